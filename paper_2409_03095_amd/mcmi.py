"""Python binding of libmcmi.so (argument marshalling only).

Every step of the Monte Carlo SPAI path runs in the HIP library; this module
moves pointers, sizes and parameters across the C ABI declared in
``include/mcmi.h``. PyTorch provides device memory and the current stream.
Importing this module fails loudly when the library has not been built: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcmi.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libmcmi.so not found at {LIB_PATH}: build it with "
                      "`python -c 'import __graft_entry__ as g; g.build()'` (hipcc, gfx950)")

# torch first: it brings its own HIP runtime (same soname as the one the library
# links), and the library must bind to that copy. Loaded the other way round the
# process ends up with two HIP runtimes, and the library's sees no device.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

MCMI_OK = 0
STATUS = {0: "ok", -1: "bad argument", -2: "bad CSR", -3: "zero or missing diagonal",
          -4: "not contractive", -5: "capacity", -6: "HIP error", -7: "out of memory"}
WALK_F64, WALK_F32 = 64, 32
FILTER_N, FILTER_M = 0, 1


class McmiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"mcmi status {status} ({STATUS.get(status, '?')}): {msg}")
        self.status = status


class CsrIn(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr_dev", ctypes.c_void_p),
                ("col_dev", ctypes.c_void_p), ("val_dev", ctypes.c_void_p)]


class CdfOpts(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("drop_frac", ctypes.c_double), ("order_cell", ctypes.c_int64),
                ("reserved", ctypes.c_int64)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("rel_residual", ctypes.c_double), ("ms", ctypes.c_double),
                ("converged", ctypes.c_int32), ("pad", ctypes.c_int32)]


class CsrOut(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr_dev", ctypes.c_void_p),
                ("col_dev", ctypes.c_void_p), ("val_dev", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("chains", ctypes.c_int32), ("walk_prec", ctypes.c_int32),
                ("delta", ctypes.c_double), ("eps", ctypes.c_double), ("max_len", ctypes.c_int32),
                ("stream_tag", ctypes.c_uint32), ("filter", ctypes.c_int32), ("lanes_per_row", ctypes.c_int32),
                ("hash_slots", ctypes.c_int32), ("sketch_slots", ctypes.c_int32), ("pool_per_row", ctypes.c_int32),
                ("heavy_weight", ctypes.c_double), ("spill_slots", ctypes.c_int32), ("topk", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("transitions", ctypes.c_uint64), ("chains", ctypes.c_uint64), ("spilled", ctypes.c_uint64),
                ("retries", ctypes.c_uint64), ("refined", ctypes.c_uint64), ("nnz", ctypes.c_int64),
                ("lmax", ctypes.c_int32), ("norm_inf", ctypes.c_float), ("ms_walk", ctypes.c_double),
                ("ms_assemble", ctypes.c_double), ("ms_total", ctypes.c_double), ("lanes_per_row", ctypes.c_int32),
                ("hash_slots", ctypes.c_int32), ("sketch_slots", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("heavy_weight", ctypes.c_double)]


_P = ctypes.POINTER
_v = ctypes.c_void_p
_sig = {
    "mcmi_build_cdf": [_P(CsrIn), _P(_v), _v],
    "mcmi_build_cdf_ex": [_P(CsrIn), _P(CdfOpts), _P(_v), _v],
    "mcmi_bicgstab": [_P(CsrIn), _P(CsrOut), _v, _v, ctypes.c_double, ctypes.c_int32, _P(SolveStats), _v],
    "mcmi_cdf_prep_info": [_v, _P(ctypes.c_double), _P(ctypes.c_double), _P(ctypes.c_int64)],
    "mcmi_cdf_order": [_v, _v, _v],
    "mcmi_cdf_info": [_v, _P(ctypes.c_int64), _P(ctypes.c_int64), _P(ctypes.c_double), _P(ctypes.c_uint64)],
    "mcmi_cdf_download": [_v, _v, _v, _v, _v],
    "mcmi_cdf_download_compact": [_v, _v, _v],
    "mcmi_build_cdf_batched": [_P(CsrIn), ctypes.c_int32, _P(_v), _v],
    "mcmi_build_cdf_batched_ex": [_P(CsrIn), ctypes.c_int32, _P(CdfOpts), _P(_v), _v],
    "mcmi_tune": [_v, _P(Params), ctypes.c_int64, ctypes.c_char_p, _P(Params), _P(ctypes.c_double), _v],
    "mcmi_plan_create": [_v, _P(Params), _v, ctypes.c_int64, _P(_v), _v],
    "mcmi_plan_launch": [_v, ctypes.c_uint64, _v],
    "mcmi_plan_result": [_v, _P(CsrOut), _P(Stats), _P(ctypes.c_int32), _v],
    "mcmi_cdf_batch_info": [_v, _P(ctypes.c_int32), _v, _v],
    "mcmi_spai": [_v, _P(Params), _v, _v, ctypes.c_int64, _P(CsrOut), _P(Stats), _v],
    "mcmi_apply": [_P(CsrOut), ctypes.c_int64, _v, _v, _v],
    "mcmi_csr_copy": [_P(CsrOut), _v, _v, _v, _v],
    "mcmi_row_features": [_v, ctypes.c_double, ctypes.c_int32, _v, _v],
    "mcmi_pilot_variance": [_v, _P(Params), ctypes.c_int32, _v, _v, _v],
    "mcmi_mlp_create": [_P(_v)],
    "mcmi_mlp_set_params": [_v, _v, _v, ctypes.c_int32],
    "mcmi_mlp_get_params": [_v, _v, _v, _v, _v, _P(ctypes.c_int64)],
    "mcmi_mlp_set_adam_state": [_v, _v, _v, ctypes.c_int64],
    "mcmi_mlp_fit_normalization": [_v, _v, ctypes.c_int64, _v],
    "mcmi_mlp_predict": [_v, _v, ctypes.c_int64, _v, _v],
    "mcmi_mlp_gradient": [_v, _v, _v, _v, ctypes.c_int64, ctypes.c_int64, _v, _P(ctypes.c_float), _v],
    "mcmi_mlp_train": [_v, _v, _v, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_uint64,
                       _v, _v],
    "mcmi_allocate": [_v, _v, ctypes.c_int64, ctypes.c_int64, _v, _P(ctypes.c_double), _P(ctypes.c_int32), _v],
    "mcmi_allocate_noalloc": [_v, _v, ctypes.c_int64, ctypes.c_int64, _v, _v, _v, _v],
    "mcmi_neyman_target": [_v, _v, ctypes.c_int64, _v, _v],
    "mcmi_chain_cost": [_v, ctypes.c_int64, _v, _P(ctypes.c_int64), _v],
    "mcmi_mlp_adam_step": [_v, _v, ctypes.c_float, _v],
}
for _name, _args in _sig.items():
    getattr(_lib, _name).argtypes = _args
    getattr(_lib, _name).restype = ctypes.c_int
_lib.mcmi_cdf_free.argtypes = [_v]
_lib.mcmi_cache_trim.argtypes = []
_lib.mcmi_cache_trim.restype = None
_lib.mcmi_cdf_free.restype = None
_lib.mcmi_plan_free.argtypes = [_v]
_lib.mcmi_plan_free.restype = None
_lib.mcmi_mlp_free.argtypes = [_v]
_lib.mcmi_mlp_free.restype = None
_lib.mcmi_csr_free.argtypes = [_P(CsrOut)]
_lib.mcmi_csr_free.restype = None
_lib.mcmi_last_error.restype = ctypes.c_char_p
_lib.mcmi_version.restype = ctypes.c_char_p

EXPORTED = ["mcmi_cache_trim", "mcmi_bicgstab", "mcmi_build_cdf", "mcmi_build_cdf_ex", "mcmi_cdf_prep_info", "mcmi_cdf_order", "mcmi_cdf_info", "mcmi_cdf_download", "mcmi_cdf_download_compact", "mcmi_spai", "mcmi_apply",
            "mcmi_csr_copy", "mcmi_cdf_free", "mcmi_csr_free", "mcmi_last_error", "mcmi_version",
            "mcmi_row_features", "mcmi_pilot_variance", "mcmi_mlp_create", "mcmi_mlp_free",
            "mcmi_mlp_set_params", "mcmi_mlp_get_params", "mcmi_mlp_set_adam_state", "mcmi_mlp_fit_normalization",
            "mcmi_mlp_predict", "mcmi_mlp_gradient", "mcmi_mlp_train", "mcmi_allocate", "mcmi_allocate_noalloc",
            "mcmi_neyman_target", "mcmi_chain_cost", "mcmi_mlp_adam_step",
            "mcmi_build_cdf_batched", "mcmi_build_cdf_batched_ex", "mcmi_cdf_batch_info", "mcmi_tune", "mcmi_plan_create", "mcmi_plan_launch",
            "mcmi_plan_result", "mcmi_plan_free"]


def _check(st):
    if st != MCMI_OK:
        raise McmiError(st, _lib.mcmi_last_error().decode(errors="replace"))


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def version() -> str:
    return _lib.mcmi_version().decode()


@dataclasses.dataclass
class DeviceCsr:
    """A CSR matrix whose arrays live in torch device tensors."""
    n: int
    row_ptr: object
    col: object
    val: object

    @property
    def nnz(self):
        return int(self.col.numel())

    @staticmethod
    def from_host(B, device="cuda"):
        import torch
        return DeviceCsr(int(B.n),
                         torch.from_numpy(np.ascontiguousarray(B.row_ptr, dtype=np.int64)).to(device),
                         torch.from_numpy(np.ascontiguousarray(B.col, dtype=np.int32)).to(device),
                         torch.from_numpy(np.ascontiguousarray(B.val, dtype=np.float64)).to(device))

    def _struct(self):
        return CsrIn(self.n, self.nnz, _ptr(self.row_ptr), _ptr(self.col), _ptr(self.val))


class Cdf:
    """Sampling records of C = I - D^-1 B (mcmi_build_cdf), or of several matrices
    in one block-diagonal row space (Cdf.batched -> mcmi_build_cdf_batched)."""

    def __init__(self, B: DeviceCsr = None, stream=None, _batch=None, alpha=0.0, drop_frac=0.0, order_cell=0):
        self._h = ctypes.c_void_p()
        self._B = B if B is not None else _batch
        if _batch is None:
            s = B._struct()
            if alpha or drop_frac or order_cell:
                opts = CdfOpts(float(alpha), float(drop_frac), int(order_cell), 0)
                _check(_lib.mcmi_build_cdf_ex(ctypes.byref(s), ctypes.byref(opts), ctypes.byref(self._h),
                                              _stream(stream)))
            else:
                _check(_lib.mcmi_build_cdf(ctypes.byref(s), ctypes.byref(self._h), _stream(stream)))
        else:
            arr = (CsrIn * len(_batch))(*[m._struct() for m in _batch])
            if order_cell:
                opts = CdfOpts(0.0, 0.0, int(order_cell), 0)
                _check(_lib.mcmi_build_cdf_batched_ex(arr, ctypes.c_int32(len(_batch)), ctypes.byref(opts),
                                                      ctypes.byref(self._h), _stream(stream)))
            else:
                _check(_lib.mcmi_build_cdf_batched(arr, ctypes.c_int32(len(_batch)), ctypes.byref(self._h),
                                                   _stream(stream)))
        n, nnz_c, nrm, units = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_uint64()
        _check(_lib.mcmi_cdf_info(self._h, ctypes.byref(n), ctypes.byref(nnz_c), ctypes.byref(nrm),
                                  ctypes.byref(units)))
        self.n, self.nnz_c, self.norm_inf, self.rec_units = n.value, nnz_c.value, nrm.value, units.value

    def prep_info(self):
        """(||B||_inf, reduction cut, entries removed) of the pre-pass."""
        nb, cut, nd = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        _check(_lib.mcmi_cdf_prep_info(self._h, ctypes.byref(nb), ctypes.byref(cut), ctypes.byref(nd)))
        return nb.value, cut.value, nd.value

    def order(self, stream=None):
        """mcmi_cdf_order: the row schedule (int32 permutation of [0, n))."""
        out = np.zeros(self.n, dtype=np.int32)
        _check(_lib.mcmi_cdf_order(self._h, out.ctypes.data_as(_v), _stream(stream)))
        return out

    @staticmethod
    def batched(mats, stream=None, order_cell=0):
        return Cdf(None, stream, _batch=list(mats), order_cell=order_cell)

    def batch_info(self):
        k = ctypes.c_int32()
        _check(_lib.mcmi_cdf_batch_info(self._h, ctypes.byref(k), None, None))
        cnt = max(k.value, 1)
        base = np.zeros(cnt + 1, dtype=np.int64)
        nrm = np.zeros(cnt, dtype=np.float64)
        _check(_lib.mcmi_cdf_batch_info(self._h, ctypes.byref(k), base.ctypes.data_as(_v), nrm.ctypes.data_as(_v)))
        return k.value, base, nrm

    def download(self, stream=None):
        rec = np.zeros(self.rec_units * 16, dtype=np.uint32)
        roff = np.zeros(self.n, dtype=np.uint32)
        diag = np.zeros(self.n, dtype=np.float64)
        _check(_lib.mcmi_cdf_download(self._h, rec.ctypes.data_as(_v), roff.ctypes.data_as(_v),
                                      diag.ctypes.data_as(_v), _stream(stream)))
        return rec, roff, diag

    def download_compact(self, stream=None):
        rec32 = np.zeros(self.rec_units * 8, dtype=np.uint32)
        _check(_lib.mcmi_cdf_download_compact(self._h, rec32.ctypes.data_as(_v), _stream(stream)))
        return rec32

    def free(self):
        if self._h:
            _lib.mcmi_cdf_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class SpaiResult:
    """Library-owned CSR M plus the run statistics."""

    def __init__(self, out: CsrOut, stats: Stats, n_cols: int):
        self._out = out
        self.stats = stats
        self.n_cols = n_cols

    @property
    def n(self):
        return self._out.n

    @property
    def nnz(self):
        return self._out.nnz

    def to_torch(self, stream=None):
        import torch
        rp = torch.empty(self.n + 1, dtype=torch.int64, device="cuda")
        col = torch.empty(max(self.nnz, 1), dtype=torch.int32, device="cuda")
        val = torch.empty(max(self.nnz, 1), dtype=torch.float64, device="cuda")
        _check(_lib.mcmi_csr_copy(ctypes.byref(self._out), _ptr(rp), _ptr(col), _ptr(val), _stream(stream)))
        return rp, col[:self.nnz], val[:self.nnz]

    def to_numpy(self, stream=None):
        import torch
        rp, col, val = self.to_torch(stream)
        torch.cuda.current_stream().synchronize()
        return rp.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy()

    def apply(self, x, y=None, stream=None):
        """y = M x (mcmi_apply); x and y are float64 device tensors."""
        import torch
        if y is None:
            y = torch.empty(self.n, dtype=torch.float64, device=x.device)
        _check(_lib.mcmi_apply(ctypes.byref(self._out), ctypes.c_int64(self.n_cols), _ptr(x), _ptr(y),
                               _stream(stream)))
        return y

    def free(self):
        if self._out.row_ptr_dev:
            _lib.mcmi_csr_free(ctypes.byref(self._out))

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def params(seed=0, chains=16, delta=1e-3, eps=1e-3, walk_prec=WALK_F64, max_len=0, tag=0, filter=FILTER_N,
           lanes_per_row=0, hash_slots=0, sketch_slots=0, heavy_weight=0.0, pool_per_row=0,
           spill_slots=0, topk=0) -> Params:
    return Params(int(seed) & 0xFFFFFFFFFFFFFFFF, int(chains), int(walk_prec), float(delta), float(eps),
                  int(max_len), int(tag) & 0xFFFFFFFF, int(filter), int(lanes_per_row), int(hash_slots),
                  int(sketch_slots), int(pool_per_row), float(heavy_weight), int(spill_slots), int(topk))


def spai(cdf: Cdf, p: Params, chains_per_row=None, rows=None, stream=None) -> SpaiResult:
    """mcmi_spai: chains_per_row / rows are int32 device tensors or None."""
    out = CsrOut()
    st = Stats()
    n_rows = int(rows.numel()) if rows is not None else 0
    _check(_lib.mcmi_spai(cdf._h, ctypes.byref(p), _ptr(chains_per_row), _ptr(rows), ctypes.c_int64(n_rows),
                          ctypes.byref(out), ctypes.byref(st), _stream(stream)))
    return SpaiResult(out, st, cdf.n)


def row_features(cdf: Cdf, delta: float, max_len: int = 0, stream=None):
    """mcmi_row_features: (n, 8) float32 device tensor."""
    import torch
    f = torch.empty((cdf.n, 8), dtype=torch.float32, device="cuda")
    _check(_lib.mcmi_row_features(cdf._h, ctypes.c_double(delta), ctypes.c_int32(max_len), _ptr(f),
                                  _stream(stream)))
    return f


def pilot_variance(cdf: Cdf, p: Params, pilot_chains: int = 64, stream=None):
    """mcmi_pilot_variance: per-row (variance, mean length), float64 device tensors."""
    import torch
    var = torch.empty(cdf.n, dtype=torch.float64, device="cuda")
    ln = torch.empty(cdf.n, dtype=torch.float64, device="cuda")
    _check(_lib.mcmi_pilot_variance(cdf._h, ctypes.byref(p), ctypes.c_int32(pilot_chains), _ptr(var), _ptr(ln),
                                    _stream(stream)))
    return var, ln


MLP_PARAMS = 4801


class Mlp:
    """The allocation network (library-owned parameters and Adam state)."""

    def __init__(self):
        self._h = ctypes.c_void_p()
        _check(_lib.mcmi_mlp_create(ctypes.byref(self._h)))

    def set_params(self, params, norm=None, reset_optimizer=True):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == MLP_PARAMS
        nm = None if norm is None else np.ascontiguousarray(norm, dtype=np.float32)
        _check(_lib.mcmi_mlp_set_params(self._h, p.ctypes.data_as(_v), None if nm is None else nm.ctypes.data_as(_v),
                                        int(bool(reset_optimizer))))

    def get_params(self):
        p = np.zeros(MLP_PARAMS, np.float32)
        nm = np.zeros(16, np.float32)
        m = np.zeros(MLP_PARAMS, np.float32)
        v = np.zeros(MLP_PARAMS, np.float32)
        t = ctypes.c_int64()
        _check(_lib.mcmi_mlp_get_params(self._h, p.ctypes.data_as(_v), nm.ctypes.data_as(_v), m.ctypes.data_as(_v),
                                        v.ctypes.data_as(_v), ctypes.byref(t)))
        return {"params": p, "norm": nm, "adam_m": m, "adam_v": v, "step": t.value}

    def set_adam_state(self, m, v, step):
        m = np.ascontiguousarray(m, np.float32)
        v = np.ascontiguousarray(v, np.float32)
        _check(_lib.mcmi_mlp_set_adam_state(self._h, m.ctypes.data_as(_v), v.ctypes.data_as(_v), int(step)))

    def fit_normalization(self, feat, stream=None):
        _check(_lib.mcmi_mlp_fit_normalization(self._h, _ptr(feat), ctypes.c_int64(feat.shape[0]), _stream(stream)))

    def predict(self, feat, stream=None):
        import torch
        out = torch.empty(feat.shape[0], dtype=torch.float32, device=feat.device)
        _check(_lib.mcmi_mlp_predict(self._h, _ptr(feat), ctypes.c_int64(feat.shape[0]), _ptr(out), _stream(stream)))
        return out

    def gradient(self, feat, target, idx, stream=None):
        g = np.zeros(MLP_PARAMS, np.float32)
        loss = ctypes.c_float()
        _check(_lib.mcmi_mlp_gradient(self._h, _ptr(feat), _ptr(target), _ptr(idx), ctypes.c_int64(idx.numel()),
                                      ctypes.c_int64(feat.shape[0]), g.ctypes.data_as(_v), ctypes.byref(loss),
                                      _stream(stream)))
        return g, loss.value

    def train(self, feat, target, steps, batch=4096, lr=1e-3, seed=0, stream=None):
        losses = np.zeros(max(steps, 1), np.float32)
        _check(_lib.mcmi_mlp_train(self._h, _ptr(feat), _ptr(target), ctypes.c_int64(feat.shape[0]),
                                   ctypes.c_int32(steps), ctypes.c_int32(batch), ctypes.c_float(lr),
                                   ctypes.c_uint64(seed), losses.ctypes.data_as(_v), _stream(stream)))
        return losses[:steps]

    def adam_step(self, grad, lr=1e-3, stream=None):
        """mcmi_mlp_adam_step: one Adam step with the float32 device gradient `grad`."""
        assert grad.numel() == MLP_PARAMS
        _check(_lib.mcmi_mlp_adam_step(self._h, _ptr(grad), ctypes.c_float(lr), _stream(stream)))

    def free(self):
        if self._h:
            _lib.mcmi_mlp_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def neyman_target(var, ln, stream=None):
    """mcmi_neyman_target: float32 regression target per row from the pilot's
    float64 variance and mean length (device tensors)."""
    import torch
    y = torch.empty(var.numel(), dtype=torch.float32, device=var.device)
    _check(_lib.mcmi_neyman_target(_ptr(var), _ptr(ln), ctypes.c_int64(var.numel()), _ptr(y), _stream(stream)))
    return y


def chain_cost(feat, stream=None):
    """mcmi_chain_cost: (int32 cost per row, total) from the (n, 8) features."""
    import torch
    cost = torch.empty(feat.shape[0], dtype=torch.int32, device=feat.device)
    tot = ctypes.c_int64()
    _check(_lib.mcmi_chain_cost(_ptr(feat), ctypes.c_int64(feat.shape[0]), _ptr(cost), ctypes.byref(tot),
                                _stream(stream)))
    return cost, tot.value


def allocate(pred, cost, budget, stream=None):
    """mcmi_allocate: chains per row (int32 device tensor), lambda, fallback flag."""
    import torch
    chains = torch.empty(pred.numel(), dtype=torch.int32, device=pred.device)
    lam = ctypes.c_double()
    fb = ctypes.c_int32()
    _check(_lib.mcmi_allocate(_ptr(pred), _ptr(cost), ctypes.c_int64(pred.numel()), ctypes.c_int64(int(budget)),
                              _ptr(chains), ctypes.byref(lam), ctypes.byref(fb), _stream(stream)))
    return chains, lam.value, bool(fb.value)


def allocate_noalloc(pred, cost, budget, chains, lam=None, fallback=None, stream=None):
    """mcmi_allocate_noalloc: writes chains (int32 device tensor of pred's length) and,
    when given, lam (float64, one element) and fallback (int32, one element), all on
    the device; asynchronous, no allocation inside the library."""
    _check(_lib.mcmi_allocate_noalloc(_ptr(pred), _ptr(cost), ctypes.c_int64(pred.numel()),
                                      ctypes.c_int64(int(budget)), _ptr(chains), _ptr(lam), _ptr(fallback),
                                      _stream(stream)))


def tune(cdf: Cdf, p: Params, sample_rows=8192, cache_path=None, stream=None):
    """mcmi_tune: (best Params, walk ms of the best candidate)."""
    best = Params()
    ms = ctypes.c_double()
    _check(_lib.mcmi_tune(cdf._h, ctypes.byref(p), ctypes.c_int64(sample_rows),
                          None if cache_path is None else str(cache_path).encode(), ctypes.byref(best),
                          ctypes.byref(ms), _stream(stream)))
    return best, ms.value


class Plan:
    """mcmi_plan: preallocated SPAI with its device work captured in a hipGraph."""

    def __init__(self, cdf: Cdf, p: Params, nnz_capacity, chains_per_row=None, stream=None):
        self._h = ctypes.c_void_p()
        self._cdf = cdf
        self._cpr = chains_per_row
        _check(_lib.mcmi_plan_create(cdf._h, ctypes.byref(p), _ptr(chains_per_row), ctypes.c_int64(nnz_capacity),
                                     ctypes.byref(self._h), _stream(stream)))

    def launch(self, seed, stream=None):
        _check(_lib.mcmi_plan_launch(self._h, ctypes.c_uint64(seed), _stream(stream)))

    def result(self, stream=None):
        """(rp, col, val) numpy copies, stats, overflow flag."""
        import torch
        out, st, ovf = CsrOut(), Stats(), ctypes.c_int32()
        _check(_lib.mcmi_plan_result(self._h, ctypes.byref(out), ctypes.byref(st), ctypes.byref(ovf), _stream(stream)))
        if ovf.value:
            return None, st, True
        rp = torch.empty(out.n + 1, dtype=torch.int64, device="cuda")
        col = torch.empty(max(out.nnz, 1), dtype=torch.int32, device="cuda")
        val = torch.empty(max(out.nnz, 1), dtype=torch.float64, device="cuda")
        _check(_lib.mcmi_csr_copy(ctypes.byref(out), _ptr(rp), _ptr(col), _ptr(val), _stream(stream)))
        torch.cuda.current_stream().synchronize()
        return (rp.cpu().numpy(), col[:out.nnz].cpu().numpy(), val[:out.nnz].cpu().numpy()), st, False

    def stats(self, stream=None):
        """(stats, overflow flag, nnz) of the last launch, without copying M."""
        out, st, ovf = CsrOut(), Stats(), ctypes.c_int32()
        _check(_lib.mcmi_plan_result(self._h, ctypes.byref(out), ctypes.byref(st), ctypes.byref(ovf), _stream(stream)))
        return st, bool(ovf.value), int(out.nnz)

    def free(self):
        if self._h:
            _lib.mcmi_plan_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def bicgstab(B: DeviceCsr, M=None, b=None, x0=None, rtol=1e-8, maxiter=5000, stream=None):
    """mcmi_bicgstab: solve B x = b on the device, M (a SpaiResult) applied on the
    right. b, x0: float64 device tensors (x0 defaults to zeros). Returns (x, SolveStats)."""
    import torch
    x = torch.zeros(B.n, dtype=torch.float64, device="cuda") if x0 is None else x0.clone()
    st = SolveStats()
    s = B._struct()
    _check(_lib.mcmi_bicgstab(ctypes.byref(s), None if M is None else ctypes.byref(M._out), _ptr(b), _ptr(x),
                              ctypes.c_double(rtol), ctypes.c_int32(maxiter), ctypes.byref(st), _stream(stream)))
    return x, st


def cache_trim():
    """mcmi_cache_trim: return the library's cached device memory to the driver."""
    _lib.mcmi_cache_trim()
