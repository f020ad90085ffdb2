"""Python face of the CPU oracle (TEST INFRASTRUCTURE ONLY).

* ctypes wrapper of ``mcmi_oracle.c`` (iteration matrix, quantized CDF, Philox,
  FP64 walks, long-double accumulation, epsilon filter, column scaling, apply,
  pilot variance, row features);
* numpy FP64 reference for the allocation network (8-64-64-1 ReLU MLP, MSE,
  Adam) and for the Neyman chain allocation;
* scipy references for the quality metric ||I - M B||_F and BiCGstab.

Nothing here imports the HIP library. Citations name the paper's sections.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mcmi_oracle.c")
LIB = os.path.join(HERE, "libmcmi_oracle.so")

ORC_OK = 0
ERRORS = {-1: "bad argument", -2: "bad CSR", -3: "zero or missing diagonal",
          -4: "not contractive (||Chat||_inf >= 1) and no max_len", -7: "out of memory"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fused multiply-add, no fast-math)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-pthread",
                               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.orc_count_c.restype = ctypes.c_int
        L.orc_build.restype = ctypes.c_int
        L.orc_lmax.restype = ctypes.c_int
        L.orc_lmax.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int]
        L.orc_spai.restype = ctypes.c_int
        L.orc_pilot.restype = ctypes.c_int
        L.orc_features.restype = None
        L.orc_features.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_void_p]
        L.orc_apply.restype = None
        L.orc_draw.restype = ctypes.c_int64
        L.orc_draw.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32]
        L.orc_build_alias.restype = ctypes.c_int
        L.orc_prepare.restype = ctypes.c_int
        L.orc_prepare.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        del i64p
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class _Mat(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("cptr", ctypes.c_void_p), ("ccol", ctypes.c_void_p),
                ("cval", ctypes.c_void_p), ("cum", ctypes.c_void_p), ("wsum", ctypes.c_void_p),
                ("shat", ctypes.c_void_p), ("diag", ctypes.c_void_p), ("norm_inf", ctypes.c_double),
                ("athr", ctypes.c_void_p), ("aidx", ctypes.c_void_p)]


class _Params(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("delta", ctypes.c_double), ("eps", ctypes.c_double),
                ("chains", ctypes.c_int32), ("fp32", ctypes.c_int32), ("max_len", ctypes.c_int32),
                ("tag", ctypes.c_uint32), ("threads", ctypes.c_int32), ("filter_on_m", ctypes.c_int32),
                ("topk", ctypes.c_int32)]


class _Result(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("row_ptr", ctypes.POINTER(ctypes.c_int64)),
                ("col", ctypes.POINTER(ctypes.c_int32)), ("val", ctypes.POINTER(ctypes.c_double)),
                ("abssum", ctypes.POINTER(ctypes.c_double)), ("cnt", ctypes.POINTER(ctypes.c_uint32)),
                ("row_transitions", ctypes.POINTER(ctypes.c_int64)), ("transitions", ctypes.c_uint64),
                ("guard", ctypes.c_int64), ("lmax", ctypes.c_int32), ("row_ambig", ctypes.POINTER(ctypes.c_int32)),
                ("row_border", ctypes.POINTER(ctypes.c_int64))]


class OracleError(RuntimeError):
    pass


def _check(st):
    if st != ORC_OK:
        raise OracleError(f"oracle status {st}: {ERRORS.get(st, '?')}")


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def prepare(B, alpha=0.0, drop_frac=0.0):
    """orc_prepare: B' (row_ptr, col, val) with the augmented diagonal and the
    reduced entries, plus (||B||_inf, cut, number dropped)."""
    L = lib()
    n = int(B.n)
    rp = np.ascontiguousarray(B.row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(B.col, dtype=np.int32)
    v = np.ascontiguousarray(B.val, dtype=np.float64)
    rp2 = np.zeros(n + 1, dtype=np.int64)
    ci2 = np.zeros(rp[-1] + n, dtype=np.int32)
    v2 = np.zeros(rp[-1] + n, dtype=np.float64)
    nrm, thr, nd = ctypes.c_double(0.0), ctypes.c_double(0.0), ctypes.c_int64(0)
    _check(L.orc_prepare(ctypes.c_int64(n), _p(rp), _p(ci), _p(v), float(alpha), float(drop_frac), _p(rp2), _p(ci2),
                         _p(v2), ctypes.byref(nrm), ctypes.byref(thr), ctypes.byref(nd)))
    e = int(rp2[-1])
    return (rp2, ci2[:e].copy(), v2[:e].copy()), (nrm.value, thr.value, nd.value)


class Oracle:
    """Iteration matrix C and its integer CDF for one input B (O1, O2), after the
    optional pre-pass (alpha-augmented diagonal, matrix reduction)."""

    def __init__(self, B, alpha=0.0, drop_frac=0.0):
        L = lib()
        self.n = int(B.n)
        self.norm_b, self.drop_thr, self.dropped = 0.0, 0.0, 0
        if alpha or drop_frac:
            (rp, ci, v), (self.norm_b, self.drop_thr, self.dropped) = prepare(B, alpha, drop_frac)
        else:
            rp = np.ascontiguousarray(B.row_ptr, dtype=np.int64)
            ci = np.ascontiguousarray(B.col, dtype=np.int32)
            v = np.ascontiguousarray(B.val, dtype=np.float64)
        nnz_c = ctypes.c_int64(0)
        _check(L.orc_count_c(ctypes.c_int64(self.n), _p(rp), _p(ci), _p(v), ctypes.byref(nnz_c)))
        m = nnz_c.value
        self.cptr = np.zeros(self.n + 1, dtype=np.int64)
        self.ccol = np.zeros(max(m, 1), dtype=np.int32)
        self.cval = np.zeros(max(m, 1), dtype=np.float64)
        self.cum = np.zeros(max(m, 1), dtype=np.uint32)
        self.wsum = np.zeros(self.n, dtype=np.uint32)
        self.shat = np.zeros(self.n, dtype=np.float64)
        self.diag = np.zeros(self.n, dtype=np.float64)
        nrm = ctypes.c_double(0.0)
        _check(L.orc_build(ctypes.c_int64(self.n), _p(rp), _p(ci), _p(v), _p(self.cptr), _p(self.ccol),
                           _p(self.cval), _p(self.cum), _p(self.wsum), _p(self.shat), _p(self.diag),
                           ctypes.byref(nrm)))
        self.norm_inf = nrm.value
        self.nnz_c = m
        self.athr = np.zeros(max(m, 1), dtype=np.uint32)
        self.aidx = np.zeros(max(m, 1), dtype=np.int32)
        _check(L.orc_build_alias(ctypes.c_int64(self.n), _p(self.cptr), _p(self.cum), _p(self.wsum),
                                 _p(self.athr), _p(self.aidx)))
        self._mat = _Mat(self.n, _p(self.cptr).value, _p(self.ccol).value, _p(self.cval).value,
                         _p(self.cum).value, _p(self.wsum).value, _p(self.shat).value,
                         _p(self.diag).value, self.norm_inf, _p(self.athr).value, _p(self.aidx).value)

    # ---- derived views (used by tests; all from the oracle's own arrays)
    def row_weights(self, i):
        b, e = self.cptr[i], self.cptr[i + 1]
        cum = self.cum[b:e].astype(np.int64)
        return np.diff(np.concatenate([[0], cum]))

    def chat_dense(self):
        """Dense quantized Chat: |chat_k| = Shat_i w_k / W_i, sign of c_k (exact rationals
        rounded once each)."""
        n = self.n
        out = np.zeros((n, n))
        for i in range(n):
            b, e = self.cptr[i], self.cptr[i + 1]
            if e == b:
                continue
            w = self.row_weights(i).astype(np.float64)
            out[i, self.ccol[b:e]] = np.sign(self.cval[b:e]) * self.shat[i] * w / float(self.wsum[i])
        return out

    def draw(self, row, u):
        """Entry of `row` (0-based inside the row) chosen by the 32-bit word u."""
        return int(lib().orc_draw(ctypes.byref(self._mat), int(row), int(u) & 0xFFFFFFFF))

    def lmax(self, delta, max_len=0):
        r = lib().orc_lmax(self.norm_inf, float(delta), int(max_len))
        _check(r if r < 0 else 0)
        return r

    def _params(self, seed, chains, delta, eps, fp32, max_len, tag, threads, filter_on_m, topk=0):
        return _Params(int(seed) & 0xFFFFFFFFFFFFFFFF, float(delta), float(eps), int(chains), int(bool(fp32)),
                       int(max_len), int(tag) & 0xFFFFFFFF,
                       int(threads if threads else default_threads()), int(bool(filter_on_m)), int(topk))

    def spai(self, seed=0, chains=16, delta=1e-3, eps=1e-3, fp32=False, max_len=0, tag=0,
             rows=None, chains_per_row=None, threads=None, filter_on_m=False, topk=0):
        """O3-O6 for all rows (rows=None) or the listed rows, in the given order.

        Returns a dict: row_ptr, col, val (M rows), abssum/cnt (per kept entry: sum of
        |W| and number of contributions), row_transitions, transitions, guard, lmax,
        row_ambig (top-k boundary order-dependent, per row), row_border (per row: chains
        with a cutoff test inside the rounding band of binary32 weights)."""
        prm = self._params(seed, chains, delta, eps, fp32, max_len, tag, threads, filter_on_m, topk)
        rows_arr = None if rows is None else np.ascontiguousarray(rows, dtype=np.int32)
        cpr = None if chains_per_row is None else np.ascontiguousarray(chains_per_row, dtype=np.int32)
        res = _Result()
        st = lib().orc_spai(ctypes.byref(self._mat), ctypes.byref(prm),
                            None if rows_arr is None else _p(rows_arr),
                            ctypes.c_int64(0 if rows_arr is None else rows_arr.size),
                            None if cpr is None else _p(cpr), ctypes.byref(res))
        try:
            _check(st)
            nr = res.nrows
            rp = np.ctypeslib.as_array(res.row_ptr, shape=(nr + 1,)).copy()
            nnz = int(rp[-1])
            out = {
                "row_ptr": rp,
                "col": np.ctypeslib.as_array(res.col, shape=(max(nnz, 1),))[:nnz].copy(),
                "val": np.ctypeslib.as_array(res.val, shape=(max(nnz, 1),))[:nnz].copy(),
                "abssum": np.ctypeslib.as_array(res.abssum, shape=(max(nnz, 1),))[:nnz].copy(),
                "cnt": np.ctypeslib.as_array(res.cnt, shape=(max(nnz, 1),))[:nnz].copy(),
                "row_transitions": np.ctypeslib.as_array(res.row_transitions, shape=(max(nr, 1),))[:nr].copy(),
                "transitions": int(res.transitions),
                "guard": int(res.guard),
                "lmax": int(res.lmax),
                "row_ambig": np.ctypeslib.as_array(res.row_ambig, shape=(max(nr, 1),))[:nr].copy(),
                "row_border": np.ctypeslib.as_array(res.row_border, shape=(max(nr, 1),))[:nr].copy(),
            }
        finally:
            lib().orc_result_free(ctypes.byref(res))
        return out

    def pilot(self, seed=0, pilot=64, delta=1e-3, fp32=False, max_len=0, tag=0, threads=None):
        """Per-row total variance of one chain's row estimate and mean chain length."""
        prm = self._params(seed, 1, delta, 0.0, fp32, max_len, tag, threads, False)
        var = np.zeros(self.n)
        ln = np.zeros(self.n)
        _check(lib().orc_pilot(ctypes.byref(self._mat), ctypes.byref(prm), ctypes.c_int32(pilot),
                               _p(var), _p(ln)))
        return var, ln

    def features(self, delta, max_len=0):
        lm = self.lmax(delta, max_len)
        f = np.zeros((self.n, 8))
        lib().orc_features(ctypes.byref(self._mat), float(delta), int(lm), _p(f))
        return f


def spai_csr(res, n, rows=None):
    """Scipy CSR of an oracle result (rows=None: all rows in order)."""
    import scipy.sparse as sp
    nr = res["row_ptr"].size - 1
    M = sp.csr_matrix((res["val"], res["col"], res["row_ptr"]), shape=(nr, n))
    return M


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(o))
    return o


def apply(M_row_ptr, M_col, M_val, x):
    """O7: y = M x, plain FP64, ascending column order."""
    n = M_row_ptr.size - 1
    rp = np.ascontiguousarray(M_row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(M_col, dtype=np.int32)
    v = np.ascontiguousarray(M_val, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros(n)
    lib().orc_apply(ctypes.c_int64(n), _p(rp), _p(ci), _p(v), _p(xx), _p(y))
    return y


# ------------------------------------------------------------ quality metric
def residual_rows(B, M_rows_csr, rows):
    """Row r of I - M B for the listed rows (M_rows_csr holds exactly those rows):
    returns the squared 2-norm of each residual row (exact, scipy sparse)."""
    import scipy.sparse as sp
    Bs = B.to_scipy() if hasattr(B, "to_scipy") else B
    R = M_rows_csr @ Bs
    E = sp.csr_matrix((np.ones(len(rows)), (np.arange(len(rows)), np.asarray(rows))),
                      shape=R.shape)
    D = (E - R).tocsr()
    return np.asarray(D.multiply(D).sum(axis=1)).ravel()


def frobenius_residual(B, M_csr):
    """||I - M B||_F (exact) and its value divided by sqrt(n)."""
    n = B.n
    sq = residual_rows(B, M_csr, np.arange(n))
    r = math.sqrt(float(sq.sum()))
    return r, r / math.sqrt(n)


def bicgstab_iters(B, M_csr=None, rtol=1e-8, maxiter=5000):
    """Iterations of scipy BiCGstab on B x = B 1, x0 = 0, optional preconditioner M."""
    import scipy.sparse.linalg as spla
    Bs = B.to_scipy()
    b = Bs @ np.ones(B.n)
    it = [0]

    def cb(_):
        it[0] += 1

    Mop = None
    if M_csr is not None:
        Mop = spla.LinearOperator(Bs.shape, matvec=lambda v: M_csr @ v)
    x, info = spla.bicgstab(Bs, b, x0=np.zeros(B.n), rtol=rtol, maxiter=maxiter, M=Mop, callback=cb)
    return it[0], info, float(np.linalg.norm(b - Bs @ x) / np.linalg.norm(b))


# ------------------------------------------------------------ MLP reference
MLP_SHAPES = [("w1", (64, 8)), ("b1", (64,)), ("w2", (64, 64)), ("b2", (64,)),
              ("w3", (64,)), ("b3", (1,))]


def mlp_init(seed=0):
    """He-uniform init of the 8-64-64-1 network (FP32 master values)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in MLP_SHAPES:
        if name.startswith("w"):
            fan_in = shape[-1] if len(shape) > 1 else 64
            lim = math.sqrt(6.0 / fan_in)
            p[name] = rng.uniform(-lim, lim, size=shape).astype(np.float32)
        else:
            p[name] = np.zeros(shape, dtype=np.float32)
    return p


def mlp_forward(p, x):
    """FP64 forward: h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = w3 . h2 + b3."""
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ p["w1"].astype(np.float64).T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["w2"].astype(np.float64).T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["w3"].astype(np.float64) + float(p["b3"][0])
    return y, (x, z1, h1, z2, h2)


def mlp_loss_grad(p, x, t):
    """Mean squared error and its FP64 gradient with respect to every parameter."""
    y, (x, z1, h1, z2, h2) = mlp_forward(p, x)
    B = x.shape[0]
    r = y - np.asarray(t, dtype=np.float64)
    loss = float(np.mean(r * r))
    dy = 2.0 * r / B
    g = {}
    g["w3"] = h2.T @ dy
    g["b3"] = np.array([dy.sum()])
    dh2 = np.outer(dy, p["w3"].astype(np.float64)) * (z2 > 0)
    g["w2"] = dh2.T @ h1
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2 @ p["w2"].astype(np.float64)) * (z1 > 0)
    g["w1"] = dh1.T @ x
    g["b1"] = dh1.sum(axis=0)
    return loss, g


def adam_step(p, g, state, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba) of the FP32 master weights, in FP64."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    out = {}
    for name, _ in MLP_SHAPES:
        m = state.setdefault("m_" + name, np.zeros_like(p[name], dtype=np.float64))
        v = state.setdefault("v_" + name, np.zeros_like(p[name], dtype=np.float64))
        m[...] = beta1 * m + (1 - beta1) * g[name]
        v[...] = beta2 * v + (1 - beta2) * g[name] * g[name]
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        out[name] = (p[name].astype(np.float64) - lr * mh / (np.sqrt(vh) + eps))
    return out


def bf16_round(a):
    """Round float32 values to bfloat16 (nearest, ties to even), returned as float32."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(a)
    out = r.astype(np.uint32).view(np.float32).copy()
    out[nan] = np.float32("nan")
    return out


# ------------------------------------------------------ Neyman allocation
def neyman_target(var, mean_len):
    """Per-row regression target y = (ln v - ln(len + 1)) / 2 (Neyman allocation:
    minimize sum v/N subject to sum N (len + 1) = T gives N proportional to
    sqrt(v / (len + 1)))."""
    v = np.maximum(np.asarray(var, dtype=np.float64), 1e-30)
    return 0.5 * (np.log(v) - np.log(np.asarray(mean_len, dtype=np.float64) + 1.0))


def chain_cost(f7):
    """Budget units of one chain per row: 1 + floor(f7), with f7 = min(L_max,
    ln delta / ln S_i) the feature as stored (binary32, so the integer decision is
    taken in the precision of the stored feature). When every row of C has the
    same |C| row sum S, a chain makes exactly floor(ln delta / ln S) transitions
    (it stops before the draw whose weight S^j would fall below delta), so the
    cost is its number of visited states."""
    f = np.asarray(f7, dtype=np.float32).astype(np.float64)
    return (1 + np.floor(np.maximum(f, 0.0))).astype(np.int64)


def allocate(pred_log, cost, budget, iters=100):
    """N_r = max(1, round(lam * exp(pred_r))) with lam found by bisection so that
    sum_r N_r cost_r is as close to `budget` as possible without exceeding it."""
    e = np.exp(np.asarray(pred_log, dtype=np.float64))
    cost = np.asarray(cost, dtype=np.int64)

    def total(lam):
        n_r = np.maximum(1, np.rint(lam * e)).astype(np.int64)
        return int((n_r * cost).sum()), n_r

    lo, hi = 0.0, 1.0
    while total(hi)[0] <= budget and hi < 1e30:
        hi *= 2.0
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if total(mid)[0] <= budget:
            lo = mid
        else:
            hi = mid
    return total(lo)[1], lo
