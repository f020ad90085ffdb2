"""Benchmark: Monte Carlo SPAI throughput (transitions/s) on one MI355X.

Workload (default): 3D 27-point anisotropic diffusion on a 160^3 grid
(n = 4,096,000, Q1 tensor stencil with conductivities 1:10:100, +-10 %
multiplicative noise on the off-diagonals, uniform diagonal so that
||C||_inf = 0.75); 64 chains per row, FP32 walk weights with FP64 sums,
delta = 1e-4, eps = 1e-3, Philox seed 0; rows walked cell by cell (cells of
4096 rows grown on B's pattern).

One step = the whole hot path over the matrix, through the C ABI:
mcmi_build_cdf (records and the row schedule) + mcmi_spai (walks,
accumulation, filter, scaling, CSR assembly) + mcmi_apply (one y = M x).
Inputs are resident in HBM before the timed region starts.

The JSON line carries, beside the throughput:
* roofline: the walk kernel's algorithmic bytes per transition x transitions
  per launch / its event-timed duration, against 8 TB/s of HBM;
* cpu_baseline: the CPU oracle (FP64) timed on a bounded uniform row sample
  on the host's cores; in the same leg the GPU's result on those rows is
  compared with the oracle's (precision: error against the FP64 oracle, and
  identity with the oracle's FP32-weight mode);
* secondary: the same figures for the random nonsymmetric n = 262144
  workload (512 chains per row, every chain exactly 25 transitions).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MC transitions/s; time to ‖I−MB‖_F≤0.3, learned vs uniform chains"
HBM_PEAK_GBS = 8000.0
# HBM bytes per walk launch from rocprofv3 DRAM request counters, keyed by the
# workload and kernel configuration they were measured on; None where no
# measurement of the current kernel exists
TRAFFIC_BYTES = {
    # FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000 (the factors that make a plain 1 GiB
    # device copy read 1 GiB), KiB -> bytes, one walk launch of the default
    # configuration of each workload
    "aniso27": (1.1611e8 * 2.0 + 8.5626e6) * 1024.0,
    "random": (1.8886e8 * 2.0 + 1.9607e6) * 1024.0,
    "batched": (1.1050e8 * 2.0 + 5.8260e7) * 1024.0,
}
# Instruction issue of the 160^3 walk (k_walk<true, 64, 1, true>) from rocprofv3 SQ
# counters of one launch (wave-summed quad cycles over SQ_WAVE_CYCLES = 1.035e11,
# 3072 waves, 3 per SIMD, the LDS tables allowing no more): the walk is bound by
# each wave's issue and waits, not by HBM (with every bucket read served from a
# 128 MB region the walk was not faster per transition)
ISSUE = {
    "aniso27": {"waves_per_simd": 3, "valu_busy_per_simd": round(2.286e10 / 1.035e11 * 3, 3),
                "salu_busy_per_simd": round(1.462e10 / 1.035e11 * 3, 3),
                "wave_issuing": round(4.626e10 / 1.035e11, 3), "wave_waiting_on_memory_or_lds": round(
                    4.471e10 / 1.035e11, 3), "valu_insts_per_transition": 3.45, "salu_insts_per_transition": 2.21,
                "lds_insts_per_transition": 0.33,
                "counters": "SQ_ACTIVE_INST_VALU, SQ_ACTIVE_INST_SCA, SQ_ACTIVE_INST_ANY, SQ_WAIT_ANY, "
                            "SQ_WAVE_CYCLES, SQ_INSTS_VALU, SQ_INSTS_SALU, SQ_INSTS_LDS"},
}
# what a draw of the implemented sampler must read per transition: the alias
# bucket's threshold and two targets (12 B) and the next state's header (row,
# m, W, Shat32: 16 B), plus Shat64 (8 B) with FP64 weights
IMPLEMENTED_DRAW_BYTES = {32: 28.0, 64: 36.0}


def algorithmic_bytes_per_transition(B, fp32: bool) -> float:
    """Bytes one transition must read by the scope table's definition, which is
    independent of the record layout: the state's header (row, m, W, Shat32:
    16 B; +8 B Shat64 in FP64 mode), the CDF words a binary search inspects
    ((ceil(log2 m) + 1) x 4 B) and the chosen target (4 B), averaged over the
    rows uniformly."""
    m = np.maximum(np.diff(B.row_ptr) - 1, 1)
    probes = np.ceil(np.log2(m)) + 1.0
    return float(np.mean((16.0 if fp32 else 24.0) + 4.0 * probes + 4.0))


def roofline_of(bpt, transitions, walk_s, prec, traffic, kernel, issue=None):
    achieved = bpt * transitions / walk_s / 1e9
    impl = IMPLEMENTED_DRAW_BYTES[prec] * transitions / walk_s / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernel,
            "bytes_per_transition": round(bpt, 2),
            "bytes_basis": "header 16 B + (ceil(log2 m)+1) x 4 B CDF probes + 4 B target"
                           + ("" if prec == 32 else " + 8 B Shat64"),
            "implemented_draw": {"bytes_per_transition": IMPLEMENTED_DRAW_BYTES[prec], "achieved": round(impl, 1),
                                 "frac": round(impl / HBM_PEAK_GBS, 4)},
            "walk_ms": round(walk_s * 1e3, 3), "walk_transitions_per_s": transitions / walk_s}
    if issue is not None:
        out["issue"] = issue
    return out


def gather_probe(units, reqs_per_step=1, steps=256, waves_per_cu=16, loads_per_req=1, mode=0):
    """Dependent random-gather ceiling (benchmark tooling, libmcmi_probe.so):
    (kernel ms, steps per second) of a chase over `units` random 64-byte units;
    mode 0: ordinary device memory, 1: non-temporal loads, 2: uncached memory."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2409_03095_amd", "bench_probe", "libmcmi_probe.so"))
    f = lib.probe_gather_chase_mode
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    ms, rate = ctypes.c_double(0.0), ctypes.c_double(0.0)
    st = f(units, reqs_per_step, loads_per_req, steps, waves_per_cu, mode, ctypes.byref(ms), ctypes.byref(rate))
    if st != 0:
        raise RuntimeError(f"probe_gather_chase_mode failed with status {st}")
    return ms.value, rate.value


def probe_main(args):
    """The dependent-gather ceiling by buffer size, load width and memory kind:
    one dependent random 64-byte unit per step, read as one 16-byte load or four,
    from ordinary memory, with non-temporal loads, or from uncached memory."""
    import torch
    torch.cuda.init()
    out = {"workload": "dependent random gather probe", "unit_bytes": 64, "waves_per_cu": 16, "results": []}
    for mb in (64, 512, 4096):
        units = mb * (1 << 20) // 64
        for mode, kind in ((0, "cached"), (1, "nontemporal"), (2, "uncached")):
            for loads in (1, 2, 4):
                ms, rate = gather_probe(units, 1, 128, 16, loads, mode)
                r = {"buffer_mb": mb, "memory": kind, "bytes_read_per_step": 16 * loads, "steps_per_s": rate,
                     "ms": ms}
                out["results"].append(r)
                print(f"[probe] {json.dumps(r)}", flush=True)
    print(json.dumps(out), flush=True)


def gpu_rows(res, rows):
    """The CSR rows `rows` (sorted) of a device result, on the host."""
    import torch
    rp_t, col_t, val_t = res.to_torch()
    torch.cuda.synchronize()
    rp = rp_t.cpu().numpy()
    lens = rp[rows + 1] - rp[rows]
    starts = rp[rows]
    sub_rp = np.concatenate([[0], np.cumsum(lens)])
    pos = np.repeat(starts - sub_rp[:-1], lens) + np.arange(sub_rp[-1])
    idx = torch.from_numpy(pos).cuda()
    return sub_rp, col_t[idx].cpu().numpy(), val_t[idx].cpu().numpy()


def compare_rows(n, a, b):
    """Pattern differences and relative value differences on the common
    pattern of two CSR row sets over the same rows."""
    (rpa, ca, va), (rpb, cb, vb) = a, b
    ka = np.repeat(np.arange(rpa.size - 1, dtype=np.int64), np.diff(rpa)) * n + ca
    kb = np.repeat(np.arange(rpb.size - 1, dtype=np.int64), np.diff(rpb)) * n + cb
    common, ia, ib = np.intersect1d(ka, kb, assume_unique=True, return_indices=True)
    rel = np.abs(va[ia] - vb[ib]) / np.abs(vb[ib])
    return {"entries_gpu": int(ka.size), "entries_oracle": int(kb.size),
            "pattern_differences": int(ka.size + kb.size - 2 * common.size),
            "max_rel_err": float(rel.max()) if rel.size else 0.0,
            "median_rel_err": float(np.median(rel)) if rel.size else 0.0,
            "entries_beyond_1e-5_rel": int(np.sum(rel > 1e-5))}, (ka, kb, ia, ib)


def fp32_weight_bound(n, g, r64, keys, o, rows, chains, eps, delta, rerun):
    """FP32 walks follow the FP64 walks' paths: a step-j weight differs by at most
    2 j u32 |W_j| (j binary32 products with Shat rounded to binary32), and a chain
    whose cutoff test falls inside that band (the oracle counts them per row, D_r)
    may add or miss one contribution of magnitude at most delta. So a value may
    differ from the FP64 oracle's by B32 = ((2 L u32 (1 + 2^-10) + 4 (k + 2) u64)
    sum|W| + D_r delta (1 + 2^-10)) / (N |d_c|). Returns the largest error /
    max(1e-5 |v64|, B32) over the common entries (<= 1: within the bound) and, for
    entries kept by one side only, the largest distance of |N64| from eps in units
    of that band (<= 1: a kept/dropped decision made by rounding), read from the
    oracle's eps = 0 run of those rows."""
    u32, u64 = 2.0 ** -24, 2.0 ** -53
    ka, kb, ia, ib = keys
    L = int(r64["lmax"])
    wb = 2.0 * L * u32 * (1.0 + 2.0 ** -10)
    D = r64["row_border"].astype(np.float64)
    loc = kb[ib] // n
    dc = np.abs(o.diag[r64["col"][ib]])
    b32 = ((wb + 4.0 * (r64["cnt"][ib] + 2.0) * u64) * r64["abssum"][ib] + D[loc] * delta * (1.0 + 2.0 ** -10)) \
        / chains / dc
    v64 = r64["val"][ib]
    ratio = np.abs(g[2][ia] - v64) / np.maximum(1e-5 * np.abs(v64), b32)
    out = {"max_err_over_bound": float(ratio.max()) if ratio.size else 0.0, "chains_near_cutoff": int(D.sum())}
    only = np.setxor1d(ka, kb, assume_unique=True)
    if only.size:
        local = np.unique(only // n)
        full = rerun(rows[local])
        kf = np.repeat(np.arange(local.size, dtype=np.int64), np.diff(full["row_ptr"])) * n + full["col"]
        want = np.searchsorted(local, only // n) * n + only % n
        pos = np.minimum(np.searchsorted(kf, want), kf.size - 1)
        found = kf[pos] == want
        nh = np.where(found, np.abs(full["val"][pos] * o.diag[only % n]), 0.0)
        ab = np.where(found, full["abssum"][pos], 0.0)
        k = np.where(found, full["cnt"][pos], 0.0)
        band = ((wb + 4.0 * (k + 2.0) * u64) * ab + D[only // n] * delta * (1.0 + 2.0 ** -10)) / chains \
            + 4.0 * u64 * eps
        out["pattern_difference_max_distance_over_band"] = float((np.abs(nh - eps) / band).max())
    return out


def cpu_baseline(B, chains, delta, eps, res, gpu_prec, budget_s=20.0, check_rows=4096):
    """The oracle as it is (FP64 walks, long-double sums), on the host's cores,
    on a bounded uniform sample of rows; one thread on the first rows of that
    sample. The same leg then compares the GPU's result `res` on the sampled
    rows with the oracle's (error against the FP64 oracle) and, for FP32 walks,
    with the oracle's FP32-weight mode on the first `check_rows` of them (same
    pattern, same values up to summation order)."""
    import oracle as O
    threads = O.default_threads()
    o = O.Oracle(B)
    rng = np.random.default_rng(123)
    probe = np.sort(rng.choice(B.n, 256, replace=False)).astype(np.int32)
    t0 = time.perf_counter()
    r = o.spai(seed=0, chains=chains, delta=delta, eps=eps, rows=probe, threads=threads)
    dt = time.perf_counter() - t0
    rate = r["transitions"] / max(dt, 1e-9)
    nrows = int(min(B.n, max(check_rows, rate * budget_s / max(r["transitions"] / 256, 1))))
    rows = np.sort(rng.choice(B.n, nrows, replace=False)).astype(np.int32)
    t0 = time.perf_counter()
    r = o.spai(seed=0, chains=chains, delta=delta, eps=eps, rows=rows, threads=threads)
    dt = time.perf_counter() - t0
    n1 = int(min(nrows, max(64, nrows * 0.2 / max(threads, 1))))
    t1 = time.perf_counter()
    r1 = o.spai(seed=0, chains=chains, delta=delta, eps=eps, rows=rows[:n1], threads=1)
    dt1 = time.perf_counter() - t1
    base = {"value": r["transitions"] / dt, "unit": "transitions/s", "cores": threads, "kind": "oracle",
            "sample": f"{nrows} uniformly sampled rows of the same matrix, FP64 walks ({r['transitions']} "
                      f"transitions, {dt:.1f} s, {threads} threads)",
            "single_core_value": r1["transitions"] / dt1,
            "single_core_sample": f"the first {n1} of those rows on one thread ({r1['transitions']} transitions, "
                                  f"{dt1:.1f} s)"}
    g = gpu_rows(res, rows)
    cmp, keys = compare_rows(B.n, g, (r["row_ptr"], r["col"], r["val"]))
    prec = {"vs": "FP64 oracle", "rows": nrows, "guard_band_entries": int(r["guard"]), **cmp}
    if gpu_prec == 32:
        prec["fp32_bound"] = fp32_weight_bound(
            B.n, g, r, keys, o, rows, chains, eps, delta,
            lambda rr: o.spai(seed=0, chains=chains, delta=delta, eps=0.0, rows=rr, threads=threads))
        sub = rows[:check_rows]
        r32 = o.spai(seed=0, chains=chains, delta=delta, eps=eps, fp32=True, rows=sub, threads=threads)
        k = int(g[0][sub.size])
        c, _ = compare_rows(B.n, (g[0][:sub.size + 1], g[1][:k], g[2][:k]), (r32["row_ptr"], r32["col"], r32["val"]))
        prec["fp32_mode"] = {"rows": int(sub.size), "pattern_differences": c["pattern_differences"],
                             "max_rel_diff": c["max_rel_err"]}
    return base, prec


def timed_steps(step, steps, warmup):
    """W untimed steps, then K steps between device synchronisations."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    walk_ms, trans, last = [], [], None
    t0 = time.perf_counter()
    for _ in range(steps):
        last = step()
        walk_ms.append(last.stats.ms_walk)
        trans.append(last.stats.transitions)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, walk_ms, trans, last


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=262144, help="rows of the random workload")
    ap.add_argument("--chains", type=int, default=0, help="chains per row (0: the workload's default)")
    ap.add_argument("--prec", type=int, default=32, choices=[32, 64])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline and the precision check")
    ap.add_argument("--no-secondary", action="store_true", help="aniso27: skip the random-workload line")
    ap.add_argument("--hash-slots", type=int, default=0)
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--sketch-slots", type=int, default=0)
    ap.add_argument("--heavy-weight", type=float, default=0.0)
    ap.add_argument("--workload", default="aniso27", choices=["random", "aniso27", "batched", "next", "probe"],
                    help="aniso27: 160^3 27-point anisotropic (default); random: n=262144 random nonsymmetric; "
                         "batched: 256 3D 7-point convection-diffusion matrices in one launch")
    ap.add_argument("--nx", type=int, default=160, help="grid side of the aniso27 workload")
    ap.add_argument("--order-cell", type=int, default=None,
                    help="row schedule cells (rows per cell; 0 = natural order). Default: 4096 for aniso27, else 0")
    ap.add_argument("--learned-alloc", action="store_true",
                    help="aniso27: chains per row from the allocation network (trained on small 27-point "
                         "matrices), same mean budget, uniform fallback; features, inference and allocation "
                         "are inside the timed step")
    ap.add_argument("--tune", action="store_true", help="batched: kernel shape from the autotuner")
    ap.add_argument("--graph", action="store_true",
                    help="batched: also time hipGraph replays of the launch on the last step's records")
    ap.add_argument("--bicgstab", action="store_true", help="aniso27: device BiCGstab iterations with and without M")
    ap.add_argument("--learned", action="store_true",
                    help="learned vs uniform chains to ||I-MB||_F/sqrt(n) <= 0.3 (allocation-network workload)")
    ap.add_argument("--train-mats", type=int, default=2000)
    ap.add_argument("--heldout", type=int, default=1024, help="held-out grid side (n = side^2)")
    ap.add_argument("--train-steps", type=int, default=3000)
    ap.add_argument("--probe", action="store_true", help="random: also run the dependent-gather ceiling probe")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run one plain 1 GiB device copy (the reference of rocprofv3's byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the Monte Carlo rows would shard across GPUs without communication, "
              "but the benchmark runs and reports a single MI355X only.", file=sys.stderr)
        sys.exit(2)

    if args.calib_copy:
        import torch
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.learned:
        return learned_main(args)
    if args.workload == "next":
        return next_main(args)
    if args.workload == "probe":
        return probe_main(args)
    if args.workload == "batched":
        return batched_main(args)
    if args.workload == "random":
        out = random_line(args, args.steps, args.warmup, budget_s=20.0)
        print(json.dumps(out), flush=True)
        return
    out = aniso_main(args)
    if not args.no_secondary and not args.learned_alloc and not args.bicgstab:
        sec = random_line(args, args.steps, args.warmup, budget_s=8.0)
        out["secondary"] = {"random_nonsym_n262144": {k: sec[k] for k in (
            "value", "unit", "ms_per_step", "dtype", "config", "roofline", "cpu_baseline", "precision") if k in sec}}
    print(json.dumps(out), flush=True)


def random_line(args, steps, warmup, budget_s):
    """Random nonsymmetric n = 262144 (5..30 off-diagonals per row, ||C||_inf
    = 0.7 in every row), 512 chains, delta = 1e-4, eps = 1e-3: every chain
    makes exactly 25 transitions."""
    import torch

    from paper_2409_03095_amd import inputs as I
    from paper_2409_03095_amd import mcmi
    delta, eps, seed = 1e-4, 1e-3, 0
    chains = args.chains or 512
    t0 = time.perf_counter()
    B = I.cfg2(args.n)
    print(f"[random] generated n={B.n} nnz={B.nnz} in {time.perf_counter() - t0:.1f} s", flush=True)
    dB = mcmi.DeviceCsr.from_host(B)
    x = torch.ones(B.n, dtype=torch.float64, device="cuda")
    y = torch.empty(B.n, dtype=torch.float64, device="cuda")
    p = mcmi.params(seed=seed, chains=chains, delta=delta, eps=eps, walk_prec=args.prec,
                    hash_slots=args.hash_slots, lanes_per_row=args.lanes, sketch_slots=args.sketch_slots,
                    heavy_weight=args.heavy_weight)
    cell = args.order_cell or 0

    def step():
        cdf = mcmi.Cdf(dB, order_cell=cell)
        res = mcmi.spai(cdf, p)
        res.apply(x, y)
        return res

    elapsed, walk_ms, trans, last = timed_steps(step, steps, warmup)
    st = last.stats
    print(f"[random] {steps} steps in {elapsed:.3f} s, walk {np.mean(walk_ms):.2f} ms", flush=True)
    walk_s = float(np.mean(walk_ms)) / 1e3
    bpt = algorithmic_bytes_per_transition(B, args.prec == 32)
    # the counters were taken on the default configuration only
    measured = (args.n == 262144 and args.prec == 32 and chains == 512 and not cell and not args.hash_slots
                and not args.lanes and not args.sketch_slots and args.heavy_weight == 0.0)
    roofline = roofline_of(bpt, trans[-1], walk_s, args.prec, TRAFFIC_BYTES["random"] if measured else None,
                           "k_walk_block")
    if args.probe:
        # memory ceiling of the access pattern: a chase over a buffer of the
        # record set's size with one dependent random 64-byte block per step
        cdf0 = mcmi.Cdf(dB)
        probe = {f"wpc{w}": gather_probe(max(1024, cdf0.rec_units), 1, 256, w, 1)[1] for w in (8, 16, 32)}
        roofline["gather_probe_steps_per_s"] = probe
        del cdf0
    out = {"metric": METRIC, "value": float(sum(trans)) / elapsed, "unit": "transitions/s", "n_gpus": 1,
           "steps": steps, "warmup": warmup, "ms_per_step": elapsed / steps * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32" if args.prec == 32 else "f64", "data": "synthetic",
           "config": {"workload": f"random nonsymmetric n={B.n}, 5-30 off-diagonals/row, ||C||_inf=0.7, "
                                  f"{chains} chains/row, delta=1e-4, eps=1e-3, FP{args.prec} walks + FP64 sums",
                      "n": B.n, "nnz_B": B.nnz, "chains_per_row": chains, "transitions_per_step": trans[-1],
                      "nnz_M": last.nnz, "spilled_contributions": st.spilled, "retries": st.retries,
                      "lanes_per_row": st.lanes_per_row, "hash_slots": st.hash_slots,
                      "sketch_slots": st.sketch_slots, "heavy_weight": st.heavy_weight,
                      "rows_replayed": st.refined, "order_cell": cell},
           "roofline": roofline}
    if not args.no_cpu:
        out["cpu_baseline"], out["precision"] = cpu_baseline(B, chains, delta, eps, last, args.prec, budget_s)
        print(f"[random] precision {json.dumps(out['precision'])}", flush=True)
    return out


def aniso_main(args):
    """3D 27-point anisotropic diffusion (1:10:100, +-10 % noise, ||C||_inf = 0.75) on
    an nx^3 grid, 64 chains/row, FP32 walks + FP64 sums, delta = 1e-4, eps = 1e-3."""
    import torch

    from paper_2409_03095_amd import inputs as I
    from paper_2409_03095_amd import mcmi
    t0 = time.perf_counter()
    B = I.cfg5(args.nx)
    print(f"[aniso27] generated n={B.n} nnz={B.nnz} in {time.perf_counter() - t0:.1f} s", flush=True)
    dB = mcmi.DeviceCsr.from_host(B)
    chains = args.chains or 64
    delta, eps = 1e-4, 1e-3
    p = mcmi.params(seed=0, chains=chains, delta=delta, eps=eps, walk_prec=args.prec, lanes_per_row=args.lanes,
                    hash_slots=args.hash_slots, sketch_slots=args.sketch_slots, heavy_weight=args.heavy_weight)
    x = torch.ones(B.n, dtype=torch.float64, device="cuda")
    y = torch.empty(B.n, dtype=torch.float64, device="cuda")
    cell = 4096 if args.order_cell is None else args.order_cell
    net, alloc = None, None
    if args.learned_alloc:
        from paper_2409_03095_amd import learned as L
        rng = np.random.default_rng(77)
        train = [I.aniso27(int(rng.integers(12, 21)), seed=1000 + k) for k in range(40)]
        net, tinfo = L.train_allocator(train, delta, steps=3000)
        alloc = {"train": tinfo}
        print(f"[aniso27] allocation network trained: {json.dumps(tinfo)}", flush=True)

    def chains_for(cdf):
        # learned allocation: features -> network -> chains per row for the same
        # mean budget (chain cost 1 + floor(f7), mcmi_chain_cost), uniform fallback inside mcmi_allocate
        if net is None:
            return None
        feat = mcmi.row_features(cdf, delta)
        pred = net.predict(feat)
        cost, total_cost = mcmi.chain_cost(feat)
        cpr, lam, fb = mcmi.allocate(pred, cost, int(chains * total_cost))
        alloc.update({"lambda": lam, "fallback": fb})
        return cpr

    rec = {}

    def step():
        cdf = mcmi.Cdf(dB, order_cell=cell)
        res = mcmi.spai(cdf, p, chains_per_row=chains_for(cdf))
        res.apply(x, y)
        rec["units"] = cdf.rec_units
        return res

    elapsed, walk_ms, trans, last = timed_steps(step, args.steps, args.warmup)
    st = last.stats
    print(f"[aniso27] {args.steps} steps in {elapsed:.3f} s, walk {np.mean(walk_ms):.2f} ms", flush=True)
    walk_s = float(np.mean(walk_ms)) / 1e3
    bpt = algorithmic_bytes_per_transition(B, args.prec == 32)
    traffic = TRAFFIC_BYTES["aniso27"] if (args.nx == 160 and args.prec == 32 and cell == 4096 and net is None
                                           and chains == 64 and not args.lanes and not args.hash_slots) else None
    out = {"metric": METRIC, "value": float(sum(trans)) / elapsed, "unit": "transitions/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32" if args.prec == 32 else "f64", "data": "synthetic",
           "config": {"workload": f"3D 27-point anisotropic diffusion {args.nx}^3 (1:10:100, +-10% noise, "
                                  f"||C||_inf=0.75), {chains} chains/row"
                                  f"{' (learned allocation, same mean)' if net is not None else ''}, delta=1e-4, "
                                  f"eps=1e-3, FP{args.prec} walks + FP64 sums",
                      "n": B.n, "nnz_B": B.nnz,
                      "chains_per_row": chains, "transitions_per_step": int(st.transitions), "nnz_M": int(last.nnz),
                      "lanes_per_row": st.lanes_per_row, "hash_slots": st.hash_slots, "spilled": int(st.spilled),
                      "retries": int(st.retries), "record_bytes": int(rec["units"]) * (32 if args.prec == 32 else 64),
                      "order_cell": cell},
           "roofline": roofline_of(bpt, st.transitions, walk_s, args.prec, traffic, "k_walk",
                                   ISSUE["aniso27"] if traffic is not None else None)}
    if net is not None:
        # quality at the same budget: learned vs uniform chains, 10^4-row sample
        cdf = mcmi.Cdf(dB, order_cell=cell)
        cpr = chains_for(cdf)
        rows = np.sort(np.random.default_rng(12345).choice(B.n, 10000, replace=False))
        ql = L.evaluate(B, cpr, delta, eps, 0, rows, args.prec, cdf)
        qu = L.evaluate(B, torch.full((B.n,), chains, dtype=torch.int32, device="cuda"), delta, eps, 0, rows,
                        args.prec, cdf)
        cq = np.percentile(cpr.cpu().numpy(), [10, 50, 90])
        alloc.update({"chains_min": int(cpr.min().item()), "chains_max": int(cpr.max().item()),
                      "chains_p10_p50_p90": [float(v) for v in cq],
                      "rows_over_64_chains": float((cpr > 64).float().mean().item()),
                      "learned": ql, "uniform": qu})
        out["config"]["allocation"] = "learned"
        out["learned_allocation"] = alloc
        print(f"[aniso27] learned r={ql['r_norm']:.4f} T={ql['transitions']} | uniform r={qu['r_norm']:.4f} "
              f"T={qu['transitions']}", flush=True)
        del cdf
    elif not args.no_cpu:
        out["cpu_baseline"], out["precision"] = cpu_baseline(B, chains, delta, eps, last, args.prec, 20.0)
        print(f"[aniso27] precision {json.dumps(out['precision'])}", flush=True)
    if args.bicgstab:
        # device BiCGstab (b = B 1, x0 = 0, rtol 1e-8): no preconditioner vs M
        Bs_ones = torch.from_numpy(B.to_scipy() @ np.ones(B.n)).cuda()
        res_it = {}
        for name, M in (("none", None), ("mcmi", last)):
            _, st_s = mcmi.bicgstab(dB, M, Bs_ones, rtol=1e-8, maxiter=5000)
            res_it[name] = {"iterations": int(st_s.iterations), "converged": int(st_s.converged),
                            "rel_residual": st_s.rel_residual, "solve_ms": st_s.ms}
            print(f"[aniso27] bicgstab {name}: {res_it[name]}", flush=True)
        res_it["mcmi"]["preconditioner_plus_solve_ms"] = elapsed / args.steps * 1e3 + res_it["mcmi"]["solve_ms"]
        out["bicgstab"] = res_it
    return out


def batched_main(args):
    """256 3D 7-point convection-diffusion matrices (n log-uniform in [1e3, 1e5],
    Peclet U[0, 5], ||C||_inf U[0.5, 0.85]; seed 3) in one batched launch: 128
    chains/row, delta = 1e-4, eps = 1e-3. Also times the same matrices one launch
    each (records built once) for comparison."""
    import torch

    from paper_2409_03095_amd import inputs as I
    from paper_2409_03095_amd import mcmi
    t0 = time.perf_counter()
    mats, _ = I.convdiff_batch(256, seed=3)
    print(f"[batched] generated {len(mats)} matrices, {sum(m.n for m in mats)} rows in "
          f"{time.perf_counter() - t0:.1f} s", flush=True)
    devs = [mcmi.DeviceCsr.from_host(B) for B in mats]
    chains = args.chains or 128
    p = mcmi.params(seed=0, chains=chains, delta=1e-4, eps=1e-3, walk_prec=args.prec, lanes_per_row=args.lanes,
                    hash_slots=args.hash_slots)
    cell = 0 if args.order_cell is None else args.order_cell
    tuned = None
    if args.tune:
        # the autotuner times candidate kernel shapes on a row sample of the set (outside
        # the timed steps; cached in a JSON file in the temporary directory)
        import tempfile
        t0 = time.perf_counter()
        p, tms = mcmi.tune(mcmi.Cdf.batched(devs, order_cell=cell), p, sample_rows=65536,
                           cache_path=os.path.join(tempfile.gettempdir(), "mcmi_tune_batched.json"))
        tuned = {"lanes_per_row": p.lanes_per_row, "hash_slots": p.hash_slots, "sketch_slots": p.sketch_slots,
                 "sample_walk_ms": tms, "tuning_s": time.perf_counter() - t0}
        print(f"[batched] tuned: {json.dumps(tuned)}", flush=True)
    for _ in range(args.warmup):
        res = mcmi.spai(mcmi.Cdf.batched(devs, order_cell=cell), p)
        del res
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    walk_ms, trans = [], 0
    for _ in range(args.steps):
        cdf = mcmi.Cdf.batched(devs, order_cell=cell)
        res = mcmi.spai(cdf, p)
        walk_ms.append(res.stats.ms_walk)
        trans += res.stats.transitions
        last = res
        cdf_last = cdf
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # one launch per matrix (records built once per matrix), same chains and seed
    cdfs = [mcmi.Cdf(d) for d in devs]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    single_trans = 0
    for i, c in enumerate(cdfs):
        r = mcmi.spai(c, mcmi.params(seed=0, chains=chains, delta=1e-4, eps=1e-3, walk_prec=args.prec, tag=i))
        single_trans += r.stats.transitions
    torch.cuda.synchronize()
    single_s = time.perf_counter() - t1
    st = last.stats
    # the same launch captured in a hipGraph plan on the last step's records: each
    # replay (new seed) resets the counters, walks, finalizes and assembles M
    graph = None
    if args.graph:
        plan = mcmi.Plan(cdf_last, p, nnz_capacity=int(last.nnz * 1.25) + (1 << 20))
        plan.launch(1000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            plan.launch(1001 + k)
        torch.cuda.synchronize()
        g_s = (time.perf_counter() - t0) / args.steps
        gst, ovf, gnnz = plan.stats()
        graph = {"ms_per_replay": g_s * 1e3, "transitions_per_replay": int(gst.transitions),
                 "transitions_per_s": gst.transitions / g_s, "overflow": ovf, "nnz_M": gnnz}
        print(f"[batched] graph replays: {json.dumps(graph)}", flush=True)
        del plan
    # algorithmic bytes per transition, the mean over all rows of the set
    nrow = np.array([m.n for m in mats], dtype=np.float64)
    bpt = float(np.dot(nrow, [algorithmic_bytes_per_transition(m, args.prec == 32) for m in mats]) / nrow.sum())
    walk_s = float(np.mean(walk_ms)) / 1e3
    traffic = TRAFFIC_BYTES["batched"] if (args.prec == 32 and chains == 128 and cell == 0 and not args.tune
                                           and not args.lanes and not args.hash_slots) else None
    roofline = roofline_of(bpt, st.transitions, walk_s, args.prec, traffic, "k_walk")
    out = {"metric": METRIC, "value": trans / elapsed, "unit": "transitions/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
           "dtype": "f32" if args.prec == 32 else "f64", "data": "synthetic",
           "config": {"workload": "batched 256 x 3D 7-point convection-diffusion", "matrices": len(mats),
                      "rows": int(sum(m.n for m in mats)), "chains_per_row": chains,
                      "transitions_per_step": int(st.transitions), "nnz_M": int(last.nnz),
                      "lanes_per_row": st.lanes_per_row, "hash_slots": st.hash_slots, "order_cell": cell,
                      "tuned": tuned},
           "walk_ms": float(np.mean(walk_ms)), "roofline": roofline, "graph_replay": graph,
           "one_launch_per_matrix": {"seconds": single_s, "transitions": int(single_trans),
                                     "transitions_per_s": single_trans / single_s}}
    print(json.dumps(out), flush=True)


def learned_main(args):
    """Allocation-network workload: train on the 5-point family with pilot-run
    variance, then time-to-quality of learned vs uniform chains on a held-out
    instance (delta = eps = 1e-3, FP64 walks)."""
    from paper_2409_03095_amd import inputs as I
    from paper_2409_03095_amd import learned as L
    delta, eps = 1e-3, 1e-3
    t0 = time.perf_counter()
    mats = I.cfg4_train(args.train_mats)
    print(f"[learned] generated {len(mats)} training matrices in {time.perf_counter() - t0:.1f} s", flush=True)
    net, info = L.train_allocator(mats, delta, steps=args.train_steps)
    print(f"[learned] trained: {json.dumps(info)}", flush=True)
    B = I.cfg4_heldout(args.heldout)
    budgets = [2, 3, 4, 6, 8, 12, 16, 24, 32]
    pts = L.compare(net, B, delta, eps, budgets)
    for p in pts:
        print(f"[learned] budget {p['mean_chains']}: learned r={p['learned']['r_norm']:.4f} "
              f"T={p['learned']['transitions']} | uniform r={p['uniform']['r_norm']:.4f} "
              f"T={p['uniform']['transitions']}", flush=True)
    lt = L.crossing([p["learned"] for p in pts], "transitions")
    ut = L.crossing([p["uniform"] for p in pts], "transitions")
    ls = L.crossing([p["learned"] for p in pts], "wall_s")
    us = L.crossing([p["uniform"] for p in pts], "wall_s")
    # control: a family whose rows differ in path variance at equal cost (a
    # deterministic-path cycle block next to random rows), where the best
    # allocation is far from uniform
    cmats = [I.cycle_plus_random(1000 + s) for s in range(40)]
    cnet, cinfo = L.train_allocator(cmats, delta, steps=args.train_steps)
    CB = I.cycle_plus_random(99, scale=200)
    cpts = L.compare(cnet, CB, delta, eps, [1, 2, 4, 8, 16])
    for p in cpts:
        print(f"[learned] control budget {p['mean_chains']}: learned r={p['learned']['r_norm']:.4f} "
              f"| uniform r={p['uniform']['r_norm']:.4f} at T={p['uniform']['transitions']}", flush=True)
    control = {"workload": f"cycle + random blocks, 40 training matrices, held-out n={CB.n}", "train": cinfo,
               "learned_transitions_to_0.3": L.crossing([p["learned"] for p in cpts], "transitions"),
               "uniform_transitions_to_0.3": L.crossing([p["uniform"] for p in cpts], "transitions"),
               "points": cpts}
    out = {"metric": METRIC, "value": lt, "unit": "transitions to ||I-MB||_F/sqrt(n) <= 0.3 (learned)",
           "uniform_value": ut, "learned_seconds": ls, "uniform_seconds": us,
           "higher_is_better": False, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"5-point family with smooth rho field: {args.train_mats} training matrices, "
                                  f"held-out {args.heldout}x{args.heldout}", "n": B.n, "train": info},
           "points": pts, "control": control}
    print(json.dumps(out), flush=True)


def next_main(args):
    """The pre-pass and output variants on a 64^3 27-point anisotropic matrix
    (1:10:100, +-10 % noise, ||C||_inf = 0.95; 32 chains/row, delta = eps = 1e-3, FP32
    walks): matrix reduction (drop shares 0-10 %), top-k retention (k = 16, 32 vs the
    eps filter), and the augmented splitting on the same stencil made non-contractive
    (||C||_inf = 1.3, alpha = 1, 2, 5). Per setting: walk time, transitions, nnz(M),
    ||I - MB||_F / sqrt(n) on a 10^4-row sample and device BiCGstab iterations on
    B x = B 1 (rtol 1e-8) with M on the right."""
    import torch

    from paper_2409_03095_amd import inputs as I
    from paper_2409_03095_amd import learned as L
    from paper_2409_03095_amd import mcmi
    nx = 64
    rows = np.sort(np.random.default_rng(12345).choice(nx ** 3, 10000, replace=False))

    def measure(B, dB, cdf_kw, p_kw, label):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cdf = mcmi.Cdf(dB, **cdf_kw)
        p = mcmi.params(seed=0, chains=32, delta=1e-3, eps=1e-3, walk_prec=32, **p_kw)
        res = mcmi.spai(cdf, p)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        sq = L.residual_sample(B, *L.sample_rows(res, rows), rows)
        b = torch.from_numpy(B.to_scipy() @ np.ones(B.n)).cuda()
        _, sn = mcmi.bicgstab(dB, None, b, rtol=1e-8, maxiter=5000)
        _, sm = mcmi.bicgstab(dB, res, b, rtol=1e-8, maxiter=5000)
        out = {"setting": label, "walk_ms": res.stats.ms_walk, "transitions": int(res.stats.transitions),
               "transitions_per_s": res.stats.transitions / (res.stats.ms_walk * 1e-3), "nnz_M": int(res.nnz),
               "r_norm": float(math.sqrt(sq.mean())), "build_and_walk_ms": build_s * 1e3,
               "bicgstab_none": {"iterations": int(sn.iterations), "converged": int(sn.converged), "ms": sn.ms},
               "bicgstab_M": {"iterations": int(sm.iterations), "converged": int(sm.converged), "ms": sm.ms}}
        print(f"[next] {label}: walk {out['walk_ms']:.2f} ms, nnz(M) {out['nnz_M']}, r {out['r_norm']:.4f}, "
              f"BiCGstab {sn.iterations} -> {sm.iterations} iterations", flush=True)
        return out

    B = I.aniso27(nx, rho=0.95, seed=5)
    dB = mcmi.DeviceCsr.from_host(B)
    results = {"reduction": [], "topk": [], "augmentation": []}
    for frac in (0.0, 0.02, 0.06, 0.10):
        results["reduction"].append(measure(B, dB, {"drop_frac": frac}, {}, f"drop {frac:.2f}"))
    for k in (16, 32):
        results["topk"].append(measure(B, dB, {}, {"topk": k}, f"top-{k}"))
    Bn = I.aniso27(nx, rho=1.3, seed=5)
    dBn = mcmi.DeviceCsr.from_host(Bn)
    for alpha in (1.0, 2.0, 5.0):
        results["augmentation"].append(measure(Bn, dBn, {"alpha": alpha}, {}, f"alpha {alpha:g} (||C||_inf 1.3)"))
    out = {"metric": METRIC, "workload": f"pre-pass and output variants, 27-point {nx}^3", "n": B.n,
           "data": "synthetic", "n_gpus": 1, "results": results}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
