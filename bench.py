"""Benchmark: Monte Carlo SPAI throughput (transitions/s) on one MI355X.

Workload (default): random nonsymmetric B, n = 262144, 5..30 off-diagonals per
row at uniform columns, log-normal magnitudes with random signs, per-row
diagonal so that every row of C = I - D^-1 B has |C| row sum 0.7; 512 chains
per row, FP32 walk weights with FP64 sums, delta = 1e-4, eps = 1e-3, Philox
seed 0. Every chain makes exactly 25 transitions, so one step is exactly
262144 * 512 * 25 = 3,355,443,200 transitions.

One step = the whole hot path over the matrix, through the C ABI:
mcmi_build_cdf (records) + mcmi_spai (walks, accumulation, filter, scaling,
CSR assembly) + mcmi_apply (one y = M x). Inputs are resident in HBM before the
timed region starts.

Prints one JSON line with, beside the throughput, the roofline of the walk
kernel (algorithmic bytes per transition x transitions per launch / the walk
kernel's event-timed duration, against 8 TB/s HBM) and the CPU oracle's rate on
a bounded row sample.
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
# rocprofv3 FETCH_SIZE/WRITE_SIZE of the walk kernel, in bytes per launch, for
# the default workload (None until measured for the current kernel)
TRAFFIC_BYTES = 3.94e11  # calibrated FETCH_SIZE + WRITE_SIZE of one walk launch (rocprofv3 --pmc)
# the same for the 160^3 27-point workload's wavefront walk (cells of 4096 rows, FP32)
TRAFFIC_BYTES_ANISO27 = 5.50e11
# and for the batched launch of the 256 convection-diffusion matrices (128 chains, FP32)
TRAFFIC_BYTES_BATCHED = 9.93e11


def algorithmic_bytes_per_transition(B, fp32: bool) -> float:
    """Bytes one transition must read, independent of the record layout: the
    state's header (row, m, W, Shat32: 16 B; +8 B Shat64 in FP64 mode), the CDF
    words a binary search inspects ((ceil(log2 m) + 1) x 4 B) and the chosen
    target (4 B). For this workload the next state is a uniformly random column,
    so the mean is taken over rows uniformly."""
    m = np.maximum(np.diff(B.row_ptr) - 1, 1)
    probes = np.ceil(np.log2(m)) + 1.0
    return float(np.mean((16.0 if fp32 else 24.0) + 4.0 * probes + 4.0))


def cpu_baseline(B, chains, delta, eps, fp32, budget_s=20.0):
    """The oracle as it is, on the host cores, on a bounded sample of rows."""
    import oracle as O
    threads = O.default_threads()
    o = O.Oracle(B)
    rng = np.random.default_rng(123)
    probe = rng.choice(B.n, 256, replace=False).astype(np.int32)
    t0 = time.perf_counter()
    r = o.spai(seed=0, chains=chains, delta=delta, eps=eps, fp32=fp32, rows=probe, threads=threads)
    dt = time.perf_counter() - t0
    rate = r["transitions"] / max(dt, 1e-9)
    nrows = int(min(B.n, max(256, rate * budget_s / max(r["transitions"] / 256, 1))))
    rows = rng.choice(B.n, nrows, replace=False).astype(np.int32)
    t0 = time.perf_counter()
    r = o.spai(seed=0, chains=chains, delta=delta, eps=eps, fp32=fp32, rows=rows, threads=threads)
    dt = time.perf_counter() - t0
    # one thread on a sample of about a fifth of the all-core run's time
    n1 = int(min(nrows, max(64, nrows * 0.2 / max(threads, 1))))
    t1 = time.perf_counter()
    r1 = o.spai(seed=0, chains=chains, delta=delta, eps=eps, fp32=fp32, rows=rows[:n1], threads=1)
    dt1 = time.perf_counter() - t1
    return {"value": r["transitions"] / dt, "unit": "transitions/s", "cores": threads, "kind": "oracle",
            "sample": f"{nrows} uniformly sampled rows of the same matrix ({r['transitions']} transitions, "
                      f"{dt:.1f} s, {threads} threads)",
            "single_core_value": r1["transitions"] / dt1,
            "single_core_sample": f"the first {n1} of those rows on one thread ({r1['transitions']} transitions, "
                                  f"{dt1:.1f} s)"}


def walk_precision(mcmi, dB, n, chains, delta, eps, seed, nrows=4096):
    """FP32 walks against FP64 walks on the same sampled rows, after the timed
    steps: the FP64 path is the one the parity tests hold to the FP64 oracle at
    1e-12, so this is the FP32 path's error against FP64 arithmetic."""
    import torch
    rows = np.sort(np.random.default_rng(7).choice(n, min(n, nrows), replace=False)).astype(np.int32)
    rows_t = torch.from_numpy(rows).cuda()
    cdf = mcmi.Cdf(dB)
    keys, vals = {}, {}
    for prec in (64, 32):
        p = mcmi.params(seed=seed, chains=chains, delta=delta, eps=eps, walk_prec=prec)
        rp, col, val = mcmi.spai(cdf, p, rows=rows_t).to_numpy()
        keys[prec] = np.repeat(rows.astype(np.int64), np.diff(rp)) * n + col
        vals[prec] = val
    common, i64, i32 = np.intersect1d(keys[64], keys[32], assume_unique=True, return_indices=True)
    v64, v32 = vals[64][i64], vals[32][i32]
    rel = np.abs(v32 - v64) / np.abs(v64)
    return {"rows": int(rows.size), "entries_f64": int(keys[64].size), "entries_f32": int(keys[32].size),
            "pattern_differences": int(keys[64].size + keys[32].size - 2 * common.size),
            "max_rel_diff_f32_vs_f64": float(rel.max()) if rel.size else 0.0,
            "median_rel_diff_f32_vs_f64": float(np.median(rel)) if rel.size else 0.0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=262144)
    ap.add_argument("--chains", type=int, default=512)
    ap.add_argument("--prec", type=int, default=32, choices=[32, 64])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--hash-slots", type=int, default=0)
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--sketch-slots", type=int, default=0)
    ap.add_argument("--heavy-weight", type=float, default=0.0)
    ap.add_argument("--workload", default="random", choices=["random", "aniso27", "batched", "next"],
                    help="random: n=262144 random nonsymmetric (default); aniso27: 160^3 27-point anisotropic; "
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
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run one plain 1 GiB device copy (reference for rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the Monte Carlo rows would shard across GPUs without communication, "
              "but the benchmark runs and reports a single MI355X only.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2409_03095_amd import inputs as I
    from paper_2409_03095_amd import mcmi

    if args.learned:
        return learned_main(args)

    delta, eps, seed = 1e-4, 1e-3, 0
    if args.workload == "next":
        return next_main(args)
    if args.workload == "aniso27":
        return aniso_main(args)
    if args.workload == "batched":
        return batched_main(args)
    B = I.cfg2(args.n)
    dB = mcmi.DeviceCsr.from_host(B)
    x = torch.ones(B.n, dtype=torch.float64, device="cuda")
    y = torch.empty(B.n, dtype=torch.float64, device="cuda")
    p = mcmi.params(seed=seed, chains=args.chains, delta=delta, eps=eps, walk_prec=args.prec,
                    hash_slots=args.hash_slots, lanes_per_row=args.lanes, sketch_slots=args.sketch_slots,
                    heavy_weight=args.heavy_weight)
    torch.cuda.synchronize()
    if args.calib_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    cell = args.order_cell or 0

    def step():
        cdf = mcmi.Cdf(dB, order_cell=cell)
        res = mcmi.spai(cdf, p)
        res.apply(x, y)
        return cdf, res

    for _ in range(args.warmup):
        cdf, res = step()
        del cdf, res
    torch.cuda.synchronize()
    walk_ms, trans = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cdf, res = step()
        walk_ms.append(res.stats.ms_walk)
        trans.append(res.stats.transitions)
        retries = res.stats.retries
        nnz = res.nnz
        spilled = res.stats.spilled
        lanes, hslots, sslots = res.stats.lanes_per_row, res.stats.hash_slots, res.stats.sketch_slots
        tau, refined = res.stats.heavy_weight, res.stats.refined
        del cdf, res
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    total_trans = float(sum(trans))
    value = total_trans / elapsed

    # memory ceiling of the access pattern: a chase over a buffer of the record
    # set's size with one dependent random 64-byte block per step (what a step of
    # the walk reads), fresh randomness each step, read as one 16-byte load
    # (loads=1) or as four (loads=4; a walk step issues three)
    probe = {}
    cdf0 = mcmi.Cdf(dB)
    for loads in (1, 4):
        for wpc in (8, 16, 32):
            ms_p, rate = mcmi.gather_probe(max(1024, cdf0.rec_units), 1, 256, wpc, loads)
            probe[f"loads{loads}_wpc{wpc}"] = rate
    del cdf0
    ceiling = max(v for k, v in probe.items() if k.startswith("loads1_"))

    bpt = algorithmic_bytes_per_transition(B, args.prec == 32)
    walk_s = float(np.mean(walk_ms)) / 1e3
    achieved = bpt * trans[-1] / walk_s / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": TRAFFIC_BYTES,
                "kernel": "k_walk_block", "bytes_per_transition": round(bpt, 2),
                "walk_ms": round(walk_s * 1e3, 3), "walk_transitions_per_s": trans[-1] / walk_s,
                "gather_ceiling_steps_per_s": ceiling, "gather_probe": probe,
                "frac_of_gather_ceiling": round(trans[-1] / walk_s / ceiling, 4)}
    precision = walk_precision(mcmi, dB, B.n, args.chains, delta, eps, seed)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "transitions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.prec == 32 else "f64",
        "data": "synthetic",
        "config": {"workload": f"random nonsymmetric n={B.n}, 5-30 off-diagonals/row, ||C||_inf=0.7, "
                               f"{args.chains} chains/row, delta=1e-4, eps=1e-3, FP{args.prec} walks + FP64 sums",
                   "n": B.n, "nnz_B": B.nnz, "chains_per_row": args.chains, "transitions_per_step": trans[-1],
                   "nnz_M": nnz, "spilled_contributions": spilled, "retries": retries,
                   "lanes_per_row": lanes, "hash_slots": hslots, "sketch_slots": sslots,
                   "heavy_weight": tau, "rows_replayed": refined, "order_cell": cell},
        "roofline": roofline,
        "precision": precision,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(B, args.chains, delta, eps, args.prec == 32)
    print(json.dumps(out), flush=True)


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
    chains = args.chains if args.chains != 512 else 64
    p = mcmi.params(seed=0, chains=chains, delta=1e-4, eps=1e-3, walk_prec=args.prec, lanes_per_row=args.lanes,
                    hash_slots=args.hash_slots, sketch_slots=args.sketch_slots, heavy_weight=args.heavy_weight)
    x = torch.ones(B.n, dtype=torch.float64, device="cuda")
    y = torch.empty(B.n, dtype=torch.float64, device="cuda")
    cell = 4096 if args.order_cell is None else args.order_cell
    net, alloc = None, None
    if args.learned_alloc:
        from paper_2409_03095_amd import learned as L
        rng = np.random.default_rng(77)
        train = [I.aniso27(int(rng.integers(12, 21)), seed=1000 + k) for k in range(40)]
        net, tinfo = L.train_allocator(train, 1e-4, steps=3000)
        alloc = {"train": tinfo}
        print(f"[aniso27] allocation network trained: {json.dumps(tinfo)}", flush=True)

    def chains_for(cdf):
        # learned allocation: features -> network -> chains per row for the same
        # mean budget (chain cost 1 + floor(f7), mcmi_chain_cost), uniform fallback inside mcmi_allocate
        if net is None:
            return None
        feat = mcmi.row_features(cdf, 1e-4)
        pred = net.predict(feat)
        cost, total_cost = mcmi.chain_cost(feat)
        cpr, lam, fb = mcmi.allocate(pred, cost, int(chains * total_cost))
        alloc.update({"lambda": lam, "fallback": fb})
        return cpr

    for _ in range(args.warmup):
        cdf = mcmi.Cdf(dB, order_cell=cell)
        res = mcmi.spai(cdf, p, chains_per_row=chains_for(cdf))
        del cdf, res
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    walk_ms = []
    for _ in range(args.steps):
        cdf = mcmi.Cdf(dB, order_cell=cell)
        cpr = chains_for(cdf)
        res = mcmi.spai(cdf, p, chains_per_row=cpr)
        res.apply(x, y)
        walk_ms.append(res.stats.ms_walk)
        last = res
        rec_units = cdf.rec_units
        del cdf
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = last.stats
    ms_p, ceiling = mcmi.gather_probe(max(1024, rec_units), 1, 128, 16)
    m = np.maximum(np.diff(B.row_ptr) - 1, 1)
    bpt = float(np.mean((16.0 if args.prec == 32 else 24.0) + 4.0 * (np.ceil(np.log2(m)) + 1.0) + 4.0))
    walk_s = float(np.mean(walk_ms)) / 1e3
    out = {"metric": METRIC, "value": st.transitions * args.steps / elapsed, "unit": "transitions/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
           "higher_is_better": True, "dtype": "f32" if args.prec == 32 else "f64", "data": "synthetic",
           "config": {"workload": f"3D 27-point anisotropic {args.nx}^3", "n": B.n, "nnz_B": B.nnz,
                      "chains_per_row": chains, "transitions_per_step": int(st.transitions), "nnz_M": int(last.nnz),
                      "lanes_per_row": st.lanes_per_row, "hash_slots": st.hash_slots, "spilled": int(st.spilled),
                      "retries": int(st.retries), "record_bytes": int(rec_units) * 64, "order_cell": cell},
           "roofline": {"bound": "hbm", "achieved": round(bpt * st.transitions / walk_s / 1e9, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(bpt * st.transitions / walk_s / 1e9 / HBM_PEAK_GBS, 4),
                        "traffic": (TRAFFIC_BYTES_ANISO27 if (args.nx == 160 and args.prec == 32 and cell == 4096
                                                              and net is None) else None),
                        "kernel": "k_walk",
                        "bytes_per_transition": round(bpt, 2), "walk_ms": round(walk_s * 1e3, 3),
                        "walk_transitions_per_s": st.transitions / walk_s, "gather_ceiling_steps_per_s": ceiling}}
    if net is not None:
        # quality at the same budget: learned vs uniform chains, 10^4-row sample
        cdf = mcmi.Cdf(dB, order_cell=cell)
        cpr = chains_for(cdf)
        rows = np.sort(np.random.default_rng(12345).choice(B.n, 10000, replace=False))
        ql = L.evaluate(B, cpr, 1e-4, 1e-3, 0, rows, args.prec, cdf)
        qu = L.evaluate(B, torch.full((B.n,), chains, dtype=torch.int32, device="cuda"), 1e-4, 1e-3, 0, rows,
                        args.prec, cdf)
        alloc.update({"chains_min": int(cpr.min().item()), "chains_max": int(cpr.max().item()),
                      "learned": ql, "uniform": qu})
        out["config"]["allocation"] = "learned"
        out["learned_allocation"] = alloc
        print(f"[aniso27] learned r={ql['r_norm']:.4f} T={ql['transitions']} | uniform r={qu['r_norm']:.4f} "
              f"T={qu['transitions']}", flush=True)
        del cdf
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
    print(json.dumps(out), flush=True)


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
    chains = args.chains if args.chains != 512 else 128
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
    achieved = bpt * st.transitions / walk_s / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": TRAFFIC_BYTES_BATCHED if (args.prec == 32 and chains == 128 and cell == 0 and not args.tune
                                                     and not args.lanes and not args.hash_slots) else None,
                "kernel": "k_walk",
                "bytes_per_transition": round(bpt, 2), "walk_ms": round(walk_s * 1e3, 3),
                "walk_transitions_per_s": st.transitions / walk_s}
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
