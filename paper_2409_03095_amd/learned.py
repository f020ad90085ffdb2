"""Learned chain allocation: train the allocation network on pilot-run variance
and compare learned vs uniform chains per row at equal transition budgets.

Pipeline (every numerical step runs in libmcmi.so through the C ABI; torch only
holds device memory):

1. training matrices -> records (mcmi_build_cdf) -> row features
   (mcmi_row_features) and pilot variance v_r and mean chain length len_r
   (mcmi_pilot_variance);
2. regression target y_r = (ln v_r - ln(len_r + 1)) / 2 (mcmi_neyman_target):
   Neyman allocation (minimise sum_r v_r / N_r subject to
   sum_r N_r (len_r + 1) = T) gives N_r proportional to exp(y_r);
3. the 8-64-64-1 network is trained on (features, y) with Adam (mcmi_mlp_train);
4. on a held-out matrix: features -> prediction (mcmi_mlp_predict) -> chains per
   row (mcmi_allocate, budget in visited states with per-row chain cost
   1 + floor(f7) from mcmi_chain_cost),
   uniform allocation gets the same budget -> mcmi_spai with the per-row chains;
5. quality: ||I - M B||_F / sqrt(n) on a uniform row sample (exact sparse
   products on the host), with a 95 % interval.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import inputs as I
from . import mcmi


def _dev(B):
    return mcmi.DeviceCsr.from_host(B)


def pilot_targets(B, delta, pilot=64, seed=0, prec=64):
    """Features and Neyman targets of every row of B (device tensors)."""
    cdf = mcmi.Cdf(_dev(B))
    feat = mcmi.row_features(cdf, delta)
    var, ln = mcmi.pilot_variance(cdf, mcmi.params(seed=seed, delta=delta, walk_prec=prec), pilot)
    return feat, mcmi.neyman_target(var, ln), cdf


def train_allocator(train_mats, delta, steps=3000, batch=4096, lr=2e-3, seed=0, pilot=64, init_seed=0):
    """Build the training set from the family (one block-diagonal matrix) and train."""
    import torch
    B = I.block_diag(train_mats)
    t0 = time.perf_counter()
    feat, y, _ = pilot_targets(B, delta, pilot=pilot, seed=seed)
    torch.cuda.synchronize()
    t_pilot = time.perf_counter() - t0
    net = mcmi.Mlp()
    net.set_params(init_params(init_seed))
    net.fit_normalization(feat)
    t0 = time.perf_counter()
    losses = net.train(feat, y, steps=steps, batch=batch, lr=lr, seed=seed + 1)
    t_train = time.perf_counter() - t0
    yv = y.cpu().numpy()
    return net, {"rows": int(B.n), "pilot_s": t_pilot, "train_s": t_train, "loss_first": float(losses[:20].mean()),
                 "loss_last": float(losses[-50:].mean()), "target_var": float(yv.var()), "steps": steps}


def init_params(seed):
    """He-uniform initial weights (zero biases), packed in the library's order."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape, fan_in in (((64, 8), 8), ((64,), None), ((64, 64), 64), ((64,), None), ((64,), 64), ((1,), None)):
        if fan_in is None:
            parts.append(np.zeros(shape, np.float32))
        else:
            lim = math.sqrt(6.0 / fan_in)
            parts.append(rng.uniform(-lim, lim, size=shape).astype(np.float32))
    return np.concatenate([p.reshape(-1) for p in parts])


def sample_rows(res, rows):
    """The listed rows of M (a SpaiResult) as host CSR arrays, gathered on the
    device so that only the sample crosses PCIe."""
    import torch
    rp, col, val = res.to_torch()
    r = torch.as_tensor(np.asarray(rows, dtype=np.int64), device="cuda")
    starts, lens = rp[r], rp[r + 1] - rp[r]
    sub_rp = torch.zeros(r.numel() + 1, dtype=torch.int64, device="cuda")
    sub_rp[1:] = torch.cumsum(lens, 0)
    total = int(sub_rp[-1].item())
    pos = torch.arange(total, device="cuda") - torch.repeat_interleave(sub_rp[:-1], lens, output_size=total)
    idx = torch.repeat_interleave(starts, lens, output_size=total) + pos
    return sub_rp.cpu().numpy(), col[idx].cpu().numpy(), val[idx].cpu().numpy()


def residual_sample(B, sub_rp, sub_col, sub_val, rows):
    """||e_r - M_r B||_2^2 for the sampled rows (exact sparse products); the
    sub_* arrays hold M's sampled rows in the order of `rows`."""
    import scipy.sparse as sp
    Bs = B.to_scipy()
    Ms = sp.csr_matrix((sub_val, sub_col, sub_rp), shape=(len(rows), B.n))
    E = sp.csr_matrix((np.ones(len(rows)), (np.arange(len(rows)), rows)), shape=(len(rows), B.n))
    R = (Ms @ Bs - E).tocsr()
    return np.asarray(R.multiply(R).sum(axis=1)).ravel()


def evaluate(B, chains_per_row, delta, eps, seed=0, rows_sample=None, prec=64, cdf=None):
    """Run mcmi_spai with the given per-row chains; return transitions, GPU time and
    the normalised residual estimate with its 95 % half-width."""
    import torch
    if cdf is None:
        cdf = mcmi.Cdf(_dev(B))
    cpr = torch.as_tensor(chains_per_row, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = mcmi.spai(cdf, mcmi.params(seed=seed, chains=1, delta=delta, eps=eps, walk_prec=prec), chains_per_row=cpr)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rows = rows_sample if rows_sample is not None else np.arange(B.n)
    sq = residual_sample(B, *sample_rows(res, rows), rows)
    mean = float(sq.mean())
    half = 1.96 * float(sq.std(ddof=1)) / math.sqrt(len(rows)) if len(rows) > 1 else 0.0
    return {"transitions": int(res.stats.transitions), "wall_s": wall, "ms_walk": float(res.stats.ms_walk),
            "r_norm": math.sqrt(mean), "r_norm_lo": math.sqrt(max(mean - half, 0.0)),
            "r_norm_hi": math.sqrt(mean + half), "nnz": int(res.nnz)}


def compare(net, B, delta, eps, budgets, seed=0, n_sample=10000, prec=64):
    """Learned vs uniform at each mean-chains budget. Budget in chain-cost units
    (mcmi_chain_cost, 1 + floor(f7_r) per chain):
    sum_r N_r cost_r <= budget_mean * sum_r cost_r."""
    import torch
    cdf = mcmi.Cdf(_dev(B))
    t0 = time.perf_counter()
    feat = mcmi.row_features(cdf, delta)
    pred = net.predict(feat)
    torch.cuda.synchronize()
    t_infer = time.perf_counter() - t0
    cost, total_cost = mcmi.chain_cost(feat)
    rng = np.random.default_rng(12345)
    rows = np.sort(rng.choice(B.n, min(n_sample, B.n), replace=False))
    out = []
    for nb in budgets:
        budget = int(nb * total_cost)
        chains_l, lam, fb = mcmi.allocate(pred, cost, budget)
        learned = evaluate(B, chains_l, delta, eps, seed, rows, prec, cdf)
        uni = max(1, budget // total_cost)
        uniform = evaluate(B, torch.full((B.n,), uni, dtype=torch.int32, device="cuda"), delta, eps, seed, rows,
                           prec, cdf)
        out.append({"mean_chains": nb, "budget": budget, "lambda": lam, "fallback": fb,
                    "learned": learned, "uniform": uniform, "infer_s": t_infer})
    return out


def crossing(points, key="transitions", thr=0.3):
    """Interpolate (log-log) the value of `key` where r_norm crosses thr."""
    pts = sorted(points, key=lambda p: p[key])
    for a, b in zip(pts, pts[1:]):
        if a["r_norm"] > thr >= b["r_norm"]:
            la, lb = math.log(a[key]), math.log(b[key])
            ra, rb = math.log(a["r_norm"]), math.log(b["r_norm"])
            return math.exp(la + (math.log(thr) - ra) * (lb - la) / (rb - ra))
    return None
