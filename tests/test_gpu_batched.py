"""GPU parity of the batched launch: many matrices of uneven size and chain
length in one persistent launch (one record space, per-matrix Philox tags)."""
import numpy as np
import pytest

import oracle as O
from paper_2409_03095_amd import inputs as I
from parity import compare_spai, fp32_walks_against_fp64

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_03095_amd import mcmi
    return mcmi


@pytest.mark.parametrize("prec,kw,cell", [(64, {}, 0), (32, {}, 0), (32, {"lanes_per_row": 256}, 0),
                                          (64, {"hash_slots": 128}, 0), (32, {}, 256), (64, {}, 64)])
def test_batched_blocks_equal_single_matrix_runs(mc, prec, kw, cell):
    mats, meta = I.convdiff_batch(count=12, seed=3, nmin=200, nmax=2500)
    print(f"[gpu] batched {[m.n for m in mats]} prec={prec} {kw} cell={cell}", flush=True)
    cdf = mc.Cdf.batched([mc.DeviceCsr.from_host(B) for B in mats], order_cell=cell)
    if cell:
        # the schedule keeps each matrix's rows in the matrix's own slice
        order = cdf.order()
        _, base0, _ = cdf.batch_info()
        for i in range(len(mats)):
            part = np.sort(order[base0[i]:base0[i + 1]])
            assert np.array_equal(part, np.arange(base0[i], base0[i + 1], dtype=np.int32))
    k, base, nrm = cdf.batch_info()
    assert k == len(mats) and base[-1] == sum(m.n for m in mats)
    N = 300 if kw.get("lanes_per_row") else 64
    res = mc.spai(cdf, mc.params(seed=1, chains=N, delta=1e-4, eps=1e-3, walk_prec=prec, tag=100, **kw))
    rp, col, val = res.to_numpy()
    total = 0
    for i, B in enumerate(mats):
        o = O.Oracle(B)
        assert nrm[i] == o.norm_inf
        orc = o.spai(seed=1, chains=N, delta=1e-4, eps=1e-3, fp32=(prec == 32), tag=100 + i)
        assert orc["guard"] == 0
        total += orc["transitions"]
        r0, r1 = base[i], base[i + 1]
        sub_rp = rp[r0:r1 + 1] - rp[r0]
        sub_col = col[rp[r0]:rp[r1]] - r0
        sub_val = val[rp[r0]:rp[r1]]
        compare_spai((sub_rp, sub_col, sub_val), orc, o.diag, N)
    assert res.stats.transitions == total


def test_batched_full_size_sampled_rows(mc):
    """The benchmark's batched set at full size (256 convection-diffusion matrices,
    5.75M rows, 128 chains, FP32 walks, delta = 1e-4, eps = 1e-3, tag 0) in one
    launch, as bench.py runs it; 48 rows of each of 8 sampled matrices compared with
    the oracle's runs of those rows under the matrix's Philox tag."""
    mats, _ = I.convdiff_batch(256, seed=3)
    devs = [mc.DeviceCsr.from_host(B) for B in mats]
    cdf = mc.Cdf.batched(devs)
    _, base, _ = cdf.batch_info()
    print(f"[gpu] batched full size: {int(base[-1])} rows", flush=True)
    res = mc.spai(cdf, mc.params(seed=0, chains=128, delta=1e-4, eps=1e-3, walk_prec=32))
    rp_t, col_t, val_t = res.to_torch()
    torch.cuda.synchronize()
    rp = rp_t.cpu().numpy()
    rng = np.random.default_rng(17)
    for k in sorted(int(x) for x in rng.choice(len(mats), 8, replace=False)):
        B = mats[k]
        rows = np.sort(rng.choice(B.n, 48, replace=False)).astype(np.int32)
        g = rows.astype(np.int64) + int(base[k])
        pos = np.concatenate([np.arange(rp[r], rp[r + 1]) for r in g])
        idx = torch.from_numpy(pos).cuda()
        sub_col = col_t[idx].cpu().numpy() - int(base[k])
        sub_val = val_t[idx].cpu().numpy()
        sub_rp = np.concatenate([[0], np.cumsum(rp[g + 1] - rp[g])])
        o = O.Oracle(B)
        orc = o.spai(seed=0, chains=128, delta=1e-4, eps=1e-3, fp32=True, tag=k, rows=rows)
        assert orc["guard"] == 0
        compare_spai((sub_rp, sub_col, sub_val), orc, o.diag, 128, rows=rows)
        # the FP32 walks' error against the FP64 oracle (1e-5 relative, or the FP32
        # weight-rounding bound where contributions cancel)
        orc64 = o.spai(seed=0, chains=128, delta=1e-4, eps=1e-3, tag=k, rows=rows)
        out = fp32_walks_against_fp64(B.n, (sub_rp, sub_col, sub_val), rows, orc64, o, 128, 1e-3, 1e-4,
                                      lambda r: o.spai(seed=0, chains=128, delta=1e-4, eps=0.0, tag=k, rows=r))
        print(f"  matrix {k}: FP32 vs FP64 oracle {out}", flush=True)


@pytest.mark.parametrize("fault", ["col_high", "col_negative", "row_ptr_end"])
def test_batched_rejects_a_bad_part(mc, fault):
    """One malformed matrix in a batch (a column outside [0, n_k) or a last row
    pointer other than nnz_k) fails the whole batch with the CSR status; the same
    batch with that matrix intact builds."""
    mats, _ = I.convdiff_batch(count=5, seed=6, nmin=200, nmax=900)
    devs = [mc.DeviceCsr.from_host(B) for B in mats]
    mc.Cdf.batched(devs)
    bad = devs[3]
    print(f"[gpu] batched bad part {fault} n={bad.n} nnz={bad.nnz}", flush=True)
    if fault == "col_high":
        bad.col[bad.nnz // 2] = bad.n
    elif fault == "col_negative":
        bad.col[0] = -1
    else:
        bad.row_ptr[-1] = bad.nnz - 1
    torch.cuda.synchronize()
    with pytest.raises(mc.McmiError) as e:
        mc.Cdf.batched(devs)
    assert e.value.status == -2


def test_batched_schedule_rejects_pre_pass_options(mc):
    import ctypes
    mats, _ = I.convdiff_batch(count=3, seed=4, nmin=200, nmax=400)
    devs = [mc.DeviceCsr.from_host(B) for B in mats]
    arr = (mc.CsrIn * 3)(*[d._struct() for d in devs])
    h = ctypes.c_void_p()
    for alpha, frac, cell in ((1.0, 0.0, 0), (0.0, 0.1, 0), (0.0, 0.0, -5)):
        opts = mc.CdfOpts(alpha, frac, cell, 0)
        st = mc._lib.mcmi_build_cdf_batched_ex(arr, ctypes.c_int32(3), ctypes.byref(opts), ctypes.byref(h),
                                                mc._stream(None))
        assert st == -1 and not h.value  # MCMI_ERR_ARG


# ------------------------------------------------------------ autotuner
def test_tune_selects_a_valid_shape_and_caches(mc, tmp_path):
    B = I.random_nonsym(20000, seed=51)
    cdf = mc.Cdf(mc.DeviceCsr.from_host(B))
    base = mc.params(seed=3, chains=512, delta=1e-4, eps=1e-3, walk_prec=32)
    cache = tmp_path / "tune.json"
    best, ms = mc.tune(cdf, base, sample_rows=2048, cache_path=cache)
    print(f"[gpu] tuned: lanes={best.lanes_per_row} H={best.hash_slots} sketch={best.sketch_slots} "
          f"tau={best.heavy_weight} ms={ms:.3f}", flush=True)
    assert best.lanes_per_row in (64, 256, 512, 1024) and ms > 0
    assert cache.exists() and "gfx950" in cache.read_text()
    best2, ms2 = mc.tune(cdf, base, sample_rows=2048, cache_path=cache)
    assert (best2.lanes_per_row, best2.hash_slots, best2.sketch_slots) == \
           (best.lanes_per_row, best.hash_slots, best.sketch_slots) and ms2 == pytest.approx(ms, rel=1e-6)
    rows = np.arange(0, B.n, 97, dtype=np.int32)
    res = mc.spai(cdf, best, rows=torch.from_numpy(rows).cuda())
    rp, col, val = res.to_numpy()
    o = O.Oracle(B)
    orc = o.spai(seed=3, chains=512, delta=1e-4, eps=1e-3, fp32=True, rows=rows)
    assert orc["guard"] == 0 and res.stats.transitions == orc["transitions"]
    compare_spai((rp, col, val), orc, o.diag, 512, rows=rows)


# ------------------------------------------------------------ hipGraph plans
@pytest.mark.parametrize("chains", [64, 512])
def test_plan_replays_match_eager_runs(mc, chains):
    """The captured plan is replayed several times with new seeds, with eager
    library work and synchronisations in between; every replay must equal the
    eager mcmi_spai result for its seed (same pattern, values to the FP64 bar)."""
    B = I.random_nonsym(6000, seed=52)
    cdf = mc.Cdf(mc.DeviceCsr.from_host(B))
    plan = mc.Plan(cdf, mc.params(seed=0, chains=chains, delta=1e-4, eps=1e-3), nnz_capacity=B.n * 400)
    for seed in (11, 12, 13):
        plan.launch(seed)
        got, st, ovf = plan.result()
        assert not ovf
        eager = mc.spai(cdf, mc.params(seed=seed, chains=chains, delta=1e-4, eps=1e-3))
        rp, col, val = eager.to_numpy()
        torch.cuda.synchronize()
        assert st.transitions == eager.stats.transitions
        assert np.array_equal(got[0], rp) and np.array_equal(got[1], col)
        assert np.allclose(got[2], val, rtol=1e-12, atol=1e-15)
    orc = O.Oracle(B).spai(seed=13, chains=chains, delta=1e-4, eps=1e-3)
    compare_spai(got, orc, O.Oracle(B).diag, chains)


def test_plan_batched_lpt_and_per_row_chains_match_eager(mc):
    """A plan over a batched record set walks the eager launch's LPT order; a
    plan with per-row chain counts sizes its tables from the largest count. Every
    replay equals the eager mcmi_spai result for its seed."""
    mats, _ = I.convdiff_batch(count=10, seed=8, nmin=300, nmax=3000)
    cdf = mc.Cdf.batched([mc.DeviceCsr.from_host(B) for B in mats])
    nrow = int(cdf.batch_info()[1][-1])
    cpr = torch.from_numpy(I.chain_counts(nrow, mean=24.0, seed=9, hi=160)).cuda()
    print(f"[gpu] batched plan: {nrow} rows, chains per row {int(cpr.min())}..{int(cpr.max())}", flush=True)
    for prec, per_row in ((32, False), (64, True)):
        base = mc.params(seed=0, chains=48, delta=1e-4, eps=1e-3, walk_prec=prec)
        plan = mc.Plan(cdf, base, nnz_capacity=nrow * 300, chains_per_row=cpr if per_row else None)
        for seed in (21, 22):
            plan.launch(seed)
            got, st, ovf = plan.result()
            assert not ovf
            eager = mc.spai(cdf, mc.params(seed=seed, chains=48, delta=1e-4, eps=1e-3, walk_prec=prec),
                            chains_per_row=cpr if per_row else None)
            rp, col, val = eager.to_numpy()
            torch.cuda.synchronize()
            assert st.transitions == eager.stats.transitions
            assert np.array_equal(got[0], rp) and np.array_equal(got[1], col)
            assert np.allclose(got[2], val, rtol=1e-12, atol=1e-15)
        del plan


@pytest.mark.parametrize("bad", ["spill_below_16", "hash_not_pow2", "lanes_odd", "chains_zero_row"])
def test_plan_create_rejects_what_spai_rejects(mc, bad):
    """mcmi_plan_create applies mcmi_spai's parameter checks (before any kernel
    runs): overflow tables below 16 slots, a hash size that is not a power of two,
    an unsupported lane count, a per-row chain count below 1."""
    B = I.random_nonsym(2000, seed=54)
    cdf = mc.Cdf(mc.DeviceCsr.from_host(B))
    kw = {"spill_below_16": dict(lanes_per_row=8, spill_slots=4), "hash_not_pow2": dict(hash_slots=96),
          "lanes_odd": dict(lanes_per_row=48), "chains_zero_row": {}}[bad]
    cpr = None
    if bad == "chains_zero_row":
        c = np.full(B.n, 8, dtype=np.int32)
        c[1234] = 0
        cpr = torch.from_numpy(c).cuda()
    p = mc.params(seed=0, chains=32, delta=1e-4, eps=1e-3, **kw)
    for call in (lambda: mc.Plan(cdf, p, nnz_capacity=B.n * 100, chains_per_row=cpr),
                 lambda: mc.spai(cdf, p, chains_per_row=cpr)):
        with pytest.raises(mc.McmiError) as ei:
            call()
        assert ei.value.status == -1


def test_plan_reports_overflow(mc):
    B = I.random_nonsym(3000, seed=53)
    cdf = mc.Cdf(mc.DeviceCsr.from_host(B))
    plan = mc.Plan(cdf, mc.params(seed=0, chains=64, delta=1e-4, eps=1e-3), nnz_capacity=1000)
    plan.launch(5)
    got, st, ovf = plan.result()
    assert ovf and got is None
