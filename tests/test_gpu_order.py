"""Row schedule with locality (mcmi_cdf_opts.order_cell): the device's cell
search equals a host breadth-first search with the same seeds and tie rule, the
schedule is a permutation, and a walk that follows it gives the oracle's estimate
(the schedule changes when a row runs, never what it computes)."""
import numpy as np
import pytest

import oracle as O
from paper_2409_03095_amd import inputs as I
from parity import compare_spai

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

UNSET = np.uint64(0xFFFFFFFF)
M32 = np.uint64(0xFFFFFFFF)


@pytest.fixture(scope="module")
def mc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_03095_amd import mcmi  # raises if libmcmi.so is missing
    return mcmi


def _fmix32(x):
    x = x ^ (x >> np.uint64(16))
    x = (x * np.uint64(0x85EBCA6B)) & M32
    x = x ^ (x >> np.uint64(13))
    x = (x * np.uint64(0xC2B2AE35)) & M32
    return x ^ (x >> np.uint64(16))


def host_order(B, cell, max_levels=64):
    """Level-synchronous multi-source BFS on the pattern of B: a row without a cell
    takes the smallest cell among its neighbours labelled at an earlier level."""
    n = B.n
    r = np.arange(n, dtype=np.uint64)
    p = 1.0 / max(cell, 1)
    thr = np.uint64(0xFFFFFFFF if p >= 1.0 else int(p * 4294967296.0))
    lab = np.where(_fmix32(r ^ np.uint64(0x6A09E667)) < thr, r, UNSET)
    rp = B.row_ptr.astype(np.int64)
    has = np.diff(rp) > 0
    for _ in range(max_levels):
        mins = np.full(n, UNSET, dtype=np.uint64)
        if B.nnz:
            red = np.minimum.reduceat(lab[B.col], np.minimum(rp[:-1], B.nnz - 1))
            mins[has] = red[has]
        new = np.where(lab == UNSET, mins, lab)
        if np.array_equal(new, lab):
            break
        lab = new
    key = np.where(lab == UNSET, r, lab)
    return np.lexsort((r, key)).astype(np.int32)


CASES = {
    "grid32_cell16": (I.cfg1, 16),
    "grid32_cell64": (I.cfg1, 64),
    "aniso27_20_cell512": (lambda: I.aniso27(20, seed=3), 512),
    "random_20000_cell4096": (lambda: I.random_nonsym(20000, seed=31), 4096),
    "cycle_50000_cell4096": (lambda: I.scaled_cycle(50000, 0.5), 4096),  # most rows beyond 64 levels
    "diag_only_cell8": (lambda: I.diag_only(3000, seed=2), 8),          # no edges: every row alone
    "grid32_cell1": (I.cfg1, 1),                                         # every row a seed
    "single_row": (lambda: I.diag_only(1, seed=3), 4096),               # n = 1
    "grid2x2": (lambda: I.grid2d_5pt(2, 2), 2),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_order_equals_host_search(mc, name):
    gen, cell = CASES[name]
    B = gen()
    print(f"[gpu] order {name}: n={B.n} nnz={B.nnz} cell={cell}", flush=True)
    cdf = mc.Cdf(mc.DeviceCsr.from_host(B), order_cell=cell)
    got = cdf.order()
    assert np.array_equal(np.sort(got), np.arange(B.n, dtype=np.int32))
    assert np.array_equal(got, host_order(B, cell))


def test_order_cells_are_compact_on_a_grid(mc):
    """On a 3D 27-point grid, 512 consecutive rows of the schedule (cells of about
    512 rows) have a smaller two-hop neighbourhood than 512 consecutive rows of the
    natural order (a flat sheet of the grid): the set a batch of walks starts in."""
    B = I.aniso27(24, seed=3)
    got = mc.Cdf(mc.DeviceCsr.from_host(B), order_cell=512).order()
    S = B.to_scipy()
    S.data[:] = 1.0
    S2 = S @ S

    def reach(order):
        return np.median([np.unique(S2[order[i:i + 512]].indices).size / 512 for i in range(0, B.n - 512, 512)])

    assert reach(got) < 0.85 * reach(np.arange(B.n))


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("chains", [64, 512])
def test_ordered_spai_matches_oracle(mc, prec, chains):
    B = I.aniso27(12, seed=4)
    print(f"[gpu] ordered spai n={B.n} chains={chains} prec={prec}", flush=True)
    cdf = mc.Cdf(mc.DeviceCsr.from_host(B), order_cell=64)
    o = O.Oracle(B)
    p = mc.params(seed=7, chains=chains, delta=1e-4, eps=1e-3, walk_prec=prec)
    res = mc.spai(cdf, p)
    orc = o.spai(seed=7, chains=chains, delta=1e-4, eps=1e-3, fp32=(prec == 32))
    assert orc["guard"] == 0 and res.stats.transitions == orc["transitions"]
    compare_spai(res.to_numpy(), orc, o.diag, chains)


def test_ordered_and_natural_runs_agree_at_size(mc):
    """40^3 27-point (64000 rows, 64 chains): the ordered and the natural schedule
    give the same pattern and the same values to the FP64 summation bar."""
    B = I.aniso27(40, seed=5)
    dB = mc.DeviceCsr.from_host(B)
    p = mc.params(seed=9, chains=64, delta=1e-4, eps=1e-3, walk_prec=32)
    a = mc.spai(mc.Cdf(dB), p)
    b = mc.spai(mc.Cdf(dB, order_cell=4096), p)
    assert a.stats.transitions == b.stats.transitions
    ra, ca, va = a.to_numpy()
    rb, cb, vb = b.to_numpy()
    assert np.array_equal(ra, rb) and np.array_equal(ca, cb)
    assert np.allclose(va, vb, rtol=1e-12, atol=1e-15)


def test_ordered_plan_matches_eager(mc):
    B = I.aniso27(16, seed=6)
    cdf = mc.Cdf(mc.DeviceCsr.from_host(B), order_cell=256)
    plan = mc.Plan(cdf, mc.params(seed=0, chains=64, delta=1e-4, eps=1e-3), nnz_capacity=B.n * 400)
    for seed in (21, 22):
        plan.launch(seed)
        got, st, ovf = plan.result()
        assert not ovf
        eager = mc.spai(cdf, mc.params(seed=seed, chains=64, delta=1e-4, eps=1e-3))
        rp, col, val = eager.to_numpy()
        torch.cuda.synchronize()
        assert st.transitions == eager.stats.transitions
        assert np.array_equal(got[0], rp) and np.array_equal(got[1], col)
        assert np.allclose(got[2], val, rtol=1e-12, atol=1e-15)


def test_order_errors(mc):
    B = I.cfg1()
    dB = mc.DeviceCsr.from_host(B)
    with pytest.raises(mc.McmiError):
        mc.Cdf(dB, order_cell=-1)
    with pytest.raises(mc.McmiError):
        mc.Cdf(dB).order()  # built without a schedule
