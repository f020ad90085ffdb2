"""GPU parity of the batched launch: many matrices of uneven size and chain
length in one persistent launch (one record space, per-matrix Philox tags)."""
import numpy as np
import pytest

import oracle as O
from paper_2409_03095_amd import inputs as I
from parity import compare_spai

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_03095_amd import mcmi
    return mcmi


@pytest.mark.parametrize("prec,kw", [(64, {}), (32, {}), (32, {"lanes_per_row": 256}),
                                     (64, {"hash_slots": 128})])
def test_batched_blocks_equal_single_matrix_runs(mc, prec, kw):
    mats, meta = I.convdiff_batch(count=12, seed=3, nmin=200, nmax=2500)
    print(f"[gpu] batched {[m.n for m in mats]} prec={prec} {kw}", flush=True)
    cdf = mc.Cdf.batched([mc.DeviceCsr.from_host(B) for B in mats])
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
