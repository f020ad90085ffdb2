"""GPU parity of top-k retention (Section IV-B: a prescribed number of the
largest entries per row) in both walk kernels, against the oracle."""
import numpy as np
import pytest

import oracle as O
from paper_2409_03095_amd import inputs as I
from parity import compare_topk

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_03095_amd import mcmi  # raises if libmcmi.so is missing
    return mcmi


CASES = {
    # name: (matrix, chains, delta, eps, topk, kernel options)
    "grid_wave_k9": (I.cfg1, 200, 1e-3, 1e-3, 9, {}),
    "grid_wave_k1": (I.cfg1, 100, 1e-3, 1e-3, 1, {}),
    "nonsym_block_k20": (lambda: I.random_nonsym(1500, seed=31), 256, 1e-4, 1e-3, 20, {"lanes_per_row": 256}),
    "nonsym_block512_k64_f32": (lambda: I.random_nonsym(1200, seed=32), 512, 1e-4, 1e-3, 64,
                                {"lanes_per_row": 512, "walk_prec": 32}),
    "nonsym_wave_k12_eps0": (lambda: I.random_nonsym(800, kmin=3, kmax=6, seed=33), 32, 1e-3, 0.0, 12, {}),
    "filter_m_k16": (lambda: I.random_nonsym(900, seed=34), 128, 1e-4, 1e-3, 16, {"filter": 1}),
    "filter_m_block_k16_f32": (lambda: I.random_nonsym(900, seed=35), 256, 1e-4, 1e-3, 16,
                               {"lanes_per_row": 256, "walk_prec": 32, "filter": 1}),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_topk_matches_oracle(mc, name):
    gen, chains, delta, eps, k, kw = CASES[name]
    B = gen()
    prec = kw.get("walk_prec", 64)
    print(f"[gpu] topk {name}: n={B.n} chains={chains} k={k} {kw}", flush=True)
    cdf = mc.Cdf(mc.DeviceCsr.from_host(B))
    res = mc.spai(cdf, mc.params(seed=3, chains=chains, delta=delta, eps=eps, topk=k, **kw))
    rp, col, val = res.to_numpy()
    o = O.Oracle(B)
    orc = o.spai(seed=3, chains=chains, delta=delta, eps=eps, topk=k, fp32=(prec == 32),
                 filter_on_m=bool(kw.get("filter", 0)))
    assert orc["guard"] == 0
    assert res.stats.transitions == orc["transitions"]
    err, amb = compare_topk((rp, col, val), orc, o.diag, chains)
    print(f"[gpu] topk {name}: max rel err {err:.2e}, order-dependent rows {amb}", flush=True)
    assert np.all(np.diff(rp) <= k)
