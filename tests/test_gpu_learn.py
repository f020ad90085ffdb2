"""GPU parity of the learned-allocation inputs: row features and pilot variance."""
import numpy as np
import pytest

import oracle as O
from paper_2409_03095_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_03095_amd import mcmi
    return mcmi


MATS = {
    "family": lambda: I.family_5pt(7),
    "nonsym": lambda: I.random_nonsym(3000, seed=41),
    "longrows": lambda: I.random_nonsym(400, kmin=60, kmax=120, seed=42),
    "signed_dense": lambda: I.dense_small(9, 0.6, 3),
    "diag_only": lambda: I.diag_only(20, seed=1),
}


@pytest.mark.parametrize("name", sorted(MATS))
def test_row_features(mc, name):
    B = MATS[name]()
    print(f"[gpu] features {name} n={B.n}", flush=True)
    cdf = mc.Cdf(mc.DeviceCsr.from_host(B))
    f = mc.row_features(cdf, 1e-3).cpu().numpy()
    ref = O.Oracle(B).features(1e-3)
    assert np.allclose(f, ref, rtol=2e-6, atol=1e-6), np.abs(f - ref).max(axis=0)


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("name", ["family", "nonsym", "signed_dense"])
def test_pilot_variance(mc, name, prec):
    B = MATS[name]()
    print(f"[gpu] pilot {name} n={B.n} prec={prec}", flush=True)
    cdf = mc.Cdf(mc.DeviceCsr.from_host(B))
    p = mc.params(seed=9, delta=1e-4, walk_prec=prec, tag=5)
    var, ln = mc.pilot_variance(cdf, p, 64)
    var, ln = var.cpu().numpy(), ln.cpu().numpy()
    rv, rl = O.Oracle(B).pilot(seed=9, pilot=64, delta=1e-4, fp32=(prec == 32), tag=5)
    assert np.array_equal(ln, rl)
    scale = np.maximum(np.abs(rv), 1e-300)
    assert np.all(np.abs(var - rv) <= 1e-10 * scale + 1e-12), np.max(np.abs(var - rv) / scale)
