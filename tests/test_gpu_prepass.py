"""GPU parity of the optional pre-pass (alpha-augmented diagonal of the
Section III-B splitting with the Section V-C sign rule; matrix reduction of
Algorithm 1 step 2): records bit-identical to the oracle's, the estimate within
the usual bar, the reported norm, cut and drop count exact."""
import numpy as np
import pytest

import oracle as O
from paper_2409_03095_amd import inputs as I
from parity import compare_spai, decode_records

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_03095_amd import mcmi  # raises if libmcmi.so is missing
    return mcmi


CASES = {
    "aug_nonddm": (lambda: I.nonddm(300, seed=4), 5.0, 0.0),
    "aug_alpha_1.5": (lambda: I.nonddm(257, seed=8), 1.5, 0.0),
    "drop_nonsym": (lambda: I.random_nonsym(3001, seed=5), 0.0, 0.1),
    "drop_half": (lambda: I.random_nonsym(2000, kmin=1, kmax=12, seed=12), 0.0, 0.5),
    "drop_ties_grid": (I.cfg1, 0.0, 0.3),
    "aug_and_drop": (lambda: I.nonddm(400, seed=9), 5.0, 0.25),
}


def _build(mc, name):
    gen, alpha, frac = CASES[name]
    B = gen()
    print(f"[gpu] prepass {name}: n={B.n} nnz={B.nnz} alpha={alpha} drop={frac}", flush=True)
    cdf = mc.Cdf(mc.DeviceCsr.from_host(B), alpha=alpha, drop_frac=frac)
    o = O.Oracle(B, alpha=alpha, drop_frac=frac)
    return B, cdf, o


@pytest.mark.parametrize("name", sorted(CASES))
def test_prepass_records_bit_identical(mc, name):
    B, cdf, o = _build(mc, name)
    nb, cut, nd = cdf.prep_info()
    assert (nb, cut, nd) == (o.norm_b, o.drop_thr, o.dropped)
    assert cdf.nnz_c == o.nnz_c and cdf.norm_inf == o.norm_inf
    rec, roff, diag = cdf.download()
    assert np.array_equal(diag, o.diag)
    for i, (row, m, W, s32, s64, cum, col, neg, thr, acol, aneg) in enumerate(decode_records(rec, roff, B.n)):
        b, e = o.cptr[i], o.cptr[i + 1]
        assert row == i and m == e - b and W == int(o.wsum[i])
        assert s64 == o.shat[i]
        assert np.array_equal(cum, o.cum[b:e].astype(np.int64))
        assert np.array_equal(col, o.ccol[b:e])
        assert np.array_equal(neg, o.cval[b:e] < 0)
        assert np.array_equal(thr, o.athr[b:e].astype(np.int64))
        assert np.array_equal(acol, o.ccol[b:e][o.aidx[b:e]])


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("name", ["aug_nonddm", "aug_and_drop", "drop_nonsym"])
def test_prepass_spai_matches_oracle(mc, name, prec):
    B, cdf, o = _build(mc, name)
    chains, delta, eps = 96, 1e-5, 1e-3
    res = mc.spai(cdf, mc.params(seed=11, chains=chains, delta=delta, eps=eps, walk_prec=prec))
    rp, col, val = res.to_numpy()
    orc = o.spai(seed=11, chains=chains, delta=delta, eps=eps, fp32=(prec == 32))
    assert orc["guard"] == 0
    assert res.stats.transitions == orc["transitions"]
    compare_spai((rp, col, val), orc, o.diag, chains)


def test_prepass_errors(mc):
    B = I.nonddm(64, seed=4)
    dB = mc.DeviceCsr.from_host(B)
    with pytest.raises(mc.McmiError):
        mc.Cdf(dB)  # zero and missing diagonals need the augmented splitting
    for alpha, frac in ((-1.0, 0.0), (0.0, 1.0), (0.0, -0.1), (float("nan"), 0.0)):
        with pytest.raises(mc.McmiError):
            mc.Cdf(dB, alpha=alpha, drop_frac=frac)


def test_prepass_full_size_cut(mc):
    """Reduction on the n = 262144 random nonsymmetric matrix (4.6M entries of C):
    the radix selection finds the oracle's cut and count exactly."""
    B = I.cfg2()
    for frac in (0.02, 0.06):
        cdf = mc.Cdf(mc.DeviceCsr.from_host(B), drop_frac=frac)
        o = O.Oracle(B, drop_frac=frac)
        assert cdf.prep_info() == (0.0, o.drop_thr, o.dropped)
        assert cdf.nnz_c == o.nnz_c and cdf.norm_inf == o.norm_inf
