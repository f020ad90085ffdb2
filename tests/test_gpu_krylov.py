"""Device BiCGstab around M (mcmi_bicgstab) against scipy's BiCGstab run with the
same matrices on the host: both converge, the iteration counts agree within
one (rounding of the inner products differs), the true residuals meet the
tolerance."""
import numpy as np
import pytest

from paper_2409_03095_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
spla = pytest.importorskip("scipy.sparse.linalg")
sp = pytest.importorskip("scipy.sparse")


@pytest.fixture(scope="module")
def mc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_03095_amd import mcmi  # raises if libmcmi.so is missing
    return mcmi


def scipy_iters(Bs, b, M=None, rtol=1e-8):
    it = [0]
    pre = None if M is None else spla.LinearOperator(Bs.shape, matvec=lambda v: M @ v)
    x, info = spla.bicgstab(Bs, b, x0=np.zeros(b.size), rtol=rtol, atol=0.0, maxiter=5000, M=pre,
                            callback=lambda _: it.__setitem__(0, it[0] + 1))
    return it[0], info, x


CASES = {
    "grid32": (I.cfg1, 2000, 1e-3),
    "convdiff": (lambda: I.convdiff3d_7pt(20000, 3.0, (0.6, 0.48, 0.64), 0.8), 128, 1e-4),
    "nonsym": (lambda: I.random_nonsym(20000, seed=41), 64, 1e-4),
}


@pytest.mark.parametrize("precond", [True, False])
@pytest.mark.parametrize("name", sorted(CASES))
def test_bicgstab_matches_scipy(mc, name, precond):
    gen, chains, delta = CASES[name]
    B = gen()
    print(f"[gpu] bicgstab {name} n={B.n} precond={precond}", flush=True)
    dB = mc.DeviceCsr.from_host(B)
    Bs = B.to_scipy()
    b = Bs @ np.ones(B.n)
    M = Ms = None
    if precond:
        M = mc.spai(mc.Cdf(dB), mc.params(seed=0, chains=chains, delta=delta, eps=1e-3))
        rp, col, val = M.to_numpy()
        Ms = sp.csr_matrix((val, col, rp), shape=(B.n, B.n))
    bt = torch.from_numpy(b).cuda()
    x, st = mc.bicgstab(dB, M, bt, rtol=1e-8, maxiter=5000)
    xs = x.cpu().numpy()
    it_ref, info, _ = scipy_iters(Bs, b, Ms)
    print(f"[gpu] bicgstab {name}: device {st.iterations} it (res {st.rel_residual:.2e}), scipy {it_ref}", flush=True)
    assert info == 0 and st.converged == 1
    assert abs(st.iterations - it_ref) <= 1
    true_res = np.linalg.norm(b - Bs @ xs) / np.linalg.norm(b)
    assert true_res <= 1e-7
    assert st.rel_residual <= 1e-8


def test_bicgstab_zero_rhs_and_errors(mc):
    B = I.cfg1()
    dB = mc.DeviceCsr.from_host(B)
    b = torch.zeros(B.n, dtype=torch.float64, device="cuda")
    x, st = mc.bicgstab(dB, None, b, x0=torch.ones(B.n, dtype=torch.float64, device="cuda"))
    assert st.converged == 1 and st.iterations == 0 and float(x.abs().max()) == 0.0
    with pytest.raises(mc.McmiError):
        mc.bicgstab(dB, None, b, rtol=0.0)
    with pytest.raises(mc.McmiError):
        mc.bicgstab(dB, None, b, maxiter=0)


def test_bicgstab_is_deterministic(mc):
    B = I.random_nonsym(5000, seed=42)
    dB = mc.DeviceCsr.from_host(B)
    b = torch.from_numpy(B.to_scipy() @ np.ones(B.n)).cuda()
    x1, s1 = mc.bicgstab(dB, None, b)
    x2, s2 = mc.bicgstab(dB, None, b)
    assert s1.iterations == s2.iterations and torch.equal(x1, x2)
