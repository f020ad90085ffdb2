"""GPU parity of the learned-allocation parts (row features, pilot variance, the
BF16 network's forward, gradient and training, the allocation, the quality
sample) and what the trained network gains over uniform chains."""
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


def test_neyman_target_matches_oracle(mc):
    """mcmi_neyman_target against the oracle's target on the same float64 inputs,
    incl. zero and subnormal variances (floored at 1e-30) and zero lengths: the
    binary32 result is within one rounding (2^-24 relative) of the FP64 value,
    plus 1e-12 for the last bits of the two logarithms."""
    rng = np.random.default_rng(4)
    n = 100003
    var = rng.lognormal(-2.0, 3.0, size=n)
    var[:50] = 0.0
    var[50:60] = 1e-310
    ln = rng.uniform(0.0, 40.0, size=n)
    ln[::7] = 0.0
    y = mc.neyman_target(torch.from_numpy(var).cuda(), torch.from_numpy(ln).cuda()).cpu().numpy()
    ref = O.neyman_target(var, ln)
    assert np.all(np.abs(y.astype(np.float64) - ref) <= np.abs(ref) * 2.0 ** -24 + 1e-12)


@pytest.mark.parametrize("name", ["family", "nonsym"])
def test_pilot_target_matches_oracle(mc, name):
    """Pilot run then target on the device against the oracle's pilot and target:
    the variances agree to 1e-10 relative (different summation order), so the
    targets agree to one binary32 rounding plus 1e-10."""
    B = MATS[name]()
    cdf = mc.Cdf(mc.DeviceCsr.from_host(B))
    var, ln = mc.pilot_variance(cdf, mc.params(seed=3, delta=1e-4, tag=2), 64)
    y = mc.neyman_target(var, ln).cpu().numpy().astype(np.float64)
    rv, rl = O.Oracle(B).pilot(seed=3, pilot=64, delta=1e-4, tag=2)
    ref = O.neyman_target(rv, rl)
    assert np.all(np.abs(y - ref) <= np.abs(ref) * 2.0 ** -24 + 1e-10)


@pytest.mark.parametrize("name", sorted(MATS))
def test_chain_cost_matches_oracle(mc, name):
    """mcmi_chain_cost against the oracle's chain cost of the same stored f7
    (the integer decision taken on the binary32 feature on both sides): equal per
    row and in total."""
    B = MATS[name]()
    cdf = mc.Cdf(mc.DeviceCsr.from_host(B))
    feat = mc.row_features(cdf, 1e-3)
    cost, total = mc.chain_cost(feat)
    ref = O.chain_cost(feat[:, 7].cpu().numpy())
    assert np.array_equal(cost.cpu().numpy().astype(np.int64), ref)
    assert total == int(ref.sum())


def test_chain_cost_total_over_many_rows(mc):
    """3,000,017 rows (a ragged grid) with f7 spread over [0, 65]: exact 64-bit total."""
    rng = np.random.default_rng(6)
    n = 3_000_017
    feat = np.zeros((n, 8), dtype=np.float32)
    feat[:, 7] = rng.uniform(0.0, 65.0, size=n).astype(np.float32)
    feat[::11, 7] = np.floor(feat[::11, 7])
    cost, total = mc.chain_cost(torch.from_numpy(feat).cuda())
    ref = O.chain_cost(feat[:, 7])
    assert np.array_equal(cost.cpu().numpy().astype(np.int64), ref) and total == int(ref.sum())
    empty, tot0 = mc.chain_cost(torch.zeros((0, 8), dtype=torch.float32, device="cuda"))
    assert empty.numel() == 0 and tot0 == 0


# ---------------------------------------------------------------- MLP (a13)
def flat(p):
    return np.concatenate([p[k].reshape(-1) for k, _ in O.MLP_SHAPES]).astype(np.float32)


def unflat(v):
    out, o = {}, 0
    for k, shape in O.MLP_SHAPES:
        size = int(np.prod(shape))
        out[k] = v[o:o + size].reshape(shape)
        o += size
    return out


def bf16_params(p):
    q = {k: v.astype(np.float64) for k, v in p.items()}
    for k in ("w1", "w2", "w3"):
        q[k] = O.bf16_round(p[k]).astype(np.float64)
    return q


@pytest.fixture(scope="module")
def net_case():
    rng = np.random.default_rng(5)
    p = O.mlp_init(11)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.normal(0, 0.1, size=p[k].shape).astype(np.float32)
    n = 1000  # not a multiple of the 16-sample tile
    x = rng.normal(1.0, 2.0, size=(n, 8)).astype(np.float32)
    mean = x.mean(axis=0).astype(np.float32)
    inv = (1.0 / x.std(axis=0)).astype(np.float32)
    t = rng.normal(0, 1, size=n).astype(np.float32)
    xn = O.bf16_round(((x - mean) * inv).astype(np.float32)).astype(np.float64)
    return p, x, mean, inv, t, xn


def test_mlp_forward_matches_reference(mc, net_case):
    p, x, mean, inv, t, xn = net_case
    net = mc.Mlp()
    net.set_params(flat(p), np.concatenate([mean, inv]))
    y = net.predict(torch.from_numpy(x).cuda()).cpu().numpy()
    ref, _ = O.mlp_forward(bf16_params(p), xn)
    err = np.abs(y - ref)
    assert err.max() <= 2e-2 * np.abs(ref).max(), (err.max(), np.abs(ref).max())
    assert np.linalg.norm(y - ref) <= 1e-2 * np.linalg.norm(ref)


def test_mlp_gradient_matches_reference(mc, net_case):
    """BF16 forward/backward on the matrix cores vs the FP64 reference on the same
    BF16-rounded weights and inputs: relative error in norm per parameter block."""
    p, x, mean, inv, t, xn = net_case
    net = mc.Mlp()
    net.set_params(flat(p), np.concatenate([mean, inv]))
    idx = np.random.default_rng(3).choice(x.shape[0], 333, replace=False).astype(np.int32)
    g, loss = net.gradient(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda(), torch.from_numpy(idx).cuda())
    rl, rg = O.mlp_loss_grad(bf16_params(p), xn[idx], t[idx])
    assert abs(loss - rl) <= 1e-2 * rl
    gg = unflat(g)
    for k, _ in O.MLP_SHAPES:
        num = np.linalg.norm(gg[k].reshape(-1) - rg[k].reshape(-1))
        den = np.linalg.norm(rg[k].reshape(-1))
        assert num <= 2e-2 * den + 1e-7, (k, num / max(den, 1e-30))


def test_mlp_training_reduces_loss_and_checkpoints(mc):
    rng = np.random.default_rng(8)
    n = 20000
    x = rng.normal(0, 1, size=(n, 8)).astype(np.float32)
    t = (np.sin(x[:, 0]) + 0.5 * x[:, 1] * x[:, 2] - 0.3 * np.abs(x[:, 3])).astype(np.float32)
    net = mc.Mlp()
    net.set_params(flat(O.mlp_init(2)))
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    net.fit_normalization(xd)
    losses = net.train(xd, td, steps=600, batch=1024, lr=3e-3, seed=4)
    assert np.all(np.isfinite(losses))
    assert losses[-50:].mean() < 0.25 * losses[:10].mean(), (losses[:10].mean(), losses[-50:].mean())
    ck = net.get_params()
    assert ck["step"] == 600
    net2 = mc.Mlp()
    net2.set_params(ck["params"], ck["norm"])
    net2.set_adam_state(ck["adam_m"], ck["adam_v"], ck["step"])
    y1 = net.predict(xd).cpu().numpy()
    y2 = net2.predict(xd).cpu().numpy()
    assert np.array_equal(y1, y2)


def test_adam_steps_match_oracle(mc):
    """25 Adam steps of k_adam (FP32 moments and master weights) against the
    oracle's FP64 Adam on the same gradients (some entries zero at some steps,
    scales from 1e-3 to 10). Tolerance from FP32 arithmetic, per step t: the
    stored weight is rounded (2^-24 |p_t|) and the update u_t carries the
    binary32 rounding of beta2 (|fl(0.999) - 0.999| / (1 - 0.999) = 1.3e-5
    relative in 1 - beta2 and in the bias correction) plus about ten binary32
    operations, 3e-5 |u_t| in all; summed over the steps."""
    rng = np.random.default_rng(21)
    p0 = O.mlp_init(4)
    for k in ("b1", "b2", "b3"):
        p0[k] = rng.normal(0, 0.2, size=p0[k].shape).astype(np.float32)
    net = mc.Mlp()
    net.set_params(flat(p0))
    lr = 3e-3
    ref = {k: v.astype(np.float64) for k, v in p0.items()}
    state = {}
    tol = np.zeros(flat(p0).size)
    tol_m = np.zeros(flat(p0).size)
    m_prev = np.zeros(flat(p0).size)
    for t in range(25):
        scale = 10.0 ** rng.uniform(-3, 1, size=flat(p0).size)
        g = (rng.normal(0, 1, size=scale.size) * scale).astype(np.float32)
        g[rng.random(g.size) < 0.05] = 0.0
        net.adam_step(torch.from_numpy(g).cuda(), lr)
        new = O.adam_step(ref, {k: v.astype(np.float64) for k, v in unflat(g).items()}, state, lr=lr)
        u = np.abs(flat({k: new[k] - ref[k] for k in ref}).astype(np.float64))
        ref = new
        tol += 2.0 ** -24 * np.abs(flat(ref).astype(np.float64)) + 3e-5 * u
        # first moment: fl(0.9) is 2.7e-8 and fl(1 - fl(0.9)) 2.4e-7 off in relative
        # terms, each product and the sum round once (2^-24); the carried error
        # decays by beta1; a factor 2 of slack. Absolute, since m cancels.
        m_now = np.concatenate([state["m_" + k].reshape(-1) for k, _ in O.MLP_SHAPES])
        tol_m = 0.9 * tol_m + 2.0 * (9e-8 * 0.9 * np.abs(m_prev) + 3e-7 * 0.1 * np.abs(g.astype(np.float64))
                                     + 6e-8 * np.abs(m_now))
        m_prev = m_now
    ck = net.get_params()
    got = ck["params"].astype(np.float64)
    want = np.concatenate([ref[k].reshape(-1) for k, _ in O.MLP_SHAPES])
    err = np.abs(got - want)
    assert ck["step"] == 25
    assert np.all(err <= tol + 1e-12), (err.max(), np.argmax(err - tol))
    m_ref = np.concatenate([state["m_" + k].reshape(-1) for k, _ in O.MLP_SHAPES])
    v_ref = np.concatenate([state["v_" + k].reshape(-1) for k, _ in O.MLP_SHAPES])
    err_m = np.abs(ck["adam_m"].astype(np.float64) - m_ref)
    assert np.all(err_m <= tol_m + 1e-30), (err_m.max(), np.argmax(err_m - tol_m))
    assert np.allclose(ck["adam_v"], v_ref, rtol=3e-5, atol=1e-20)
    # the BF16 copies follow the masters: the network's prediction equals one made
    # from a fresh network loaded with the same masters
    x = torch.from_numpy(rng.normal(0, 1, size=(300, 8)).astype(np.float32)).cuda()
    net2 = mc.Mlp()
    net2.set_params(ck["params"])
    assert np.array_equal(net.predict(x).cpu().numpy(), net2.predict(x).cpu().numpy())


@pytest.mark.parametrize("n", [1, 5000, 400000])
def test_allocation_matches_reference(mc, n):
    """Grid-wide bisection on the device vs the sequential numpy reference."""
    rng = np.random.default_rng(9)
    pred = rng.normal(0, 0.7, size=n).astype(np.float32)
    cost = rng.integers(5, 40, size=n).astype(np.int32)
    budget = int(24 * cost.sum())
    chains, lam, fb = mc.allocate(torch.from_numpy(pred).cuda(), torch.from_numpy(cost).cuda(), budget)
    chains = chains.cpu().numpy()
    assert not fb
    ref, rlam = O.allocate(pred.astype(np.float64), cost, budget)
    assert (chains.astype(np.int64) * cost).sum() <= budget
    assert abs(lam - rlam) <= 1e-9 * rlam
    assert np.mean(chains != ref) < 1e-3 and np.max(np.abs(chains - ref)) <= 1
    bad = pred.copy()
    bad[min(7, n - 1)] = np.nan
    chains, lam, fb = mc.allocate(torch.from_numpy(bad).cuda(), torch.from_numpy(cost).cuda(), budget)
    assert fb and np.all(chains.cpu().numpy() == budget // cost.sum())


def test_quality_sample_matches_oracle_residual(mc):
    """The learned-allocation quality estimate: rows of M gathered on the device
    equal the full download's rows, and the sampled ||e_r - M_r B||^2 equals the
    oracle's residual rows of the same M."""
    import scipy.sparse as sp
    from paper_2409_03095_amd import learned as L
    B = I.family_5pt(7, 30, 34)
    dB = mc.DeviceCsr.from_host(B)
    res = mc.spai(mc.Cdf(dB), mc.params(seed=2, chains=24, delta=1e-3, eps=1e-3))
    rp, col, val = res.to_numpy()
    rows = np.sort(np.random.default_rng(0).choice(B.n, 200, replace=False))
    srp, scol, sval = L.sample_rows(res, rows)
    for t, r in enumerate(rows):
        assert np.array_equal(scol[srp[t]:srp[t + 1]], col[rp[r]:rp[r + 1]])
        assert np.array_equal(sval[srp[t]:srp[t + 1]], val[rp[r]:rp[r + 1]])
    got = L.residual_sample(B, srp, scol, sval, rows)
    Msub = sp.csr_matrix((sval, scol, srp), shape=(rows.size, B.n))
    ref = O.residual_rows(B, Msub, rows)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-15)


# ------------------------------------------------ what the network gains
@pytest.mark.parametrize("family", ["cycle_plus_random", "family_5pt"])
def test_learned_allocation_against_uniform(mc, family):
    """Train the network on pilot variance of 40 matrices of a family and compare
    learned vs uniform chains on a held-out matrix at equal total transitions
    (||I - M B||_F / sqrt(n) on a 4000-row sample, 95 % intervals).
    cycle_plus_random (half the rows follow one deterministic path, so one chain
    estimates them exactly): the learned allocation moves chains to the random
    rows and wins with disjoint intervals at every budget. family_5pt (the
    grid family of the learned-allocation workload: per-row variance and chain
    cost both grow like 1 / (1 - rho_i), so the best allocation is nearly
    uniform): the two agree within their intervals."""
    from paper_2409_03095_amd import learned as L
    gen = I.cycle_plus_random if family == "cycle_plus_random" else I.family_5pt
    train = [gen(1000 + s) for s in range(40)]
    held = I.cycle_plus_random(99, scale=20) if family == "cycle_plus_random" else I.family_5pt(555, 200, 200)
    print(f"[gpu] learned vs uniform on {family}: train rows {sum(m.n for m in train)}, held-out n={held.n}",
          flush=True)
    net, info = L.train_allocator(train, 1e-3, steps=3000)
    assert info["loss_last"] < info["loss_first"]
    pts = L.compare(net, held, 1e-3, 1e-3, [2, 8], n_sample=4000)
    for p in pts:
        lr, ur = p["learned"], p["uniform"]
        print(f"  mean chains {p['mean_chains']}: learned {lr['r_norm']:.4f} [{lr['r_norm_lo']:.4f}, "
              f"{lr['r_norm_hi']:.4f}] at {lr['transitions']} | uniform {ur['r_norm']:.4f} "
              f"[{ur['r_norm_lo']:.4f}, {ur['r_norm_hi']:.4f}] at {ur['transitions']}", flush=True)
        assert not p["fallback"]
        assert abs(lr["transitions"] - ur["transitions"]) <= 0.01 * ur["transitions"]
        if family == "cycle_plus_random":
            assert lr["r_norm_hi"] < ur["r_norm_lo"]
        else:
            assert lr["r_norm_lo"] <= ur["r_norm_hi"] and ur["r_norm_lo"] <= lr["r_norm_hi"]
