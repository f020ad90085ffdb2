"""Host-side checks that need no GPU: the synthetic input recipes have the
structure the workloads promise (row counts, patterns, contraction norms,
determinism), the benchmark refuses more than one GPU before touching a device,
and the learned-allocation crossing interpolation is exact on a power law."""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2409_03095_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def c_abs_row_sums(B):
    """sum_j |b_ij| / |b_ii| over j != i (the row sums of |C|), in numpy."""
    S = B.to_scipy().tocsr()
    d = S.diagonal()
    absS = abs(S)
    return (np.asarray(absS.sum(axis=1)).ravel() - np.abs(d)) / np.abs(d)


def check_csr(B):
    rp, col = B.row_ptr, B.col
    assert rp.dtype == np.int64 and col.dtype == np.int32 and B.val.dtype == np.float64
    assert rp[0] == 0 and rp[-1] == col.size == B.val.size
    for r in range(0, B.n, max(1, B.n // 257)):
        c = col[rp[r]:rp[r + 1]]
        assert np.all(np.diff(c) > 0) and c[0] >= 0 and c[-1] < B.n


def test_random_nonsym_recipe():
    B = I.random_nonsym(4000, seed=7)
    check_csr(B)
    off = np.diff(B.row_ptr) - 1
    assert off.min() >= 5 and off.max() <= 30
    S = B.to_scipy().tocsr()
    assert np.all(S.diagonal() != 0.0)
    np.testing.assert_allclose(c_abs_row_sums(B), 0.7, rtol=1e-12)
    # nonsymmetric pattern, mixed signs
    assert (S != S.T).nnz > 0
    offv = S.copy()
    offv.setdiag(0.0)
    offv.eliminate_zeros()
    assert (offv.data > 0).any() and (offv.data < 0).any()
    B2 = I.random_nonsym(4000, seed=7)
    assert np.array_equal(B.col, B2.col) and np.array_equal(B.val, B2.val)


def test_grid_recipe_matches_the_small_workload():
    B = I.cfg1()
    check_csr(B)
    assert B.n == 1024 and B.nnz == 4992
    S = B.to_scipy().tocsr()
    assert np.all(S.diagonal() == 5.0)
    offv = S.copy()
    offv.setdiag(0.0)
    offv.eliminate_zeros()
    assert np.all(offv.data == -1.0)
    assert c_abs_row_sums(B).max() == pytest.approx(0.8, abs=0.0)


def test_aniso27_recipe():
    nx = 10
    B = I.aniso27(nx, seed=5)
    check_csr(B)
    assert B.n == nx ** 3
    cnt = np.diff(B.row_ptr)
    idx = np.arange(B.n)
    x, y, z = idx % nx, (idx // nx) % nx, idx // (nx * nx)
    interior = (x > 0) & (x < nx - 1) & (y > 0) & (y < nx - 1) & (z > 0) & (z < nx - 1)
    assert np.all(cnt[interior] == 27) and cnt.min() == 8
    assert c_abs_row_sums(B).max() == pytest.approx(0.75, rel=1e-12)
    S = B.to_scipy().tocsr()
    assert abs(S - S.T).max() > 0.0  # coefficient noise makes it nonsymmetric
    # anisotropy 1:10:100 through the Q1 mass factors: the z face coupling is the
    # largest and negative (Kz S_z M_x M_y = -100 * 16/36 = -44.4 before the other
    # two terms and the noise), the x face coupling is positive
    r = int(np.flatnonzero(interior)[0])
    row = S.getrow(r).toarray().ravel()
    assert row[r + nx * nx] < 0.0 < row[r + 1]
    assert abs(row[r + nx * nx]) > 1.5 * abs(row[r + 1])


def test_convdiff_batch_recipe():
    mats, meta = I.convdiff_batch(count=24, seed=3)
    assert len(mats) == 24
    for B, m in zip(mats, meta):
        check_csr(B)
        assert 1e3 * 0.8 <= B.n <= 1e5 * 1.2
        assert 0.5 <= m["rho"] <= 0.85 and 0.0 <= m["peclet"] <= 5.0
        assert np.diff(B.row_ptr).max() <= 7
        assert c_abs_row_sums(B).max() == pytest.approx(m["rho"], rel=1e-12)
    ns = np.array([m["n_target"] for m in meta])
    assert ns.min() >= 1e3 and ns.max() <= 1e5


def test_nonddm_has_the_two_degenerate_rows():
    B = I.nonddm(50, seed=4)
    S = B.to_scipy().tocsr()
    assert S[1, 1] == 0.0 and 1 in S.getrow(1).indices  # explicit zero diagonal
    assert 2 not in S.getrow(2).indices  # no diagonal entry at all


def test_bench_refuses_more_than_one_gpu():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120, cwd=ROOT)
    assert out.returncode == 2
    assert "one GPU" in out.stderr or "single MI355X" in out.stderr
    assert out.stdout == ""


def test_crossing_interpolates_a_power_law_exactly():
    from paper_2409_03095_amd import learned as L
    # r = 3 * T^-0.5 crosses 0.3 at T = 100 exactly in log-log
    pts = [{"transitions": t, "r_norm": 3.0 * t ** -0.5} for t in (10.0, 50.0, 400.0, 1000.0)]
    assert L.crossing(pts, "transitions") == pytest.approx(100.0, rel=1e-12)
    assert L.crossing([{"transitions": 1.0, "r_norm": 0.1}], "transitions") is None


def test_cycle_plus_random_recipe():
    B = I.cycle_plus_random(5)
    check_csr(B)
    m = np.diff(B.row_ptr) - 1
    S = B.to_scipy().tocsr()
    n1 = int(np.argmax(m > 1))  # the cycle block comes first: one entry of C per row
    assert n1 >= 500 and np.all(m[:n1] == 1) and np.all(m[n1:] >= 5)
    assert S[:n1, n1:].nnz == 0 and S[n1:, :n1].nnz == 0  # decoupled blocks
    sums = c_abs_row_sums(B)
    np.testing.assert_allclose(sums, sums[0], rtol=1e-12)  # one ||C||_inf for both blocks
    assert 0.5 <= sums[0] <= 0.8


def test_wide_rows_recipe():
    B = I.wide_rows(2001, {0: 2000, 7: 900}, seed=3)
    check_csr(B)
    m = np.diff(B.row_ptr) - 1
    assert m[0] == 2000 and m[7] == 900
    rest = np.delete(m, [0, 7])
    assert rest.min() >= 5 and rest.max() <= 30
    np.testing.assert_allclose(c_abs_row_sums(B), 0.7, rtol=1e-12)
