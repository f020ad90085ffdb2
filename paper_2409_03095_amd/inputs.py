"""Seeded synthetic input matrices B (CSR) for the Monte Carlo SPAI path.

This module only builds input matrices and draws random numbers for them. It
holds none of the method's arithmetic: no iteration matrix, no transition
probabilities, no walks. Both the CPU oracle and the HIP path read the same
arrays produced here, so both sides see identical bits.

Every generator returns a ``Csr`` with int64 row pointers, int32 column
indices (ascending, unique per row) and float64 values; each row holds its
diagonal entry. The paper's test matrices (Section VI, Table I) are not
available, so these families stand in for them with similar row densities:

* ``grid2d_5pt``      - 2D 5-point stencil (rdb2048-like, about 5 entries/row)
* ``random_nonsym``   - random nonsymmetric rows with 5..30 off-diagonals
                        (nonsym_r3_a11-like, about 30 entries/row)
* ``convdiff3d_7pt``  - 3D 7-point convection-diffusion (batched family)
* ``family_5pt``      - 5-point stencil with edge noise and a smooth
                        per-row contraction field (learned-allocation family)
* ``aniso27``         - 3D 27-point anisotropic Q1 stencil (sym_r6_a11-like,
                        about 27 entries/row)
* ``cycle_plus_random`` - allocation control: a deterministic-path block next to
                        a random block
* small pin matrices  - diagonal-only, nilpotent shift, scaled cycle, torus,
                        tiny dense.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Csr:
    n: int
    row_ptr: np.ndarray  # int64, n + 1
    col: np.ndarray      # int32, nnz
    val: np.ndarray      # float64, nnz

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))

    def to_dense(self) -> np.ndarray:
        return self.to_scipy().toarray()


def from_coo(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray) -> Csr:
    """Sort COO triplets by (row, col) and pack them as CSR. Duplicates are an error."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    if rows.size > 1:
        dup = (rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])
        if dup.any():
            raise ValueError("duplicate (row, col) entries")
    counts = np.bincount(rows, minlength=n).astype(np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Csr(n, row_ptr, cols.astype(np.int32), vals)


def from_dense(a: np.ndarray) -> Csr:
    a = np.asarray(a, dtype=np.float64)
    r, c = np.nonzero(a)
    diag = np.arange(a.shape[0])
    missing = np.setdiff1d(diag, r[r == c])
    r = np.concatenate([r, missing])
    c = np.concatenate([c, missing])
    return from_coo(a.shape[0], r, c, a[r, c])


def _with_row_diagonal(n, rows, cols, offv, rho):
    """Append a positive diagonal d_i = sum_j |b_ij| / rho_i to off-diagonal triplets.

    rho may be a scalar or a per-row array. Rows without off-diagonals get d = 1.
    """
    absum = np.bincount(rows, weights=np.abs(offv), minlength=n)
    rho = np.broadcast_to(np.asarray(rho, dtype=np.float64), (n,))
    d = np.where(absum > 0, absum / rho, 1.0)
    i = np.arange(n, dtype=np.int64)
    return from_coo(n, np.concatenate([rows, i]), np.concatenate([cols, i]),
                    np.concatenate([offv, d]))


def _with_uniform_diagonal(n, rows, cols, offv, rho):
    """Append one diagonal value d = max_i sum_j |b_ij| / rho to every row."""
    absum = np.bincount(rows, weights=np.abs(offv), minlength=n)
    d = float(absum.max()) / rho if absum.size and absum.max() > 0 else 1.0
    i = np.arange(n, dtype=np.int64)
    return from_coo(n, np.concatenate([rows, i]), np.concatenate([cols, i]),
                    np.concatenate([offv, np.full(n, d)]))


# ---------------------------------------------------------------- stencils
def _grid_edges_2d(nx, ny, periodic=False):
    """Directed 4-neighbour edges (src, dst) on an nx-by-ny grid, row index x + nx*y."""
    x, y = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    x = x.ravel().astype(np.int64)
    y = y.ravel().astype(np.int64)
    src, dst = [], []
    for dx, dy in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        xx, yy = x + dx, y + dy
        if periodic:
            xx %= nx
            yy %= ny
            ok = np.ones_like(xx, dtype=bool)
        else:
            ok = (xx >= 0) & (xx < nx) & (yy >= 0) & (yy < ny)
        src.append((x + nx * y)[ok])
        dst.append((xx + nx * yy)[ok])
    return np.concatenate(src), np.concatenate(dst)


def grid2d_5pt(nx: int = 32, ny: int = 32, diag: float = 5.0, off: float = -1.0,
               periodic: bool = False) -> Csr:
    """2D 5-point stencil, constant diagonal and off-diagonals (Dirichlet unless periodic)."""
    n = nx * ny
    src, dst = _grid_edges_2d(nx, ny, periodic)
    if periodic and (nx <= 2 or ny <= 2):
        raise ValueError("periodic grid needs nx, ny >= 3 so the 4 neighbours are distinct")
    i = np.arange(n, dtype=np.int64)
    return from_coo(n, np.concatenate([src, i]), np.concatenate([dst, i]),
                    np.concatenate([np.full(src.size, off), np.full(n, diag)]))


def random_nonsym(n: int = 262144, kmin: int = 5, kmax: int = 30, rho: float = 0.7,
                  seed: int = 2) -> Csr:
    """Random nonsymmetric rows: k_i ~ U{kmin..kmax} off-diagonals at distinct uniform
    columns != i, magnitudes lognormal(0, 1), signs +-1 with p = 1/2, and a per-row
    diagonal d_i = sum_j |b_ij| / rho, so every row of C has absolute row sum rho."""
    rng = np.random.default_rng(seed)
    k = rng.integers(kmin, kmax + 1, size=n)
    rows = np.repeat(np.arange(n, dtype=np.int64), k)
    cols = rng.integers(0, n - 1, size=rows.size)
    cols = cols + (cols >= rows)  # skip the diagonal
    # resample duplicate (row, col) pairs until each row's columns are distinct
    for _ in range(100):
        key = rows * n + cols
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup = np.zeros(ks.size, dtype=bool)
        dup[1:] = ks[1:] == ks[:-1]
        if not dup.any():
            break
        bad = order[dup]
        newc = rng.integers(0, n - 1, size=bad.size)
        cols[bad] = newc + (newc >= rows[bad])
    else:
        raise RuntimeError("could not draw distinct columns")
    mag = rng.lognormal(0.0, 1.0, size=rows.size)
    sign = np.where(rng.random(rows.size) < 0.5, -1.0, 1.0)
    return _with_row_diagonal(n, rows, cols, sign * mag, rho)


def _edges_3d(nx, ny, nz, offsets):
    idx = np.arange(nx * ny * nz, dtype=np.int64)
    x = idx % nx
    y = (idx // nx) % ny
    z = idx // (nx * ny)
    out = []
    for off in offsets:
        dx, dy, dz = off
        xx, yy, zz = x + dx, y + dy, z + dz
        ok = (xx >= 0) & (xx < nx) & (yy >= 0) & (yy < ny) & (zz >= 0) & (zz < nz)
        out.append((idx[ok], (xx + nx * (yy + ny * zz))[ok], off))
    return out


def convdiff3d_7pt(n_target: int, peclet: float, velocity, rho: float) -> Csr:
    """3D 7-point central-difference convection-diffusion on nx = ny = floor(n^(1/3)),
    nz = round(n / (nx*ny)). Off-diagonal along axis a, direction s = +-1:
    -1 + s * Pe * v_a / 2 (nonsymmetric, mixed signs for Pe |v_a| > 2); uniform
    diagonal d = max_i sum_j |b_ij| / rho."""
    nx = max(2, int(math.floor(n_target ** (1.0 / 3.0))))
    ny = nx
    nz = max(1, int(round(n_target / (nx * ny))))
    n = nx * ny * nz
    v = np.asarray(velocity, dtype=np.float64)
    rows, cols, vals = [], [], []
    offs = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    for src, dst, off in _edges_3d(nx, ny, nz, offs):
        a = int(np.nonzero(off)[0][0])
        s = float(off[a])
        rows.append(src)
        cols.append(dst)
        vals.append(np.full(src.size, -1.0 + s * peclet * v[a] / 2.0))
    rows, cols, vals = map(np.concatenate, (rows, cols, vals))
    keep = vals != 0.0
    return _with_uniform_diagonal(n, rows[keep], cols[keep], vals[keep], rho)


def convdiff_batch(count: int = 256, seed: int = 3, nmin: float = 1e3, nmax: float = 1e5):
    """The batched family: n log-uniform in [nmin, nmax], Peclet U[0, 5], random unit
    velocity, rho = ||C||_inf U[0.5, 0.85]. Returns (list of Csr, list of dict)."""
    rng = np.random.default_rng(seed)
    mats, meta = [], []
    for _ in range(count):
        n = float(np.exp(rng.uniform(math.log(nmin), math.log(nmax))))
        pe = float(rng.uniform(0.0, 5.0))
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        rho = float(rng.uniform(0.5, 0.85))
        mats.append(convdiff3d_7pt(int(round(n)), pe, v, rho))
        meta.append({"n_target": n, "peclet": pe, "velocity": v.tolist(), "rho": rho})
    return mats, meta


def family_5pt(seed: int, nx: int | None = None, ny: int | None = None) -> Csr:
    """Learned-allocation family: 5-point stencil on nx-by-ny (each U{24..40} unless
    given), off-diagonal -(1 + 0.5 U[-1, 1]) per directed edge, and a per-row
    diagonal d_i = sum_j |b_ij| / rho_i with rho a smooth random field in [0.6, 0.9]."""
    rng = np.random.default_rng(seed)
    if nx is None:
        nx = int(rng.integers(24, 41))
    if ny is None:
        ny = int(rng.integers(24, 41))
    n = nx * ny
    src, dst = _grid_edges_2d(nx, ny)
    offv = -(1.0 + 0.5 * rng.uniform(-1.0, 1.0, size=src.size))
    fx, fy = rng.integers(1, 4, size=2)
    px, py = rng.uniform(0.0, 2.0 * math.pi, size=2)
    x = (np.arange(n) % nx) / nx
    y = (np.arange(n) // nx) / ny
    field = np.cos(2.0 * math.pi * fx * x + px) * np.cos(2.0 * math.pi * fy * y + py)
    rho = 0.75 + 0.15 * field
    return _with_row_diagonal(n, src, dst, offv, rho)


def aniso27(nx: int = 160, kx: float = 1.0, ky: float = 10.0, kz: float = 100.0,
            noise: float = 0.1, rho: float = 0.75, seed: int = 5) -> Csr:
    """3D 27-point Q1 tensor stencil Kx S(x)M(x)M + Ky M(x)S(x)M + Kz M(x)M(x)S with
    S = [-1, 2, -1], M = [1, 4, 1] / 6 on an nx^3 grid (Dirichlet truncation), each
    off-diagonal scaled by 1 + noise U[-1, 1] independently (nonsymmetric), and a
    uniform diagonal d = max_i sum_j |b_ij| / rho."""
    rng = np.random.default_rng(seed)
    S = {-1: -1.0, 0: 2.0, 1: -1.0}
    M = {-1: 1.0 / 6.0, 0: 4.0 / 6.0, 1: 1.0 / 6.0}
    offs = [(a, b, c) for c in (-1, 0, 1) for b in (-1, 0, 1) for a in (-1, 0, 1)
            if (a, b, c) != (0, 0, 0)]
    n = nx ** 3
    rows, cols, vals = [], [], []
    for src, dst, (a, b, c) in _edges_3d(nx, nx, nx, offs):
        w = kx * S[a] * M[b] * M[c] + ky * M[a] * S[b] * M[c] + kz * M[a] * M[b] * S[c]
        rows.append(src)
        cols.append(dst)
        vals.append(np.full(src.size, w))
    rows, cols, vals = map(np.concatenate, (rows, cols, vals))
    vals = vals * (1.0 + noise * rng.uniform(-1.0, 1.0, size=vals.size))
    return _with_uniform_diagonal(n, rows, cols, vals, rho)


def cycle_plus_random(seed: int, scale: int = 1) -> Csr:
    """Allocation control family: two decoupled blocks, a scaled cycle (one entry
    per row of C: every chain from such a row follows the same path) and random
    nonsymmetric rows (5..30 entries), n1, n2 ~ scale * U{500..1499}, common
    ||C||_inf = a ~ U[0.5, 0.8]. Rows differ in how much a chain's path varies at
    equal cost, which is what a per-row chain allocation can exploit."""
    rng = np.random.default_rng(seed)
    n1 = int(rng.integers(500, 1500)) * scale
    n2 = int(rng.integers(500, 1500)) * scale
    a = float(rng.uniform(0.5, 0.8))
    return block_diag([scaled_cycle(n1, a), random_nonsym(n2, rho=a, seed=seed + 7)])


def block_diag(mats) -> Csr:
    """Stack matrices into one block-diagonal CSR (walks never leave their block)."""
    n = sum(m.n for m in mats)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    cols, vals = [], []
    r0 = 0
    base = 0
    for m in mats:
        row_ptr[r0 + 1:r0 + m.n + 1] = m.row_ptr[1:] + base
        cols.append(m.col.astype(np.int64) + r0)
        vals.append(m.val)
        base += m.nnz
        r0 += m.n
    return Csr(n, row_ptr, np.concatenate(cols).astype(np.int32), np.concatenate(vals))


# ---------------------------------------------------------------- pin matrices
def nonddm(n: int, seed: int, k: int = 6) -> Csr:
    """A general (not diagonally dominant) sparse B for the augmented splitting:
    k off-diagonals per row at distinct random columns, lognormal(0, 1) magnitudes
    with random signs, diagonals of random sign and magnitude in [0.1, 1]; row 1
    stores an explicit zero diagonal and row 2 stores no diagonal at all."""
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    for i in range(n):
        others = rng.choice(n - 1, size=min(k, n - 1), replace=False)
        others = others + (others >= i)
        mags = rng.lognormal(0.0, 1.0, size=others.size) * np.where(rng.random(others.size) < 0.5, -1.0, 1.0)
        rows.extend([i] * others.size)
        cols.extend(others.tolist())
        vals.extend(mags.tolist())
        if i == 2:
            continue
        d = 0.0 if i == 1 else rng.uniform(0.1, 1.0) * (-1.0 if rng.random() < 0.5 else 1.0)
        rows.append(i)
        cols.append(i)
        vals.append(d)
    return from_coo(n, np.array(rows), np.array(cols), np.array(vals))


def wide_rows(n: int, widths: dict, seed: int = 0, rho: float = 0.7) -> Csr:
    """random_nonsym-style rows (5..30 off-diagonals) except the rows in `widths`,
    which get that many off-diagonals at distinct uniform columns (n - 1: every
    other column); per-row diagonal sum_j |b_ij| / rho."""
    rng = np.random.default_rng(seed)
    k = rng.integers(5, 31, size=n)
    for r, m in widths.items():
        k[r] = m
    rows, cols = [], []
    for r in range(n):
        c = rng.choice(n - 1, size=int(k[r]), replace=False)
        cols.append(c + (c >= r))
        rows.append(np.full(int(k[r]), r, dtype=np.int64))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols).astype(np.int64)
    mag = rng.lognormal(0.0, 1.0, size=rows.size)
    sign = np.where(rng.random(rows.size) < 0.5, -1.0, 1.0)
    return _with_row_diagonal(n, rows, cols, sign * mag, rho)


def diag_only(n: int, seed: int = 0) -> Csr:
    """B diagonal (so C = 0), diagonal values of both signs."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(0.5, 4.0, size=n) * np.where(rng.random(n) < 0.5, -1.0, 1.0)
    i = np.arange(n)
    return from_coo(n, i, i, d)


def nilpotent_shift(n: int, seed: int = 0, amax: float = 0.9) -> Csr:
    """B = D - D*U with U the strictly upper shift scaled by random signed a_i:
    row i has one off-diagonal at column i + 1 (none in the last row), so C is
    nilpotent with c_{i,i+1} = a_i."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(0.5, 3.0, size=n) * np.where(rng.random(n) < 0.5, -1.0, 1.0)
    a = rng.uniform(0.2, amax, size=n - 1) * np.where(rng.random(n - 1) < 0.5, -1.0, 1.0)
    i = np.arange(n - 1)
    rows = np.concatenate([np.arange(n), i])
    cols = np.concatenate([np.arange(n), i + 1])
    vals = np.concatenate([d, -a * d[:-1]])
    return from_coo(n, rows, cols, vals)


def scaled_cycle(n: int, a: float, d: float = 2.0) -> Csr:
    """B = d (I - a P) with P the cyclic shift i -> i+1 mod n (C = a P)."""
    i = np.arange(n)
    return from_coo(n, np.concatenate([i, i]), np.concatenate([i, (i + 1) % n]),
                    np.concatenate([np.full(n, d), np.full(n, -a * d)]))


def dense_small(n: int, norm: float, seed: int, signed: bool = True) -> Csr:
    """Tiny dense B = D (I - C) with random C of infinity norm <= `norm` and random
    positive/negative diagonal D."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.1, 1.0, size=(n, n))
    if signed:
        c *= np.where(rng.random((n, n)) < 0.5, -1.0, 1.0)
    np.fill_diagonal(c, 0.0)
    c *= (norm * rng.uniform(0.6, 1.0, size=(n, 1))) / np.abs(c).sum(axis=1, keepdims=True)
    d = rng.uniform(0.5, 3.0, size=n) * np.where(rng.random(n) < 0.5, -1.0, 1.0)
    b = d[:, None] * (np.eye(n) - c)
    return from_dense(b)


# ---------------------------------------------------------------- named configs
def cfg1() -> Csr:
    """2D 5-point, 32 x 32, diagonal 5, off-diagonals -1 (||C||_inf = 0.8)."""
    return grid2d_5pt(32, 32, 5.0, -1.0)


def cfg2(n: int = 262144) -> Csr:
    """Random nonsymmetric, n = 262144, 5..30 off-diagonals/row, ||C||_inf = 0.7."""
    return random_nonsym(n, 5, 30, 0.7, seed=2)


def cfg5(nx: int = 160) -> Csr:
    """3D 27-point anisotropic (1:10:100), +-10% noise, ||C||_inf = 0.75, 160^3 grid."""
    return aniso27(nx, 1.0, 10.0, 100.0, 0.1, 0.75, seed=5)


def cfg4_train(count: int = 2000, seed0: int = 1000):
    return [family_5pt(seed0 + k) for k in range(count)]


def cfg4_heldout(nx: int = 1024, seed: int = 999_999) -> Csr:
    return family_5pt(seed, nx, nx)


def chain_counts(n: int, mean: float = 12.0, seed: int = 41, lo: int = 1, hi: int = 96) -> np.ndarray:
    """Per-row chain counts shaped like an allocation that moves chains between
    rows: log-normal with sigma 0.6 scaled to the given mean, rounded, clipped to
    [lo, hi] (int32). A test input only: both sides read the same array."""
    rng = np.random.default_rng(seed)
    x = rng.lognormal(0.0, 0.6, size=n)
    return np.clip(np.rint(x * (mean / x.mean())), lo, hi).astype(np.int32)
