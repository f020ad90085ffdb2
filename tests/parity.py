"""Helpers for comparing the HIP library with the oracle (test code only)."""
import numpy as np

U64 = 2.0 ** -53


def decode_records(rec, roff, n):
    """Decode the library's records (64-byte units: header {row, m, W, S32},
    {S64, 0, 0} and zeros, then one bucket per entry: {T, target, alias target,
    w}, the target's header words, the alias target's header words, their S64s)
    into per-row (row, m, W, S32, S64, cum[], col[], neg[], thr[], alias_col[],
    alias_neg[]) in column order, checking padding and every copied header."""
    inv = {int(o): i for i, o in enumerate(roff)}
    out = []
    for i in range(n):
        base = int(roff[i]) * 16
        row, m, W = int(rec[base]), int(rec[base + 1]), int(rec[base + 2])
        s32 = rec[base + 3:base + 4].view(np.float32)[0]
        s64 = rec[base + 4:base + 6].view(np.float64)[0]
        assert not rec[base + 6:base + 16].any(), ("header padding", i)
        ent = rec[base + 16:base + 16 + 16 * m].reshape(m, 16)
        thr, tg, al, w = (ent[:, k].astype(np.int64) for k in range(4))
        for k in range(m):
            for t, words, sw in ((int(tg[k]), ent[k, 4:8], ent[k, 12:14]), (int(al[k]), ent[k, 8:12], ent[k, 14:16])):
                hb = (t & 0x7FFFFFFF) * 16
                assert np.array_equal(words, rec[hb:hb + 4]), ("copied header", i, k)
                assert np.array_equal(sw, rec[hb + 4:hb + 6]), ("copied Shat64", i, k)
        cum = np.cumsum(w)
        col = np.array([inv[int(t) & 0x7FFFFFFF] for t in tg], dtype=np.int64)
        neg = (tg >> 31) & 1 == 1
        acol = np.array([inv[int(t) & 0x7FFFFFFF] for t in al], dtype=np.int64)
        aneg = (al >> 31) & 1 == 1
        out.append((row, m, W, s32, s64, cum, col, neg, thr, acol, aneg))
    return out


def compare_spai(gpu, orc, diag, chains, rel=1e-12, rows=None, check_pattern=True):
    """Pattern must be identical; each value within rel * |oracle| or the FP64
    summation-order bound 4 (k + 2) u sum|W| / (N |d_c|) (the two sides add the
    same terms in different orders)."""
    rp, col, val = gpu
    assert rp.size == orc["row_ptr"].size
    if check_pattern:
        assert np.array_equal(rp, orc["row_ptr"]), "row lengths differ"
        assert np.array_equal(col, orc["col"]), "columns differ"
    nrows = rp.size - 1
    N = np.broadcast_to(np.asarray(chains, dtype=np.float64), (diag.size,))
    row_of_entry = np.repeat(np.arange(nrows), np.diff(orc["row_ptr"]))
    grow = row_of_entry if rows is None else np.asarray(rows)[row_of_entry]
    bound = 4.0 * (orc["cnt"] + 2.0) * U64 * orc["abssum"] / N[grow] / np.abs(diag[orc["col"]])
    tol = np.maximum(rel * np.abs(orc["val"]), bound)
    err = np.abs(val - orc["val"])
    bad = np.nonzero(err > tol)[0]
    assert bad.size == 0, f"{bad.size} values out of tolerance, worst {err[bad].max()} vs {tol[bad].min()}"
    return float((err / np.maximum(np.abs(orc["val"]), 1e-300)).max()) if err.size else 0.0


def common_entries(rp_a, col_a, val_a, rp_b, col_b, val_b):
    """Values of two CSR matrices on their common pattern."""
    va, vb = [], []
    for r in range(rp_a.size - 1):
        ca = col_a[rp_a[r]:rp_a[r + 1]]
        cb = col_b[rp_b[r]:rp_b[r + 1]]
        _, ia, ib = np.intersect1d(ca, cb, assume_unique=True, return_indices=True)
        va.append(val_a[rp_a[r]:rp_a[r + 1]][ia])
        vb.append(val_b[rp_b[r]:rp_b[r + 1]][ib])
    return np.concatenate(va), np.concatenate(vb)


def compare_topk(gpu, orc, diag, chains):
    """Top-k retention: rows whose boundary the oracle marks order-dependent
    (row_ambig) must keep as many entries, with equal values on the columns both
    keep; every other row must match as in compare_spai."""
    rp, col, val = gpu
    orp = orc["row_ptr"]
    amb = orc["row_ambig"].astype(bool)
    assert np.array_equal(np.diff(rp), np.diff(orp)), "row lengths differ"
    clean = np.nonzero(~amb)[0]

    def sub(r_p, arrays, rows):
        lens = r_p[rows + 1] - r_p[rows]
        idx = np.concatenate([np.arange(r_p[r], r_p[r + 1]) for r in rows]) if rows.size else np.zeros(0, int)
        return np.concatenate([[0], np.cumsum(lens)]), [a[idx] for a in arrays]

    g_rp, (g_col, g_val) = sub(rp, [col, val], clean)
    o_rp, (o_col, o_val, o_abs, o_cnt) = sub(orp, [orc["col"], orc["val"], orc["abssum"], orc["cnt"]], clean)
    ref = {"row_ptr": o_rp, "col": o_col, "val": o_val, "abssum": o_abs, "cnt": o_cnt}
    err = compare_spai((g_rp, g_col, g_val), ref, diag, chains, rows=clean)
    for r in np.nonzero(amb)[0]:
        gc, gv = col[rp[r]:rp[r + 1]], val[rp[r]:rp[r + 1]]
        sl = slice(orp[r], orp[r + 1])
        oc, ov = orc["col"][sl], orc["val"][sl]
        _, ia, ib = np.intersect1d(gc, oc, return_indices=True)
        bound = 4.0 * (orc["cnt"][sl][ib] + 2.0) * U64 * orc["abssum"][sl][ib] / chains / np.abs(diag[oc[ib]])
        tol = np.maximum(1e-12 * np.abs(ov[ib]), bound)
        assert np.all(np.abs(gv[ia] - ov[ib]) <= tol), ("ambiguous row values", r)
    return err, int(amb.sum())


U32 = 2.0 ** -24


def fp32_walks_against_fp64(n, gpu, rows, orc64, o, chains, eps, delta, rerun):
    """FP32 walks (binary32 weights and Shat32, binary64 sums) against the FP64
    oracle on sampled rows. The draws do not depend on the weights, so the two
    walks follow the same paths and differ in two ways only:
      * a step-j weight by at most 2 j u32 |W_j| (j binary32 products, each with
        the rounding of Shat to binary32);
      * a chain whose cutoff test lies inside that band (the oracle counts them
        per row: row_border = D_r) may stop one step earlier or later, adding or
        missing one contribution of magnitude at most delta (1 + 2^-10) (one step,
        as ||Chat||_inf < 1 - 2^-16 takes the next weight below delta).
    So an entry may differ by B32 = ((2 L u32 (1 + 2^-10) + 4 (k + 2) u64) sum|W|
    + D_r delta (1 + 2^-10)) / (N |d_c|) (L: the longest chain, k: contributions),
    which where contributions cancel exceeds any relative bar. Checked:
      * every common entry within max(1e-5 |v64|, B32);
      * an entry kept by one side only lies within B32 |d_c| of eps (kept or
        dropped by rounding): `rerun(rows)` must give the FP64 oracle's run of
        those rows with eps = 0, from which such entries' sums are read (an entry
        no FP64 chain reached counts as 0 with no contributions).
    Returns (common entries, worst relative error, entries beyond 1e-5 relative,
    pattern differences, chains near the cutoff)."""
    rp, col, val = gpu
    L = int(orc64["lmax"])
    N = np.broadcast_to(np.asarray(chains, dtype=np.float64), (n,))
    rows = np.asarray(rows)
    D = orc64["row_border"].astype(np.float64)
    assert o.norm_inf < 1.0 - 2.0 ** -16
    wb = 2.0 * L * U32 * (1.0 + 2.0 ** -10)

    def keyed(r_p, c):
        return np.repeat(np.arange(r_p.size - 1, dtype=np.int64), np.diff(r_p)) * n + c

    kg, ko = keyed(rp, col), keyed(orc64["row_ptr"], orc64["col"])
    common, ig, io = np.intersect1d(kg, ko, assume_unique=True, return_indices=True)
    loc = ko[io] // n
    dcol = np.abs(o.diag[orc64["col"][io]])
    b32 = ((wb + 4.0 * (orc64["cnt"][io] + 2.0) * U64) * orc64["abssum"][io] + D[loc] * delta * (1.0 + 2.0 ** -10)) \
        / N[rows[loc]] / dcol
    v64 = orc64["val"][io]
    err = np.abs(val[ig] - v64)
    rel = err / np.abs(v64)
    bad = np.nonzero(err > np.maximum(1e-5 * np.abs(v64), b32))[0]
    assert bad.size == 0, f"{bad.size} FP32 values beyond the bound, worst {err[bad].max()}"
    only = np.setxor1d(kg, ko, assume_unique=True)
    if only.size:
        local = np.unique(only // n)
        full = rerun(rows[local])
        kf = keyed(full["row_ptr"], full["col"])
        want = np.searchsorted(local, only // n) * n + only % n
        pos = np.minimum(np.searchsorted(kf, want), max(kf.size - 1, 0))
        found = kf[pos] == want  # (never empty: the diagonal is always kept)
        c = only % n
        nh = np.where(found, np.abs(full["val"][pos] * o.diag[c]), 0.0)
        ab = np.where(found, full["abssum"][pos], 0.0)
        k = np.where(found, full["cnt"][pos], 0.0)
        Dr = D[only // n]
        band = (((wb + 4.0 * (k + 2.0) * U64) * ab + Dr * delta * (1.0 + 2.0 ** -10)) / N[rows[only // n]]
                + 4.0 * U64 * eps)
        assert np.all(np.abs(nh - eps) <= band), "a pattern difference away from eps"
    return (int(common.size), float(rel.max()) if rel.size else 0.0, int(np.sum(rel > 1e-5)), int(only.size),
            int(D.sum()))


def check_compact_records(rec32, roff, o, rng, draws=64):
    """Compact records (8 words per unit: header {row, m, W, Shat32}, {Shat64,
    b_ii}; bucket j {T'_j, target_j, m_j, Shat32_j}, {w_j, alias target, its m, its
    Shat32}) against the oracle's arrays: T'_j = ceil(T_j 2^32 / W) (2^32 - 1 and
    the alias half equal to the own half when T_j = W), targets as record offsets
    with the sign of c, the targets' m and Shat32, w_j. Then the draw rule
    'target_j iff (u m mod 2^32) < T'_j' picks the oracle's entry for random words
    and for the words on both sides of every threshold of a sample of rows."""
    n = o.n
    cm = np.diff(o.cptr)
    inv = {int(x): i for i, x in enumerate(roff)}
    for i in range(n):
        base = int(roff[i]) * 8
        h = rec32[base:base + 8]
        b, e = int(o.cptr[i]), int(o.cptr[i + 1])
        m = e - b
        assert int(h[0]) == i and int(h[1]) == m and int(h[2]) == int(o.wsum[i]), ("compact header", i)
        assert h[3:4].view(np.float32)[0] == np.float32(o.shat[i])
        assert h[4:6].view(np.float64)[0] == o.shat[i] and h[6:8].view(np.float64)[0] == o.diag[i]
        if m == 0:
            continue
        W = int(o.wsum[i])
        ent = rec32[base + 8:base + 8 + 8 * m].reshape(m, 8).astype(np.int64)
        cum = o.cum[b:e].astype(np.int64)
        w = np.diff(np.concatenate([[0], cum]))
        thr = o.athr[b:e].astype(np.int64)
        ali = o.aidx[b:e]
        for k in range(m):
            full = thr[k] >= W
            tp = 0xFFFFFFFF if full else -((-(thr[k] << 32)) // W)
            assert int(ent[k, 0]) == tp, ("T'", i, k)
            assert int(ent[k, 4]) == int(w[k]), ("w", i, k)
            for half, kk in ((0, k), (1, k if full else int(ali[k]))):
                tg = int(ent[k, 4 * half + 1])
                col = int(o.ccol[b + kk])
                assert inv[tg & 0x7FFFFFFF] == col and ((tg >> 31) & 1) == int(o.cval[b + kk] < 0), ("target", i, k)
                assert int(ent[k, 4 * half + 2]) == int(cm[col]), ("target m", i, k)
                assert np.uint32(ent[k, 4 * half + 3]).view(np.float32) == np.float32(o.shat[col]), ("target S", i, k)
    rows = rng.choice(n, min(n, 40), replace=False)
    for i in rows:
        b, e = int(o.cptr[i]), int(o.cptr[i + 1])
        m = e - b
        if m == 0:
            continue
        ent = rec32[int(roff[i]) * 8 + 8:int(roff[i]) * 8 + 8 + 8 * m].reshape(m, 8).astype(np.int64)
        words = [int(x) for x in rng.integers(0, 2 ** 32, size=draws)]
        for k in range(m):
            # the last word below T'_k and the first at or above it, inside bucket k
            u_hi = -(-((k << 32) + int(ent[k, 0])) // m)
            words += [u for u in (u_hi - 1, u_hi) if 0 <= u < 2 ** 32 and (u * m) >> 32 == k]
        for u in words:
            j = (u * m) >> 32
            f = (u * m) & 0xFFFFFFFF
            full = int(o.athr[b + j]) >= int(o.wsum[i])
            pick = j if (f < int(ent[j, 0]) or full) else int(o.aidx[b + j])
            assert pick == o.draw(int(i), u), ("draw", i, u)
