/*
 * mcmi_oracle.c - plain, slow, FP64 CPU oracle for the Monte Carlo sparse
 * approximate inverse (Markov Chain Monte Carlo Matrix Inversion).
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library. It shares no code, header, table or
 * constant generator with the HIP library; the two meet only in the seeded
 * input matrices.
 *
 * What it computes, in the paper's order (Section III-A, eq. (2); Section IV,
 * phases 2-4; Section IV-A for the column scaling):
 *   O1  iteration matrix   C = I - D^-1 B, c_ij = (-b_ij) / b_ii, zeros dropped
 *   O2  transition CDF     p_ij proportional to |c_ij| (the paper never defines P;
 *                          this is the almost-optimal choice), quantized to
 *                          integer weights so both sides sample the same Chat
 *   O3  random numbers     Philox4x32-10 (Salmon et al., SC'11), counter-based;
 *                          a word picks the next state by the alias method
 *                          (Walker; Vose's exact-integer tables)
 *   O4  walk               eq. (2): W_0 = 1 at s_0 = r, W_j = W_{j-1} c/p; stop
 *                          when the next weight falls below delta (checked before
 *                          the draw) or the row of C is empty
 *   O5  accumulate         sum of W_j over chains per (r, s_j), long double
 *   O6  finalize           N_rc = acc / N_r; keep iff c = r or |N_rc| >= eps;
 *                          M_rc = N_rc / d_c (column scaling by the diagonal);
 *                          optionally only the k largest per row (Section IV-B)
 *   O7  apply              y = M x
 * an optional pre-pass before O1 (orc_prepare: the alpha-augmented diagonal of
 * Section III-B / V-C and the matrix reduction of Algorithm 1 step 2), and
 * the two per-row side products of the learned allocation:
 *   pilot variance (total variance of a chain's row estimate, mean chain length)
 *   row features (8 per row).
 *
 * Every floating-point step is one IEEE operation in source order; build with
 * -ffp-contract=off and without -ffast-math so nothing is fused or reordered.
 * Parity of the pilot and feature side products against the paper is
 * unpinned by any printed value (the paper has neither); they are pinned by
 * closed forms in the tests.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_ARG -1
#define ORC_ERR_CSR -2
#define ORC_ERR_ZERO_DIAG -3
#define ORC_ERR_NOT_CONTRACTIVE -4
#define ORC_ERR_NOMEM -7

#define ORC_LMAX_CAP 65536

/* ------------------------------------------------------------------ Philox */
/* Philox4x32 with 10 rounds as defined in Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3" (SC'11): each round multiplies
 * words 0 and 2 by two fixed 32-bit multipliers, and rebuilds the block from
 * the high/low halves xor'ed with words 1, 3 and the round key; the key is
 * bumped by two Weyl constants between rounds. */
static void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        x0 = y0;
        x1 = lo1;
        x2 = y2;
        x3 = lo0;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

/* Exposed for the pin against an independent Philox implementation. */
void orc_philox4x32_10(const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    orc_philox(ctr, key, out);
}

/* -------------------------------------------------------- O1 + O2: C, CDF */
/* The oracle's view of C and its sampling tables, natural column order. */
typedef struct {
    int64_t n;
    int64_t *cptr;    /* n+1: row i of C is entries [cptr[i], cptr[i+1]) */
    int32_t *ccol;    /* column of each entry, ascending within a row */
    double *cval;     /* c_ij (exact, unquantized) */
    uint32_t *cum;    /* inclusive prefix sum of the integer weights */
    uint32_t *wsum;   /* n: W_i = total integer weight of row i */
    double *shat;     /* n: Shat_i = a_max * W_i * 2^-Q (one rounding) */
    double *diag;     /* n: d_i = b_ii */
    double norm_inf;  /* max_i Shat_i */
    uint32_t *athr;   /* alias table: threshold T of each entry's bucket (O3) */
    int32_t *aidx;    /* alias table: alias of each entry's bucket, 0-based within the row */
} orc_mat;

static int ceil_log2_u64(uint64_t m)
{
    int q = 0;
    while (((uint64_t)1 << q) < m)
        ++q;
    return q;
}

/* Count entries of C per row (for the caller's allocation). Validates B.
 * Returns ORC_OK and *nnz_c, or an error code. */
int orc_count_c(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, int64_t *nnz_c)
{
    if (n <= 0 || !rp || !ci || !v || !nnz_c)
        return ORC_ERR_ARG;
    if (rp[0] != 0)
        return ORC_ERR_CSR;
    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (rp[i + 1] < rp[i])
            return ORC_ERR_CSR;
        int have_diag = 0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            if (ci[k] < 0 || ci[k] >= n)
                return ORC_ERR_CSR;
            if (k > rp[i] && ci[k] <= ci[k - 1])
                return ORC_ERR_CSR;
            if (ci[k] == i) {
                have_diag = 1;
                if (v[k] == 0.0)
                    return ORC_ERR_ZERO_DIAG;
            }
        }
        if (!have_diag)
            return ORC_ERR_ZERO_DIAG;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] != i && v[k] != 0.0)
                total += 1;
    }
    *nnz_c = total;
    return ORC_OK;
}

/* ----------------------------------------- phase 1 and matrix reduction
 * Optional pre-pass that turns B into B' before O1 (B' is CSR with ascending
 * columns and a stored diagonal in every row; capacity of ci2/v2: nnz + n):
 *  - augmentation, the splitting of Section III-B (b^_ii = b_ii + alpha ||B||)
 *    with the sign rule of Section V-C:
 *        b'_ii = b_ii + s_i * (alpha * ||B||_inf),  s_i = -1 if b_ii < 0, else +1,
 *    a missing diagonal counting as b_ii = 0; ||B||_inf = max over rows of the
 *    row's sum of |b_ij| taken in column order. alpha = 0 leaves B alone.
 *  - reduction, Algorithm 1 step 2 and Section V-A (drop a set share of the
 *    smallest entries of the iteration matrix): the K = floor(drop_frac * cnt)
 *    smallest of the cnt nonzero off-diagonal |c_ij| = |(-b_ij) / b'_ii| go; the
 *    cut is the (K+1)-th smallest value, entries strictly below it are removed
 *    and entries equal to it stay (so ties never split). drop_frac = 0 keeps all.
 * Explicit zeros off the diagonal are removed (they give c = 0 anyway). */
static int cmp_f64(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

int orc_prepare(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, double alpha,
                double drop_frac, int64_t *rp2, int32_t *ci2, double *v2, double *norm_b,
                double *thr_out, int64_t *dropped)
{
    if (n <= 0 || !rp || !ci || !v || !rp2 || !ci2 || !v2)
        return ORC_ERR_ARG;
    if (!(alpha >= 0.0) || !(drop_frac >= 0.0 && drop_frac < 1.0))
        return ORC_ERR_ARG;
    if (rp[0] != 0)
        return ORC_ERR_CSR;
    for (int64_t i = 0; i < n; ++i) {
        if (rp[i + 1] < rp[i])
            return ORC_ERR_CSR;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            if (ci[k] < 0 || ci[k] >= n)
                return ORC_ERR_CSR;
            if (k > rp[i] && ci[k] <= ci[k - 1])
                return ORC_ERR_CSR;
        }
    }
    double nrm = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
            s += fabs(v[k]);
        if (s > nrm)
            nrm = s;
    }
    double aug = alpha * nrm;
    double *dh = (double *)malloc((size_t)n * sizeof(double));
    if (!dh)
        return ORC_ERR_NOMEM;
    for (int64_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] == i)
                d = v[k];
        if (alpha > 0.0)
            d = d + (d < 0.0 ? -aug : aug);
        if (d == 0.0) {
            free(dh);
            return ORC_ERR_ZERO_DIAG;
        }
        dh[i] = d;
    }
    double thr = 0.0;
    if (drop_frac > 0.0) {
        int64_t cnt = 0;
        double *mag = (double *)malloc((size_t)(rp[n] > 0 ? rp[n] : 1) * sizeof(double));
        if (!mag) {
            free(dh);
            return ORC_ERR_NOMEM;
        }
        for (int64_t i = 0; i < n; ++i)
            for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
                if (ci[k] == i)
                    continue;
                double c = (-v[k]) / dh[i];
                if (c != 0.0)
                    mag[cnt++] = fabs(c);
            }
        if (cnt > 0) {
            qsort(mag, (size_t)cnt, sizeof(double), cmp_f64);
            int64_t K = (int64_t)floor(drop_frac * (double)cnt);
            thr = mag[K];
        }
        free(mag);
    }
    int64_t pos = 0, nd = 0;
    for (int64_t i = 0; i < n; ++i) {
        rp2[i] = pos;
        int placed = 0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            if (ci[k] == i)
                continue;
            if (!placed && ci[k] > i) {
                ci2[pos] = (int32_t)i;
                v2[pos++] = dh[i];
                placed = 1;
            }
            double c = (-v[k]) / dh[i];
            if (c == 0.0)
                continue;
            if (fabs(c) < thr) {
                ++nd;
                continue;
            }
            ci2[pos] = ci[k];
            v2[pos++] = v[k];
        }
        if (!placed) {
            ci2[pos] = (int32_t)i;
            v2[pos++] = dh[i];
        }
    }
    rp2[n] = pos;
    free(dh);
    if (norm_b)
        *norm_b = alpha > 0.0 ? nrm : 0.0; /* reported only when it was used */
    if (thr_out)
        *thr_out = thr;
    if (dropped)
        *dropped = nd;
    return ORC_OK;
}

/* Fill C and its CDF into caller-owned arrays sized by orc_count_c. */
int orc_build(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
              int64_t *cptr, int32_t *ccol, double *cval, uint32_t *cum,
              uint32_t *wsum, double *shat, double *diag, double *norm_inf)
{
    int64_t nnz_c = 0;
    int st = orc_count_c(n, rp, ci, v, &nnz_c);
    if (st != ORC_OK)
        return st;
    double nrm = 0.0;
    int64_t pos = 0;
    for (int64_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] == i)
                d = v[k];
        diag[i] = d;
        cptr[i] = pos;
        /* O1: c_ij = (-b_ij) / b_ii, entries equal to zero are dropped */
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            if (ci[k] == i)
                continue;
            double c = (-v[k]) / d;
            if (c == 0.0)
                continue;
            ccol[pos] = ci[k];
            cval[pos] = c;
            ++pos;
        }
        int64_t m = pos - cptr[i];
        if (m == 0) {
            wsum[i] = 0;
            shat[i] = 0.0;
            continue;
        }
        /* O2: a_k = |c_k|, a_max, Q = 31 - ceil(log2 m),
         *     w_k = max(1, floor(2^Q a_k / a_max)), cum = running sum. */
        double amax = 0.0;
        for (int64_t k = cptr[i]; k < pos; ++k)
            if (fabs(cval[k]) > amax)
                amax = fabs(cval[k]);
        int q = 31 - ceil_log2_u64((uint64_t)m);
        uint64_t run = 0;
        for (int64_t k = cptr[i]; k < pos; ++k) {
            double ratio = fabs(cval[k]) / amax;
            double scaled = floor(ldexp(ratio, q));
            uint64_t w = (uint64_t)scaled;
            if (w < 1)
                w = 1;
            run += w;
            cum[k] = (uint32_t)run;
        }
        if (run >= ((uint64_t)1 << 32))
            return ORC_ERR_ARG; /* cannot happen: sum <= 2^31 */
        wsum[i] = (uint32_t)run;
        shat[i] = ldexp(amax * (double)run, -q);
        if (shat[i] > nrm)
            nrm = shat[i];
    }
    cptr[n] = pos;
    *norm_inf = nrm;
    return ORC_OK;
}

/* O3 tables: the alias method of Walker in the exact-integer construction of
 * Vose ("A linear algorithm for generating random numbers with a given
 * distribution", IEEE TSE 17(9), 1991), one table per row. With m entries,
 * weights w_k (from cum) and W = sum w_k, entry k has the integer mass
 * q_k = m w_k and every one of the m buckets holds W units. The entries are
 * put, in column order, on a `small` stack (q < W) or a `large` stack (q >= W).
 * While both stacks are non-empty, the top s of small and the top l of large are
 * popped; bucket s keeps T_s = q_s units for entry s and gives the other W - q_s
 * to l (A_s = l, q_l -= W - q_s), and l is pushed back on small if now q_l < W,
 * else on large. Buckets left over hold exactly W for their own entry
 * (T = W, A = self). Each entry's mass is conserved exactly:
 * T_k + sum over buckets j with A_j = k of (W - T_j) = m w_k. */
int orc_build_alias(int64_t n, const int64_t *cptr, const uint32_t *cum, const uint32_t *wsum,
                    uint32_t *athr, int32_t *aidx)
{
    int64_t mmax = 0;
    for (int64_t i = 0; i < n; ++i)
        if (cptr[i + 1] - cptr[i] > mmax)
            mmax = cptr[i + 1] - cptr[i];
    uint64_t *q = (uint64_t *)malloc((size_t)(mmax + 1) * sizeof(uint64_t));
    int64_t *small = (int64_t *)malloc((size_t)(mmax + 1) * sizeof(int64_t));
    int64_t *large = (int64_t *)malloc((size_t)(mmax + 1) * sizeof(int64_t));
    if (!q || !small || !large) {
        free(q);
        free(small);
        free(large);
        return ORC_ERR_NOMEM;
    }
    for (int64_t i = 0; i < n; ++i) {
        int64_t b = cptr[i], m = cptr[i + 1] - cptr[i];
        uint64_t W = wsum[i];
        int64_t ns = 0, nl = 0;
        for (int64_t k = 0; k < m; ++k) {
            uint64_t w = (uint64_t)cum[b + k] - (k ? (uint64_t)cum[b + k - 1] : 0);
            q[k] = (uint64_t)m * w;
            if (q[k] < W)
                small[ns++] = k;
            else
                large[nl++] = k;
        }
        while (ns > 0 && nl > 0) {
            int64_t sm = small[--ns], lg = large[--nl];
            athr[b + sm] = (uint32_t)q[sm];
            aidx[b + sm] = (int32_t)lg;
            q[lg] -= W - q[sm];
            if (q[lg] < W)
                small[ns++] = lg;
            else
                large[nl++] = lg;
        }
        while (nl > 0) {
            int64_t k = large[--nl];
            athr[b + k] = (uint32_t)W;
            aidx[b + k] = (int32_t)k;
        }
        while (ns > 0) { /* cannot happen with exact masses */
            int64_t k = small[--ns];
            athr[b + k] = (uint32_t)W;
            aidx[b + k] = (int32_t)k;
        }
    }
    free(q);
    free(small);
    free(large);
    return ORC_OK;
}

/* L_max: max_len if given; otherwise the smallest L with p_L < delta, where
 * p_0 = 1 and p_j = p_{j-1} * ||Chat||_inf (one IEEE product per step). */
int orc_lmax(double norm_inf, double delta, int max_len)
{
    if (max_len > 0)
        return max_len > ORC_LMAX_CAP ? ORC_ERR_ARG : max_len;
    if (!(norm_inf < 1.0))
        return ORC_ERR_NOT_CONTRACTIVE;
    if (!(delta > 0.0))
        return ORC_ERR_ARG;
    double p = 1.0;
    int L = 0;
    while (p >= delta) {
        p = p * norm_inf;
        ++L;
        if (L > ORC_LMAX_CAP)
            return ORC_ERR_ARG;
    }
    return L;
}

/* ------------------------------------------------------------- O3 + O4 */
typedef struct {
    uint64_t seed;
    double delta, eps;
    int32_t chains;       /* uniform N_r when chains_per_row is NULL */
    int32_t fp32;         /* 1: binary32 weights, Shat32 and delta compare */
    int32_t max_len;      /* 0: derive L_max from ||Chat||_inf */
    uint32_t tag;         /* fourth Philox counter word */
    int32_t threads;
    int32_t filter_on_m;  /* 1: keep iff |M_rc| >= eps instead of |N_rc| >= eps */
    int32_t topk;         /* > 0: keep at most topk entries per row (see O6) */
} orc_params;

/* Draw step j >= 1 of chain c of row r: returns the chosen entry index of row s. */
typedef struct {
    uint32_t key[2];
    uint32_t ctr[4];
    uint32_t blk[4];
    int64_t loaded;
} orc_stream;

static void stream_init(orc_stream *st, uint64_t seed, uint32_t chain, uint32_t row, uint32_t tag)
{
    st->key[0] = (uint32_t)(seed & 0xffffffffu);
    st->key[1] = (uint32_t)(seed >> 32);
    st->ctr[0] = 0;
    st->ctr[1] = chain;
    st->ctr[2] = row;
    st->ctr[3] = tag;
    st->loaded = -1;
}

static uint32_t stream_word(orc_stream *st, int j)
{
    int64_t q = (int64_t)((j - 1) >> 2);
    if (q != st->loaded) {
        st->ctr[0] = (uint32_t)q;
        orc_philox(st->ctr, st->key, st->blk);
        st->loaded = q;
    }
    return st->blk[(j - 1) & 3];
}

/* O3: with m entries, the product u m < m 2^32 names the bucket j = floor(u m / 2^32)
 * (uniform over the m buckets) and its low 32 bits f the position inside it:
 * r = floor(f W_s / 2^32) is uniform over the bucket's W_s units; units r < T_j
 * belong to entry j, the others to its alias A_j. Entry k is drawn with
 * probability m w_k / (m W_s) = w_k / W_s, up to the 2^-32 grain of u. */
static int64_t draw_entry(const orc_mat *A, int64_t s, uint32_t u)
{
    int64_t b = A->cptr[s];
    uint64_t m = (uint64_t)(A->cptr[s + 1] - b);
    uint64_t um = (uint64_t)u * m;
    uint64_t j = um >> 32;
    uint64_t f = um & 0xFFFFFFFFull;
    uint64_t r = (f * (uint64_t)A->wsum[s]) >> 32;
    if (r < (uint64_t)A->athr[b + (int64_t)j])
        return b + (int64_t)j;
    return b + A->aidx[b + (int64_t)j];
}

/* Exposed for the pins: the entry of row s (0-based within the row) chosen by
 * the random word u, or -1 for an empty row. */
int64_t orc_draw(const orc_mat *A, int64_t s, uint32_t u)
{
    if (A->cptr[s + 1] == A->cptr[s])
        return -1;
    return draw_entry(A, s, u) - A->cptr[s];
}

/* One chain: calls visit(ctx, s, W) for every contribution (j = 0 included).
 * Returns the number of transitions (draws). */
typedef void (*visit_fn)(void *ctx, int64_t s, double w);

/* Is the cutoff test of step j (|wn| < delta) within the rounding band of a walk
 * with binary32 weights? Such a walk follows the same path, and its step-j weight
 * differs from this one by at most 2 j products' rounding of 2^-24 each (Shat
 * rounded to binary32, then the product), its delta by one more: a test inside
 * the band may go the other way there. Test instrumentation only: the count of
 * such chains bounds how many contributions of magnitude about delta a
 * binary32-weight run can add or miss. */
static int near_cutoff(double wn, double delta, int j)
{
    const double u32 = ldexp(1.0, -24);
    double a = fabs(wn);
    double big = a > delta ? a : delta;
    return fabs(a - delta) <= (2.0 * (double)j + 1.0) * u32 * (1.0 + ldexp(1.0, -10)) * big;
}

static int64_t run_chain(const orc_mat *A, const orc_params *p, int lmax, int64_t r,
                         uint32_t chain, uint32_t tag, visit_fn visit, void *ctx, int *border)
{
    orc_stream st;
    stream_init(&st, p->seed, chain, (uint32_t)r, tag);
    int64_t s = r;
    int64_t steps = 0;
    int near = 0;
    if (!p->fp32) {
        double w = 1.0;
        visit(ctx, s, w);
        for (int j = 1; j <= lmax; ++j) {
            if (A->cptr[s + 1] == A->cptr[s])
                break;
            double wn = w * A->shat[s];
            near |= near_cutoff(wn, p->delta, j);
            if (fabs(wn) < p->delta)
                break;
            int64_t k = draw_entry(A, s, stream_word(&st, j));
            w = (A->cval[k] < 0.0) ? -wn : wn;
            s = A->ccol[k];
            visit(ctx, s, w);
            ++steps;
        }
    } else {
        float w = 1.0f;
        float delta32 = (float)p->delta;
        visit(ctx, s, (double)w);
        for (int j = 1; j <= lmax; ++j) {
            if (A->cptr[s + 1] == A->cptr[s])
                break;
            float s32 = (float)A->shat[s];
            float wn = w * s32;
            near |= near_cutoff((double)wn, p->delta, j);
            if (fabsf(wn) < delta32)
                break;
            int64_t k = draw_entry(A, s, stream_word(&st, j));
            w = (A->cval[k] < 0.0) ? -wn : wn;
            s = A->ccol[k];
            visit(ctx, s, (double)w);
            ++steps;
        }
    }
    if (border)
        *border = near;
    return steps;
}

/* ------------------------------------------------------------- O5 + O6 */
typedef struct {
    long double *acc;
    double *abssum;
    uint32_t *cnt;
    int32_t *touched;
    int64_t ntouched;
} row_accum;

static void accum_visit(void *ctx, int64_t s, double w)
{
    row_accum *ra = (row_accum *)ctx;
    if (ra->cnt[s] == 0)
        ra->touched[ra->ntouched++] = (int32_t)s;
    ra->acc[s] += (long double)w;
    ra->abssum[s] += fabs(w);
    ra->cnt[s] += 1;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

typedef struct {
    int64_t nnz;
    int32_t *col;
    double *val;
    double *abssum;
    uint32_t *cnt;
    int64_t guard;
    int64_t transitions;
    int64_t border;
    int32_t ambig;
} row_out;

typedef struct {
    const orc_mat *A;
    const orc_params *p;
    const int32_t *rows;
    int64_t nrows;
    const int32_t *chains_per_row;
    int lmax;
    row_out *out;
    int64_t next;
    pthread_mutex_t lock;
    int failed;
} spai_job;

static int64_t take_rows(spai_job *job, int64_t want, int64_t *begin)
{
    pthread_mutex_lock(&job->lock);
    int64_t b = job->next;
    int64_t e = b + want;
    if (e > job->nrows)
        e = job->nrows;
    job->next = e;
    pthread_mutex_unlock(&job->lock);
    *begin = b;
    return e - b;
}

/* Top-k retention (Section IV-B: only a prescribed number of the entries
 * largest in magnitude are retained per row). Of the entries that passed the
 * eps rule, the diagonal stays and the topk - 1 off-diagonal entries with the
 * largest test value (|N_rc|, or |M_rc| with filter_on_m) stay; equal values go
 * by ascending column. The row is marked ambiguous when the last kept and the
 * first dropped entry are within the sum-order band of each other (sums of at
 * most two terms are order-free and have no band), so that another summation
 * order could swap them. Entries stay in column order. */
typedef struct {
    double test;
    int32_t col;
    int64_t idx;
} top_item;

static int cmp_top(const void *a, const void *b)
{
    const top_item *x = (const top_item *)a, *y = (const top_item *)b;
    if (x->test != y->test)
        return x->test > y->test ? -1 : 1;
    return (x->col > y->col) - (x->col < y->col);
}

static double order_band(uint32_t cnt, double abssum, int32_t nr, double scale)
{
    if (cnt <= 2)
        return 0.0;
    return 4.0 * ((double)cnt + 2.0) * ldexp(1.0, -53) * abssum / (double)nr * scale;
}

static int keep_top(const orc_mat *A, const orc_params *p, int64_t r, int32_t nr, row_out *ro, const double *tv)
{
    int64_t nc = 0;
    top_item *it = (top_item *)malloc((size_t)(ro->nnz + 1) * sizeof(top_item));
    char *sel = (char *)calloc((size_t)(ro->nnz + 1), 1);
    if (!it || !sel) {
        free(it);
        free(sel);
        return -1;
    }
    for (int64_t q = 0; q < ro->nnz; ++q) {
        if (ro->col[q] == r) {
            sel[q] = 1;
            continue;
        }
        it[nc].test = tv[q];
        it[nc].col = ro->col[q];
        it[nc].idx = q;
        ++nc;
    }
    qsort(it, (size_t)nc, sizeof(top_item), cmp_top);
    int64_t want = (int64_t)p->topk - 1;
    for (int64_t q = 0; q < nc && q < want; ++q)
        sel[it[q].idx] = 1;
    if (want >= 1 && nc > want) {
        const top_item *a = &it[want - 1], *b = &it[want];
        double sa = p->filter_on_m ? 1.0 / fabs(A->diag[a->col]) : 1.0;
        double sb = p->filter_on_m ? 1.0 / fabs(A->diag[b->col]) : 1.0;
        double band = order_band(ro->cnt[a->idx], ro->abssum[a->idx], nr, sa) +
                      order_band(ro->cnt[b->idx], ro->abssum[b->idx], nr, sb);
        if (band > 0.0 && fabs(a->test - b->test) <= band)
            ro->ambig = 1;
    }
    int64_t w = 0;
    for (int64_t q = 0; q < ro->nnz; ++q) {
        if (!sel[q])
            continue;
        ro->col[w] = ro->col[q];
        ro->val[w] = ro->val[q];
        ro->abssum[w] = ro->abssum[q];
        ro->cnt[w] = ro->cnt[q];
        ++w;
    }
    ro->nnz = w;
    free(it);
    free(sel);
    return 0;
}

static void *spai_worker(void *arg)
{
    spai_job *job = (spai_job *)arg;
    const orc_mat *A = job->A;
    const orc_params *p = job->p;
    int64_t n = A->n;
    row_accum ra;
    ra.acc = (long double *)calloc((size_t)n, sizeof(long double));
    ra.abssum = (double *)calloc((size_t)n, sizeof(double));
    ra.cnt = (uint32_t *)calloc((size_t)n, sizeof(uint32_t));
    ra.touched = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!ra.acc || !ra.abssum || !ra.cnt || !ra.touched) {
        job->failed = 1;
        goto done;
    }
    const double u = ldexp(1.0, -53);
    for (;;) {
        int64_t b;
        int64_t cnt = take_rows(job, 8, &b);
        if (cnt <= 0)
            break;
        for (int64_t t = b; t < b + cnt; ++t) {
            int64_t r = job->rows ? job->rows[t] : t;
            int32_t nr = job->chains_per_row ? job->chains_per_row[r] : p->chains;
            ra.ntouched = 0;
            int64_t steps = 0, border = 0;
            for (int32_t c = 0; c < nr; ++c) {
                int near = 0;
                steps += run_chain(A, p, job->lmax, r, (uint32_t)c, p->tag, accum_visit, &ra, &near);
                border += near;
            }
            qsort(ra.touched, (size_t)ra.ntouched, sizeof(int32_t), cmp_i32);
            row_out *ro = &job->out[t];
            ro->transitions = steps;
            ro->border = border;
            ro->guard = 0;
            ro->col = (int32_t *)malloc((size_t)(ra.ntouched + 1) * sizeof(int32_t));
            ro->val = (double *)malloc((size_t)(ra.ntouched + 1) * sizeof(double));
            ro->abssum = (double *)malloc((size_t)(ra.ntouched + 1) * sizeof(double));
            ro->cnt = (uint32_t *)malloc((size_t)(ra.ntouched + 1) * sizeof(uint32_t));
            double *tv = (double *)malloc((size_t)(ra.ntouched + 1) * sizeof(double));
            if (!ro->col || !ro->val || !ro->abssum || !ro->cnt || !tv) {
                free(tv);
                job->failed = 1;
                goto done;
            }
            int64_t kept = 0;
            for (int64_t q = 0; q < ra.ntouched; ++q) {
                int32_t col = ra.touched[q];
                double acc = (double)ra.acc[col];
                double nhat = acc / (double)nr;
                double m = nhat / A->diag[col];
                double test = p->filter_on_m ? fabs(m) : fabs(nhat);
                int keep = (col == r) || (nhat != 0.0 && test >= p->eps);
                /* guard band: a summation order other than this one can only flip
                 * the decision inside |test - eps| <= band (standard recursive
                 * summation bound with k terms, widened by a factor 4). */
                double scale = p->filter_on_m ? 1.0 / fabs(A->diag[col]) : 1.0;
                double band = 4.0 * ((double)ra.cnt[col] + 2.0) * u * ra.abssum[col] / (double)nr * scale
                              + 4.0 * u * p->eps;
                if (col != r && fabs(test - p->eps) <= band)
                    ro->guard += 1;
                if (keep) {
                    tv[kept] = test;
                    ro->col[kept] = col;
                    ro->val[kept] = m;
                    ro->abssum[kept] = ra.abssum[col];
                    ro->cnt[kept] = ra.cnt[col];
                    ++kept;
                }
                ra.acc[col] = 0.0L;
                ra.abssum[col] = 0.0;
                ra.cnt[col] = 0;
            }
            ro->nnz = kept;
            ro->ambig = 0;
            int top_failed = p->topk > 0 && keep_top(A, p, r, nr, ro, tv) != 0;
            free(tv);
            if (top_failed) {
                job->failed = 1;
                goto done;
            }
        }
    }
done:
    free(ra.acc);
    free(ra.abssum);
    free(ra.cnt);
    free(ra.touched);
    return NULL;
}

typedef struct {
    int64_t nrows;
    int64_t *row_ptr;     /* nrows + 1 */
    int32_t *col;
    double *val;
    double *abssum;       /* per kept entry: sum of |W| of its contributions */
    uint32_t *cnt;        /* per kept entry: number of contributions */
    int64_t *row_transitions;
    uint64_t transitions;
    int64_t guard;
    int32_t lmax;
    int32_t *row_ambig;   /* nrows: 1 where the top-k boundary is order-dependent */
    int64_t *row_border;  /* nrows: chains with a cutoff test inside the binary32 band (near_cutoff) */
} orc_result;

static int run_threads(void *(*fn)(void *), void *job, int threads)
{
    if (threads < 1)
        threads = 1;
    if (threads > 256)
        threads = 256;
    pthread_t tid[256];
    int started = 0;
    for (int t = 0; t < threads; ++t) {
        if (pthread_create(&tid[t], NULL, fn, job) != 0)
            break;
        ++started;
    }
    if (started == 0) {
        fn(job);
        return ORC_OK;
    }
    for (int t = 0; t < started; ++t)
        pthread_join(tid[t], NULL);
    return ORC_OK;
}

/* O4-O6 for a list of rows (rows == NULL: all rows, in order). Output rows are
 * in the order given. chains_per_row (nullable) is indexed by global row. */
int orc_spai(const orc_mat *A, const orc_params *p, const int32_t *rows, int64_t nrows,
             const int32_t *chains_per_row, orc_result *res)
{
    memset(res, 0, sizeof(*res));
    if (!A || !p || A->n <= 0)
        return ORC_ERR_ARG;
    if (!rows)
        nrows = A->n;
    if (nrows < 0 || p->eps < 0.0 || !(p->delta >= 0.0) || p->topk < 0)
        return ORC_ERR_ARG;
    if (!chains_per_row && p->chains < 1)
        return ORC_ERR_ARG;
    for (int64_t t = 0; rows && t < nrows; ++t)
        if (rows[t] < 0 || rows[t] >= A->n)
            return ORC_ERR_ARG;
    if (chains_per_row)
        for (int64_t i = 0; i < A->n; ++i)
            if (chains_per_row[i] < 1)
                return ORC_ERR_ARG;
    int lmax = orc_lmax(A->norm_inf, p->delta, p->max_len);
    if (lmax < 0)
        return lmax;
    spai_job job;
    memset(&job, 0, sizeof(job));
    job.A = A;
    job.p = p;
    job.rows = rows;
    job.nrows = nrows;
    job.chains_per_row = chains_per_row;
    job.lmax = lmax;
    job.out = (row_out *)calloc((size_t)(nrows > 0 ? nrows : 1), sizeof(row_out));
    if (!job.out)
        return ORC_ERR_NOMEM;
    pthread_mutex_init(&job.lock, NULL);
    run_threads(spai_worker, &job, p->threads);
    pthread_mutex_destroy(&job.lock);
    int status = job.failed ? ORC_ERR_NOMEM : ORC_OK;
    int64_t total = 0;
    for (int64_t t = 0; t < nrows; ++t)
        total += job.out[t].nnz;
    res->nrows = nrows;
    res->lmax = lmax;
    res->row_ptr = (int64_t *)malloc((size_t)(nrows + 1) * sizeof(int64_t));
    res->col = (int32_t *)malloc((size_t)(total + 1) * sizeof(int32_t));
    res->val = (double *)malloc((size_t)(total + 1) * sizeof(double));
    res->abssum = (double *)malloc((size_t)(total + 1) * sizeof(double));
    res->cnt = (uint32_t *)malloc((size_t)(total + 1) * sizeof(uint32_t));
    res->row_transitions = (int64_t *)malloc((size_t)(nrows + 1) * sizeof(int64_t));
    res->row_ambig = (int32_t *)malloc((size_t)(nrows + 1) * sizeof(int32_t));
    res->row_border = (int64_t *)malloc((size_t)(nrows + 1) * sizeof(int64_t));
    if (!res->row_ptr || !res->col || !res->val || !res->abssum || !res->cnt || !res->row_transitions ||
        !res->row_ambig || !res->row_border)
        status = ORC_ERR_NOMEM;
    int64_t pos = 0;
    for (int64_t t = 0; t < nrows; ++t) {
        row_out *ro = &job.out[t];
        if (status == ORC_OK) {
            res->row_ptr[t] = pos;
            if (ro->nnz > 0) {
                memcpy(res->col + pos, ro->col, (size_t)ro->nnz * sizeof(int32_t));
                memcpy(res->val + pos, ro->val, (size_t)ro->nnz * sizeof(double));
                memcpy(res->abssum + pos, ro->abssum, (size_t)ro->nnz * sizeof(double));
                memcpy(res->cnt + pos, ro->cnt, (size_t)ro->nnz * sizeof(uint32_t));
            }
            pos += ro->nnz;
            res->row_transitions[t] = ro->transitions;
            res->row_ambig[t] = ro->ambig;
            res->row_border[t] = ro->border;
            res->transitions += (uint64_t)ro->transitions;
            res->guard += ro->guard;
        }
        free(ro->col);
        free(ro->val);
        free(ro->abssum);
        free(ro->cnt);
    }
    if (status == ORC_OK)
        res->row_ptr[nrows] = pos;
    free(job.out);
    return status;
}

void orc_result_free(orc_result *res)
{
    if (!res)
        return;
    free(res->row_ptr);
    free(res->col);
    free(res->val);
    free(res->abssum);
    free(res->cnt);
    free(res->row_transitions);
    free(res->row_border);
    free(res->row_ambig);
    memset(res, 0, sizeof(*res));
}

/* -------------------------------------------------------------------- O7 */
/* y_i = sum_k M_ik x_k, ascending column order, plain FP64. */
void orc_apply(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
               const double *x, double *y)
{
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
            s += v[k] * x[ci[k]];
        y[i] = s;
    }
}

/* ------------------------------------------------------ pilot variance */
/* Per row r with P pilot chains (Philox tag with bit 31 set): each chain's row
 * estimate is the sparse vector X_c with X_c[s] = sum of its W_j at s. Returns
 *   v_r  = mean_c ||X_c||^2 - ||mean_c X_c||^2   (total variance of one chain)
 *   len_r = mean_c (number of transitions of chain c).
 * Revisits inside one chain are merged before squaring. */
typedef struct {
    int64_t *cols;
    double *vals;
    int64_t n;
} chain_list;

static void list_visit(void *ctx, int64_t s, double w)
{
    chain_list *cl = (chain_list *)ctx;
    for (int64_t k = 0; k < cl->n; ++k)
        if (cl->cols[k] == s) {
            cl->vals[k] += w;
            return;
        }
    cl->cols[cl->n] = s;
    cl->vals[cl->n] = w;
    cl->n += 1;
}

typedef struct {
    const orc_mat *A;
    const orc_params *p;
    int lmax;
    int32_t pilot;
    double *var;
    double *len;
    int64_t next;
    pthread_mutex_t lock;
    int failed;
} pilot_job;

static void *pilot_worker(void *arg)
{
    pilot_job *job = (pilot_job *)arg;
    const orc_mat *A = job->A;
    int64_t n = A->n;
    chain_list cl;
    cl.cols = (int64_t *)malloc((size_t)(job->lmax + 2) * sizeof(int64_t));
    cl.vals = (double *)malloc((size_t)(job->lmax + 2) * sizeof(double));
    long double *mean = (long double *)calloc((size_t)n, sizeof(long double));
    int32_t *touched = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    uint8_t *seen = (uint8_t *)calloc((size_t)n, 1);
    if (!cl.cols || !cl.vals || !mean || !touched || !seen) {
        job->failed = 1;
        goto done;
    }
    for (;;) {
        pthread_mutex_lock(&job->lock);
        int64_t r = job->next++;
        pthread_mutex_unlock(&job->lock);
        if (r >= n)
            break;
        int64_t nt = 0;
        long double sq = 0.0L;
        int64_t steps = 0;
        for (int32_t c = 0; c < job->pilot; ++c) {
            cl.n = 0;
            steps += run_chain(A, job->p, job->lmax, r, (uint32_t)c, job->p->tag | 0x80000000u,
                               list_visit, &cl, NULL);
            for (int64_t k = 0; k < cl.n; ++k) {
                int64_t s = cl.cols[k];
                sq += (long double)cl.vals[k] * (long double)cl.vals[k];
                if (!seen[s]) {
                    seen[s] = 1;
                    touched[nt++] = (int32_t)s;
                }
                mean[s] += (long double)cl.vals[k];
            }
        }
        long double msq = 0.0L;
        for (int64_t k = 0; k < nt; ++k) {
            long double mu = mean[touched[k]] / (long double)job->pilot;
            msq += mu * mu;
            mean[touched[k]] = 0.0L;
            seen[touched[k]] = 0;
        }
        job->var[r] = (double)(sq / (long double)job->pilot - msq);
        job->len[r] = (double)steps / (double)job->pilot;
    }
done:
    free(cl.cols);
    free(cl.vals);
    free(mean);
    free(touched);
    free(seen);
    return NULL;
}

int orc_pilot(const orc_mat *A, const orc_params *p, int32_t pilot, double *var, double *len)
{
    if (!A || !p || pilot < 1 || !var || !len)
        return ORC_ERR_ARG;
    int lmax = orc_lmax(A->norm_inf, p->delta, p->max_len);
    if (lmax < 0)
        return lmax;
    pilot_job job;
    memset(&job, 0, sizeof(job));
    job.A = A;
    job.p = p;
    job.lmax = lmax;
    job.pilot = pilot;
    job.var = var;
    job.len = len;
    pthread_mutex_init(&job.lock, NULL);
    run_threads(pilot_worker, &job, p->threads);
    pthread_mutex_destroy(&job.lock);
    return job.failed ? ORC_ERR_NOMEM : ORC_OK;
}

/* --------------------------------------------------------- row features */
/* Eight features per row i of the sampled matrix Chat (O2: |chat_ij| = S_i w_ij
 * / W_i with the sign of c_ij; p_ij = w_ij / W_i its transition probabilities,
 * S = Shat, m = entries of the row of C):
 *   f0 = ln(max(m_i, 1))          f1 = S_i
 *   f2 = max_j |chat_ij|           f3 = sum_j p_ij S_j
 *   f4 = max_j S_j                 f5 = sum_j p_ij m_j
 *   f6 = |sum_j chat_ij| / S_i     f7 = min(L_max, ln(delta) / ln(S_i))
 * with f2..f6 = 0 for an empty row, f7 = L_max when S_i >= 1 and f7 = 0 when
 * S_i = 0. These are inputs of the learned allocation, not part of the paper. */
void orc_features(const orc_mat *A, double delta, int lmax, double *feat)
{
    for (int64_t i = 0; i < A->n; ++i) {
        double *f = feat + 8 * i;
        int64_t b = A->cptr[i], e = A->cptr[i + 1];
        int64_t m = e - b;
        double s = A->shat[i];
        f[0] = log((double)(m > 1 ? m : 1));
        f[1] = s;
        double cmax = 0.0, ps = 0.0, smax = 0.0, pm = 0.0, csum = 0.0;
        uint32_t prev = 0;
        for (int64_t k = b; k < e; ++k) {
            uint32_t w = A->cum[k] - prev;
            prev = A->cum[k];
            double pk = (double)w / (double)A->wsum[i];
            double chat = s * (double)w / (double)A->wsum[i];
            int64_t j = A->ccol[k];
            if (chat > cmax)
                cmax = chat;
            ps += pk * A->shat[j];
            if (A->shat[j] > smax)
                smax = A->shat[j];
            pm += pk * (double)(A->cptr[j + 1] - A->cptr[j]);
            csum += A->cval[k] < 0.0 ? -chat : chat;
        }
        f[2] = cmax;
        f[3] = ps;
        f[4] = smax;
        f[5] = pm;
        f[6] = (m > 0 && s > 0.0) ? fabs(csum) / s : 0.0;
        if (s > 0.0 && s < 1.0 && delta > 0.0) {
            double l = log(delta) / log(s);
            f[7] = l < (double)lmax ? l : (double)lmax;
        } else {
            f[7] = s > 0.0 ? (double)lmax : 0.0;
        }
    }
}
