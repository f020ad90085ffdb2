/*
 * Test driver for the CPU oracle under AddressSanitizer + UndefinedBehaviorSanitizer
 * and under ThreadSanitizer (test infrastructure only; built and run by
 * tests/test_oracle_sanitize.py with gcc, never by the library).
 *
 * It builds small input matrices itself, runs every entry point of the oracle
 * (pre-pass, iteration matrix, alias tables, walks with several thread counts,
 * top-k and M filter, pilot variance, features, apply) and checks a few facts
 * that hold exactly:
 *   - B diagonal: zero transitions, M = D^-1 (C = 0 leaves only the j = 0 term);
 *   - periodic 5-point torus with diagonal 5 (every |C| row sum 0.8, delta 1e-3):
 *     every chain makes 30 transitions, so the total is n * N * 30;
 *   - results with 1 thread and with 8 threads are bit-identical (each row's
 *     result depends only on its own chains).
 * A sanitizer report makes the process exit non-zero.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t n;
    int64_t *cptr;
    int32_t *ccol;
    double *cval;
    uint32_t *cum;
    uint32_t *wsum;
    double *shat;
    double *diag;
    double norm_inf;
    uint32_t *athr;
    int32_t *aidx;
} orc_mat;

typedef struct {
    uint64_t seed;
    double delta, eps;
    int32_t chains, fp32, max_len;
    uint32_t tag;
    int32_t threads, filter_on_m, topk;
} orc_params;

typedef struct {
    int64_t nrows;
    int64_t *row_ptr;
    int32_t *col;
    double *val;
    double *abssum;
    uint32_t *cnt;
    int64_t *row_transitions;
    uint64_t transitions;
    int64_t guard;
    int32_t lmax;
    int32_t *row_ambig;
    int64_t *row_border;
} orc_result;

int orc_count_c(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, int64_t *nnz_c);
int orc_build(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, int64_t *cptr, int32_t *ccol,
              double *cval, uint32_t *cum, uint32_t *wsum, double *shat, double *diag, double *norm_inf);
int orc_build_alias(int64_t n, const int64_t *cptr, const uint32_t *cum, const uint32_t *wsum, uint32_t *athr,
                    int32_t *aidx);
int orc_prepare(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, double alpha, double drop_frac,
                int64_t *rp2, int32_t *ci2, double *v2, double *norm_b, double *thr_out, int64_t *dropped);
int orc_spai(const orc_mat *A, const orc_params *p, const int32_t *rows, int64_t nrows,
             const int32_t *chains_per_row, orc_result *res);
void orc_result_free(orc_result *res);
void orc_apply(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, const double *x, double *y);
int orc_pilot(const orc_mat *A, const orc_params *p, int32_t pilot, double *var, double *len);
void orc_features(const orc_mat *A, double delta, int lmax, double *feat);
int orc_lmax(double norm_inf, double delta, int max_len);

#define CHECK(cond, msg)                                             \
    do {                                                             \
        if (!(cond)) {                                               \
            fprintf(stderr, "FAILED: %s (line %d)\n", msg, __LINE__); \
            exit(2);                                                 \
        }                                                            \
    } while (0)

typedef struct {
    int64_t n;
    int64_t *rp;
    int32_t *ci;
    double *v;
} csr;

static void csr_free(csr *B) {
    free(B->rp);
    free(B->ci);
    free(B->v);
}

/* periodic nx x ny 5-point stencil, diagonal d, off-diagonals o */
static csr torus(int nx, int ny, double d, double o) {
    csr B;
    B.n = (int64_t)nx * ny;
    B.rp = malloc((B.n + 1) * sizeof(int64_t));
    B.ci = malloc(B.n * 5 * sizeof(int32_t));
    B.v = malloc(B.n * 5 * sizeof(double));
    int64_t k = 0;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int32_t c[5] = {y * nx + x, y * nx + (x + 1) % nx, y * nx + (x + nx - 1) % nx,
                            ((y + 1) % ny) * nx + x, ((y + ny - 1) % ny) * nx + x};
            /* insertion sort of the five columns */
            for (int a = 1; a < 5; ++a)
                for (int b = a; b > 0 && c[b] < c[b - 1]; --b) {
                    int32_t t = c[b];
                    c[b] = c[b - 1];
                    c[b - 1] = t;
                }
            B.rp[y * nx + x] = k;
            for (int a = 0; a < 5; ++a) {
                B.ci[k] = c[a];
                B.v[k] = c[a] == y * nx + x ? d : o;
                ++k;
            }
        }
    B.rp[B.n] = k;
    return B;
}

/* rows with 1..kmax off-diagonals at pseudo-random distinct columns, random signs,
 * diagonal sum|b| / rho; a plain LCG makes the input (no method arithmetic) */
static csr random_rows(int64_t n, int kmax, double rho, uint64_t seed) {
    csr B;
    B.n = n;
    B.rp = malloc((n + 1) * sizeof(int64_t));
    B.ci = malloc(n * (kmax + 1) * sizeof(int32_t));
    B.v = malloc(n * (kmax + 1) * sizeof(double));
    uint64_t s = seed * 6364136223846793005ull + 1442695040888963407ull;
#define NEXT() (s = s * 6364136223846793005ull + 1442695040888963407ull, (uint32_t)(s >> 33))
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i) {
        int m = 1 + (int)(NEXT() % (uint32_t)kmax);
        int32_t cols[64];
        int got = 0;
        while (got < m) {
            int32_t c = (int32_t)(NEXT() % (uint32_t)n);
            int dup = c == i;
            for (int a = 0; a < got; ++a) dup |= cols[a] == c;
            if (!dup) cols[got++] = c;
        }
        cols[got++] = (int32_t)i;
        for (int a = 1; a < got; ++a)
            for (int b = a; b > 0 && cols[b] < cols[b - 1]; --b) {
                int32_t t = cols[b];
                cols[b] = cols[b - 1];
                cols[b - 1] = t;
            }
        B.rp[i] = k;
        double sum = 0.0;
        int64_t dpos = -1;
        for (int a = 0; a < got; ++a) {
            B.ci[k] = cols[a];
            if (cols[a] == i) {
                dpos = k;
                B.v[k] = 0.0;
            } else {
                double mag = 0.1 + (double)(NEXT() % 1000u) / 100.0;
                B.v[k] = (NEXT() & 1u) ? mag : -mag;
                sum += mag;
            }
            ++k;
        }
        B.v[dpos] = sum / rho;
    }
    B.rp[n] = k;
#undef NEXT
    return B;
}

typedef struct {
    orc_mat A;
    int64_t nnz_c;
} built;

static built build(const csr *B) {
    built r;
    memset(&r, 0, sizeof(r));
    CHECK(orc_count_c(B->n, B->rp, B->ci, B->v, &r.nnz_c) == 0, "orc_count_c");
    int64_t m = r.nnz_c > 0 ? r.nnz_c : 1;
    r.A.n = B->n;
    r.A.cptr = calloc(B->n + 1, sizeof(int64_t));
    r.A.ccol = calloc(m, sizeof(int32_t));
    r.A.cval = calloc(m, sizeof(double));
    r.A.cum = calloc(m, sizeof(uint32_t));
    r.A.wsum = calloc(B->n, sizeof(uint32_t));
    r.A.shat = calloc(B->n, sizeof(double));
    r.A.diag = calloc(B->n, sizeof(double));
    r.A.athr = calloc(m, sizeof(uint32_t));
    r.A.aidx = calloc(m, sizeof(int32_t));
    CHECK(orc_build(B->n, B->rp, B->ci, B->v, r.A.cptr, r.A.ccol, r.A.cval, r.A.cum, r.A.wsum, r.A.shat, r.A.diag,
                    &r.A.norm_inf) == 0,
          "orc_build");
    CHECK(orc_build_alias(B->n, r.A.cptr, r.A.cum, r.A.wsum, r.A.athr, r.A.aidx) == 0, "orc_build_alias");
    return r;
}

static void built_free(built *b) {
    free(b->A.cptr);
    free(b->A.ccol);
    free(b->A.cval);
    free(b->A.cum);
    free(b->A.wsum);
    free(b->A.shat);
    free(b->A.diag);
    free(b->A.athr);
    free(b->A.aidx);
}

static orc_params params(int chains, double delta, double eps, int threads) {
    orc_params p;
    memset(&p, 0, sizeof(p));
    p.seed = 0x1234abcdull;
    p.delta = delta;
    p.eps = eps;
    p.chains = chains;
    p.threads = threads;
    return p;
}

static int same_result(const orc_result *a, const orc_result *b) {
    if (a->nrows != b->nrows || a->transitions != b->transitions) return 0;
    int64_t nnz = a->row_ptr[a->nrows];
    return memcmp(a->row_ptr, b->row_ptr, (a->nrows + 1) * sizeof(int64_t)) == 0 &&
           memcmp(a->col, b->col, nnz * sizeof(int32_t)) == 0 && memcmp(a->val, b->val, nnz * sizeof(double)) == 0;
}

int main(void) {
    /* 1. diagonal B: zero transitions, M = D^-1 */
    {
        csr B;
        B.n = 40;
        B.rp = malloc(41 * sizeof(int64_t));
        B.ci = malloc(40 * sizeof(int32_t));
        B.v = malloc(40 * sizeof(double));
        for (int i = 0; i < 40; ++i) {
            B.rp[i] = i;
            B.ci[i] = i;
            B.v[i] = (i % 3 == 0 ? -1.0 : 1.0) * (1.0 + i);
        }
        B.rp[40] = 40;
        built b = build(&B);
        orc_params p = params(50, 1e-3, 1e-3, 4);
        orc_result r;
        CHECK(orc_spai(&b.A, &p, NULL, 0, NULL, &r) == 0, "orc_spai diagonal");
        CHECK(r.transitions == 0, "diagonal: transitions");
        for (int i = 0; i < 40; ++i) {
            CHECK(r.row_ptr[i + 1] - r.row_ptr[i] == 1 && r.col[r.row_ptr[i]] == i, "diagonal: pattern");
            CHECK(r.val[r.row_ptr[i]] == 1.0 / B.v[i], "diagonal: value");
        }
        orc_result_free(&r);
        built_free(&b);
        csr_free(&B);
    }
    /* 2. torus: exact transition count, 1 vs 8 threads bit-identical */
    {
        csr B = torus(12, 10, 5.0, -1.0);
        built b = build(&B);
        orc_params p1 = params(64, 1e-3, 1e-3, 1), p8 = params(64, 1e-3, 1e-3, 8);
        orc_result r1, r8;
        CHECK(orc_spai(&b.A, &p1, NULL, 0, NULL, &r1) == 0, "orc_spai torus 1 thread");
        CHECK(orc_spai(&b.A, &p8, NULL, 0, NULL, &r8) == 0, "orc_spai torus 8 threads");
        CHECK(r1.transitions == (uint64_t)B.n * 64u * 30u, "torus: n N 30 transitions");
        CHECK(same_result(&r1, &r8), "torus: thread counts give different results");
        double *x = malloc(B.n * sizeof(double)), *y = malloc(B.n * sizeof(double));
        for (int64_t i = 0; i < B.n; ++i) x[i] = 1.0;
        orc_apply(B.n, r1.row_ptr, r1.col, r1.val, x, y);
        for (int64_t i = 0; i < B.n; ++i) CHECK(isfinite(y[i]) && y[i] > 0.0, "torus: apply");
        double *var = malloc(B.n * sizeof(double)), *len = malloc(B.n * sizeof(double));
        CHECK(orc_pilot(&b.A, &p8, 32, var, len) == 0, "orc_pilot torus");
        for (int64_t i = 0; i < B.n; ++i) CHECK(len[i] == 30.0, "torus: pilot length");
        double *feat = malloc(B.n * 8 * sizeof(double));
        orc_features(&b.A, 1e-3, orc_lmax(b.A.norm_inf, 1e-3, 0), feat);
        for (int64_t i = 0; i < B.n * 8; ++i) CHECK(isfinite(feat[i]), "torus: features");
        free(x);
        free(y);
        free(var);
        free(len);
        free(feat);
        orc_result_free(&r1);
        orc_result_free(&r8);
        built_free(&b);
        csr_free(&B);
    }
    /* 3. random rows: pre-pass, row subsets, per-row chains, FP32 mode, top-k, M filter */
    {
        csr B0 = random_rows(700, 12, 0.9, 7);
        int64_t cap = B0.rp[B0.n] + B0.n;
        csr B;
        B.n = B0.n;
        B.rp = calloc(B.n + 1, sizeof(int64_t));
        B.ci = calloc(cap, sizeof(int32_t));
        B.v = calloc(cap, sizeof(double));
        double norm_b = 0.0, thr = 0.0;
        int64_t dropped = 0;
        CHECK(orc_prepare(B0.n, B0.rp, B0.ci, B0.v, 0.5, 0.05, B.rp, B.ci, B.v, &norm_b, &thr, &dropped) == 0,
              "orc_prepare");
        CHECK(dropped > 0 && norm_b > 0.0, "prepare: something dropped");
        built b = build(&B);
        int32_t rows[300];
        int32_t *cpr = malloc(B.n * sizeof(int32_t));
        for (int i = 0; i < 300; ++i) rows[i] = (int32_t)((i * 37) % B.n);
        for (int64_t i = 0; i < B.n; ++i) cpr[i] = 1 + (int32_t)(i % 50);
        for (int variant = 0; variant < 4; ++variant) {
            orc_params p1 = params(40, 1e-4, 1e-3, 1), p8 = params(40, 1e-4, 1e-3, 8);
            p1.fp32 = p8.fp32 = variant == 1;
            p1.topk = p8.topk = variant == 2 ? 5 : 0;
            p1.filter_on_m = p8.filter_on_m = variant == 3;
            orc_result r1, r8;
            CHECK(orc_spai(&b.A, &p1, rows, 300, variant == 3 ? cpr : NULL, &r1) == 0, "orc_spai random 1");
            CHECK(orc_spai(&b.A, &p8, rows, 300, variant == 3 ? cpr : NULL, &r8) == 0, "orc_spai random 8");
            CHECK(same_result(&r1, &r8), "random: thread counts give different results");
            orc_result_free(&r1);
            orc_result_free(&r8);
        }
        free(cpr);
        built_free(&b);
        csr_free(&B);
        csr_free(&B0);
    }
    printf("oracle sanitize driver ok\n");
    return 0;
}
