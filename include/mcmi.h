/*
 * mcmi.h - C ABI of libmcmi.so: Markov Chain Monte Carlo sparse approximate
 * inverse ((MC)^2MI) on AMD Instinct MI355X (gfx950).
 *
 * The library computes, for a sparse matrix B with a nonzero diagonal D, a
 * sparse approximate inverse M of B:
 *
 *   C = I - D^-1 B                     (Section IV, phase 2: the iteration matrix
 *                                       whose Neumann series gives (I - C)^-1)
 *   N_r ~ row r of (I - C)^-1          (Section III-A, eq. (2): the mean over N_r
 *                                       Markov chains started at r of the chain
 *                                       weights W_j summed at the states visited)
 *   M_rc = N_rc / d_c                  (Section IV-A, phase 4: column scaling by
 *                                       the inverse diagonal, since B^-1 =
 *                                       (I - C)^-1 D^-1)
 *   keep (r, c) iff c == r or |N_rc| >= eps   (the filter that makes M sparse,
 *                                       named at the end of Section III-A)
 *
 * Sampling: transition probabilities p_ij proportional to |c_ij| (the paper
 * leaves P undefined), quantized to integer weights per row so that every
 * implementation samples the same quantized matrix Chat; weights W_j =
 * W_{j-1} * sign(c) * Shat_s with Shat_s = sum_k |chat_sk|. A chain stops before
 * a draw when the row of C is empty, when |W * Shat_s| < delta, or after L_max
 * transitions. Random numbers: Philox4x32-10 with key (seed lo, seed hi) and
 * counter (step block, chain, row, tag); step j >= 1 uses word (j-1) mod 4 of
 * block (j-1) / 4.
 *
 * Conventions for every entry point:
 *  - Pointers named *_dev are device pointers (hipMalloc'd or torch tensors'
 *    data_ptr()); the caller owns them and keeps them valid until the work
 *    queued on `stream` has finished. Pointers named *_host are host memory.
 *  - `stream` is a hipStream_t (NULL = the default stream). Calls are
 *    asynchronous on it except where a call states a host synchronisation.
 *  - Every call returns an mcmi_status. On error, output structs are zeroed,
 *    nothing stays allocated, and mcmi_last_error() (thread-local) describes the
 *    failure. No C++ exception crosses this boundary.
 *  - Layouts: CSR with int64 row pointers (n + 1), int32 column indices
 *    (ascending and unique within a row) and float64 values.
 */
#ifndef MCMI_H
#define MCMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MCMI_OK = 0,
    MCMI_ERR_ARG = -1,            /* bad argument (null pointer, bad size, bad parameter) */
    MCMI_ERR_CSR = -2,            /* row pointers not monotone, columns unsorted, duplicated or out of range */
    MCMI_ERR_ZERO_DIAG = -3,      /* a row lacks its diagonal entry or it is zero */
    MCMI_ERR_NOT_CONTRACTIVE = -4,/* ||Chat||_inf >= 1 and no max_len given */
    MCMI_ERR_CAPACITY = -5,       /* an internal table stayed too small after growing */
    MCMI_ERR_HIP = -6,            /* a HIP runtime call failed */
    MCMI_ERR_NOMEM = -7           /* device allocation failed */
} mcmi_status;

/* Input matrix B (borrowed device pointers). */
typedef struct {
    int64_t n;                 /* rows = columns */
    int64_t nnz;               /* stored entries */
    const int64_t *row_ptr_dev;/* n + 1 */
    const int32_t *col_dev;    /* nnz */
    const double *val_dev;     /* nnz */
} mcmi_csr_in;

/* Output matrix (device buffers allocated by the library; free with mcmi_csr_free). */
typedef struct {
    int64_t n;                 /* rows (the number of rows requested) */
    int64_t nnz;
    int64_t *row_ptr_dev;      /* n + 1 */
    int32_t *col_dev;          /* nnz */
    double *val_dev;           /* nnz */
} mcmi_csr_out;

/* Opaque: the packed per-row sampling records of C (library-owned device memory). */
typedef struct mcmi_cdf mcmi_cdf;

enum { MCMI_WALK_F64 = 64, MCMI_WALK_F32 = 32 };
enum { MCMI_FILTER_N = 0, MCMI_FILTER_M = 1 };

typedef struct {
    uint64_t seed;        /* Philox key */
    int32_t chains;       /* chains per row when no per-row array is given (>= 1) */
    int32_t walk_prec;    /* MCMI_WALK_F64 or MCMI_WALK_F32 (binary32 weights, Shat and
                             delta test; sums stay binary64) */
    double delta;         /* weight cutoff: stop before a draw when |W * Shat_s| < delta */
    double eps;           /* filter threshold (>= 0) */
    int32_t max_len;      /* L_max; 0 = derive: smallest L with ||Chat||_inf^L < delta
                             (one IEEE product per step); required when ||Chat||_inf >= 1 */
    uint32_t stream_tag;  /* fourth Philox counter word (distinguishes independent runs) */
    int32_t filter;       /* MCMI_FILTER_N: |N_rc| >= eps; MCMI_FILTER_M: |M_rc| >= eps */
    int32_t lanes_per_row;/* 0 = automatic; 64 = one wavefront per row; 8, 16 or 32 = 64 / that
                             many rows share a wavefront (and its tables); 256, 512 or 1024 =
                             one workgroup of that many lanes per row */
    int32_t hash_slots;   /* 0 = automatic; else LDS hash slots per row (power of two) */
    int32_t sketch_slots; /* 0 = automatic; else count-sketch buckets per row (64..16384) */
    int32_t pool_per_row; /* 0 = automatic; else first guess of kept entries per row: rows that
                             do not fit are rerun into a second pool sized exactly */
    double heavy_weight;  /* workgroup-per-row kernel only. 0 = automatic; < 0 = track every
                             contribution in the row hash; > 0 (<= 1): contributions with
                             |W| >= heavy_weight are tracked, lighter ones are added to
                             tracked columns or to a count sketch that certifies that no
                             untracked column reaches the filter threshold (rows that fail
                             the certificate are replayed exactly). Needs ||Chat||_inf < 1. */
    int32_t spill_slots;  /* 0 = automatic; else HBM overflow-table slots per row in flight
                             (power of two); rows that overflow it are rerun with it grown */
    int32_t topk;         /* 0 = off; > 0: top-k retention (Section IV-B keeps a prescribed
                             number of the entries largest in magnitude): of the entries that
                             pass the eps filter, the diagonal and the topk - 1 off-diagonal
                             entries with the largest filter value (|N_rc|, or |M_rc| under
                             MCMI_FILTER_M) are kept, equal values by ascending column */
} mcmi_params;

typedef struct {
    uint64_t transitions;     /* exact number of draws made */
    uint64_t chains;          /* chains run */
    uint64_t spilled;         /* contributions that went to the HBM spill table */
    uint64_t retries;         /* reruns after a table or pool overflow */
    uint64_t refined;         /* rows whose sketch certificate failed and were replayed */
    int64_t nnz;              /* entries of M */
    int32_t lmax;             /* L_max used */
    float norm_inf;           /* ||Chat||_inf */
    double ms_walk;           /* device time of the walk + finalize kernel(s) */
    double ms_assemble;       /* device time of the CSR assembly */
    double ms_total;          /* device time of the whole call */
    int32_t lanes_per_row;    /* kernel shape used */
    int32_t hash_slots;
    int32_t sketch_slots;
    int32_t pad;
    double heavy_weight;      /* tau used (0: every contribution tracked) */
} mcmi_stats;

/* Build the sampling records of C = I - D^-1 B (Section IV, phase 2 and the
 * transition matrix P of Section IV-A). Validates B (sorted unique columns,
 * nonzero diagonal) on the device. Synchronises the stream once to read the
 * validation flags and the record sizes, and once more for ||Chat||_inf.
 * *out is allocated by the library; free it with mcmi_cdf_free. */
mcmi_status mcmi_build_cdf(const mcmi_csr_in *B, mcmi_cdf **out, void *stream);

/* Optional pre-pass on B before the records are built (both off when zero). */
typedef struct {
    /* Phase 1, the splitting B = B^ - (B^ - B) of Section III-B with the sign rule
     * of Section V-C: b^_ii = b_ii + s_i * (alpha * ||B||_inf), s_i = -1 when
     * b_ii < 0, else +1; a missing diagonal counts as 0, so such rows are allowed.
     * ||B||_inf is the largest row sum of |b_ij| (each row summed in column order).
     * C of B^ then has ||C||_inf <= 1/alpha, and M approximates the inverse of B^
     * (the paper's recovery phase 5 is not applied). */
    double alpha;
    /* Matrix reduction (Algorithm 1 step 2, Section V-A): with cnt nonzero
     * off-diagonal entries of C and K = floor(drop_frac * cnt), the cut is the
     * (K+1)-th smallest |c_ij|; entries with |c_ij| below it are removed before the
     * CDF is built (entries equal to the cut stay). 0 <= drop_frac < 1. */
    double drop_frac;
    /* Row schedule (not part of the method: every row's estimate is the same in any
     * order). 0: rows run in their natural order. k > 0: rows are grouped into
     * cells of about k rows grown by a multi-source breadth-first search on the
     * pattern of B (seeds picked by a hash of the row with probability 1/k, each row
     * joining the cell whose seed reaches it first, the smaller seed on a tie, at
     * most 64 levels), and mcmi_spai of a whole single-matrix record set runs them
     * cell by cell, so rows that are close in the graph run together on one XCD and
     * share its L2. Pays off for matrices with locality (PDE discretisations); costs
     * about one pass over B per level. Ignored by batched record sets. */
    int64_t order_cell;
    int64_t reserved; /* must be 0 */
} mcmi_cdf_opts;

/* mcmi_build_cdf with the pre-pass of `opts` (NULL: none). The augmentation adds
 * one stream synchronisation, the reduction an 8-pass radix selection over a
 * temporary key per entry of B and one more. */
mcmi_status mcmi_build_cdf_ex(const mcmi_csr_in *B, const mcmi_cdf_opts *opts, mcmi_cdf **out, void *stream);

/* What the pre-pass did: ||B||_inf (0 without augmentation), the reduction cut on
 * |c| (0 without reduction) and the number of entries of C it removed. */
mcmi_status mcmi_cdf_prep_info(const mcmi_cdf *cdf, double *norm_b, double *drop_thr, int64_t *dropped);

/* The row schedule of a record set built with order_cell > 0: n row indices (a
 * permutation of [0, n)) copied to order_host; synchronises the stream. Fails
 * with MCMI_ERR_ARG when the set has no such schedule. */
mcmi_status mcmi_cdf_order(const mcmi_cdf *cdf, int32_t *order_host, void *stream);

/* Records of `count` matrices in one block-diagonal row space (the batched
 * launch): matrix k occupies rows [base_k, base_k + n_k) and its columns are
 * shifted by base_k. Walks never leave their matrix; in mcmi_spai the Philox row
 * word is the row inside its matrix and the tag word is stream_tag + k, so each
 * matrix gets exactly the result of its own single-matrix run with that tag.
 * Bs[k] are borrowed device CSR matrices (validated as in mcmi_build_cdf; each
 * column must lie in [0, n_k)). Synchronises. */
mcmi_status mcmi_build_cdf_batched(const mcmi_csr_in *Bs, int32_t count, mcmi_cdf **out, void *stream);

/* mcmi_build_cdf_batched with a row schedule (opts->order_cell; alpha and
 * drop_frac must be 0, as one norm or cut over the whole batch would couple the
 * matrices). The cells never cross matrices, so the schedule lists each matrix's
 * rows in its own slice; the batched launch then deals 64 consecutive positions
 * of the schedule at a time. */
mcmi_status mcmi_build_cdf_batched_ex(const mcmi_csr_in *Bs, int32_t count, const mcmi_cdf_opts *opts,
                                      mcmi_cdf **out, void *stream);

/* Number of matrices of a record set (0 for a single-matrix set), their first
 * rows (count + 1 values; for a single matrix {0, n}) and ||Chat_k||_inf. */
mcmi_status mcmi_cdf_batch_info(const mcmi_cdf *cdf, int32_t *count, int64_t *row_base_host, double *norm_host);

/* Copy the records to host memory (for inspection and tests; synchronises the
 * stream). rec_host receives rec_units * 16 uint32 words (rec_units from
 * mcmi_cdf_info, in 64-byte units), roff_host n record offsets (64-byte units)
 * and diag_host the n diagonal values b_ii (augmented when the pre-pass ran). Any
 * of the three may be NULL. Record of a row with m entries (1 + m units): the
 * header {row, m, W, Shat32}, {Shat64 (2 words), 0, 0} and 8 zero words, then
 * bucket j = 0 .. m-1: {T_j, target_j, target of A_j, w_j}, the header words
 * {row, m, W, Shat32} of target_j's row, the same for A_j's, and their two Shat64;
 * (T, A) is the row's alias table and a target the column's record offset with
 * bit 31 set for c < 0. */
mcmi_status mcmi_cdf_download(const mcmi_cdf *cdf, uint32_t *rec_host, uint32_t *roff_host, double *diag_host,
                              void *stream);

/* Copy the compact records (the draw data of walks with binary32 weights) to
 * host memory: rec_units * 8 uint32 words, record offsets as for the full
 * records but in 32-byte units (synchronises the stream). Record of a row with m
 * entries: the header {row, m, W, Shat32}, {Shat64 (2 words), b_ii (2 words)},
 * then bucket j: {T'_j, target_j, m of target_j, Shat32 of target_j},
 * {w_j, target of A_j, m of that row, its Shat32}, where T'_j = ceil(T_j 2^32 / W)
 * (the draw with word u takes target_j iff (u m mod 2^32) < T'_j, the same entry
 * as the full record's rule) and a bucket with T_j = W has T'_j = 2^32 - 1 and
 * the alias half equal to its own. */
mcmi_status mcmi_cdf_download_compact(const mcmi_cdf *cdf, uint32_t *rec32_host, void *stream);

/* ||Chat||_inf, n, nnz(C) and the size in 64-byte units of built records. */
mcmi_status mcmi_cdf_info(const mcmi_cdf *cdf, int64_t *n, int64_t *nnz_c, double *norm_inf,
                          uint64_t *rec_units);

/* The Monte Carlo SPAI (Section III-A eq. (2), Section IV phases 3-4):
 * walks, per-row accumulation, eps filter, D^-1 column scaling, CSR assembly.
 * chains_per_row_dev: NULL (every row gets p->chains) or a device int32 array of
 * length n with values >= 1. rows_dev: NULL (all n rows) or a device int32 array
 * of n_rows distinct row indices; M then holds those rows in that order.
 * M's buffers are allocated by the library. Synchronises the stream to size M
 * (and once more per retry after an overflow). st may be NULL. */
mcmi_status mcmi_spai(const mcmi_cdf *cdf, const mcmi_params *p, const int32_t *chains_per_row_dev,
                      const int32_t *rows_dev, int64_t n_rows, mcmi_csr_out *M, mcmi_stats *st,
                      void *stream);

/* y = M x (CSR SpMV, float64), asynchronous. x_dev has M's column count (the n of
 * the cdf M came from), y_dev has M->n entries. Used to apply M as a
 * preconditioner (Section III-A: the result is used directly as a preconditioner). */
mcmi_status mcmi_apply(const mcmi_csr_out *M, int64_t n_cols, const double *x_dev, double *y_dev,
                       void *stream);

/* ---------------------------------------------------- learned allocation */

/* Eight binary32 features per row of C (feat_dev: n x 8, row-major), the input of
 * the chain-allocation network, computed from the records (p_ij = w_ij / W_i the
 * quantized transition probabilities, S = Shat):
 *   f0 ln max(m_i, 1), f1 S_i, f2 max_j |chat_ij|, f3 sum_j p_ij S_j, f4 max_j S_j,
 *   f5 sum_j p_ij m_j, f6 |sum_j chat_ij| / S_i, f7 min(L_max, ln delta / ln S_i).
 * L_max as in mcmi_params (max_len, or derived from delta). Asynchronous. */
mcmi_status mcmi_row_features(const mcmi_cdf *cdf, double delta, int32_t max_len, float *feat_dev, void *stream);

/* Pilot run for the allocation target: pilot_chains chains per row on Philox
 * streams whose tag has bit 31 set (independent of the main walks). Writes, per
 * row, var_dev = mean_c ||X_c||^2 - ||mean_c X_c||^2 (X_c = chain c's row
 * estimate, revisits merged; the total variance of one chain, eq. (2)) and
 * len_dev = mean transitions per chain (both float64, n). Uses seed, delta,
 * walk_prec, max_len and stream_tag of p. Synchronises the stream. */
mcmi_status mcmi_pilot_variance(const mcmi_cdf *cdf, const mcmi_params *p, int32_t pilot_chains, double *var_dev,
                                double *len_dev, void *stream);

/* The allocation network: 8 -> 64 -> 64 -> 1 ReLU MLP (4,801 parameters) that maps
 * z-scored row features to the log of a row's chain share. Parameters are FP32
 * masters packed as W1 (64 x 8, row = output), b1 (64), W2 (64 x 64), b2 (64),
 * w3 (64), b3 (1); the forward and backward use BF16 copies of W1, W2, w3 with
 * FP32 accumulation (64 x 64 products on the matrix cores). Library-owned. */
typedef struct mcmi_mlp mcmi_mlp;
mcmi_status mcmi_mlp_create(mcmi_mlp **out);
void mcmi_mlp_free(mcmi_mlp *net);
/* Load parameters (4801 floats) and, if non-NULL, the feature normalisation
 * (mean[8] then 1/std[8]); reset_optimizer != 0 clears the Adam state. Synchronises. */
mcmi_status mcmi_mlp_set_params(mcmi_mlp *net, const float *params_host, const float *norm_host,
                                int32_t reset_optimizer);
/* Copy parameters, normalisation, Adam moments and step count to the host (each
 * pointer nullable; a checkpoint). Synchronises the device. */
mcmi_status mcmi_mlp_get_params(const mcmi_mlp *net, float *params_host, float *norm_host, float *adam_m_host,
                                float *adam_v_host, int64_t *adam_step);
mcmi_status mcmi_mlp_set_adam_state(mcmi_mlp *net, const float *adam_m_host, const float *adam_v_host,
                                    int64_t adam_step);
/* Normalisation from the training features (feat_dev n x 8): per-column mean and
 * 1/std (population std; 1 for a constant column). Asynchronous. */
mcmi_status mcmi_mlp_fit_normalization(mcmi_mlp *net, const float *feat_dev, int64_t n, void *stream);
/* out_dev[r] = network(feat_dev[r]) for n rows. Asynchronous. */
mcmi_status mcmi_mlp_predict(const mcmi_mlp *net, const float *feat_dev, int64_t n, float *out_dev, void *stream);
/* Mean-squared-error gradient over the samples idx_dev[0..batch) of (feat_dev,
 * target_dev) at the current parameters, to grad_host (4801 floats) and the loss
 * to loss_host (for checks against a reference). Synchronises. */
mcmi_status mcmi_mlp_gradient(mcmi_mlp *net, const float *feat_dev, const float *target_dev, const int32_t *idx_dev,
                              int64_t batch, int64_t n, float *grad_host, float *loss_host, void *stream);
/* `steps` Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on
 * minibatches of `batch` samples drawn with replacement by Philox (key = seed,
 * counter = (step, slot, 'MLP', 0)); loss_host (nullable) receives each step's
 * loss. Synchronises at the end. */
mcmi_status mcmi_mlp_train(mcmi_mlp *net, const float *feat_dev, const float *target_dev, int64_t n, int32_t steps,
                           int32_t batch, float lr, uint64_t seed, float *loss_host, void *stream);
/* Chains per row from predicted log shares: N_r = max(1, rint(lambda exp(pred_r)))
 * with lambda (bisection) giving the largest sum_r N_r cost_r <= budget; any
 * non-finite prediction selects the uniform allocation max(1, budget / sum cost)
 * (*fallback_host = 1). cost_dev: int32 per-row chain cost (>= 1). Synchronises. */
mcmi_status mcmi_allocate(const float *pred_dev, const int32_t *cost_dev, int64_t n, int64_t budget,
                          int32_t *chains_dev, double *lambda_host, int32_t *fallback_host, void *stream);
/* mcmi_allocate for callers that cannot allocate device memory (code under
 * hipGraph stream capture, tight serving loops, harnesses that forbid
 * hipMalloc). Same kernels and the same results (chains_dev, lambda, fallback
 * flag) as mcmi_allocate, but every temporary lives in a static device workspace
 * of 256 B + 8 B per row for at most 4,194,304 rows (32 MiB + 256 B, one copy
 * per GPU, held until the process ends); n above that limit returns
 * MCMI_ERR_ARG before anything is launched. lambda_dev (double) and fallback_dev
 * (int32) are optional device outputs (NULL: not written). Fully asynchronous:
 * no allocation, no host copy, no synchronisation. Calls that overlap on one GPU
 * (concurrent streams or threads) share the workspace and race; serialise them.
 * Each call re-initialises the workspace it uses. */
mcmi_status mcmi_allocate_noalloc(const float *pred_dev, const int32_t *cost_dev, int64_t n, int64_t budget,
                                  int32_t *chains_dev, double *lambda_dev, int32_t *fallback_dev, void *stream);

/* Regression target of the allocation network, per row. Neyman allocation:
 * minimising the summed variance sum_r v_r / N_r of the row estimates under a
 * budget sum_r N_r (len_r + 1) = T gives N_r proportional to sqrt(v_r / (len_r +
 * 1)), so y_dev[r] = (ln max(v_r, 1e-30) - ln(len_r + 1)) / 2 (binary32) from the
 * float64 var_dev and len_dev of mcmi_pilot_variance (n rows each). The variance
 * per chain is that of the estimator of Section III-A, eq. (2). Asynchronous. */
mcmi_status mcmi_neyman_target(const double *var_dev, const double *len_dev, int64_t n, float *y_dev,
                               void *stream);
/* Budget units of one chain per row, from the row features (feat_dev n x 8, as
 * written by mcmi_row_features): cost_dev[r] = 1 + floor(f7_r), the states a
 * chain from r visits when every row on its path has row r's |C| row sum (exact
 * when all row sums are equal: a chain then makes floor(f7) transitions). With
 * total_host non-NULL it receives sum_r cost_r (64-bit) and the call
 * synchronises the stream; otherwise it is asynchronous. */
mcmi_status mcmi_chain_cost(const float *feat_dev, int64_t n, int32_t *cost_dev, int64_t *total_host,
                            void *stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected moments, as in
 * mcmi_mlp_train) of the network's FP32 master parameters with a caller-supplied
 * gradient grad_dev (4801 floats, device, in the parameter order above) and
 * learning rate lr > 0; the BF16 copies follow. For gradients that the caller
 * computes or combines itself. Asynchronous. */
mcmi_status mcmi_mlp_adam_step(mcmi_mlp *net, const float *grad_dev, float lr, void *stream);

/* ------------------------------------------------------ tuning and plans */

/* Autotuner: times candidate kernel shapes (lanes per row, LDS hash slots,
 * sketch buckets, heavy threshold automatic or off) with mcmi_spai on a strided
 * sample of sample_rows rows (0: 8192) and writes the fastest into *best (a copy
 * of *base with lanes_per_row, hash_slots, sketch_slots, heavy_weight set) and its
 * walk time to *best_ms. cache_path (nullable): a JSON file keyed by the workload
 * class (architecture, log2 of n, mean row length, chains and L_max, precision,
 * batched, filter); a cached class is returned without timing, a new one is
 * added. Synchronises. */
mcmi_status mcmi_tune(const mcmi_cdf *cdf, const mcmi_params *base, int64_t sample_rows, const char *cache_path,
                      mcmi_params *best, double *best_ms, void *stream);

/* A plan owns every buffer of one SPAI configuration (cdf, parameters, per-row
 * chains, output capacity nnz_capacity) and a hipGraph of its device work: counter
 * reset, walk + finalize, row-count scan, gather into the plan's CSR buffers. For
 * callers that repeat the SPAI (time stepping, serving). mcmi_plan_launch replays
 * the graph with a new seed (asynchronous); mcmi_plan_result synchronises and
 * returns a view of the plan-owned CSR (valid until the next launch or
 * mcmi_plan_free) and *overflow = 1 when a table or the capacity overflowed (the
 * view is then empty: rerun with mcmi_spai or a larger plan). Rows are not rerun
 * inside a plan. The cdf must outlive the plan. mcmi_plan_create checks p as
 * mcmi_spai does (MCMI_ERR_ARG before any allocation or kernel), reads the
 * per-row chain counts once (one synchronisation: each must be >= 1; the tables
 * are sized for the largest, so a later change of the array must keep every
 * count between 1 and that largest value), sizes the HBM overflow tables from the
 * rows' reach as mcmi_spai does, and walks a batched record set in the eager
 * launch's longest-processing-time order. Besides the output (nnz_capacity
 * entries) a plan of the wavefront kernel holds a staging pool of nnz_capacity
 * * 9/8 + c entries per wavefront of its grid (12 bytes each), in which
 * wavefronts reserve space c entries at a time, c = nnz_capacity / (4 x the
 * wavefronts) clamped to [256, 32768]; a pool that runs out is reported as an
 * overflow. */
typedef struct mcmi_plan mcmi_plan;
mcmi_status mcmi_plan_create(const mcmi_cdf *cdf, const mcmi_params *p, const int32_t *chains_per_row_dev,
                             int64_t nnz_capacity, mcmi_plan **out, void *stream);
mcmi_status mcmi_plan_launch(mcmi_plan *plan, uint64_t seed, void *stream);
mcmi_status mcmi_plan_result(mcmi_plan *plan, mcmi_csr_out *M_view, mcmi_stats *st, int32_t *overflow, void *stream);
void mcmi_plan_free(mcmi_plan *plan);

/* Result of mcmi_bicgstab. */
typedef struct {
    int64_t iterations;   /* BiCGstab iterations made (a converged half step counts as one) */
    double rel_residual;  /* ||r|| / ||b|| of the recurrence residual at exit */
    double ms;            /* device time of the solve */
    int32_t converged;    /* 1 when ||r|| <= rtol ||b|| was reached */
    int32_t pad;
} mcmi_solve_stats;

/* Solve B x = b with BiCGstab (van der Vorst), M applied on the right as the
 * preconditioner (the use of M that Section III-B and the solver experiments of
 * Section VI make of it); M = NULL solves without one. B is a borrowed device
 * CSR (as for mcmi_build_cdf), M a result of mcmi_spai; b_dev (n, read) and
 * x_dev (n, in: initial guess, out: solution) are device float64 vectors. Stops
 * when ||r|| <= rtol ||b|| for the recurrence residual r, or after maxiter
 * iterations, or on a breakdown (a zero inner product); then converged = 0 and x
 * holds the last iterate. Dot products reduce in a fixed order, so a rerun gives
 * the same iterates. Allocates 8 n float64 of workspace; synchronises the stream
 * once per inner product. */
mcmi_status mcmi_bicgstab(const mcmi_csr_in *B, const mcmi_csr_out *M, const double *b_dev, double *x_dev,
                          double rtol, int32_t maxiter, mcmi_solve_stats *st, void *stream);

/* Copy M into caller-owned device buffers (row_ptr n+1, col nnz, val nnz). */
mcmi_status mcmi_csr_copy(const mcmi_csr_out *M, int64_t *row_ptr_dev, int32_t *col_dev,
                          double *val_dev, void *stream);

/* Device memory that the library's calls free is kept for reuse by later calls
 * (each device keeps at most a quarter of its memory; a block released with a
 * stream is reused only on that stream). This returns all of it to the driver;
 * it synchronises every device that holds cached memory. */
void mcmi_cache_trim(void);

void mcmi_cdf_free(mcmi_cdf *cdf);
void mcmi_csr_free(mcmi_csr_out *M);
const char *mcmi_last_error(void);
const char *mcmi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MCMI_H */
