// Autotuner and captured plans (gfx950).
//
// mcmi_tune: times candidate kernel shapes (lanes per row, rows sharing a
// wavefront, LDS hash slots,
// count-sketch buckets, heavy threshold) on a strided sample of rows and keeps the
// fastest walk; results are cached in a JSON file keyed by the workload class
// (architecture, log2 buckets of n, mean entries per row, chains, chain length,
// precision, batched or not).
//
// mcmi_plan: everything of one SPAI configuration allocated once and its device
// work captured in a hipGraph (counter reset kernel -> walk -> row-count scan ->
// gather into fixed-capacity CSR buffers); each launch replays the graph with a
// new seed. No memset node is recorded: counters are cleared by a kernel, and the
// walk leaves its HBM overflow tables clean. The walk runs as the eager launch
// does: the same task order (locality schedule, or LPT order on batched sets) and
// wavefronts reserving output space in chunks (pool_chunk_for) in a pool of the
// plan's own, sized for the caller's capacity plus those reservations.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "common.hpp"
#include "walk_args.hpp"

namespace mcmi {

size_t walk_lds_bytes(int hash_slots, int waves);
hipError_t launch_walk(const WalkArgs &a, bool f32, int blocks, int waves, hipStream_t s);
hipError_t walk_occupancy(bool f32, int hash_slots, int waves, int *blocks_per_cu);
bool walk_block_supported(int lanes, int hash_slots);
hipError_t launch_walk_block(const WalkArgs &a, bool f32, int lanes, int blocks, hipStream_t s);
hipError_t walk_block_occupancy(bool f32, int lanes, int hash_slots, int sketch_slots, int *bpc);
hipError_t batched_lpt_map(const mcmi_cdf *cdf, double delta, int lmax, int n_hint, int32_t *map, hipStream_t s);
hipError_t gather_rows(int64_t n_rows, const int64_t *row_start, const uint32_t *row_cnt, const int64_t *row_ptr,
                       const PoolSet &pools, int64_t cap, int32_t *col, double *val, hipStream_t s);

namespace {

__global__ void k_zero_words(uint32_t *p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

// seed from device memory so that each graph replay can use a new one
__global__ void k_set_keys(const uint64_t *seed, uint32_t *keys) {
    if (threadIdx.x == 0) {
        keys[0] = (uint32_t)(*seed & 0xffffffffu);
        keys[1] = (uint32_t)(*seed >> 32);
    }
}

std::string tune_key(const mcmi_cdf *cdf, const mcmi_params *p, int lmax) {
    auto lg = [](double x) { return x > 0 ? (int)std::floor(std::log2(x)) : -1; };
    char buf[256];
    const double m_bar = cdf->n ? (double)cdf->nnz_c / (double)cdf->n : 0.0;
    snprintf(buf, sizeof(buf), "gfx950|n%d|m%d|N%d|L%d|p%d|b%d|f%d", lg((double)cdf->n), lg(m_bar),
             lg((double)std::max(p->chains, 1)), lg((double)lmax), p->walk_prec, cdf->batch > 0 ? 1 : 0, p->filter);
    return buf;
}

struct TuneEntry {
    int lanes, hash, sketch;
    double tau, ms;
};

std::map<std::string, TuneEntry> read_cache(const char *path) {
    std::map<std::string, TuneEntry> out;
    if (!path) return out;
    FILE *f = fopen(path, "r");
    if (!f) return out;
    char line[512];
    while (fgets(line, sizeof(line), f)) {
        char key[256];
        TuneEntry e;
        if (sscanf(line, " \"%255[^\"]\" : [ %d , %d , %d , %lf , %lf ]", key, &e.lanes, &e.hash, &e.sketch, &e.tau,
                   &e.ms) == 6)
            out[key] = e;
    }
    fclose(f);
    return out;
}

bool write_cache(const char *path, const std::map<std::string, TuneEntry> &m) {
    if (!path) return true;
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return false;
    fprintf(f, "{\n");
    size_t k = 0;
    for (const auto &kv : m) {
        fprintf(f, "  \"%s\": [%d, %d, %d, %.17g, %.6f]%s\n", kv.first.c_str(), kv.second.lanes, kv.second.hash,
                kv.second.sketch, kv.second.tau, kv.second.ms, ++k < m.size() ? "," : "");
    }
    fprintf(f, "}\n");
    fclose(f);
    return rename(tmp.c_str(), path) == 0;
}

}  // namespace
}  // namespace mcmi

using namespace mcmi;

extern "C" mcmi_status mcmi_tune(const mcmi_cdf *cdf, const mcmi_params *base, int64_t sample_rows,
                                 const char *cache_path, mcmi_params *best, double *best_ms, void *stream) {
    if (!cdf || !base || !best) return fail(MCMI_ERR_ARG, "mcmi_tune: null argument");
    if (base->chains < 1) return fail(MCMI_ERR_ARG, "mcmi_tune: needs a uniform chain count (chains >= 1)");
    const int lmax = derive_lmax(cdf->norm_inf, base->delta, base->max_len);
    if (lmax < 0) return fail(MCMI_ERR_ARG, "mcmi_tune: bad delta / max_len or not contractive");
    const std::string key = tune_key(cdf, base, lmax);
    auto cache = read_cache(cache_path);
    *best = *base;
    auto it = cache.find(key);
    if (it != cache.end()) {
        best->lanes_per_row = it->second.lanes;
        best->hash_slots = it->second.hash;
        best->sketch_slots = it->second.sketch;
        best->heavy_weight = it->second.tau;
        if (best_ms) *best_ms = it->second.ms;
        return MCMI_OK;
    }
    hipStream_t s = (hipStream_t)stream;
    // strided row sample (for batched sets it spans every matrix)
    const int64_t ns = std::max<int64_t>(1, std::min<int64_t>(sample_rows > 0 ? sample_rows : 8192, cdf->n));
    std::vector<int32_t> rows(ns);
    for (int64_t k = 0; k < ns; ++k) rows[k] = (int32_t)((k * cdf->n) / ns);
    int32_t *rows_dev = nullptr;
    MCMI_HIP(hipMalloc(&rows_dev, ns * sizeof(int32_t)));
    MCMI_HIP(hipMemcpy(rows_dev, rows.data(), ns * sizeof(int32_t), hipMemcpyHostToDevice));
    struct Cand {
        int lanes, hash, sketch;
        double tau;
    };
    std::vector<Cand> cands = {{64, 512, 0, 0},  {64, 1024, 0, 0}, {64, 2048, 0, 0},
                               {32, 1024, 0, 0}, {32, 2048, 0, 0}, {16, 1024, 0, 0}, {8, 1024, 0, 0}};
    for (int lanes : {256, 512, 1024})
        for (int hash : {2048, 4096})
            if (walk_block_supported(lanes, hash))
                for (int sk : {0, 4096, 16384}) {  // 0: the largest sketch leaving two workgroups
                                                     // per CU; 16384: one workgroup per CU
                    cands.push_back({lanes, hash, sk, 0.0});  // automatic tau
                    if (sk == 0) cands.push_back({lanes, hash, sk, -1.0});  // track everything
                }
    double best_t = 1e300;
    Cand win = cands[0];
    for (const Cand &c : cands) {
        mcmi_params q = *base;
        q.lanes_per_row = c.lanes;
        q.hash_slots = c.hash;
        q.sketch_slots = c.sketch;
        q.heavy_weight = c.tau;
        double t = 0.0;
        bool ok = true;
        for (int rep = 0; rep < 2 && ok; ++rep) {
            mcmi_csr_out M;
            mcmi_stats st;
            if (mcmi_spai(cdf, &q, nullptr, rows_dev, ns, &M, &st, s) != MCMI_OK) {
                ok = false;
                break;
            }
            mcmi_csr_free(&M);
            t = st.ms_walk;  // second run's time
        }
        if (ok && t < best_t) {
            best_t = t;
            win = c;
        }
    }
    (void)hipFree(rows_dev);
    if (best_t >= 1e300) return fail(MCMI_ERR_CAPACITY, "mcmi_tune: no candidate ran");
    best->lanes_per_row = win.lanes;
    best->hash_slots = win.hash;
    best->sketch_slots = win.sketch;
    best->heavy_weight = win.tau;
    if (best_ms) *best_ms = best_t;
    cache[key] = TuneEntry{win.lanes, win.hash, win.sketch, win.tau, best_t};
    if (!write_cache(cache_path, cache)) return fail(MCMI_ERR_ARG, "mcmi_tune: cannot write the cache file");
    set_error("");
    return MCMI_OK;
}

// ---------------------------------------------------------------- plans
struct mcmi_plan {
    const mcmi_cdf *cdf = nullptr;
    int64_t n = 0, cap = 0, pool_cap = 0;
    void *ctrl = nullptr;       // queue counters, pool_used, stats, flags, keys
    int64_t *row_start = nullptr, *row_ptr = nullptr;
    uint32_t *row_cnt = nullptr;
    int32_t *pool_col = nullptr, *col = nullptr, *sk = nullptr, *su = nullptr;
    double *pool_val = nullptr, *val = nullptr, *sv = nullptr;
    uint64_t *seed = nullptr;
    void *scan_tmp = nullptr;
    int32_t *lpt = nullptr;     // batched sets: longest-processing-time task order
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int lmax = 0;
    int32_t chunk = 0;  // pool entries a wavefront reserves at a time
    KernelShape shape;
};

extern "C" void mcmi_plan_free(mcmi_plan *pl) {
    if (!pl) return;
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    for (void *p : {(void *)pl->ctrl, (void *)pl->row_start, (void *)pl->row_ptr, (void *)pl->row_cnt,
                    (void *)pl->pool_col, (void *)pl->col, (void *)pl->sk, (void *)pl->su, (void *)pl->pool_val,
                    (void *)pl->val, (void *)pl->sv, (void *)pl->seed, pl->scan_tmp, (void *)pl->lpt})
        (void)hipFree(p);
    delete pl;
}

extern "C" mcmi_status mcmi_plan_create(const mcmi_cdf *cdf, const mcmi_params *p, const int32_t *chains_per_row_dev,
                                        int64_t nnz_capacity, mcmi_plan **out, void *stream) {
    if (out) *out = nullptr;
    if (!cdf || !p || !out || nnz_capacity < 1) return fail(MCMI_ERR_ARG, "mcmi_plan_create: bad argument");
    {
        const mcmi_status cst = check_walk_params(p, chains_per_row_dev != nullptr, "mcmi_plan_create");
        if (cst != MCMI_OK) return cst;
    }
    const int lmax = derive_lmax(cdf->norm_inf, p->delta, p->max_len);
    if (lmax < 0) return fail(MCMI_ERR_ARG, "mcmi_plan_create: bad delta / max_len or not contractive");
    hipStream_t s = (hipStream_t)stream;
    // the per-row chain counts are read once here (checked, largest and mean); a
    // replay walks the counts the array holds at that time, which must stay >= 1
    // and at most the largest seen here (the tables are sized for it)
    int n_max = p->chains, n_typ = p->chains;
    {
        const mcmi_status rst = read_chain_counts(cdf, p, nullptr, 0, chains_per_row_dev, n_max, n_typ, s,
                                                  "mcmi_plan_create");
        if (rst != MCMI_OK) return rst;
    }
    mcmi_plan *pl = new mcmi_plan();
    pl->cdf = cdf;
    pl->n = cdf->n;
    pl->cap = nnz_capacity;
    pl->pool_cap = nnz_capacity;
    pl->lmax = lmax;
    mcmi_status sst = choose_shape(cdf, p, lmax, n_max, n_typ, pl->shape);
    if (sst != MCMI_OK) {
        delete pl;
        return sst;
    }
    const WaveLayout layout = wave_layout(pl->shape, p->spill_slots, n_max, lmax);
    pl->shape.lanes = layout.lanes;
    const bool f32 = p->walk_prec == MCMI_WALK_F32;
    const bool block_kernel = pl->shape.lanes > 64;
    if (!f32) {  // FP32 walks read the compact records only
        const hipError_t fe = ensure_full_records(cdf, s);
        if (fe != hipSuccess) {
            delete pl;
            return fail(MCMI_ERR_HIP, std::string("mcmi_plan_create: ") + hipGetErrorString(fe));
        }
    }
    const int waves = 4;
    int bpc = 0;
    hipError_t e = block_kernel ? walk_block_occupancy(f32, pl->shape.lanes, pl->shape.hash, pl->shape.sketch, &bpc)
                                : walk_occupancy(f32, pl->shape.hash, waves, &bpc);
    if (e != hipSuccess || bpc < 1) {
        mcmi_plan_free(pl);
        return fail(MCMI_ERR_CAPACITY, "mcmi_plan_create: kernel does not fit");
    }
    int64_t blocks = (int64_t)bpc * device_cus();
    int64_t regions;
    if (block_kernel) {
        blocks = std::min<int64_t>(blocks, pl->n);
        regions = blocks;
    } else {
        if (blocks * waves > pl->n) blocks = std::max<int64_t>(1, (pl->n + waves - 1) / waves);
        regions = blocks * waves;
        // chunked reservations (as the eager launch's first pass makes them) leave
        // the tail of each wavefront's last chunk and the ends of chunks too short
        // for the next row unused: an eighth of the capacity plus one chunk per
        // wavefront covers them (a pool that still runs out is reported as an
        // overflow, like the output capacity)
        pl->chunk = pool_chunk_for(nnz_capacity, regions);
        pl->pool_cap = nnz_capacity + nnz_capacity / 8 + regions * (int64_t)pl->chunk;
    }
    const int spill_slots = layout.spill_slots;
    const size_t ctrl_bytes = kCtrlBytes;
#define TRYP(call)                                                                           \
    do {                                                                                     \
        hipError_t _e = (call);                                                              \
        if (_e != hipSuccess) {                                                              \
            mcmi_plan_free(pl);                                                              \
            return fail(MCMI_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(_e));    \
        }                                                                                    \
    } while (0)
    TRYP(hipMalloc(&pl->ctrl, ctrl_bytes));
    TRYP(hipMalloc(&pl->row_start, pl->n * sizeof(int64_t)));
    TRYP(hipMalloc(&pl->row_ptr, (pl->n + 1) * sizeof(int64_t)));
    TRYP(hipMalloc(&pl->row_cnt, pl->n * sizeof(uint32_t)));
    TRYP(hipMalloc(&pl->pool_col, pl->pool_cap * sizeof(int32_t)));
    TRYP(hipMalloc(&pl->pool_val, pl->pool_cap * sizeof(double)));
    TRYP(hipMalloc(&pl->col, pl->cap * sizeof(int32_t)));
    TRYP(hipMalloc(&pl->val, pl->cap * sizeof(double)));
    TRYP(hipMalloc(&pl->sk, (size_t)regions * spill_slots * sizeof(int32_t)));
    TRYP(hipMalloc(&pl->sv, (size_t)regions * spill_slots * sizeof(double)));
    TRYP(hipMalloc(&pl->su, (size_t)regions * spill_slots * sizeof(int32_t)));
    TRYP(hipMalloc(&pl->seed, sizeof(uint64_t)));
    TRYP(hipMalloc(&pl->scan_tmp, scan_tmp_bytes(pl->n)));
    if (cdf->batch > 0) {
        // the eager launch's order of a batched set, computed once for every replay
        TRYP(hipMalloc(&pl->lpt, pl->n * sizeof(int32_t)));
        TRYP(batched_lpt_map(cdf, p->delta, lmax, p->chains >= 1 ? p->chains : 64, pl->lpt, s));
    }
    // overflow tables start clean once; every walk leaves them clean again
    TRYP(hipMemsetAsync(pl->sk, 0xFF, (size_t)regions * spill_slots * sizeof(int32_t), s));
    TRYP(hipMemsetAsync(pl->sv, 0, (size_t)regions * spill_slots * sizeof(double), s));
    TRYP(hipStreamSynchronize(s));

    unsigned char *ctrl = (unsigned char *)pl->ctrl;
    WalkArgs a;
    memset(&a, 0, sizeof(a));
    a.rec = cdf->rec;
    a.rec32 = cdf->rec32;
    a.roff = cdf->roff;
    a.diag = cdf->diag;
    a.n_tasks = pl->n;
    a.row_lanes = block_kernel ? 0 : pl->shape.lanes;
    a.lane_chains = (!block_kernel && pl->shape.lanes == 64) ? pl->shape.lane_chains : 1;
    a.task_map = cdf->batch == 0 ? cdf->order : pl->lpt;  // locality schedule or LPT order, if any
    a.chains_per_row = chains_per_row_dev;
    a.chains = p->chains;
    a.keys_dev = (const uint32_t *)(ctrl + kCtrlKeys);
    a.tag = p->stream_tag;
    a.row_mat = cdf->batch > 0 ? cdf->row_mat : nullptr;
    a.mat_base = cdf->batch > 0 ? cdf->mat_base : nullptr;
    a.delta = p->delta;
    a.delta32 = (float)p->delta;
    a.eps = p->eps;
    a.lmax = lmax;
    a.filter_m = p->filter == MCMI_FILTER_M;
    a.topk = p->topk;
    a.hash_slots = pl->shape.hash;
    a.hash_shift = 32 - __builtin_ctz((unsigned)pl->shape.hash);
    a.queue_ctr = (uint32_t *)ctrl;
    a.row_start = pl->row_start;
    a.row_cnt = pl->row_cnt;
    a.pool_col = pl->pool_col;
    a.pool_val = pl->pool_val;
    a.pool_cap = pl->pool_cap;
    a.pool_chunk = block_kernel ? 0 : pl->chunk;
    a.pool_used = (unsigned long long *)(ctrl + kCtrlPool);
    a.spill_keys = pl->sk;
    a.spill_vals = pl->sv;
    a.spill_used = pl->su;
    a.spill_slots = spill_slots;
    a.stats = (unsigned long long *)(ctrl + kCtrlStats);
    a.flags = (uint32_t *)(ctrl + kCtrlFlags);
    a.tau = pl->shape.tau;
    a.tau32 = (float)pl->shape.tau;
    a.sketch_slots = pl->shape.sketch;

    hipStream_t cs;
    TRYP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t ce = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (ce == hipSuccess) {
        // counters, stats and flags (everything before the keys)
        k_zero_words<<<1, 256, 0, cs>>>((uint32_t *)ctrl, (int)(kCtrlKeys / 4));
        k_set_keys<<<1, 64, 0, cs>>>(pl->seed, (uint32_t *)(ctrl + kCtrlKeys));
        if (block_kernel)
            ce = launch_walk_block(a, f32, pl->shape.lanes, (int)blocks, cs);
        else
            ce = launch_walk(a, f32, (int)blocks, waves, cs);
        if (ce == hipSuccess)
            ce = scan_exclusive_u32_to_i64(pl->row_cnt, pl->row_ptr, pl->n, pl->row_ptr + pl->n, pl->scan_tmp, cs);
        PoolSet pools;
        memset(&pools, 0, sizeof(pools));
        pools.col[0] = pl->pool_col;
        pools.val[0] = pl->pool_val;
        if (ce == hipSuccess)
            ce = gather_rows(pl->n, pl->row_start, pl->row_cnt, pl->row_ptr, pools, pl->cap, pl->col, pl->val, cs);
        hipError_t ee = hipStreamEndCapture(cs, &pl->graph);
        if (ce == hipSuccess) ce = ee;
    }
    if (ce == hipSuccess) ce = hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
#undef TRYP
    if (ce != hipSuccess) {
        mcmi_plan_free(pl);
        return fail(MCMI_ERR_HIP, std::string("mcmi_plan_create: capture: ") + hipGetErrorString(ce));
    }
    *out = pl;
    return MCMI_OK;
}

extern "C" mcmi_status mcmi_plan_launch(mcmi_plan *pl, uint64_t seed, void *stream) {
    if (!pl || !pl->exec) return fail(MCMI_ERR_ARG, "mcmi_plan_launch: bad plan");
    hipStream_t s = (hipStream_t)stream;
    MCMI_HIP(hipMemcpyAsync(pl->seed, &seed, sizeof(seed), hipMemcpyHostToDevice, s));
    MCMI_HIP(hipGraphLaunch(pl->exec, s));
    return MCMI_OK;
}

extern "C" mcmi_status mcmi_plan_result(mcmi_plan *pl, mcmi_csr_out *M_view, mcmi_stats *st, int32_t *overflow,
                                        void *stream) {
    if (!pl) return fail(MCMI_ERR_ARG, "mcmi_plan_result: bad plan");
    hipStream_t s = (hipStream_t)stream;
    const unsigned char *ctrl = (const unsigned char *)pl->ctrl;
    int64_t nnz = 0;
    uint32_t flags = 0;
    unsigned long long stats[4] = {0, 0, 0, 0};
    MCMI_HIP(hipMemcpyAsync(&flags, ctrl + kCtrlFlags, sizeof(flags), hipMemcpyDeviceToHost, s));
    MCMI_HIP(hipMemcpyAsync(stats, ctrl + kCtrlStats, sizeof(stats), hipMemcpyDeviceToHost, s));
    MCMI_HIP(hipMemcpyAsync(&nnz, pl->row_ptr + pl->n, sizeof(nnz), hipMemcpyDeviceToHost, s));
    MCMI_HIP(hipStreamSynchronize(s));
    const int ovf = (flags & (kFlagPool | kFlagSpill | kFlagStage)) || nnz > pl->cap ? 1 : 0;
    if (overflow) *overflow = ovf;
    if (M_view) {
        M_view->n = pl->n;
        M_view->nnz = ovf ? 0 : nnz;
        M_view->row_ptr_dev = pl->row_ptr;
        M_view->col_dev = pl->col;
        M_view->val_dev = pl->val;
    }
    if (st) {
        memset(st, 0, sizeof(*st));
        st->transitions = stats[0];
        st->spilled = stats[1];
        st->chains = stats[2];
        st->refined = stats[3];
        st->nnz = nnz;
        st->lmax = pl->lmax;
        st->norm_inf = (float)pl->cdf->norm_inf;
        st->lanes_per_row = pl->shape.lanes;
        st->hash_slots = pl->shape.hash;
        st->sketch_slots = pl->shape.sketch;
        st->heavy_weight = pl->shape.tau;
    }
    return MCMI_OK;
}
