// Host side of the C ABI: parameter checks, workspace sizing, launches and
// the grow-and-rerun policy for the output pool and the hash tables.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "common.hpp"
#include "walk_args.hpp"

namespace mcmi {

size_t walk_lds_bytes(int hash_slots, int waves);
hipError_t launch_walk(const WalkArgs &a, bool f32, int blocks, int waves, hipStream_t s);
hipError_t walk_occupancy(bool f32, int hash_slots, int waves, int *blocks_per_cu);
size_t walk_block_lds_bytes(int hash_slots, int sketch_slots);
bool walk_block_supported(int lanes, int hash_slots);
hipError_t launch_walk_block(const WalkArgs &a, bool f32, int lanes, int blocks, hipStream_t s);
hipError_t walk_block_occupancy(bool f32, int lanes, int hash_slots, int sketch_slots, int *bpc);
hipError_t gather_rows(int64_t n_rows, const int64_t *row_start, const uint32_t *row_cnt, const int64_t *row_ptr,
                       const PoolSet &pools, int64_t cap, int32_t *col, double *val, hipStream_t s);
hipError_t collect_failed(int64_t n_slots, const int64_t *row_start, const uint32_t *row_cnt, int32_t *list,
                          unsigned long long *ctr, hipStream_t s);
hipError_t validate_rows(const int32_t *rows, int64_t n_rows, const int32_t *cpr, int64_t n, uint32_t *bad,
                         hipStream_t s);
hipError_t expand_blocks(int64_t nblocks, const int32_t *start, const int32_t *cnt, const int64_t *pos,
                         const int32_t *order, int32_t *out, hipStream_t s);
hipError_t spmv(int64_t n, int64_t nnz, const int64_t *rp, const int32_t *ci, const double *v, const double *x,
                double *y, hipStream_t s);

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

mcmi_status fail(mcmi_status st, const std::string &msg) {
    set_error(msg);
    return st;
}

// L_max: max_len if given, else the smallest L with p_L < delta where p_0 = 1
// and p_j = p_{j-1} * ||Chat||_inf, one IEEE product per step.
int derive_lmax(double norm_inf, double delta, int max_len) {
    constexpr int kCap = 65536;
    if (max_len > 0) return max_len <= kCap ? max_len : (int)MCMI_ERR_ARG;
    if (!(norm_inf < 1.0)) return (int)MCMI_ERR_NOT_CONTRACTIVE;
    if (!(delta > 0.0)) return (int)MCMI_ERR_ARG;
    double prod = 1.0;
    int steps = 0;
    while (prod >= delta) {
        prod = prod * norm_inf;
        if (++steps > kCap) return (int)MCMI_ERR_ARG;
    }
    return steps;
}

int device_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        hipGetDevice(&dev);
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (cus <= 0) cus = 256;
    }
    return cus;
}


// Task order of a batched record set (longest-processing-time first): matrix k
// costs about N (L_k + 1) per row with L_k its chain-length bound; blocks of 64
// consecutive rows (of the set's schedule, if it has one) in decreasing cost are
// dealt round-robin to the eight XCD queue slices. Writes cdf->n row indices to
// `map` (device); synchronises the stream before it returns.
hipError_t batched_lpt_map(const mcmi_cdf *cdf, double delta, int lmax, int n_hint, int32_t *map, hipStream_t s) {
    {  // host tables of the order, freed at the end of this scope
        const int K = cdf->batch;
        std::vector<double> cost(K);
        for (int k = 0; k < K; ++k) {
            const double S = cdf->mat_norm[k];
            double L = (double)lmax;
            if (S > 0.0 && S < 1.0 && delta > 0.0) L = std::min(L, std::ceil(std::log(delta) / std::log(S)));
            if (S == 0.0) L = 0.0;
            cost[k] = (double)n_hint * (L + 1.0);
        }
        std::vector<int> ord(K);
        for (int k = 0; k < K; ++k) ord[k] = k;
        std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return cost[x] > cost[y]; });
        // the host orders blocks (start, count) only; the device expands them to rows
        std::vector<std::vector<std::pair<int32_t, int32_t>>> lists(8);
        int64_t blk = 0;
        for (int k : ord) {
            for (int64_t r0 = cdf->mat_base_host[k]; r0 < cdf->mat_base_host[k + 1]; r0 += 64, ++blk) {
                const int64_t r1 = std::min<int64_t>(r0 + 64, cdf->mat_base_host[k + 1]);
                lists[blk % 8].push_back({(int32_t)r0, (int32_t)(r1 - r0)});
            }
        }
        std::vector<int32_t> bstart, bcnt;
        std::vector<int64_t> bpos;
        bstart.reserve(blk);
        bcnt.reserve(blk);
        bpos.reserve(blk);
        int64_t at = 0;
        for (auto &L : lists)
            for (auto &b : L) {
                bstart.push_back(b.first);
                bcnt.push_back(b.second);
                bpos.push_back(at);
                at += b.second;
            }
        const size_t nb = bstart.size();
        void *bdesc = nullptr;
        hipError_t e = dev_alloc(&bdesc, nb * 16 + 16, s);
        if (e != hipSuccess) return e;
        int32_t *d_start = (int32_t *)bdesc, *d_cnt = d_start + nb;
        int64_t *d_pos = (int64_t *)((unsigned char *)bdesc + ((nb * 8 + 15) / 16) * 16);
        e = hipMemcpyAsync(d_start, bstart.data(), nb * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(d_cnt, bcnt.data(), nb * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(d_pos, bpos.data(), nb * 8, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = expand_blocks((int64_t)nb, d_start, d_cnt, d_pos, cdf->order, map, s);
        // the host vectors die at the end of this scope: nothing may still read them
        const hipError_t se = hipStreamSynchronize(s);
        if (e == hipSuccess) e = se;
        dev_release(bdesc, s);
        return e;
    }
}

// Kernel shape of a run: lanes per row (64 = wavefront kernel), LDS hash slots,
// count-sketch buckets and heavy threshold tau (0 = track every contribution).
// n_max: the largest chain count of a row.
mcmi_status choose_shape(const mcmi_cdf *cdf, const mcmi_params *p, int lmax, int n_max, int n_typ,
                         KernelShape &out) {
    const double m_bar = cdf->n > 0 ? (double)cdf->nnz_c / (double)cdf->n : 0.0;
    const int n_hint = p->chains >= 1 ? p->chains : 64;
    int lanes = p->lanes_per_row;
    // One row per wavefront by default. Rows of few chains can share a wavefront
    // (lanes_per_row 8, 16 or 32), but measured slower on the learned-allocation
    // workloads: the rows of a wavefront finish together, so one row with many
    // chains holds the others, and the shared table leaves fewer wavefronts per CU
    // than small one-row tables do.
    if (lanes == 0) lanes = n_hint >= 384 ? 512 : (n_hint >= 192 ? 256 : 64);
    const bool block_kernel = lanes > 64;
    int H = p->hash_slots;
    if (!H && block_kernel) H = 4096;
    if (!H && lanes == 64) {
        // one row per wavefront: a row's chains reach at most N (L + 1) columns; a
        // table of that size (128 to 1024 slots) lets more wavefronts share a CU's
        // LDS, which is what keeps enough rows in flight when rows have few chains
        const double reach = (double)std::max(n_max, 1) * ((double)std::max(lmax, 0) + 1.0);
        H = 128;
        while (H < 1024 && (double)H < reach) H *= 2;
    }
    if (!H) {
        // 64 / lanes rows per wavefront, each with a table for its typical reach; at
        // most 2048 slots (24 KB of LDS) per wavefront, so long chains mean fewer rows
        const double reach = (double)std::max(n_typ, 1) * ((double)std::max(lmax, 0) + 1.0);
        int Hg = 64;
        while (Hg < 1024 && (double)Hg < reach) Hg *= 2;
        while (lanes < 64 && Hg * (64 / lanes) > 2048) lanes *= 2;
        H = lanes == 64 ? std::max(Hg, 128) : Hg * (64 / lanes);
    }
    if (block_kernel && !walk_block_supported(lanes, H))
        return fail(MCMI_ERR_ARG, "mcmi_spai: unsupported (lanes_per_row, hash_slots) for the workgroup kernel");
    int sketch = 0;
    double tau = 0.0;
    if (block_kernel && cdf->norm_inf < 1.0 && p->heavy_weight >= 0.0) {
        if (p->heavy_weight > 0.0) {
            tau = p->heavy_weight;
        } else {
            // distinct columns reached by step j are at most min(N, m^j, n); track every
            // contribution when all steps fit in half the table, else the first J steps
            // whose bound fits in 72 % of it (on the n = 262144 random matrix: J = 7,
            // 3 rows replayed instead of 3317 at J = 5, walk about 1 % faster)
            const double S = cdf->norm_inf;
            const int steps = S > 0.0 ? std::min(lmax, (int)std::ceil(std::log(p->delta > 0 ? p->delta : 1e-300) /
                                                                        std::log(S))) : 0;
            double reach = 1.0, total = 1.0;
            int J = 0;
            bool fits = true;
            for (int jj = 1; jj <= steps; ++jj) {
                reach = std::min({reach * std::max(m_bar, 1.0), (double)n_hint, (double)cdf->n});
                total += reach;
                if (fits && total <= 0.72 * H)
                    J = jj;
                else
                    fits = false;
            }
            if (std::min(total, (double)cdf->n) > 0.5 * H) tau = std::pow(S, std::max(J, 1)) * (1.0 - 1.0 / 1048576.0);
        }
        // default sketch: the largest that still lets two workgroups share a CU's
        // LDS. With one random 64-byte block per transition, the walk is bound by
        // HBM line traffic, and two workgroups per CU keep more lines in flight than
        // one with a bigger sketch saves in replays (measured: 59.2 vs 66.2 ms).
        if (tau > 0.0)
            sketch = p->sketch_slots ? p->sketch_slots
                                     : (int)std::max<int64_t>(1024, ((int64_t)81920 - (int64_t)H * 12 - 256) / 4);
    }
    out.lanes = lanes;
    out.hash = H;
    out.sketch = sketch;
    out.tau = tau;
    // one row per wavefront with more chains than lanes: each lane keeps two of the
    // row's chains in flight (two independent bucket loads per step, same table)
    out.lane_chains = (lanes == 64 && n_typ > 64) ? 2 : 1;
    return MCMI_OK;
}

}  // namespace mcmi

using namespace mcmi;

namespace {

struct DevBuf {
    void *p = nullptr;
    hipStream_t s = nullptr;
    ~DevBuf() {
        if (p) dev_release(p, s);
    }
    hipError_t alloc(size_t bytes, hipStream_t st) {
        if (p) dev_release(p, s);
        p = nullptr;
        s = st;
        return dev_alloc(&p, bytes ? bytes : 16, st);
    }
    template <typename T>
    T *as() const {
        return (T *)p;
    }
};

int pow2_at_least(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

}  // namespace

namespace mcmi {

// Checks of a walk's parameters, shared by mcmi_spai and mcmi_plan_create.
mcmi_status check_walk_params(const mcmi_params *p, bool per_row_chains, const char *who) {
    auto bad = [who](const char *m) { return fail(MCMI_ERR_ARG, std::string(who) + ": " + m); };
    if (p->chains < 1 && !per_row_chains) return bad("chains must be >= 1");
    if (p->walk_prec != MCMI_WALK_F64 && p->walk_prec != MCMI_WALK_F32) return bad("walk_prec must be 64 or 32");
    if (!(p->eps >= 0.0) || !(p->delta >= 0.0)) return bad("eps and delta must be >= 0");
    if (p->filter != MCMI_FILTER_N && p->filter != MCMI_FILTER_M) return bad("bad filter");
    if (p->topk < 0) return bad("topk < 0");
    if (p->pool_per_row < 0) return bad("pool_per_row must be >= 0");
    if (p->spill_slots && (p->spill_slots < 16 || (p->spill_slots & (p->spill_slots - 1))))
        return bad("spill_slots must be a power of two >= 16");
    if (p->hash_slots && (p->hash_slots < 64 || p->hash_slots > 8192 || (p->hash_slots & (p->hash_slots - 1))))
        return bad("hash_slots must be a power of two in [64, 8192]");
    if (p->sketch_slots && (p->sketch_slots < 64 || p->sketch_slots > 16384))
        return bad("sketch_slots must be in [64, 16384]");
    if (p->lanes_per_row && p->lanes_per_row != 8 && p->lanes_per_row != 16 && p->lanes_per_row != 32 &&
        p->lanes_per_row != 64 && p->lanes_per_row != 256 && p->lanes_per_row != 512 && p->lanes_per_row != 1024)
        return bad("lanes_per_row must be 0, 8, 16, 32, 64, 256, 512 or 1024");
    if (!(p->heavy_weight <= 1.0)) return bad("heavy_weight must be <= 1");
    return MCMI_OK;
}

// Largest and mean chain count of a row, with the row list and the per-row
// counts checked on the device (one synchronisation when either is given).
mcmi_status read_chain_counts(const mcmi_cdf *cdf, const mcmi_params *p, const int32_t *rows_dev, int64_t n_rows,
                              const int32_t *cpr_dev, int &n_max, int &n_typ, hipStream_t s, const char *who) {
    n_max = p->chains;
    n_typ = p->chains;
    if (!rows_dev && !cpr_dev) return MCMI_OK;
    uint32_t hv[4] = {0, 0, 0, 0};
    DevBuf vb;
    MCMI_HIP(vb.alloc(sizeof(hv), s));
    MCMI_HIP(hipMemsetAsync(vb.p, 0, sizeof(hv), s));
    MCMI_HIP(validate_rows(rows_dev, rows_dev ? n_rows : 0, cpr_dev, cdf->n, vb.as<uint32_t>(), s));
    MCMI_HIP(hipMemcpyAsync(hv, vb.p, sizeof(hv), hipMemcpyDeviceToHost, s));
    MCMI_HIP(hipStreamSynchronize(s));
    if (hv[0] & 1u) return fail(MCMI_ERR_ARG, std::string(who) + ": a row index is outside [0, n)");
    if (hv[0] & 2u) return fail(MCMI_ERR_ARG, std::string(who) + ": chains_per_row holds a value < 1");
    if (cpr_dev) {
        unsigned long long sum = 0;
        ::memcpy(&sum, hv + 2, sizeof(sum));
        n_max = (int)std::min<uint32_t>(hv[1], 1u << 30);
        n_typ = (int)std::min<unsigned long long>((sum + (unsigned long long)cdf->n - 1) / (unsigned long long)cdf->n,
                                                   1ull << 30);
    }
    return MCMI_OK;
}

// Rows per wavefront and HBM overflow slots per region of a launch. Unless
// given, the wavefront kernel's overflow table has room for every column a
// row's chains can reach, N_max (L + 1), shared out among the rows of a
// wavefront (a row with many more chains than its neighbours would otherwise
// overflow and be rerun); rows stop sharing a wavefront when given tables are
// too small to share out.
WaveLayout wave_layout(const KernelShape &shape, int spill_given, int n_max, int lmax) {
    WaveLayout w;
    w.lanes = shape.lanes;
    const bool block_kernel = w.lanes > 64;
    w.rows_per_wave = block_kernel ? 1 : 64 / w.lanes;
    w.spill_slots = spill_given;
    if (!w.spill_slots) {
        const double reach = (double)std::max(n_max, 1) * ((double)std::max(lmax, 0) + 1.0);
        if (block_kernel) {
            w.spill_slots = 16384;
        } else if (w.rows_per_wave == 1) {
            w.spill_slots = 4096;
            while (w.spill_slots < 32768 && (double)w.spill_slots < reach) w.spill_slots *= 2;
        } else {
            int sg = 1024;
            while (sg < 32768 / w.rows_per_wave && (double)sg < reach) sg *= 2;
            w.spill_slots = sg * w.rows_per_wave;
        }
    }
    while (!block_kernel && w.rows_per_wave > 1 &&
           (w.spill_slots / w.rows_per_wave < 16 || shape.hash / w.rows_per_wave < 64)) {
        w.lanes *= 2;
        w.rows_per_wave /= 2;
    }
    return w;
}

}  // namespace mcmi

extern "C" mcmi_status mcmi_spai(const mcmi_cdf *cdf, const mcmi_params *p, const int32_t *chains_per_row_dev,
                                 const int32_t *rows_dev, int64_t n_rows, mcmi_csr_out *M, mcmi_stats *st,
                                 void *stream) {
    if (M) memset(M, 0, sizeof(*M));
    if (st) memset(st, 0, sizeof(*st));
    if (!cdf || !p || !M) return fail(MCMI_ERR_ARG, "mcmi_spai: null argument");
    {
        const mcmi_status cst = check_walk_params(p, chains_per_row_dev != nullptr, "mcmi_spai");
        if (cst != MCMI_OK) return cst;
    }
    const int64_t n_tasks = rows_dev ? n_rows : cdf->n;
    if (rows_dev && (n_rows < 1 || n_rows > cdf->n)) return fail(MCMI_ERR_ARG, "mcmi_spai: bad n_rows");
    const int lmax = derive_lmax(cdf->norm_inf, p->delta, p->max_len);
    if (lmax < 0) {
        if (lmax == (int)MCMI_ERR_NOT_CONTRACTIVE)
            return fail(MCMI_ERR_NOT_CONTRACTIVE, "mcmi_spai: ||Chat||_inf >= 1; give max_len");
        return fail(MCMI_ERR_ARG, "mcmi_spai: bad delta / max_len");
    }
    hipStream_t s = (hipStream_t)stream;
    const bool f32 = p->walk_prec == MCMI_WALK_F32;

    hipEvent_t ev0, ev1, ev2;
    MCMI_HIP(hipEventCreate(&ev0));
    MCMI_HIP(hipEventCreate(&ev1));
    MCMI_HIP(hipEventCreate(&ev2));
    struct EvGuard {
        hipEvent_t a, b, c;
        ~EvGuard() {
            hipEventDestroy(a);
            hipEventDestroy(b);
            hipEventDestroy(c);
        }
    } evg{ev0, ev1, ev2};

    // ---- row list and chain counts (one synchronisation), then the kernel shape
    int n_max = p->chains, n_typ = p->chains;  // largest and mean chains of a row
    {
        const mcmi_status rst = read_chain_counts(cdf, p, rows_dev, n_rows, chains_per_row_dev, n_max, n_typ, s,
                                                  "mcmi_spai");
        if (rst != MCMI_OK) return rst;
    }
    const int cus = device_cus();
    const int n_hint = p->chains >= 1 ? p->chains : 64;
    KernelShape shape;
    {
        const mcmi_status sst = choose_shape(cdf, p, lmax, n_max, n_typ, shape);
        if (sst != MCMI_OK) return sst;
    }
    const bool block_kernel = shape.lanes > 64;
    // FP32 walks read the compact records only
    if (!f32) MCMI_HIP(ensure_full_records(cdf, s));
    int H = shape.hash;
    const int sketch = shape.sketch;
    const double tau = shape.tau;
    int waves = 4;
    const WaveLayout layout = wave_layout(shape, p->spill_slots, n_max, lmax);
    int lanes = layout.lanes;
    int rows_per_wave = layout.rows_per_wave;
    int spill_slots = layout.spill_slots;
    // first guess of the output size; rows that do not fit are rerun into a new pool
    // a quarter of the row table per row: rows that overflow the first pool are
    // walked again, so a generous first guess (HBM is large) is the cheap side
    const int h_row = H / rows_per_wave;
    int64_t per_row = p->pool_per_row ? p->pool_per_row : std::max(h_row / 4, std::min(h_row, 256));
    if (!p->pool_per_row && p->topk > 0) per_row = std::min<int64_t>(per_row, p->topk);  // exact bound
    int64_t pool_cap = n_tasks * per_row;
    pool_cap = std::min<int64_t>(pool_cap, (int64_t)1 << 31);
    if (!p->pool_per_row) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && free_b > 0)
            pool_cap = std::min<int64_t>(pool_cap, (int64_t)(free_b / 4 / 12));  // at most a quarter of free HBM
        pool_cap = std::max<int64_t>(pool_cap, 1 << 16);
    }
    pool_cap = std::max<int64_t>(pool_cap, 1);
    uint64_t retries = 0;

    DevBuf row_start, row_cnt, sk, sv, su, ctrl, row_ptr, scan_tmp, failed;
    DevBuf pool_col[kMaxPools], pool_val[kMaxPools];
    // the control block (kCtrl* offsets): queue counters, pool position, stats, flags, collect
    const size_t ctrl_bytes = kCtrlBytes;
    MCMI_HIP(ctrl.alloc(ctrl_bytes, s));
    MCMI_HIP(row_start.alloc(n_tasks * sizeof(int64_t), s));
    MCMI_HIP(row_cnt.alloc(n_tasks * sizeof(uint32_t), s));
    MCMI_HIP(row_ptr.alloc((n_tasks + 1) * sizeof(int64_t), s));
    MCMI_HIP(scan_tmp.alloc(scan_tmp_bytes(n_tasks), s));
    uint32_t *qctr = ctrl.as<uint32_t>();
    unsigned long long *pool_used = (unsigned long long *)(ctrl.as<unsigned char>() + kCtrlPool);
    unsigned long long *stats = (unsigned long long *)(ctrl.as<unsigned char>() + kCtrlStats);
    uint32_t *flags = (uint32_t *)(ctrl.as<unsigned char>() + kCtrlFlags);
    unsigned long long *collect = (unsigned long long *)(ctrl.as<unsigned char>() + kCtrlCollect);


    // batched record sets: longest-processing-time order (batched_lpt_map)
    DevBuf lpt;
    const int32_t *task_map = nullptr;
    if (cdf->batch > 0 && !rows_dev) {
        MCMI_HIP(lpt.alloc((size_t)n_tasks * sizeof(int32_t), s));
        MCMI_HIP(batched_lpt_map(cdf, p->delta, lmax, n_hint, lpt.as<int32_t>(), s));
        task_map = lpt.as<int32_t>();
    } else if (cdf->batch == 0 && !rows_dev && cdf->order) {
        task_map = cdf->order;  // locality schedule of the record set
    }

    int64_t nnz = 0;
    unsigned long long tot_stats[4] = {0, 0, 0, 0};
    float ms_walk = 0.f;
    PoolSet pools;
    memset(&pools, 0, sizeof(pools));
    int64_t pass_tasks = n_tasks;
    MCMI_HIP(hipEventRecord(ev0, s));
    for (int pass = 0;; ++pass) {
        if (pass >= kMaxPools) return fail(MCMI_ERR_CAPACITY, "mcmi_spai: rows still overflow after regrowing tables");
        int bpc = 0;
        int64_t blocks = 0, regions = 0;
        if (block_kernel) {
            MCMI_HIP(walk_block_occupancy(f32, lanes, H, sketch, &bpc));
            if (bpc < 1) return fail(MCMI_ERR_CAPACITY, "mcmi_spai: workgroup kernel does not fit in LDS");
            blocks = std::min<int64_t>((int64_t)bpc * cus, pass_tasks);
            regions = blocks;
        } else {
            MCMI_HIP(walk_occupancy(f32, H, waves, &bpc));
            while (bpc < 1 && waves > 1) {
                waves >>= 1;
                MCMI_HIP(walk_occupancy(f32, H, waves, &bpc));
            }
            if (bpc < 1) return fail(MCMI_ERR_CAPACITY, "mcmi_spai: hash table does not fit in LDS");
            blocks = (int64_t)bpc * cus;
            if (blocks * waves > pass_tasks) blocks = std::max<int64_t>(1, (pass_tasks + waves - 1) / waves);
            regions = blocks * waves;
        }
        MCMI_HIP(pool_col[pass].alloc((size_t)pool_cap * sizeof(int32_t), s));
        MCMI_HIP(pool_val[pass].alloc((size_t)pool_cap * sizeof(double), s));
        pools.col[pass] = pool_col[pass].as<int32_t>();
        pools.val[pass] = pool_val[pass].as<double>();
        MCMI_HIP(sk.alloc((size_t)regions * spill_slots * sizeof(int32_t), s));
        MCMI_HIP(sv.alloc((size_t)regions * spill_slots * sizeof(double), s));
        MCMI_HIP(su.alloc((size_t)regions * spill_slots * sizeof(int32_t), s));
        MCMI_HIP(hipMemsetAsync(sk.p, 0xFF, (size_t)regions * spill_slots * sizeof(int32_t), s));
        MCMI_HIP(hipMemsetAsync(sv.p, 0, (size_t)regions * spill_slots * sizeof(double), s));
        MCMI_HIP(hipMemsetAsync(ctrl.p, 0, ctrl_bytes, s));

        WalkArgs a;
        memset(&a, 0, sizeof(a));
        a.rec = cdf->rec;
        a.rec32 = cdf->rec32;
        a.roff = cdf->roff;
        a.diag = cdf->diag;
        a.rows = rows_dev;
        a.n_tasks = pass_tasks;
        a.task_map = task_map;
        a.pool_tag = (int64_t)pass << kPoolShift;
        a.row_mat = cdf->batch > 0 ? cdf->row_mat : nullptr;
        a.mat_base = cdf->batch > 0 ? cdf->mat_base : nullptr;
        a.chains_per_row = chains_per_row_dev;
        a.chains = p->chains;
        a.key0 = (uint32_t)(p->seed & 0xffffffffu);
        a.key1 = (uint32_t)(p->seed >> 32);
        a.tag = p->stream_tag;
        a.delta = p->delta;
        a.delta32 = (float)p->delta;
        a.eps = p->eps;
        a.lmax = lmax;
        a.filter_m = p->filter == MCMI_FILTER_M;
        a.topk = p->topk;
        a.hash_slots = H;
        a.hash_shift = 32 - __builtin_ctz((unsigned)H);
        a.row_lanes = block_kernel ? 0 : lanes;
        a.lane_chains = (!block_kernel && lanes == 64) ? shape.lane_chains : 1;
        a.queue_ctr = qctr;
        a.row_start = row_start.as<int64_t>();
        a.row_cnt = row_cnt.as<uint32_t>();
        a.pool_col = pool_col[pass].as<int32_t>();
        a.pool_val = pool_val[pass].as<double>();
        a.pool_cap = pool_cap;
        a.pool_used = pool_used;
        // reruns size their pool exactly and reserve per row
        a.pool_chunk = (pass == 0 && !block_kernel) ? pool_chunk_for(pool_cap, regions) : 0;
        a.spill_keys = sk.as<int32_t>();
        a.spill_vals = sv.as<double>();
        a.spill_used = su.as<int32_t>();
        a.spill_slots = spill_slots;
        a.stats = stats;
        a.flags = flags;
        a.tau = tau;
        a.tau32 = (float)tau;
        a.sketch_slots = sketch;
        if (pass == 0) MCMI_HIP(hipEventRecord(ev1, s));
        if (block_kernel)
            MCMI_HIP(launch_walk_block(a, f32, lanes, (int)blocks, s));
        else
            MCMI_HIP(launch_walk(a, f32, (int)blocks, waves, s));
        MCMI_HIP(hipEventRecord(ev2, s));
        uint32_t hflags = 0;
        unsigned long long hstats[4] = {0, 0, 0, 0};
        MCMI_HIP(hipMemcpyAsync(&hflags, flags, sizeof(hflags), hipMemcpyDeviceToHost, s));
        MCMI_HIP(hipMemcpyAsync(hstats, stats, sizeof(hstats), hipMemcpyDeviceToHost, s));
        MCMI_HIP(hipStreamSynchronize(s));
        for (int k = 0; k < 4; ++k) tot_stats[k] += hstats[k];
        if (!(hflags & (kFlagPool | kFlagSpill | kFlagStage))) break;
        // rerun only the rows that overflowed, with the overflowing tables grown
        ++retries;
        if (!failed.p) MCMI_HIP(failed.alloc((size_t)n_tasks * sizeof(int32_t), s));
        unsigned long long hcol[2] = {0, 0};
        MCMI_HIP(collect_failed(n_tasks, row_start.as<int64_t>(), row_cnt.as<uint32_t>(), failed.as<int32_t>(),
                                collect, s));
        MCMI_HIP(hipMemcpyAsync(hcol, collect, sizeof(hcol), hipMemcpyDeviceToHost, s));
        MCMI_HIP(hipStreamSynchronize(s));
        // the failed list is read by the next pass while `collect` is cleared with ctrl
        DevBuf next_map;
        MCMI_HIP(next_map.alloc((size_t)std::max<unsigned long long>(hcol[0], 1) * sizeof(int32_t), s));
        MCMI_HIP(hipMemcpyAsync(next_map.p, failed.p, (size_t)hcol[0] * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        std::swap(failed.p, next_map.p);
        task_map = failed.as<int32_t>();
        pass_tasks = (int64_t)hcol[0];
        pool_cap = std::max<int64_t>((int64_t)(hcol[1] + hcol[1] / 4) + 1024, pass_tasks * 64);
        if (hflags & kFlagSpill) spill_slots *= 4;
        if (hflags & kFlagStage) {
            if (block_kernel) {
                if (!walk_block_supported(lanes, H * 2))
                    return fail(MCMI_ERR_CAPACITY, "mcmi_spai: more survivors per row than the workgroup table holds");
                H *= 2;
            } else if (rows_per_wave > 1) {
                // the rerun gives each row a wavefront and twice its table
                H = 2 * (H / rows_per_wave);
                lanes = 64;
                rows_per_wave = 1;
            } else {
                if (H >= 8192) return fail(MCMI_ERR_CAPACITY, "mcmi_spai: more survivors per row than 8192 slots");
                H *= 2;
            }
        }
    }
    MCMI_HIP(hipEventElapsedTime(&ms_walk, ev1, ev2));
    MCMI_HIP(scan_exclusive_u32_to_i64(row_cnt.as<uint32_t>(), row_ptr.as<int64_t>(), n_tasks,
                                       row_ptr.as<int64_t>() + n_tasks, scan_tmp.p, s));
    MCMI_HIP(hipMemcpyAsync(&nnz, row_ptr.as<int64_t>() + n_tasks, sizeof(nnz), hipMemcpyDeviceToHost, s));
    MCMI_HIP(hipStreamSynchronize(s));
    unsigned long long *hstats = tot_stats;

    // ---- CSR assembly
    hipEvent_t ev3;
    MCMI_HIP(hipEventCreate(&ev3));
    int32_t *col = nullptr;
    double *val = nullptr;
    int64_t *rp = nullptr;
    hipError_t e1 = dev_alloc((void **)&col, (size_t)std::max<int64_t>(nnz, 1) * sizeof(int32_t), s);
    hipError_t e2 = dev_alloc((void **)&val, (size_t)std::max<int64_t>(nnz, 1) * sizeof(double), s);
    hipError_t e3 = dev_alloc((void **)&rp, (size_t)(n_tasks + 1) * sizeof(int64_t), s);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
        dev_release(col, s);
        dev_release(val, s);
        dev_release(rp, s);
        hipEventDestroy(ev3);
        return fail(MCMI_ERR_NOMEM, "mcmi_spai: cannot allocate M");
    }
    hipError_t ge = hipMemcpyAsync(rp, row_ptr.p, (size_t)(n_tasks + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, s);
    if (ge == hipSuccess)
        ge = gather_rows(n_tasks, row_start.as<int64_t>(), row_cnt.as<uint32_t>(), rp, pools, nnz, col, val, s);
    if (ge == hipSuccess) ge = hipEventRecord(ev3, s);
    if (ge == hipSuccess) ge = hipEventSynchronize(ev3);
    if (ge != hipSuccess) {
        dev_release(col, s);
        dev_release(val, s);
        dev_release(rp, s);
        hipEventDestroy(ev3);
        return fail(MCMI_ERR_HIP, std::string("mcmi_spai: assembly: ") + hipGetErrorString(ge));
    }
    M->n = n_tasks;
    M->nnz = nnz;
    M->row_ptr_dev = rp;
    M->col_dev = col;
    M->val_dev = val;
    if (st) {
        float ms_tot = 0.f, ms_asm = 0.f;
        hipEventElapsedTime(&ms_tot, ev0, ev3);
        hipEventElapsedTime(&ms_asm, ev2, ev3);
        st->transitions = hstats[0];
        st->spilled = hstats[1];
        st->chains = hstats[2];
        st->retries = retries;
        st->refined = hstats[3];
        st->lanes_per_row = lanes;
        st->hash_slots = H;
        st->sketch_slots = sketch;
        st->heavy_weight = tau;
        st->nnz = nnz;
        st->lmax = lmax;
        st->norm_inf = (float)cdf->norm_inf;
        st->ms_walk = ms_walk;
        st->ms_assemble = ms_asm;
        st->ms_total = ms_tot;
    }
    hipEventDestroy(ev3);
    return MCMI_OK;
}

extern "C" mcmi_status mcmi_apply(const mcmi_csr_out *M, int64_t n_cols, const double *x_dev, double *y_dev,
                                  void *stream) {
    if (!M || !x_dev || !y_dev || n_cols < 1) return fail(MCMI_ERR_ARG, "mcmi_apply: bad argument");
    if (M->n < 0 || (M->n > 0 && !M->row_ptr_dev)) return fail(MCMI_ERR_ARG, "mcmi_apply: bad M");
    MCMI_HIP(spmv(M->n, M->nnz, M->row_ptr_dev, M->col_dev, M->val_dev, x_dev, y_dev, (hipStream_t)stream));
    return MCMI_OK;
}

extern "C" mcmi_status mcmi_csr_copy(const mcmi_csr_out *M, int64_t *row_ptr_dev, int32_t *col_dev,
                                     double *val_dev, void *stream) {
    if (!M || !row_ptr_dev || (M->nnz > 0 && (!col_dev || !val_dev))) return fail(MCMI_ERR_ARG, "mcmi_csr_copy: bad argument");
    hipStream_t s = (hipStream_t)stream;
    MCMI_HIP(hipMemcpyAsync(row_ptr_dev, M->row_ptr_dev, (size_t)(M->n + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    if (M->nnz > 0) {
        MCMI_HIP(hipMemcpyAsync(col_dev, M->col_dev, (size_t)M->nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        MCMI_HIP(hipMemcpyAsync(val_dev, M->val_dev, (size_t)M->nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    return MCMI_OK;
}

extern "C" void mcmi_csr_free(mcmi_csr_out *M) {
    if (!M) return;
    dev_release_idle(M->row_ptr_dev);
    dev_release_idle(M->col_dev);
    dev_release_idle(M->val_dev);
    memset(M, 0, sizeof(*M));
}

extern "C" const char *mcmi_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *mcmi_version(void) { return "mcmi 0.1 gfx950"; }
