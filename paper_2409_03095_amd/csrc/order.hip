// Row schedule with locality (an execution order of the rows; the estimate of
// every row is the same in any order).
//
// Chains started at rows that are close in the graph of B visit overlapping sets
// of records, so the walk kernels find more of their buckets in the XCD's L2 when
// such rows run at the same time on the same XCD (each XCD takes a contiguous
// slice of the task list). The rows are grouped into cells of about `cell` rows
// by a multi-source breadth-first search on the pattern of B: the seeds are the
// rows whose hash falls below 2^32 / cell, and at each level a row without a cell
// joins the cell with the smallest seed among its neighbours that already have
// one. Rows that no seed reaches within kMaxGrow levels are cells of their own.
// The order lists the rows by (seed, row), which a stable radix sort on the seed
// gives directly.
#include <rocprim/device/device_radix_sort.hpp>

#include "common.hpp"

namespace mcmi {
namespace {

constexpr uint32_t kUnset = 0xFFFFFFFFu;
constexpr int kMaxGrow = 64;
constexpr int kGrowBatch = 16;
// lanes per row in a level (fewer lanes, more rows per wave in flight: on the
// 160^3 27-point matrix 60 us per level with 8 lanes, 44 us with 4, 50 and 52 us
// with 2 and 1)
constexpr int kGrowLanes = 4;

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    // MurmurHash3's 32-bit finaliser
    x ^= x >> 16;
    x *= 0x85EBCA6Bu;
    x ^= x >> 13;
    x *= 0xC2B2AE35u;
    x ^= x >> 16;
    return x;
}

__global__ void __launch_bounds__(256) k_seed(int64_t n, uint32_t thr, uint32_t *lab, uint32_t *changed) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (gid < kMaxGrow) changed[gid] = 0u;
    for (int64_t r = gid; r < n; r += stride) lab[r] = mix32((uint32_t)r ^ 0x6A09E667u) < thr ? (uint32_t)r : kUnset;
}

// One level of the search, G lanes per row, each lane issuing the loads of 32 / G
// of the row's columns before their labels (a row of up to 32 entries costs two
// dependent loads; past the end a lane re-reads the row's last column, which
// leaves the minimum as it is). A level runs only if the one before it labelled
// a row; when a level labels nothing, its output equals its input, so after the
// search both buffers hold the final labels (or, if all kMaxGrow levels ran, the
// buffer the last level wrote).
template <int G>
__global__ void __launch_bounds__(256) k_grow(int64_t n, const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                                              const uint32_t *__restrict__ lin, uint32_t *__restrict__ lout,
                                              uint32_t *changed, int level) {
    constexpr int U = 32 / G;
    if (level > 0 && changed[level - 1] == 0u) return;
    const int sub = threadIdx.x & (G - 1);
    const int64_t groups = ((int64_t)gridDim.x * blockDim.x) / G;
    bool any = false;
    for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G; r < n; r += groups) {
        uint32_t v = lin[r];
        if (v == kUnset) {  // uniform over the row's G lanes
            uint32_t m = kUnset;
            const int64_t b = rp[r], e = rp[r + 1];
            for (int64_t k0 = b + sub; k0 < e; k0 += 32) {
                int32_t c[U];
#pragma unroll
                for (int j = 0; j < U; ++j) c[j] = col[k0 + G * j < e ? k0 + G * j : e - 1];
#pragma unroll
                for (int j = 0; j < U; ++j) m = min(m, lin[c[j]]);
            }
#pragma unroll
            for (int off = 1; off < G; off <<= 1) m = min(m, (uint32_t)__shfl_xor((int)m, off, G));
            v = m;
            any |= m != kUnset;
        }
        if (sub == 0) lout[r] = v;
    }
    if (__any(any) && (threadIdx.x & 63) == 0 && __atomic_load_n(&changed[level], __ATOMIC_RELAXED) == 0u)
        changed[level] = 1u;
}

__global__ void __launch_bounds__(256) k_order_keys(int64_t n, uint32_t *lab, int32_t *idx) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
        const uint32_t v = lab[r];
        lab[r] = v == kUnset ? (uint32_t)r : v;
        idx[r] = (int32_t)r;
    }
}

// blocks for `lanes` threads per row, at most `cap` (grid-stride beyond)
unsigned grid_rows(int64_t n, int lanes, int64_t cap) {
    int64_t b = (n * lanes + 255) / 256;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

}  // namespace

hipError_t build_locality_order(int64_t n, const int64_t *row_ptr, const int32_t *col, int64_t cell, int32_t *order,
                                hipStream_t s) {
    uint32_t *lab0 = nullptr, *lab1 = nullptr, *changed = nullptr;
    int32_t *idx = nullptr;
    void *tmp = nullptr;
    size_t tmp_bytes = 0;
    int end_bit = 1;
    while (end_bit < 32 && ((uint64_t)(n - 1) >> end_bit) != 0) ++end_bit;
    // rocPRIM's LSD radix sort (stable) on the labels' low end_bit bits
    hipError_t e = rocprim::radix_sort_pairs(nullptr, tmp_bytes, (const uint32_t *)nullptr, (uint32_t *)nullptr,
                                             (const int32_t *)nullptr, (int32_t *)nullptr, (size_t)n, 0u,
                                             (unsigned)end_bit, s);
    if (e == hipSuccess) e = dev_alloc((void **)&lab0, (size_t)n * 4, s);
    if (e == hipSuccess) e = dev_alloc((void **)&lab1, (size_t)n * 4, s);
    if (e == hipSuccess) e = dev_alloc((void **)&idx, (size_t)n * 4, s);
    if (e == hipSuccess) e = dev_alloc((void **)&changed, kMaxGrow * 4, s);
    if (e == hipSuccess) e = dev_alloc(&tmp, tmp_bytes > 0 ? tmp_bytes : 16, s);
    if (e == hipSuccess) {
        const double p = 1.0 / (double)(cell > 1 ? cell : 1);
        const uint32_t thr = p >= 1.0 ? 0xFFFFFFFFu : (uint32_t)(p * 4294967296.0);
        k_seed<<<grid_rows(n, 1, 65536), 256, 0, s>>>(n, thr, lab0, changed);
        e = hipGetLastError();
        // levels go out kGrowBatch at a time; the search stops after a batch whose
        // last level labelled nothing (a level after the first empty one returns at
        // once, and the empty one copied the final labels into both buffers)
        for (int level = 0; e == hipSuccess && level < kMaxGrow; ++level) {
            const bool even = (level & 1) == 0;
            k_grow<kGrowLanes><<<grid_rows(n, kGrowLanes, 4096), 256, 0, s>>>(n, row_ptr, col, even ? lab0 : lab1,
                                                                           even ? lab1 : lab0, changed, level);
            e = hipGetLastError();
            if (e == hipSuccess && (level + 1) % kGrowBatch == 0 && level + 1 < kMaxGrow) {
                uint32_t last = 1u;
                e = hipMemcpyAsync(&last, changed + level, sizeof(last), hipMemcpyDeviceToHost, s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                if (e == hipSuccess && last == 0u) break;
            }
        }
    }
    // kMaxGrow and kGrowBatch are even: the last level that runs writes lab0
    if (e == hipSuccess) {
        k_order_keys<<<grid_rows(n, 1, 65536), 256, 0, s>>>(n, lab0, idx);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = rocprim::radix_sort_pairs(tmp, tmp_bytes, (const uint32_t *)lab0, lab1, (const int32_t *)idx, order,
                                      (size_t)n, 0u, (unsigned)end_bit, s);
    for (void *t : {(void *)lab0, (void *)lab1, (void *)idx, (void *)changed, tmp})
        if (t) dev_release(t, s);
    return e;
}

}  // namespace mcmi
