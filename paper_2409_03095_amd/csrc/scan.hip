// Device prefix sums, CSR assembly helpers and the SpMV y = M x (gfx950).
#include "common.hpp"

namespace mcmi {

namespace {
constexpr int kScanThreads = 256;
constexpr int kScanPer = 4;
constexpr int kScanTile = kScanThreads * kScanPer;

template <typename T>
__device__ __forceinline__ int64_t load_as_i64(const T *p, int64_t i, int64_t n) {
    return i < n ? (int64_t)p[i] : 0;
}

// block-wide exclusive scan of one int64 per thread; returns the block total
__device__ int64_t block_excl_scan(int64_t v, int64_t *out_excl) {
    __shared__ int64_t warp_tot[kScanThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t incl = wave_incl_scan(v);
    if (lane == 63) warp_tot[w] = incl;
    __syncthreads();
    int64_t base = 0, total = 0;
    for (int k = 0; k < kScanThreads / 64; ++k) {
        if (k < w) base += warp_tot[k];
        total += warp_tot[k];
    }
    __syncthreads();
    *out_excl = base + incl - v;
    return total;
}

template <typename T>
__global__ void __launch_bounds__(kScanThreads) k_tile_sums(const T *in, int64_t n, int64_t *sums) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    int64_t v = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) v += load_as_i64(in, base + k, n);
    int64_t ex;
    int64_t tot = block_excl_scan(v, &ex);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_sums(int64_t *sums, int64_t nb, int64_t *total) {
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kScanThreads) {
        const int64_t i = b0 + threadIdx.x;
        int64_t v = i < nb ? sums[i] : 0;
        int64_t ex;
        int64_t tot = block_excl_scan(v, &ex);
        if (i < nb) sums[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

template <typename T>
__global__ void __launch_bounds__(kScanThreads) k_tile_scan(const T *in, int64_t *out, int64_t n,
                                                           const int64_t *sums) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    int64_t v[kScanPer];
    int64_t tsum = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        v[k] = load_as_i64(in, base + k, n);
        tsum += v[k];
    }
    int64_t ex;
    block_excl_scan(tsum, &ex);
    int64_t run = sums[blockIdx.x] + ex;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
}

template <typename T>
hipError_t scan_impl(const T *in, int64_t *out, int64_t n, int64_t *total_dev, void *tmp, hipStream_t s) {
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    int64_t *sums = (int64_t *)tmp;
    if (nb > 0) {
        k_tile_sums<T><<<(unsigned)nb, kScanThreads, 0, s>>>(in, n, sums);
    }
    k_scan_sums<<<1, kScanThreads, 0, s>>>(sums, nb, total_dev);
    if (nb > 0) {
        k_tile_scan<T><<<(unsigned)nb, kScanThreads, 0, s>>>(in, out, n, sums);
    }
    return hipGetLastError();
}
}  // namespace

size_t scan_tmp_bytes(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile + 1) * sizeof(int64_t); }

hipError_t scan_exclusive_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *total_dev, void *tmp,
                              hipStream_t s) {
    return scan_impl<int64_t>(in, out, n, total_dev, tmp, s);
}

hipError_t scan_exclusive_u32_to_i64(const uint32_t *in, int64_t *out, int64_t n, int64_t *total_dev, void *tmp,
                                     hipStream_t s) {
    return scan_impl<uint32_t>(in, out, n, total_dev, tmp, s);
}

// ------------------------------------------------------------- assembly
// Copy each row's survivors from its pool into the CSR arrays (row_ptr is the
// exclusive scan of row_cnt, n_rows + 1 entries). A workgroup takes kGatherRows
// consecutive rows, whose output is one contiguous range: it stages the rows'
// source pointers and output starts in LDS, then its threads stride over the
// range (coalesced stores, kGatherU positions per thread in flight), each
// following which row its position falls in. row_start holds the position in the
// low 56 bits and the pool index above. Rows without a pool position (row_start <
// 0) and positions at or past `cap` are not written (captured plans report them
// as an overflow).
constexpr int kGatherRows = 256;
constexpr int kGatherU = 4;

__global__ void __launch_bounds__(256) k_gather_rows(int64_t n_rows, const int64_t *__restrict__ row_start,
                                                     const int64_t *__restrict__ row_ptr, PoolSet pools,
                                                     int64_t cap, int32_t *__restrict__ col,
                                                     double *__restrict__ val) {
    __shared__ int64_t s_ptr[kGatherRows + 1];
    __shared__ const int32_t *s_col[kGatherRows];
    __shared__ const double *s_val[kGatherRows];
    constexpr int64_t kPosMask = ((int64_t)1 << kPoolShift) - 1;
    const int t = threadIdx.x;
    const int nt = blockDim.x;
    for (int64_t r0 = (int64_t)blockIdx.x * kGatherRows; r0 < n_rows; r0 += (int64_t)gridDim.x * kGatherRows) {
        const int nr = (int)(n_rows - r0 < kGatherRows ? n_rows - r0 : kGatherRows);
        __syncthreads();  // the previous range's readers are done with the staging arrays
        for (int i = t; i <= nr; i += nt) s_ptr[i] = row_ptr[r0 + i];
        for (int i = t; i < nr; i += nt) {
            const int64_t tagged = row_start[r0 + i];
            const int32_t *pc = nullptr;
            const double *pv = nullptr;
            if (tagged >= 0) {
                const int pool = (int)(tagged >> kPoolShift);
                const int64_t src = tagged & kPosMask;
#pragma unroll
                for (int q = 0; q < kMaxPools; ++q)
                    if (pool == q) {
                        pc = pools.col[q] + src;
                        pv = pools.val[q] + src;
                    }
            }
            s_col[i] = pc;
            s_val[i] = pv;
        }
        __syncthreads();
        const int64_t d0 = s_ptr[0], d1 = s_ptr[nr];
        int i = 0;  // the row of this thread's current position (positions only grow)
        for (int64_t p0 = d0 + t; p0 < d1; p0 += (int64_t)nt * kGatherU) {
            int32_t c[kGatherU];
            double w[kGatherU];
            int64_t q[kGatherU];
#pragma unroll
            for (int u = 0; u < kGatherU; ++u) {
                const int64_t p = p0 + (int64_t)u * nt;
                q[u] = -1;
                if (p < d1) {
                    while (s_ptr[i + 1] <= p) ++i;
                    const int32_t *pc = s_col[i];
                    if (pc != nullptr && p < cap) {
                        const int64_t k = p - s_ptr[i];
                        c[u] = pc[k];
                        w[u] = s_val[i][k];
                        q[u] = p;
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < kGatherU; ++u)
                if (q[u] >= 0) {
                    col[q[u]] = c[u];
                    val[q[u]] = w[u];
                }
        }
    }
}

hipError_t gather_rows(int64_t n_rows, const int64_t *row_start, const uint32_t *row_cnt, const int64_t *row_ptr,
                       const PoolSet &pools, int64_t cap, int32_t *col, double *val, hipStream_t s) {
    (void)row_cnt;  // the counts are the differences of row_ptr
    if (n_rows <= 0) return hipSuccess;
    int64_t blocks = (n_rows + kGatherRows - 1) / kGatherRows;
    if (blocks > 65536) blocks = 65536;
    k_gather_rows<<<(unsigned)blocks, 256, 0, s>>>(n_rows, row_start, row_ptr, pools, cap, col, val);
    return hipGetLastError();
}

// Slots whose row must be rerun (row_start < 0): appended to `list`, count in
// ctr[0], their survivor counts summed in ctr[1] (pool overflows know theirs).
__global__ void __launch_bounds__(256) k_collect_failed(int64_t n_slots, const int64_t *row_start,
                                                        const uint32_t *row_cnt, int32_t *list,
                                                        unsigned long long *ctr) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_slots; i += stride) {
        if (row_start[i] < 0) {
            const unsigned long long k = atomicAdd(&ctr[0], 1ull);
            list[k] = (int32_t)i;
            atomicAdd(&ctr[1], (unsigned long long)row_cnt[i]);
        }
    }
}

hipError_t collect_failed(int64_t n_slots, const int64_t *row_start, const uint32_t *row_cnt, int32_t *list,
                          unsigned long long *ctr, hipStream_t s) {
    int64_t blocks = (n_slots + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    k_collect_failed<<<(unsigned)blocks, 256, 0, s>>>(n_slots, row_start, row_cnt, list, ctr);
    return hipGetLastError();
}

// ------------------------------------------------------------ validation
// rows[i] in [0, n) and chains_per_row[r] >= 1; sets bit 1 / bit 2 of bad[0], the
// largest chains_per_row value in bad[1] and their sum in bad[2..3] (a u64); all
// cleared by the caller. One atomic per workgroup and quantity.
__global__ void __launch_bounds__(256) k_validate(const int32_t *rows, int64_t n_rows, const int32_t *cpr,
                                                  int64_t n, uint32_t *bad) {
    __shared__ uint32_t red_max[4];
    __shared__ unsigned long long red_sum[4];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint32_t most = 0;
    unsigned long long sum = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_rows || i < n; i += stride) {
        if (rows && i < n_rows && (rows[i] < 0 || (int64_t)rows[i] >= n)) atomicOr(bad, 1u);
        if (cpr && i < n) {
            const int32_t c = cpr[i];
            if (c < 1) atomicOr(bad, 2u);
            most = c > (int32_t)most ? (uint32_t)c : most;
            sum += c > 0 ? (unsigned long long)c : 0ull;
        }
    }
    most = wave_max(most);
    sum = wave_sum(sum);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red_max[w] = most;
        red_sum[w] = sum;
    }
    __syncthreads();
    if (threadIdx.x == 0 && cpr) {
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
            most = red_max[k] > most ? red_max[k] : most;
            sum += red_sum[k];
        }
        if (most > __atomic_load_n(&bad[1], __ATOMIC_RELAXED)) atomicMax(&bad[1], most);
        if (sum) atomicAdd((unsigned long long *)(bad + 2), sum);
    }
}

hipError_t validate_rows(const int32_t *rows, int64_t n_rows, const int32_t *cpr, int64_t n, uint32_t *bad,
                         hipStream_t s) {
    const int64_t m = n_rows > n ? n_rows : n;
    int64_t blocks = (m + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    k_validate<<<(unsigned)blocks, 256, 0, s>>>(rows, n_rows, cpr, n, bad);
    return hipGetLastError();
}

// Task map of the batched launch from its row blocks: block b lists `cnt[b]`
// consecutive positions from `start[b]`, written at `pos[b]`; a position is a row,
// or, with a schedule, the row the schedule puts there.
__global__ void __launch_bounds__(64) k_expand_blocks(int64_t nblocks, const int32_t *__restrict__ start,
                                                      const int32_t *__restrict__ cnt, const int64_t *__restrict__ pos,
                                                      const int32_t *__restrict__ order, int32_t *__restrict__ out) {
    for (int64_t b = blockIdx.x; b < nblocks; b += gridDim.x)
        for (int t = threadIdx.x; t < cnt[b]; t += blockDim.x) {
            const int32_t p = start[b] + t;
            out[pos[b] + t] = order ? order[p] : p;
        }
}

hipError_t expand_blocks(int64_t nblocks, const int32_t *start, const int32_t *cnt, const int64_t *pos,
                         const int32_t *order, int32_t *out, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    const int64_t g = nblocks < 65536 ? nblocks : 65536;
    k_expand_blocks<<<(unsigned)g, 64, 0, s>>>(nblocks, start, cnt, pos, order, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ SpMV
// y = M x, float64. A group of G lanes per row (G and the loads per lane U from
// the average row length, so that G U covers a typical row in one pass), strided
// partial sums then a butterfly reduction inside the group; grid-stride over
// rows. Each lane issues the loads of its U entries before it adds them (in the
// same order as one at a time), and the next row's bounds load while the current
// row is summed, so a row costs two dependent memory latencies, not three.
template <int G, int U>
__global__ void __launch_bounds__(256) k_spmv(int64_t n, const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                              const double *__restrict__ v, const double *__restrict__ x,
                                              double *__restrict__ y) {
    const int sub = threadIdx.x & (G - 1);
    const int64_t groups = ((int64_t)gridDim.x * blockDim.x) / G;
    int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    int64_t b = 0, e = 0;
    if (row < n) {
        b = rp[row];
        e = rp[row + 1];
    }
    for (; row < n; row += groups) {
        const int64_t nrow = row + groups;
        int64_t nb = 0, ne = 0;
        if (nrow < n) {
            nb = rp[nrow];
            ne = rp[nrow + 1];
        }
        double acc = 0.0;
        for (int64_t k0 = b + sub; k0 < e; k0 += (int64_t)G * U) {
            int32_t c[U];
            double w[U], xv[U];
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int64_t k = k0 + (int64_t)j * G < e ? k0 + (int64_t)j * G : e - 1;
                c[j] = ci[k];
                w[j] = v[k];
            }
#pragma unroll
            for (int j = 0; j < U; ++j) xv[j] = x[c[j]];
#pragma unroll
            for (int j = 0; j < U; ++j)
                if (k0 + (int64_t)j * G < e) acc += w[j] * xv[j];
        }
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
        if (sub == 0) y[row] = acc;
        b = nb;
        e = ne;
    }
}

template <int G, int U>
hipError_t launch_spmv(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, const double *x, double *y,
                       hipStream_t s) {
    int64_t blocks = (n * G + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    k_spmv<G, U><<<(unsigned)blocks, 256, 0, s>>>(n, rp, ci, v, x, y);
    return hipGetLastError();
}

hipError_t spmv(int64_t n, int64_t nnz, const int64_t *rp, const int32_t *ci, const double *v, const double *x,
                double *y, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const double per_row = (double)nnz / (double)n;
    if (per_row < 12.0) return launch_spmv<8, 4>(n, rp, ci, v, x, y, s);
    if (per_row < 24.0) return launch_spmv<16, 4>(n, rp, ci, v, x, y, s);
    if (per_row < 96.0) return launch_spmv<32, 4>(n, rp, ci, v, x, y, s);
    // rows of 96-191 entries (the 160^3 27-point M: 165): 16 lanes per row with
    // twelve entries each in flight measured 2.07 vs 2.43 ms for 32 x 6
    if (per_row < 192.0) return launch_spmv<16, 12>(n, rp, ci, v, x, y, s);
    return launch_spmv<64, 4>(n, rp, ci, v, x, y, s);
}

}  // namespace mcmi
