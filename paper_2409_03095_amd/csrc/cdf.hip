// Row records of C = I - D^-1 B and their integer CDFs (gfx950).
//
// Section IV, phase 2 forms the iteration matrix; the transition matrix P of
// Section IV-A is, here, p_ij proportional to |c_ij|, quantized per row:
//   a_k = |c_k|, a_max = max_k a_k, Q = 31 - ceil(log2 m),
//   w_k = max(1, floor(2^Q a_k / a_max)), cum_k = w_1 + ... + w_k (exact uint32),
//   W = cum_m, Shat = (a_max * W) * 2^-Q (one rounding).
// The integer scan is order-free, so a wavefront prefix scan gives exactly the
// sequential sums. Each row's alias table (the sampler of a step) is then built
// from the weights by Vose's exact-integer construction.
#include <string.h>

#include "common.hpp"

namespace mcmi {

namespace {

__device__ __forceinline__ int ceil_log2_u32(uint32_t m) {
    int q = 0;
    while ((1u << q) < m) ++q;  // m < 2^31 here
    return q;
}

// An off-diagonal quotient c is an entry of C when it is nonzero and, with a
// reduction cut, |c| is not below the cut (compared as the bits of |c|, which
// order non-negative doubles like their values).
__device__ __forceinline__ bool keep_c(double c, const unsigned long long *cut) {
    return c != 0.0 && (!cut || (unsigned long long)__double_as_longlong(fabs(c)) >= *cut);
}

// Groups of G lanes (G divides 64), each owning one row at a time: reductions,
// scans and broadcasts stay inside the group; a ballot is the wave's ballot
// masked to the group's lanes (so mask_rank counts the group's lanes below).
template <int G>
struct Group {
    int sub;        // lane inside the group
    uint64_t mask;  // the group's lanes in a wave ballot
    __device__ __forceinline__ Group() {
        const int lane = threadIdx.x & 63;
        sub = lane & (G - 1);
        mask = G == 64 ? ~0ull : (((1ull << (G & 63)) - 1ull) << (lane & ~(G - 1)));
    }
    __device__ __forceinline__ uint64_t ballot(bool p) const { return __ballot(p) & mask; }
    template <typename T>
    __device__ __forceinline__ T sum(T v) const {
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
        return v;
    }
    template <typename T>
    __device__ __forceinline__ T max(T v) const {
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) {
            T o = __shfl_xor(v, off, G);
            v = o > v ? o : v;
        }
        return v;
    }
    template <typename T>
    __device__ __forceinline__ T incl_scan(T v) const {
#pragma unroll
        for (int off = 1; off < G; off <<= 1) {
            T o = __shfl_up(v, off, G);
            if (sub >= off) v += o;
        }
        return v;
    }
    template <typename T>
    __device__ __forceinline__ T bcast(T v, int src) const { return __shfl(v, src, G); }
    // lane (inside the group) of the lowest set bit of a group ballot
    __device__ __forceinline__ int first(uint64_t b) const { return (__builtin_ctzll(b)) & (G - 1); }
};

// Maximum of non-negative doubles kept as their bits (which order like the
// values). The atomic is skipped when the stored value is already as large:
// with one call per wave, tens of thousands of atomics on one address would
// otherwise serialise at its L2 channel.
__device__ __forceinline__ void atomic_max_bits(unsigned long long *bits, double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    if (__atomic_load_n(bits, __ATOMIC_RELAXED) < b) atomicMax(bits, b);
}

// ||B||_inf for the augmented splitting: each thread sums one row's |b_ij| in
// column order (one IEEE add at a time, so the sums are those of a sequential
// loop), the maximum is an integer max on the bits of the non-negative sums.
__global__ void __launch_bounds__(256) k_row_abs_max(int64_t n, const int64_t *__restrict__ rp,
                                                     const double *__restrict__ v, unsigned long long *bits) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    double best = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
        double sum = 0.0;
        for (int64_t k = rp[r]; k < rp[r + 1]; ++k) sum += fabs(v[k]);
        best = sum > best ? sum : best;
    }
    best = wave_max(best);
    if ((threadIdx.x & 63) == 0) atomic_max_bits(bits, best);
}

// Reduction keys: the bits of |c| for every entry of C, all ones for the rest
// (diagonal, zero quotients), in B's entry order.
__global__ void __launch_bounds__(256) k_cut_keys(int64_t n, const int64_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                  const double *__restrict__ diag, unsigned long long *__restrict__ keys) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t r = wave; r < n; r += nwaves) {
        const double d = diag[r];
        for (int64_t k = rp[r] + lane; k < rp[r + 1]; k += 64) {
            const double c = (int64_t)ci[k] != r ? (-v[k]) / d : 0.0;
            keys[k] = c != 0.0 ? (unsigned long long)__double_as_longlong(fabs(c)) : ~0ull;
        }
    }
}

// Radix selection of the key of rank sel[1] (0-based), 8 bits per pass from the
// top: sel[0] holds the bits fixed so far. Each pass histograms the next digit of
// the keys that match them (LDS histogram per workgroup), then one thread fixes
// the digit and the rank inside it.
__global__ void __launch_bounds__(256) k_radix_hist(const unsigned long long *__restrict__ keys, int64_t nk,
                                                    int shift, const unsigned long long *__restrict__ sel,
                                                    unsigned long long *__restrict__ hist) {
    __shared__ unsigned int h[256];
    for (int i = threadIdx.x; i < 256; i += blockDim.x) h[i] = 0u;
    __syncthreads();
    const unsigned long long prefix = sel[0];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nk; i += stride) {
        const unsigned long long key = keys[i];
        if (shift == 56 || (key >> (shift + 8)) == (prefix >> (shift + 8)))
            atomicAdd(&h[(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 256; i += blockDim.x)
        if (h[i]) atomicAdd(&hist[i], (unsigned long long)h[i]);
}

__global__ void k_radix_pick(unsigned long long *sel, unsigned long long *hist, int shift) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const unsigned long long rank = sel[1];
    unsigned long long below = 0;
    for (int dgt = 0; dgt < 256; ++dgt) {
        const unsigned long long c = hist[dgt];
        if (rank < below + c) {
            sel[0] |= (unsigned long long)dgt << shift;
            sel[1] = rank - below;
            break;
        }
        below += c;
    }
    for (int dgt = 0; dgt < 256; ++dgt) hist[dgt] = 0ull;
}

// Validate row r of B, find its diagonal and count its nonzero off-diagonals.
template <int G>
__global__ void __launch_bounds__(256) k_count(int64_t n, int64_t nnz, const int64_t *__restrict__ rp,
                                               const int32_t *__restrict__ ci, const double *__restrict__ v,
                                               double aug, const unsigned long long *__restrict__ cut,
                                               uint32_t *__restrict__ mrow, uint32_t *__restrict__ units,
                                               double *__restrict__ diag, uint32_t *__restrict__ flags) {
    const Group<G> g;
    const int sub = g.sub;
    const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int64_t ngrp = ((int64_t)gridDim.x * blockDim.x) / G;
    if (grp == 0 && sub == 0 && (rp[0] != 0 || rp[n] != nnz)) atomicOr(flags, kFlagCsr);
    for (int64_t r = grp; r < n; r += ngrp) {
        const int64_t b = rp[r], e = rp[r + 1];
        if (b < 0 || e < b || e > nnz) {
            if (sub == 0) {
                atomicOr(flags, kFlagCsr);
                mrow[r] = 0;
                units[r] = record_units(0);
                diag[r] = 0.0;
            }
            continue;
        }
        bool bad = false, found = false;
        double dv = 0.0;
        for (int64_t k = b + sub; k < e; k += G) {
            const int32_t c = ci[k];
            bad |= (c < 0) || ((int64_t)c >= n) || (k > b && ci[k - 1] >= c);
            if ((int64_t)c == r) {
                found = true;
                dv = v[k];
            }
        }
        const uint64_t fb = g.ballot(found);
        const uint64_t bb = g.ballot(bad);
        double d = g.bcast(dv, fb ? g.first(fb) : 0);
        if (!fb) d = 0.0;
        if (aug > 0.0) d = d + (d < 0.0 ? -aug : aug);  // augmented splitting (a missing diagonal is 0)
        // entries of C: off-diagonals whose quotient (-b_ij) / b_ii is nonzero
        // and not below the reduction cut
        uint32_t cnt = 0;
        if (d != 0.0)
            for (int64_t k = b + sub; k < e; k += G)
                if ((int64_t)ci[k] != r && keep_c((-v[k]) / d, cut)) ++cnt;
        cnt = g.sum(cnt);
        if (sub == 0) {
            if (bb) atomicOr(flags, kFlagCsr);
            if (d == 0.0) atomicOr(flags, kFlagZeroDiag);
            mrow[r] = cnt;
            units[r] = record_units(cnt);
            diag[r] = d;
        }
    }
}

// Write each row's header and its sorted {cum, target row} nodes into `sorted`
// (C-row order, at cptr[r]; the target's sign bit set for a negative c), the
// row's record offset as 32 bits, and {offset, m, Shat32} into the dense per-row
// table `tinfo` (what a bucket copies of its targets).
template <int G>
__global__ void __launch_bounds__(256) k_fill(int64_t n, const int64_t *__restrict__ rp,
                                              const int32_t *__restrict__ ci, const double *__restrict__ v,
                                              const double *__restrict__ diag, const uint32_t *__restrict__ mrow,
                                              const int64_t *__restrict__ roff64, const int64_t *__restrict__ cptr,
                                              const unsigned long long *__restrict__ cut,
                                              uint32_t *__restrict__ roff32, uint32_t *__restrict__ rec32,
                                              uint2 *__restrict__ sorted, uint4 *__restrict__ tinfo,
                                              unsigned long long *__restrict__ norm_bits) {
    const Group<G> g;
    const int sub = g.sub;
    const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int64_t ngrp = ((int64_t)gridDim.x * blockDim.x) / G;
    double best = 0.0;  // the wave's largest Shat (one atomic per wave, not per row)
    for (int64_t r = grp; r < n; r += ngrp) {
        const int64_t b = rp[r], e = rp[r + 1];
        const uint32_t m = mrow[r];
        const double d = diag[r];
        const uint32_t off = (uint32_t)roff64[r];
        uint32_t *hdc = rec32 + (size_t)off * kUnitWords32;
        if (sub == 0) roff32[r] = off;
        if (m == 0) {
            if (sub == 0) {
                tinfo[r] = make_uint4(off, 0u, __float_as_uint(0.0f), 0u);
                *(uint4 *)hdc = make_uint4((uint32_t)r, 0u, 0u, __float_as_uint(0.0f));
                *(double2 *)(hdc + 4) = make_double2(0.0, d);
            }
            continue;
        }
        // a_max over the row's entries of C (order-free)
        double amax = 0.0;
        for (int64_t k = b + sub; k < e; k += G) {
            const int32_t c = ci[k];
            if ((int64_t)c != r) {
                const double cv = (-v[k]) / d;
                const double a = keep_c(cv, cut) ? fabs(cv) : 0.0;
                amax = a > amax ? a : amax;
            }
        }
        amax = g.max(amax);
        const int q = 31 - ceil_log2_u32(m);
        // quantize and scan in column order, G entries at a time
        uint32_t carry = 0, placed = 0;
        const int64_t base = cptr[r];
        for (int64_t k0 = b; k0 < e; k0 += G) {
            const int64_t k = k0 + sub;
            bool valid = false;
            uint32_t w = 0, tgt = 0;
            if (k < e) {
                const int32_t c = ci[k];
                if ((int64_t)c != r) {
                    const double cv = (-v[k]) / d;
                    if (keep_c(cv, cut)) {
                        valid = true;
                        const double scaled = floor(ldexp(fabs(cv) / amax, q));
                        w = scaled < 1.0 ? 1u : (uint32_t)scaled;
                        tgt = (uint32_t)c | (cv < 0.0 ? kSignBit : 0u);
                    }
                }
            }
            const uint64_t vm = g.ballot(valid);
            const uint32_t incl = g.incl_scan(w);
            if (valid) {
                const uint32_t pos = placed + (uint32_t)mask_rank(vm);
                sorted[base + pos] = make_uint2(carry + incl, tgt);
            }
            carry += g.bcast(incl, G - 1);
            placed += (uint32_t)__popcll(vm);
        }
        if (sub == 0) {
            const double shat = ldexp(amax * (double)carry, -q);
            tinfo[r] = make_uint4(off, m, __float_as_uint((float)shat), 0u);
            *(uint4 *)hdc = make_uint4((uint32_t)r, m, carry, __float_as_uint((float)shat));
            *(double2 *)(hdc + 4) = make_double2(shat, d);
            best = shat > best ? shat : best;
        }
    }
    best = wave_max(best);
    if ((threadIdx.x & 63) == 0 && best > 0.0) atomic_max_bits(norm_bits, best);
}

// Alias table of each row (Walker's method, Vose's exact-integer construction;
// one lane per row, as the construction is sequential): masses q_k = m w_k
// (w_k from the row's cums), bucket capacity W. Entries go, in column order, on
// a `small` (q < W) or `large` stack; while both are non-empty the tops s and l
// are popped, bucket s keeps T_s = q_s and gives W - q_s to l (A_s = l,
// q_l -= W - q_s), and l goes back on small if q_l < W, else on large. Leftover
// buckets keep all W units (T = W, A = self). Every entry's final q is its
// threshold. Both stacks live in one scratch array of the row's length (small
// grows up from the front, large down from the back), q and A in two more, at
// stride sc (vose_row); the scratch is in LDS for rows of up to kAliasLds
// entries (in the row's slice of a global scratch otherwise). The thresholds and
// alias indices end in thr_g and ali_g, indexed like the entries of C.
constexpr int kAliasLds = 32;    // rows up to this long keep their scratch in LDS
constexpr int kAliasPitch = 65;  // LDS words per entry index: the lanes of a wave hit distinct banks

template <typename I>
__device__ __forceinline__ void vose_row(uint32_t m, const uint2 *__restrict__ row, uint32_t *q, I *st, I *al,
                                         int sc) {
    const uint32_t W = row[m - 1].x;
    int ns = 0, nl = 0;
    uint32_t prev = 0;
    for (uint32_t k = 0; k < m; ++k) {
        const uint32_t cum = row[k].x;
        const uint32_t qk = m * (cum - prev);  // m w_k <= m 2^Q <= 2^31
        prev = cum;
        q[k * sc] = qk;
        al[k * sc] = (I)k;
        if (qk < W)
            st[(ns++) * sc] = (I)k;
        else
            st[(m - 1 - nl++) * sc] = (I)k;
    }
    while (ns > 0 && nl > 0) {
        const int sm = (int)st[(--ns) * sc];
        const int lg = (int)st[(m - nl--) * sc];
        al[sm * sc] = (I)lg;
        const uint32_t ql = q[lg * sc] - (W - q[sm * sc]);
        q[lg * sc] = ql;
        if (ql < W)
            st[(ns++) * sc] = (I)lg;
        else
            st[(m - 1 - nl++) * sc] = (I)lg;
    }
}

// LDS rows keep their stack and alias indices in bytes (entry indices < 32):
// 12.5 KB per wave instead of 25 KB, twice the waves per CU.
__global__ void __launch_bounds__(64) k_alias(int64_t n, const uint32_t *__restrict__ mrow,
                                              const int64_t *__restrict__ cptr, const uint2 *__restrict__ sorted,
                                              uint32_t *__restrict__ thr_g, int32_t *__restrict__ stk_g,
                                              int32_t *__restrict__ ali_g) {
    __shared__ uint32_t q_l[kAliasLds * kAliasPitch];
    __shared__ uint8_t st_l[kAliasLds * kAliasPitch];
    __shared__ uint8_t al_l[kAliasLds * kAliasPitch];
    const int lane = threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + lane; r < n; r += stride) {
        const uint32_t m = mrow[r];
        if (m == 0) continue;
        const int64_t base = cptr[r];
        if (m <= (uint32_t)kAliasLds) {
            vose_row<uint8_t>(m, sorted + base, q_l + lane, st_l + lane, al_l + lane, kAliasPitch);
            for (uint32_t k = 0; k < m; ++k) {
                thr_g[base + k] = q_l[k * kAliasPitch + lane];
                ali_g[base + k] = (int32_t)al_l[k * kAliasPitch + lane];
            }
        } else {
            vose_row<int32_t>(m, sorted + base, thr_g + base, stk_g + base, ali_g + base, 1);
        }
    }
}

constexpr int kBucketSlots = 4;
// buckets per lane in flight in k_buckets32: fewer registers, more waves (on the
// 160^3 27-point records 1.83 ms with 2, 1.93 ms with 4, 2.60 ms with 8)
constexpr int kBucketSlots32 = 2;

// Full records from the compact ones (see common.hpp). Header units: thread per
// row. Buckets: a wave takes 64 consecutive rows and writes their buckets as one
// run, four lanes per 64-byte bucket, 64 buckets per pass: {T_j, target_j,
// target_{A_j}, w_j} with T_j = floor(T'_j W / 2^32) (T_j = W where T'_j = 2^32 - 1;
// T is the only integer in ((T' - 1) W / 2^32, T' W / 2^32], an interval shorter
// than 1 as W <= 2^31), then the two targets' header words and their Shat64.
__global__ void __launch_bounds__(256) k_expand_headers(int64_t n, const uint32_t *__restrict__ roff32,
                                                        const uint32_t *__restrict__ rec32,
                                                        uint32_t *__restrict__ rec) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
        const uint32_t off = roff32[r];
        const uint4 h = *(const uint4 *)(rec32 + (size_t)off * kUnitWords32);
        const uint2 s64 = *(const uint2 *)(rec32 + (size_t)off * kUnitWords32 + 4);
        uint4 *u = (uint4 *)(rec + (size_t)off * kUnitWords);
        u[0] = h;
        u[1] = make_uint4(s64.x, s64.y, 0u, 0u);
        u[2] = make_uint4(0u, 0u, 0u, 0u);
        u[3] = make_uint4(0u, 0u, 0u, 0u);
    }
}

__global__ void __launch_bounds__(256) k_expand_buckets(int64_t n, const uint32_t *__restrict__ mrow,
                                                        const uint32_t *__restrict__ roff32,
                                                        const uint32_t *__restrict__ rec32,
                                                        uint32_t *__restrict__ rec) {
    __shared__ uint32_t pm_s[4][65];
    __shared__ uint32_t po_s[4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t *pm = pm_s[wv];
    uint32_t *po = po_s[wv];
    const int64_t wstride = (int64_t)gridDim.x * 4 * 64;
    for (int64_t r0 = ((int64_t)blockIdx.x * 4 + wv) * 64; r0 < n; r0 += wstride) {
        const int64_t r = r0 + lane;
        const uint32_t m = r < n ? mrow[r] : 0u;
        const uint32_t incl = wave_incl_scan(m);
        pm[lane + 1] = incl;
        if (lane == 0) pm[0] = 0u;
        po[lane] = r < n ? roff32[r] : 0u;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t total = (uint32_t)__shfl((int)incl, 63, 64);
        const int part = lane & 3;
        int row[kBucketSlots];
#pragma unroll
        for (int j = 0; j < kBucketSlots; ++j) row[j] = 0;
        for (uint32_t t0 = 0; t0 < total; t0 += 16 * kBucketSlots) {
            uint4 v[kBucketSlots];
            size_t dst[kBucketSlots];
#pragma unroll
            for (int j = 0; j < kBucketSlots; ++j) {
                const uint32_t t = t0 + (uint32_t)(j * 16 + (lane >> 2));
                dst[j] = ~(size_t)0;
                if (t >= total) continue;
                while (pm[row[j] + 1] <= t) ++row[j];
                const int i = row[j];
                const uint32_t k = t - pm[i];
                const uint32_t *cb = rec32 + ((size_t)po[i] + 1u + k) * kUnitWords32;
                const uint4 q0 = *(const uint4 *)cb, q1 = *(const uint4 *)(cb + 4);
                if (part == 0) {
                    const uint32_t W = rec32[(size_t)po[i] * kUnitWords32 + 2];
                    const uint32_t T = q0.x == 0xFFFFFFFFu ? W : (uint32_t)(((uint64_t)q0.x * W) >> 32);
                    v[j] = make_uint4(T, q0.y, q1.y, q1.x);
                } else if (part == 1) {
                    v[j] = *(const uint4 *)(rec32 + (size_t)(q0.y & ~kSignBit) * kUnitWords32);
                } else if (part == 2) {
                    v[j] = *(const uint4 *)(rec32 + (size_t)(q1.y & ~kSignBit) * kUnitWords32);
                } else {
                    const uint2 so = *(const uint2 *)(rec32 + (size_t)(q0.y & ~kSignBit) * kUnitWords32 + 4);
                    const uint2 sa = *(const uint2 *)(rec32 + (size_t)(q1.y & ~kSignBit) * kUnitWords32 + 4);
                    v[j] = make_uint4(so.x, so.y, sa.x, sa.y);
                }
                dst[j] = ((size_t)po[i] + 1u + k) * kUnitWords + (size_t)part * 4u;
            }
#pragma unroll
            for (int j = 0; j < kBucketSlots; ++j)
                if (dst[j] != ~(size_t)0) *(uint4 *)(rec + dst[j]) = v[j];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// The compact buckets (8 words each, see common.hpp): a wave takes 64
// consecutive rows as in k_expand_buckets, two lanes per bucket (its own half, its alias
// half) and 32 buckets per pass; the targets' record offsets, m and Shat32 come
// from the dense per-row table k_fill writes (16 bytes a row, so that neighbouring
// targets share cache lines, which their header units spread over the records
// do not).
__global__ void __launch_bounds__(256) k_buckets32(int64_t n, const uint32_t *__restrict__ mrow,
                                                   const uint32_t *__restrict__ roff32,
                                                   const int64_t *__restrict__ cptr, const uint2 *__restrict__ sorted,
                                                   const uint32_t *__restrict__ thr_g,
                                                   const int32_t *__restrict__ ali_g, const uint4 *__restrict__ tinfo,
                                                   uint32_t *__restrict__ rec32) {
    __shared__ uint32_t pm_s[4][65];
    __shared__ int64_t pb_s[4][64];
    __shared__ uint32_t po_s[4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t *pm = pm_s[wv];
    int64_t *pb = pb_s[wv];
    uint32_t *po = po_s[wv];
    const int64_t wstride = (int64_t)gridDim.x * 4 * 64;
    for (int64_t r0 = ((int64_t)blockIdx.x * 4 + wv) * 64; r0 < n; r0 += wstride) {
        const int64_t r = r0 + lane;
        const uint32_t m = r < n ? mrow[r] : 0u;
        const uint32_t incl = wave_incl_scan(m);
        pm[lane + 1] = incl;
        if (lane == 0) pm[0] = 0u;
        pb[lane] = r < n ? cptr[r] : 0;
        po[lane] = r < n ? roff32[r] : 0u;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t total = (uint32_t)__shfl((int)incl, 63, 64);
        const int half = lane & 1;
        int row[kBucketSlots32];
#pragma unroll
        for (int j = 0; j < kBucketSlots32; ++j) row[j] = 0;
        for (uint32_t t0 = 0; t0 < total; t0 += 32 * kBucketSlots32) {
            uint4 v[kBucketSlots32];
            size_t dst[kBucketSlots32];
#pragma unroll
            for (int j = 0; j < kBucketSlots32; ++j) {
                const uint32_t t = t0 + (uint32_t)(j * 32 + (lane >> 1));
                dst[j] = ~(size_t)0;
                if (t >= total) continue;
                while (pm[row[j] + 1] <= t) ++row[j];
                const int i = row[j];
                const uint32_t k = t - pm[i];
                const int64_t e = pb[i] + k;
                const uint2 own = sorted[e];
                const uint32_t W = sorted[pb[i] + pm[i + 1] - pm[i] - 1].x;
                const uint32_t T = thr_g[e];
                const bool full = T >= W;  // no alias: both halves lead to target_j
                const uint32_t trow = (half == 0 || full) ? own.y : sorted[pb[i] + ali_g[e]].y;
                const uint4 ti = tinfo[trow & ~kSignBit];
                const uint32_t tgt = ti.x | (trow & kSignBit);
                uint32_t first;
                if (half == 0) {
                    // T' = ceil(T 2^32 / W) (< 2^32 when T < W)
                    first = full ? 0xFFFFFFFFu : (uint32_t)((((uint64_t)T << 32) + (uint64_t)W - 1u) / (uint64_t)W);
                } else {
                    const uint32_t prev = k > 0 ? sorted[e - 1].x : 0u;
                    first = own.x - prev;  // w_j
                }
                v[j] = make_uint4(first, tgt, ti.y, ti.z);
                dst[j] = ((size_t)po[i] + 1u + k) * kUnitWords32 + (size_t)half * 4u;
            }
#pragma unroll
            for (int j = 0; j < kBucketSlots32; ++j)
                if (dst[j] != ~(size_t)0) *(uint4 *)(rec32 + dst[j]) = v[j];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

unsigned grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    return (unsigned)(b < 1 ? 1 : b);
}

unsigned grid_for_rows(int64_t n) {
    int64_t blocks = (n + 3) / 4;  // 4 waves per block, one row per wave
    if (blocks > 16384) blocks = 16384;
    if (blocks < 1) blocks = 1;
    return (unsigned)blocks;
}

}  // namespace

hipError_t ensure_full_records(const mcmi_cdf *cdf_c, hipStream_t s) {
    mcmi_cdf *cdf = const_cast<mcmi_cdf *>(cdf_c);
    std::lock_guard<std::mutex> guard(cdf->full_lock);
    if (cdf->rec) return hipSuccess;
    uint32_t *rec = nullptr;
    hipError_t e = dev_alloc((void **)&rec, (size_t)cdf->rec_units * kUnitWords * 4u + 64u, s);
    if (e != hipSuccess) return e;
    k_expand_headers<<<grid_for(cdf->n), 256, 0, s>>>(cdf->n, cdf->roff, cdf->rec32, rec);
    e = hipGetLastError();
    if (e == hipSuccess) {
        int64_t bb = (cdf->n + 255) / 256;
        if (bb > 16384) bb = 16384;
        k_expand_buckets<<<(unsigned)bb, 256, 0, s>>>(cdf->n, cdf->mrow, cdf->roff, cdf->rec32, rec);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        dev_release_idle(rec);
        return e;
    }
    cdf->rec = rec;
    return hipSuccess;
}

}  // namespace mcmi

using namespace mcmi;

extern "C" mcmi_status mcmi_build_cdf(const mcmi_csr_in *B, mcmi_cdf **out, void *stream) {
    return mcmi_build_cdf_ex(B, nullptr, out, stream);
}

extern "C" mcmi_status mcmi_build_cdf_ex(const mcmi_csr_in *B, const mcmi_cdf_opts *opts, mcmi_cdf **out,
                                         void *stream) {
    if (out) *out = nullptr;
    if (!B || !out) return fail(MCMI_ERR_ARG, "mcmi_build_cdf: null argument");
    const double alpha = opts ? opts->alpha : 0.0;
    const double drop_frac = opts ? opts->drop_frac : 0.0;
    const int64_t order_cell = opts ? opts->order_cell : 0;
    if (!(alpha >= 0.0) || !(alpha < 1e300) || !(drop_frac >= 0.0) || !(drop_frac < 1.0))
        return fail(MCMI_ERR_ARG, "mcmi_build_cdf_ex: need alpha >= 0 and 0 <= drop_frac < 1");
    if (order_cell < 0 || (opts && opts->reserved != 0))
        return fail(MCMI_ERR_ARG, "mcmi_build_cdf_ex: need order_cell >= 0 and reserved == 0");
    if (B->n <= 0 || B->n >= (int64_t)INT32_MAX || B->nnz < (alpha > 0.0 ? 0 : B->n) || !B->row_ptr_dev ||
        !B->col_dev || !B->val_dev)
        return fail(MCMI_ERR_ARG, "mcmi_build_cdf: need 0 < n < 2^31, nnz >= n (or alpha > 0) and device pointers");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = B->n;
    mcmi_cdf *cdf = new mcmi_cdf();
    cdf->n = n;
    uint32_t *units = nullptr, *flags = nullptr;
    int64_t *roff64 = nullptr, *cptr = nullptr, *totals = nullptr;
    unsigned long long *norm_bits = nullptr;
    void *tmp = nullptr;
    uint2 *sorted = nullptr;
    uint4 *tinfo = nullptr;
    uint32_t *qs = nullptr;
    int32_t *stk = nullptr;
    unsigned long long *cut_keys = nullptr, *sel = nullptr;
    mcmi_status st = MCMI_OK;
    auto cleanup = [&]() {
        // temporaries are stream-ordered: released behind the last kernel that uses them
        for (void *t : {(void *)cut_keys, (void *)sel, (void *)units, (void *)flags, (void *)roff64, (void *)cptr,
                        (void *)totals, (void *)norm_bits, tmp, (void *)sorted, (void *)tinfo, (void *)qs,
                        (void *)stk})
            if (t) dev_release(t, s);
    };
    auto bail = [&](mcmi_status code, const std::string &msg) {
        cleanup();
        mcmi_cdf_free(cdf);
        return fail(code, msg);
    };
#define TRY(call)                                                                             \
    do {                                                                                      \
        hipError_t _e = (call);                                                               \
        if (_e != hipSuccess) return bail(MCMI_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(_e)); \
    } while (0)
    TRY(dev_alloc((void **)&cdf->mrow, n * sizeof(uint32_t), s));
    TRY(dev_alloc((void **)&cdf->diag, n * sizeof(double), s));
    TRY(dev_alloc((void **)&cdf->roff, n * sizeof(uint32_t), s));
    TRY(dev_alloc((void **)&units, n * sizeof(uint32_t), s));
    TRY(dev_alloc((void **)&flags, sizeof(uint32_t), s));
    TRY(dev_alloc((void **)&roff64, n * sizeof(int64_t), s));
    TRY(dev_alloc((void **)&cptr, n * sizeof(int64_t), s));
    TRY(dev_alloc((void **)&totals, 2 * sizeof(int64_t), s));
    TRY(dev_alloc((void **)&norm_bits, sizeof(unsigned long long), s));
    TRY(dev_alloc((void **)&tmp, scan_tmp_bytes(n), s));
    TRY(hipMemsetAsync(flags, 0, sizeof(uint32_t), s));
    TRY(hipMemsetAsync(norm_bits, 0, sizeof(unsigned long long), s));
    const unsigned grid = grid_for_rows(n);
    // phase 1 (optional): ||B||_inf for the augmented diagonal
    double aug = 0.0;
    if (alpha > 0.0) {
        k_row_abs_max<<<grid_for(n), 256, 0, s>>>(n, B->row_ptr_dev, B->val_dev, norm_bits);
        TRY(hipGetLastError());
        unsigned long long hb = 0;
        TRY(hipMemcpyAsync(&hb, norm_bits, sizeof(hb), hipMemcpyDeviceToHost, s));
        TRY(hipStreamSynchronize(s));
        ::memcpy(&cdf->norm_b, &hb, sizeof(double));
        aug = alpha * cdf->norm_b;
        TRY(hipMemsetAsync(norm_bits, 0, sizeof(unsigned long long), s));
    }
    uint32_t hflags = 0;
    int64_t htot[2] = {0, 0};
    // lanes per row: k_count about one lane per three entries of an average row,
    // k_fill (two passes over the row, a scan per G entries) one per two. More
    // rows per wave hide more of each row's dependent loads: on the 160^3
    // 27-point matrix k_count 0.87 -> 0.60 ms (32 -> 8 lanes), k_fill 1.43 ->
    // 1.13 ms (32 -> 16 lanes; 8 lanes: 1.23 ms)
    const double per_row = (double)B->nnz / (double)n;
    const int lanes_c = per_row <= 40.0 ? 8 : per_row <= 80.0 ? 16 : per_row <= 160.0 ? 32 : 64;
    const int lanes_f = per_row <= 12.0 ? 8 : per_row <= 48.0 ? 16 : per_row <= 96.0 ? 32 : 64;
    auto count_pass = [&](const unsigned long long *cut) -> hipError_t {
        if (lanes_c == 8)
            k_count<8><<<grid, 256, 0, s>>>(n, B->nnz, B->row_ptr_dev, B->col_dev, B->val_dev, aug, cut, cdf->mrow,
                                            units, cdf->diag, flags);
        else if (lanes_c == 16)
            k_count<16><<<grid, 256, 0, s>>>(n, B->nnz, B->row_ptr_dev, B->col_dev, B->val_dev, aug, cut, cdf->mrow,
                                             units, cdf->diag, flags);
        else if (lanes_c == 32)
            k_count<32><<<grid, 256, 0, s>>>(n, B->nnz, B->row_ptr_dev, B->col_dev, B->val_dev, aug, cut, cdf->mrow,
                                             units, cdf->diag, flags);
        else
            k_count<64><<<grid, 256, 0, s>>>(n, B->nnz, B->row_ptr_dev, B->col_dev, B->val_dev, aug, cut, cdf->mrow,
                                             units, cdf->diag, flags);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = scan_exclusive_u32_to_i64(units, roff64, n, totals + 0, tmp, s);
        if (e == hipSuccess) e = scan_exclusive_u32_to_i64(cdf->mrow, cptr, n, totals + 1, tmp, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&hflags, flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(htot, totals, sizeof(htot), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        return e;
    };
    TRY(count_pass(nullptr));
    if (hflags & kFlagCsr) return bail(MCMI_ERR_CSR, "mcmi_build_cdf: invalid CSR (row_ptr, column range or order)");
    if (hflags & kFlagZeroDiag) return bail(MCMI_ERR_ZERO_DIAG, "mcmi_build_cdf: missing or zero diagonal");
    // row schedule (optional), on the pattern of B now that it is validated
    if (order_cell > 0) {
        TRY(dev_alloc((void **)&cdf->order, n * sizeof(int32_t), s));
        TRY(build_locality_order(n, B->row_ptr_dev, B->col_dev, order_cell, cdf->order, s));
    }
    // matrix reduction (optional): the cut is the key of rank K among the |c|
    const unsigned long long *cut = nullptr;
    if (drop_frac > 0.0 && htot[1] > 0) {
        const int64_t cnt = htot[1];
        const int64_t K = (int64_t)floor(drop_frac * (double)cnt);
        const int64_t nk = B->nnz;
        TRY(dev_alloc((void **)&cut_keys, (size_t)(nk > 0 ? nk : 1) * sizeof(unsigned long long), s));
        TRY(dev_alloc((void **)&sel, (2 + 256) * sizeof(unsigned long long), s));
        const unsigned long long init[2] = {0ull, (unsigned long long)K};
        TRY(hipMemcpyAsync(sel, init, sizeof(init), hipMemcpyHostToDevice, s));
        TRY(hipMemsetAsync(sel + 2, 0, 256 * sizeof(unsigned long long), s));
        k_cut_keys<<<grid, 256, 0, s>>>(n, B->row_ptr_dev, B->col_dev, B->val_dev, cdf->diag, cut_keys);
        TRY(hipGetLastError());
        for (int shift = 56; shift >= 0; shift -= 8) {
            k_radix_hist<<<grid_for(nk), 256, 0, s>>>(cut_keys, nk, shift, sel, sel + 2);
            TRY(hipGetLastError());
            k_radix_pick<<<1, 64, 0, s>>>(sel, sel + 2, shift);
            TRY(hipGetLastError());
        }
        unsigned long long hcut = 0;
        TRY(hipMemcpyAsync(&hcut, sel, sizeof(hcut), hipMemcpyDeviceToHost, s));
        cut = sel;
        TRY(count_pass(cut));
        ::memcpy(&cdf->drop_thr, &hcut, sizeof(double));
        cdf->dropped = cnt - htot[1];
    }
    if (htot[0] >= (int64_t)kSignBit) return bail(MCMI_ERR_CAPACITY, "mcmi_build_cdf: records exceed 128 GiB");
    cdf->rec_units = (uint64_t)htot[0];
    cdf->nnz_c = htot[1];
    TRY(dev_alloc((void **)&cdf->rec32, (size_t)htot[0] * kUnitWords32 * 4u + 32u, s));
    TRY(dev_alloc((void **)&sorted, (size_t)(htot[1] > 0 ? htot[1] : 1) * sizeof(uint2), s));
    TRY(dev_alloc((void **)&tinfo, (size_t)n * sizeof(uint4), s));
    if (lanes_f == 8)
        k_fill<8><<<grid, 256, 0, s>>>(n, B->row_ptr_dev, B->col_dev, B->val_dev, cdf->diag, cdf->mrow, roff64, cptr,
                                       cut, cdf->roff, cdf->rec32, sorted, tinfo, norm_bits);
    else if (lanes_f == 16)
        k_fill<16><<<grid, 256, 0, s>>>(n, B->row_ptr_dev, B->col_dev, B->val_dev, cdf->diag, cdf->mrow, roff64, cptr,
                                        cut, cdf->roff, cdf->rec32, sorted, tinfo, norm_bits);
    else if (lanes_f == 32)
        k_fill<32><<<grid, 256, 0, s>>>(n, B->row_ptr_dev, B->col_dev, B->val_dev, cdf->diag, cdf->mrow, roff64, cptr,
                                        cut, cdf->roff, cdf->rec32, sorted, tinfo, norm_bits);
    else
        k_fill<64><<<grid, 256, 0, s>>>(n, B->row_ptr_dev, B->col_dev, B->val_dev, cdf->diag, cdf->mrow, roff64, cptr,
                                        cut, cdf->roff, cdf->rec32, sorted, tinfo, norm_bits);
    TRY(hipGetLastError());
    TRY(dev_alloc((void **)&qs, (size_t)(htot[1] > 0 ? htot[1] : 1) * sizeof(uint32_t), s));
    TRY(dev_alloc((void **)&stk, (size_t)(htot[1] > 0 ? 2 * htot[1] : 2) * sizeof(int32_t), s));
    {
        int64_t ab = (n + 63) / 64;
        if (ab > 32768) ab = 32768;
        int32_t *ali = stk + (htot[1] > 0 ? htot[1] : 1);
        k_alias<<<(unsigned)ab, 64, 0, s>>>(n, cdf->mrow, cptr, sorted, qs, stk, ali);
        TRY(hipGetLastError());
        int64_t bb = (n + 255) / 256;
        if (bb > 16384) bb = 16384;
        k_buckets32<<<(unsigned)bb, 256, 0, s>>>(n, cdf->mrow, cdf->roff, cptr, sorted, qs, ali, tinfo, cdf->rec32);
    }
    TRY(hipGetLastError());
    unsigned long long hnorm = 0;
    TRY(hipMemcpyAsync(&hnorm, norm_bits, sizeof(hnorm), hipMemcpyDeviceToHost, s));
    TRY(hipStreamSynchronize(s));
    double nrm;
    ::memcpy(&nrm, &hnorm, sizeof(nrm));
    cdf->norm_inf = nrm;
#undef TRY
    cleanup();
    *out = cdf;
    return st;
}

extern "C" mcmi_status mcmi_cdf_prep_info(const mcmi_cdf *cdf, double *norm_b, double *drop_thr,
                                          int64_t *dropped) {
    if (!cdf) return fail(MCMI_ERR_ARG, "mcmi_cdf_prep_info: null cdf");
    if (norm_b) *norm_b = cdf->norm_b;
    if (drop_thr) *drop_thr = cdf->drop_thr;
    if (dropped) *dropped = cdf->dropped;
    return MCMI_OK;
}

extern "C" mcmi_status mcmi_cdf_order(const mcmi_cdf *cdf, int32_t *order_host, void *stream) {
    if (!cdf || !order_host) return fail(MCMI_ERR_ARG, "mcmi_cdf_order: null argument");
    if (!cdf->order) return fail(MCMI_ERR_ARG, "mcmi_cdf_order: the record set was built without a row schedule");
    hipStream_t s = (hipStream_t)stream;
    MCMI_HIP(hipMemcpyAsync(order_host, cdf->order, (size_t)cdf->n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MCMI_HIP(hipStreamSynchronize(s));
    return MCMI_OK;
}

extern "C" mcmi_status mcmi_cdf_info(const mcmi_cdf *cdf, int64_t *n, int64_t *nnz_c, double *norm_inf,
                                     uint64_t *rec_units) {
    if (!cdf) return fail(MCMI_ERR_ARG, "mcmi_cdf_info: null cdf");
    if (n) *n = cdf->n;
    if (nnz_c) *nnz_c = cdf->nnz_c;
    if (norm_inf) *norm_inf = cdf->norm_inf;
    if (rec_units) *rec_units = cdf->rec_units;
    return MCMI_OK;
}

extern "C" mcmi_status mcmi_cdf_download_compact(const mcmi_cdf *cdf, uint32_t *rec32_host, void *stream) {
    if (!cdf || !rec32_host) return fail(MCMI_ERR_ARG, "mcmi_cdf_download_compact: null argument");
    hipStream_t s = (hipStream_t)stream;
    MCMI_HIP(hipMemcpyAsync(rec32_host, cdf->rec32, (size_t)cdf->rec_units * kUnitWords32 * 4u, hipMemcpyDeviceToHost,
                            s));
    MCMI_HIP(hipStreamSynchronize(s));
    return MCMI_OK;
}

extern "C" mcmi_status mcmi_cdf_download(const mcmi_cdf *cdf, uint32_t *rec_host, uint32_t *roff_host,
                                         double *diag_host, void *stream) {
    if (!cdf) return fail(MCMI_ERR_ARG, "mcmi_cdf_download: null cdf");
    hipStream_t s = (hipStream_t)stream;
    if (rec_host) {
        MCMI_HIP(ensure_full_records(cdf, s));
        MCMI_HIP(hipMemcpyAsync(rec_host, cdf->rec, (size_t)cdf->rec_units * kUnitWords * 4u, hipMemcpyDeviceToHost, s));
    }
    if (roff_host) MCMI_HIP(hipMemcpyAsync(roff_host, cdf->roff, (size_t)cdf->n * 4u, hipMemcpyDeviceToHost, s));
    if (diag_host) MCMI_HIP(hipMemcpyAsync(diag_host, cdf->diag, (size_t)cdf->n * 8u, hipMemcpyDeviceToHost, s));
    MCMI_HIP(hipStreamSynchronize(s));
    return MCMI_OK;
}

// ------------------------------------------------------------ batched sets
namespace mcmi {
namespace {

// One matrix of a batch: its CSR (device) and where it starts in the
// block-diagonal row and entry spaces.
struct BatchPart {
    const int64_t *rp;
    const int32_t *col;
    const double *val;
    int64_t n, nnz, row_base, nnz_base;
};

// All matrices of a batch into one block-diagonal CSR in one launch: the blocks
// of row y of the grid take matrix y. Row pointers are shifted by the matrix's
// first entry, columns by its first row (each must lie in [0, n_k)), values
// copied; row_mat records each row's matrix. Matrix k = k_first + blockIdx.y.
__global__ void __launch_bounds__(256) k_concat(const BatchPart *parts, int32_t k_first, int64_t *rp_out,
                                                int32_t *col_out, double *val_out, int32_t *row_mat,
                                                uint32_t *flags) {
    const int32_t k = k_first + (int32_t)blockIdx.y;
    const BatchPart p = parts[k];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    for (int64_t i = t0; i < p.n; i += stride) {
        rp_out[p.row_base + i] = p.rp[i] + p.nnz_base;
        row_mat[p.row_base + i] = k;
        if (i == 0) bad |= p.rp[0] != 0 || p.rp[p.n] != p.nnz;
    }
    for (int64_t j = t0; j < p.nnz; j += stride) {
        const int32_t c = p.col[j];
        bad |= c < 0 || (int64_t)c >= p.n;
        col_out[p.nnz_base + j] = (int32_t)(c + p.row_base);
        val_out[p.nnz_base + j] = p.val[j];
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flags, kFlagCsr);
}

// ||Chat_k||_inf per matrix: the largest Shat64 of its rows (bits of non-negative
// doubles). A wave whose 64 rows belong to one matrix reduces them first.
__global__ void __launch_bounds__(256) k_matrix_norms(int64_t n, const uint32_t *rec32, const uint32_t *roff,
                                                      const int32_t *row_mat, unsigned long long *bits) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r0 = (int64_t)blockIdx.x * blockDim.x; r0 < n; r0 += stride) {  // uniform per wave
        const int64_t r = r0 + threadIdx.x;
        const bool ok = r < n;
        unsigned long long b = 0;
        int32_t k = -1;
        if (ok) {
            const uint32_t *h = rec32 + (size_t)roff[r] * kUnitWords32;  // Shat64 in words 4-5
            b = ((unsigned long long)h[5] << 32) | h[4];
            k = row_mat[r];
        }
        if (!__any(ok)) continue;  // lane 0 holds the wave's first row, so it is in range
        const int32_t k0 = __shfl(k, 0, 64);
        if (__all(!ok || k == k0)) {
            const unsigned long long m = wave_max(b);
            if ((threadIdx.x & 63) == 0 && __atomic_load_n(&bits[k0], __ATOMIC_RELAXED) < m) atomicMax(&bits[k0], m);
        } else if (ok && __atomic_load_n(&bits[k], __ATOMIC_RELAXED) < b) {
            atomicMax(&bits[k], b);
        }
    }
}


}  // namespace
}  // namespace mcmi

extern "C" mcmi_status mcmi_build_cdf_batched(const mcmi_csr_in *Bs, int32_t count, mcmi_cdf **out, void *stream) {
    return mcmi_build_cdf_batched_ex(Bs, count, nullptr, out, stream);
}

extern "C" mcmi_status mcmi_build_cdf_batched_ex(const mcmi_csr_in *Bs, int32_t count, const mcmi_cdf_opts *opts,
                                                 mcmi_cdf **out, void *stream) {
    if (out) *out = nullptr;
    if (!Bs || !out || count < 1) return fail(MCMI_ERR_ARG, "mcmi_build_cdf_batched: bad argument");
    if (opts && (opts->alpha != 0.0 || opts->drop_frac != 0.0 || opts->order_cell < 0 || opts->reserved != 0))
        return fail(MCMI_ERR_ARG, "mcmi_build_cdf_batched_ex: only order_cell >= 0 applies to a batch");
    hipStream_t s = (hipStream_t)stream;
    std::vector<int64_t> rb(count + 1, 0), zb(count + 1, 0);
    for (int32_t k = 0; k < count; ++k) {
        if (Bs[k].n <= 0 || Bs[k].nnz < Bs[k].n || !Bs[k].row_ptr_dev || !Bs[k].col_dev || !Bs[k].val_dev)
            return fail(MCMI_ERR_ARG, "mcmi_build_cdf_batched: matrix " + std::to_string(k) + " is malformed");
        rb[k + 1] = rb[k] + Bs[k].n;
        zb[k + 1] = zb[k] + Bs[k].nnz;
    }
    if (rb[count] >= (int64_t)INT32_MAX) return fail(MCMI_ERR_ARG, "mcmi_build_cdf_batched: more than 2^31 rows");
    const int64_t n = rb[count], nnz = zb[count];
    int64_t *rp = nullptr;
    int32_t *col = nullptr, *row_mat = nullptr;
    double *val = nullptr;
    uint32_t *flags = nullptr;
    int64_t *base_dev = nullptr;
    unsigned long long *nb = nullptr;
    BatchPart *parts_dev = nullptr;
    auto cleanup = [&]() {  // stream-ordered: behind the last kernel that reads them
        for (void *t : {(void *)rp, (void *)col, (void *)val, (void *)flags, (void *)nb, (void *)parts_dev})
            if (t) dev_release(t, s);
    };
#define TRYB(call)                                                                          \
    do {                                                                                    \
        hipError_t _e = (call);                                                             \
        if (_e != hipSuccess) {                                                             \
            cleanup();                                                                      \
            dev_release_idle(row_mat);                                                      \
            dev_release_idle(base_dev);                                                     \
            return fail(MCMI_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(_e));   \
        }                                                                                   \
    } while (0)
    TRYB(dev_alloc((void **)&rp, (n + 1) * sizeof(int64_t), s));
    TRYB(dev_alloc((void **)&col, nnz * sizeof(int32_t), s));
    TRYB(dev_alloc((void **)&val, nnz * sizeof(double), s));
    TRYB(dev_alloc((void **)&row_mat, n * sizeof(int32_t), s));
    TRYB(dev_alloc((void **)&base_dev, (count + 1) * sizeof(int64_t), s));
    TRYB(dev_alloc((void **)&flags, sizeof(uint32_t), s));
    TRYB(dev_alloc((void **)&nb, count * sizeof(unsigned long long), s));
    TRYB(hipMemsetAsync(flags, 0, sizeof(uint32_t), s));
    TRYB(hipMemsetAsync(nb, 0, count * sizeof(unsigned long long), s));
    // the parts table lives until the synchronisation below, which the copy precedes
    std::vector<BatchPart> parts(count);
    int64_t most = 0;
    for (int32_t k = 0; k < count; ++k) {
        parts[k] = {Bs[k].row_ptr_dev, Bs[k].col_dev, Bs[k].val_dev, Bs[k].n, Bs[k].nnz, rb[k], zb[k]};
        most = std::max(most, Bs[k].nnz);
    }
    TRYB(dev_alloc((void **)&parts_dev, count * sizeof(BatchPart), s));
    TRYB(hipMemcpyAsync(parts_dev, parts.data(), count * sizeof(BatchPart), hipMemcpyHostToDevice, s));
    {
        int64_t gx = (most + 255) / 256;
        if (gx > 64) gx = 64;  // a few blocks per matrix; 256 matrices fill the chip
        for (int32_t k0 = 0; k0 < count; k0 += 65535) {  // the grid's y extent is at most 65535
            const int32_t ky = std::min<int32_t>(65535, count - k0);
            k_concat<<<dim3((unsigned)gx, (unsigned)ky), 256, 0, s>>>(parts_dev, k0, rp, col, val, row_mat, flags);
        }
    }
    TRYB(hipGetLastError());
    TRYB(hipMemcpyAsync(rp + n, &nnz, sizeof(int64_t), hipMemcpyHostToDevice, s));
    TRYB(hipMemcpyAsync(base_dev, rb.data(), (count + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    uint32_t hflags = 0;
    TRYB(hipMemcpyAsync(&hflags, flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    TRYB(hipStreamSynchronize(s));
    if (hflags & kFlagCsr) {
        cleanup();
        dev_release_idle(row_mat);
        dev_release_idle(base_dev);
        return fail(MCMI_ERR_CSR, "mcmi_build_cdf_batched: a matrix has bad row pointers or columns");
    }
    mcmi_csr_in all{n, nnz, rp, col, val};
    mcmi_cdf *cdf = nullptr;
    mcmi_status st = mcmi_build_cdf_ex(&all, opts, &cdf, stream);
    if (st != MCMI_OK) {
        cleanup();
        dev_release_idle(row_mat);
        dev_release_idle(base_dev);
        return st;
    }
    cdf->batch = count;
    cdf->row_mat = row_mat;
    cdf->mat_base = base_dev;
    cdf->mat_base_host = rb;
    k_matrix_norms<<<grid_for(n), 256, 0, s>>>(n, cdf->rec32, cdf->roff, row_mat, nb);
    std::vector<unsigned long long> hb(count);
    hipError_t e = hipMemcpyAsync(hb.data(), nb, count * sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
#undef TRYB
    cleanup();
    if (e != hipSuccess) {
        mcmi_cdf_free(cdf);
        return fail(MCMI_ERR_HIP, std::string("mcmi_build_cdf_batched: ") + hipGetErrorString(e));
    }
    cdf->mat_norm.resize(count);
    for (int32_t k = 0; k < count; ++k) ::memcpy(&cdf->mat_norm[k], &hb[k], sizeof(double));
    *out = cdf;
    return MCMI_OK;
}

extern "C" mcmi_status mcmi_cdf_batch_info(const mcmi_cdf *cdf, int32_t *count, int64_t *row_base_host,
                                           double *norm_host) {
    if (!cdf) return fail(MCMI_ERR_ARG, "mcmi_cdf_batch_info: null cdf");
    const int32_t k = cdf->batch;
    if (count) *count = k;
    if (row_base_host) {
        if (k) ::memcpy(row_base_host, cdf->mat_base_host.data(), (k + 1) * sizeof(int64_t));
        else {
            row_base_host[0] = 0;
            row_base_host[1] = cdf->n;
        }
    }
    if (norm_host) {
        if (k) ::memcpy(norm_host, cdf->mat_norm.data(), k * sizeof(double));
        else norm_host[0] = cdf->norm_inf;
    }
    return MCMI_OK;
}

extern "C" void mcmi_cdf_free(mcmi_cdf *cdf) {
    if (!cdf) return;
    dev_release_idle(cdf->row_mat);
    dev_release_idle(cdf->mat_base);
    dev_release_idle(cdf->rec);
    dev_release_idle(cdf->rec32);
    dev_release_idle(cdf->roff);
    dev_release_idle(cdf->diag);
    dev_release_idle(cdf->mrow);
    dev_release_idle(cdf->order);
    delete cdf;
}
