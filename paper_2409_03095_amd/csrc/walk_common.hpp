// Device helpers shared by the walk kernels (internal).
#pragma once
#include "common.hpp"
#include "walk_args.hpp"

namespace mcmi {
namespace walkdev {

constexpr int32_t kEmpty = -1;
constexpr int kMaxLdsProbe = 32;

__device__ __forceinline__ uint32_t hash_key(int32_t key, int shift) {
    return ((uint32_t)key * 2654435761u) >> shift;
}

__device__ __forceinline__ bool lds_add(int32_t *keys, double *vals, uint32_t mask, uint32_t h, int32_t key,
                                        double w) {
    for (int p = 0; p < kMaxLdsProbe; ++p) {
        int32_t k = __atomic_load_n(&keys[h], __ATOMIC_RELAXED);
        if (k == kEmpty) {
            const int32_t prev = atomicCAS(&keys[h], kEmpty, key);
            k = prev == kEmpty ? key : prev;
        }
        if (k == key) {
            atomicAdd(&vals[h], w);
            return true;
        }
        h = (h + 1) & mask;
    }
    return false;
}

// per-wave HBM hash; returns false when the table is full
__device__ __forceinline__ bool spill_add(int32_t *keys, double *vals, int32_t *used, int *used_cnt, uint32_t mask,
                                          int32_t key, double w) {
    uint32_t h = ((uint32_t)key * 0x85EBCA6Bu) & mask;
    for (uint32_t p = 0; p <= mask; ++p) {
        int32_t k = __atomic_load_n(&keys[h], __ATOMIC_RELAXED);
        if (k == kEmpty) {
            const int32_t prev = atomicCAS(&keys[h], kEmpty, key);
            if (prev == kEmpty) {
                const int u = atomicAdd(used_cnt, 1);
                used[u] = (int32_t)h;
                k = key;
            } else {
                k = prev;
            }
        }
        if (k == key) {
            atomicAdd(&vals[h], w);
            return true;
        }
        h = (h + 1) & mask;
    }
    return false;
}

// Hash of a column onto the count-sketch buckets [0, nb) by a multiply-high
// (any bucket count, independent of the slot hash's multiplier).
__device__ __forceinline__ uint32_t bucket_of(int32_t key, uint32_t nb) {
    const uint32_t h = ((uint32_t)key * 0x9E3779B1u ^ 0x5bd1e995u) * 0x85EBCA77u;
    return __umulhi(h, nb);
}

// Philox row and tag words of the chains of global row r
__device__ __forceinline__ void philox_ids(const WalkArgs &a, int32_t r, uint32_t &prow, uint32_t &ptag) {
    if (a.row_mat) {
        const int32_t k = a.row_mat[r];
        prow = (uint32_t)((int64_t)r - a.mat_base[k]);
        ptag = a.tag + (uint32_t)k;
    } else {
        prow = (uint32_t)r;
        ptag = a.tag;
    }
}

// ------------------------------------------------------------- one step
// The header unit of the current state: h0 = {row, m, W, Shat32},
// h1 = {Shat64 lo, Shat64 hi, summary 0, summary 1}, h2/h3 = summaries 2..9.
struct StepHdr {
    uint4 h0, h1, h2, h3;
};

__device__ __forceinline__ void load_header(const uint32_t *rec, uint32_t off, StepHdr &H) {
    const uint4 *p = (const uint4 *)(rec + (size_t)off * kUnitWords);
    H.h0 = p[0];
    H.h1 = p[1];
    H.h2 = p[2];
    H.h3 = p[3];
}

__device__ __forceinline__ double header_shat64(const StepHdr &H) {
    return __hiloint2double((int)H.h1.y, (int)H.h1.x);
}

__device__ __forceinline__ uint32_t count_le(const uint4 &v, uint32_t t) {
    return (uint32_t)(v.x <= t) + (uint32_t)(v.y <= t) + (uint32_t)(v.z <= t) + (uint32_t)(v.w <= t);
}

// Target word (record offset | sign bit) of the first entry of the row with
// t < cum: group = number of group summaries <= t, entry = number of the
// group's cums <= t (padding words never compare <= t because t < W < 2^31).
__device__ __forceinline__ uint32_t draw_target(const uint32_t *rec, uint32_t off, const StepHdr &H, uint32_t t) {
    const uint32_t m = H.h0.y;
    const uint32_t G = record_groups(m);
    uint32_t g;
    if (G <= (uint32_t)(kUnitWords - kHdrWords)) {
        g = (uint32_t)(H.h1.z <= t) + (uint32_t)(H.h1.w <= t) + count_le(H.h2, t) + count_le(H.h3, t);
    } else {
        const uint32_t *summ = rec + (size_t)off * kUnitWords + kHdrWords;
        uint32_t lo = 0, hi = G;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (summ[mid] <= t)
                lo = mid + 1;
            else
                hi = mid;
        }
        g = lo;
    }
    const uint4 *grp = (const uint4 *)(rec + ((size_t)off + header_units(m) + g) * kUnitWords);
    const uint4 c0 = grp[0], c1 = grp[1], t0 = grp[2], t1 = grp[3];
    const uint32_t k = count_le(c0, t) + count_le(c1, t);
    uint32_t tg = t0.x;
    tg = k == 1u ? t0.y : tg;
    tg = k == 2u ? t0.z : tg;
    tg = k == 3u ? t0.w : tg;
    tg = k == 4u ? t1.x : tg;
    tg = k == 5u ? t1.y : tg;
    tg = k == 6u ? t1.z : tg;
    tg = k == 7u ? t1.w : tg;
    return tg;
}

}  // namespace walkdev
}  // namespace mcmi
