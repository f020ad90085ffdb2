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

// The LDS hash is probed a bucket of 4 slots at a time (two relaxed 64-bit
// reads), so a lookup in a table at moderate load ends after about one read
// instead of walking a run of slots one by one; in a wavefront the slowest lane's
// probe sets the time. Slots fill lowest first within a bucket and never empty
// during a phase, so a bucket with an empty slot ends every search, and a full
// bucket stays full.
__device__ __forceinline__ void read_bucket(const int32_t *keys, uint32_t b, int32_t k[4]) {
    const uint64_t lo = __atomic_load_n((const uint64_t *)(keys + b), __ATOMIC_RELAXED);
    const uint64_t hi = __atomic_load_n((const uint64_t *)(keys + b + 2), __ATOMIC_RELAXED);
    k[0] = (int32_t)(uint32_t)lo;
    k[1] = (int32_t)(uint32_t)(lo >> 32);
    k[2] = (int32_t)(uint32_t)hi;
    k[3] = (int32_t)(uint32_t)(hi >> 32);
}

// index in the bucket of `key` (-1 if absent) and of its lowest empty slot (-1 if full)
__device__ __forceinline__ void scan_bucket(const int32_t k[4], int32_t key, int &hit, int &emp) {
    hit = -1;
    emp = -1;
#pragma unroll
    for (int i = 3; i >= 0; --i) {
        if (k[i] == key) hit = i;
        if (k[i] == kEmpty) emp = i;
    }
}

// Adds w to key's slot, inserting the key if absent; false when the kMaxLdsProbe
// slots from the key's bucket on are all held by other keys.
__device__ __forceinline__ bool lds_add(int32_t *keys, double *vals, uint32_t mask, uint32_t h, int32_t key,
                                        double w) {
    uint32_t b = h & ~3u;
    int nb = 0;
    while (nb < kMaxLdsProbe / 4) {
        int32_t k[4];
        read_bucket(keys, b, k);
        int hit, emp;
        scan_bucket(k, key, hit, emp);
        if (hit >= 0) {
            atomicAdd(&vals[b + hit], w);
            return true;
        }
        if (emp < 0) {
            b = (b + 4u) & mask;
            ++nb;
            continue;
        }
        const int32_t prev = atomicCAS(&keys[b + emp], kEmpty, key);
        if (prev == kEmpty || prev == key) {
            atomicAdd(&vals[b + emp], w);
            return true;
        }
        // another key took the slot (at most 4 times per bucket): read it again
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

// Top-k retention order (the row's diagonal first, then decreasing filter
// value |N_rc|, or |M_rc| = |N_rc / d_c| under the M filter, equal values by
// ascending column, padding keys INT32_MAX last): true when entry (ka, va) comes
// after entry (kb, vb). Values are N_rc here.
__device__ __forceinline__ bool top_after(const WalkArgs &a, int32_t r, int32_t ka, double va, int32_t kb,
                                          double vb) {
    const bool pa = ka == INT32_MAX, pb = kb == INT32_MAX;
    if (pa || pb) return pa && !pb;
    if (ka == r || kb == r) return kb == r && ka != r;
    const double ta = a.filter_m ? fabs(va / a.diag[ka]) : fabs(va);
    const double tb = a.filter_m ? fabs(vb / a.diag[kb]) : fabs(vb);
    if (ta != tb) return ta < tb;
    return ka > kb;
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
// Summary i is the cumulative weight at the end of group i; the last group's
// summary equals W, which no draw t < W reaches, so a row with G groups needs
// summaries 0..G-2 only.
struct StepHdr {
    uint4 h0, h1, h2, h3;
};

// h0..h2 are loaded together (a dependent load of a random unit waits a full
// memory latency when the line has left the L1 meanwhile); h3 only when the row
// needs summaries 6..9. Words not loaded read as padding.
__device__ __forceinline__ void load_header(const uint32_t *rec, uint32_t off, StepHdr &H) {
    const uint4 *u = (const uint4 *)(rec + (size_t)off * kUnitWords);
    H.h0 = u[0];
    H.h1 = u[1];
    H.h2 = u[2];
    H.h3 = make_uint4(kPad, kPad, kPad, kPad);
    const uint32_t G = record_groups(H.h0.y);
    if (G >= 8u && G <= (uint32_t)(kUnitWords - kHdrWords)) H.h3 = u[3];
}

__device__ __forceinline__ double header_shat64(const StepHdr &H) {
    return __hiloint2double((int)H.h1.y, (int)H.h1.x);
}

__device__ __forceinline__ uint32_t count_le(const uint4 &v, uint32_t t) {
    return (uint32_t)(v.x <= t) + (uint32_t)(v.y <= t) + (uint32_t)(v.z <= t) + (uint32_t)(v.w <= t);
}

// Target word (record offset | sign bit) of the first entry of the row with
// t < cum: group = number of group summaries <= t, entry = number of the
// group's cums <= t (padding words never compare <= t because t < W <= 2^31).
// The group's cums and targets are loaded together.
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
    const uint4 *grp = (const uint4 *)(rec + ((size_t)off + header_units(m)) * kUnitWords + (size_t)g * kGroupWords);
    const uint4 c = grp[0], tg = grp[1];
    const uint32_t k = count_le(c, t);
    uint32_t r = tg.x;
    r = k == 1u ? tg.y : r;
    r = k == 2u ? tg.z : r;
    r = k == 3u ? tg.w : r;
    return r;
}

}  // namespace walkdev
}  // namespace mcmi
