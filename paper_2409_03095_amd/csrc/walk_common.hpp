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
// reads, or one 16-byte read where one wavefront owns the table), so a lookup in a table at moderate load ends after about one read
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

// The same as one 16-byte LDS read (buckets are 16-byte aligned), for tables that
// only one wavefront updates (its LDS operations take effect in program order; a
// probe that finds the bucket taken by another lane's compare-and-swap reads it
// again).
typedef int i32x4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void read_bucket_wave(const int32_t *keys, uint32_t b, int32_t k[4]) {
    const i32x4v q = *(const i32x4v *)(keys + b);
    k[0] = q.x;
    k[1] = q.y;
    k[2] = q.z;
    k[3] = q.w;
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

// lds_add for a table one wavefront owns, whose bucket b0 (the key's home bucket)
// was read into kp earlier, while the previous step's bucket load was in flight.
// A copy that has gone stale is safe: keys never move, slots fill lowest first,
// so a key missing from the copy is either absent or in a slot the copy shows
// empty, and the compare-and-swap of the copy's first empty slot then reports it.
__device__ __forceinline__ bool lds_add_pre(int32_t *keys, double *vals, uint32_t mask, uint32_t b0,
                                            const int32_t kp[4], int32_t key, double w) {
    uint32_t b = b0;
    int nb = 0;
    bool first = true;
    while (nb < kMaxLdsProbe / 4) {
        int32_t k[4];
        if (first) {
            k[0] = kp[0];
            k[1] = kp[1];
            k[2] = kp[2];
            k[3] = kp[3];
        } else {
            read_bucket_wave(keys, b, k);
        }
        first = false;
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
        // another key took the slot: read the bucket again
    }
    return false;
}

// Adds w to key's slot, inserting the key if absent; false when the kMaxLdsProbe
// slots from the key's bucket on are all held by other keys.
// kWave: the table belongs to one wavefront (16-byte bucket reads)
template <bool kWave = false>
__device__ __forceinline__ bool lds_add(int32_t *keys, double *vals, uint32_t mask, uint32_t h, int32_t key,
                                        double w) {
    uint32_t b = h & ~3u;
    int nb = 0;
    while (nb < kMaxLdsProbe / 4) {
        int32_t k[4];
        if (kWave)
            read_bucket_wave(keys, b, k);
        else
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

// One slot of an HBM hash probe: claim it if empty, add if it holds the key.
// Returns 1 when w was added, 0 when the slot holds another key.
__device__ __forceinline__ int spill_try(int32_t *keys, double *vals, int32_t *used, int *used_cnt, uint32_t h,
                                         int32_t key, double w) {
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
    if (k != key) return 0;
    atomicAdd(&vals[h], w);
    return 1;
}

// Per-wave HBM hash of the wavefront kernel (nothing else looks keys up in it):
// a key first tries 16 slots of the table's first kSpillWindow, where a row's
// overflow usually fits, so that it occupies few cache lines of a table sized for
// the worst case; then the whole table. Returns false when the table is full.
constexpr uint32_t kSpillWindow = 2048;
__device__ __forceinline__ bool spill_add_window(int32_t *keys, double *vals, int32_t *used, int *used_cnt,
                                                 uint32_t mask, int32_t key, double w) {
    const uint32_t hk = (uint32_t)key * 0x85EBCA6Bu;
    const uint32_t wmask = mask < kSpillWindow - 1u ? mask : kSpillWindow - 1u;
    uint32_t h = hk & wmask;
    for (int p = 0; p < 16; ++p) {
        if (spill_try(keys, vals, used, used_cnt, h, key, w)) return true;
        h = (h + 1) & wmask;
    }
    h = hk & mask;
    for (uint32_t p = 0; p <= mask; ++p) {
        if (spill_try(keys, vals, used, used_cnt, h, key, w)) return true;
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
// Header of a chain's current state, kept in registers: h0 = {row, m, W,
// Shat32}; s64 = Shat as binary64 (FP64 weights only).
struct StepHdr {
    uint4 h0;
    uint2 s64;
};

// The header unit of a record (read when a chain starts at its row).
template <bool kF32>
__device__ __forceinline__ void load_header(const uint32_t *rec, uint32_t off, StepHdr &H) {
    const uint4 *u = (const uint4 *)(rec + (size_t)off * kUnitWords);
    H.h0 = u[0];
    H.s64 = kF32 ? make_uint2(0u, 0u) : make_uint2(u[1].x, u[1].y);
}

__device__ __forceinline__ double header_shat64(const StepHdr &H) {
    return __hiloint2double((int)H.s64.y, (int)H.s64.x);
}

// One transition drawn by the 32-bit word u: bucket j = (u m) >> 32 of the
// current row, position r = ((u m mod 2^32) W) >> 32 among its W units; the
// bucket's own entry if r < T_j, else its alias. The bucket's loads are issued
// together and also deliver the next state's header into N. Returns the target
// word (record offset | sign bit).
template <bool kF32>
__device__ __forceinline__ uint32_t draw_next(const uint32_t *rec, uint32_t off, const StepHdr &H, uint32_t u,
                                              StepHdr &N) {
    const uint32_t m = H.h0.y, W = H.h0.z;
    const uint32_t j = __umulhi(u, m);
    const uint32_t f = u * m;
    const uint32_t r = __umulhi(f, W);
    const uint4 *b = (const uint4 *)(rec + ((size_t)off + 1u + j) * kUnitWords);
    const uint4 q0 = b[0], q1 = b[1], q2 = b[2];
    const uint4 q3 = kF32 ? make_uint4(0u, 0u, 0u, 0u) : b[3];
    const bool own = r < q0.x;
    N.h0 = own ? q1 : q2;
    N.s64 = own ? make_uint2(q3.x, q3.y) : make_uint2(q3.z, q3.w);
    return own ? q0.y : q0.z;
}

// draw_next in two halves, so that other work can run while the bucket is in
// flight: bucket_issue picks the bucket and position and issues its loads,
// bucket_resolve picks the entry once they have arrived.
struct BucketLd {
    uint4 q0, q1, q2, q3;
    uint32_t r;
};

template <bool kF32>
__device__ __forceinline__ void bucket_issue(const uint32_t *rec, uint32_t off, const StepHdr &H, uint32_t u,
                                             BucketLd &b) {
    const uint32_t m = H.h0.y, W = H.h0.z;
    const uint32_t j = __umulhi(u, m);
    const uint32_t f = u * m;
    b.r = __umulhi(f, W);
    const uint4 *p = (const uint4 *)(rec + ((size_t)off + 1u + j) * kUnitWords);
    b.q0 = p[0];
    b.q1 = p[1];
    b.q2 = p[2];
    b.q3 = kF32 ? make_uint4(0u, 0u, 0u, 0u) : p[3];
}

template <bool kF32>
__device__ __forceinline__ uint32_t bucket_resolve(const BucketLd &b, StepHdr &N) {
    const bool own = b.r < b.q0.x;
    N.h0 = own ? b.q1 : b.q2;
    N.s64 = own ? make_uint2(b.q3.x, b.q3.y) : make_uint2(b.q3.z, b.q3.w);
    return own ? b.q0.y : b.q0.z;
}

// ---------------------------------------------------- compact records (FP32)
// A chain's state in compact records: h0 = {record offset (the accumulation
// key), m, 0, Shat32}.
__device__ __forceinline__ void load_header_c(const uint32_t *rec32, uint32_t off, StepHdr &H) {
    const uint4 h = *(const uint4 *)(rec32 + (size_t)off * kUnitWords32);
    H.h0 = make_uint4(off, h.y, 0u, h.w);
    H.s64 = make_uint2(0u, 0u);
}

// A compact draw: bucket j = (u m) >> 32, f = u m mod 2^32; target_j iff f < T'_j.
__device__ __forceinline__ void bucket_issue_c(const uint32_t *rec32, uint32_t off, const StepHdr &H, uint32_t u,
                                               BucketLd &b) {
    const uint64_t um = (uint64_t)u * H.h0.y;
    const uint32_t j = (uint32_t)(um >> 32);
    b.r = (uint32_t)um;
    const uint4 *p = (const uint4 *)(rec32 + ((size_t)off + 1u + j) * kUnitWords32);
    b.q0 = p[0];
    b.q1 = p[1];
}

__device__ __forceinline__ uint32_t bucket_resolve_c(const BucketLd &b, StepHdr &N) {
    const bool own = b.r < b.q0.x;
    const uint32_t tgt = own ? b.q0.y : b.q1.y;
    N.h0 = make_uint4(tgt & ~kSignBit, own ? b.q0.z : b.q1.z, 0u, own ? b.q0.w : b.q1.w);
    N.s64 = make_uint2(0u, 0u);
    return tgt;
}

// Row (column index) and d of the row whose compact record starts at unit `off`.
__device__ __forceinline__ int32_t row_of_c(const uint32_t *rec32, uint32_t off) {
    return (int32_t)rec32[(size_t)off * kUnitWords32];
}
__device__ __forceinline__ double diag_of_c(const uint32_t *rec32, uint32_t off) {
    return *(const double *)(rec32 + (size_t)off * kUnitWords32 + 6);
}

}  // namespace walkdev
}  // namespace mcmi
