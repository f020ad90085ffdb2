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

// Fibonacci hash of a column into the count-sketch buckets (independent of the
// slot hash, which uses a different multiplier).
__device__ __forceinline__ uint32_t bucket_of(int32_t key, int shift) {
    return ((uint32_t)key * 0x9E3779B1u ^ 0x5bd1e995u) * 0x85EBCA77u >> shift;
}

}  // namespace walkdev
}  // namespace mcmi
