// Kernel arguments of the walk kernels (internal).
#pragma once
#include "common.hpp"

namespace mcmi {

struct WalkArgs {
    const uint32_t *rec;
    const uint32_t *rec32;         // compact records (FP32 walks)
    const uint32_t *roff;
    const double *diag;
    const int32_t *rows;           // nullable: output slot t is row t
    int64_t n_tasks;
    const int32_t *task_map;       // nullable: task k works on output slot task_map[k]
    int64_t pool_tag;              // (pool index) << 56, or-ed into row_start
    const int32_t *chains_per_row; // nullable
    int32_t chains;
    uint32_t key0, key1, tag;
    const uint32_t *keys_dev;      // nullable: read the Philox key from device memory (graph replays)
    // batched record sets: the Philox row word is the row inside its matrix and the
    // tag word is tag + matrix index (nullable: row word = global row, tag word = tag)
    const int32_t *row_mat;
    const int64_t *mat_base;
    double delta;
    float delta32;
    double eps;
    int32_t lmax;
    int32_t filter_m;
    int32_t topk;
    int32_t pool_chunk;  // > 0: a wave reserves pool space this many entries at a time
    int32_t hash_slots;            // power of two (wavefront kernel: all rows of a wavefront together)
    int32_t hash_shift;            // 32 - log2(hash_slots)
    int32_t row_lanes;             // wavefront kernel: lanes per row (8, 16, 32 or 64; 0 = 64)
    int32_t lane_chains;           // wavefront kernel, 64 lanes per row: chains a lane keeps in flight (1 or 2)
    uint32_t *queue_ctr;           // 8 counters, kQueueStride elements apart
    int64_t *row_start;            // pool position | pool_tag, or -1 when the row must be rerun
    uint32_t *row_cnt;
    int32_t *pool_col;
    double *pool_val;
    int64_t pool_cap;
    unsigned long long *pool_used;
    int32_t *spill_keys;
    double *spill_vals;
    int32_t *spill_used;
    int32_t spill_slots;           // power of two, per wave
    unsigned long long *stats;     // [0] transitions, [1] spilled, [2] chains, [3] rows refined
    uint32_t *flags;
    // workgroup-per-row kernel: contributions with |W| >= tau are tracked in the
    // LDS hash; lighter ones only update tracked columns or the count sketch
    double tau;                    // 0: track every contribution
    float tau32;
    int32_t sketch_slots;          // count-sketch buckets (0 when tau == 0)
};

}  // namespace mcmi
