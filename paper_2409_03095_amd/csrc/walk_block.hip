// Workgroup-per-row Monte Carlo walks with heavy/light accumulation (gfx950).
//
// Same estimator as the wavefront-per-row kernel (Section III-A, eq. (2);
// Section IV-A phase 4 scaling; the eps filter), for rows whose chains touch
// more distinct columns than an LDS hash can hold (random sparsity: with m
// entries per row, a row's chains reach ~m^j columns at step j).
//
// A contribution is heavy when |W| >= tau, light otherwise. With ||Chat||_inf < 1
// weights never grow along a chain, so each chain's heavy contributions form a
// prefix. The row is processed in phases, each over all N_r chains:
//   H  heavy contributions are accumulated in the LDS hash (spilling to HBM);
//      a chain pauses at its first light contribution;
//   L  light contributions are added to the column's slot when the column is
//      tracked; otherwise |W| is added to a count sketch bucket chosen by hashing
//      the column. An untracked column's |sum| is at most its bucket total, so
//      when every bucket stays below eps * N_r (with a 1/16 margin that covers
//      binary32 bucket sums) no untracked column can pass the filter, and every
//      tracked column has its complete sum;
//   R  only if some bucket fails that bound: replay every chain from its start
//      (counter-based random numbers make the replay exact) and track the light
//      contributions whose bucket failed, as new columns.
// The kept set and the values are then those of full accumulation.
//
// With N_r <= lanes each lane keeps its chain's state in registers across H and
// L; otherwise phase L replays chains from their start, skipping the heavy prefix.
//
// FP32 walks read the compact records (32-byte units, two loads per step); their
// accumulation key is the state's record offset, which orders like the column
// and becomes it at the finalize (one header read per kept entry). FP64 walks
// read the full records and key by column.
#include "common.hpp"
#include "walk_args.hpp"
#include "walk_common.hpp"

namespace mcmi {

namespace {

using namespace walkdev;

constexpr uint32_t kRBit = 0x80000000u;  // marks columns first tracked in phase R

enum Mode { kAll = 0, kHeavy = 1, kLight = 2, kRefine = 3 };

struct Chain {
    int32_t c;
    uint32_t off, j;
    double w64;
    float w32;
    u32x4 blk;
    StepHdr h;  // header of the current state
    bool active;
};

struct RowCtx {
    int32_t r, N;
    uint32_t prow, ptag;  // Philox row and tag words
    uint32_t k0, k1;      // Philox key
    uint32_t r_off;
    int32_t rk;  // the key of row r itself: its record offset (FP32), else r
    StepHdr h0;  // header of row r, where every chain starts
    int32_t *keys;
    double *vals;
    float *sketch;
    int *spill_cnt;
    int32_t *skeys;
    double *svals;
    int32_t *sused;
    bool row_spilled;  // phase H spilled at least one column
    float hot_thr;     // bucket total that fails the certificate
};

__device__ __forceinline__ void chain_start(Chain &st, int32_t c, const RowCtx &rc) {
    st.c = c;
    st.off = rc.r_off;
    st.h = rc.h0;
    st.j = 0;
    st.w64 = 1.0;
    st.w32 = 1.0f;
    st.active = c < rc.N;
}

// header of the record at unit off: compact (FP32 walks) or full
template <bool kF32>
__device__ __forceinline__ void row_header(const WalkArgs &a, uint32_t off, StepHdr &H) {
    if (kF32)
        load_header_c(a.rec32, off, H);
    else
        load_header<false>(a.rec, off, H);
}

// d of an accumulation key's column
template <bool kF32>
__device__ __forceinline__ double key_diag(const WalkArgs &a, int32_t key) {
    return kF32 ? diag_of_c(a.rec32, (uint32_t)key) : a.diag[key];
}

// light contribution: add to the tracked column, else to its sketch bucket
template <bool kF32>
__device__ __forceinline__ void light_add(const WalkArgs &a, const RowCtx &rc, int32_t key, double w,
                                          unsigned long long &spilled) {
    const uint32_t hmask = (uint32_t)a.hash_slots - 1u;
    uint32_t b = hash_key(key, a.hash_shift) & ~3u;
    bool full_run = true;
    for (int nb = 0; nb < kMaxLdsProbe / 4; ++nb) {
        int32_t k[4];
        read_bucket(rc.keys, b, k);
        int hit, emp;
        scan_bucket(k, key, hit, emp);
        if (hit >= 0) {
            atomicAdd(&rc.vals[b + hit], w);
            return;
        }
        if (emp >= 0) {
            full_run = false;
            break;
        }
        b = (b + 4u) & hmask;
    }
    if (full_run && rc.row_spilled) {
        const uint32_t smask = (uint32_t)a.spill_slots - 1u;
        uint32_t g = ((uint32_t)key * 0x85EBCA6Bu) & smask;
        for (uint32_t p = 0; p <= smask; ++p) {
            const int32_t k = __atomic_load_n(&rc.skeys[g], __ATOMIC_RELAXED);
            if (k == key) {
                atomicAdd(&rc.svals[g], w);
                ++spilled;
                return;
            }
            if (k == kEmpty) break;
            g = (g + 1) & smask;
        }
    }
    double mag = fabs(w);
    if (a.filter_m) mag = mag / fabs(key_diag<kF32>(a, key));
    atomicAdd(&rc.sketch[bucket_of(key, (uint32_t)a.sketch_slots)], (float)mag);
}

// refine: track light contributions of columns whose bucket failed the bound
__device__ __forceinline__ void refine_add(const WalkArgs &a, const RowCtx &rc, int32_t key, double w,
                                           bool &spill_full, unsigned long long &spilled) {
    if (rc.sketch[bucket_of(key, (uint32_t)a.sketch_slots)] < rc.hot_thr) return;
    const int32_t rkey = (int32_t)((uint32_t)key | kRBit);
    const uint32_t hmask = (uint32_t)a.hash_slots - 1u;
    uint32_t b = hash_key(key, a.hash_shift) & ~3u;
    int nb = 0;
    while (nb < kMaxLdsProbe / 4) {
        int32_t k[4];
        read_bucket(rc.keys, b, k);
        int hit, emp, rhit, remp;
        scan_bucket(k, key, hit, emp);
        if (hit >= 0) return;  // tracked since phase H: already complete
        scan_bucket(k, rkey, rhit, remp);
        if (rhit >= 0) {
            atomicAdd(&rc.vals[b + rhit], w);
            return;
        }
        if (emp < 0) {
            b = (b + 4u) & hmask;
            ++nb;
            continue;
        }
        const int32_t prev = atomicCAS(&rc.keys[b + emp], kEmpty, rkey);
        if (prev == kEmpty || prev == rkey) {
            atomicAdd(&rc.vals[b + emp], w);
            return;
        }
        // another column took the slot: read the bucket again
    }
    // HBM table: a heavy column may live there; else track the light column there
    const uint32_t smask = (uint32_t)a.spill_slots - 1u;
    uint32_t g = ((uint32_t)key * 0x85EBCA6Bu) & smask;
    ++spilled;
    for (uint32_t p = 0; p <= smask; ++p) {
        int32_t k = __atomic_load_n(&rc.skeys[g], __ATOMIC_RELAXED);
        if (k == kEmpty) {
            const int32_t prev = atomicCAS(&rc.skeys[g], kEmpty, rkey);
            if (prev == kEmpty) {
                const int u = atomicAdd(rc.spill_cnt, 1);
                rc.sused[u] = (int32_t)g;
                k = rkey;
            } else {
                k = prev;
            }
        }
        if (k == key) return;
        if (k == rkey) {
            atomicAdd(&rc.svals[g], w);
            return;
        }
        g = (g + 1) & smask;
    }
    spill_full = true;
}

// Run this lane's chains (c, c + stride, ...) in one phase. In kHeavy mode a
// chain pauses (stays active, state kept) at its first light contribution.
template <bool kF32, int kMode>
__device__ __forceinline__ void run_chains(const WalkArgs &a, const RowCtx &rc, Chain &st, int stride, bool count,
                           unsigned long long &trans, unsigned long long &spilled, bool &spill_full,
                           bool &paused) {
    const uint32_t hmask = (uint32_t)a.hash_slots - 1u;
    const uint32_t smask = (uint32_t)a.spill_slots - 1u;
    paused = false;
    while (st.active) {
        const StepHdr H = st.h;
        const uint4 h = H.h0;  // row, m, W, Shat32
        const double s64 = kF32 ? 0.0 : header_shat64(H);
        if (st.j > 0) {
            const int32_t key = (int32_t)h.x;
            const double w = kF32 ? (double)st.w32 : st.w64;
            const bool heavy = kF32 ? (fabsf(st.w32) >= a.tau32) : (fabs(st.w64) >= a.tau);
            if (kMode == kAll || (kMode == kHeavy && heavy)) {
                if (!lds_add(rc.keys, rc.vals, hmask, hash_key(key, a.hash_shift), key, w)) {
                    ++spilled;
                    if (!spill_add(rc.skeys, rc.svals, rc.sused, rc.spill_cnt, smask, key, w)) spill_full = true;
                }
            } else if (kMode == kHeavy) {
                paused = true;
                break;
            } else if (kMode == kLight) {
                if (!heavy) light_add<kF32>(a, rc, key, w, spilled);
            } else {
                if (!heavy) refine_add(a, rc, key, w, spill_full, spilled);
            }
        }
        bool stop = (h.y == 0u) || (st.j >= (uint32_t)a.lmax);
        double wn64 = 0.0;
        float wn32 = 0.0f;
        if (kF32) {
            wn32 = st.w32 * __uint_as_float(h.w);
            stop = stop || (fabsf(wn32) < a.delta32);
        } else {
            wn64 = st.w64 * s64;
            stop = stop || (fabs(wn64) < a.delta);
        }
        if (stop) {
            if (count) trans += st.j;
            chain_start(st, st.c + stride, rc);
        } else {
            if ((st.j & 3u) == 0u)
                st.blk = philox4x32_10(st.j >> 2, (uint32_t)st.c, rc.prow, rc.ptag, rc.k0, rc.k1);
            const uint32_t u = st.blk.x;
            st.blk.x = st.blk.y;
            st.blk.y = st.blk.z;
            st.blk.z = st.blk.w;
            uint32_t tgt;
            if (kF32) {
                BucketLd b;
                bucket_issue_c(a.rec32, st.off, H, u, b);
                tgt = bucket_resolve_c(b, st.h);
            } else {
                tgt = draw_next<false>(a.rec, st.off, H, u, st.h);
            }
            const bool neg = (tgt & kSignBit) != 0u;
            if (kF32)
                st.w32 = neg ? -wn32 : wn32;
            else
                st.w64 = neg ? -wn64 : wn64;
            st.off = tgt & ~kSignBit;
            ++st.j;
        }
    }
}

// Compare-exchange of a bitonic pass on (column, value) pairs: the first keeps
// the smaller column of an ascending pair (up), the larger of a descending one.
__device__ __forceinline__ void exch_kv(int32_t &ka, double &va, int32_t &kb, double &vb, bool up) {
    if ((ka > kb) == up) {
        const int32_t tk = ka;
        ka = kb;
        kb = tk;
        const double tv = va;
        va = vb;
        vb = tv;
    }
}

template <int kLPR>
__device__ __forceinline__ float block_max(float v, float *red) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    v = wave_max(v);
    if (lane == 0) red[w] = v;
    __syncthreads();
    float m = red[0];
#pragma unroll
    for (int k = 1; k < kLPR / 64; ++k) m = red[k] > m ? red[k] : m;
    __syncthreads();
    return m;
}

// exclusive scan of one int per thread over the block; *total receives the sum
template <int kLPR>
__device__ __forceinline__ int block_scan(int v, int *red, int *total) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int incl = wave_incl_scan(v);
    if (lane == 63) red[w] = incl;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kLPR / 64; ++k) {
        base += k < w ? red[k] : 0;
        tot += red[k];
    }
    __syncthreads();
    *total = tot;
    return base + incl - v;
}

// Next row from the XCD queues (called by one thread; -1 when all are drained).
__device__ __forceinline__ int64_t grab_task(const WalkArgs &a, int &queue) {
    for (int tries = 0; tries < 8; ++tries) {
        const int q = (queue + tries) & 7;
        const int64_t lo = a.n_tasks * q / 8, hi = a.n_tasks * (q + 1) / 8;
        if (hi > lo && __atomic_load_n(&a.queue_ctr[q * kQueueStride], __ATOMIC_RELAXED) < (uint32_t)(hi - lo)) {
            const uint32_t idx = atomicAdd(&a.queue_ctr[q * kQueueStride], 1u);
            if ((int64_t)idx < hi - lo) {
                queue = q;
                return lo + idx;
            }
        }
    }
    return -1;
}

__device__ __forceinline__ void put_task(int *ctl, int64_t task) {
    ctl[8] = (int)(task & 0xffffffff);
    ctl[9] = (int)(task >> 32);
}

__device__ __forceinline__ int64_t get_task(const int *ctl) {
    return (int64_t)(((uint64_t)(uint32_t)ctl[9] << 32) | (uint32_t)ctl[8]);
}

// A row's record offset and header, loaded ahead of its walk.
struct RowPre {
    int64_t task;
    uint32_t r_off;
    StepHdr h0;
};

__device__ __forceinline__ int32_t task_row(const WalkArgs &a, int64_t task, int64_t &slot) {
    slot = a.task_map ? (int64_t)a.task_map[task] : task;
    return a.rows ? a.rows[slot] : (int32_t)slot;
}

template <bool kF32, int kLPR, int kQ>
__device__ __forceinline__ void block_row(const WalkArgs &a, const RowPre &cur, RowPre &nxt, int &queue, RowCtx &rc,
                          int *ctl, float *redf, int *redi,
                          unsigned long long &trans, unsigned long long &spilled, bool &spill_full,
                          bool &stage_full) {
    constexpr int H = kLPR * kQ;
    const int tid = threadIdx.x;
    const int64_t task = cur.task;
    int64_t slot;
    const int32_t r = task_row(a, task, slot);
    const int32_t N = a.chains_per_row ? a.chains_per_row[r] : a.chains;
    unsigned long long row_trans = 0;
    spill_full = false;
    stage_full = false;
    rc.r = r;
    rc.N = N;
    philox_ids(a, r, rc.prow, rc.ptag);
    rc.r_off = cur.r_off;
    rc.rk = kF32 ? (int32_t)cur.r_off : r;
    rc.h0 = cur.h0;
    const bool split = a.tau > 0.0;
    const bool reg = N <= kLPR;
    if (tid == 0) lds_add(rc.keys, rc.vals, H - 1u, hash_key(rc.rk, a.hash_shift), rc.rk, (double)N);
    __syncthreads();

    Chain st;
    bool paused;
    chain_start(st, tid, rc);
    if (!split) {
        run_chains<kF32, kAll>(a, rc, st, kLPR, true, row_trans, spilled, spill_full, paused);
        __syncthreads();
    } else {
        run_chains<kF32, kHeavy>(a, rc, st, kLPR, reg, row_trans, spilled, spill_full, paused);
        if (!reg) {
            // the other chains of this lane must finish phase H before any light sum
            for (;;) {
                if (paused) chain_start(st, st.c + kLPR, rc);
                if (!st.active) break;
                run_chains<kF32, kHeavy>(a, rc, st, kLPR, false, row_trans, spilled, spill_full, paused);
            }
        }
        __syncthreads();
        rc.row_spilled = *rc.spill_cnt > 0;  // some heavy column lives in the HBM table
        if (!reg) chain_start(st, tid, rc);
        run_chains<kF32, kLight>(a, rc, st, kLPR, true, row_trans, spilled, spill_full, paused);
        __syncthreads();
        // certificate: every untracked column is bounded by its bucket total
        float mx = 0.f;
        for (int b = tid; b < a.sketch_slots; b += kLPR) mx = fmaxf(mx, rc.sketch[b]);
        mx = block_max<kLPR>(mx, redf);
        const float thr = (float)(a.eps * (double)N) * (15.0f / 16.0f);
        if (mx >= thr) {
            rc.hot_thr = thr;
            chain_start(st, tid, rc);
            run_chains<kF32, kRefine>(a, rc, st, kLPR, false, row_trans, spilled, spill_full, paused);
            if (tid == 0) atomicAdd(&a.stats[3], 1ull);
            __syncthreads();
        }
    }

    // ------------------------------------------------------------ finalize
    // the next row: taken now, its offset and header loaded during this finalize
    if (tid == 0) put_task(ctl, grab_task(a, queue));
    const double nd = (double)N;
    // compaction in one pass: each lane reads its kQ consecutive slots, one block
    // scan places the survivors (all reads precede the scan's barrier, so writing
    // in place is safe)
    int32_t ks[kQ];
    double vs[kQ];
    int cnt = 0;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        const int s = tid * kQ + q;
        const int32_t raw = rc.keys[s];
        const double acc = rc.vals[s];
        ks[q] = kEmpty;
        vs[q] = 0.0;
        if (raw != kEmpty) {
            const int32_t key = (int32_t)((uint32_t)raw & ~kRBit);
            const double nhat = acc / nd;  // N_rc; scaled by 1 / d_c once the kept set is final
            const double test = a.filter_m ? fabs(nhat / key_diag<kF32>(a, key)) : fabs(nhat);
            if (key == rc.rk || (nhat != 0.0 && test >= a.eps)) {
                ks[q] = key;
                vs[q] = nhat;
                ++cnt;
            }
        }
    }
    int K;
    int pos = block_scan<kLPR>(cnt, redi, &K);
#pragma unroll
    for (int q = 0; q < kQ; ++q)
        if (ks[q] != kEmpty) {
            rc.keys[pos] = ks[q];
            rc.vals[pos] = vs[q];
            ++pos;
        }
    __syncthreads();
    nxt.task = get_task(ctl);
    int64_t nslot = 0;
    const int32_t nr = nxt.task >= 0 ? task_row(a, nxt.task, nslot) : 0;
    nxt.r_off = nxt.task >= 0 ? a.roff[nr] : 0u;
    // spilled columns
    const int nsp = *rc.spill_cnt;
    for (int base = 0; base < nsp; base += kLPR) {
        const int u = base + tid;
        int32_t key = kEmpty;
        double nhat = 0.0;
        int keep = 0;
        if (u < nsp) {
            const int32_t sl = rc.sused[u];
            key = (int32_t)((uint32_t)rc.skeys[sl] & ~kRBit);
            nhat = rc.svals[sl] / nd;
            const double test = a.filter_m ? fabs(nhat / key_diag<kF32>(a, key)) : fabs(nhat);
            keep = (key == rc.rk || (nhat != 0.0 && test >= a.eps)) ? 1 : 0;
            rc.skeys[sl] = kEmpty;
            rc.svals[sl] = 0.0;
        }
        int added;
        const int p = K + block_scan<kLPR>(keep, redi, &added);
        if (keep) {
            if (p < H) {
                rc.keys[p] = key;
                rc.vals[p] = nhat;
            } else {
                stage_full = true;
            }
        }
        K += added;
    }
    if (K > H) K = H;
    __syncthreads();
    if (nxt.task >= 0) row_header<kF32>(a, nxt.r_off, nxt.h0);
    if (kF32) {
        // record offsets -> columns (the same order)
        for (int i = tid; i < K; i += kLPR) rc.keys[i] = row_of_c(a.rec32, (uint32_t)rc.keys[i]);
        __syncthreads();
    }
    // top-k retention: bitonic sort in retention order, keep the first topk,
    // then turn N_rc into M_rc = N_rc / d_c
    if (a.topk > 0) {
        if (K > a.topk) {
            int PT = 1;
            while (PT < K) PT <<= 1;
            for (int s = K + tid; s < PT; s += kLPR) rc.keys[s] = INT32_MAX;
            __syncthreads();
            for (int k = 2; k <= PT; k <<= 1) {
                for (int jj = k >> 1; jj > 0; jj >>= 1) {
                    for (int i = tid; i < PT; i += kLPR) {
                        const int ixj = i ^ jj;
                        if (ixj > i) {
                            const int32_t ka = rc.keys[i], kb = rc.keys[ixj];
                            const double va = rc.vals[i], vb = rc.vals[ixj];
                            if (top_after(a, r, ka, va, kb, vb) == ((i & k) == 0)) {
                                rc.keys[i] = kb;
                                rc.keys[ixj] = ka;
                                rc.vals[i] = vb;
                                rc.vals[ixj] = va;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            K = a.topk;
        }
    }
    // M_rc = N_rc / d_c for the kept entries only (the eps test on N_rc needs no
    // diagonal)
    for (int i = tid; i < K; i += kLPR) rc.vals[i] = rc.vals[i] / a.diag[rc.keys[i]];
    __syncthreads();
    int P = 1;
    while (P < K) P <<= 1;
    for (int s = K + tid; s < P; s += kLPR) rc.keys[s] = INT32_MAX;
    __syncthreads();
    // two bitonic passes per barrier: a thread takes the entries b, b + h, b + jj,
    // b + jj + h (h = jj / 2; b with bits h and jj clear) and applies the
    // exchanges at distance jj, then at distance h
    for (int k = 2; k <= P; k <<= 1) {
        int jj = k >> 1;
        for (; jj >= 2; jj >>= 2) {
            const int h = jj >> 1;
            const int ph = __builtin_ctz((unsigned)h);
            for (int g = tid; g < (P >> 2); g += kLPR) {
                const int b = ((g >> ph) << (ph + 2)) | (g & (h - 1));
                const bool up = (b & k) == 0;
                int32_t k0 = rc.keys[b], k1 = rc.keys[b + h], k2 = rc.keys[b + jj], k3 = rc.keys[b + jj + h];
                double v0 = rc.vals[b], v1 = rc.vals[b + h], v2 = rc.vals[b + jj], v3 = rc.vals[b + jj + h];
                exch_kv(k0, v0, k2, v2, up);
                exch_kv(k1, v1, k3, v3, up);
                exch_kv(k0, v0, k1, v1, up);
                exch_kv(k2, v2, k3, v3, up);
                rc.keys[b] = k0;
                rc.keys[b + h] = k1;
                rc.keys[b + jj] = k2;
                rc.keys[b + jj + h] = k3;
                rc.vals[b] = v0;
                rc.vals[b + h] = v1;
                rc.vals[b + jj] = v2;
                rc.vals[b + jj + h] = v3;
            }
            __syncthreads();
        }
        if (jj == 1) {
            for (int pr = tid; pr < (P >> 1); pr += kLPR) {
                const int i = pr << 1;
                int32_t ka = rc.keys[i], kb = rc.keys[i + 1];
                double va = rc.vals[i], vb = rc.vals[i + 1];
                exch_kv(ka, va, kb, vb, (i & k) == 0);
                rc.keys[i] = ka;
                rc.keys[i + 1] = kb;
                rc.vals[i] = va;
                rc.vals[i + 1] = vb;
            }
            __syncthreads();
        }
    }
    // row-wide overflow flags: a row whose tables overflowed is rerun, not written
    if (spill_full) atomicOr(&ctl[6], 1);
    if (stage_full) atomicOr(&ctl[6], 2);
    __syncthreads();
    const int row_fail = ctl[6];
    unsigned long long *pool_pos = (unsigned long long *)(ctl + 4);
    if (tid == 0) *pool_pos = row_fail ? 0ull : atomicAdd(a.pool_used, (unsigned long long)K);
    __syncthreads();
    const unsigned long long pos0 = *pool_pos;
    const bool fits = (int64_t)(pos0 + (unsigned long long)K) <= a.pool_cap;
    const bool ok = fits && !row_fail;
    if (ok) {
        for (int i = tid; i < K; i += kLPR) {
            a.pool_col[pos0 + i] = rc.keys[i];
            a.pool_val[pos0 + i] = rc.vals[i];
        }
        trans += row_trans;
    }
    if (tid == 0) {
        a.row_start[slot] = ok ? ((int64_t)pos0 | a.pool_tag) : -1;
        a.row_cnt[slot] = (uint32_t)K;
        uint32_t f = 0;
        if (!fits && !row_fail) f |= kFlagPool;
        if (row_fail & 1) f |= kFlagSpill;
        if (row_fail & 2) f |= kFlagStage;
        if (f) atomicOr(a.flags, f);
        if (ok) atomicAdd(&a.stats[2], (unsigned long long)N);
        ctl[6] = 0;
    }
    __syncthreads();
    for (int s = tid; s < H; s += kLPR) {
        rc.keys[s] = kEmpty;
        rc.vals[s] = 0.0;
    }
    for (int b = tid; b < a.sketch_slots; b += kLPR) rc.sketch[b] = 0.f;
    if (tid == 0) *rc.spill_cnt = 0;
    __syncthreads();
}

template <bool kF32, int kLPR, int kQ>
__global__ void __launch_bounds__(kLPR, 4) k_walk_block(WalkArgs a) {
    constexpr int H = kLPR * kQ;
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x;
    double *vals = (double *)smem;
    int32_t *keys = (int32_t *)(smem + (size_t)H * 8u);
    float *sketch = (float *)(smem + (size_t)H * 12u);
    int *ctl = (int *)(smem + (size_t)H * 12u + (size_t)a.sketch_slots * 4u);  // 16 ints
    float *redf = (float *)(ctl + 16);
    int *redi = (int *)(redf + 16);
    for (int s = tid; s < H; s += kLPR) {
        keys[s] = kEmpty;
        vals[s] = 0.0;
    }
    for (int b = tid; b < a.sketch_slots; b += kLPR) sketch[b] = 0.f;
    if (tid < 16) ctl[tid] = 0;
    __syncthreads();
    RowCtx rc;
    rc.keys = keys;
    rc.vals = vals;
    rc.sketch = sketch;
    rc.spill_cnt = &ctl[0];
    rc.skeys = a.spill_keys + (int64_t)blockIdx.x * a.spill_slots;
    rc.svals = a.spill_vals + (int64_t)blockIdx.x * a.spill_slots;
    rc.sused = a.spill_used + (int64_t)blockIdx.x * a.spill_slots;
    rc.row_spilled = false;
    rc.hot_thr = 0.f;
    rc.k0 = a.keys_dev ? a.keys_dev[0] : a.key0;
    rc.k1 = a.keys_dev ? a.keys_dev[1] : a.key1;
    unsigned long long trans = 0, spilled = 0;
    bool spill_full = false, stage_full = false;
    int queue = (int)(blockIdx.x & 7u);
    RowPre cur;
    if (tid == 0) put_task(ctl, grab_task(a, queue));
    __syncthreads();
    cur.task = get_task(ctl);
    __syncthreads();
    if (cur.task >= 0) {
        int64_t slot;
        cur.r_off = a.roff[task_row(a, cur.task, slot)];
        row_header<kF32>(a, cur.r_off, cur.h0);
    }
    while (cur.task >= 0) {
        RowPre nxt;
        block_row<kF32, kLPR, kQ>(a, cur, nxt, queue, rc, ctl, redf, redi, trans, spilled, spill_full, stage_full);
        cur = nxt;
    }
    // one set of atomics per workgroup
    trans = wave_sum(trans);
    spilled = wave_sum(spilled);
    if ((tid & 63) == 0) {
        if (trans) atomicAdd(&a.stats[0], trans);
        if (spilled) atomicAdd(&a.stats[1], spilled);
    }
}

template <bool kF32, int kLPR, int kQ>
hipError_t launch_one(const WalkArgs &a, int blocks, hipStream_t s, size_t lds) {
    k_walk_block<kF32, kLPR, kQ><<<blocks, kLPR, lds, s>>>(a);
    return hipGetLastError();
}

template <bool kF32, int kLPR, int kQ>
hipError_t occ_one(int *bpc, size_t lds) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(bpc, k_walk_block<kF32, kLPR, kQ>, kLPR, lds);
}

}  // namespace

size_t walk_block_lds_bytes(int hash_slots, int sketch_slots) {
    return (size_t)hash_slots * 12u + (size_t)sketch_slots * 4u + 16 * 4 + 16 * 4 + 16 * 4;
}

// Supported shapes: lanes in {256, 512, 1024}, slots per lane in {2, 4, 8, 16}.
#define MCMI_BLOCK_SHAPES(X) \
    X(256, 4) X(256, 8) X(256, 16) X(512, 2) X(512, 4) X(512, 8) X(1024, 2) X(1024, 4)

bool walk_block_supported(int lanes, int hash_slots) {
#define X(L, Q) if (lanes == L && hash_slots == L * Q) return true;
    MCMI_BLOCK_SHAPES(X)
#undef X
    return false;
}

hipError_t launch_walk_block(const WalkArgs &a, bool f32, int lanes, int blocks, hipStream_t s) {
    const size_t lds = walk_block_lds_bytes(a.hash_slots, a.sketch_slots);
#define X(L, Q)                                                                   \
    if (lanes == L && a.hash_slots == L * Q)                                      \
        return f32 ? launch_one<true, L, Q>(a, blocks, s, lds) : launch_one<false, L, Q>(a, blocks, s, lds);
    MCMI_BLOCK_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t walk_block_occupancy(bool f32, int lanes, int hash_slots, int sketch_slots, int *bpc) {
    const size_t lds = walk_block_lds_bytes(hash_slots, sketch_slots);
#define X(L, Q) \
    if (lanes == L && hash_slots == L * Q) return f32 ? occ_one<true, L, Q>(bpc, lds) : occ_one<false, L, Q>(bpc, lds);
    MCMI_BLOCK_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace mcmi
