// Monte Carlo walks, per-row accumulation and finalize (gfx950).
//
// Section III-A, eq. (2): row r of (I - C)^-1 is estimated by the mean over N_r
// chains started at r of sum_j W_j e_{s_j}, with W_0 = 1 and
// W_j = W_{j-1} * c_{s_{j-1} s_j} / p_{s_{j-1} s_j} = W_{j-1} * sign * Shat.
// Section IV-A, phase 4 scales column c by 1 / d_c, and the filter keeps the
// diagonal and every entry with |N_rc| >= eps.
//
// Design (one wavefront owns one row at a time, or 64 / G rows of G lanes each when
// rows have few chains; persistent grid):
//  * rows come from eight work queues, one per XCD (workgroups are dispatched
//    round-robin over the XCDs, so blockIdx % 8 picks the XCD), each a contiguous
//    slice of the rows so that neighbouring rows share their L2; a wave whose
//    queue is empty steals from the next queue;
//  * each lane runs one chain at a time and starts the row's next unstarted chain
//    as soon as its chain stops, so short and long chains do not wait for each
//    other;
//  * a step draws one Philox word and reads the 64-byte alias bucket it names,
//    which also carries the next state's header: one random line per step;
//  * contributions go to an open-addressing hash per row in LDS (key = column,
//    value = float64 sum, LDS float64 atomics; the wave's table split among its
//    rows); a full neighbourhood spills to a per-row share of the wave's HBM hash;
//  * the rows of a wave start together and are finalized one after the other;
//  * at the end of the row the wave filters the slots with a ballot, compacts the
//    survivors in place, scales them by 1 / d_c, sorts them by column with a
//    bitonic network in LDS and appends them to an output pool.
#include "common.hpp"
#include "walk_args.hpp"
#include "walk_common.hpp"

namespace mcmi {

namespace {

using namespace walkdev;

// Wave-uniform task fetch from the eight per-XCD queues.
// Rows are taken from the XCD queues kTaskChunk at a time (one atomic per chunk);
// [lo, hi) is the wave's current chunk. The chunk sets the locality of an XCD's
// rows in flight (about chunk x its wavefronts consecutive rows of the schedule)
// against the atomics on the queue counters: on the 160^3 27-point walk chunks of
// 2, 3, 4, 8 and 16 rows took 63.0, 61.9, 61.7, 62.2 and 71.5 ms.
constexpr int kTaskChunk = 4;

// Compare-exchange of a bitonic pass: a keeps the smaller word of an ascending
// pair (up), the larger of a descending one.
__device__ __forceinline__ void exch(uint64_t &a, uint64_t &b, bool up) {
    const uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
    a = up ? lo : hi;
    b = up ? hi : lo;
}

__device__ __forceinline__ int64_t next_task(const WalkArgs &a, int &queue, int64_t &lo, int64_t &hi) {
    if (lo < hi) return lo++;
    const int lane = lane_id();
    int64_t clo = -1, chi = -1;
    if (lane == 0) {
        for (int tries = 0; tries < 8; ++tries) {
            const int q = (queue + tries) & 7;
            const int64_t qlo = a.n_tasks * q / 8, qhi = a.n_tasks * (q + 1) / 8;
            if (qhi > qlo && __atomic_load_n(&a.queue_ctr[q * kQueueStride], __ATOMIC_RELAXED) < (uint32_t)(qhi - qlo)) {
                const uint32_t idx = atomicAdd(&a.queue_ctr[q * kQueueStride], (uint32_t)kTaskChunk);
                if ((int64_t)idx < qhi - qlo) {
                    clo = qlo + idx;
                    chi = qlo + (int64_t)idx + kTaskChunk < qhi ? qlo + (int64_t)idx + kTaskChunk : qhi;
                    queue = q;
                    break;
                }
            }
        }
    }
    clo = __shfl(clo, 0, 64);
    chi = __shfl(chi, 0, 64);
    queue = __shfl(queue, 0, 64);
    if (clo < 0) return -1;
    lo = clo + 1;
    hi = chi;
    return clo;
}

// A row's ids, record offset and header, loaded ahead of its walk: row_ids issues
// the offset load, row_hdr (later, once that has arrived) the header load.
struct RowPre {
    int64_t task, slot;
    int32_t r, N;
    uint32_t r_off;
    StepHdr h0;
};

__device__ __forceinline__ void row_ids(const WalkArgs &a, int64_t task, RowPre &p) {
    p.task = task;
    if (task < 0) return;
    p.slot = a.task_map ? (int64_t)a.task_map[task] : task;
    p.r = a.rows ? a.rows[p.slot] : (int32_t)p.slot;
    p.N = a.chains_per_row ? a.chains_per_row[p.r] : a.chains;
    p.r_off = a.roff[p.r];
}

template <bool kF32, bool kCmp>
__device__ __forceinline__ void row_hdr(const WalkArgs &a, RowPre &p) {
    if (p.task < 0) return;
    if (kCmp)
        load_header_c(a.rec32, p.r_off, p.h0);
    else
        load_header<kF32>(a.rec, p.r_off, p.h0);
}

// One chain of a lane: its index in the row, state, weight and Philox block.
struct ChainSt {
    int32_t c;
    bool active;
    uint32_t off, j;
    double w64;
    float w32;
    StepHdr H;
    u32x4 blk;
    int32_t pk[4];  // the home bucket of the next contribution's key, read ahead
    uint32_t pb;
};

// One step of a chain: stop (and start the lane's next chain of the row, `stride`
// further on) or draw the next state, and add the current state's weight (j > 0).
// The next bucket's loads go out first; the weight's accumulation (from the copy of
// its key's home bucket read at the end of the previous step) and the Philox
// block of the next four steps run while they are in flight. `blk` holds the
// words of the chain's next draws (step j + 1 takes word j mod 4 of block j / 4).
template <bool kF32, bool kCmp>
__device__ __forceinline__ void chain_step(const WalkArgs &a, ChainSt &ch, int stride, int32_t N, uint32_t r_off,
                                           const StepHdr &H0, uint32_t prow, uint32_t ptag, uint32_t k0, uint32_t k1,
                                           int32_t *gkeys, double *gvals, uint32_t hmask, int hshift, int32_t *gskeys,
                                           double *gsvals, int32_t *gsused, int *gspill, uint32_t smask,
                                           unsigned long long &trans, unsigned long long &spilled, bool &spill_full) {
    const uint4 h = ch.H.h0;  // row, m, W, Shat32
    const double s64 = kF32 ? 0.0 : header_shat64(ch.H);
    const double wcur = kF32 ? (double)ch.w32 : ch.w64;
    bool stop = (h.y == 0u) || (ch.j >= (uint32_t)a.lmax);
    double wn64 = 0.0;
    float wn32 = 0.0f;
    if (kF32) {
        wn32 = ch.w32 * __uint_as_float(h.w);
        stop = stop || (fabsf(wn32) < a.delta32);
    } else {
        wn64 = ch.w64 * s64;
        stop = stop || (fabs(wn64) < a.delta);
    }
    BucketLd bl;
    if (!stop) {
        const uint32_t u = ch.blk.x;
        ch.blk.x = ch.blk.y;
        ch.blk.y = ch.blk.z;
        ch.blk.z = ch.blk.w;
        if (kCmp)
            bucket_issue_c(a.rec32, ch.off, ch.H, u, bl);
        else
            bucket_issue<kF32>(a.rec, ch.off, ch.H, u, bl);
        // the last word of the block went to this draw: the next block now
        if ((ch.j & 3u) == 3u) ch.blk = philox4x32_10((ch.j + 1u) >> 2, (uint32_t)ch.c, prow, ptag, k0, k1);
    }
    if (ch.j > 0) {
        const int32_t key = (int32_t)h.x;  // the row, or its compact record offset
        if (!lds_add_pre(gkeys, gvals, hmask, ch.pb, ch.pk, key, wcur)) {
            ++spilled;
            if (!spill_add_window(gskeys, gsvals, gsused, gspill, smask, key, wcur)) spill_full = true;
        }
    }
    if (stop) {
        trans += ch.j;
        ch.c += stride;
        if (ch.c < N) {
            ch.off = r_off;
            ch.H = H0;
            ch.j = 0;
            ch.w64 = 1.0;
            ch.w32 = 1.0f;
            ch.blk = philox4x32_10(0u, (uint32_t)ch.c, prow, ptag, k0, k1);
        } else {
            ch.active = false;
        }
    } else {
        StepHdr Nx;
        const uint32_t tgt = kCmp ? bucket_resolve_c(bl, Nx) : bucket_resolve<kF32>(bl, Nx);
        const bool neg = (tgt & kSignBit) != 0u;
        if (kF32)
            ch.w32 = neg ? -wn32 : wn32;
        else
            ch.w64 = neg ? -wn64 : wn64;
        ch.off = tgt & ~kSignBit;
        ch.H = Nx;
        ++ch.j;
        // the next step adds this state's weight: its key's home bucket is read
        // now, so that the read has a whole bucket load's latency to complete
        ch.pb = hash_key((int32_t)Nx.h0.x, hshift) & ~3u;
        read_bucket_wave(gkeys, ch.pb, ch.pk);
    }
}

// The 64 / kG rows of one wave (one per group of kG lanes; cur and nxt hold each
// lane's own group's row); each lane keeps kC of its row's chains in flight.
template <bool kF32, int kG, int kC, bool kCmp>
__device__ __forceinline__ void walk_rows(const WalkArgs &a, const RowPre &cur, RowPre &nxt, int &queue, int64_t &tlo,
                         int64_t &thi, int32_t *keys, double *vals, int *spill_cnt,
                         int32_t *skeys, double *svals, int32_t *sused, uint32_t k0, uint32_t k1,
                         unsigned long long &pcur, unsigned long long &pend, unsigned long long *wstats) {
    constexpr int P = 64 / kG;  // rows per wave
    constexpr int kLogP = P == 1 ? 0 : P == 2 ? 1 : P == 4 ? 2 : 3;
    const int lane = lane_id();
    const int grp = lane / kG;
    const int sub = lane & (kG - 1);
    const int Hg = a.hash_slots / P;  // slots per row
    const int hshift = a.hash_shift + kLogP;
    const uint32_t hmask = (uint32_t)Hg - 1u;
    const int Sg = a.spill_slots / P;
    const uint32_t smask = (uint32_t)Sg - 1u;
    int32_t *gkeys = keys + grp * Hg;
    double *gvals = vals + grp * Hg;
    int32_t *gskeys = skeys + (size_t)grp * Sg;
    double *gsvals = svals + (size_t)grp * Sg;
    int32_t *gsused = sused + (size_t)grp * Sg;
    const bool has = cur.task >= 0;
    const int32_t r = has ? cur.r : 0;
    const int32_t N = has ? cur.N : 0;
    const uint32_t r_off = has ? cur.r_off : 0u;
    uint32_t prow = 0, ptag = 0;
    if (has) philox_ids(a, r, prow, ptag);

    // j = 0: every chain contributes W_0 = 1 at (r, r); N ones sum exactly to N.
    // Keys are rows, or record offsets with compact records (turned into rows once
    // the kept set is known).
    const int32_t rkey = kCmp ? (int32_t)r_off : r;
    if (sub == 0 && has) lds_add<true>(gkeys, gvals, hmask, hash_key(rkey, hshift), rkey, (double)N);
    wave_sync();

    // the row's own header (every chain starts there, loaded ahead); later
    // states' headers arrive with the bucket of the step that reaches them
    const StepHdr H0 = cur.h0;
    ChainSt ch[kC];
#pragma unroll
    for (int k = 0; k < kC; ++k) {
        ch[k].c = sub + k * kG;
        ch[k].active = has && ch[k].c < N;
        ch[k].off = r_off;
        ch[k].j = 0;
        ch[k].w64 = 1.0;
        ch[k].w32 = 1.0f;
        ch[k].H = H0;
        ch[k].blk = ch[k].active ? philox4x32_10(0u, (uint32_t)ch[k].c, prow, ptag, k0, k1) : u32x4{0, 0, 0, 0};
    }
    unsigned long long trans = 0, spilled = 0;
    bool spill_full = false;

    while (true) {
        bool any = false;
#pragma unroll
        for (int k = 0; k < kC; ++k) any |= ch[k].active;
        if (!__any(any)) break;
#pragma unroll
        for (int k = 0; k < kC; ++k)
            if (ch[k].active)
                chain_step<kF32, kCmp>(a, ch[k], kG * kC, N, r_off, H0, prow, ptag, k0, k1, gkeys, gvals, hmask, hshift,
                                 gskeys, gsvals, gsused, spill_cnt + grp, smask, trans, spilled, spill_full);
    }
    wave_sync();
    // the next rows' ids and record offsets load now, their headers during the
    // finalize: both latencies hide behind these rows' finalize
#pragma unroll
    for (int g = 0; g < P; ++g) {
        const int64_t t = next_task(a, queue, tlo, thi);
        if (grp == g) row_ids(a, t, nxt);
    }

    // ---------------------------------------------------------- finalize, row by row
    bool hdr_issued = false;
#pragma unroll 1
    for (int g = 0; g < P; ++g) {
        if (__shfl((int)has, g * kG, 64) == 0) continue;  // no row in this group
        const int32_t rg = __shfl(r, g * kG, 64);
        const int32_t kg = kCmp ? __shfl(rkey, g * kG, 64) : rg;  // the row's own key
        const int32_t Ng = __shfl(N, g * kG, 64);
        const int64_t slot = (int64_t)(((uint64_t)(uint32_t)__shfl((int)(cur.slot >> 32), g * kG, 64) << 32) |
                                       (uint32_t)__shfl((int)(uint32_t)cur.slot, g * kG, 64));
        int32_t *tk = keys + g * Hg;
        double *tv = vals + g * Hg;
        int32_t *tsk = skeys + (size_t)g * Sg;
        double *tsv = svals + (size_t)g * Sg;
        const int32_t *tsu = sused + (size_t)g * Sg;
        const double nd = (double)Ng;
        // The eps test needs N_rc = fl(acc / N) only near the cutoff: |acc| above
        // hi = fl(fl(eps N) (1 + 2^-50)) gives fl(acc / N) >= eps for certain, below lo
        // = fl(fl(eps N) (1 - 2^-50)) gives < eps; in between (and for the M filter or
        // eps = 0) the quotient itself decides. Survivors keep acc until the kept set
        // is known.
        const bool exact = a.filter_m || !(a.eps > 0.0);
        const double en = a.eps * nd;
        const double hi = en * (1.0 + 0x1p-50), lo = en * (1.0 - 0x1p-50);
        auto keep_test = [&](int32_t key, double acc) -> bool {
            const double aa = fabs(acc);
            if (key == kg || (!exact && aa > hi)) return true;
            if (!exact && !(aa >= lo)) return false;
            const double nhat = acc / nd;
            const double test =
                a.filter_m ? fabs(nhat / (kCmp ? diag_of_c(a.rec32, (uint32_t)key) : a.diag[key])) : fabs(nhat);
            return nhat != 0.0 && test >= a.eps;
        };
        int K = 0;
        for (int base = 0; base < Hg; base += 64) {
            const int s = base + lane;
            int32_t key = kEmpty;
            double acc = 0.0;
            if (s < Hg) {
                key = tk[s];
                acc = tv[s];
            }
            const bool keep = key != kEmpty && keep_test(key, acc);
            const uint64_t km = ballot(keep);
            wave_sync();
            if (keep) {
                const int pos = K + mask_rank(km);
                tk[pos] = key;
                tv[pos] = acc;
            }
            K += __popcll(km);
        }
        wave_sync();
        if (!hdr_issued) {
            row_hdr<kF32, kCmp>(a, nxt);
            hdr_issued = true;
        }
        const int nsp = spill_cnt[g];
        bool stage_full = false;
        for (int base = 0; base < nsp; base += 64) {
            const int u = base + lane;
            bool keep = false;
            int32_t key = kEmpty;
            double acc = 0.0;
            if (u < nsp) {
                const int32_t sl = tsu[u];
                key = tsk[sl];
                acc = tsv[sl];
                keep = keep_test(key, acc);
                tsk[sl] = kEmpty;
                tsv[sl] = 0.0;
            }
            const uint64_t km = ballot(keep);
            if (keep) {
                const int pos = K + mask_rank(km);
                if (pos < Hg) {
                    tk[pos] = key;
                    tv[pos] = acc;
                } else {
                    stage_full = true;
                }
            }
            K += __popcll(km);
        }
        if (K > Hg) K = Hg;
        wave_sync();
        // the survivors: record offsets -> rows (compact records: row and d from the
        // header unit, loaded together), N_rc = acc / N, and without top-k at once
        // M_rc = N_rc / d_c; four entries per lane in flight
        const bool scale_now = a.topk <= 0;
        // Compact records: record offsets order like the rows they start, so the
        // survivors (up to 256, no top-k) are sorted by their keys while the loads
        // of their rows and d_c are in flight; the rows and M_rc = (acc / N) / d_c
        // replace the keys and sums after the sort.
        int PS0 = 1;
        while (PS0 < K) PS0 <<= 1;
        const bool early = kCmp && scale_now && K <= 256 && K + PS0 <= Hg;
        int32_t erw[4];
        double ed[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            erw[q] = 0;
            ed[q] = 1.0;
        }
        if (early) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = lane + 64 * q;
                if (i < K) {
                    const uint32_t *h = a.rec32 + (size_t)(uint32_t)tk[i] * kUnitWords32;
                    erw[q] = (int32_t)h[0];
                    ed[q] = *(const double *)(h + 6);
                }
            }
        } else {
            for (int i0 = lane; i0 < K; i0 += 256) {
                int32_t rw[4];
                double d[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = i0 + 64 * q;
                    rw[q] = i < K ? tk[i] : 0;
                    d[q] = 1.0;
                    if (i < K) {
                        if (kCmp) {
                            const uint32_t *h = a.rec32 + (size_t)(uint32_t)rw[q] * kUnitWords32;
                            rw[q] = (int32_t)h[0];
                            if (scale_now) d[q] = *(const double *)(h + 6);
                        } else if (scale_now) {
                            d[q] = a.diag[rw[q]];
                        }
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = i0 + 64 * q;
                    if (i < K) {
                        const double nhat = tv[i] / nd;
                        tk[i] = rw[q];
                        tv[i] = scale_now ? nhat / d[q] : nhat;
                    }
                }
            }
            wave_sync();

            // top-k retention: bitonic sort in retention order, keep the first topk,
            // then turn N_rc into M_rc = N_rc / d_c
            if (!scale_now) {
                if (K > a.topk) {
                    int PT = 1;
                    while (PT < K) PT <<= 1;
                    for (int s = K + lane; s < PT; s += 64) tk[s] = INT32_MAX;
                    wave_sync();
                    for (int k = 2; k <= PT; k <<= 1) {
                        for (int jj = k >> 1; jj > 0; jj >>= 1) {
                            for (int pr = lane; pr < (PT >> 1); pr += 64) {
                                const int i = ((pr & ~(jj - 1)) << 1) | (pr & (jj - 1));
                                const int ixj = i | jj;
                                const int32_t ka = tk[i], kb = tk[ixj];
                                const double va = tv[i], vb = tv[ixj];
                                if (top_after(a, rg, ka, va, kb, vb) == ((i & k) == 0)) {
                                    tk[i] = kb;
                                    tk[ixj] = ka;
                                    tv[i] = vb;
                                    tv[ixj] = va;
                                }
                            }
                            wave_sync();
                        }
                    }
                    K = a.topk;
                }
                for (int i0 = lane; i0 < K; i0 += 256) {
                    double d[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) d[q] = i0 + 64 * q < K ? a.diag[tk[i0 + 64 * q]] : 1.0;
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (i0 + 64 * q < K) tv[i0 + 64 * q] = tv[i0 + 64 * q] / d[q];
                }
                wave_sync();
            }
        }

        // Bitonic sort by column (on the early path by record offset, which orders
        // the same way). A pass has PS / 2 compare-exchange pairs, pair p
        // joining i (p with a zero bit inserted at jj) and i | jj, so every lane has a
        // pair. When the value slots past the survivors have room, the sort moves
        // one word per entry, (column << 13) | position, in that free part of the
        // value table, and the values stay where they are; otherwise it moves
        // (column, value) pairs, padding with INT32_MAX.
        int PS = 1;
        while (PS < K) PS <<= 1;
        const bool packed = K + PS <= Hg;
        uint64_t *pk = (uint64_t *)(tv + (Hg - PS));
        if (packed) {
            for (int s = lane; s < PS; s += 64) pk[s] = s < K ? ((uint64_t)(uint32_t)tk[s] << 13) | (uint64_t)s : ~0ull;
            wave_sync();
            for (int k = 2; k <= PS; k <<= 1) {
                int jj = k >> 1;
                // two passes per LDS round trip: a lane takes the four words b, b + h,
                // b + jj, b + jj + h (h = jj / 2; b with bits h and jj clear) and
                // applies the exchanges at distance jj, then at distance h
                for (; jj >= 2; jj >>= 2) {
                    const int h = jj >> 1;
                    const int ph = __builtin_ctz((unsigned)h);
                    for (int g = lane; g < (PS >> 2); g += 64) {
                        const int b = ((g >> ph) << (ph + 2)) | (g & (h - 1));
                        const bool up = (b & k) == 0;
                        uint64_t e0 = pk[b], e1 = pk[b + h], e2 = pk[b + jj], e3 = pk[b + jj + h];
                        exch(e0, e2, up);
                        exch(e1, e3, up);
                        exch(e0, e1, up);
                        exch(e2, e3, up);
                        pk[b] = e0;
                        pk[b + h] = e1;
                        pk[b + jj] = e2;
                        pk[b + jj + h] = e3;
                    }
                    wave_sync();
                }
                if (jj == 1) {
                    for (int pr = lane; pr < (PS >> 1); pr += 64) {
                        const int i = pr << 1;
                        uint64_t ea = pk[i], eb = pk[i + 1];
                        exch(ea, eb, (i & k) == 0);
                        pk[i] = ea;
                        pk[i + 1] = eb;
                    }
                    wave_sync();
                }
            }
        } else {
            for (int s = K + lane; s < PS; s += 64) tk[s] = INT32_MAX;
            wave_sync();
            for (int k = 2; k <= PS; k <<= 1) {
                for (int jj = k >> 1; jj > 0; jj >>= 1) {
                    for (int pr = lane; pr < (PS >> 1); pr += 64) {
                        const int i = ((pr & ~(jj - 1)) << 1) | (pr & (jj - 1));
                        const int ixj = i | jj;
                        const int32_t ka = tk[i], kb = tk[ixj];
                        const bool up = (i & k) == 0;
                        if ((ka > kb) == up) {
                            const double va = tv[i], vb = tv[ixj];
                            tk[i] = kb;
                            tk[ixj] = ka;
                            tv[i] = vb;
                            tv[ixj] = va;
                        }
                    }
                    wave_sync();
                }
            }
        }

        if (early) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = lane + 64 * q;
                if (i < K) {
                    const double nhat = tv[i] / nd;
                    tk[i] = erw[q];
                    tv[i] = nhat / ed[q];
                }
            }
            wave_sync();
        }

        // append to the pool unless a table overflowed for this row (then it is rerun)
        const bool row_spill_full = __any(spill_full && grp == g);
        const bool row_stage_full = __any(stage_full);
        unsigned long long pos0 = 0;
        if (lane == 0 && !row_spill_full && !row_stage_full) {
            if (a.pool_chunk > 0) {
                // the wave's reservation: one global atomic per pool_chunk entries
                if (pcur + (unsigned long long)K > pend) {
                    const unsigned long long grab = (unsigned long long)(K > a.pool_chunk ? K : a.pool_chunk);
                    pcur = atomicAdd(a.pool_used, grab);
                    pend = pcur + grab;
                }
                pos0 = pcur;
                pcur += (unsigned long long)K;
            } else {
                pos0 = atomicAdd(a.pool_used, (unsigned long long)K);
            }
        }
        pos0 = __shfl(pos0, 0, 64);
        const bool fits = (int64_t)(pos0 + (unsigned long long)K) <= a.pool_cap;
        const bool ok = fits && !row_spill_full && !row_stage_full;
        if (ok) {
            for (int i = lane; i < K; i += 64) {
                if (packed) {
                    const uint64_t e = pk[i];
                    a.pool_col[pos0 + i] = tk[e & 8191u];
                    a.pool_val[pos0 + i] = tv[e & 8191u];
                } else {
                    a.pool_col[pos0 + i] = tk[i];
                    a.pool_val[pos0 + i] = tv[i];
                }
            }
        }
        const unsigned long long tg = wave_sum(grp == g ? trans : 0ull);
        const unsigned long long sg = wave_sum(grp == g ? spilled : 0ull);
        if (lane == 0) {
            a.row_start[slot] = ok ? ((int64_t)pos0 | a.pool_tag) : -1;
            a.row_cnt[slot] = (uint32_t)K;
            uint32_t f = 0;
            if (!fits && !row_spill_full && !row_stage_full) f |= kFlagPool;
            if (row_spill_full) f |= kFlagSpill;
            if (row_stage_full) f |= kFlagStage;
            if (f) atomicOr(a.flags, f);
            if (ok) {
                wstats[0] += tg;
                wstats[2] += (unsigned long long)Ng;
            }
            wstats[1] += sg;
        }
        // clear this row's table for the next row of its group
        wave_sync();
        for (int s = lane; s < Hg; s += 64) {
            tk[s] = kEmpty;
            tv[s] = 0.0;
        }
        if (lane == 0) spill_cnt[g] = 0;
        wave_sync();
    }
    if (!hdr_issued) row_hdr<kF32, kCmp>(a, nxt);
}

template <bool kF32, int kG, int kC, bool kCmp>
__global__ void __launch_bounds__(256) k_walk(WalkArgs a) {
    constexpr int P = 64 / kG;
    extern __shared__ __align__(16) unsigned char smem[];
    const int waves = blockDim.x >> 6;
    const int w = threadIdx.x >> 6;
    const int lane = lane_id();
    const int H = a.hash_slots;
    // per wave: vals[H] (f64), keys[H] (i32), one spill counter per row (64 bytes)
    const size_t per_wave = (size_t)H * 12u + 64u;
    unsigned char *mine = smem + (size_t)w * per_wave;
    double *vals = (double *)mine;
    int32_t *keys = (int32_t *)(mine + (size_t)H * 8u);
    int *spill_cnt = (int *)(mine + (size_t)H * 12u);
    for (int s = lane; s < H; s += 64) {
        keys[s] = kEmpty;
        vals[s] = 0.0;
    }
    if (lane < P) spill_cnt[lane] = 0;
    wave_sync();
    const int64_t gw = (int64_t)blockIdx.x * waves + w;
    int32_t *skeys = a.spill_keys + gw * a.spill_slots;
    double *svals = a.spill_vals + gw * a.spill_slots;
    int32_t *sused = a.spill_used + gw * a.spill_slots;
    int queue = (int)(blockIdx.x & 7u);
    const uint32_t k0 = a.keys_dev ? a.keys_dev[0] : a.key0;
    const uint32_t k1 = a.keys_dev ? a.keys_dev[1] : a.key1;
    unsigned long long pcur = 0, pend = 0, wstats[3] = {0, 0, 0};
    int64_t tlo = 0, thi = 0;
    const int grp = lane / kG;
    RowPre cur;
#pragma unroll
    for (int g = 0; g < P; ++g) {
        const int64_t t = next_task(a, queue, tlo, thi);
        if (grp == g) row_ids(a, t, cur);
    }
    row_hdr<kF32, kCmp>(a, cur);
    while (__any(cur.task >= 0)) {
        RowPre nxt;
        walk_rows<kF32, kG, kC, kCmp>(a, cur, nxt, queue, tlo, thi, keys, vals, spill_cnt, skeys, svals, sused, k0,
                                      k1, pcur, pend, wstats);
        cur = nxt;
    }
    // statistics: one set of atomics per wave
    if (lane == 0) {
        if (wstats[0]) atomicAdd(&a.stats[0], wstats[0]);
        if (wstats[1]) atomicAdd(&a.stats[1], wstats[1]);
        if (wstats[2]) atomicAdd(&a.stats[2], wstats[2]);
    }
}

}  // namespace

size_t walk_lds_bytes(int hash_slots, int waves) { return (size_t)waves * ((size_t)hash_slots * 12u + 64u); }

template <bool kF32, bool kCmp>
hipError_t launch_walk_t(const WalkArgs &a, int blocks, int waves, hipStream_t s) {
    const size_t lds = walk_lds_bytes(a.hash_slots, waves);
    switch (a.row_lanes) {
        case 8: k_walk<kF32, 8, 1, kCmp><<<blocks, waves * 64, lds, s>>>(a); break;
        case 16: k_walk<kF32, 16, 1, kCmp><<<blocks, waves * 64, lds, s>>>(a); break;
        case 32: k_walk<kF32, 32, 1, kCmp><<<blocks, waves * 64, lds, s>>>(a); break;
        default:
            if (a.lane_chains == 2)
                k_walk<kF32, 64, 2, kCmp><<<blocks, waves * 64, lds, s>>>(a);
            else
                k_walk<kF32, 64, 1, kCmp><<<blocks, waves * 64, lds, s>>>(a);
            break;
    }
    return hipGetLastError();
}

// FP32 walks read the compact records, FP64 walks the full ones (which carry Shat64).
hipError_t launch_walk(const WalkArgs &a, bool f32, int blocks, int waves, hipStream_t s) {
    if (a.row_lanes != 0 && a.row_lanes != 8 && a.row_lanes != 16 && a.row_lanes != 32 && a.row_lanes != 64)
        return hipErrorInvalidValue;
    if (a.lane_chains == 2 && a.row_lanes != 0 && a.row_lanes != 64) return hipErrorInvalidValue;
    if (f32 && !a.rec32) return hipErrorInvalidValue;
    return f32 ? launch_walk_t<true, true>(a, blocks, waves, s) : launch_walk_t<false, false>(a, blocks, waves, s);
}

hipError_t walk_occupancy(bool f32, int hash_slots, int waves, int *blocks_per_cu) {
    // the instances differ only in loop bounds; the 64-lane one stands for all
    const size_t lds = walk_lds_bytes(hash_slots, waves);
    if (f32)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_walk<true, 64, 1, true>, waves * 64, lds);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_walk<false, 64, 1, false>, waves * 64, lds);
}

}  // namespace mcmi
