// Per-row inputs of the learned chain allocation (gfx950): row features and
// pilot-run variance.
//
// Features (8 per row, binary32, row-major), with p_ij = w_ij / W_i the
// quantized transition probabilities and S = Shat:
//   f0 = ln max(m_i, 1)      f1 = S_i               f2 = max_j |chat_ij|
//   f3 = sum_j p_ij S_j      f4 = max_j S_j          f5 = sum_j p_ij m_j
//   f6 = |sum_j chat_ij| / S_i (sign balance)        f7 = min(L_max, ln delta / ln S_i)
// (f3..f6 = 0 for an empty row; f7 = L_max when S_i >= 1 and 0 when S_i = 0).
//
// Pilot variance (the per-row target of the allocation): P chains per row on
// their own Philox streams (tag bit 31 set). Each chain's row estimate is the
// sparse vector X_c with X_c[s] = sum of its W_j at s (revisits merged);
// v_r = mean_c ||X_c||^2 - ||mean_c X_c||^2 and len_r = mean transitions per chain.
#include <string.h>

#include <algorithm>
#include <string>

#include "common.hpp"
#include "walk_args.hpp"
#include "walk_common.hpp"

namespace mcmi {

namespace {

using namespace walkdev;

__global__ void __launch_bounds__(256) k_features(int64_t n, const uint32_t *__restrict__ rec,
                                                  const uint32_t *__restrict__ roff, double delta, int lmax,
                                                  float *__restrict__ feat) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t r = wave; r < n; r += nwaves) {
        const uint32_t *recp = rec + (size_t)roff[r] * kUnitWords;
        const uint32_t m = recp[1], W = recp[2];
        const double S = __hiloint2double((int)recp[5], (int)recp[4]);
        double ps = 0.0, pm = 0.0, sgn = 0.0, smax = 0.0;
        uint32_t wmax = 0;
        for (uint32_t k = lane; k < m; k += 64) {
            // bucket k: {T, target, alias target, w}, target's header, alias's header, Shat64s
            const uint4 *e = (const uint4 *)(recp + (size_t)(1u + k) * kUnitWords);
            const uint4 q0 = e[0], q1 = e[1], q3 = e[3];
            const uint32_t w = q0.w;
            const uint32_t tgt = q0.y;
            const double St = __hiloint2double((int)q3.y, (int)q3.x);
            const double mt = (double)q1.y;
            ps += (double)w * St;
            pm += (double)w * mt;
            sgn += (tgt & kSignBit) ? -(double)w : (double)w;
            smax = St > smax ? St : smax;
            wmax = w > wmax ? w : wmax;
        }
        ps = wave_sum(ps);
        pm = wave_sum(pm);
        sgn = wave_sum(sgn);
        smax = wave_max(smax);
        wmax = wave_max(wmax);
        if (lane == 0) {
            float *f = feat + 8 * r;
            const double Wd = (double)W;
            f[0] = (float)log((double)(m > 1u ? m : 1u));
            f[1] = (float)S;
            f[2] = m ? (float)(S * (double)wmax / Wd) : 0.f;
            f[3] = m ? (float)(ps / Wd) : 0.f;
            f[4] = (float)smax;
            f[5] = m ? (float)(pm / Wd) : 0.f;
            f[6] = (m && S > 0.0) ? (float)(fabs(sgn) / Wd) : 0.f;
            double f7;
            if (S > 0.0 && S < 1.0 && delta > 0.0) {
                const double l = log(delta) / log(S);
                f7 = l < (double)lmax ? l : (double)lmax;
            } else {
                f7 = S > 0.0 ? (double)lmax : 0.0;
            }
            f[7] = (float)f7;
        }
    }
}

// One wavefront per row, one chain per lane (with refill). Per lane a list of
// the chain's distinct states in LDS (interleaved by lane), per wave an LDS hash
// for the row mean (spilling to HBM like the walk).
template <bool kF32>
__global__ void __launch_bounds__(64) k_pilot(WalkArgs a, int pilot, int cap, double *__restrict__ var,
                                              double *__restrict__ len) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int H = a.hash_slots;
    double *vals = (double *)smem;
    int32_t *keys = (int32_t *)(smem + (size_t)H * 8u);
    int *spill_cnt = (int *)(smem + (size_t)H * 12u);
    double *lv = (double *)(smem + (size_t)H * 12u + 16u);          // cap x 64
    int32_t *lk = (int32_t *)(smem + (size_t)H * 12u + 16u + (size_t)cap * 64u * 8u);
    const uint32_t hmask = (uint32_t)H - 1u, smask = (uint32_t)a.spill_slots - 1u;
    for (int s = lane; s < H; s += 64) {
        keys[s] = kEmpty;
        vals[s] = 0.0;
    }
    if (lane == 0) *spill_cnt = 0;
    wave_sync();
    int32_t *skeys = a.spill_keys + (int64_t)blockIdx.x * a.spill_slots;
    double *svals = a.spill_vals + (int64_t)blockIdx.x * a.spill_slots;
    int32_t *sused = a.spill_used + (int64_t)blockIdx.x * a.spill_slots;
    int queue = (int)(blockIdx.x & 7u);
    const uint32_t tag = a.tag | 0x80000000u;
    for (;;) {
        int64_t task = -1;
        if (lane == 0) {
            for (int tries = 0; tries < 8; ++tries) {
                const int q = (queue + tries) & 7;
                const int64_t lo = a.n_tasks * q / 8, hi = a.n_tasks * (q + 1) / 8;
                if (hi > lo && __atomic_load_n(&a.queue_ctr[q * kQueueStride], __ATOMIC_RELAXED) < (uint32_t)(hi - lo)) {
                    const uint32_t idx = atomicAdd(&a.queue_ctr[q * kQueueStride], 1u);
                    if ((int64_t)idx < hi - lo) {
                        task = lo + idx;
                        queue = q;
                        break;
                    }
                }
            }
        }
        task = __shfl(task, 0, 64);
        queue = __shfl(queue, 0, 64);
        if (task < 0) break;
        const int32_t r = (int32_t)task;
        const uint32_t r_off = a.roff[r];
        int32_t c = lane;
        bool active = c < pilot;
        uint32_t off = r_off, j = 0;
        double w64 = 1.0;
        float w32 = 1.0f;
        u32x4 blk = {0, 0, 0, 0};
        StepHdr H0;
        load_header<kF32>(a.rec, r_off, H0);
        StepHdr Hd = H0;  // header of the current state
        int nl = 0;
        bool overflow = false, spill_full = false;
        double sq = 0.0;
        unsigned long long steps = 0;
        while (__any(active)) {
            if (active) {
                const uint4 h = Hd.h0;
                const double s64 = kF32 ? 0.0 : header_shat64(Hd);
                // contribution (j = 0 included: the start state gets W_0 = 1)
                const int32_t key = (int32_t)h.x;
                const double w = kF32 ? (double)w32 : w64;
                int e = 0;
                while (e < nl && lk[e * 64 + lane] != key) ++e;
                if (e < nl) {
                    lv[e * 64 + lane] += w;
                } else if (nl < cap) {
                    lk[nl * 64 + lane] = key;
                    lv[nl * 64 + lane] = w;
                    ++nl;
                } else {
                    overflow = true;
                }
                if (!lds_add(keys, vals, hmask, hash_key(key, a.hash_shift), key, w))
                    if (!spill_add(skeys, svals, sused, spill_cnt, smask, key, w)) spill_full = true;
                bool stop = (h.y == 0u) || (j >= (uint32_t)a.lmax);
                double wn64 = 0.0;
                float wn32 = 0.0f;
                if (kF32) {
                    wn32 = w32 * __uint_as_float(h.w);
                    stop = stop || (fabsf(wn32) < a.delta32);
                } else {
                    wn64 = w64 * s64;
                    stop = stop || (fabs(wn64) < a.delta);
                }
                if (stop) {
                    for (int q = 0; q < nl; ++q) sq += lv[q * 64 + lane] * lv[q * 64 + lane];
                    steps += j;
                    nl = 0;
                    c += 64;
                    if (c < pilot) {
                        off = r_off;
                        Hd = H0;
                        j = 0;
                        w64 = 1.0;
                        w32 = 1.0f;
                    } else {
                        active = false;
                    }
                } else {
                    if ((j & 3u) == 0u) blk = philox4x32_10(j >> 2, (uint32_t)c, (uint32_t)r, tag, a.key0, a.key1);
                    const uint32_t u = blk.x;
                    blk.x = blk.y;
                    blk.y = blk.z;
                    blk.z = blk.w;
                    StepHdr Nx;
                    const uint32_t tgt = draw_next<kF32>(a.rec, off, Hd, u, Nx);
                    const bool neg = (tgt & kSignBit) != 0u;
                    if (kF32)
                        w32 = neg ? -wn32 : wn32;
                    else
                        w64 = neg ? -wn64 : wn64;
                    off = tgt & ~kSignBit;
                    Hd = Nx;
                    ++j;
                }
            }
        }
        wave_sync();
        // ||mean||^2 over the row hash and the spilled columns
        const double P = (double)pilot;
        double msq = 0.0;
        for (int s = lane; s < H; s += 64) {
            if (keys[s] != kEmpty) {
                const double mu = vals[s] / P;
                msq += mu * mu;
            }
        }
        const int nsp = *spill_cnt;
        for (int u = lane; u < nsp; u += 64) {
            const int32_t sl = sused[u];
            const double mu = svals[sl] / P;
            msq += mu * mu;
            skeys[sl] = kEmpty;
            svals[sl] = 0.0;
        }
        msq = wave_sum(msq);
        sq = wave_sum(sq);
        steps = wave_sum(steps);
        const bool bad_cap = __any(overflow), bad_spill = __any(spill_full);
        if (lane == 0) {
            var[r] = sq / P - msq;
            len[r] = (double)steps / P;
            if (bad_cap) atomicOr(a.flags, kFlagStage);
            if (bad_spill) atomicOr(a.flags, kFlagSpill);
            atomicAdd(&a.stats[0], steps);
        }
        wave_sync();
        for (int s = lane; s < H; s += 64) {
            keys[s] = kEmpty;
            vals[s] = 0.0;
        }
        if (lane == 0) *spill_cnt = 0;
        wave_sync();
    }
}

// Neyman allocation target of each row: minimising sum_r v_r / N_r under
// sum_r N_r (len_r + 1) = T gives N_r proportional to sqrt(v_r / (len_r + 1)), so
// the network regresses y_r = (ln v_r - ln(len_r + 1)) / 2 (v floored at 1e-30 so
// that rows with a deterministic chain get a finite, very small share).
__global__ void __launch_bounds__(256) k_neyman_target(int64_t n, const double *__restrict__ var,
                                                       const double *__restrict__ len, float *__restrict__ y) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
        const double v = var[r] > 1e-30 ? var[r] : 1e-30;
        y[r] = (float)(0.5 * (log(v) - log(len[r] + 1.0)));
    }
}

// Budget units of one chain of each row: the states it visits when every row on
// its path has the row's own |C| row sum, 1 + floor(f7) (f7 = min(L_max,
// ln delta / ln S), the feature the network also sees); exact for matrices with
// equal row sums. Partial sums of the costs per workgroup, in 64-bit integers.
__global__ void __launch_bounds__(256) k_chain_cost(int64_t n, const float *__restrict__ feat,
                                                    int32_t *__restrict__ cost,
                                                    unsigned long long *__restrict__ total) {
    __shared__ unsigned long long red[4];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long sum = 0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
        const float f7 = feat[8 * r + 7];
        const int32_t c = 1 + (int32_t)floorf(f7 > 0.f ? f7 : 0.f);
        cost[r] = c;
        sum += (unsigned long long)c;
    }
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_down(sum, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(total, red[0] + red[1] + red[2] + red[3]);
}

}  // namespace

hipError_t launch_features(const mcmi_cdf *cdf, double delta, int lmax, float *feat, hipStream_t s) {
    const hipError_t fe = ensure_full_records(cdf, s);
    if (fe != hipSuccess) return fe;
    int64_t blocks = (cdf->n + 3) / 4;
    if (blocks > 16384) blocks = 16384;
    k_features<<<(unsigned)blocks, 256, 0, s>>>(cdf->n, cdf->rec, cdf->roff, delta, lmax, feat);
    return hipGetLastError();
}

size_t pilot_lds_bytes(int hash_slots, int cap) { return (size_t)hash_slots * 12u + 16u + (size_t)cap * 64u * 12u; }

hipError_t launch_pilot(const WalkArgs &a, bool f32, int pilot, int cap, int blocks, double *var, double *len,
                        hipStream_t s) {
    const size_t lds = pilot_lds_bytes(a.hash_slots, cap);
    if (f32)
        k_pilot<true><<<blocks, 64, lds, s>>>(a, pilot, cap, var, len);
    else
        k_pilot<false><<<blocks, 64, lds, s>>>(a, pilot, cap, var, len);
    return hipGetLastError();
}

hipError_t pilot_occupancy(bool f32, int hash_slots, int cap, int *bpc) {
    const size_t lds = pilot_lds_bytes(hash_slots, cap);
    if (f32) return hipOccupancyMaxActiveBlocksPerMultiprocessor(bpc, k_pilot<true>, 64, lds);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(bpc, k_pilot<false>, 64, lds);
}

}  // namespace mcmi

// ------------------------------------------------------------------ C ABI
using namespace mcmi;

extern "C" mcmi_status mcmi_row_features(const mcmi_cdf *cdf, double delta, int32_t max_len, float *feat_dev,
                                         void *stream) {
    if (!cdf || !feat_dev) return fail(MCMI_ERR_ARG, "mcmi_row_features: null argument");
    if (!(delta >= 0.0) || max_len < 0) return fail(MCMI_ERR_ARG, "mcmi_row_features: bad delta / max_len");
    int lmax = derive_lmax(cdf->norm_inf, delta, max_len);
    if (lmax < 0) lmax = max_len;  // not contractive and no max_len: f7 uses 0
    MCMI_HIP(launch_features(cdf, delta, lmax, feat_dev, (hipStream_t)stream));
    return MCMI_OK;
}

extern "C" mcmi_status mcmi_pilot_variance(const mcmi_cdf *cdf, const mcmi_params *p, int32_t pilot_chains,
                                           double *var_dev, double *len_dev, void *stream) {
    if (!cdf || !p || !var_dev || !len_dev) return fail(MCMI_ERR_ARG, "mcmi_pilot_variance: null argument");
    if (pilot_chains < 1) return fail(MCMI_ERR_ARG, "mcmi_pilot_variance: pilot_chains must be >= 1");
    if (p->walk_prec != MCMI_WALK_F64 && p->walk_prec != MCMI_WALK_F32)
        return fail(MCMI_ERR_ARG, "mcmi_pilot_variance: walk_prec must be 64 or 32");
    const int lmax = derive_lmax(cdf->norm_inf, p->delta, p->max_len);
    if (lmax < 0) return fail(lmax == (int)MCMI_ERR_NOT_CONTRACTIVE ? MCMI_ERR_NOT_CONTRACTIVE : MCMI_ERR_ARG,
                              "mcmi_pilot_variance: ||Chat||_inf >= 1 needs max_len, or bad delta");
    hipStream_t s = (hipStream_t)stream;
    const bool f32 = p->walk_prec == MCMI_WALK_F32;
    int H = 1024, cap = lmax + 1 < 48 ? lmax + 1 : 48, spill_slots = 4096;
    unsigned char *ctrl = nullptr;
    int32_t *sk = nullptr, *su = nullptr;
    double *sv = nullptr;
    const size_t ctrl_bytes = kCtrlBytes;
    auto cleanup = [&]() {
        (void)hipFree(ctrl);
        (void)hipFree(sk);
        (void)hipFree(sv);
        (void)hipFree(su);
        ctrl = nullptr;
        sk = su = nullptr;
        sv = nullptr;
    };
    // the pilot walks read the full records: build them before the arguments take their address
    {
        const hipError_t fe = ensure_full_records(cdf, s);
        if (fe != hipSuccess) return fail(MCMI_ERR_HIP, std::string("mcmi_pilot_variance: ") + hipGetErrorString(fe));
    }
    for (int attempt = 0; attempt < 6; ++attempt) {
        int bpc = 0;
        hipError_t e = pilot_occupancy(f32, H, cap, &bpc);
        if (e != hipSuccess || bpc < 1) {
            cleanup();
            return fail(MCMI_ERR_CAPACITY, "mcmi_pilot_variance: per-chain state lists do not fit in LDS");
        }
        const int64_t blocks = std::min<int64_t>((int64_t)bpc * device_cus(), cdf->n);
#define TRYP(call)                                                                              \
    do {                                                                                        \
        hipError_t _e = (call);                                                                 \
        if (_e != hipSuccess) {                                                                 \
            cleanup();                                                                          \
            return fail(MCMI_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(_e));       \
        }                                                                                       \
    } while (0)
        TRYP(hipMalloc(&ctrl, ctrl_bytes));
        TRYP(hipMalloc(&sk, (size_t)blocks * spill_slots * 4));
        TRYP(hipMalloc(&sv, (size_t)blocks * spill_slots * 8));
        TRYP(hipMalloc(&su, (size_t)blocks * spill_slots * 4));
        TRYP(hipMemsetAsync(ctrl, 0, ctrl_bytes, s));
        TRYP(hipMemsetAsync(sk, 0xFF, (size_t)blocks * spill_slots * 4, s));
        TRYP(hipMemsetAsync(sv, 0, (size_t)blocks * spill_slots * 8, s));
        WalkArgs a;
        memset(&a, 0, sizeof(a));
        a.rec = cdf->rec;
        a.roff = cdf->roff;
        a.diag = cdf->diag;
        a.n_tasks = cdf->n;
        a.key0 = (uint32_t)(p->seed & 0xffffffffu);
        a.key1 = (uint32_t)(p->seed >> 32);
        a.tag = p->stream_tag;
        a.delta = p->delta;
        a.delta32 = (float)p->delta;
        a.lmax = lmax;
        a.hash_slots = H;
        a.hash_shift = 32 - __builtin_ctz((unsigned)H);
        a.queue_ctr = (uint32_t *)ctrl;
        a.stats = (unsigned long long *)(ctrl + kCtrlStats);
        a.flags = (uint32_t *)(ctrl + kCtrlFlags);
        a.spill_keys = sk;
        a.spill_vals = sv;
        a.spill_used = su;
        a.spill_slots = spill_slots;
        TRYP(launch_pilot(a, f32, pilot_chains, cap, (int)blocks, var_dev, len_dev, s));
        uint32_t hflags = 0;
        TRYP(hipMemcpyAsync(&hflags, a.flags, sizeof(hflags), hipMemcpyDeviceToHost, s));
        TRYP(hipStreamSynchronize(s));
#undef TRYP
        cleanup();
        if (!(hflags & (kFlagStage | kFlagSpill))) return MCMI_OK;
        if (hflags & kFlagStage) {
            if (cap >= lmax + 1 || cap >= 160) return fail(MCMI_ERR_CAPACITY, "mcmi_pilot_variance: state list overflow");
            cap = cap * 2 < lmax + 1 ? cap * 2 : lmax + 1;
            if (cap > 160) cap = 160;
        }
        if (hflags & kFlagSpill) spill_slots *= 4;
    }
    return fail(MCMI_ERR_CAPACITY, "mcmi_pilot_variance: tables still overflow");
}

extern "C" mcmi_status mcmi_neyman_target(const double *var_dev, const double *len_dev, int64_t n, float *y_dev,
                                          void *stream) {
    if (n < 0 || (n > 0 && (!var_dev || !len_dev || !y_dev)))
        return fail(MCMI_ERR_ARG, "mcmi_neyman_target: bad argument");
    if (n == 0) return MCMI_OK;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    k_neyman_target<<<(unsigned)blocks, 256, 0, (hipStream_t)stream>>>(n, var_dev, len_dev, y_dev);
    MCMI_HIP(hipGetLastError());
    return MCMI_OK;
}

extern "C" mcmi_status mcmi_chain_cost(const float *feat_dev, int64_t n, int32_t *cost_dev, int64_t *total_host,
                                       void *stream) {
    if (n < 0 || (n > 0 && (!feat_dev || !cost_dev)))
        return fail(MCMI_ERR_ARG, "mcmi_chain_cost: bad argument");
    if (total_host) *total_host = 0;
    if (n == 0) return MCMI_OK;
    if (n > (int64_t)INT32_MAX * 4) return fail(MCMI_ERR_ARG, "mcmi_chain_cost: too many rows");
    hipStream_t s = (hipStream_t)stream;
    unsigned long long *tot = nullptr;
    MCMI_HIP(hipMallocAsync((void **)&tot, sizeof(unsigned long long), s));
    hipError_t e = hipMemsetAsync(tot, 0, sizeof(unsigned long long), s);
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    if (e == hipSuccess) {
        k_chain_cost<<<(unsigned)blocks, 256, 0, s>>>(n, feat_dev, cost_dev, tot);
        e = hipGetLastError();
    }
    unsigned long long h = 0;
    if (e == hipSuccess && total_host) e = hipMemcpyAsync(&h, tot, sizeof(h), hipMemcpyDeviceToHost, s);
    const hipError_t ef = hipFreeAsync(tot, s);
    if (e == hipSuccess) e = ef;
    if (e == hipSuccess && total_host) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(MCMI_ERR_HIP, std::string("mcmi_chain_cost: ") + hipGetErrorString(e));
    if (total_host) *total_host = (int64_t)h;
    return MCMI_OK;
}
