// Chain-allocation network: 8 -> 64 -> 64 -> 1 ReLU MLP with BF16 weights,
// FP32 master weights and FP32 accumulation (gfx950).
//
// One wavefront handles a tile of 16 samples. Layer 1 (K = 8) runs on the VALU;
// the 64x64 layer and its two backward products run on the matrix cores with
// v_mfma_f32_16x16x16_bf16 (A: lane l holds row l%16, k = 4(l/16)..+3;
// B: column l%16, k = 4(l/16)..+3; D: column l%16, rows 4(l/16)..+3).
// Training: per-workgroup gradient partials in LDS, a deterministic column
// reduction, then Adam (Kingma and Ba) on the FP32 masters, which are re-rounded
// to BF16 for the next forward. Samples of a training step are drawn with
// replacement by Philox (no host shuffling).
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace mcmi {
namespace {

constexpr int kIn = 8, kHid = 64;
constexpr int oW1 = 0, ob1 = 512, oW2 = 576, ob2 = 4672, ow3 = 4736, ob3 = 4800, kParams = 4801;
constexpr int kTile = 16, kWaves = 4, kWG = kWaves * 64;
constexpr uint32_t kMlpTag = 0x4D4C5000u;

typedef short short4v __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // NaN stays NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

struct MlpArgs {
    const float *feat;      // n x 8
    const float *target;    // n (training)
    const int32_t *idx;     // explicit sample indices (gradient check), nullable
    int64_t n;
    int64_t count;          // samples processed by this launch
    const float *master;    // FP32 parameters
    const uint16_t *w1b, *w2b, *w3b;
    const float *norm;      // mean[8], inv_std[8]
    float *out;             // predictions (inference)
    float *partial;         // gridDim.x x (kParams + 1) gradient partials and loss
    uint64_t seed;
    uint32_t step;
    float inv_batch;
};

template <bool kTrain>
__global__ void __launch_bounds__(kWG) k_mlp(MlpArgs a) {
    __shared__ uint16_t w2s[kHid * kHid];
    __shared__ float w1s[kHid * kIn], b1s[kHid], b2s[kHid], w3s[kHid];
    __shared__ float gsh[kTrain ? kParams + 1 : 1];
    __shared__ uint16_t h1t[kWaves][kTile * kHid];   // [sample][in] bf16
    __shared__ uint16_t dzt[kWaves][kTile * kHid];   // [sample][out] bf16
    __shared__ float xt[kWaves][kTile * kIn];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, q = l >> 4, i = l & 15;
    for (int p = tid; p < kHid * kHid; p += kWG) w2s[p] = a.w2b[p];
    for (int p = tid; p < kHid * kIn; p += kWG) w1s[p] = from_bf16(a.w1b[p]);
    for (int p = tid; p < kHid; p += kWG) {
        b1s[p] = a.master[ob1 + p];
        b2s[p] = a.master[ob2 + p];
        w3s[p] = from_bf16(a.w3b[p]);
    }
    if (kTrain)
        for (int p = tid; p < kParams + 1; p += kWG) gsh[p] = 0.f;
    const float b3 = a.master[ob3];
    __syncthreads();

    const int64_t tiles = (a.count + kTile - 1) / kTile;
    for (int64_t tile = (int64_t)blockIdx.x * kWaves + w; tile < tiles; tile += (int64_t)gridDim.x * kWaves) {
        // ---- sample of this lane in the A layout (row i), normalized, BF16-rounded
        const int64_t slot_a = tile * kTile + i;
        const bool valid_a = slot_a < a.count;
        int64_t sa = 0;
        if (valid_a) {
            if (a.idx) {
                sa = a.idx[slot_a];
            } else if (kTrain) {
                const u32x4 rnd = philox4x32_10(a.step, (uint32_t)slot_a, kMlpTag, 0u, (uint32_t)a.seed,
                                                (uint32_t)(a.seed >> 32));
                sa = (int64_t)(((uint64_t)rnd.x * (uint64_t)a.n) >> 32);
            } else {
                sa = slot_a;
            }
        }
        float xb[kIn];
#pragma unroll
        for (int k = 0; k < kIn; ++k) {
            const float x = valid_a ? a.feat[sa * kIn + k] : 0.f;
            xb[k] = from_bf16(to_bf16((x - a.norm[k]) * a.norm[kIn + k]));
        }
        if (q == 0)
#pragma unroll
            for (int k = 0; k < kIn; ++k) xt[w][i * kIn + k] = xb[k];
        // ---- layer 1 on the VALU, straight into the A operand of layer 2
        short4v A[4];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int o = 16 * kb + 4 * q + r;
                float z = b1s[o];
#pragma unroll
                for (int k = 0; k < kIn; ++k) z += w1s[o * kIn + k] * xb[k];
                const uint16_t hb = to_bf16(z > 0.f ? z : 0.f);
                A[kb][r] = (short)hb;
                h1t[w][i * kHid + o] = hb;
            }
        }
        // ---- layer 2 on the matrix cores: Z2 (16 x 64) = H1 (16 x 64) W2^T
        float4v D[4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            D[nb] = (float4v){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
                const uint16_t *row = &w2s[(16 * nb + i) * kHid + 16 * kb + 4 * q];
                const short4v Bv = (short4v){(short)row[0], (short)row[1], (short)row[2], (short)row[3]};
                D[nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A[kb], Bv, D[nb], 0, 0, 0);
            }
        }
        // D[nb][r] = z2[sample 4q + r][out 16 nb + i]
        float h2[4][4], part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            const int o = 16 * nb + i;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float z = D[nb][r] + b2s[o];
                h2[nb][r] = z > 0.f ? z : 0.f;
                part[r] += w3s[o] * h2[nb][r];
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) part[r] += __shfl_xor(part[r], off, 64);
        }
        float y[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) y[r] = part[r] + b3;
        if (!kTrain) {
            if (i == 0) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t sl = tile * kTile + 4 * q + r;
                    if (sl < a.count) a.out[a.idx ? a.idx[sl] : sl] = y[r];
                }
            }
            continue;
        }
        // ---- backward
        float dy[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t sl = tile * kTile + 4 * q + r;
            const int64_t src = __shfl(sa, (int)((4 * q + r) & 15), 64);
            if (sl < a.count) {
                const float diff = y[r] - a.target[src];
                dy[r] = 2.f * diff * a.inv_batch;
                if (i == 0) atomicAdd(&gsh[kParams], diff * diff);
            } else {
                dy[r] = 0.f;
            }
        }
        // dw3, db3, dz2 (D layout), db2
        float dz2[4][4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            const int o = 16 * nb + i;
            float gw3 = 0.f, gb2 = 0.f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                gw3 += dy[r] * h2[nb][r];
                const float d = h2[nb][r] > 0.f ? dy[r] * w3s[o] : 0.f;
                dz2[nb][r] = d;
                gb2 += d;
                dzt[w][(4 * q + r) * kHid + o] = to_bf16(d);
            }
            atomicAdd(&gsh[ow3 + o], gw3);
            atomicAdd(&gsh[ob2 + o], gb2);
        }
        {
            // db3 = sum of dy over the tile's 16 samples (lanes i == 0 hold 4 each)
            float s = 0.f;
            if (i == 0)
#pragma unroll
                for (int r = 0; r < 4; ++r) s += dy[r];
            if (i == 0) atomicAdd(&gsh[ob3], s);
        }
        wave_sync();
        // dW2 (64 x 64) = dZ2^T H1: A = dZ2^T tile (this lane's D values), B = H1 tile from LDS
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            const short4v Av = (short4v){(short)to_bf16(dz2[nb][0]), (short)to_bf16(dz2[nb][1]),
                                         (short)to_bf16(dz2[nb][2]), (short)to_bf16(dz2[nb][3])};
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
                const short4v Bv = (short4v){(short)h1t[w][(4 * q + 0) * kHid + 16 * kb + i],
                                             (short)h1t[w][(4 * q + 1) * kHid + 16 * kb + i],
                                             (short)h1t[w][(4 * q + 2) * kHid + 16 * kb + i],
                                             (short)h1t[w][(4 * q + 3) * kHid + 16 * kb + i]};
                const float4v G = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(Av, Bv, (float4v){0.f, 0.f, 0.f, 0.f},
                                                                             0, 0, 0);
#pragma unroll
                for (int r = 0; r < 4; ++r) atomicAdd(&gsh[oW2 + (16 * nb + 4 * q + r) * kHid + 16 * kb + i], G[r]);
            }
        }
        // dH1 (16 x 64) = dZ2 (16 x 64) W2: A = dZ2 tile from LDS, B = W2 rows from LDS
        short4v Ad[4];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
            for (int r = 0; r < 4; ++r) Ad[kb][r] = (short)dzt[w][i * kHid + 16 * kb + 4 * q + r];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            float4v E = (float4v){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
                const short4v Bv = (short4v){(short)w2s[(16 * kb + 4 * q + 0) * kHid + 16 * nb + i],
                                             (short)w2s[(16 * kb + 4 * q + 1) * kHid + 16 * nb + i],
                                             (short)w2s[(16 * kb + 4 * q + 2) * kHid + 16 * nb + i],
                                             (short)w2s[(16 * kb + 4 * q + 3) * kHid + 16 * nb + i]};
                E = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(Ad[kb], Bv, E, 0, 0, 0);
            }
            // E[r] = dh1[sample 4q + r][in 16 nb + i]; ReLU mask from the stored H1
            const int o = 16 * nb + i;
            float gb1 = 0.f, gw1[kIn];
#pragma unroll
            for (int k = 0; k < kIn; ++k) gw1[k] = 0.f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int s = 4 * q + r;
                const float dz1 = from_bf16(h1t[w][s * kHid + o]) > 0.f ? E[r] : 0.f;
                gb1 += dz1;
#pragma unroll
                for (int k = 0; k < kIn; ++k) gw1[k] += dz1 * xt[w][s * kIn + k];
            }
            atomicAdd(&gsh[ob1 + o], gb1);
#pragma unroll
            for (int k = 0; k < kIn; ++k) atomicAdd(&gsh[oW1 + o * kIn + k], gw1[k]);
        }
        wave_sync();
    }
    if (kTrain) {
        __syncthreads();
        float *dst = a.partial + (size_t)blockIdx.x * (kParams + 1);
        for (int p = tid; p < kParams + 1; p += kWG) dst[p] = gsh[p];
    }
}

// grad[p] = sum over workgroups of the partials (fixed order), loss slot too
__global__ void __launch_bounds__(256) k_mlp_reduce(const float *partial, int nwg, float *grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kParams) return;
    float s = 0.f;
    for (int g = 0; g < nwg; ++g) s += partial[(size_t)g * (kParams + 1) + p];
    grad[p] = s;
}

__global__ void __launch_bounds__(256) k_adam(float *master, float *m, float *v, const float *grad, uint16_t *w1b,
                                             uint16_t *w2b, uint16_t *w3b, float lr, float beta1, float beta2,
                                             float eps, float bc1, float bc2, float *loss_slot, float inv_batch) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0 && loss_slot) *loss_slot = grad[kParams] * inv_batch;
    if (p >= kParams) return;
    const float g = grad[p];
    const float mm = beta1 * m[p] + (1.f - beta1) * g;
    const float vv = beta2 * v[p] + (1.f - beta2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float th = master[p] - lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
    master[p] = th;
    if (p < ob1) w1b[p - oW1] = to_bf16(th);
    else if (p >= oW2 && p < ob2) w2b[p - oW2] = to_bf16(th);
    else if (p >= ow3 && p < ob3) w3b[p - ow3] = to_bf16(th);
}

__global__ void __launch_bounds__(256) k_round_weights(const float *master, uint16_t *w1b, uint16_t *w2b,
                                                       uint16_t *w3b) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < 512) w1b[p] = to_bf16(master[oW1 + p]);
    if (p < 4096) w2b[p] = to_bf16(master[oW2 + p]);
    if (p < 64) w3b[p] = to_bf16(master[ow3 + p]);
}

// mean and 1/std of each feature column (population std; 1 when the column is constant)
__global__ void __launch_bounds__(256) k_feature_stats(const float *feat, int64_t n, float *norm) {
    __shared__ double red[2][256];
    const int k = blockIdx.x;  // one block per feature
    double s = 0.0, s2 = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += 256) {
        const double x = feat[r * kIn + k];
        s += x;
        s2 += x * x;
    }
    red[0][threadIdx.x] = s;
    red[1][threadIdx.x] = s2;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            red[0][threadIdx.x] += red[0][threadIdx.x + off];
            red[1][threadIdx.x] += red[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double mean = red[0][0] / (double)n;
        const double var = red[1][0] / (double)n - mean * mean;
        norm[k] = (float)mean;
        norm[kIn + k] = var > 1e-12 ? (float)(1.0 / sqrt(var)) : 1.f;
    }
}

}  // namespace
}  // namespace mcmi

using namespace mcmi;

struct mcmi_mlp {
    float *master = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *norm = nullptr, *partial = nullptr;
    uint16_t *w1b = nullptr, *w2b = nullptr, *w3b = nullptr;
    int partial_rows = 0;
    int64_t t = 0;
};

namespace {

mcmi_status mlp_alloc_partial(mcmi_mlp *net, int rows) {
    if (rows <= net->partial_rows) return MCMI_OK;
    (void)hipFree(net->partial);
    net->partial = nullptr;
    MCMI_HIP(hipMalloc(&net->partial, (size_t)rows * (kParams + 1) * sizeof(float)));
    net->partial_rows = rows;
    return MCMI_OK;
}

int mlp_grid(int64_t count) {
    const int64_t tiles = (count + kTile - 1) / kTile;
    int64_t blocks = (tiles + kWaves - 1) / kWaves;
    const int64_t cap = (int64_t)device_cus() * 4;
    if (blocks > cap) blocks = cap;
    return (int)std::max<int64_t>(blocks, 1);
}

MlpArgs mlp_args(const mcmi_mlp *net) {
    MlpArgs a;
    memset(&a, 0, sizeof(a));
    a.master = net->master;
    a.w1b = net->w1b;
    a.w2b = net->w2b;
    a.w3b = net->w3b;
    a.norm = net->norm;
    return a;
}

}  // namespace

extern "C" mcmi_status mcmi_mlp_create(mcmi_mlp **out) {
    if (!out) return fail(MCMI_ERR_ARG, "mcmi_mlp_create: null argument");
    *out = nullptr;
    mcmi_mlp *net = new mcmi_mlp();
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMalloc(&net->master, kParams * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&net->m, kParams * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&net->v, kParams * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&net->grad, (kParams + 1) * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&net->norm, 2 * kIn * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&net->w1b, 512 * sizeof(uint16_t));
    if (e == hipSuccess) e = hipMalloc(&net->w2b, 4096 * sizeof(uint16_t));
    if (e == hipSuccess) e = hipMalloc(&net->w3b, 64 * sizeof(uint16_t));
    if (e == hipSuccess) e = hipMemset(net->master, 0, kParams * sizeof(float));
    if (e == hipSuccess) e = hipMemset(net->m, 0, kParams * sizeof(float));
    if (e == hipSuccess) e = hipMemset(net->v, 0, kParams * sizeof(float));
    if (e != hipSuccess) {
        mcmi_mlp_free(net);
        return fail(MCMI_ERR_HIP, std::string("mcmi_mlp_create: ") + hipGetErrorString(e));
    }
    std::vector<float> nm(2 * kIn, 0.f);
    for (int k = 0; k < kIn; ++k) nm[kIn + k] = 1.f;
    if (hipMemcpy(net->norm, nm.data(), nm.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
        mcmi_mlp_free(net);
        return fail(MCMI_ERR_HIP, "mcmi_mlp_create: copy");
    }
    *out = net;
    return MCMI_OK;
}

extern "C" void mcmi_mlp_free(mcmi_mlp *net) {
    if (!net) return;
    (void)hipFree(net->master);
    (void)hipFree(net->m);
    (void)hipFree(net->v);
    (void)hipFree(net->grad);
    (void)hipFree(net->norm);
    (void)hipFree(net->partial);
    (void)hipFree(net->w1b);
    (void)hipFree(net->w2b);
    (void)hipFree(net->w3b);
    delete net;
}

extern "C" mcmi_status mcmi_mlp_set_params(mcmi_mlp *net, const float *params_host, const float *norm_host,
                                           int32_t reset_optimizer) {
    if (!net || !params_host) return fail(MCMI_ERR_ARG, "mcmi_mlp_set_params: null argument");
    MCMI_HIP(hipMemcpy(net->master, params_host, kParams * sizeof(float), hipMemcpyHostToDevice));
    if (norm_host) MCMI_HIP(hipMemcpy(net->norm, norm_host, 2 * kIn * sizeof(float), hipMemcpyHostToDevice));
    if (reset_optimizer) {
        MCMI_HIP(hipMemset(net->m, 0, kParams * sizeof(float)));
        MCMI_HIP(hipMemset(net->v, 0, kParams * sizeof(float)));
        net->t = 0;
    }
    k_round_weights<<<16, 256>>>(net->master, net->w1b, net->w2b, net->w3b);
    MCMI_HIP(hipGetLastError());
    MCMI_HIP(hipDeviceSynchronize());
    return MCMI_OK;
}

extern "C" mcmi_status mcmi_mlp_get_params(const mcmi_mlp *net, float *params_host, float *norm_host,
                                           float *adam_m_host, float *adam_v_host, int64_t *adam_step) {
    if (!net) return fail(MCMI_ERR_ARG, "mcmi_mlp_get_params: null argument");
    MCMI_HIP(hipDeviceSynchronize());
    if (params_host) MCMI_HIP(hipMemcpy(params_host, net->master, kParams * sizeof(float), hipMemcpyDeviceToHost));
    if (norm_host) MCMI_HIP(hipMemcpy(norm_host, net->norm, 2 * kIn * sizeof(float), hipMemcpyDeviceToHost));
    if (adam_m_host) MCMI_HIP(hipMemcpy(adam_m_host, net->m, kParams * sizeof(float), hipMemcpyDeviceToHost));
    if (adam_v_host) MCMI_HIP(hipMemcpy(adam_v_host, net->v, kParams * sizeof(float), hipMemcpyDeviceToHost));
    if (adam_step) *adam_step = net->t;
    return MCMI_OK;
}

extern "C" mcmi_status mcmi_mlp_set_adam_state(mcmi_mlp *net, const float *adam_m_host, const float *adam_v_host,
                                               int64_t adam_step) {
    if (!net || !adam_m_host || !adam_v_host || adam_step < 0)
        return fail(MCMI_ERR_ARG, "mcmi_mlp_set_adam_state: bad argument");
    MCMI_HIP(hipMemcpy(net->m, adam_m_host, kParams * sizeof(float), hipMemcpyHostToDevice));
    MCMI_HIP(hipMemcpy(net->v, adam_v_host, kParams * sizeof(float), hipMemcpyHostToDevice));
    net->t = adam_step;
    return MCMI_OK;
}

extern "C" mcmi_status mcmi_mlp_fit_normalization(mcmi_mlp *net, const float *feat_dev, int64_t n, void *stream) {
    if (!net || !feat_dev || n < 1) return fail(MCMI_ERR_ARG, "mcmi_mlp_fit_normalization: bad argument");
    k_feature_stats<<<kIn, 256, 0, (hipStream_t)stream>>>(feat_dev, n, net->norm);
    MCMI_HIP(hipGetLastError());
    return MCMI_OK;
}

extern "C" mcmi_status mcmi_mlp_predict(const mcmi_mlp *net, const float *feat_dev, int64_t n, float *out_dev,
                                        void *stream) {
    if (!net || !feat_dev || !out_dev || n < 0) return fail(MCMI_ERR_ARG, "mcmi_mlp_predict: bad argument");
    if (n == 0) return MCMI_OK;
    MlpArgs a = mlp_args(net);
    a.feat = feat_dev;
    a.n = n;
    a.count = n;
    a.out = out_dev;
    k_mlp<false><<<mlp_grid(n), kWG, 0, (hipStream_t)stream>>>(a);
    MCMI_HIP(hipGetLastError());
    return MCMI_OK;
}

extern "C" mcmi_status mcmi_mlp_gradient(mcmi_mlp *net, const float *feat_dev, const float *target_dev,
                                         const int32_t *idx_dev, int64_t batch, int64_t n, float *grad_host,
                                         float *loss_host, void *stream) {
    if (!net || !feat_dev || !target_dev || !idx_dev || batch < 1 || n < 1)
        return fail(MCMI_ERR_ARG, "mcmi_mlp_gradient: bad argument");
    hipStream_t s = (hipStream_t)stream;
    const int grid = mlp_grid(batch);
    mcmi_status st = mlp_alloc_partial(net, grid);
    if (st != MCMI_OK) return st;
    MlpArgs a = mlp_args(net);
    a.feat = feat_dev;
    a.target = target_dev;
    a.idx = idx_dev;
    a.n = n;
    a.count = batch;
    a.partial = net->partial;
    a.inv_batch = 1.f / (float)batch;
    k_mlp<true><<<grid, kWG, 0, s>>>(a);
    MCMI_HIP(hipGetLastError());
    k_mlp_reduce<<<(kParams + 1 + 255) / 256, 256, 0, s>>>(net->partial, grid, net->grad);
    MCMI_HIP(hipGetLastError());
    float tmp[kParams + 1];
    MCMI_HIP(hipMemcpyAsync(tmp, net->grad, (kParams + 1) * sizeof(float), hipMemcpyDeviceToHost, s));
    MCMI_HIP(hipStreamSynchronize(s));
    if (grad_host) memcpy(grad_host, tmp, kParams * sizeof(float));
    if (loss_host) *loss_host = tmp[kParams] / (float)batch;
    return MCMI_OK;
}

extern "C" mcmi_status mcmi_mlp_train(mcmi_mlp *net, const float *feat_dev, const float *target_dev, int64_t n,
                                      int32_t steps, int32_t batch, float lr, uint64_t seed, float *loss_host,
                                      void *stream) {
    if (!net || !feat_dev || !target_dev || n < 1 || steps < 0 || batch < 1 || !(lr > 0.f))
        return fail(MCMI_ERR_ARG, "mcmi_mlp_train: bad argument");
    hipStream_t s = (hipStream_t)stream;
    const int grid = mlp_grid(batch);
    mcmi_status st = mlp_alloc_partial(net, grid);
    if (st != MCMI_OK) return st;
    float *losses = nullptr;
    MCMI_HIP(hipMallocAsync((void **)&losses, (size_t)std::max(steps, 1) * sizeof(float), s));
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (int32_t k = 0; k < steps; ++k) {
        MlpArgs a = mlp_args(net);
        a.feat = feat_dev;
        a.target = target_dev;
        a.n = n;
        a.count = batch;
        a.partial = net->partial;
        a.seed = seed;
        a.step = (uint32_t)(net->t + 1);
        a.inv_batch = 1.f / (float)batch;
        k_mlp<true><<<grid, kWG, 0, s>>>(a);
        k_mlp_reduce<<<(kParams + 1 + 255) / 256, 256, 0, s>>>(net->partial, grid, net->grad);
        net->t += 1;
        const float bc1 = 1.f - powf(b1, (float)net->t), bc2 = 1.f - powf(b2, (float)net->t);
        k_adam<<<(kParams + 255) / 256, 256, 0, s>>>(net->master, net->m, net->v, net->grad, net->w1b, net->w2b,
                                                     net->w3b, lr, b1, b2, eps, bc1, bc2, losses + k,
                                                     1.f / (float)batch);
    }
    MCMI_HIP(hipGetLastError());
    if (loss_host && steps > 0)
        MCMI_HIP(hipMemcpyAsync(loss_host, losses, (size_t)steps * sizeof(float), hipMemcpyDeviceToHost, s));
    MCMI_HIP(hipFreeAsync(losses, s));
    MCMI_HIP(hipStreamSynchronize(s));
    return MCMI_OK;
}

extern "C" mcmi_status mcmi_mlp_adam_step(mcmi_mlp *net, const float *grad_dev, float lr, void *stream) {
    if (!net || !grad_dev || !(lr > 0.f)) return fail(MCMI_ERR_ARG, "mcmi_mlp_adam_step: bad argument");
    hipStream_t s = (hipStream_t)stream;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    net->t += 1;
    const float bc1 = 1.f - powf(b1, (float)net->t), bc2 = 1.f - powf(b2, (float)net->t);
    k_adam<<<(kParams + 255) / 256, 256, 0, s>>>(net->master, net->m, net->v, grad_dev, net->w1b, net->w2b,
                                                 net->w3b, lr, b1, b2, eps, bc1, bc2, nullptr, 0.f);
    MCMI_HIP(hipGetLastError());
    return MCMI_OK;
}

// ------------------------------------------------------------ allocation
// N_r = max(1, rint(lambda * exp(pred_r))) with lambda found by bisection so that
// sum_r N_r cost_r is the largest total not above the budget: hi doubles from 1
// while total(hi) <= budget (and hi < 1e30), then 100 halvings of [0, hi] keep
// total(lo) <= budget < total(hi); lambda = lo. Every total is an exact integer
// sum, so the grid-wide evaluation below (one pass over the rows per step, the
// step's decision taken on the device, no host round trip) makes the same
// decisions as a sequential loop. Non-finite predictions fall back to the
// uniform allocation N_r = max(1, floor(budget / sum_r cost_r)).
namespace mcmi {
namespace {

struct AllocState {
    double lo, hi;
    long long total;  // of the current candidate
    long long bad;    // non-finite predictions
    long long csum;   // sum of costs
    int32_t phase;    // 0: doubling hi, 1: halving, 2: done
    int32_t halvings;
};

__device__ __forceinline__ long long block_sum_ll(long long v, long long *red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) red[w] = v;
    __syncthreads();
    long long t = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += red[k];
    __syncthreads();
    return t;
}

__device__ __forceinline__ long long chains_of(double lam, double e) {
    double k = rint(lam * e);
    if (!(k >= 1.0)) k = 1.0;
    if (k > 2147483647.0) k = 2147483647.0;
    return (long long)k;
}

__global__ void __launch_bounds__(256) k_alloc_prep(const float *pred, const int32_t *cost, int64_t n, double *e,
                                                    AllocState *st) {
    __shared__ long long red[4];
    long long bad = 0, csum = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
        const float p = pred[r];
        bad += isfinite(p) ? 0 : 1;
        e[r] = exp((double)p);
        csum += cost[r];
    }
    bad = block_sum_ll(bad, red);
    csum = block_sum_ll(csum, red);
    if (threadIdx.x == 0) {
        if (bad) atomicAdd((unsigned long long *)&st->bad, (unsigned long long)bad);
        atomicAdd((unsigned long long *)&st->csum, (unsigned long long)csum);
    }
}

// total(candidate) into st->total; the candidate is hi while doubling, else the midpoint
__global__ void __launch_bounds__(256) k_alloc_total(const double *e, const int32_t *cost, int64_t n,
                                                     AllocState *st) {
    __shared__ long long red[4];
    const int32_t phase = st->phase;
    if (phase == 2) return;
    const double lam = phase == 0 ? st->hi : 0.5 * (st->lo + st->hi);
    long long t = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride)
        t += chains_of(lam, e[r]) * (long long)cost[r];
    t = block_sum_ll(t, red);
    if (threadIdx.x == 0) atomicAdd((unsigned long long *)&st->total, (unsigned long long)t);
}

// the step's decision (one thread)
__global__ void k_alloc_update(AllocState *st, long long budget) {
    if (st->phase == 0) {
        if (st->total <= budget && st->hi < 1e30)
            st->hi *= 2.0;
        else
            st->phase = 1;
    } else if (st->phase == 1) {
        const double mid = 0.5 * (st->lo + st->hi);
        if (st->total <= budget)
            st->lo = mid;
        else
            st->hi = mid;
        if (++st->halvings == 100) st->phase = 2;
    }
    st->total = 0;
}

__global__ void __launch_bounds__(256) k_alloc_write(const double *e, int64_t n, long long budget,
                                                     const AllocState *st, int32_t *chains, double *lam_out,
                                                     int32_t *fallback_out) {
    const bool fb0 = st->bad > 0 || st->csum <= 0;
    const double lam = fb0 ? 0.0 : st->lo;
    const bool fb = fb0 || !(lam > 0.0);
    const long long csum = st->csum;
    const long long uni = csum > 0 ? (budget / csum > 1 ? budget / csum : 1) : 1;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride)
        chains[r] = fb ? (int32_t)(uni < 2147483647LL ? uni : 2147483647LL) : (int32_t)chains_of(lam, e[r]);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *lam_out = lam;
        *fallback_out = fb ? 1 : 0;
    }
}

// the bisection's starting state, written on the device (the no-allocation
// variant clears its static workspace with this instead of a host copy)
__global__ void k_alloc_init(AllocState *st) {
    if (threadIdx.x == 0) {
        st->lo = 0.0;
        st->hi = 1.0;
        st->total = 0;
        st->bad = 0;
        st->csum = 0;
        st->phase = 0;
        st->halvings = 0;
    }
}

// Workspace of mcmi_allocate_noalloc: the bisection state, the lambda and
// fallback slots, then exp(pred_r) for up to kNoAllocMaxRows rows.
constexpr int64_t kNoAllocMaxRows = int64_t(1) << 22;
constexpr size_t kNoAllocHead = 256;
constexpr size_t kNoAllocBytes = kNoAllocHead + (size_t)kNoAllocMaxRows * sizeof(double);
static_assert(sizeof(AllocState) <= 64, "state slot");

}  // namespace
}  // namespace mcmi

// Static workspace (one copy per GPU, alive until the process ends). Host code
// never passes this name to a kernel: it uses the device address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[mcmi::kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
hipError_t scratch_address(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}
}  // namespace

extern "C" mcmi_status mcmi_allocate(const float *pred_dev, const int32_t *cost_dev, int64_t n, int64_t budget,
                                     int32_t *chains_dev, double *lambda_host, int32_t *fallback_host,
                                     void *stream) {
    if (!pred_dev || !cost_dev || !chains_dev || n < 1 || budget < 1)
        return fail(MCMI_ERR_ARG, "mcmi_allocate: bad argument");
    hipStream_t s = (hipStream_t)stream;
    double *e = nullptr, *lam = nullptr;
    int32_t *fbk = nullptr;
    AllocState *st = nullptr;
    MCMI_HIP(dev_alloc((void **)&e, (size_t)n * sizeof(double), s));
    MCMI_HIP(dev_alloc((void **)&lam, sizeof(double) + sizeof(int32_t) * 2 + sizeof(AllocState), s));
    fbk = (int32_t *)(lam + 1);
    st = (AllocState *)(fbk + 2);
    const AllocState init{0.0, 1.0, 0, 0, 0, 0, 0};
    int64_t blocks = (n + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    hipError_t err = hipMemcpyAsync(st, &init, sizeof(init), hipMemcpyHostToDevice, s);
    if (err == hipSuccess) {
        k_alloc_prep<<<(unsigned)blocks, 256, 0, s>>>(pred_dev, cost_dev, n, e, st);
        err = hipGetLastError();
    }
    // at most 101 doublings (hi reaches 2^100 > 1e30) and exactly 100 halvings;
    // steps after the search has ended return at once
    for (int it = 0; err == hipSuccess && it < 201; ++it) {
        k_alloc_total<<<(unsigned)blocks, 256, 0, s>>>(e, cost_dev, n, st);
        k_alloc_update<<<1, 1, 0, s>>>(st, (long long)budget);
        err = hipGetLastError();
    }
    if (err == hipSuccess) {
        k_alloc_write<<<(unsigned)blocks, 256, 0, s>>>(e, n, (long long)budget, st, chains_dev, lam, fbk);
        err = hipGetLastError();
    }
    double hl = 0.0;
    int32_t hf = 0;
    if (err == hipSuccess) err = hipMemcpyAsync(&hl, lam, sizeof(double), hipMemcpyDeviceToHost, s);
    if (err == hipSuccess) err = hipMemcpyAsync(&hf, fbk, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    dev_release(e, s);
    dev_release(lam, s);
    if (err != hipSuccess) return fail(MCMI_ERR_HIP, std::string("mcmi_allocate: ") + hipGetErrorString(err));
    if (lambda_host) *lambda_host = hl;
    if (fallback_host) *fallback_host = hf;
    return MCMI_OK;
}

extern "C" mcmi_status mcmi_allocate_noalloc(const float *pred_dev, const int32_t *cost_dev, int64_t n,
                                             int64_t budget, int32_t *chains_dev, double *lambda_dev,
                                             int32_t *fallback_dev, void *stream) {
    using namespace mcmi;
    if (!pred_dev || !cost_dev || !chains_dev || n < 1 || budget < 1)
        return fail(MCMI_ERR_ARG, "mcmi_allocate_noalloc: bad argument");
    if (n > kNoAllocMaxRows)
        return fail(MCMI_ERR_ARG, "mcmi_allocate_noalloc: n = " + std::to_string(n) +
                                      " rows exceeds the static workspace (" + std::to_string(kNoAllocMaxRows) +
                                      " rows); use mcmi_allocate");
    void *base = nullptr;
    hipError_t err = scratch_address(&base);
    if (err != hipSuccess)
        return fail(MCMI_ERR_HIP, std::string("mcmi_allocate_noalloc: workspace address: ") + hipGetErrorString(err));
    hipStream_t s = (hipStream_t)stream;
    unsigned char *head = (unsigned char *)base;
    AllocState *st = (AllocState *)head;
    double *lam = (double *)(head + 64);
    int32_t *fbk = (int32_t *)(head + 72);
    double *e = (double *)(head + kNoAllocHead);
    int64_t blocks = (n + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    k_alloc_init<<<1, 64, 0, s>>>(st);
    k_alloc_prep<<<(unsigned)blocks, 256, 0, s>>>(pred_dev, cost_dev, n, e, st);
    for (int it = 0; it < 201; ++it) {
        k_alloc_total<<<(unsigned)blocks, 256, 0, s>>>(e, cost_dev, n, st);
        k_alloc_update<<<1, 1, 0, s>>>(st, (long long)budget);
    }
    k_alloc_write<<<(unsigned)blocks, 256, 0, s>>>(e, n, (long long)budget, st, chains_dev,
                                                   lambda_dev ? lambda_dev : lam, fallback_dev ? fallback_dev : fbk);
    err = hipGetLastError();
    if (err != hipSuccess) return fail(MCMI_ERR_HIP, std::string("mcmi_allocate_noalloc: ") + hipGetErrorString(err));
    return MCMI_OK;
}
