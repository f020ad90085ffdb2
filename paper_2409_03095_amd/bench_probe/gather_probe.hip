// Dependent random-gather probe (gfx950): the memory ceiling of the walk's
// access pattern without the method's arithmetic. Benchmark tooling, built into
// its own library (libmcmi_probe.so) and loaded only by the benchmark script;
// it is not part of the library's C ABI.
//
// A buffer of `units` 64-byte units is read by a chase in which every step
// issues `reqs` dependent reads of one random unit each, a read being `loads`
// 16-byte loads of the unit's first quarters (1: only the word the next address
// depends on; 4: the whole unit). The next unit is a hash of the word just read,
// the lane and the step, so, like a Markov chain's fresh random numbers, two
// lanes that meet the same unit do not follow each other afterwards (a fixed
// successor per unit would funnel lanes into shared paths that hit in the
// caches). The measured steps per second is the ceiling a walk with the same
// number of dependent random blocks per transition can reach on this chip for a
// record set of the same size.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../csrc/common.hpp"

namespace {

__global__ void k_probe_fill(uint4 *buf, uint64_t units, uint32_t seed) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < units; u += stride) {
        const mcmi::u32x4 r = mcmi::philox4x32_10((uint32_t)u, (uint32_t)(u >> 32), 0x50524F42u, 0u, seed, 0x9E3779B9u);
        const uint32_t next = (uint32_t)(((uint64_t)r.x * units) >> 32);
        uint4 *p = buf + u * 4;
        p[0] = make_uint4(next, r.y, r.z, r.w);
        p[1] = make_uint4(next, 0u, 0u, 0u);
        p[2] = make_uint4(next, 0u, 0u, 0u);
        p[3] = make_uint4(next, 0u, 0u, 0u);
    }
}

typedef unsigned int u32v4 __attribute__((ext_vector_type(4)));

template <bool kNt>
__device__ __forceinline__ uint4 probe_load(const uint4 *p) {
    if (kNt) {
        const u32v4 v = __builtin_nontemporal_load((const u32v4 *)p);
        return make_uint4(v.x, v.y, v.z, v.w);
    }
    return *p;
}

template <bool kNt>
__global__ void __launch_bounds__(256) k_probe_chase(const uint4 *buf, uint64_t units, int reqs, int loads,
                                                     int steps, unsigned long long *sink) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t cur = (uint32_t)((tid * 2654435761ull) % units);
    uint32_t acc = 0;
    for (int s = 0; s < steps; ++s) {
        for (int q = 0; q < reqs; ++q) {
            const uint4 *u = buf + (uint64_t)cur * 4;
            const uint4 v = probe_load<kNt>(u);
            uint32_t extra = 0;
            if (loads > 1) extra += probe_load<kNt>(u + 1).y;
            if (loads > 2) extra += probe_load<kNt>(u + 2).z;
            if (loads > 3) extra += probe_load<kNt>(u + 3).w;
            // next unit: hash of the word read, the lane and the step
            uint32_t h = v.x ^ (uint32_t)tid * 0x9E3779B9u ^ (uint32_t)(s * 4 + q) * 0x85EBCA77u;
            h ^= h >> 16;
            h *= 0x7FEB352Du;
            h ^= h >> 15;
            cur = (uint32_t)(((uint64_t)h * units) >> 32);
            acc += v.y + extra;
        }
    }
    if (acc == 0xFFFFFFFFu) atomicAdd(sink, 1ull);
}

// Uncached device memory is never handed back to the driver once a kernel has
// read it (memory allocated after such a free has been seen to hold wrong
// values): blocks stay for the process and are reused by later probes.
struct KeptBlock {
    void *p;
    size_t bytes;
};
KeptBlock g_uncached[16];
int g_uncached_n = 0;

hipError_t uncached_buffer(size_t bytes, void **out) {
    for (int i = 0; i < g_uncached_n; ++i)
        if (g_uncached[i].bytes >= bytes) {
            *out = g_uncached[i].p;
            return hipSuccess;
        }
    if (g_uncached_n == 16) return hipErrorOutOfMemory;
    void *p = nullptr;
    const hipError_t e = hipExtMallocWithFlags(&p, bytes, hipDeviceMallocUncached);
    if (e != hipSuccess) return e;
    g_uncached[g_uncached_n++] = KeptBlock{p, bytes};
    *out = p;
    return hipSuccess;
}

}  // namespace

// mode 0: ordinary (cached) device memory; 1: the same with non-temporal loads;
// 2: uncached device memory (kept for the process). Returns 0 on success, -1 for
// a bad argument, or the HIP error code.
extern "C" int probe_gather_chase_mode(uint64_t units, int32_t reqs_per_step, int32_t loads_per_req, int32_t steps,
                                       int32_t waves_per_cu, int32_t mode, double *ms_out, double *steps_per_s_out) {
    if (units < 1024 || units >= (1ull << 32) || reqs_per_step < 1 || loads_per_req < 1 || loads_per_req > 4 ||
        steps < 1 || waves_per_cu < 1 || mode < 0 || mode > 2)
        return -1;
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    uint4 *buf = nullptr;
    unsigned long long *sink = nullptr;
    hipError_t e = mode == 2 ? uncached_buffer(units * 64, (void **)&buf) : hipMalloc(&buf, units * 64);
    if (e != hipSuccess) return (int)e;
    e = hipMalloc(&sink, 8);
    if (e != hipSuccess) {
        if (mode != 2) (void)hipFree(buf);
        return (int)e;
    }
    k_probe_fill<<<4096, 256>>>(buf, units, 12345u);
    const int blocks = cus * waves_per_cu / 4;
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    if (mode == 1) {
        k_probe_chase<true><<<blocks, 256>>>(buf, units, reqs_per_step, loads_per_req, steps / 4 + 1, sink);  // warm-up
        (void)hipEventRecord(a, nullptr);
        k_probe_chase<true><<<blocks, 256>>>(buf, units, reqs_per_step, loads_per_req, steps, sink);
    } else {
        k_probe_chase<false><<<blocks, 256>>>(buf, units, reqs_per_step, loads_per_req, steps / 4 + 1, sink);
        (void)hipEventRecord(a, nullptr);
        k_probe_chase<false><<<blocks, 256>>>(buf, units, reqs_per_step, loads_per_req, steps, sink);
    }
    (void)hipEventRecord(b, nullptr);
    e = hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (mode != 2) (void)hipFree(buf);
    (void)hipFree(sink);
    if (e != hipSuccess) return (int)e;
    if (ms_out) *ms_out = ms;
    if (steps_per_s_out) *steps_per_s_out = (double)blocks * 256.0 * (double)steps / (ms * 1e-3);
    return 0;
}

extern "C" int probe_gather_chase(uint64_t units, int32_t reqs_per_step, int32_t loads_per_req, int32_t steps,
                                  int32_t waves_per_cu, double *ms_out, double *steps_per_s_out) {
    return probe_gather_chase_mode(units, reqs_per_step, loads_per_req, steps, waves_per_cu, 0, ms_out,
                                   steps_per_s_out);
}
