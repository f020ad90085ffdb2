// Internal header of libmcmi.so (gfx950). Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/mcmi.h"

namespace mcmi {

// ------------------------------------------------------------------ errors
void set_error(const std::string &msg);
mcmi_status fail(mcmi_status st, const std::string &msg);

#define MCMI_HIP(call)                                                                     \
    do {                                                                                   \
        hipError_t _e = (call);                                                            \
        if (_e != hipSuccess)                                                              \
            return ::mcmi::fail(MCMI_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(_e)); \
    } while (0)

// ----------------------------------------------------------- record layout
// One record per row s of C, 64-byte aligned, addressed by its offset in
// 64-byte units (31 bits: up to 128 GiB of records). With m entries (column
// order) it is 1 + m units of 16 words:
//   unit 0    header of s: {row s, m, W = total integer weight, Shat_s as
//             binary32}, {Shat_s as binary64 (2 words), 0, 0}, 8 zero words
//   unit 1+j  bucket j = 0 .. m-1 of the row's alias table:
//             {T_j, target_j, target_{A_j}, w_j},
//             the header words {row, m, W, Shat32} of the row target_j points to,
//             the same for target_{A_j},
//             {Shat64 of target_j (2 words), Shat64 of target_{A_j} (2 words)}
// (T, A) is the alias table (Walker's method in Vose's exact-integer
// construction: bucket j keeps T_j of its W units for entry j and gives the
// rest to entry A_j); a target is the record offset of the column's row with bit
// 31 set when c < 0. A draw with the 32-bit word u takes bucket j = (u m) >> 32
// and r = ((u m mod 2^32) W) >> 32: the next state is target_j if r < T_j, else
// target_{A_j}. Because the bucket carries the next state's header, a transition
// reads one 64-byte block (three 16-byte loads issued together, four with
// binary64 weights): one random line per transition; the header unit is read
// only when a chain starts.
constexpr int kUnitWords = 16;
constexpr uint32_t kSignBit = 0x80000000u;
//
// Compact records (the wavefront kernel's FP32 walks): the same unit offsets in
// units of 32 bytes (8 words), so a row of m entries again takes 1 + m units:
//   unit 0    {row s, m, W, Shat32}, {Shat64 (2 words), d_s (2 words)}
//   unit 1+j  {T'_j, target_j, m of target_j, Shat32 of target_j},
//             {w_j, target_{A_j}, m of target_{A_j}, Shat32 of target_{A_j}}
// with the threshold moved onto the draw's word: the entry is target_j iff
// f < T'_j, where f = u m mod 2^32 and T'_j = ceil(T_j 2^32 / W) (exactly the
// r < T_j test of the full record, as floor(f W / 2^32) < T_j <=> f W < T_j 2^32);
// a bucket that keeps all W units has T'_j = 2^32 - 1 and target_{A_j} =
// target_j, so f = 2^32 - 1 leads to the same state. A draw reads 32 bytes
// (two 16-byte loads) of a record half the size; the state's key in the walk is
// its record offset (unique and increasing with the row), turned into the row at
// the finalize from the header unit.
constexpr int kUnitWords32 = 8;

__host__ __device__ inline uint32_t record_units(uint32_t m) { return 1u + m; }

// Error flags raised by device-side validation (bit set).
enum : uint32_t {
    kFlagCsr = 1u,        // unsorted / duplicate / out-of-range column or bad row_ptr
    kFlagZeroDiag = 2u,   // missing or zero diagonal
    kFlagTooBig = 4u,     // record area above 2^31 units
    kFlagPool = 8u,       // output pool overflow
    kFlagSpill = 16u,     // spill table overflow
    kFlagStage = 32u,     // more survivors than the staging area holds
};
constexpr int kPoolShift = 56;   // row_start = position | (pool index << kPoolShift)
constexpr int kMaxPools = 8;
struct PoolSet {
    const int32_t *col[kMaxPools];
    const double *val[kMaxPools];
};

// ------------------------------------------------------------------ Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds; each round
// takes the 64-bit products of counter words 0 and 2 with two fixed odd
// multipliers and forms the next block from their halves, words 1 and 3 and the
// round key; the key advances by two Weyl increments between rounds.
struct u32x4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ u32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1) {
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        // one 32 x 32 -> 64-bit product per multiplier (both halves from one instruction)
        const uint64_t pA = (uint64_t)kMulA * c0, pB = (uint64_t)kMulB * c2;
        const uint32_t hiA = (uint32_t)(pA >> 32), loA = (uint32_t)pA;
        const uint32_t hiB = (uint32_t)(pB >> 32), loB = (uint32_t)pB;
        const uint32_t n0 = hiB ^ c1 ^ k0;
        const uint32_t n2 = hiA ^ c3 ^ k1;
        c0 = n0;
        c1 = loB;
        c2 = n2;
        c3 = loA;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    return {c0, c1, c2, c3};
}

// ---------------------------------------------------------- wave helpers
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// number of set bits of `mask` below this lane
__device__ __forceinline__ int mask_rank(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        T o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// inclusive prefix sum over the 64 lanes
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        T o = __shfl_up(v, off, 64);
        if (lane >= off) v += o;
    }
    return v;
}

// Shared host helpers (api.hip)
int derive_lmax(double norm_inf, double delta, int max_len);
int device_cus();

// --------------------------------------------------------------- scans
// Exclusive prefix sum of n int64 values (out may alias in); writes the total
// to *total_dev (device). Temporary memory comes from `tmp` (>= scan_tmp_bytes(n)).
size_t scan_tmp_bytes(int64_t n);
hipError_t scan_exclusive_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *total_dev, void *tmp,
                              hipStream_t s);
hipError_t scan_exclusive_u32_to_i64(const uint32_t *in, int64_t *out, int64_t n, int64_t *total_dev, void *tmp,
                                     hipStream_t s);

}  // namespace mcmi

// Kernel shape of a walk launch (api.hip: choose_shape)
struct KernelShape {
    int lanes = 64, hash = 1024, sketch = 0;
    int lane_chains = 1;  // wavefront kernel: chains a lane keeps in flight
    double tau = 0.0;
};
struct mcmi_cdf;
namespace mcmi {
mcmi_status choose_shape(const mcmi_cdf *cdf, const mcmi_params *p, int lmax, int n_max, int n_typ,
                         KernelShape &out);
// Checks shared by every walk launch (api.hip).
mcmi_status check_walk_params(const mcmi_params *p, bool per_row_chains, const char *who);
mcmi_status read_chain_counts(const mcmi_cdf *cdf, const mcmi_params *p, const int32_t *rows_dev, int64_t n_rows,
                              const int32_t *cpr_dev, int &n_max, int &n_typ, hipStream_t s, const char *who);
// Control block of a walk launch. Every counter that wavefronts update with
// device-wide atomics (the eight row queues, the pool position, statistics, flags)
// sits on a 4 KB line of its own: atomics on one cache line are performed one
// after the other, so counters sharing a line would queue behind each other.
constexpr size_t kCtrlLine = 4096;
constexpr int kQueueStride = (int)(kCtrlLine / 4);  // uint32 elements between queue counters
constexpr size_t kCtrlPool = 8 * kCtrlLine;         // u64 pool position
constexpr size_t kCtrlStats = 9 * kCtrlLine;        // u64 stats[4]
constexpr size_t kCtrlFlags = 10 * kCtrlLine;       // u32 flags
constexpr size_t kCtrlCollect = 11 * kCtrlLine;     // u64 collect[2] (failed rows of a pass)
constexpr size_t kCtrlKeys = 12 * kCtrlLine;        // u32 Philox keys (captured plans)
constexpr size_t kCtrlBytes = 13 * kCtrlLine;

// Entries a wavefront of the wavefront kernel reserves in the output pool with one
// atomic: a quarter of the pool spread over the wavefronts, between 256 and 32768.
// The reservation is a device-wide atomic on one counter with a return value the
// wavefront waits for; on the 160^3 27-point walk, chunks of 2048 entries (one
// atomic per 12 rows) cost 3 % of the walk against chunks of 32768.
inline int32_t pool_chunk_for(int64_t pool_cap, int64_t wavefronts) {
    int64_t c = wavefronts > 0 ? pool_cap / (4 * wavefronts) : 32768;
    if (c > 32768) c = 32768;
    if (c < 256) c = 256;
    return (int32_t)c;
}

struct WaveLayout {
    int lanes = 64, rows_per_wave = 1, spill_slots = 0;
};
WaveLayout wave_layout(const KernelShape &shape, int spill_given, int n_max, int lmax);
}

// Full records from the compact ones (cdf.hip), once per record set: every
// consumer other than the FP32 walks of the wavefront kernel calls this first
// (FP64 walks, the workgroup kernel, row features, pilot walks, downloads).
// Synchronises the stream the first time, so that every stream sees them.
namespace mcmi {
hipError_t ensure_full_records(const mcmi_cdf *cdf, hipStream_t s);
}

// Device-memory cache (alloc.hip): dev_alloc reuses a block released on the
// same stream (dev_release, stream-ordered) or released idle (dev_release_idle,
// which synchronises the device first); otherwise it calls hipMalloc.
namespace mcmi {
hipError_t dev_alloc(void **p, size_t bytes, hipStream_t s);
void dev_release(void *p, hipStream_t s);
void dev_release_idle(void *p);
// Locality order of the rows (order.hip): a permutation of [0, n) in `order`.
hipError_t build_locality_order(int64_t n, const int64_t *row_ptr, const int32_t *col, int64_t cell, int32_t *order,
                                hipStream_t s);
}  // namespace mcmi

// The opaque record set.
#include <mutex>
#include <vector>
struct mcmi_cdf {
    int64_t n = 0;
    int64_t nnz_c = 0;
    double norm_inf = 0.0;
    double norm_b = 0.0;    // ||B||_inf when the diagonal was augmented
    double drop_thr = 0.0;  // reduction cut on |c| (0: none)
    int64_t dropped = 0;    // entries of C removed by the reduction
    uint64_t rec_units = 0;
    uint32_t *rec = nullptr;       // full records, 16 words per unit (built on first use)
    uint32_t *rec32 = nullptr;     // compact records, 8 words per unit (same offsets)
    std::mutex full_lock;          // guards the first build of the full records
    uint32_t *roff = nullptr;      // n: record offset (64-byte units) of each row
    double *diag = nullptr;        // n: b_ii
    uint32_t *mrow = nullptr;      // n: entries of each row of C
    int32_t *order = nullptr;      // n: locality order of the rows (null: natural order)
    // batched record sets (several matrices, block-diagonal row space)
    int32_t batch = 0;                   // number of matrices (0: a single matrix)
    int32_t *row_mat = nullptr;          // n: matrix of each row
    int64_t *mat_base = nullptr;         // batch + 1: first row of each matrix (device)
    std::vector<int64_t> mat_base_host;  // same, on the host
    std::vector<double> mat_norm;        // ||Chat_k||_inf per matrix
};
