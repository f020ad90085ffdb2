// BiCGstab on the device around the sparse approximate inverse (gfx950).
//
// The paper uses M directly as a preconditioner of a Krylov solver (Section III-B,
// last paragraph; the solver experiments of Section VI). This is van der Vorst's
// BiCGstab with M applied on the right (solve B M y = b, x = M y): every step
// applies B and M once per half step (CSR SpMV, 8 lanes per row), reduces dot
// products deterministically (fixed grid, per-workgroup partials summed by one
// workgroup in index order) and updates the vectors in fused elementwise kernels.
// The scalars are read back once per reduction; the iteration stops when the
// recurrence residual satisfies ||r|| <= rtol ||b||.
#include <math.h>
#include <string.h>

#include <string>

#include "common.hpp"

namespace mcmi {
hipError_t spmv(int64_t n, int64_t nnz, const int64_t *rp, const int32_t *ci, const double *v, const double *x,
                double *y, hipStream_t s);

namespace {

constexpr int kDotBlocks = 1024;

__global__ void __launch_bounds__(256) k_dot_partial(int64_t n, const double *__restrict__ a,
                                                     const double *__restrict__ b, double *__restrict__ part) {
    __shared__ double red[4];
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) acc += a[i] * b[i];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void __launch_bounds__(256) k_dot_final(int nb, const double *__restrict__ part, double *__restrict__ out) {
    __shared__ double red[4];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += part[i];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) *out = (red[0] + red[1]) + (red[2] + red[3]);
}

// r = b - y, rhat = r
__global__ void __launch_bounds__(256) k_residual(int64_t n, const double *__restrict__ b,
                                                  const double *__restrict__ y, double *__restrict__ r,
                                                  double *__restrict__ rhat) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double v = b[i] - y[i];
        r[i] = v;
        rhat[i] = v;
    }
}

// p = r + beta (p - omega v)
__global__ void __launch_bounds__(256) k_dir(int64_t n, const double *__restrict__ r, const double *__restrict__ v,
                                             double beta, double omega, double *__restrict__ p) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = r[i] + beta * (p[i] - omega * v[i]);
}

// y = x + a z (in place when y == x)
__global__ void __launch_bounds__(256) k_axpy(int64_t n, const double *__restrict__ x, double a,
                                              const double *__restrict__ z, double *y) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) y[i] = x[i] + a * z[i];
}

// x += alpha phat + omega shat, r = s - omega t
__global__ void __launch_bounds__(256) k_step(int64_t n, double alpha, const double *__restrict__ phat, double omega,
                                              const double *__restrict__ shat, const double *__restrict__ s,
                                              const double *__restrict__ t, double *__restrict__ x,
                                              double *__restrict__ r) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        x[i] = x[i] + alpha * phat[i] + omega * shat[i];
        r[i] = s[i] - omega * t[i];
    }
}

unsigned grid_elem(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    return (unsigned)(b < 1 ? 1 : b);
}

struct Solver {
    int64_t n;
    const mcmi_csr_in *B;
    const mcmi_csr_out *M;
    hipStream_t s;
    double *part = nullptr, *dres = nullptr;

    hipError_t dot(const double *a, const double *b, double *out) {
        k_dot_partial<<<kDotBlocks, 256, 0, s>>>(n, a, b, part);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        k_dot_final<<<1, 256, 0, s>>>(kDotBlocks, part, dres);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(out, dres, sizeof(double), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(s);
    }
    hipError_t applyB(const double *x, double *y) {
        return spmv(n, B->nnz, B->row_ptr_dev, B->col_dev, B->val_dev, x, y, s);
    }
    // y = M x, or a copy without a preconditioner
    hipError_t applyM(const double *x, double *y) {
        if (!M) return hipMemcpyAsync(y, x, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s);
        return spmv(n, M->nnz, M->row_ptr_dev, M->col_dev, M->val_dev, x, y, s);
    }
};

}  // namespace
}  // namespace mcmi

using namespace mcmi;

extern "C" mcmi_status mcmi_bicgstab(const mcmi_csr_in *B, const mcmi_csr_out *M, const double *b_dev, double *x_dev,
                                     double rtol, int32_t maxiter, mcmi_solve_stats *st, void *stream) {
    if (st) ::memset(st, 0, sizeof(*st));
    if (!B || !b_dev || !x_dev || !(rtol > 0.0) || maxiter < 1)
        return fail(MCMI_ERR_ARG, "mcmi_bicgstab: need B, b, x, rtol > 0 and maxiter >= 1");
    if (B->n <= 0 || !B->row_ptr_dev || !B->col_dev || !B->val_dev)
        return fail(MCMI_ERR_ARG, "mcmi_bicgstab: bad B");
    if (M && (M->n != B->n || !M->row_ptr_dev)) return fail(MCMI_ERR_ARG, "mcmi_bicgstab: M must be n x n");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = B->n;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    MCMI_HIP(hipEventCreate(&e0));
    MCMI_HIP(hipEventCreate(&e1));
    double *w = nullptr;
    const size_t vec = (size_t)n * sizeof(double);
    MCMI_HIP(hipMalloc(&w, 8 * vec + (kDotBlocks + 1) * sizeof(double)));
    double *r = w, *rhat = w + n, *p = w + 2 * n, *v = w + 3 * n, *phat = w + 4 * n, *sv = w + 5 * n,
           *shat = w + 6 * n, *t = w + 7 * n;
    Solver S{n, B, M, s, w + 8 * n, w + 8 * n + kDotBlocks};
    mcmi_status status = MCMI_OK;
    std::string why;
    const unsigned g = grid_elem(n);
    int64_t it = 0;
    int converged = 0;
    double bnrm = 0.0, rr = 0.0;
#define STEP(call)                                         \
    do {                                                   \
        hipError_t _e = (call);                            \
        if (_e != hipSuccess) {                            \
            status = MCMI_ERR_HIP;                         \
            why = std::string(#call) + ": " + hipGetErrorString(_e); \
            goto done;                                     \
        }                                                  \
    } while (0)
    STEP(hipEventRecord(e0, s));
    STEP(S.dot(b_dev, b_dev, &bnrm));
    bnrm = sqrt(bnrm);
    STEP(S.applyB(x_dev, v));
    k_residual<<<g, 256, 0, s>>>(n, b_dev, v, r, rhat);
    STEP(hipGetLastError());
    STEP(S.dot(r, r, &rr));
    if (bnrm == 0.0) {
        STEP(hipMemsetAsync(x_dev, 0, vec, s));
        converged = 1;
    } else if (sqrt(rr) <= rtol * bnrm) {
        converged = 1;
    } else {
        double rho_prev = 1.0, alpha = 1.0, omega = 1.0;
        STEP(hipMemsetAsync(p, 0, vec, s));
        STEP(hipMemsetAsync(v, 0, vec, s));
        for (it = 1; it <= maxiter; ++it) {
            double rho = 0.0, rv = 0.0, ss = 0.0, ts = 0.0, tt = 0.0;
            STEP(S.dot(rhat, r, &rho));
            if (rho == 0.0) break;  // breakdown
            const double beta = (rho / rho_prev) * (alpha / omega);
            k_dir<<<g, 256, 0, s>>>(n, r, v, it == 1 ? 0.0 : beta, omega, p);
            STEP(hipGetLastError());
            STEP(S.applyM(p, phat));
            STEP(S.applyB(phat, v));
            STEP(S.dot(rhat, v, &rv));
            if (rv == 0.0) break;
            alpha = rho / rv;
            k_axpy<<<g, 256, 0, s>>>(n, r, -alpha, v, sv);
            STEP(hipGetLastError());
            STEP(S.dot(sv, sv, &ss));
            if (sqrt(ss) <= rtol * bnrm) {
                k_axpy<<<g, 256, 0, s>>>(n, x_dev, alpha, phat, x_dev);
                STEP(hipGetLastError());
                rr = ss;
                converged = 1;
                break;
            }
            STEP(S.applyM(sv, shat));
            STEP(S.applyB(shat, t));
            STEP(S.dot(t, sv, &ts));
            STEP(S.dot(t, t, &tt));
            if (tt == 0.0) break;
            omega = ts / tt;
            k_step<<<g, 256, 0, s>>>(n, alpha, phat, omega, shat, sv, t, x_dev, r);
            STEP(hipGetLastError());
            STEP(S.dot(r, r, &rr));
            if (sqrt(rr) <= rtol * bnrm) {
                converged = 1;
                break;
            }
            if (omega == 0.0) break;
            rho_prev = rho;
        }
        if (it > maxiter) it = maxiter;
    }
    STEP(hipEventRecord(e1, s));
    STEP(hipEventSynchronize(e1));
done:
#undef STEP
    float ms = 0.f;
    if (status == MCMI_OK) (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipStreamSynchronize(s);
    (void)hipFree(w);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status != MCMI_OK) return fail(status, "mcmi_bicgstab: " + why);
    if (st) {
        st->iterations = it;
        st->rel_residual = bnrm > 0.0 ? sqrt(rr) / bnrm : 0.0;
        st->ms = ms;
        st->converged = converged;
    }
    return MCMI_OK;
}
