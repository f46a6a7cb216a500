// Diagnostics of the macroscopic fields on the device: integrals of a field
// over a window of cells (the integrated heat flux q and shear pressure Pi
// around a discontinuity, Sec. IV B 3, eqs. intq, intpi), the error measure of
// the Sod convergence test (Sec. IV E, eq. eps_def) and the L2 norm of the
// Bjorken convergence test (Sec. V E, eq. bjork_L2).
//
// Inputs are rows of per-cell (or per-sample) fields as rsl_moments writes
// them.  Every reduction runs in one workgroup in a fixed order (a strided
// per-thread pass, then a tree in LDS), so results do not depend on
// scheduling.
#include <hip/hip_runtime.h>

#include "rsl_impl.h"

namespace rsl {

namespace {

constexpr int kDiagThreads = 256;

// Tree reduction of one value per thread (sum or max), result in thread 0.
template <bool MAX>
__device__ double block_reduce(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = kDiagThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const double a = red[threadIdx.x], b = red[threadIdx.x + o];
            red[threadIdx.x] = MAX ? fmax(a, b) : a + b;
        }
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// out[c] = dz sum_{r in [r0, r1)} m[r * ncols + c], c < ncols (midpoint rule over the cells).
__global__ void __launch_bounds__(kDiagThreads) window_integral_kernel(const double* __restrict__ m, int ncols,
                                                                      int r0, int r1, double dz,
                                                                      double* __restrict__ out) {
    __shared__ double red[kDiagThreads];
    for (int c = 0; c < ncols; ++c) {
        double s = 0.0;
        for (int r = r0 + (int)threadIdx.x; r < r1; r += kDiagThreads) s += m[(size_t)r * ncols + c];
        const double tot = block_reduce<false>(s, red);
        if (threadIdx.x == 0) out[c] = dz * tot;
    }
}

// Field of a rsl_moments row used by the convergence tests: n, T, gamma
// (from beta), P, Pi.
enum DiagField { kN = 0, kT = 1, kGamma = 2, kP = 3, kPi = 4 };
__device__ __forceinline__ double diag_field(const double* row, int f) {
    switch (f) {
        case kN: return row[5];
        case kT: return row[8];
        case kGamma: return 1.0 / sqrt((1.0 - row[9]) * (1.0 + row[9]));
        case kP: return row[7];
        default: return row[12];
    }
}

// eps_j = max_z |d_j - d_j,ref| / (max_z d_j - min_z d_j) for d_j = n, T, gamma
// (eq. eps_def as read here: the largest pointwise deviation over the range of
// the profile); out = {eps_n, eps_T, eps_gamma, eps = max_j eps_j}.
__global__ void __launch_bounds__(kDiagThreads) sod_eps_kernel(const double* __restrict__ m,
                                                              const double* __restrict__ ref, int nz,
                                                              double* __restrict__ out) {
    __shared__ double red[kDiagThreads];
    double eps = 0.0;
    for (int f = 0; f < 3; ++f) {
        double dmax = -HUGE_VAL, dmin = HUGE_VAL, dev = 0.0;
        for (int s = threadIdx.x; s < nz; s += kDiagThreads) {
            const double d = diag_field(m + (size_t)s * RSL_NMOM, f);
            const double r = diag_field(ref + (size_t)s * RSL_NMOM, f);
            dmax = fmax(dmax, d);
            dmin = fmin(dmin, d);
            dev = fmax(dev, fabs(d - r));
        }
        dmax = block_reduce<true>(dmax, red);
        dmin = -block_reduce<true>(-dmin, red);
        dev = block_reduce<true>(dev, red);
        const double e = dev / (dmax - dmin);
        if (threadIdx.x == 0) out[f] = e;
        eps = fmax(eps, e);
    }
    if (threadIdx.x == 0) out[3] = eps;
}

// L2(A) = sqrt( int_1^tau_f dtau / (tau_f - 1) [A - A_ref]^2 ) for A = n, T, P,
// Pi from samples at tau = 1 + i dtau, i = 0..ns-1 (trapezoid rule), and
// out[4] = max_A L2(A) (eq. bjork_L2).
__global__ void __launch_bounds__(kDiagThreads) bjorken_l2_kernel(const double* __restrict__ h,
                                                                 const double* __restrict__ ref, int ns,
                                                                 double dtau, double* __restrict__ out) {
    __shared__ double red[kDiagThreads];
    const int fields[4] = {kN, kT, kP, kPi};
    const double span = dtau * (ns - 1);
    double worst = 0.0;
    for (int a = 0; a < 4; ++a) {
        double s = 0.0;
        for (int i = threadIdx.x; i < ns; i += kDiagThreads) {
            const double d = diag_field(h + (size_t)i * RSL_NMOM, fields[a]) -
                             diag_field(ref + (size_t)i * RSL_NMOM, fields[a]);
            const double w = (i == 0 || i == ns - 1) ? 0.5 : 1.0;
            s += w * d * d;
        }
        const double tot = block_reduce<false>(s, red);
        const double l2 = sqrt(tot * dtau / span);
        if (threadIdx.x == 0) out[a] = l2;
        worst = fmax(worst, l2);
    }
    if (threadIdx.x == 0) out[4] = worst;
}

}  // namespace

}  // namespace rsl

using namespace rsl;

extern "C" {

int rsl_window_integral(const double* m_dev, int nrows, int ncols, double dz, int row_lo, int row_hi, double* out_dev,
                        void* hip_stream) {
    if (!m_dev || !out_dev || ncols <= 0 || nrows < 0 || !(dz > 0.0))
        return set_error(RSL_EINVAL, "window integral: bad argument");
    if (row_lo < 0 || row_hi > nrows || row_lo > row_hi) return set_error(RSL_EINVAL, "window integral: bad window");
    hipLaunchKernelGGL(window_integral_kernel, dim3(1), dim3(kDiagThreads), 0, (hipStream_t)hip_stream, m_dev, ncols,
                       row_lo, row_hi, dz, out_dev);
    return hip_check(hipGetLastError(), "window_integral_kernel launch");
}

int rsl_sod_eps(const double* m_dev, const double* ref_dev, int nz, double* out_dev, void* hip_stream) {
    if (!m_dev || !ref_dev || !out_dev || nz < 2) return set_error(RSL_EINVAL, "eps: bad argument");
    hipLaunchKernelGGL(sod_eps_kernel, dim3(1), dim3(kDiagThreads), 0, (hipStream_t)hip_stream, m_dev, ref_dev, nz,
                       out_dev);
    return hip_check(hipGetLastError(), "sod_eps_kernel launch");
}

int rsl_bjorken_l2(const double* hist_dev, const double* ref_dev, int nsamples, double dtau, double* out_dev,
                   void* hip_stream) {
    if (!hist_dev || !ref_dev || !out_dev || nsamples < 2 || !(dtau > 0.0))
        return set_error(RSL_EINVAL, "L2: bad argument");
    hipLaunchKernelGGL(bjorken_l2_kernel, dim3(1), dim3(kDiagThreads), 0, (hipStream_t)hip_stream, hist_dev, ref_dev,
                       nsamples, dtau, out_dev);
    return hip_check(hipGetLastError(), "bjorken_l2_kernel launch");
}

}  // extern "C"
