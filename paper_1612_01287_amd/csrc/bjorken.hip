// Bjorken flow in Milne coordinates (Sec. V): one workgroup integrates one
// instance for all requested steps, with the populations resident in LDS.
//
// L_Bjorken (eq. L_Bjorken):
//   -f_jk/tau + (xi_j^2/tau) sum_k' K^L_{kk'} f_jk' + (1/tau) sum_j' K^P_{jj'} f_j'k
//   - (f_jk - f^eq_jk)/tau_AW,
// with the fluid at rest (u = (1,0,0,0)), so f^eq is the rest-frame expansion
// f^eq_jk = (n_eq/4) w_j w_k [1 + (1 - theta) L_1(pbar_k)], theta = T/T0.
// Ideal gas: n_eq = n = N^tau, T = P/n, tau_AW of eq. bjorken_tauAW_mu (the
// eta/s law with lambda_bar = n/T^3); parton gas: T = P^{1/4}, n_eq = T^3,
// tau_AW = tau_AW0/T (Sec. V D).  RK3 stage times tau_n, tau_n + dtau,
// tau_n + dtau/2 (Table II).
#include <hip/hip_runtime.h>

#include "rsl_math.h"

namespace rsl {

namespace {

constexpr int kBjBlock = 256;

template <typename Tf>
__device__ void bj_moments(const InstDesc& d, const double* f, double* red, double& n, double& E, double& PL) {
    double a = 0.0, b = 0.0, c = 0.0;
    for (int v = threadIdx.x; v < d.V; v += blockDim.x) {
        const int k = v / d.Q, j = v - k * d.Q;
        const double p = d.tab.pk[k], x = d.tab.xi[j];
        a += f[v];
        b += p * f[v];
        c += p * x * x * f[v];
    }
    // block reduction in a fixed order
    red[threadIdx.x] = a;
    red[blockDim.x + threadIdx.x] = b;
    red[2 * blockDim.x + threadIdx.x] = c;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[threadIdx.x] += red[threadIdx.x + h];
            red[blockDim.x + threadIdx.x] += red[blockDim.x + threadIdx.x + h];
            red[2 * blockDim.x + threadIdx.x] += red[2 * blockDim.x + threadIdx.x + h];
        }
        __syncthreads();
    }
    n = red[0];
    E = red[blockDim.x];
    PL = red[2 * blockDim.x];
    __syncthreads();
}

template <typename Tf>
__device__ void bj_L(const InstDesc& d, const double* f, double tau, double* L, double* red, unsigned& bad) {
    double n, E, PL;
    bj_moments<Tf>(d, f, red, n, E, PL);
    const double P = E / 3.0;
    const bool collide = d.tau_mode != RSL_TAU_INF;
    double neq = 1.0, T = 1.0, itaw = 0.0;
    if (collide) {
        if (d.gas == RSL_GAS_IDEAL) {
            if (!(n > 0.0) || !(P > 0.0)) bad |= 1u;
            T = P / n;
            neq = n;
            double taw = d.tau_r;
            if (d.tau_mode == RSL_TAU_ETAS)
                taw = d.tau_aw0 / T * (1.0 - 0.25 * log(n / (T * T * T) * d.lambda_ref));
            itaw = 1.0 / taw;
        } else {
            if (!(P > 0.0)) bad |= 1u;
            T = sqrt(sqrt(P));
            neq = T * T * T;
            itaw = 1.0 / (d.tau_mode == RSL_TAU_ETAS ? d.tau_aw0 / T : d.tau_r);
        }
    }
    const double th1 = 1.0 - T / d.T0, it = 1.0 / tau;
    const int Q = d.Q, QL = d.QL;
    for (int v = threadIdx.x; v < d.V; v += blockDim.x) {
        const int k = v / Q, j = v - k * Q;
        const double x = d.tab.xi[j];
        double sl = 0.0;
        for (int kp = 0; kp < QL; ++kp) sl += d.tab.KL[k * QL + kp] * f[kp * Q + j];
        double sp = 0.0;
        const double* Kr = d.tab.KP + (size_t)j * Q;
        const double* fk = f + k * Q;
        for (int jp = 0; jp < Q; ++jp) sp = fma(Kr[jp], fk[jp], sp);
        double acc = (-f[v] + x * x * sl + sp) * it;
        if (collide) {
            const double feq = d.tab.wxw[v] * 0.25 * neq * (1.0 + th1 * d.tab.L1[k]);
            acc -= (f[v] - feq) * itaw;
        }
        L[v] = acc;
    }
    __syncthreads();
}

template <typename Tf>
__device__ void bj_run(const InstDesc& d, double tau0, double dtau, int nsteps, double* sm) {
    double* f = sm;
    double* f1 = f + d.V;
    double* f2 = f1 + d.V;
    double* L = f2 + d.V;
    double* red = L + d.V;
    Tf* g = (Tf*)d.f;
    for (int v = threadIdx.x; v < d.V; v += blockDim.x) f[v] = (double)g[v];
    __syncthreads();
    unsigned bad = 0;
    for (int it = 0; it < nsteps; ++it) {
        const double t = tau0 + it * dtau;
        bj_L<Tf>(d, f, t, L, red, bad);
        for (int v = threadIdx.x; v < d.V; v += blockDim.x) f1[v] = (double)(Tf)(f[v] + dtau * L[v]);
        __syncthreads();
        bj_L<Tf>(d, f1, t + dtau, L, red, bad);
        for (int v = threadIdx.x; v < d.V; v += blockDim.x)
            f2[v] = (double)(Tf)(0.75 * f[v] + 0.25 * f1[v] + 0.25 * dtau * L[v]);
        __syncthreads();
        bj_L<Tf>(d, f2, t + 0.5 * dtau, L, red, bad);
        for (int v = threadIdx.x; v < d.V; v += blockDim.x)
            f[v] = (double)(Tf)(kThird * f[v] + kTwoThirds * (f2[v] + dtau * L[v]));
        __syncthreads();
    }
    for (int v = threadIdx.x; v < d.V; v += blockDim.x) {
        g[v] = (Tf)f[v];
        if (!isfinite(f[v])) bad |= 2u;
    }
    if (bad) atomicOr(d.status, bad);
}

template <typename Tf>
__global__ void __launch_bounds__(kBjBlock) bj_steps_kernel(InstDesc d, double tau0, double dtau, int nsteps) {
    extern __shared__ double sm[];
    bj_run<Tf>(d, tau0, dtau, nsteps, sm);
}

// Batched Bjorken: one workgroup per instance; each instance keeps its proper
// time in its work area and advances it by nsteps * dt.
template <typename Tf>
__global__ void __launch_bounds__(kBjBlock) bj_batch_steps_kernel(const InstDesc* __restrict__ descs, char* fbase,
                                                                 char* wbase, int nsteps) {
    extern __shared__ double sm[];
    InstDesc d = descs[blockIdx.x];
    rebase(d, fbase, wbase);
    const double tau0 = *d.clock;
    bj_run<Tf>(d, tau0, d.dt, nsteps, sm);
    __syncthreads();
    if (threadIdx.x == 0) *d.clock = tau0 + nsteps * d.dt;
}

template <typename Tf>
__global__ void bj_init_kernel(InstDesc d, double n0, double T, double tau0) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v == 0) *d.clock = tau0;
    if (v >= d.V) return;
    const int k = v / d.Q;
    const double val = d.tab.wxw[v] * 0.25 * n0 * (1.0 + (1.0 - T / d.T0) * d.tab.L1[k]);
    ((Tf*)d.f)[v] = (Tf)val;
}

template <typename Tf>
__global__ void bj_moments_kernel(InstDesc d, const Tf* f, double* out, int nf) {
    __shared__ double red[3 * kBjBlock];
    __shared__ double fs[4096];
    for (int v = threadIdx.x; v < d.V; v += blockDim.x) fs[v] = (double)f[v];
    __syncthreads();
    double n, E, PL;
    bj_moments<Tf>(d, fs, red, n, E, PL);
    if (threadIdx.x == 0) {
        const double P = E / 3.0;
        const double T = d.gas == RSL_GAS_IDEAL ? P / n : sqrt(sqrt(P));
        const double row[RSL_NMOM] = {n, 0.0, E, 0.0, PL, n, E, P, T, 0.0, n / (T * T * T), 0.0, PL - P};
        for (int q = 0; q < nf; ++q) out[q] = row[q];
    }
}

}  // namespace

int launch_bj_init(const InstDesc& d, double n0, double T, double tau0, hipStream_t s) {
    if (d.dtype == RSL_F64)
        hipLaunchKernelGGL(bj_init_kernel<double>, dim3((d.V + 63) / 64), dim3(64), 0, s, d, n0, T, tau0);
    else
        hipLaunchKernelGGL(bj_init_kernel<float>, dim3((d.V + 63) / 64), dim3(64), 0, s, d, n0, T, tau0);
    return hip_check(hipGetLastError(), "bj_init_kernel launch");
}

int launch_bj_steps(const InstDesc& d, double tau0, double dtau, int nsteps, hipStream_t s) {
    const size_t lds = sizeof(double) * (4 * (size_t)d.V + 3 * kBjBlock);
    if (lds > 150 * 1024) return set_error(RSL_EUNSUPPORTED, "Bjorken: velocity set too large for one workgroup");
    static const hipError_t a64 = hipFuncSetAttribute((const void*)bj_steps_kernel<double>,
                                                      hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    static const hipError_t a32 = hipFuncSetAttribute((const void*)bj_steps_kernel<float>,
                                                      hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    if (a64 != hipSuccess) return hip_check(a64, "hipFuncSetAttribute(bj_steps_kernel)");
    if (a32 != hipSuccess) return hip_check(a32, "hipFuncSetAttribute(bj_steps_kernel)");
    if (d.dtype == RSL_F64)
        hipLaunchKernelGGL(bj_steps_kernel<double>, dim3(1), dim3(kBjBlock), lds, s, d, tau0, dtau, nsteps);
    else
        hipLaunchKernelGGL(bj_steps_kernel<float>, dim3(1), dim3(kBjBlock), lds, s, d, tau0, dtau, nsteps);
    return hip_check(hipGetLastError(), "bj_steps_kernel launch");
}

int launch_bj_batch_steps(const InstDesc* descs, int n, size_t lds, int dtype, char* fbase, char* wbase,
                          double, double, int nsteps, hipStream_t s) {
    if (lds > 150 * 1024) return set_error(RSL_EUNSUPPORTED, "Bjorken: velocity set too large for one workgroup");
    static const hipError_t a64 = hipFuncSetAttribute((const void*)bj_batch_steps_kernel<double>,
                                                      hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    static const hipError_t a32 = hipFuncSetAttribute((const void*)bj_batch_steps_kernel<float>,
                                                      hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    if (a64 != hipSuccess) return hip_check(a64, "hipFuncSetAttribute(bj_batch_steps_kernel)");
    if (a32 != hipSuccess) return hip_check(a32, "hipFuncSetAttribute(bj_batch_steps_kernel)");
    if (dtype == RSL_F64)
        hipLaunchKernelGGL(bj_batch_steps_kernel<double>, dim3(n), dim3(kBjBlock), lds, s, descs, fbase, wbase, nsteps);
    else
        hipLaunchKernelGGL(bj_batch_steps_kernel<float>, dim3(n), dim3(kBjBlock), lds, s, descs, fbase, wbase, nsteps);
    return hip_check(hipGetLastError(), "bj_batch_steps_kernel launch");
}

size_t bj_lds_bytes(int V) { return sizeof(double) * (4 * (size_t)V + 3 * kBjBlock); }

int launch_bj_moments(const InstDesc& d, const void* f, double* out, int nf, hipStream_t s) {
    if (d.V > 4096) return set_error(RSL_EUNSUPPORTED, "Bjorken moments: more than 4096 velocities");
    if (d.dtype == RSL_F64)
        hipLaunchKernelGGL(bj_moments_kernel<double>, dim3(1), dim3(kBjBlock), 0, s, d, (const double*)f, out, nf);
    else
        hipLaunchKernelGGL(bj_moments_kernel<float>, dim3(1), dim3(kBjBlock), 0, s, d, (const float*)f, out, nf);
    return hip_check(hipGetLastError(), "bj_moments_kernel launch");
}

}  // namespace rsl
