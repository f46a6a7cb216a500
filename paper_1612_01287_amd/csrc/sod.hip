// Sod shock-tube kernels around the stage kernel: initial state, boundary
// states, cell moments (the fused RK3 stage is in sod_stage.hip).
#include <hip/hip_runtime.h>

#include "rsl_math.h"

namespace rsl {

namespace {



// Initial value of cell s, velocity v (Sec. IV A): the left or right state's
// f^eq, the mean of the two in a cell centred on the membrane.
__device__ __forceinline__ double sod_initial(const InstDesc& d, int s, int v) {
    const double z = d.z_lo + (s + 0.5) * d.dz;
    const double zm = d.z_lo + 0.5 * d.nz * d.dz;
    if (z < zm && fabs(z - zm) > 0.25 * d.dz) return d.feqL[v];
    if (z > zm && fabs(z - zm) > 0.25 * d.dz) return d.feqR[v];
    return 0.5 * (d.feqL[v] + d.feqR[v]);
}

template <typename Tf>
__global__ void sod_fill_kernel(InstDesc d) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y;
    if (s >= d.nz) return;
    ((Tf*)d.f)[(size_t)v * d.pitch + s] = (Tf)sod_initial(d, s, v);
}

// f^eq at velocity v of a state at rest (truncated expansion at the nodes).
__device__ __forceinline__ double rest_feq(const InstDesc& d, double n, double T, int v) {
    const int k = v / d.Q, j = v - k * d.Q;
    double c0[kMaxNOm + 1], c1[kMaxNOm + 1];
    feq_coef(n, T, 0.0, 1.0, d.T0, d.NOm, d.beta_series, d.tab.ser, 1, c0, c1);
    double g = 0.0;
    for (int m = 0; m <= d.NOm; ++m) g += d.tab.Pm[m * d.Q + j] * (c0[m] + d.tab.L1[k] * c1[m]);
    return d.tab.wxw[v] * g;
}

// f^eq at the nodes of two states at rest, one thread per velocity.
__global__ void boundary_state_kernel(InstDesc d, double nL, double TL, double nR, double TR,
                                      double* outL, double* outR) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= d.V) return;
    outL[v] = rest_feq(d, nL, TL, v);
    outR[v] = rest_feq(d, nR, TR, v);
}

// Batch initialisation, step 1: one workgroup per instance writes the
// boundary states and clears the status word and clock.
__global__ void batch_boundary_kernel(const InstDesc* __restrict__ descs, const double* __restrict__ states,
                                      char* fbase, char* wbase) {
    InstDesc d = descs[blockIdx.x];
    rebase(d, fbase, wbase);
    const double* st = states + 4 * (size_t)blockIdx.x;
    for (int v = threadIdx.x; v < d.V; v += blockDim.x) {
        ((double*)d.feqL)[v] = rest_feq(d, st[0], st[1], v);
        ((double*)d.feqR)[v] = rest_feq(d, st[2], st[3], v);
    }
    if (threadIdx.x == 0) {
        *d.status = 0u;
        *d.clock = 0.0;
    }
}

// Batch initialisation, step 2: one workgroup per (instance, 64-cell tile).
template <typename Tf>
__global__ void batch_fill_kernel(const InstDesc* __restrict__ descs, const int2* __restrict__ items, char* fbase,
                                  char* wbase) {
    const int2 it = items[blockIdx.x];
    if (it.x < 0) return;
    InstDesc d = descs[it.x];
    rebase(d, fbase, wbase);
    const int s = it.y * kCellTile + threadIdx.x;
    if (s >= d.nz) return;
    for (int v = 0; v < d.V; ++v) ((Tf*)d.f)[(size_t)v * d.pitch + s] = (Tf)sod_initial(d, s, v);
}

// nf = 5: the raw moments only; nf = RSL_NMOM: raw and derived fields.
template <typename Tf>
__global__ void sod_moments_kernel(InstDesc d, const Tf* __restrict__ f, double* __restrict__ out, int nf) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= d.nz) return;
    double M[5] = {0, 0, 0, 0, 0};
    for (int v = 0; v < d.V; ++v) {
        const int k = v / d.Q, j = v - k * d.Q;
        const double val = (double)f[(size_t)v * d.pitch + s];
        const double x = d.tab.xi[j], pv = d.tab.pk[k] * val;
        M[0] += val;
        M[1] += x * val;
        M[2] += pv;
        M[3] += x * pv;
        M[4] += x * x * pv;
    }
    double* o = out + (size_t)s * nf;
    for (int q = 0; q < 5; ++q) o[q] = M[q];
    if (nf == 5) return;
    const CellState cs = landau(M[0], M[1], M[2], M[3], M[4]);
    if (!cs.ok) {
        for (int q = 5; q < RSL_NMOM; ++q) o[q] = NAN;
        atomicOr(d.status, 1u);
        return;
    }
    const double P = cs.E / 3.0;
    o[5] = cs.n;
    o[6] = cs.E;
    o[7] = P;
    o[8] = cs.T;
    o[9] = cs.beta;
    o[10] = cs.n / (cs.T * cs.T * cs.T);
    o[11] = -4.0 * cs.T * (M[1] - cs.n * cs.beta * cs.gamma);
    o[12] = 2.0 * cs.E / 3.0 - M[2] + M[4];
}

}  // namespace

int launch_boundary_states(const InstDesc& d, double nL, double TL, double nR, double TR, hipStream_t s) {
    hipLaunchKernelGGL(boundary_state_kernel, dim3((d.V + 63) / 64), dim3(64), 0, s, d, nL, TL, nR, TR,
                       (double*)d.feqL, (double*)d.feqR);
    return hip_check(hipGetLastError(), "boundary_state_kernel launch");
}

int launch_sod_batch_init(const InstDesc* descs, const double* states, int n, const int2* items, int nitems,
                          int dtype, char* fbase, char* wbase, hipStream_t s) {
    hipLaunchKernelGGL(batch_boundary_kernel, dim3(n), dim3(64), 0, s, descs, states, fbase, wbase);
    int rc = hip_check(hipGetLastError(), "batch_boundary_kernel launch");
    if (rc || nitems == 0) return rc;
    if (dtype == RSL_F64)
        hipLaunchKernelGGL(batch_fill_kernel<double>, dim3(nitems), dim3(kCellTile), 0, s, descs, items, fbase, wbase);
    else
        hipLaunchKernelGGL(batch_fill_kernel<float>, dim3(nitems), dim3(kCellTile), 0, s, descs, items, fbase, wbase);
    return hip_check(hipGetLastError(), "batch_fill_kernel launch");
}

int launch_sod_init(const InstDesc& d, hipStream_t s) {
    dim3 grid((d.nz + 255) / 256, d.V);
    if (d.dtype == RSL_F64) hipLaunchKernelGGL(sod_fill_kernel<double>, grid, dim3(256), 0, s, d);
    else hipLaunchKernelGGL(sod_fill_kernel<float>, grid, dim3(256), 0, s, d);
    return hip_check(hipGetLastError(), "sod_fill_kernel launch");
}

int launch_sod_moments(const InstDesc& d, const void* f, double* out, int nf, hipStream_t s) {
    dim3 grid((d.nz + 127) / 128);
    if (d.dtype == RSL_F64)
        hipLaunchKernelGGL(sod_moments_kernel<double>, grid, dim3(128), 0, s, d, (const double*)f, out, nf);
    else
        hipLaunchKernelGGL(sod_moments_kernel<float>, grid, dim3(128), 0, s, d, (const float*)f, out, nf);
    return hip_check(hipGetLastError(), "sod_moments_kernel launch");
}

}  // namespace rsl
