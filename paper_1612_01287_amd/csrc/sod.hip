// Sod shock-tube kernels: initial state, one fused RK3 stage, cell moments.
//
// One RK3 stage (eq. rk3) evaluates L_Sod (eq. L_Sod) on the stage field and
// combines it with f_n.  A workgroup owns one tile: 64 consecutive cells
// (lane l <-> cell c = z0 - 1 + l) of one instance and all V velocities,
// split over its four waves (wave w takes v = w, w+4, ...).
//   phase 1  each wave streams its planes once (coalesced along z), sums the
//            five moments of its lane's cell (eq. macro_jk) and keeps the
//            values, with a 3-cell halo on either side, in an LDS window
//            [V][72] (cells z0-3 .. z0+65);
//   reduce   the four partial moment sets meet in LDS;
//   cell     each lane solves its cell's Landau frame (eqs. E_landau,
//            u_landau), relaxation time and equilibrium coefficients in FP64;
//   phase 2  per plane: WENO5 flux at face c+1/2 (Sec. III F) from the LDS
//            window, the face c-1/2 flux from the neighbouring lane, the
//            AW term -gamma (1 - beta xi_j)/tau (f - f^eq), the RK
//            combination, one store.
// Lane 0 only supplies the flux of face z0-1/2, so a tile advances 63 cells.
// If the window does not fit in LDS the stencil is read from global memory
// (L2) instead.
#include <hip/hip_runtime.h>

#include "rsl_math.h"

namespace rsl {

namespace {

constexpr int kWaves = 4;
constexpr int kBlock = kWaves * kLanes;
constexpr size_t kRedBytes = sizeof(double) * kWaves * 5 * kLanes;
constexpr size_t kMaxLds = 150 * 1024;

template <typename Tf>
__device__ __forceinline__ double cell_value(const InstDesc& d, const Tf* __restrict__ f, int v, int c) {
    if (c >= 0 && c < d.nz) return (double)f[(size_t)v * d.pitch + c];
    if (d.bc == RSL_BC_EQ) return c < 0 ? d.feqL[v] : d.feqR[v];
    const int cc = c < 0 ? 0 : d.nz - 1;
    return (double)f[(size_t)v * d.pitch + cc];
}

// Tile index with consecutive tiles on one XCD (workgroups are dealt to the
// eight XCDs round-robin), so that halo cells shared by neighbouring tiles
// are fetched into the same L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int per = nb >> 3;
    return (b & 7) * per + (b >> 3);
}

template <typename Tf, int STAGE>
__device__ __forceinline__ void sod_tile(const InstDesc& d, int tile, int use_stash, double* smem) {
    const int lane = threadIdx.x & (kLanes - 1);
    const int w = threadIdx.x / kLanes;
    const int z0 = tile * kTileCells;
    const int c = z0 - 1 + lane;
    const bool own = (c >= 0) && (c < d.nz);

    const Tf* __restrict__ fcur = (const Tf*)(STAGE == 1 ? d.f : (STAGE == 2 ? d.f1 : d.f2));
    Tf* __restrict__ fout = (Tf*)(STAGE == 1 ? d.f1 : (STAGE == 2 ? d.f2 : d.f));
    const Tf* __restrict__ fn = (const Tf*)d.f;
    double* red = smem;
    Tf* win = (Tf*)((char*)smem + kRedBytes);
    const int Q = d.Q;
    const double* __restrict__ xi = d.tab.xi;
    const double* __restrict__ pk = d.tab.pk;

    // ---- phase 1: moments of the stage field, LDS window
    double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0, m4 = 0.0;
    for (int v = w; v < d.V; v += kWaves) {
        const int k = v / Q, j = v - k * Q;
        const double val = cell_value(d, fcur, v, c);
        if (own) {
            const double x = xi[j], pv = pk[k] * val;
            m0 += val;
            m1 += x * val;
            m2 += pv;
            m3 += x * pv;
            m4 += x * x * pv;
        }
        if (use_stash) {
            Tf* row = win + (size_t)v * kWin;
            row[lane + 2] = (Tf)val;
            if (lane < 2) row[lane] = (Tf)cell_value(d, fcur, v, z0 - 3 + lane);
            else if (lane < 5) row[lane + 64] = (Tf)cell_value(d, fcur, v, z0 + 61 + lane);
        }
    }
    red[(w * 5 + 0) * kLanes + lane] = m0;
    red[(w * 5 + 1) * kLanes + lane] = m1;
    red[(w * 5 + 2) * kLanes + lane] = m2;
    red[(w * 5 + 3) * kLanes + lane] = m3;
    red[(w * 5 + 4) * kLanes + lane] = m4;
    __syncthreads();
    double M[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        double s = red[q * kLanes + lane];
#pragma unroll
        for (int ww = 1; ww < kWaves; ++ww) s += red[(ww * 5 + q) * kLanes + lane];
        M[q] = s;
    }

    // ---- per-cell state (FP64)
    const bool collide = d.tau_mode != RSL_TAU_INF;
    double cA = 0.0, cB = 0.0;
    double c0[kMaxNOm + 1], c1[kMaxNOm + 1];
#pragma unroll
    for (int m = 0; m <= kMaxNOm; ++m) c0[m] = c1[m] = 0.0;
    unsigned bad = 0;
    if (collide) {
        CellState cs = landau(M[0], M[1], M[2], M[3], M[4]);
        if (own && !cs.ok) bad |= 1u;
        if (!cs.ok) {   // keep the arithmetic finite; the cell is flagged
            cs.n = 1.0; cs.T = 1.0; cs.beta = 0.0; cs.gamma = 1.0;
        }
        double tau = d.tau_r;
        if (d.tau_mode == RSL_TAU_ETAS) {
            const double lam = cs.n / (cs.T * cs.T * cs.T);
            tau = d.tau_aw0 / cs.T * (1.0 - 0.25 * log(lam * d.lambda_ref));
        }
        const double it = 1.0 / tau;
        cA = cs.gamma * it;
        cB = cs.gamma * cs.beta * it;
        feq_coef(cs.n, cs.T, cs.beta, cs.gamma, d.T0, d.NOm, d.beta_series, d.tab.ser, d.tab.thr, c0, c1);
    }

    // ---- phase 2: flux, collision, RK combination
    const double dt = d.dt;
    for (int v = w; v < d.V; v += kWaves) {
        const int k = v / Q, j = v - k * Q;
        const double x = xi[j];
        double s[6];
        if (use_stash) {
            const Tf* row = win + (size_t)v * kWin + lane;
#pragma unroll
            for (int i = 0; i < 6; ++i) s[i] = (double)row[i];
        } else {
#pragma unroll
            for (int i = 0; i < 6; ++i) s[i] = cell_value(d, fcur, v, c - 2 + i);
        }
        double F = 0.0;
        if (x > 0.0) F = x * weno5(s[0], s[1], s[2], s[3], s[4]);
        else if (x < 0.0) F = x * weno5(s[5], s[4], s[3], s[2], s[1]);
        const double Fm = __shfl_up(F, 1);
        if (lane >= 1 && own) {
            const double fc = s[2];
            double L = -(F - Fm) * d.dz_inv;
            if (collide) {
                const double l1 = d.tab.L1[k];
                double g = 0.0;
#pragma unroll
                for (int m = 0; m <= kMaxNOm; ++m)
                    if (m <= d.NOm) g = fma(d.tab.Pm[m * Q + j], fma(l1, c1[m], c0[m]), g);
                const double feq = d.tab.wxw[v] * g;
                L -= (cA - cB * x) * (fc - feq);
            }
            double out;
            if (STAGE == 1) {
                out = fc + dt * L;
            } else if (STAGE == 2) {
                const double fv = (double)fn[(size_t)v * d.pitch + c];
                out = 0.75 * fv + 0.25 * fc + 0.25 * dt * L;
            } else {
                const double fv = (double)fn[(size_t)v * d.pitch + c];
                out = fv / 3.0 + 2.0 * fc / 3.0 + 2.0 * dt * L / 3.0;
            }
            const Tf o = (Tf)out;
            if (!isfinite((double)o)) bad |= 2u;
            fout[(size_t)v * d.pitch + c] = o;
        }
    }
    if (bad) atomicOr(d.status, bad);
}

template <typename Tf, int STAGE>
__global__ void __launch_bounds__(kBlock) sod_stage_kernel(InstDesc d, int ntiles, int use_stash) {
    extern __shared__ double smem[];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    sod_tile<Tf, STAGE>(d, tile, use_stash, smem);
}

// Batched stage: one workgroup per (instance, tile) item.  The host orders the
// items so that block b runs on XCD b % 8 with that XCD's share of the work,
// costliest first; padding items carry inst = -1.  Descriptors hold byte
// offsets into the batch's f and work buffers.
template <typename Tf, int STAGE>
__global__ void __launch_bounds__(kBlock) sod_batch_stage_kernel(const InstDesc* __restrict__ descs,
                                                                 const int2* __restrict__ items, char* fbase,
                                                                 char* wbase, int stash_limit) {
    extern __shared__ double smem[];
    const int2 it = items[blockIdx.x];
    if (it.x < 0) return;
    InstDesc d = descs[it.x];
    rebase(d, fbase, wbase);
    const int use_stash = (int)(d.V * kWin * sizeof(Tf)) <= stash_limit;
    sod_tile<Tf, STAGE>(d, it.y, use_stash, smem);
}

template <typename Tf>
__global__ void sod_fill_kernel(InstDesc d) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y;
    if (s >= d.nz) return;
    const double z = d.z_lo + (s + 0.5) * d.dz;
    const double zm = d.z_lo + 0.5 * d.nz * d.dz;
    double val;
    if (z < zm && fabs(z - zm) > 0.25 * d.dz) val = d.feqL[v];
    else if (z > zm && fabs(z - zm) > 0.25 * d.dz) val = d.feqR[v];
    else val = 0.5 * (d.feqL[v] + d.feqR[v]);
    ((Tf*)d.f)[(size_t)v * d.pitch + s] = (Tf)val;
}

// f^eq at the nodes of two states at rest, one thread per velocity.
__global__ void boundary_state_kernel(InstDesc d, double nL, double TL, double nR, double TR,
                                      double* outL, double* outR) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= d.V) return;
    const int k = v / d.Q, j = v - k * d.Q;
    double c0[kMaxNOm + 1], c1[kMaxNOm + 1];
    for (int side = 0; side < 2; ++side) {
        const double n = side ? nR : nL, T = side ? TR : TL;
        feq_coef(n, T, 0.0, 1.0, d.T0, d.NOm, d.beta_series, d.tab.ser, d.tab.thr, c0, c1);
        double g = 0.0;
        for (int m = 0; m <= d.NOm; ++m) g += d.tab.Pm[m * d.Q + j] * (c0[m] + d.tab.L1[k] * c1[m]);
        (side ? outR : outL)[v] = d.tab.wxw[v] * g;
    }
}

template <typename Tf>
__global__ void sod_moments_kernel(InstDesc d, const Tf* __restrict__ f, double* __restrict__ out) {
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
    double* o = out + (size_t)s * RSL_NMOM;
    for (int q = 0; q < 5; ++q) o[q] = M[q];
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

template <typename Tf>
size_t stash_bytes(const InstDesc& d) { return (size_t)d.V * kWin * sizeof(Tf); }

template <typename Tf, int STAGE>
int stage_t(const InstDesc& d, hipStream_t s) {
    const int ntiles = (d.nz + kTileCells - 1) / kTileCells;
    const int nb = (ntiles + 7) / 8 * 8;
    const size_t sb = stash_bytes<Tf>(d);
    const int use_stash = (kRedBytes + sb) <= kMaxLds;
    const size_t lds = kRedBytes + (use_stash ? sb : 0);
    static const hipError_t attr = hipFuncSetAttribute((const void*)sod_stage_kernel<Tf, STAGE>,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
    if (attr != hipSuccess) return hip_check(attr, "hipFuncSetAttribute(sod_stage_kernel)");
    hipLaunchKernelGGL((sod_stage_kernel<Tf, STAGE>), dim3(nb), dim3(kBlock), lds, s, d, ntiles, use_stash);
    return hip_check(hipGetLastError(), "sod_stage_kernel launch");
}

template <typename Tf, int STAGE>
int batch_stage_t(const BatchLaunch& b, char* fbase, char* wbase, hipStream_t s) {
    static const hipError_t attr = hipFuncSetAttribute((const void*)sod_batch_stage_kernel<Tf, STAGE>,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
    if (attr != hipSuccess) return hip_check(attr, "hipFuncSetAttribute(sod_batch_stage_kernel)");
    hipLaunchKernelGGL((sod_batch_stage_kernel<Tf, STAGE>), dim3(b.nitems), dim3(kBlock), b.lds_bytes, s, b.descs,
                       b.items, fbase, wbase, b.stash_limit);
    return hip_check(hipGetLastError(), "sod_batch_stage_kernel launch");
}

}  // namespace

size_t sod_red_bytes() { return kRedBytes; }
size_t sod_max_lds() { return kMaxLds; }

int launch_sod_batch_stage(const BatchLaunch& b, int dtype, int stage, char* fbase, char* wbase, hipStream_t s) {
    if (dtype == RSL_F64) {
        if (stage == 1) return batch_stage_t<double, 1>(b, fbase, wbase, s);
        if (stage == 2) return batch_stage_t<double, 2>(b, fbase, wbase, s);
        return batch_stage_t<double, 3>(b, fbase, wbase, s);
    }
    if (stage == 1) return batch_stage_t<float, 1>(b, fbase, wbase, s);
    if (stage == 2) return batch_stage_t<float, 2>(b, fbase, wbase, s);
    return batch_stage_t<float, 3>(b, fbase, wbase, s);
}

int launch_sod_stage(const InstDesc& d, int stage, hipStream_t s) {
    if (d.dtype == RSL_F64) {
        if (stage == 1) return stage_t<double, 1>(d, s);
        if (stage == 2) return stage_t<double, 2>(d, s);
        return stage_t<double, 3>(d, s);
    }
    if (stage == 1) return stage_t<float, 1>(d, s);
    if (stage == 2) return stage_t<float, 2>(d, s);
    return stage_t<float, 3>(d, s);
}

int launch_boundary_states(const InstDesc& d, double nL, double TL, double nR, double TR, hipStream_t s) {
    hipLaunchKernelGGL(boundary_state_kernel, dim3((d.V + 63) / 64), dim3(64), 0, s, d, nL, TL, nR, TR,
                       (double*)d.feqL, (double*)d.feqR);
    return hip_check(hipGetLastError(), "boundary_state_kernel launch");
}

int launch_sod_init(const InstDesc& d, hipStream_t s) {
    dim3 grid((d.nz + 255) / 256, d.V);
    if (d.dtype == RSL_F64) hipLaunchKernelGGL(sod_fill_kernel<double>, grid, dim3(256), 0, s, d);
    else hipLaunchKernelGGL(sod_fill_kernel<float>, grid, dim3(256), 0, s, d);
    return hip_check(hipGetLastError(), "sod_fill_kernel launch");
}

int launch_sod_moments(const InstDesc& d, const void* f, double* out, hipStream_t s) {
    dim3 grid((d.nz + 127) / 128);
    if (d.dtype == RSL_F64)
        hipLaunchKernelGGL(sod_moments_kernel<double>, grid, dim3(128), 0, s, d, (const double*)f, out);
    else
        hipLaunchKernelGGL(sod_moments_kernel<float>, grid, dim3(128), 0, s, d, (const float*)f, out);
    return hip_check(hipGetLastError(), "sod_moments_kernel launch");
}

}  // namespace rsl
