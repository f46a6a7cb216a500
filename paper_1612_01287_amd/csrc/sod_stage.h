#pragma once
// The fused Sod RK3-stage kernel (included by sod_stage_f64.hip and
// sod_stage_f32.hip, one instantiation per storage type).
//
// One stage of eq. rk3 applied to L_Sod (eq. L_Sod): for every cell s and
// velocity (j,k) of a 63-cell tile,
//   out = a f_n + b [ f + dt ( -(F_{s+1/2} - F_{s-1/2})/dz
//                              - gamma (1 - beta xi_j)/tau (f - f^eq_jk) ) ]
// with (a, b) = (0, 1), (3/4, 1/4), (1/3, 2/3) for the three stages.
//
// Work decomposition.  A workgroup of W waves owns one tile; lane l of every
// wave holds cell c = z0 - 1 + l (lane 0 only supplies the flux of face
// z0 - 1/2, so 63 cells advance), and wave w owns the velocities
// v = w, w + W, ... (at most NV of them).
//   phase 1  every wave issues all its stage-field loads at once (own cells
//            and a 3+2 cell halo), then per velocity: moments of the lane's cell
//            (eq. macro_jk), the 69-cell plane segment through a
//            double-buffered per-wave LDS window, the WENO5 flux at face
//            c + 1/2 (Sec. III F) and the face c - 1/2 flux from lane - 1,
//            and the advective update f - dt dF/dz, kept in registers with
//            the cell value; the f_n loads are issued next;
//   reduce   partial moments of the W waves meet in LDS in a fixed order;
//   cell     wave 0 solves each cell's Landau frame (eqs. E_landau,
//            u_landau), relaxation time and equilibrium coefficients in FP64
//            and publishes them in LDS;
//   phase 2  per velocity: f^eq_jk from the coefficients, the AW term, the
//            RK combination, one store.
// HBM traffic per cell and velocity: the stage field once (plus 5/64 halo,
// mostly L2 hits), f_n once (stages 2, 3), one store.
#include <hip/hip_runtime.h>

#include "rsl_math.h"

namespace rsl {

namespace {

constexpr int kPar = 16;   // per-cell coefficients in LDS: cA, cB, c0[7], c1[7]
constexpr int kGroup = 4;  // velocities per LDS window round

// Value of lane l - 1 (lane 0 gets its own value back): a DPP wave shift,
// no LDS round trip.
__device__ __forceinline__ double shift_up(double x) {
    const int lo = __double2loint(x), hi = __double2hiint(x);
    const int slo = __builtin_amdgcn_update_dpp(lo, lo, 0x138, 0xf, 0xf, false);
    const int shi = __builtin_amdgcn_update_dpp(hi, hi, 0x138, 0xf, 0xf, false);
    return __hiloint2double(shi, slo);
}

__device__ __forceinline__ float shift_up(float x) {
    const int b = __float_as_int(x);
    return __int_as_float(__builtin_amdgcn_update_dpp(b, b, 0x138, 0xf, 0xf, false));
}


// Orders LDS accesses of one wave: LDS executes a wave's instructions in
// issue order, so keeping the compiler from moving them is enough.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Read-only tables indexed by a wave-uniform velocity: going through the
// constant address space lets the compiler use scalar loads, which do not
// wait behind the vector loads in flight.
template <typename T>
__device__ __forceinline__ T ldc(const T* p, int i) {
    return ((const __attribute__((address_space(4))) T*)p)[i];
}

// Per-lane choice between the constants of the two velocity slots of a wave
// (both loaded with scalar loads; a lane-dependent branch would turn the loads
// into vector loads).
template <int S>
__device__ __forceinline__ double pick(int slot, double a, double b) {
    return (S == 2 && slot) ? b : a;
}

__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int per = nb >> 3;
    return (b & 7) * per + (b >> 3);
}

// Velocities of step i for wave w.  One slot (64 lanes per velocity): v = w + i W.
// Two slots (32 lanes each): the pair vperm[2p], vperm[2p+1], p = w + i W, taken
// from a list ordered by the sign of xi_j so that both slots usually move the
// same way (the upwind branch then stays uniform).  All values are scalars.
struct VelPair {
    int va, vb;
    bool ok_a, ok_b;
};

template <int S, int W>
__device__ __forceinline__ VelPair vel_pair(const InstDesc& d, int w, int i) {
    VelPair r;
    if (S == 1) {
        const int v = w + i * W;
        r.ok_a = r.ok_b = v < d.V;
        r.va = r.vb = min(v, d.V - 1);
    } else {
        const int ia = 2 * (w + i * W), ib = ia + 1;
        r.ok_a = ia < d.V;
        r.ok_b = ib < d.V;
        r.va = ldc(d.tab.vperm, min(ia, d.V - 1));
        r.vb = ldc(d.tab.vperm, min(ib, d.V - 1));
    }
    return r;
}

template <typename Tf, int STAGE, int W, int NV, int TW>
__device__ __forceinline__ void stage_tile(const InstDesc& d, int tile, char* lds) {
    constexpr int G = kGroup;
    constexpr int S = kLanes / TW;        // velocity slots per wave
    constexpr int VS = W * S;             // velocity streams per workgroup
    constexpr int WN = TW + 8;            // window entries per slot (TW + 5 used)
    const int lane = threadIdx.x & (kLanes - 1);
    // wave index as a scalar: the per-velocity tables then come through
    // scalar loads and the upwind branch on xi_j is uniform
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
    const int slot = S == 1 ? 0 : lane / TW;
    const int cl = lane & (TW - 1);
    const int z0 = tile * (TW - 1);
    const int c = z0 - 1 + cl;
    const bool ghost = (c < 0) || (c >= d.nz);
    const int cc = min(max(c, 0), d.nz - 1);
    const int hc = cl < 2 ? z0 - 3 + cl : z0 + TW - 3 + cl;   // halo cell of lanes cl = 0..4
    const bool hghost = (hc < 0) || (hc >= d.nz);
    const int hcc = min(max(hc, 0), d.nz - 1);
    const bool eqbc = d.bc == RSL_BC_EQ;
    const int V = d.V;

    double* red = (double*)lds;
    double* par = red + VS * 5 * TW;
    Tf* win = (Tf*)(par + TW * kPar) + w * 2 * G * S * WN + slot * WN;

    const Tf* __restrict__ fcur = (const Tf*)(STAGE == 1 ? d.f : (STAGE == 2 ? d.f1 : d.f2));
    Tf* __restrict__ fout = (Tf*)(STAGE == 1 ? d.f1 : (STAGE == 2 ? d.f2 : d.f));
    const Tf* __restrict__ fn = (const Tf*)d.f;
    const size_t pitch = (size_t)d.pitch;
    const double* __restrict__ xv = d.tab.xv;
    const double* __restrict__ pv = d.tab.pv;

    // ---- all stage-field loads of this wave in flight at once (clamped,
    //      branch-free addresses so the compiler keeps them outstanding)
    Tf ra[NV], rh[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const VelPair vp = vel_pair<S, W>(d, w, i);
        const Tf* row = fcur + (size_t)(slot ? vp.vb : vp.va) * pitch;
        ra[i] = row[cc];
        rh[i] = cl < 5 ? row[hcc] : Tf(0);
    }

    // ---- phase 1: moments, WENO5 flux, advective update y = f - dt dF/dz
    //      (y and f kept in the storage type: binary32 rounding of y is within
    //      the binary32 parity bar, binary64 keeps it exact)
    const double dt = d.dt, dzi = d.dz_inv;
    double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0, m4 = 0.0;
    Tf fcv[NV], yv[NV];
    // velocities go through the LDS window in groups of G: one wave-level
    // ordering point per group, and G independent WENO evaluations after it
#pragma unroll
    for (int i0 = 0; i0 < NV; i0 += G) {
        if (!vel_pair<S, W>(d, w, i0).ok_a) break;
#pragma unroll
        for (int i = i0; i < i0 + G && i < NV; ++i) {
            const VelPair vp = vel_pair<S, W>(d, w, i);
            if (vp.ok_a) {
                const bool valid = slot ? vp.ok_b : vp.ok_a;
                // per-velocity constants: scalar loads for both slots, lane select
                const double x = pick<S>(slot, ldc(xv, vp.va), ldc(xv, vp.vb));
                const double pk = pick<S>(slot, ldc(pv, vp.va), ldc(pv, vp.vb));
                double fc = (double)ra[i];
                double h = (double)rh[i];
                if (eqbc) {
                    const double gl = pick<S>(slot, ldc(d.feqL, vp.va), ldc(d.feqL, vp.vb));
                    const double gr = pick<S>(slot, ldc(d.feqR, vp.va), ldc(d.feqR, vp.vb));
                    fc = ghost ? (c < 0 ? gl : gr) : fc;
                    h = hghost ? (hc < 0 ? gl : gr) : h;
                }
                const double fo = (ghost || !valid) ? 0.0 : fc;
                const double p = pk * fo;
                m0 += fo;
                m1 += x * fo;
                m2 += p;
                m3 += x * p;
                m4 += x * x * p;
                Tf* wb = win + (((i0 / G) & 1) * G + (i - i0)) * S * WN;
                wb[cl + 2] = (Tf)fc;
                if (cl < 2) wb[cl] = (Tf)h;
                else if (cl < 5) wb[TW + cl] = (Tf)h;
            }
        }
        wave_lds_sync();
#pragma unroll
        for (int i = i0; i < i0 + G && i < NV; ++i) {
            const VelPair vp = vel_pair<S, W>(d, w, i);
            if (vp.ok_a) {
                const double xa = ldc(xv, vp.va), xb = ldc(xv, vp.vb);
                const double x = pick<S>(slot, xa, xb);
                const Tf* wb = win + (((i0 / G) & 1) * G + (i - i0)) * S * WN;
                double sv[6];
#pragma unroll
                for (int q = 0; q < 6; ++q) sv[q] = (double)wb[cl + q];
                // both slots move the same way unless the pair straddles xi = 0
                const bool same = S == 1 || !vp.ok_b || ((xa > 0.0) == (xb > 0.0) && (xa < 0.0) == (xb < 0.0));
                double F = 0.0;
                if (same) {
                    if (xa > 0.0) F = x * weno5(sv[0], sv[1], sv[2], sv[3], sv[4]);
                    else if (xa < 0.0) F = x * weno5(sv[5], sv[4], sv[3], sv[2], sv[1]);
                } else {
                    const bool up = x > 0.0;
                    F = x * weno5(up ? sv[0] : sv[5], up ? sv[1] : sv[4], up ? sv[2] : sv[3], up ? sv[3] : sv[2],
                                  up ? sv[4] : sv[1]);
                    if (x == 0.0) F = 0.0;
                }
                const double Fm = shift_up(F);
                yv[i] = (Tf)(sv[2] + dt * (-(F - Fm) * dzi));
                fcv[i] = wb[cl + 2];
            }
        }
    }

    // ---- f_n loads (stages 2, 3) go in flight before the barriers when the
    //      registers allow it
    Tf rn[NV];
    constexpr bool kEarlyFn = TW == 64 && NV * sizeof(Tf) <= 32 * sizeof(double);
    if (STAGE > 1 && kEarlyFn) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const VelPair vp = vel_pair<S, W>(d, w, i);
            rn[i] = fn[(size_t)(slot ? vp.vb : vp.va) * pitch + cc];
        }
    }

    // ---- moments of the VS streams, then per-cell coefficients by wave 0
    const int g = w * S + slot;
    red[(g * 5 + 0) * TW + cl] = m0;
    red[(g * 5 + 1) * TW + cl] = m1;
    red[(g * 5 + 2) * TW + cl] = m2;
    red[(g * 5 + 3) * TW + cl] = m3;
    red[(g * 5 + 4) * TW + cl] = m4;
    __syncthreads();
    const bool collide = d.tau_mode != RSL_TAU_INF;
    unsigned bad = 0;
    if (collide && w == 0 && slot == 0) {
        double M[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            double sum = red[q * TW + cl];
#pragma unroll
            for (int gg = 1; gg < VS; ++gg) sum += red[(gg * 5 + q) * TW + cl];
            M[q] = sum;
        }
        CellState cs = landau(M[0], M[1], M[2], M[3], M[4]);
        if (!ghost && !cs.ok) bad |= 1u;
        if (!cs.ok) {
            cs.n = 1.0; cs.T = 1.0; cs.beta = 0.0; cs.gamma = 1.0;
        }
        double tau = d.tau_r;
        if (d.tau_mode == RSL_TAU_ETAS) {
            const double lam = cs.n / (cs.T * cs.T * cs.T);
            tau = d.tau_aw0 / cs.T * (1.0 - 0.25 * log(lam * d.lambda_ref));
        }
        const double it = 1.0 / tau;
        double c0[kMaxNOm + 1], c1[kMaxNOm + 1];
        const int nt = series_terms(cs.beta * cs.beta, d.tab.thr);
        feq_coef(cs.n, cs.T, cs.beta, cs.gamma, d.T0, d.NOm, d.beta_series, d.tab.ser, nt, c0, c1);
        double* pp = par + cl * kPar;
        pp[0] = cs.gamma * it;
        pp[1] = cs.gamma * cs.beta * it;
#pragma unroll
        for (int m = 0; m <= kMaxNOm; ++m) {
            pp[2 + m] = c0[m];
            pp[2 + kMaxNOm + 1 + m] = c1[m];
        }
    }
    __syncthreads();

    // ---- phase 2: f_n, equilibrium, AW relaxation, RK combination, store
    if (STAGE > 1 && !kEarlyFn) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const VelPair vp = vel_pair<S, W>(d, w, i);
            rn[i] = fn[(size_t)(slot ? vp.vb : vp.va) * pitch + cc];
        }
    }
    double cA = 0.0, cB = 0.0, c0[kMaxNOm + 1], c1[kMaxNOm + 1];
    if (collide) {
        const double* pp = par + cl * kPar;
        cA = pp[0];
        cB = pp[1];
#pragma unroll
        for (int m = 0; m <= kMaxNOm; ++m) {
            c0[m] = pp[2 + m];
            c1[m] = pp[2 + kMaxNOm + 1 + m];
        }
    }
    const bool out_lane = !ghost && cl >= 1;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const VelPair vp = vel_pair<S, W>(d, w, i);
        if (vp.ok_a) {
            const int v = slot ? vp.vb : vp.va;
            const bool valid = slot ? vp.ok_b : vp.ok_a;
            double y = (double)yv[i];
            if (collide) {
                const double l1 = pick<S>(slot, ldc(d.tab.l1v, vp.va), ldc(d.tab.l1v, vp.vb));
                const double wx = pick<S>(slot, ldc(d.tab.wxw, vp.va), ldc(d.tab.wxw, vp.vb));
                const double x = pick<S>(slot, ldc(xv, vp.va), ldc(xv, vp.vb));
                double gsum = 0.0;
#pragma unroll
                for (int m = 0; m <= kMaxNOm; ++m)
                    if (m <= d.NOm) {
                        const double P = pick<S>(slot, ldc(d.tab.Pv, m * V + vp.va), ldc(d.tab.Pv, m * V + vp.vb));
                        gsum = fma(P, fma(l1, c1[m], c0[m]), gsum);
                    }
                y += dt * (cA - cB * x) * (wx * gsum - (double)fcv[i]);
            }
            double out;
            if (STAGE == 1) out = y;
            else if (STAGE == 2) out = 0.75 * (double)rn[i] + 0.25 * y;
            else out = fma(kTwoThirds, y, kThird * (double)rn[i]);
            if (out_lane && valid) {
                const Tf o = (Tf)out;
                if (!isfinite((double)o)) bad |= 2u;
                fout[(size_t)v * pitch + c] = o;
            }
        }
    }
    if (bad) atomicOr(d.status, bad);
}

template <typename Tf, int STAGE, int W, int NV, int TW>
__global__ void __launch_bounds__(W * 64) stage_single_kernel(InstDesc d, int ntiles) {
    extern __shared__ double lds_d[];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    stage_tile<Tf, STAGE, W, NV, TW>(d, tile, (char*)lds_d);
}

template <typename Tf, int STAGE, int W, int NV, int TW>
__global__ void __launch_bounds__(W * 64) stage_batch_kernel(const InstDesc* __restrict__ descs,
                                                             const int2* __restrict__ items, char* fbase,
                                                             char* wbase) {
    extern __shared__ double lds_d[];
    const int2 it = items[blockIdx.x];
    if (it.x < 0) return;
    InstDesc d = descs[it.x];
    rebase(d, fbase, wbase);
    stage_tile<Tf, STAGE, W, NV, TW>(d, it.y, (char*)lds_d);
}

template <int W, int TW, typename Tf>
constexpr size_t lds_bytes_t() {
    constexpr int S = kLanes / TW;
    return sizeof(double) * (W * S * 5 * TW + TW * kPar) + sizeof(Tf) * W * 2 * kGroup * S * (TW + 8);
}

template <typename Tf, int STAGE, int W, int NV, int TW>
int launch_t(const InstDesc* d, const StageClass* cl, char* fb, char* wb, hipStream_t s) {
    const size_t lds = lds_bytes_t<W, TW, Tf>();
    static_assert(lds_bytes_t<W, TW, Tf>() <= 160 * 1024, "stage kernel LDS above 160 KiB");
    if (lds > 64 * 1024) {
        static const hipError_t a1 = hipFuncSetAttribute((const void*)stage_single_kernel<Tf, STAGE, W, NV, TW>,
                                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        static const hipError_t a2 = hipFuncSetAttribute((const void*)stage_batch_kernel<Tf, STAGE, W, NV, TW>,
                                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (a1 != hipSuccess) return hip_check(a1, "hipFuncSetAttribute(stage kernel)");
        if (a2 != hipSuccess) return hip_check(a2, "hipFuncSetAttribute(stage kernel)");
    }
    if (d) {
        const int ntiles = (d->nz + TW - 2) / (TW - 1);
        const int nb = (ntiles + 7) / 8 * 8;
        hipLaunchKernelGGL((stage_single_kernel<Tf, STAGE, W, NV, TW>), dim3(nb), dim3(W * 64), lds, s, *d, ntiles);
    } else {
        hipLaunchKernelGGL((stage_batch_kernel<Tf, STAGE, W, NV, TW>), dim3(cl->nitems), dim3(W * 64), lds, s,
                           cl->descs, cl->items, fb, wb);
    }
    return hip_check(hipGetLastError(), "sod stage kernel launch");
}

// Kernel variants of the fused form: (waves W, velocities per slot NV, lanes
// per velocity TW); a variant covers V <= W * (64 / TW) * NV velocities.
#define RSL_STAGE_VARIANTS(X) \
    X(0, 4, 8, 64) X(1, 8, 4, 64) X(2, 4, 16, 64) X(3, 8, 8, 64) X(4, 8, 16, 64) X(5, 16, 8, 64) \
    X(6, 16, 4, 32) X(7, 8, 16, 32) X(8, 8, 20, 32) X(9, 8, 24, 32)
// Variants of the two-kernel form (sod_split.h): stream-kernel waves W,
// velocities per wave NV, cell-kernel waves WC; any V.
#define RSL_SPLIT_VARIANTS(X) \
    X(10, 4, 2, 8) X(11, 4, 4, 8) X(12, 4, 8, 8) X(13, 4, 2, 16) X(14, 4, 4, 16) X(15, 4, 8, 16) \
    X(16, 8, 2, 16) X(17, 8, 1, 16) X(18, 2, 4, 16)
// Variants of the loop form (sod_split.h): waves W walking the velocity set
// NV velocities at a time with K rounds of loads in flight, cell-kernel waves
// WC for the first stage of a call.
#define RSL_LOOP_VARIANTS(X) \
    X(19, 8, 2, 8, 2) X(20, 8, 1, 8, 4) X(21, 8, 1, 8, 2) X(22, 8, 1, 8, 3) X(23, 4, 1, 8, 4) X(24, 4, 1, 8, 5) \
    X(25, 4, 1, 8, 6) X(26, 4, 1, 8, 3) X(27, 4, 1, 8, 2) X(28, 4, 2, 8, 3)

}  // namespace

int launch_stage_f64(int stage, int var, const InstDesc* d, const StageClass* cl, char* fb, char* wb, hipStream_t s,
                     int seq);
int launch_stage_f32(int stage, int var, const InstDesc* d, const StageClass* cl, char* fb, char* wb, hipStream_t s,
                     int seq);

}  // namespace rsl
