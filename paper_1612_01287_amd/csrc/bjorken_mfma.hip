// Batched Bjorken flow with the momentum-space projection on the matrix cores.
//
// L_Bjorken (eq. L_Bjorken) for a group of up to 16 instances that share one
// velocity set is
//   L = ( -F + xi^2 (F K^L^T) + K^P F ) / tau - (F - F^eq) / tau_AW ,
// with F the Q_xi x (16 Q_L) matrix whose column (i, k) holds instance i's
// populations at radial node k.  The dense K^P F product (Q_xi^2 per column,
// eq. K_leg_disc) runs as v_mfma_f64_16x16x4f64 on 16x16 output tiles; the
// K^L term (Q_L x Q_L, eq. K_lag_disc), the moments, the relaxation and the
// RK3 combination (eq. rk3, stage times of Table II) run on the vector units.
//
// One workgroup (4 waves) owns one group for all requested steps: the stage
// field F lives in LDS (row j, column i Q_L + k), f_n in registers in the
// accumulator layout of the tiles each wave owns, K^P streams from global
// memory pre-arranged in A-operand tile order (one coalesced 512-byte load
// per wave and k-step).
#include <hip/hip_runtime.h>

#include "rsl_math.h"

namespace rsl {

namespace {

constexpr int kGI = 16;        // instances per group
constexpr int kBW = 4;         // waves per workgroup
constexpr int kMaxTilesPerWave = 16;

typedef double d4 __attribute__((ext_vector_type(4)));

template <typename Tf>
__global__ void __launch_bounds__(kBW * 64) bj_mfma_kernel(const InstDesc* __restrict__ descs,
                                                           const int* __restrict__ groups, char* fbase,
                                                           char* wbase, int nsteps) {
    extern __shared__ double X[];   // [Qp][NC] stage field, then per-instance scalars
    const int* gi = groups + blockIdx.x * kGI;
    const InstDesc d0 = descs[gi[0]];
    const int Q = d0.Q, QL = d0.QL, NC = kGI * QL;
    const int Qp = (Q + 15) & ~15;
    const int RT = Qp / 16, CT = NC / 16, KT = Qp / 4;
    const int ntiles = RT * CT;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    double* P = X + (size_t)Qp * NC;          // per instance: itaw, neq, th1, clock (4 x 16)

    // ---- load the group's populations into LDS (padding rows/columns zero)
    for (int e = threadIdx.x; e < Qp * NC; e += blockDim.x) X[e] = 0.0;
    __syncthreads();
    for (int i = 0; i < kGI; ++i) {
        if (gi[i] < 0) continue;
        InstDesc d = descs[gi[i]];
        rebase(d, fbase, wbase);
        const Tf* f = (const Tf*)d.f;
        for (int e = threadIdx.x; e < QL * Q; e += blockDim.x) {
            const int k = e / Q, j = e - k * Q;
            X[j * NC + i * QL + k] = (double)f[e];
        }
    }
    __syncthreads();

    // ---- f_n in registers, accumulator layout: tile t = w + kBW*u, element r
    //      sits at row 16*rt + lane/16 + 4*r, column 16*ct + lane%16 (the
    //      v_mfma_f64_16x16x4f64 result layout, checked on the device)
    double fn[kMaxTilesPerWave][4];
#pragma unroll
    for (int u = 0; u < kMaxTilesPerWave; ++u) {
        const int t = w + kBW * u;
        if (t < ntiles) {
            const int rt = t / CT, ct = t - rt * CT;
#pragma unroll
            for (int r = 0; r < 4; ++r) fn[u][r] = X[(16 * rt + (lane >> 4) + 4 * r) * NC + 16 * ct + (lane & 15)];
        }
    }

    const double* KPt = d0.tab.KPt;
    unsigned bad = 0;
    if (threadIdx.x < kGI) P[3 * kGI + threadIdx.x] =
        gi[threadIdx.x] >= 0 ? *((const double*)(wbase + (size_t)descs[gi[threadIdx.x]].clock)) : 1.0;
    __syncthreads();

    for (int it = 0; it < nsteps; ++it) {
#pragma unroll 1
        for (int st = 1; st <= 3; ++st) {
            // ---- per-instance moments and closure: 16 threads per instance
            {
                const int i = threadIdx.x >> 4, sub = threadIdx.x & 15;
                double n = 0.0, E = 0.0, PL = 0.0;
                if (gi[i] >= 0)
                    for (int e = sub; e < QL * Q; e += 16) {
                        const int j = e / QL, k = e - j * QL;
                        const double v = X[j * NC + i * QL + k], p = d0.tab.pk[k], x = d0.tab.xi[j];
                        n += v;
                        E += p * v;
                        PL += p * x * x * v;
                    }
#pragma unroll
                for (int o = 8; o > 0; o >>= 1) {
                    n += __shfl_xor(n, o, 16);
                    E += __shfl_xor(E, o, 16);
                    PL += __shfl_xor(PL, o, 16);
                }
                if (sub == 0) {
                    double itaw = 0.0, neq = 0.0, th1 = 0.0;
                    if (gi[i] >= 0) {
                        const InstDesc& d = descs[gi[i]];
                        const double P3 = E / 3.0;
                        double T = 1.0;
                        if (d.tau_mode != RSL_TAU_INF) {
                            if (d.gas == RSL_GAS_IDEAL) {
                                if (!(n > 0.0) || !(P3 > 0.0)) bad |= 1u;
                                T = P3 / n;
                                neq = n;
                                double taw = d.tau_r;
                                if (d.tau_mode == RSL_TAU_ETAS)
                                    taw = d.tau_aw0 / T * (1.0 - 0.25 * log(n / (T * T * T) * d.lambda_ref));
                                itaw = 1.0 / taw;
                            } else {
                                if (!(P3 > 0.0)) bad |= 1u;
                                T = sqrt(sqrt(P3));
                                neq = T * T * T;
                                itaw = 1.0 / (d.tau_mode == RSL_TAU_ETAS ? d.tau_aw0 / T : d.tau_r);
                            }
                        }
                        th1 = 1.0 - T / d.T0;
                    }
                    P[0 * kGI + i] = itaw;
                    P[1 * kGI + i] = neq;
                    P[2 * kGI + i] = th1;
                }
            }
            __syncthreads();

            // ---- K^P F on the matrix cores, then the vector epilogue
            double out[kMaxTilesPerWave][4];
#pragma unroll
            for (int u = 0; u < kMaxTilesPerWave; ++u) {
                const int t = w + kBW * u;
                if (t < ntiles) {
                    const int rt = t / CT, ct = t - rt * CT;
                    d4 acc = {0.0, 0.0, 0.0, 0.0};
                    const double* ap = KPt + ((size_t)rt * KT) * 64 + lane;
                    const int bcol = 16 * ct + (lane & 15);
                    for (int kk = 0; kk < KT; ++kk) {
                        const double a = ap[(size_t)kk * 64];
                        const double b = X[(4 * kk + (lane >> 4)) * NC + bcol];
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
                    }
                    const int col = bcol, i = col / QL, k = col - i * QL;
                    const bool live = gi[i] >= 0;
                    const double dti = live ? descs[gi[i]].dt : 0.0;
                    // stage time of instance i (Table II)
                    const double tst = P[3 * kGI + i] + it * dti + (st == 1 ? 0.0 : (st == 2 ? dti : 0.5 * dti));
                    const double ti = 1.0 / tst;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int j = 16 * rt + (lane >> 4) + 4 * r;
                        double o = 0.0;
                        if (live && j < Q) {
                            const double f = X[j * NC + col];
                            double sl = 0.0;
                            for (int kp = 0; kp < QL; ++kp) sl += d0.tab.KL[k * QL + kp] * X[j * NC + i * QL + kp];
                            const double x = d0.tab.xi[j];
                            double L = (-f + x * x * sl + acc[r]) * ti;
                            const double itaw = P[i], neq = P[kGI + i], th1 = P[2 * kGI + i];
                            const double feq = d0.tab.wxw[k * Q + j] * 0.25 * neq * (1.0 + th1 * d0.tab.L1[k]);
                            L -= (f - feq) * itaw;
                            if (st == 1) o = (double)(Tf)(fn[u][r] + dti * L);
                            else if (st == 2) o = (double)(Tf)(0.75 * fn[u][r] + 0.25 * f + 0.25 * dti * L);
                            else o = (double)(Tf)(kThird * fn[u][r] + kTwoThirds * (f + dti * L));
                        }
                        out[u][r] = o;
                    }
                }
            }
            __syncthreads();   // every read of the stage field is done
#pragma unroll
            for (int u = 0; u < kMaxTilesPerWave; ++u) {
                const int t = w + kBW * u;
                if (t < ntiles) {
                    const int rt = t / CT, ct = t - rt * CT;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        X[(16 * rt + (lane >> 4) + 4 * r) * NC + 16 * ct + (lane & 15)] = out[u][r];
                        if (st == 3) fn[u][r] = out[u][r];
                    }
                }
            }
            __syncthreads();
        }
    }

    // ---- write back, advance the clocks
    for (int i = 0; i < kGI; ++i) {
        if (gi[i] < 0) continue;
        InstDesc d = descs[gi[i]];
        rebase(d, fbase, wbase);
        Tf* f = (Tf*)d.f;
        for (int e = threadIdx.x; e < QL * Q; e += blockDim.x) {
            const int k = e / Q, j = e - k * Q;
            const double v = X[j * NC + i * QL + k];
            if (!isfinite(v)) bad |= 2u;
            f[e] = (Tf)v;
        }
        __syncthreads();
        if (threadIdx.x == 0) *d.clock = P[3 * kGI + i] + nsteps * d.dt;
        if (bad) atomicOr(d.status, bad);
    }
}

}  // namespace

size_t bj_mfma_lds_bytes(int Q, int QL) {
    const size_t Qp = (size_t)(Q + 15) / 16 * 16;
    return sizeof(double) * (Qp * kGI * QL + 4 * kGI);
}

bool bj_mfma_fits(int Q, int QL) {
    const int tiles = (Q + 15) / 16 * QL;     // (Qp/16) x (16 QL / 16)
    return QL >= 1 && QL <= 4 && tiles <= kBW * kMaxTilesPerWave && bj_mfma_lds_bytes(Q, QL) <= 150 * 1024;
}

int launch_bj_mfma(const InstDesc* descs, const int* groups, int ngroups, size_t lds, int dtype, char* fbase,
                   char* wbase, int nsteps, hipStream_t s) {
    static const hipError_t a64 = hipFuncSetAttribute((const void*)bj_mfma_kernel<double>,
                                                      hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    static const hipError_t a32 = hipFuncSetAttribute((const void*)bj_mfma_kernel<float>,
                                                      hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    if (a64 != hipSuccess) return hip_check(a64, "hipFuncSetAttribute(bj_mfma_kernel)");
    if (a32 != hipSuccess) return hip_check(a32, "hipFuncSetAttribute(bj_mfma_kernel)");
    if (dtype == RSL_F64)
        hipLaunchKernelGGL(bj_mfma_kernel<double>, dim3(ngroups), dim3(kBW * 64), lds, s, descs, groups, fbase, wbase,
                           nsteps);
    else
        hipLaunchKernelGGL(bj_mfma_kernel<float>, dim3(ngroups), dim3(kBW * 64), lds, s, descs, groups, fbase, wbase,
                           nsteps);
    return hip_check(hipGetLastError(), "bj_mfma_kernel launch");
}

}  // namespace rsl
