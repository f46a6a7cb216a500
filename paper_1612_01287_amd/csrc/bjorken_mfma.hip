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
// One workgroup (8 waves) owns one group for all requested steps: the stage
// field F lives in LDS (row j, column i Q_L + k), f_n in registers in the
// accumulator layout of the row blocks each wave owns, K^P streams from
// global memory pre-arranged in A-operand tile order (one coalesced 512-byte
// load per wave, row block and k-step, issued four to eight k-steps ahead and
// shared by the Q_L column tiles of the row block).
#include <hip/hip_runtime.h>

#include "rsl_math.h"

namespace rsl {

namespace {

constexpr int kGI = 16;        // instances per group
constexpr int kBW = 8;         // waves per workgroup
constexpr int kTPI = kBW * 64 / kGI;   // threads per instance in the moment sums
constexpr int kMaxRB = 2;      // 16-row blocks of K^P F per wave (Q_xi <= 256)
constexpr int kMaxCT = 4;      // 16-column tiles per row block (Q_L <= 4)
static_assert(kMaxRB == 2, "the product loop below is written for two row blocks per wave");
// k-steps per block of A-fragment loads: deeper for fewer column tiles (less
// matrix-core work per k-step to cover the latency, fewer accumulators),
// shallower at Q_L = 4, whose accumulators and f_n leave fewer registers
template <int QL, int NT>
constexpr int kPD = QL >= 4 ? (NT == 1 ? 4 : 2) : (NT == 1 ? 8 : 4);

typedef double d4 __attribute__((ext_vector_type(4)));

// K^P F over the first NT column tiles for row block w (and w + kBW when TWO)
// of one wave: the row blocks advance together, so that the B fragments of a
// k-step (LDS) serve both, and one A fragment serves every column tile; the A
// fragments (K^P in A-operand tile order, from the L2 or HBM, far slower than
// one k-step) are loaded 2-8 k-steps ahead.
template <int QL, int NT, bool TWO, int CT>
__device__ __forceinline__ void kp_product(d4 (&acc)[kMaxRB][CT], const double* X, const double* KPt, int w,
                                           int lane, int KT) {
    constexpr int NC = kGI * QL;
    constexpr int PD = kPD<QL, NT>;
    const double* ap0 = KPt + ((size_t)w * KT) * 64 + lane;
    const double* ap1 = KPt + ((size_t)(w + (TWO ? kBW : 0)) * KT) * 64 + lane;
    double a0[PD], a1[PD];
#pragma unroll
    for (int p = 0; p < PD; ++p) {
        const size_t k0 = (size_t)min(p, KT - 1) * 64;
        a0[p] = ap0[k0];
        if (TWO) a1[p] = ap1[k0];
    }
    // KT is a multiple of 4 (Q_xi is padded to 16 rows); a block of 8 may
    // overhang it by 4 (loads clamped, products skipped)
    for (int kb = 0; kb < KT; kb += PD) {
        double n0[PD], n1[PD];
#pragma unroll
        for (int p = 0; p < PD; ++p) {
            const size_t kn = (size_t)min(kb + PD + p, KT - 1) * 64;
            n0[p] = ap0[kn];
            if (TWO) n1[p] = ap1[kn];
        }
#pragma unroll
        for (int p = 0; p < PD; ++p) {
            if (PD > 4 && kb + p >= KT) break;
            const double* brow = X + (4 * (kb + p) + (lane >> 4)) * NC + (lane & 15);
            double b[NT];
#pragma unroll
            for (int ct = 0; ct < NT; ++ct) b[ct] = brow[16 * ct];
#pragma unroll
            for (int ct = 0; ct < NT; ++ct)
                acc[0][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[p], b[ct], acc[0][ct], 0, 0, 0);
            if (TWO) {
#pragma unroll
                for (int ct = 0; ct < NT; ++ct)
                    acc[1][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[p], b[ct], acc[1][ct], 0, 0, 0);
            }
        }
#pragma unroll
        for (int p = 0; p < PD; ++p) {
            a0[p] = n0[p];
            if (TWO) a1[p] = n1[p];
        }
    }
}

// The product with the group's live column tiles (nct, wave-uniform) as a
// compile-time count: no per-MFMA branches.
template <int QL, bool TWO, int CT>
__device__ __forceinline__ void kp_product_nt(d4 (&acc)[kMaxRB][CT], const double* X, const double* KPt, int w,
                                              int lane, int KT, int nct) {
    if (nct >= CT) kp_product<QL, CT, TWO>(acc, X, KPt, w, lane, KT);
    else if (nct == 1) kp_product<QL, 1, TWO>(acc, X, KPt, w, lane, KT);
    else if constexpr (CT > 2) {
        if (nct == 2) kp_product<QL, 2, TWO>(acc, X, KPt, w, lane, KT);
        else if constexpr (CT > 3) kp_product<QL, 3, TWO>(acc, X, KPt, w, lane, KT);
    }
}

// Orders one wave's LDS accesses (LDS executes a wave's instructions in issue
// order, so keeping the compiler from moving them across is enough).
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename Tf, int QL>
__global__ void __launch_bounds__(kBW * 64) bj_mfma_kernel(const InstDesc* __restrict__ descs,
                                                           const int* __restrict__ groups, char* fbase,
                                                           char* wbase, int nsteps) {
    extern __shared__ double X[];   // [Qp][NC] stage field, then per-instance scalars and tables
    const int* gi = groups + blockIdx.x * kGI;
    const InstDesc d0 = descs[gi[0]];
    constexpr int NC = kGI * QL, CT = QL;      // one 16-column tile per radial node
    const int Q = d0.Q;
    const int Qp = (Q + 15) & ~15;
    const int RT = Qp / 16, KT = Qp / 4;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    // live instances come first in a group; column tiles past the last live
    // column are skipped (groups smaller than 16 shorten the critical path of
    // a batch with a few large velocity sets)
    int nlive = 0;
    while (nlive < kGI && gi[nlive] >= 0) ++nlive;
    const int nct = __builtin_amdgcn_readfirstlane((nlive * QL + 15) / 16);
    double* P = X + (size_t)Qp * NC;          // per instance: itaw, neq, th1, clock, dt, tau mode, gas,
                                              // tau_r, tau_aw0, lambda_ref, T0, 1 / stage time (12 x 16)
    // status bits of each instance (bit 0: unphysical state met by its
    // closure; bit 1: a non-finite population written back), one word each
    unsigned* flag = (unsigned*)(P + 12 * kGI);
    // velocity-set tables read by the epilogue (from LDS, so that the
    // compiler does not keep per-element copies in registers across steps)
    double* Tx2 = P + 13 * kGI;               // [Qp]      xi_j^2
    double* Tw = Tx2 + Qp;                    // [QL][Qp]  w_j w_k / 4
    double* TL1 = Tw + (size_t)QL * Qp;       // [QL]      L_1(pbar_k)
    double* TKL = TL1 + QL;                   // [QL][QL]  K^L
    double* Tpk = TKL + QL * QL;              // [QL]      p_k
    for (int e = threadIdx.x; e < Qp; e += blockDim.x) {
        const double x = e < Q ? d0.tab.xi[e] : 0.0;
        Tx2[e] = x * x;
    }
    for (int e = threadIdx.x; e < QL * Qp; e += blockDim.x) {
        const int k = e / Qp, j = e - k * Qp;
        Tw[e] = j < Q ? 0.25 * d0.tab.wxw[k * Q + j] : 0.0;
    }
    for (int e = threadIdx.x; e < QL; e += blockDim.x) TL1[e] = d0.tab.L1[e];
    for (int e = threadIdx.x; e < QL * QL; e += blockDim.x) TKL[e] = d0.tab.KL[e];
    for (int e = threadIdx.x; e < QL; e += blockDim.x) Tpk[e] = d0.tab.pk[e];

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

    // ---- f_n in registers, accumulator layout: row block rb = w + kBW u,
    //      column tile ct, element r at row 16 rb + lane/16 + 4 r, column
    //      16 ct + lane%16 (the v_mfma_f64_16x16x4f64 result layout, checked
    //      on the device)
    double fn[kMaxRB][CT][4];
#pragma unroll
    for (int u = 0; u < kMaxRB; ++u) {
        const int rb = w + kBW * u;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
            if (rb < RT) {
#pragma unroll
                for (int r = 0; r < 4; ++r) fn[u][ct][r] = X[(16 * rb + (lane >> 4) + 4 * r) * NC + 16 * ct + (lane & 15)];
            }
    }

    const double* KPt = d0.tab.KPt;
    if (threadIdx.x < kGI) {
        flag[threadIdx.x] = 0u;
        const int i = threadIdx.x;
        const bool live = gi[i] >= 0;
        const InstDesc& d = descs[live ? gi[i] : gi[0]];
        P[3 * kGI + i] = live ? *((const double*)(wbase + (size_t)d.clock)) : 1.0;
        P[4 * kGI + i] = live ? d.dt : 0.0;
        P[5 * kGI + i] = (double)d.tau_mode;
        P[6 * kGI + i] = (double)d.gas;
        P[7 * kGI + i] = d.tau_r;
        P[8 * kGI + i] = d.tau_aw0;
        P[9 * kGI + i] = d.lambda_ref;
        P[10 * kGI + i] = d.T0;
    }
    __syncthreads();

    for (int it = 0; it < nsteps; ++it) {
#pragma unroll 1
        for (int st = 1; st <= 3; ++st) {
            // ---- per-instance moments and closure: kTPI threads per instance
            {
                const int i = threadIdx.x / kTPI, sub = threadIdx.x % kTPI;
                double n = 0.0, E = 0.0;
                if (gi[i] >= 0)
                    for (int e = sub; e < QL * Q; e += kTPI) {
                        const int j = e / QL, k = e - j * QL;
                        const double v = X[j * NC + i * QL + k];
                        n += v;
                        E += Tpk[k] * v;
                    }
#pragma unroll
                for (int o = kTPI / 2; o > 0; o >>= 1) {
                    n += __shfl_xor(n, o, kTPI);
                    E += __shfl_xor(E, o, kTPI);
                }
                if (sub == 0) {
                    double itaw = 0.0, neq = 0.0, th1 = 0.0;
                    unsigned bad = 0;
                    if (gi[i] >= 0) {
                        // the instance's parameters, staged in LDS at the start
                        const int mode = (int)P[5 * kGI + i], gas = (int)P[6 * kGI + i];
                        const double tau_r = P[7 * kGI + i], tau_aw0 = P[8 * kGI + i];
                        const double lambda_ref = P[9 * kGI + i], T0 = P[10 * kGI + i];
                        const double P3 = E / 3.0;
                        double T = 1.0;
                        if (mode != RSL_TAU_INF) {
                            if (gas == RSL_GAS_IDEAL) {
                                if (!(n > 0.0) || !(P3 > 0.0)) bad |= 1u;
                                T = P3 / n;
                                neq = n;
                                double taw = tau_r;
                                if (mode == RSL_TAU_ETAS)
                                    taw = tau_aw0 / T * (1.0 - 0.25 * log(n / (T * T * T) * lambda_ref));
                                itaw = 1.0 / taw;
                            } else {
                                if (!(P3 > 0.0)) bad |= 1u;
                                T = sqrt(sqrt(P3));
                                neq = T * T * T;
                                itaw = 1.0 / (mode == RSL_TAU_ETAS ? tau_aw0 / T : tau_r);
                            }
                        }
                        th1 = 1.0 - T / T0;
                    }
                    if (bad) flag[i] |= bad;   // only this thread writes instance i's word here
                    P[0 * kGI + i] = itaw;
                    P[1 * kGI + i] = neq;
                    P[2 * kGI + i] = th1;
                    // stage time of the instance (Table II)
                    const double dti = P[4 * kGI + i];
                    P[11 * kGI + i] = 1.0 / (P[3 * kGI + i] + it * dti + (st == 1 ? 0.0 : (st == 2 ? dti : 0.5 * dti)));
                }
            }
            __syncthreads();

            // ---- K^P F on the matrix cores
            d4 acc[kMaxRB][CT];
#pragma unroll
            for (int u = 0; u < kMaxRB; ++u)
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) acc[u][ct] = d4{0.0, 0.0, 0.0, 0.0};
            if (w < RT) {
                const bool two = w + kBW < RT;   // wave-uniform
                if (two) kp_product_nt<QL, true>(acc, X, KPt, w, lane, KT, nct);
                else kp_product_nt<QL, false>(acc, X, KPt, w, lane, KT, nct);
            }
            __syncthreads();   // every read of the stage field by the products is done

            // ---- vector epilogue, in place: the rows of a row block belong to
            //      one wave, which reads all of them before writing any
#pragma unroll
            for (int u = 0; u < kMaxRB; ++u) {
                const int rb = w + kBW * u;
                if (rb >= RT) continue;
                double out[CT][4];
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) {
                    const int col = 16 * ct + (lane & 15), i = col / QL, k = col - i * QL;
                    const bool live = ct < nct && gi[i] >= 0;
                    const double dti = P[4 * kGI + i];
                    const double ti = P[11 * kGI + i];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int j = 16 * rb + (lane >> 4) + 4 * r;
                        double o = 0.0;
                        if (live && j < Q) {
                            const double f = X[j * NC + col];
                            double sl = 0.0;
                            for (int kp = 0; kp < QL; ++kp) sl += TKL[k * QL + kp] * X[j * NC + i * QL + kp];
                            double L = (-f + Tx2[j] * sl + acc[u][ct][r]) * ti;
                            const double itaw = P[i], neq = P[kGI + i], th1 = P[2 * kGI + i];
                            const double feq = Tw[k * Qp + j] * neq * (1.0 + th1 * TL1[k]);
                            L -= (f - feq) * itaw;
                            if (st == 1) o = (double)(Tf)(fn[u][ct][r] + dti * L);
                            else if (st == 2) o = (double)(Tf)(0.75 * fn[u][ct][r] + 0.25 * f + 0.25 * dti * L);
                            else o = (double)(Tf)(kThird * fn[u][ct][r] + kTwoThirds * (f + dti * L));
                        }
                        out[ct][r] = o;
                    }
                }
                wave_sync_lds();
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            X[(16 * rb + (lane >> 4) + 4 * r) * NC + 16 * ct + (lane & 15)] = out[ct][r];
                            if (st == 3) fn[u][ct][r] = out[ct][r];
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
        int nonfinite = 0;
        for (int e = threadIdx.x; e < QL * Q; e += blockDim.x) {
            const int k = e / Q, j = e - k * Q;
            const double v = X[j * NC + i * QL + k];
            if (!isfinite(v)) nonfinite = 1;
            f[e] = (Tf)v;
        }
        // this instance's flags only: its closure's word and its own populations
        const unsigned bad = flag[i] | (__syncthreads_or(nonfinite) ? 2u : 0u);
        if (threadIdx.x == 0) {
            *d.clock = P[3 * kGI + i] + nsteps * d.dt;
            if (bad) atomicOr(d.status, bad);
        }
    }
}

}  // namespace

size_t bj_mfma_lds_bytes(int Q, int QL) {
    const size_t Qp = (size_t)(Q + 15) / 16 * 16;
    return sizeof(double) * (Qp * kGI * QL + 13 * kGI + Qp * (1 + QL) + 2 * QL + QL * QL);
}

bool bj_mfma_fits(int Q, int QL) {
    const int RT = (Q + 15) / 16;
    return QL >= 1 && QL <= kMaxCT && RT <= kBW * kMaxRB && bj_mfma_lds_bytes(Q, QL) <= 150 * 1024;
}

template <typename Tf, int QL>
int launch_bj_mfma_t(const InstDesc* descs, const int* groups, int ngroups, size_t lds, char* fbase, char* wbase,
                     int nsteps, hipStream_t s) {
    static const hipError_t attr = hipFuncSetAttribute((const void*)bj_mfma_kernel<Tf, QL>,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    if (attr != hipSuccess) return hip_check(attr, "hipFuncSetAttribute(bj_mfma_kernel)");
    hipLaunchKernelGGL((bj_mfma_kernel<Tf, QL>), dim3(ngroups), dim3(kBW * 64), lds, s, descs, groups, fbase, wbase,
                       nsteps);
    return hip_check(hipGetLastError(), "bj_mfma_kernel launch");
}

template <typename Tf>
int launch_bj_mfma_q(int QL, const InstDesc* descs, const int* groups, int ngroups, size_t lds, char* fbase,
                     char* wbase, int nsteps, hipStream_t s) {
    switch (QL) {
        case 1: return launch_bj_mfma_t<Tf, 1>(descs, groups, ngroups, lds, fbase, wbase, nsteps, s);
        case 2: return launch_bj_mfma_t<Tf, 2>(descs, groups, ngroups, lds, fbase, wbase, nsteps, s);
        case 3: return launch_bj_mfma_t<Tf, 3>(descs, groups, ngroups, lds, fbase, wbase, nsteps, s);
        case 4: return launch_bj_mfma_t<Tf, 4>(descs, groups, ngroups, lds, fbase, wbase, nsteps, s);
        default: return set_error(RSL_EUNSUPPORTED, "matrix-core Bjorken path: Q_L > 4");
    }
}

int launch_bj_mfma(const InstDesc* descs, const int* groups, int ngroups, int QL, size_t lds, int dtype, char* fbase,
                   char* wbase, int nsteps, hipStream_t s) {
    if (dtype == RSL_F64) return launch_bj_mfma_q<double>(QL, descs, groups, ngroups, lds, fbase, wbase, nsteps, s);
    return launch_bj_mfma_q<float>(QL, descs, groups, ngroups, lds, fbase, wbase, nsteps, s);
}

}  // namespace rsl
