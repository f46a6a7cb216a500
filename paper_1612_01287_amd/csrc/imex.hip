// An implicit-explicit time step of the Sod operator (eq. L_Sod), so that dt is
// not bound by the relaxation time (the option Sec. I names in place of
// dt < tau_AW; Sec. III F): the WENO5 advection explicit, the Anderson-Witting
// term implicit, in the IMEX-SSP2(2,2,2) scheme of Pareschi and Russo
// (g = 1 - 1/sqrt(2)):
//   F1 = f + g dt Q(F1)
//   F2 = f + dt A(F1) + (1 - 2g) dt Q(F1) + g dt Q(F2)
//   f' = f + dt/2 (A(F1) + A(F2)) + dt/2 (Q(F1) + Q(F2)),
// Q(F1) = (F1 - f) / (g dt), Q(F2) = (F2 - F2*) / (g dt).
//
// An implicit stage G = F + h Q(G) is solved cell by cell: the collision has
// no N^0, T^00, T^0z (they are its zero moments in the Landau frame of G), so
// G keeps those of F and the unknowns are X = (N^z, T^zz) of G.  For a guess X
// the frame of (N^0, X_0, T^00, T^0z, X_1) gives c_j = gamma (1 - beta xi_j)
// / tau and f^eq, and G = (F + h c f^eq) / (1 + h c); the guess must reproduce
// itself.  Broyden's method from the moments of F, started with a
// finite-difference Jacobian.  c_j does not depend on the radial node, so an evaluation needs the
// radial sums of F (once) and two radial sums of f^eq per angular node,
// which follow from g_j, h_j and fixed quadrature sums; L lanes share a
// cell, each taking every L-th angular node.
//
// Fields (binary64): f the state, F1 in the work buffer's first stage slot,
// F2* then F2 (in place) in the second.
#include <hip/hip_runtime.h>

#include <cmath>

#include "rsl_impl.h"
#include "rsl_math.h"

namespace rsl {

namespace {

constexpr int kImexThreads = 64;
constexpr double kImexG = 0.29289321881345247560;   // 1 - 1/sqrt(2)

struct Frame {
    CellState cs;
    double rate;                       // gamma / tau (0 when collisionless)
    double c0[kMaxNOm + 1], c1[kMaxNOm + 1];
};

template <typename TP>
__device__ __forceinline__ bool frame_of(const InstDesc& d, double N0, double Nz, double T00, double T0z, double Tzz, TP ser,
                         TP thr, Frame& fr) {
    fr.cs = landau(N0, Nz, T00, T0z, Tzz);
    if (!fr.cs.ok) return false;
    const CellState& cs = fr.cs;
    double tau = d.tau_r;
    if (d.tau_mode == RSL_TAU_ETAS)
        tau = d.tau_aw0 / cs.T * (1.0 - 0.25 * log(cs.n / (cs.T * cs.T * cs.T) * d.lambda_ref));
    fr.rate = d.tau_mode == RSL_TAU_INF ? 0.0 : cs.gamma / tau;
    const int nt = series_terms_uniform(fmin(cs.beta * cs.beta, d.beta_series * d.beta_series), thr);
    feq_coef(cs.n, cs.T, cs.beta, cs.gamma, d.T0, d.NOm, d.beta_series, ser, nt, fr.c0, fr.c1);
    return true;
}

// Sum over the L lanes of a cell's group (xor butterfly: every lane of the
// group ends with the same bits, since each addition pairs the same operands).
template <int L>
__device__ __forceinline__ double group_sum(double x) {
#pragma unroll
    for (int o = 1; o < L; o <<= 1) x += __shfl_xor(x, o, L);
    return x;
}

// A lane's angular nodes j = r + i L (i < JM) with what an evaluation needs
// of them that does not depend on the frame: xi_j, the radial sums a_j =
// sum_k F_jk, b_j = sum_k p_k F_jk of the cell, the quadrature sums
// w0..w3 = sum_k w_j w_k {1, L_1(pbar_k), p_k, p_k L_1(pbar_k)}, and (for
// JM <= 2) P_m(xi_j).  Nodes past Q_xi carry zeros.
template <int JM>
struct LaneNodes {
    double x[JM], a[JM], b[JM], w0[JM], w1[JM], w2[JM], w3[JM];
    double P[JM <= 2 ? JM : 1][kMaxNOm + 1];
};

template <int L, int JM>
__device__ __forceinline__ void load_nodes(const InstDesc& d, const double* __restrict__ F, int s, int r, LaneNodes<JM>& n) {
#pragma unroll
    for (int i = 0; i < JM; ++i) {
        const int j = r + i * L;
        n.x[i] = n.a[i] = n.b[i] = n.w0[i] = n.w1[i] = n.w2[i] = n.w3[i] = 0.0;
        if (j >= d.Q) continue;
        n.x[i] = d.tab.xi[j];
        for (int k = 0; k < d.QL; ++k) {
            const int v = k * d.Q + j;
            const double fv = F[(size_t)v * d.pitch + s], w = d.tab.wxw[v], p = d.tab.pk[k], l1 = d.tab.L1[k];
            n.a[i] += fv;
            n.b[i] = fma(p, fv, n.b[i]);
            n.w0[i] += w;
            n.w1[i] = fma(w, l1, n.w1[i]);
            n.w2[i] = fma(w, p, n.w2[i]);
            n.w3[i] = fma(w * p, l1, n.w3[i]);
        }
        if constexpr (JM <= 2) {
#pragma unroll
            for (int m = 0; m <= kMaxNOm; ++m) n.P[i][m] = m <= d.NOm ? d.tab.Pm[(size_t)m * d.Q + j] : 0.0;
        }
    }
}

// (N^z, T^zz) of the relaxed stage G = (F + h c f^eq) / (1 + h c) for the
// frame fr, summed over the cell's group of L lanes.
template <int L, int JM>
__device__ __forceinline__ void relaxed_moments(const InstDesc& d, const LaneNodes<JM>& n, int r, const Frame& fr, double h,
                                double (&out)[2]) {
    double nzs = 0.0, tzz = 0.0;
#pragma unroll
    for (int i = 0; i < JM; ++i) {
        const int j = min(r + i * L, d.Q - 1);          // past Q_xi: any node (the sums are zero)
        double g = 0.0, hh = 0.0;
#pragma unroll
        for (int m = 0; m <= kMaxNOm; ++m) {       // fixed bounds keep c0, c1 in registers
            if (m > d.NOm) break;
            double P;
            if constexpr (JM <= 2) P = n.P[i][m];
            else P = d.tab.Pm[(size_t)m * d.Q + j];
            g = fma(P, fr.c0[m], g);
            hh = fma(P, fr.c1[m], hh);
        }
        const double e0 = fma(g, n.w0[i], hh * n.w1[i]), e1 = fma(g, n.w2[i], hh * n.w3[i]);
        const double hc = h * fr.rate * (1.0 - fr.cs.beta * n.x[i]);
        const double den = 1.0 / (1.0 + hc);
        nzs = fma(n.x[i], fma(hc, e0, n.a[i]) * den, nzs);
        tzz = fma(n.x[i] * n.x[i], fma(hc, e1, n.b[i]) * den, tzz);
    }
    out[0] = group_sum<L>(nzs);
    out[1] = group_sum<L>(tzz);
}

// One cell per group of L lanes; the groups of a wave are independent and
// every lane of a group takes the same branches (its sums are bitwise equal).
template <int L, int JM>
__global__ void __launch_bounds__(kImexThreads) imex_implicit_kernel(InstDesc d, const double* Fs, double* G,
                                                                      double h) {
    const int r = threadIdx.x % L;
    const int s0 = blockIdx.x * (kImexThreads / L) + threadIdx.x / L;
    const bool live = s0 < d.nz;
    const int s = live ? s0 : d.nz - 1;           // dead groups repeat the last cell and store nothing
    // the Maclaurin tables of K_{3,m}, K_{4,m} in LDS (read by every frame)
    constexpr int kSer = kSeriesTerms * 2 * (kMaxNOm + 1);
    __shared__ double ser[kSer], thr[kSeriesTerms];
    for (int i = threadIdx.x; i < kSer; i += kImexThreads) ser[i] = d.tab.ser[i];
    for (int i = threadIdx.x; i < kSeriesTerms; i += kImexThreads) thr[i] = d.tab.thr[i];
    __syncthreads();
    LaneNodes<JM> nd;
    load_nodes<L, JM>(d, Fs, s, r, nd);
    double M[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < JM; ++i) {
        M[0] += nd.a[i];
        M[1] = fma(nd.x[i], nd.a[i], M[1]);
        M[2] += nd.b[i];
        M[3] = fma(nd.x[i], nd.b[i], M[3]);
        M[4] = fma(nd.x[i] * nd.x[i], nd.b[i], M[4]);
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) M[i] = group_sum<L>(M[i]);
    double X[2] = {M[1], M[4]};
    const double sc[2] = {fabs(M[0]), fabs(M[2])};   // scales of the two unknowns
    // Broyden's method: a finite-difference Jacobian of R(X) = (relaxed
    // moments - X) at the start, rank-one updates after each step above
    // 1e-10 of the scales; one more step once a step is at 1e-13 of them
    Frame fr;
    bool ok = frame_of(d, M[0], X[0], M[2], M[3], X[1], ser, thr, fr), conv = false;
    double R[2] = {0.0, 0.0}, J[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    if (ok) {
        double r0[2], rp[2], rq[2];
        relaxed_moments<L, JM>(d, nd, r, fr, h, r0);
        const double e0 = 1e-7 * sc[0], e1 = 1e-7 * sc[1];
        ok = frame_of(d, M[0], X[0] + e0, M[2], M[3], X[1], ser, thr, fr);
        if (ok) relaxed_moments<L, JM>(d, nd, r, fr, h, rp);
        ok = ok && frame_of(d, M[0], X[0], M[2], M[3], X[1] + e1, ser, thr, fr);
        if (ok) {
            relaxed_moments<L, JM>(d, nd, r, fr, h, rq);
            R[0] = r0[0] - X[0];
            R[1] = r0[1] - X[1];
            J[0][0] = (rp[0] - r0[0]) / e0 - 1.0;
            J[1][0] = (rp[1] - r0[1]) / e0;
            J[0][1] = (rq[0] - r0[0]) / e1;
            J[1][1] = (rq[1] - r0[1]) / e1 - 1.0;
        }
    }
    bool last = false;
    for (int it = 0; it < 40 && ok && !conv; ++it) {
        const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        if (!(fabs(det) > 0.0)) { ok = false; break; }
        const double s0 = -(J[1][1] * R[0] - J[0][1] * R[1]) / det;
        const double s1 = -(J[0][0] * R[1] - J[1][0] * R[0]) / det;
        X[0] += s0;
        X[1] += s1;
        if (!frame_of(d, M[0], X[0], M[2], M[3], X[1], ser, thr, fr)) { ok = false; break; }
        if (last) { conv = true; break; }            // fr is the frame of the final X
        last = fabs(s0) <= 1e-13 * sc[0] && fabs(s1) <= 1e-13 * sc[1];
        double rn[2];
        relaxed_moments<L, JM>(d, nd, r, fr, h, rn);
        const double y0 = rn[0] - X[0] - R[0], y1 = rn[1] - X[1] - R[1];
        R[0] = rn[0] - X[0];
        R[1] = rn[1] - X[1];
        // no update from steps near the rounding level of R (its differences
        // are noise there): the last Jacobian is kept
        if (fabs(s0) <= 1e-10 * sc[0] && fabs(s1) <= 1e-10 * sc[1]) continue;
        const double ss = s0 * s0 + s1 * s1;
        const double u0 = (y0 - (J[0][0] * s0 + J[0][1] * s1)) / ss;
        const double u1 = (y1 - (J[1][0] * s0 + J[1][1] * s1)) / ss;
        J[0][0] += u0 * s0;
        J[0][1] += u0 * s1;
        J[1][0] += u1 * s0;
        J[1][1] += u1 * s1;
    }
    if (!live) return;
    if (!ok || !conv) {
        if (r == 0) atomicOr(d.status, 1u);
        for (int j = r; j < d.Q; j += L)
            for (int k = 0; k < d.QL; ++k) G[(size_t)(k * d.Q + j) * d.pitch + s] = __builtin_nan("");
        return;
    }
    for (int j = r; j < d.Q; j += L) {
        double g = 0.0, hh = 0.0;
#pragma unroll
        for (int m = 0; m <= kMaxNOm; ++m) {
            if (m > d.NOm) break;
            const double P = d.tab.Pm[(size_t)m * d.Q + j];
            g = fma(P, fr.c0[m], g);
            hh = fma(P, fr.c1[m], hh);
        }
        const double hc = h * fr.rate * (1.0 - fr.cs.beta * d.tab.xi[j]);
        const double den = 1.0 / (1.0 + hc);
        for (int k = 0; k < d.QL; ++k) {
            const int v = k * d.Q + j;
            const double fe = d.tab.wxw[v] * fma(d.tab.L1[k], hh, g);
            const double fv = Fs[(size_t)v * d.pitch + s];
            G[(size_t)v * d.pitch + s] = fma(hc, fe, fv) * den;
        }
    }
}

// Population of velocity v at cell c (ghosts per the instance's rule).
__device__ __forceinline__ double at(const InstDesc& d, const double* F, int v, int c) {
    if (c < 0) return d.bc == RSL_BC_EQ ? d.feqL[v] : F[(size_t)v * d.pitch];
    if (c >= d.nz) return d.bc == RSL_BC_EQ ? d.feqR[v] : F[(size_t)v * d.pitch + d.nz - 1];
    return F[(size_t)v * d.pitch + c];
}

// A(F) at cell s, velocity v: -(Phi_{s+1/2} - Phi_{s-1/2}) / dz with the WENO5
// flux Phi = xi_j weno5(upwind stencil) (Sec. III F).
__device__ double advection(const InstDesc& d, const double* F, int v, int s) {
    const double x = d.tab.xv[v];
    if (x == 0.0) return 0.0;
    double u[7];
    for (int q = 0; q < 7; ++q) u[q] = at(d, F, v, s - 3 + q);
    double fp, fm;
    if (x > 0.0) {
        fp = weno5(u[1], u[2], u[3], u[4], u[5]);
        fm = weno5(u[0], u[1], u[2], u[3], u[4]);
    } else {
        fp = weno5(u[6], u[5], u[4], u[3], u[2]);
        fm = weno5(u[5], u[4], u[3], u[2], u[1]);
    }
    return -x * (fp - fm) * d.dz_inv;
}

// mode 0: F2* = f + dt A(F1) + (1 - 2g)/g (F1 - f) into the second slot;
// mode 1: f <- f + dt/2 (A(F1) + A(F2)) + (F1 - f)/(2g) + (F2 - F2*)/(2g),
// F2* recomputed from f, F1 and A(F1).  One thread per (cell, velocity v =
// blockIdx.y).
__global__ void __launch_bounds__(kImexThreads) imex_explicit_kernel(InstDesc d, int mode) {
    const int s = blockIdx.x * kImexThreads + threadIdx.x;
    const int v = blockIdx.y;
    if (s >= d.nz) return;
    double* f = (double*)d.f;
    const double* F1 = (const double*)d.f1;
    double* F2 = (double*)d.f2;
    const double dt = d.dt, g = kImexG;
    const size_t i = (size_t)v * d.pitch + s;
    const double fn = f[i], f1 = F1[i];
    const double a1 = advection(d, F1, v, s);
    const double fs2 = fn + dt * a1 + (1.0 - 2.0 * g) / g * (f1 - fn);
    if (mode == 0) {
        F2[i] = fs2;
    } else {
        const double a2 = advection(d, F2, v, s);
        const double out = fn + 0.5 * dt * (a1 + a2) + (f1 - fn) / (2.0 * g) + (F2[i] - fs2) / (2.0 * g);
        if (!isfinite(out)) atomicOr(d.status, 2u);
        f[i] = out;
    }
}

}  // namespace

template <int L, int JM>
static void implicit_stage(const InstDesc& d, const double* F, double* G, double h, hipStream_t s) {
    const int cells = kImexThreads / L;
    hipLaunchKernelGGL((imex_implicit_kernel<L, JM>), dim3((d.nz + cells - 1) / cells), dim3(kImexThreads), 0, s,
                       d, F, G, h);
}

int launch_imex_steps(const InstDesc& d, int nsteps, hipStream_t s) {
    const dim3 gx((d.nz + kImexThreads - 1) / kImexThreads, d.V);
    const double h = kImexG * d.dt;
    // lanes per cell: enough to cover the angular nodes, at most a wave;
    // past 64 nodes each lane takes up to 16 (Q_xi <= 1024)
    using Stage = void (*)(const InstDesc&, const double*, double*, double, hipStream_t);
    const Stage stage = d.Q <= 4    ? implicit_stage<4, 1>
                        : d.Q <= 8   ? implicit_stage<8, 1>
                        : d.Q <= 16  ? implicit_stage<16, 1>
                        : d.Q <= 32  ? implicit_stage<32, 1>
                        : d.Q <= 64  ? implicit_stage<64, 1>
                        : d.Q <= 128 ? implicit_stage<64, 2>
                        : d.Q <= 256 ? implicit_stage<64, 4>
                        : d.Q <= 512 ? implicit_stage<64, 8>
                                     : implicit_stage<64, 16>;
    for (int it = 0; it < nsteps; ++it) {
        stage(d, (const double*)d.f, (double*)d.f1, h, s);
        hipLaunchKernelGGL(imex_explicit_kernel, gx, dim3(kImexThreads), 0, s, d, 0);
        stage(d, (const double*)d.f2, (double*)d.f2, h, s);
        hipLaunchKernelGGL(imex_explicit_kernel, gx, dim3(kImexThreads), 0, s, d, 1);
    }
    return hip_check(hipGetLastError(), "imex step launch");
}

}  // namespace rsl
