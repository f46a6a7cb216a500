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
// Fields (binary64 or binary32 storage, arithmetic in binary64): f the state,
// F1 in the work buffer's first stage slot, F2* then F2 (in place) in the
// second.  One instance per call, or a Sod batch (work items of one instance
// each, per lanes-per-cell class).
#include <hip/hip_runtime.h>

#include <cmath>

#include "imex.h"
#include "rsl_impl.h"
#include "rsl_math.h"

namespace rsl {

namespace {

constexpr int kImexThreads = 64;        // single-instance workgroups
constexpr int kImexBatchThreads = 256;  // batch implicit-stage workgroups (one instance each)
constexpr double kImexG = 0.29289321881345247560;   // 1 - 1/sqrt(2)

struct Frame {
    CellState cs;
    double rate;                       // gamma / tau (0 when collisionless)
    double c0[kMaxNOm + 1], c1[kMaxNOm + 1];
};

// nt: the series length of the cell's previous evaluation (0: none), kept
// when it is still the first length whose threshold covers beta^2 (the
// binary search's answer; consecutive evaluations of a solve barely move
// beta), else searched.
template <typename TP>
__device__ __forceinline__ bool frame_of(const InstDesc& d, double N0, double Nz, double T00, double T0z, double Tzz,
                                         TP ser, TP thr, Frame& fr, int& nt) {
    fr.cs = landau(N0, Nz, T00, T0z, Tzz);
    if (!fr.cs.ok) return false;
    const CellState& cs = fr.cs;
    double tau = d.tau_r;
    if (d.tau_mode == RSL_TAU_ETAS)
        tau = d.tau_aw0 / cs.T * (1.0 - 0.25 * log(cs.n / (cs.T * cs.T * cs.T) * d.lambda_ref));
    fr.rate = d.tau_mode == RSL_TAU_INF ? 0.0 : cs.gamma / tau;
    const double x = fmin(cs.beta * cs.beta, d.beta_series * d.beta_series);
    const bool keep = nt > 0 && (nt == 1 || x > thr[nt - 1]) && (nt == kSeriesTerms || x <= thr[nt]);
    if (!keep) nt = series_terms_uniform(x, thr);
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
// w0..w3 = sum_k w_j w_k {1, L_1(pbar_k), p_k, p_k L_1(pbar_k)}.  Nodes past
// Q_xi carry zeros.
template <int JM>
struct LaneNodes {
    double x[JM], a[JM], b[JM], w0[JM], w1[JM], w2[JM], w3[JM];
};

template <typename Tf, int L, int JM>
__device__ __forceinline__ void load_nodes(const InstDesc& d, const Tf* __restrict__ F, int s, int r,
                                           LaneNodes<JM>& n) {
#pragma unroll
    for (int i = 0; i < JM; ++i) {
        const int j = r + i * L;
        n.x[i] = n.a[i] = n.b[i] = n.w0[i] = n.w1[i] = n.w2[i] = n.w3[i] = 0.0;
        if (j >= d.Q) continue;
        n.x[i] = d.tab.xi[j];
        for (int k = 0; k < d.QL; ++k) {
            const int v = k * d.Q + j;
            const double fv = (double)F[(size_t)v * d.pitch + s], w = d.tab.wxw[v], p = d.tab.pk[k];
            const double l1 = d.tab.L1[k];
            n.a[i] += fv;
            n.b[i] = fma(p, fv, n.b[i]);
            n.w0[i] += w;
            n.w1[i] = fma(w, l1, n.w1[i]);
            n.w2[i] = fma(w, p, n.w2[i]);
            n.w3[i] = fma(w * p, l1, n.w3[i]);
        }
    }
}

// (N^z, T^zz) of the relaxed stage G = (F + h c f^eq) / (1 + h c) for the
// frame fr, summed over the cell's group of L lanes.
template <int L, int JM>
__device__ __forceinline__ void relaxed_moments(const InstDesc& d, const LaneNodes<JM>& n, const double* Pm, int r,
                                                const Frame& fr, double h, double (&out)[2]) {
    double nzs = 0.0, tzz = 0.0;
#pragma unroll
    for (int i = 0; i < JM; ++i) {
        const int j = min(r + i * L, d.Q - 1);          // past Q_xi: any node (the sums are zero)
        double g = 0.0, hh = 0.0;
#pragma unroll
        for (int m = 0; m <= kMaxNOm; ++m) {       // fixed bounds keep c0, c1 in registers
            if (m > d.NOm) break;
            const double P = Pm[m * d.Q + j];
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

// The K-series tables of the instance's velocity set into LDS (read by every
// frame evaluation).
constexpr int kSer = kSeriesTerms * 2 * (kMaxNOm + 1);
constexpr int kPmLds = (kMaxNOm + 1) * 128;   // P_m(xi_j) staged for Q_xi <= 128

struct ImexLds {
    double ser[kSer], thr[kSeriesTerms], Pm[kPmLds];
};

// The tables into LDS; returns the P_m(xi_j) rows to read (the LDS copy, or
// the global table past 128 nodes).
__device__ __forceinline__ const double* stage_tables(const InstDesc& d, ImexLds& t) {
    for (int i = threadIdx.x; i < kSer; i += blockDim.x) t.ser[i] = d.tab.ser[i];
    for (int i = threadIdx.x; i < kSeriesTerms; i += blockDim.x) t.thr[i] = d.tab.thr[i];
    const int np = (d.NOm + 1) * d.Q;
    const bool lds = np <= kPmLds;
    if (lds)
        for (int i = threadIdx.x; i < np; i += blockDim.x) t.Pm[i] = d.tab.Pm[i];
    __syncthreads();
    return lds ? t.Pm : d.tab.Pm;
}

// One cell per group of L lanes (cell s0 + threadIdx.x / L of a workgroup);
// the groups of a wave are independent and every lane of a group takes the
// same branches (its sums are bitwise equal).  In place (Fs == G) is safe: a
// group reads its cell's column before it writes any of it.
template <typename Tf, int L, int JM>
__device__ __forceinline__ void implicit_cells(const InstDesc& d, const Tf* Fs, Tf* G, double h, int s_first,
                                               const double* ser, const double* thr, const double* Pm,
                                               double* jac, int reuse) {
    const int r = threadIdx.x % L;
    const int s0 = s_first + threadIdx.x / L;
    const bool live = s0 < d.nz;
    const int s = live ? s0 : d.nz - 1;           // dead groups repeat the last cell and store nothing
    LaneNodes<JM> nd;
    load_nodes<Tf, L, JM>(d, Fs, s, r, nd);
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
    // Broyden's method.  The Jacobian of R(X) = (relaxed moments - X) comes
    // from finite differences (evaluations at X, X + e0, X + e1) or, with
    // reuse, from the cell's previous solve in this call (kept in the work
    // buffer's per-cell rows: the states of consecutive stages are close);
    // rank-one updates after each step above 1e-10 of the scales.  The X that
    // a step of at most 1e-13 of them reaches is the solution (the next step
    // would be far smaller still), provided the residual before that step is
    // below 1e-9 of the scales (a carried Jacobian far off cannot pass for
    // convergence); a carried Jacobian that is singular or needs more than 12
    // steps is replaced by finite differences at the current X.  One
    // evaluation site (frame, K-series, relaxed moments) serves all phases.
    const double e0 = 1e-7 * sc[0], e1 = 1e-7 * sc[1];
    Frame fr;
    bool ok = true, conv = false, fresh = !reuse;
    double R[2] = {0.0, 0.0}, J[2][2] = {{0.0, 0.0}, {0.0, 0.0}}, r0[2] = {0.0, 0.0}, st[2] = {0.0, 0.0};
    int phase = 0, nst = 0;        // phases 0-2: finite differences; 4: residual only; 3: steps
    int nt_cell = 0;               // series length of the cell's last frame
    if (reuse) {
        J[0][0] = jac[s];
        J[0][1] = jac[(size_t)d.pitch + s];
        J[1][0] = jac[2 * (size_t)d.pitch + s];
        J[1][1] = jac[3 * (size_t)d.pitch + s];
        phase = 4;
    }
    for (int it = 0; it < 48 && ok && !conv; ++it) {
        if (phase == 3 && !fresh && nst >= 12) {
            phase = 0;
            fresh = true;
        }
        double xe0 = X[0], xe1 = X[1];
        if (phase == 1) xe0 += e0;
        if (phase == 2) xe1 += e1;
        if (phase == 3) {
            const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
            if (!(fabs(det) > 0.0)) {
                if (fresh) { ok = false; break; }
                phase = 0;
                fresh = true;
                continue;
            }
            st[0] = -(J[1][1] * R[0] - J[0][1] * R[1]) / det;
            st[1] = -(J[0][0] * R[1] - J[1][0] * R[0]) / det;
            X[0] += st[0];
            X[1] += st[1];
            xe0 = X[0];
            xe1 = X[1];
            ++nst;
        }
        if (!frame_of(d, M[0], xe0, M[2], M[3], xe1, ser, thr, fr, nt_cell)) { ok = false; break; }
        if (phase == 3 && fabs(st[0]) <= 1e-13 * sc[0] && fabs(st[1]) <= 1e-13 * sc[1] &&
            fabs(R[0]) <= 1e-9 * sc[0] && fabs(R[1]) <= 1e-9 * sc[1]) {
            conv = true;                                      // fr is the frame of the final X
            break;
        }
        double rn[2];
        relaxed_moments<L, JM>(d, nd, Pm, r, fr, h, rn);
        if (phase == 0) {
            r0[0] = rn[0];
            r0[1] = rn[1];
            R[0] = rn[0] - X[0];
            R[1] = rn[1] - X[1];
            phase = 1;
        } else if (phase == 1) {
            J[0][0] = (rn[0] - r0[0]) / e0 - 1.0;
            J[1][0] = (rn[1] - r0[1]) / e0;
            phase = 2;
        } else if (phase == 2) {
            J[0][1] = (rn[0] - r0[0]) / e1;
            J[1][1] = (rn[1] - r0[1]) / e1 - 1.0;
            phase = 3;
            nst = 0;
        } else if (phase == 4) {
            R[0] = rn[0] - X[0];
            R[1] = rn[1] - X[1];
            phase = 3;
            nst = 0;
        } else {
            const double y0 = rn[0] - X[0] - R[0], y1 = rn[1] - X[1] - R[1];
            R[0] = rn[0] - X[0];
            R[1] = rn[1] - X[1];
            // no update from steps near the rounding level of R (its
            // differences are noise there): the last Jacobian is kept
            if (fabs(st[0]) <= 1e-10 * sc[0] && fabs(st[1]) <= 1e-10 * sc[1]) continue;
            const double ss = st[0] * st[0] + st[1] * st[1];
            const double u0 = (y0 - (J[0][0] * st[0] + J[0][1] * st[1])) / ss;
            const double u1 = (y1 - (J[1][0] * st[0] + J[1][1] * st[1])) / ss;
            J[0][0] += u0 * st[0];
            J[0][1] += u0 * st[1];
            J[1][0] += u1 * st[0];
            J[1][1] += u1 * st[1];
        }
    }
    if (live && ok && conv && r == 0) {           // the Jacobian for this cell's next solve
        jac[s] = J[0][0];
        jac[(size_t)d.pitch + s] = J[0][1];
        jac[2 * (size_t)d.pitch + s] = J[1][0];
        jac[3 * (size_t)d.pitch + s] = J[1][1];
    }
    if (!live) return;
    if (!ok || !conv) {
        if (r == 0) atomicOr(d.status, 1u);
        for (int j = r; j < d.Q; j += L)
            for (int k = 0; k < d.QL; ++k) G[(size_t)(k * d.Q + j) * d.pitch + s] = (Tf)__builtin_nan("");
        return;
    }
    for (int j = r; j < d.Q; j += L) {
        double g = 0.0, hh = 0.0;
#pragma unroll
        for (int m = 0; m <= kMaxNOm; ++m) {
            if (m > d.NOm) break;
            const double P = Pm[m * d.Q + j];
            g = fma(P, fr.c0[m], g);
            hh = fma(P, fr.c1[m], hh);
        }
        const double hc = h * fr.rate * (1.0 - fr.cs.beta * d.tab.xi[j]);
        const double den = 1.0 / (1.0 + hc);
        for (int k = 0; k < d.QL; ++k) {
            const int v = k * d.Q + j;
            const double fe = d.tab.wxw[v] * fma(d.tab.L1[k], hh, g);
            const double fv = (double)Fs[(size_t)v * d.pitch + s];
            G[(size_t)v * d.pitch + s] = (Tf)(fma(hc, fe, fv) * den);
        }
    }
}

template <typename Tf, int L, int JM>
__global__ void __launch_bounds__(kImexThreads) imex_implicit_kernel(InstDesc d, const Tf* Fs, Tf* G, double h,
                                                                      int reuse) {
    __shared__ ImexLds t;
    const double* Pm = stage_tables(d, t);
    implicit_cells<Tf, L, JM>(d, Fs, G, h, blockIdx.x * (kImexThreads / L), t.ser, t.thr, Pm, d.cell, reuse);
}

// Batch form: item (instance, first cell); second = 0 solves F1 from f,
// second = 1 solves F2 from F2* in place.  One node per lane fits three waves
// per SIMD without spills (164 VGPRs); two nodes per lane stay at two (three
// would spill, measured slower).
template <typename Tf, int L, int JM>
__global__ void __launch_bounds__(kImexBatchThreads, JM == 1 ? 3 : 1) imex_implicit_batch_kernel(const InstDesc* __restrict__ descs,
                                                                            const int2* __restrict__ items,
                                                                            char* fbase, char* wbase, int second,
                                                                            int reuse) {
    const int2 it = items[blockIdx.x];
    InstDesc d = descs[it.x];
    rebase(d, fbase, wbase);
    __shared__ ImexLds t;
    const double* Pm = stage_tables(d, t);
    const Tf* F = (const Tf*)(second ? d.f2 : d.f);
    Tf* G = (Tf*)(second ? d.f2 : d.f1);
    implicit_cells<Tf, L, JM>(d, F, G, kImexG * d.dt, it.y, t.ser, t.thr, Pm, d.cell, reuse);
}

// Population of velocity v at cell c (ghosts per the instance's rule).
template <typename Tf>
__device__ __forceinline__ double at(const InstDesc& d, const Tf* F, int v, int c) {
    if (c < 0) return d.bc == RSL_BC_EQ ? d.feqL[v] : (double)F[(size_t)v * d.pitch];
    if (c >= d.nz) return d.bc == RSL_BC_EQ ? d.feqR[v] : (double)F[(size_t)v * d.pitch + d.nz - 1];
    return (double)F[(size_t)v * d.pitch + c];
}

// Explicit passes: each thread takes RUN consecutive cells of one velocity
// plane, so that the run's RUN + 1 interface fluxes come from one window of
// RUN + 6 values (each face's WENO5 once, shared by the two cells it bounds).
// Batches take runs of kImexRun cells; a single instance, short of threads,
// one cell per thread.
constexpr int kImexRun = 4;

// Interface fluxes Phi_{s0 + f - 1/2}, f = 0..RUN, of velocity v (without
// the factor xi_j), from the WENO5 upwind stencil (Sec. III F) in the storage
// precision (binary32 storage: the binary32 weights of the explicit stages,
// with their limiting cases).
template <typename Tf, int RUN>
__device__ __forceinline__ void run_fluxes(const InstDesc& d, const Tf* F, int v, int s0, double x,
                                           Tf (&ph)[RUN + 1]) {
    Tf u[RUN + 6];
#pragma unroll
    for (int q = 0; q < RUN + 6; ++q) u[q] = (Tf)at(d, F, v, s0 - 3 + q);
#pragma unroll
    for (int f = 0; f <= RUN; ++f)
        ph[f] = x > 0.0 ? weno5(u[f], u[f + 1], u[f + 2], u[f + 3], u[f + 4])
                        : weno5(u[f + 5], u[f + 4], u[f + 3], u[f + 2], u[f + 1]);
}

// mode 0: F2* = f + dt A(F1) + (1 - 2g)/g (F1 - f) into the second slot, and
//         Y = f + dt/2 A(F1) + (F1 - f)/(2g) - F2*/(2g) (F2* unrounded) over f
//         (each thread reads f at its own elements only);
// mode 1: f <- Y + dt/2 A(F2) + F2/(2g), which is
//         f + dt/2 (A(F1) + A(F2)) + (F1 - f)/(2g) + (F2 - F2*)/(2g);
// A(F) = -xi_j (Phi_{s+1/2} - Phi_{s-1/2}) / dz, the difference in binary64.
template <typename Tf, int RUN>
__device__ __forceinline__ void explicit_run(const InstDesc& d, int v, int s0, int mode) {
    Tf* f = (Tf*)d.f;
    Tf* F2 = (Tf*)d.f2;
    const double dt = d.dt, g = kImexG, x = d.tab.xv[v];
    const Tf* A = mode == 0 ? (const Tf*)d.f1 : (const Tf*)F2;   // the field advected
    Tf ph[RUN + 1];
#pragma unroll
    for (int q = 0; q <= RUN; ++q) ph[q] = (Tf)0;
    if (x != 0.0) run_fluxes<Tf, RUN>(d, A, v, s0, x, ph);
    unsigned bad = 0;
#pragma unroll
    for (int c = 0; c < RUN; ++c) {
        const int s = s0 + c;
        if (s >= d.nz) break;
        const size_t i = (size_t)v * d.pitch + s;
        const double a = -x * ((double)ph[c + 1] - (double)ph[c]) * d.dz_inv;
        if (mode == 0) {
            const double fn = (double)f[i], f1 = (double)A[i];
            const double fs2 = fn + dt * a + (1.0 - 2.0 * g) / g * (f1 - fn);
            F2[i] = (Tf)fs2;
            f[i] = (Tf)(fn + 0.5 * dt * a + (f1 - fn - fs2) / (2.0 * g));
        } else {
            const Tf o = (Tf)((double)f[i] + 0.5 * dt * a + (double)A[i] / (2.0 * g));
            if (!isfinite(o)) bad = 2u;
            f[i] = o;
        }
    }
    if (bad) atomicOr(d.status, bad);
}

// One thread per cell and velocity v = blockIdx.y.
template <typename Tf>
__global__ void __launch_bounds__(kImexThreads) imex_explicit_kernel(InstDesc d, int mode) {
    const int s = blockIdx.x * kImexThreads + threadIdx.x;
    if (s < d.nz) explicit_run<Tf, 1>(d, blockIdx.y, s, mode);
}

// Batch form: item (instance, first cell of kImexThreads runs); velocities
// v = blockIdx.y, blockIdx.y + kImexVY, ...
constexpr int kImexVY = 8;

template <typename Tf>
__global__ void __launch_bounds__(kImexThreads) imex_explicit_batch_kernel(const InstDesc* __restrict__ descs,
                                                                            const int2* __restrict__ items,
                                                                            char* fbase, char* wbase, int mode) {
    const int2 it = items[blockIdx.x];
    InstDesc d = descs[it.x];
    rebase(d, fbase, wbase);
    const int s0 = it.y + threadIdx.x * kImexRun;
    if (s0 >= d.nz) return;
    for (int v = blockIdx.y; v < d.V; v += kImexVY) explicit_run<Tf, kImexRun>(d, v, s0, mode);
}

// Lanes per cell (L) and angular nodes per lane (JM) of each class.  A single
// instance spreads a cell over enough lanes to cover its angular nodes (at
// most a wave; past 64 nodes each lane takes up to 16), since its few cells
// leave the GPU short of waves.  A batch fills the GPU, so there each lane
// takes two nodes (up to 128 nodes) and a wave serves twice the cells: the
// frame of a cell, which every lane of its group evaluates, is then formed
// for half the waves.  More nodes per lane push the registers past two waves
// per SIMD, which costs more than the saved frames (measured).
constexpr int kImexBatchL[kImexClasses] = {4, 8, 8, 16, 32, 64, 64, 64, 64};

template <typename Tf, int C>
struct ImexClass;
#define RSL_IMEX_CLASS(C, L, JM, LB, JMB)                                                                     \
    template <typename Tf>                                                                                    \
    struct ImexClass<Tf, C> {                                                                                 \
        static void single(const InstDesc& d, const Tf* F, Tf* G, double h, int reuse, hipStream_t s) {      \
            const int cells = kImexThreads / L;                                                               \
            hipLaunchKernelGGL((imex_implicit_kernel<Tf, L, JM>), dim3((d.nz + cells - 1) / cells),           \
                               dim3(kImexThreads), 0, s, d, F, G, h, reuse);                                  \
        }                                                                                                     \
        static void batch(const InstDesc* descs, const int2* items, int n, char* fb, char* wb, int second,    \
                          int reuse, hipStream_t s) {                                                         \
            static_assert(LB == kImexBatchL[C], "batch lanes per cell");                                      \
            hipLaunchKernelGGL((imex_implicit_batch_kernel<Tf, LB, JMB>), dim3(n), dim3(kImexBatchThreads), 0, \
                               s, descs, items, fb, wb, second, reuse);                                       \
        }                                                                                                     \
    };
//              class  single    batch      angular nodes
RSL_IMEX_CLASS(0, 4, 1, 4, 1)     // Q_xi <= 4
RSL_IMEX_CLASS(1, 8, 1, 8, 1)     // <= 8
RSL_IMEX_CLASS(2, 16, 1, 8, 2)    // <= 16
RSL_IMEX_CLASS(3, 32, 1, 16, 2)   // <= 32
RSL_IMEX_CLASS(4, 64, 1, 32, 2)   // <= 64
RSL_IMEX_CLASS(5, 64, 2, 64, 2)   // <= 128
RSL_IMEX_CLASS(6, 64, 4, 64, 4)   // <= 256
RSL_IMEX_CLASS(7, 64, 8, 64, 8)   // <= 512
RSL_IMEX_CLASS(8, 64, 16, 64, 16) // <= 1024
#undef RSL_IMEX_CLASS

template <typename Tf>
void implicit_single(int c, const InstDesc& d, const Tf* F, Tf* G, double h, int reuse, hipStream_t s) {
    switch (c) {
        case 0: ImexClass<Tf, 0>::single(d, F, G, h, reuse, s); break;
        case 1: ImexClass<Tf, 1>::single(d, F, G, h, reuse, s); break;
        case 2: ImexClass<Tf, 2>::single(d, F, G, h, reuse, s); break;
        case 3: ImexClass<Tf, 3>::single(d, F, G, h, reuse, s); break;
        case 4: ImexClass<Tf, 4>::single(d, F, G, h, reuse, s); break;
        case 5: ImexClass<Tf, 5>::single(d, F, G, h, reuse, s); break;
        case 6: ImexClass<Tf, 6>::single(d, F, G, h, reuse, s); break;
        case 7: ImexClass<Tf, 7>::single(d, F, G, h, reuse, s); break;
        default: ImexClass<Tf, 8>::single(d, F, G, h, reuse, s); break;
    }
}

template <typename Tf>
void implicit_batch(int c, const InstDesc* descs, const int2* items, int n, char* fb, char* wb, int second, int reuse,
                    hipStream_t s) {
    switch (c) {
        case 0: ImexClass<Tf, 0>::batch(descs, items, n, fb, wb, second, reuse, s); break;
        case 1: ImexClass<Tf, 1>::batch(descs, items, n, fb, wb, second, reuse, s); break;
        case 2: ImexClass<Tf, 2>::batch(descs, items, n, fb, wb, second, reuse, s); break;
        case 3: ImexClass<Tf, 3>::batch(descs, items, n, fb, wb, second, reuse, s); break;
        case 4: ImexClass<Tf, 4>::batch(descs, items, n, fb, wb, second, reuse, s); break;
        case 5: ImexClass<Tf, 5>::batch(descs, items, n, fb, wb, second, reuse, s); break;
        case 6: ImexClass<Tf, 6>::batch(descs, items, n, fb, wb, second, reuse, s); break;
        case 7: ImexClass<Tf, 7>::batch(descs, items, n, fb, wb, second, reuse, s); break;
        default: ImexClass<Tf, 8>::batch(descs, items, n, fb, wb, second, reuse, s); break;
    }
}

template <typename Tf>
int imex_steps_t(const InstDesc& d, int nsteps, hipStream_t s) {
    const dim3 gx((d.nz + kImexThreads - 1) / kImexThreads, d.V);
    const double h = kImexG * d.dt;
    const int c = imex_class(d.Q);
    for (int it = 0; it < nsteps; ++it) {
        implicit_single<Tf>(c, d, (const Tf*)d.f, (Tf*)d.f1, h, it > 0, s);   // fresh Jacobians first
        hipLaunchKernelGGL(imex_explicit_kernel<Tf>, gx, dim3(kImexThreads), 0, s, d, 0);
        implicit_single<Tf>(c, d, (const Tf*)d.f2, (Tf*)d.f2, h, 1, s);
        hipLaunchKernelGGL(imex_explicit_kernel<Tf>, gx, dim3(kImexThreads), 0, s, d, 1);
    }
    return hip_check(hipGetLastError(), "imex step launch");
}

template <typename Tf>
int imex_batch_steps_t(const InstDesc* descs, const ImexItems& it, char* fb, char* wb, int nsteps, hipStream_t s) {
    const dim3 gx(it.nx, kImexVY);
    for (int step = 0; step < nsteps; ++step) {
        for (int second = 0; second < 2; ++second) {
            for (int c = 0; c < kImexClasses; ++c)
                if (it.n[c]) implicit_batch<Tf>(c, descs, it.items[c], it.n[c], fb, wb, second, step > 0 || second, s);
            if (it.nx) hipLaunchKernelGGL(imex_explicit_batch_kernel<Tf>, gx, dim3(kImexThreads), 0, s, descs, it.x,
                                          fb, wb, second);
        }
    }
    return hip_check(hipGetLastError(), "imex batch step launch");
}

}  // namespace

int imex_class(int Q) {
    return Q <= 4 ? 0 : Q <= 8 ? 1 : Q <= 16 ? 2 : Q <= 32 ? 3 : Q <= 64 ? 4 : Q <= 128 ? 5 : Q <= 256 ? 6
                                                                                            : Q <= 512 ? 7 : 8;
}

int imex_cells_per_item(int Q) { return kImexBatchThreads / kImexBatchL[imex_class(Q)]; }

int imex_cells_per_explicit_item() { return kImexThreads * kImexRun; }

int launch_imex_steps(const InstDesc& d, int dtype, int nsteps, hipStream_t s) {
    return dtype == RSL_F64 ? imex_steps_t<double>(d, nsteps, s) : imex_steps_t<float>(d, nsteps, s);
}

int launch_imex_batch_steps(const InstDesc* descs, const ImexItems& items, int dtype, char* fbase, char* wbase,
                            int nsteps, hipStream_t s) {
    return dtype == RSL_F64 ? imex_batch_steps_t<double>(descs, items, fbase, wbase, nsteps, s)
                            : imex_batch_steps_t<float>(descs, items, fbase, wbase, nsteps, s);
}

}  // namespace rsl
