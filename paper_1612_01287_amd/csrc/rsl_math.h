// Per-cell and per-interface arithmetic of the R-SLB step, as device functions.
//
// Equilibrium coefficients.  The truncated expansion of f^eq (Sec. III D,
// eq. feq_trunc with N_L = 1) mapped to the populations by eq. fjk reads
//
//   f^eq_jk = (n gamma / 2) w_j w_k sum_{l<=1} L_l(pbar_k) sum_{m<=N_Omega}
//             (2m+1)/2 a~_{l,m} P_m(xi_j),
//
// with a~_{l,m} the normalised coefficients of App. A.  Writing the angular
// integral that defines them (eq. aeq_aux) with u^0 - u cos = gamma (1 - beta cos)
// gives a~_{0,m} = K_{3,m} / (2 gamma^4) and
// a~_{1,m} = (K_{3,m} - (theta/gamma) K_{4,m}) / (2 gamma^4), where
//
//   K_{k,m}(beta) = int_{-1}^{1} P_m(c) (1 - beta c)^{-k} dc ,  theta = T / T0.
//
// Instead of the closed forms printed in App. A (which lose digits to
// cancellation as u -> 0) the kernels evaluate K_{k,m}:
//  * for |beta| < beta_s by its Maclaurin series  beta^m sum_i a_i beta^{2i}
//    (all terms positive; coefficients tabulated on the host, the number of
//    terms chosen per cell from beta^2);
//  * for |beta| >= beta_s by the Legendre three-term recurrence in m,
//    (m+1) K_{k,m+1} = (2m+1)(K_{k,m} - K_{k-1,m})/beta - m K_{k,m-1},
//    started from the closed forms K_{0,m} = 2 delta_{m0},
//    K_{1,0} = ln((1+beta)/(1-beta))/beta, K_{2,0} = 2/(1-beta^2),
//    K_{3,0} = 2/(1-beta^2)^2, K_{4,0} = 2(3+beta^2)/(3(1-beta^2)^3).
//  beta_s grows with N_Omega so that the recurrence (which loses about a
//  factor 1/beta per order) stays at the 1e-15 level.
#pragma once

#include <hip/hip_runtime.h>

#include "rsl_impl.h"

namespace rsl {

struct CellState {
    double n, T, beta, gamma, E;
    bool ok;
};

// Landau frame of the Sod moments (Sec. II E, eqs. E_landau, u_landau):
// E = [T00 - Tzz + sqrt((T00 + Tzz)^2 - 4 T0z^2)]/2, beta = T0z/(E + Tzz),
// n = gamma (N0 - beta Nz), P = E/3, T = P/n.
__device__ __forceinline__ CellState landau(double N0, double Nz, double T00, double T0z,
                                            double Tzz) {
    CellState c;
    const double s = T00 + Tzz;
    const double disc = s * s - 4.0 * T0z * T0z;
    const double E = 0.5 * (T00 - Tzz + sqrt(disc));
    const double beta = T0z / (E + Tzz);
    const double g = 1.0 / sqrt((1.0 - beta) * (1.0 + beta));
    const double n = g * (N0 - beta * Nz);
    c.E = E;
    c.beta = beta;
    c.gamma = g;
    c.n = n;
    c.T = E / (3.0 * n);
    c.ok = (disc >= 0.0) && (fabs(beta) < 1.0) && (n > 0.0) && (E > 0.0) && isfinite(c.T);
    return c;
}

// Number of Maclaurin terms that carry K_{3,m}, K_{4,m} to full precision for
// every beta^2 <= x (thr is ascending).
__device__ __forceinline__ int series_terms(double x, const double* __restrict__ thr) {
    int nt = 1;
    while (nt < kSeriesTerms && x > thr[nt]) ++nt;
    return nt;
}

// The same count for a wave-uniform x (binary search; thr a copy in LDS, or
// the table itself through scalar loads when TP is a constant-space pointer).
template <typename TP>
__device__ __forceinline__ int series_terms_uniform(double x, TP thr) {
    TP t = thr;
    int lo = 1, hi = kSeriesTerms;      // first nt in [1, kSeriesTerms) with x <= thr[nt], else kSeriesTerms
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (x > t[mid]) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Largest x over the 64 lanes of a wave (all lanes active), as a wave-uniform value.
__device__ __forceinline__ double wave_max_uniform(double x) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) x = fmax(x, __shfl_xor(x, o));
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(x));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(x));
    return __hiloint2double(hi, lo);
}

// K_{3,m}, K_{4,m} for m = 0..nom (nom <= kMaxNOm); nt terms of the series
// when |beta| < beta_s (nt from series_terms for beta^2 or anything larger:
// extra terms only add values below the last bit).  ser is the term-major
// coefficient table, in global memory or staged in LDS by the caller.
// The series sums for a fixed order N, without per-term branches.
template <int N, typename TP>
__device__ __forceinline__ void kint_series(double x, TP ser, int nt, double* s3, double* s4) {
    double p = 1.0;
#pragma unroll 1
    for (int i = 0; i < nt; ++i) {
        TP a = ser + i * 2 * (kMaxNOm + 1);
#pragma unroll
        for (int m = 0; m <= N; ++m) {
            s3[m] = fma(a[m], p, s3[m]);
            s4[m] = fma(a[kMaxNOm + 1 + m], p, s4[m]);
        }
        p *= x;
    }
}

template <typename TP>
__device__ __forceinline__ void kint(double beta, int nom, double beta_s, TP ser, int nt, double* K3, double* K4) {
    const double ab = fabs(beta);
    if (ab < beta_s) {
        const double x = beta * beta;
        double s3[kMaxNOm + 1], s4[kMaxNOm + 1];
#pragma unroll
        for (int m = 0; m <= kMaxNOm; ++m) s3[m] = s4[m] = 0.0;
        switch (nom) {
            case 3: kint_series<3>(x, ser, nt, s3, s4); break;
            case 4: kint_series<4>(x, ser, nt, s3, s4); break;
            case 5: kint_series<5>(x, ser, nt, s3, s4); break;
            case 6: kint_series<6>(x, ser, nt, s3, s4); break;
            default: {
                double p = 1.0;
                for (int i = 0; i < nt; ++i) {
                    TP a = ser + i * 2 * (kMaxNOm + 1);
#pragma unroll
                    for (int m = 0; m <= kMaxNOm; ++m) {
                        if (m <= nom) {
                            s3[m] = fma(a[m], p, s3[m]);
                            s4[m] = fma(a[kMaxNOm + 1 + m], p, s4[m]);
                        }
                    }
                    p *= x;
                }
            }
        }
        double bm = 1.0;
#pragma unroll
        for (int m = 0; m <= kMaxNOm; ++m) {
            K3[m] = bm * s3[m];
            K4[m] = bm * s4[m];
            bm *= beta;
        }
    } else {
        const double omb2 = (1.0 - beta) * (1.0 + beta);
        double k0 = 2.0, k1 = log1p(2.0 * beta / (1.0 - beta)) / beta;
        double k2 = 2.0 / omb2, k3 = k2 / omb2;
        double k4 = 2.0 * (3.0 + beta * beta) / (3.0 * omb2 * omb2 * omb2);
        double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0, p4 = 0.0;   // order m-1
        const double ib = 1.0 / beta;
        K3[0] = k3;
        K4[0] = k4;
#pragma unroll
        for (int m = 0; m < kMaxNOm; ++m) {
            const double a = (2.0 * m + 1.0) * ib, inv = 1.0 / (m + 1.0);
            const double n1 = (a * (k1 - k0) - m * p1) * inv;
            const double n2 = (a * (k2 - k1) - m * p2) * inv;
            const double n3 = (a * (k3 - k2) - m * p3) * inv;
            const double n4 = (a * (k4 - k3) - m * p4) * inv;
            p0 = k0; p1 = k1; p2 = k2; p3 = k3; p4 = k4;
            k0 = 0.0; k1 = n1; k2 = n2; k3 = n3; k4 = n4;
            K3[m + 1] = k3;
            K4[m + 1] = k4;
        }
        (void)p0;
    }
}

// Coefficients of the equilibrium at the nodes:
//   f^eq_jk = w_j w_k sum_m P_m(xi_j) (c0[m] + L_1(pbar_k) c1[m]),
//   c0[m] = h_m K_{3,m},  c1[m] = h_m (K_{3,m} - (theta/gamma) K_{4,m}),
//   h_m = n (2m+1) / (8 gamma^3).
// nt: series terms (see kint).
template <typename TP>
__device__ __forceinline__ void feq_coef(double n, double T, double beta, double gamma, double T0,
                                         int nom, double beta_s, TP ser, int nt, double* c0, double* c1) {
    double K3[kMaxNOm + 1], K4[kMaxNOm + 1];
    kint(beta, nom, beta_s, ser, nt, K3, K4);
    const double h0 = n / (8.0 * gamma * gamma * gamma);
    const double tg = T / (T0 * gamma);
#pragma unroll
    for (int m = 0; m <= kMaxNOm; ++m) {
        const double h = h0 * (2.0 * m + 1.0);
        c0[m] = h * K3[m];
        c1[m] = h * (K3[m] - tg * K4[m]);
    }
}

// WENO5 flux at one interface from five values in upwind order
// (a, b, c, d, e) = (f_{s-2}, ..., f_{s+2}) for a right-moving population
// (Sec. III F, eqs. flux_weno, weno5_omega).  Nonlinear weights
// w_q ~ delta_q / sigma_q^2 with delta = (1/10, 6/10, 3/10) and no epsilon
// regulariser; the paper's limiting cases for vanishing indicators are
// honoured: all equal -> ideal weights; two zero -> the two share by their
// ideal weights; one zero -> that stencil alone.
//
// weno5_6 returns six times the interface value: the three candidates are
// taken without their common factor 1/6 (callers fold it into the velocity
// xi_j / 6), and the indicators are taken four times larger,
// (13/3) r^2 + t^2, which leaves the normalised weights and the tests for
// equal or vanishing indicators unchanged (scaling by 4 is exact).  The
// common case uses the common denominator sigma_1^2 sigma_2^2 sigma_3^2
// (equal indicators then give the ideal weights to rounding) and a reciprocal
// refined by two Newton steps; exact zeros and products outside
// [1e-280, 1e280] take the explicit branch.
__device__ __forceinline__ double weno5_6(double a, double b, double c, double d, double e) {
    const double q1 = 2.0 * a - 7.0 * b + 11.0 * c;
    const double q2 = -b + 5.0 * c + 2.0 * d;
    const double q3 = 2.0 * c + 5.0 * d - e;
    const double r1 = a - 2.0 * b + c, t1 = a - 4.0 * b + 3.0 * c;
    const double r2 = b - 2.0 * c + d, t2 = b - d;
    const double r3 = c - 2.0 * d + e, t3 = 3.0 * c - 4.0 * d + e;
    const double s1 = (13.0 / 3.0) * r1 * r1 + t1 * t1;
    const double s2 = (13.0 / 3.0) * r2 * r2 + t2 * t2;
    const double s3 = (13.0 / 3.0) * r3 * r3 + t3 * t3;
    const double u1 = s1 * s1, u2 = s2 * s2, u3 = s3 * s3;
    const double w1 = 0.1 * u2 * u3, w2 = 0.6 * u1 * u3, w3 = 0.3 * u1 * u2;
    const double den = w1 + w2 + w3;
    if (den > 1e-280 && den < 1e280) {
        double r = __builtin_amdgcn_rcp(den);
        double err = fma(-den, r, 1.0);
        r = fma(r, err, r);
        err = fma(-den, r, 1.0);
        r = fma(r, err, r);
        return (w1 * q1 + w2 * q2 + w3 * q3) * r;
    }
    if (s1 == s2 && s2 == s3) return 0.1 * q1 + 0.6 * q2 + 0.3 * q3;    // case (i), incl. all zero
    const int z1 = s1 == 0.0, z2 = s2 == 0.0, z3 = s3 == 0.0;
    const int nz = z1 + z2 + z3;
    if (nz == 2) {                                                        // case (ii)
        const double dsum = 0.1 * z1 + 0.6 * z2 + 0.3 * z3;
        return (0.1 * z1 * q1 + 0.6 * z2 * q2 + 0.3 * z3 * q3) / dsum;
    }
    if (nz == 1) return z1 ? q1 : (z2 ? q2 : q3);                         // case (iii)
    // no zero but the product form left the safe range: weights relative to the
    // smallest indicator, delta_q (sigma_min / sigma_q)^2, all in [0, 1]
    const double sm = fmin(s1, fmin(s2, s3));
    const double g1 = sm / s1, g2 = sm / s2, g3 = sm / s3;
    const double v1 = 0.1 * g1 * g1, v2 = 0.6 * g2 * g2, v3 = 0.3 * g3 * g3;
    return (v1 * q1 + v2 * q2 + v3 * q3) / (v1 + v2 + v3);
}

// The same in binary32, for populations stored in binary32.  The weights are
// formed as ratios, w_q ~ delta_q (sigma_min / sigma_q)^2 in [0, delta_q],
// which neither overflow nor underflow whatever the scale of the populations
// (delta_q / sigma_q^2 itself overflows binary32 for smooth data); equal
// indicators give exactly the ideal weights.  The limiting cases are decided
// on the binary32 indicators: all equal (flat data) takes the ideal weights,
// exact zeros among unequal indicators (the edges of flat regions) weight the
// vanishing stencils by their ideal weights (two zero: they share; one zero:
// it alone).  Only a smallest indicator that is not zero but below 4e-30
// (where the squared ratio would lose digits in the denormal range) goes
// through the binary64 form above.
__device__ __forceinline__ float weno5_6(float a, float b, float c, float d, float e) {
    const float q1 = 2.0f * a - 7.0f * b + 11.0f * c;
    const float q2 = -b + 5.0f * c + 2.0f * d;
    const float q3 = 2.0f * c + 5.0f * d - e;
    const float r1 = a - 2.0f * b + c, t1 = a - 4.0f * b + 3.0f * c;
    const float r2 = b - 2.0f * c + d, t2 = b - d;
    const float r3 = c - 2.0f * d + e, t3 = 3.0f * c - 4.0f * d + e;
    const float s1 = (13.0f / 3.0f) * r1 * r1 + t1 * t1;
    const float s2 = (13.0f / 3.0f) * r2 * r2 + t2 * t2;
    const float s3 = (13.0f / 3.0f) * r3 * r3 + t3 * t3;
    const float sm = fminf(s1, fminf(s2, s3));
    if (sm > 4e-30f) {
        const float g1 = sm * __builtin_amdgcn_rcpf(s1);
        const float g2 = sm * __builtin_amdgcn_rcpf(s2);
        const float g3 = sm * __builtin_amdgcn_rcpf(s3);
        const float v1 = 0.1f * g1 * g1, v2 = 0.6f * g2 * g2, v3 = 0.3f * g3 * g3;
        return (v1 * q1 + v2 * q2 + v3 * q3) * __builtin_amdgcn_rcpf(v1 + v2 + v3);
    }
    if (s1 == s2 && s2 == s3) return 0.1f * q1 + 0.6f * q2 + 0.3f * q3;   // case (i), incl. all zero
    if (sm == 0.0f) {                                                        // cases (ii), (iii)
        const float v1 = s1 == 0.0f ? 0.1f : 0.0f, v2 = s2 == 0.0f ? 0.6f : 0.0f, v3 = s3 == 0.0f ? 0.3f : 0.0f;
        return (v1 * q1 + v2 * q2 + v3 * q3) * __builtin_amdgcn_rcpf(v1 + v2 + v3);
    }
    return (float)weno5_6((double)a, (double)b, (double)c, (double)d, (double)e);
}

// The interface value itself.
template <typename T>
__device__ __forceinline__ T weno5(T a, T b, T c, T d, T e) {
    return weno5_6(a, b, c, d, e) * (T)(1.0 / 6.0);
}

}  // namespace rsl
