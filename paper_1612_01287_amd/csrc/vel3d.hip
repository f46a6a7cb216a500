// Velocity sets with azimuthal nodes, for flows whose velocity is not along z
// (Sec. III D, eq. leg_product and its azimuthal rule): the discrete
// equilibrium for a fluid four-velocity in any direction, and the moments
// N^mu, T^{mu nu} of a population field with the Landau frame of T^{mu nu}.
//
// Node v = (k Q_phi + l) Q_xi + j = k A + a, with a = l Q_xi + j the angular
// node.  Angular record [a] = (Omega_x, Omega_y, Omega_z, w_j / Q_phi), radial
// record [k] = (p_k, w_k, L_1(pbar_k), 0).  Fields are [V][pitch], one lane per
// cell.
#include <hip/hip_runtime.h>

#include "rsl_impl.h"
#include "rsl_math.h"

namespace rsl {

namespace {

using CP = const __attribute__((address_space(4))) double*;

constexpr int kV3Threads = 256;

// f_v = (w_j w_k / Q_phi) sum_m P_m(cos gamma_u) (c0_m + L_1(pbar_k) c1_m),
// cos gamma_u = Omega_a . u_hat: the truncated expansion (eq. feq_trunc) mapped
// by eq. fjk with the azimuthal weight 2 pi / Q_phi; the coefficients c0, c1
// are those of the aligned flow at |u| (they depend on |u| only).
template <typename Tf>
__global__ void __launch_bounds__(kV3Threads) feq3_kernel(const double* __restrict__ state, int ncell, CP arec,
                                                           CP rrec, int A, int QL, int NOm, double T0,
                                                           double beta_s, CP ser, CP thr, Tf* __restrict__ f,
                                                           int pitch) {
    const int cell = blockIdx.x * kV3Threads + threadIdx.x;
    const bool live = cell < ncell;
    const int c = live ? cell : ncell - 1;
    const double n = state[5 * (size_t)c], T = state[5 * (size_t)c + 1];
    const double ux = state[5 * (size_t)c + 2], uy = state[5 * (size_t)c + 3], uz = state[5 * (size_t)c + 4];
    const double u = sqrt(ux * ux + uy * uy + uz * uz);
    const double gam = sqrt(1.0 + u * u), beta = u / gam;
    const double iu = u > 0.0 ? 1.0 / u : 0.0;
    const double hx = ux * iu, hy = uy * iu, hz = u > 0.0 ? uz * iu : 1.0;
    // series terms for the lanes on the Maclaurin branch, uniform over the wave
    const int nt = series_terms_uniform(wave_max_uniform(fmin(beta * beta, beta_s * beta_s)), thr);
    double c0[kMaxNOm + 1], c1[kMaxNOm + 1];
    feq_coef(n, T, beta, gam, T0, NOm, beta_s, ser, nt, c0, c1);
    // radial weights and L_1 values, loaded once (Q_L <= 8)
    double wk[8], lk[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        wk[k] = k < QL ? rrec[4 * k + 1] : 0.0;
        lk[k] = k < QL ? rrec[4 * k + 2] : 0.0;
    }
#pragma unroll 2
    for (int a = 0; a < A; ++a) {
        CP r = arec + 4 * (size_t)a;
        const double x = r[0] * hx + r[1] * hy + r[2] * hz, wa = r[3];
        // P_m(x) by the three-term recurrence, summed against the coefficients
        double pm1 = 1.0, pm = x;
        double g = c0[0], h = c1[0];
        if (NOm >= 1) {
            g = fma(x, c0[1], g);
            h = fma(x, c1[1], h);
        }
#pragma unroll
        for (int m = 1; m < kMaxNOm; ++m) {
            if (m < NOm) {
                const double pn = ((2.0 * m + 1.0) * x * pm - m * pm1) * (1.0 / (m + 1.0));
                pm1 = pm;
                pm = pn;
                g = fma(pn, c0[m + 1], g);
                h = fma(pn, c1[m + 1], h);
            }
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (k < QL) {
                const double fv = wa * wk[k] * fma(lk[k], h, g);
                if (live) f[((size_t)k * A + a) * pitch + cell] = (Tf)fv;
            }
        }
    }
}

// N^mu = sum_v f_v Omega^mu, T^{mu nu} = sum_v f_v p_k Omega^mu Omega^nu
// (discrete eq. macro_jk), then the Landau frame T^{mu nu} u_nu = E u^mu:
// with u = gamma (1, v), Newton's method on
//   F_i(v) = (T^00 - T^0k v_k) v_i - T^0i + T^ij v_j = 0
// from v = (3/4) T^0i / T^00, the step halved while it leaves |v| < 1, and
// two full steps more once a step is below 1e-12.
// Output per cell (RSL_NMOM3 doubles): N^0..N^3, T^00, T^01, T^02, T^03,
// T^11, T^12, T^13, T^22, T^23, T^33, n, E, P, T, u^0..u^3; the derived
// fields are NaN where no timelike frame with E > 0 and n > 0 exists.
__device__ __forceinline__ bool landau3(const double (&N)[4], const double (&M)[10], double* out) {
    const double T00 = M[0], T0[3] = {M[1], M[2], M[3]};
    const double Tij[3][3] = {{M[4], M[5], M[6]}, {M[5], M[7], M[8]}, {M[6], M[8], M[9]}};
    if (!(T00 > 0.0)) return false;
    double v[3] = {0.75 * T0[0] / T00, 0.75 * T0[1] / T00, 0.75 * T0[2] / T00};
    {
        const double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        if (v2 >= 0.81) {
            const double s = 0.9 / sqrt(v2);
            v[0] *= s; v[1] *= s; v[2] *= s;
        }
    }
    bool conv = false;
    int polish = -1;   // steps still to take once the step length is at 1e-12
    for (int it = 0; it < 60 && !conv; ++it) {
        const double e = T00 - (T0[0] * v[0] + T0[1] * v[1] + T0[2] * v[2]);
        double F[3], J[3][3];
        for (int i = 0; i < 3; ++i) {
            F[i] = e * v[i] - T0[i] + Tij[i][0] * v[0] + Tij[i][1] * v[1] + Tij[i][2] * v[2];
            for (int l = 0; l < 3; ++l) J[i][l] = -v[i] * T0[l] + (i == l ? e : 0.0) + Tij[i][l];
        }
        // J d = F by Cramer's rule
        const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
        if (!(fabs(det) > 0.0)) return false;
        const double id = 1.0 / det;
        const double d0 = (F[0] * c00 + F[1] * (J[0][2] * J[2][1] - J[0][1] * J[2][2]) +
                           F[2] * (J[0][1] * J[1][2] - J[0][2] * J[1][1])) * id;
        const double d1 = (F[0] * c01 + F[1] * (J[0][0] * J[2][2] - J[0][2] * J[2][0]) +
                           F[2] * (J[0][2] * J[1][0] - J[0][0] * J[1][2])) * id;
        const double d2 = (F[0] * c02 + F[1] * (J[0][1] * J[2][0] - J[0][0] * J[2][1]) +
                           F[2] * (J[0][0] * J[1][1] - J[0][1] * J[1][0])) * id;
        double s = 1.0, w[3];
        for (int h = 0; h < 40; ++h) {
            w[0] = v[0] - s * d0; w[1] = v[1] - s * d1; w[2] = v[2] - s * d2;
            if (w[0] * w[0] + w[1] * w[1] + w[2] * w[2] < 1.0) break;
            s *= 0.5;
        }
        const double dn = s * sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        v[0] = w[0]; v[1] = w[1]; v[2] = w[2];
        // quadratic convergence: two more full steps after 1e-12 reach the last
        // bit; a step cut back at |v| = 1 is no convergence (the root, if any,
        // lies outside: no timelike eigenvector)
        if (s < 1.0) polish = -1;
        else if (polish < 0 && dn <= 1e-12) polish = 2;
        else if (polish > 0 && --polish == 0) conv = true;
    }
    const double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    if (!conv || !(v2 < 1.0)) return false;
    const double E = T00 - (T0[0] * v[0] + T0[1] * v[1] + T0[2] * v[2]);
    const double gam = 1.0 / sqrt(1.0 - v2);
    const double n = gam * (N[0] - (N[1] * v[0] + N[2] * v[1] + N[3] * v[2]));
    if (!(E > 0.0) || !(n > 0.0)) return false;
    out[0] = n;
    out[1] = E;
    out[2] = E / 3.0;
    out[3] = E / (3.0 * n);
    out[4] = gam;
    out[5] = gam * v[0];
    out[6] = gam * v[1];
    out[7] = gam * v[2];
    return true;
}

template <typename Tf>
__global__ void __launch_bounds__(kV3Threads) moments3_kernel(const Tf* __restrict__ f, int pitch, int ncell,
                                                               CP arec, CP rrec, int A, int QL,
                                                               double* __restrict__ out) {
    const int cell = blockIdx.x * kV3Threads + threadIdx.x;
    if (cell >= ncell) return;
    double N[4] = {0.0, 0.0, 0.0, 0.0};
    double M[10] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    // plane by plane (radial node outer): consecutive loads walk neighbouring
    // velocity rows of one plane
    for (int k = 0; k < QL; ++k) {
        const double p = rrec[4 * k];
        const Tf* fk = f + (size_t)k * A * pitch + cell;
#pragma unroll 8
        for (int a = 0; a < A; ++a) {
            CP r = arec + 4 * (size_t)a;
            const double ox = r[0], oy = r[1], oz = r[2];
            const double fv = (double)fk[(size_t)a * pitch];
            const double pf = p * fv;
            N[0] += fv;
            N[1] = fma(ox, fv, N[1]);
            N[2] = fma(oy, fv, N[2]);
            N[3] = fma(oz, fv, N[3]);
            M[0] += pf;
            const double px = ox * pf, py = oy * pf, pz = oz * pf;
            M[1] += px;
            M[2] += py;
            M[3] += pz;
            M[4] = fma(ox, px, M[4]);
            M[5] = fma(oy, px, M[5]);
            M[6] = fma(oz, px, M[6]);
            M[7] = fma(oy, py, M[7]);
            M[8] = fma(oz, py, M[8]);
            M[9] = fma(oz, pz, M[9]);
        }
    }
    double* o = out + (size_t)cell * RSL_NMOM3;
    for (int i = 0; i < 4; ++i) o[i] = N[i];
    for (int i = 0; i < 10; ++i) o[4 + i] = M[i];
    double d[8];
    if (!landau3(N, M, d))
        for (int i = 0; i < 8; ++i) d[i] = __builtin_nan("");
    for (int i = 0; i < 8; ++i) o[14 + i] = d[i];
}

}  // namespace

int launch_feq3(const Quad3Dev& q, const double* state, int ncell, int dtype, void* f, int pitch, hipStream_t s) {
    const int nb = (ncell + kV3Threads - 1) / kV3Threads;
    if (dtype == RSL_F32)
        hipLaunchKernelGGL(feq3_kernel<float>, dim3(nb), dim3(kV3Threads), 0, s, state, ncell, (CP)q.arec,
                           (CP)q.rrec, q.A, q.QL, q.NOm, q.T0, q.beta_series, (CP)q.ser, (CP)q.thr, (float*)f,
                           pitch);
    else
        hipLaunchKernelGGL(feq3_kernel<double>, dim3(nb), dim3(kV3Threads), 0, s, state, ncell, (CP)q.arec,
                           (CP)q.rrec, q.A, q.QL, q.NOm, q.T0, q.beta_series, (CP)q.ser, (CP)q.thr, (double*)f,
                           pitch);
    return hip_check(hipGetLastError(), "feq3 launch");
}

int launch_moments3(const Quad3Dev& q, const void* f, int dtype, int ncell, int pitch, double* out, hipStream_t s) {
    const int nb = (ncell + kV3Threads - 1) / kV3Threads;
    if (dtype == RSL_F32)
        hipLaunchKernelGGL(moments3_kernel<float>, dim3(nb), dim3(kV3Threads), 0, s, (const float*)f, pitch, ncell,
                           (CP)q.arec, (CP)q.rrec, q.A, q.QL, out);
    else
        hipLaunchKernelGGL(moments3_kernel<double>, dim3(nb), dim3(kV3Threads), 0, s, (const double*)f, pitch,
                           ncell, (CP)q.arec, (CP)q.rrec, q.A, q.QL, out);
    return hip_check(hipGetLastError(), "moments3 launch");
}

}  // namespace rsl
