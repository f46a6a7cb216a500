/*
 * rslo.c -- plain FP64 CPU oracle for the R-SLB time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this code.  It shares no code, header
 * or table generator with the HIP library: velocity-set tables come from
 * oracle/quadrature.py, everything else is written out here from the paper.
 *
 * Compiled with  gcc -O2 -ffp-contract=off -fPIC -shared  (no FMA contraction,
 * summation in the written order: radial index k outer, angular index j inner,
 * both ascending).
 *
 * Notation (Ambrus & Blaga, arXiv:1612.01287):
 *   f[v][s], v = k*Q + j          distribution f_{jk} in cell s     (eq. fjk)
 *   xi[j], wx[j]                  Gauss-Legendre nodes/weights      (eq. quad_xi)
 *   pb[k], wl[k]                  Gauss-Laguerre(alpha=2)           (eq. wL, Table I)
 *   T0                            radial reference temperature, p_k = T0 * pb[k]
 *
 * Every function says which passage it follows.  Parity pins live in
 * tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define O_OK 0
#define O_EBADSTATE (-1)
#define O_ENOMEM (-2)

/* ---------------------------------------------------------------- tables */

/* Legendre polynomials P_0..P_mmax at x by the Bonnet recurrence. */
static void o_legendre(int mmax, double x, double *P)
{
    P[0] = 1.0;
    if (mmax >= 1) P[1] = x;
    for (int m = 1; m < mmax; ++m)
        P[m + 1] = ((2.0 * m + 1.0) * x * P[m] - m * P[m - 1]) / (m + 1.0);
}

/* ------------------------------------------------ equilibrium coefficients */

/*
 * a~_{l,m}(u, theta) for l = 0,1 and m = 0..NOm, written out from its
 * definition (Sec. III D, eq. aeq_aux, with the normalisation of App. A):
 *   a_{l,m} = n (l+1)(l+2)/(8 pi) Int_{-1}^{1} dc (u0 - u c)^{-3}
 *                                   (1 - theta/(u0 - u c))^l P_m(c),
 *   a_{l,m} = n (l+1)(l+2) u0 a~_{l,m} / (4 pi)
 * so  a~_{l,m} = 1/(2 u0) Int dc (u0 - u c)^{-3} (1 - theta/(u0 - u c))^l P_m(c).
 * The c-integral is done with the ng-point Gauss-Legendre rule (xg, wg);
 * u is the signed spatial four-velocity beta*gamma (cos gamma_u = sgn(u) xi).
 * Output at[l*(NOm+1) + m].
 */
void o_atilde(int NOm, double beta, double theta, int ng, const double *xg,
              const double *wg, double *at)
{
    double gam = 1.0 / sqrt(1.0 - beta * beta);
    double u0 = gam, u = beta * gam;
    double P[64];
    for (int i = 0; i < 2 * (NOm + 1); ++i) at[i] = 0.0;
    for (int g = 0; g < ng; ++g) {
        double c = xg[g];
        double D = u0 - u * c;
        double base = 1.0 / (D * D * D);
        double corr = 1.0 - theta / D;
        o_legendre(NOm, c, P);
        for (int m = 0; m <= NOm; ++m) {
            at[m] += wg[g] * base * P[m];
            at[(NOm + 1) + m] += wg[g] * base * corr * P[m];
        }
    }
    for (int i = 0; i < 2 * (NOm + 1); ++i) at[i] /= (2.0 * u0);
}

/*
 * f^eq_{jk} of the truncated expansion (Sec. III D, eq. feq_trunc, N_L = 1)
 * mapped to the discrete populations by eq. fjk:
 *   f^eq(p, xi) = T0^-3 e^{-pb} sum_{l<=1} L_l(pb)/((l+1)(l+2))
 *                 sum_{m<=NOm} (2m+1)/2 a_{l,m} P_m(xi)
 *   f_{jk}     = 2 pi T0^3 e^{pb_k} w_j w_k f(p_k, xi_j)
 * with L_0 = 1, L_1 = 3 - x (eq. lag_expl).  feq[k*Q + j].
 */
void o_feq(int QL, int Q, int NOm, const double *xi, const double *wx,
           const double *pb, const double *wl, double T0,
           int ng, const double *xg, const double *wg,
           double n, double T, double beta, double *feq)
{
    const double PI = 3.14159265358979323846;
    double at[32], a[32], P[64];
    double gam = 1.0 / sqrt(1.0 - beta * beta);
    double theta = T / T0;
    o_atilde(NOm, beta, theta, ng, xg, wg, at);
    for (int l = 0; l <= 1; ++l)
        for (int m = 0; m <= NOm; ++m)
            a[l * (NOm + 1) + m] = n * (l + 1.0) * (l + 2.0) * gam * at[l * (NOm + 1) + m] / (4.0 * PI);
    for (int k = 0; k < QL; ++k) {
        double x = pb[k];
        double Ll[2] = {1.0, 3.0 - x};
        for (int j = 0; j < Q; ++j) {
            o_legendre(NOm, xi[j], P);
            double fc = 0.0;
            for (int l = 0; l <= 1; ++l) {
                double s = 0.0;
                for (int m = 0; m <= NOm; ++m)
                    s += (2.0 * m + 1.0) / 2.0 * a[l * (NOm + 1) + m] * P[m];
                fc += Ll[l] / ((l + 1.0) * (l + 2.0)) * s;
            }
            fc *= exp(-x) / (T0 * T0 * T0);
            feq[k * Q + j] = 2.0 * PI * T0 * T0 * T0 * exp(x) * wx[j] * wl[k] * fc;
        }
    }
}

/* ---------------------------------------------------------------- moments */

/* N^0, N^z, T^00, T^0z, T^zz of one cell (Sec. III E, eq. macro_jk);
 * f is strided: population v at f[v*stride]. */
static void o_cell_moments(int QL, int Q, const double *xi, const double *pb,
                           double T0, const double *f, long stride, double *M)
{
    M[0] = M[1] = M[2] = M[3] = M[4] = 0.0;
    for (int k = 0; k < QL; ++k) {
        double p = T0 * pb[k];
        for (int j = 0; j < Q; ++j) {
            double v = f[(long)(k * Q + j) * stride];
            M[0] += v;
            M[1] += xi[j] * v;
            M[2] += p * v;
            M[3] += p * xi[j] * v;
            M[4] += p * xi[j] * xi[j] * v;
        }
    }
}

/*
 * Landau frame of the Sod stress tensor (Sec. II E, eqs. E_landau, u_landau)
 * and n = -u.N, P = E/3, T = P/n (eqs. EL_def, T_def).
 * out = {E, beta, gamma, n, P, T}.  Returns O_EBADSTATE for an unphysical
 * state (negative discriminant, |beta| >= 1, n <= 0 or non-finite values).
 */
int o_landau(const double *M, double *out)
{
    double T00 = M[2], T0z = M[3], Tzz = M[4];
    double disc = (T00 + Tzz) * (T00 + Tzz) - 4.0 * T0z * T0z;
    if (!(disc >= 0.0)) return O_EBADSTATE;
    double E = 0.5 * (T00 - Tzz + sqrt(disc));
    double beta = T0z / (E + Tzz);
    if (!(fabs(beta) < 1.0)) return O_EBADSTATE;
    double gam = 1.0 / sqrt(1.0 - beta * beta);
    double n = gam * (M[0] - beta * M[1]);
    if (!(n > 0.0) || !(E > 0.0)) return O_EBADSTATE;
    double P = E / 3.0;
    out[0] = E; out[1] = beta; out[2] = gam; out[3] = n; out[4] = P; out[5] = P / n;
    return O_OK;
}

/*
 * Derived output fields of one Sod cell:
 * {N0, Nz, T00, T0z, Tzz, n, E, P, T, beta, lambda_bar, q, Pi}
 * lambda_bar = n/T^3 (relative fugacity, eq. lambda), q = -4T(N^z - n beta gamma)
 * (eq. q_val), Pi = 2E/3 - T^00 + T^zz (eq. pi_val).
 */
int o_sod_moments(int QL, int Q, const double *xi, const double *pb, double T0,
                  int nz, const double *f, double *out)
{
    int rc = O_OK;
    for (int s = 0; s < nz; ++s) {
        double M[5], L[6];
        o_cell_moments(QL, Q, xi, pb, T0, f + s, nz, M);
        double *o = out + 13L * s;
        for (int i = 0; i < 5; ++i) o[i] = M[i];
        if (o_landau(M, L) != O_OK) {
            rc = O_EBADSTATE;
            for (int i = 5; i < 13; ++i) o[i] = NAN;
            continue;
        }
        double E = L[0], beta = L[1], gam = L[2], n = L[3], P = L[4], T = L[5];
        o[5] = n; o[6] = E; o[7] = P; o[8] = T; o[9] = beta;
        o[10] = n / (T * T * T);
        o[11] = -4.0 * T * (M[1] - n * beta * gam);
        o[12] = 2.0 * E / 3.0 - M[2] + M[4];
    }
    return rc;
}

/* ------------------------------------------------------------------ WENO5 */

/*
 * WENO5 numerical flux at one interface (Sec. III F, eqs. flux_weno,
 * weno5_omega).  The five values are given in upwind order: for xi > 0,
 * (a,b,c,d,e) = (J_{s-2}, J_{s-1}, J_s, J_{s+1}, J_{s+2}) for F_{s+1/2}; for
 * xi < 0 the mirror image (J_{s+3}, J_{s+2}, J_{s+1}, J_s, J_{s-1}).
 * Limiting cases (i)-(iii) of the paper are applied, in that order, on exact
 * zeros / exact equality of the smoothness indicators; no epsilon regulariser.
 */
double o_weno5(double a, double b, double c, double d, double e)
{
    const double dl[3] = {0.1, 0.6, 0.3};
    double F[3], sg[3], w[3];
    F[0] = a / 3.0 - 7.0 * b / 6.0 + 11.0 * c / 6.0;
    F[1] = -b / 6.0 + 5.0 * c / 6.0 + d / 3.0;
    F[2] = c / 3.0 + 5.0 * d / 6.0 - e / 6.0;
    sg[0] = 13.0 / 12.0 * (a - 2.0 * b + c) * (a - 2.0 * b + c) + 0.25 * (a - 4.0 * b + 3.0 * c) * (a - 4.0 * b + 3.0 * c);
    sg[1] = 13.0 / 12.0 * (b - 2.0 * c + d) * (b - 2.0 * c + d) + 0.25 * (b - d) * (b - d);
    sg[2] = 13.0 / 12.0 * (c - 2.0 * d + e) * (c - 2.0 * d + e) + 0.25 * (3.0 * c - 4.0 * d + e) * (3.0 * c - 4.0 * d + e);
    int nzero = (sg[0] == 0.0) + (sg[1] == 0.0) + (sg[2] == 0.0);
    if (sg[0] == sg[1] && sg[1] == sg[2]) {                 /* case (i) */
        w[0] = dl[0]; w[1] = dl[1]; w[2] = dl[2];
    } else if (nzero == 2) {                                /* case (ii) */
        double den = 0.0;
        for (int q = 0; q < 3; ++q) if (sg[q] == 0.0) den += dl[q];
        for (int q = 0; q < 3; ++q) w[q] = (sg[q] == 0.0) ? dl[q] / den : 0.0;
    } else if (nzero == 1) {                                /* case (iii) */
        for (int q = 0; q < 3; ++q) w[q] = (sg[q] == 0.0) ? 1.0 : 0.0;
    } else {
        double wt[3], sum = 0.0;
        for (int q = 0; q < 3; ++q) { wt[q] = dl[q] / (sg[q] * sg[q]); sum += wt[q]; }
        for (int q = 0; q < 3; ++q) w[q] = wt[q] / sum;
    }
    return w[0] * F[0] + w[1] * F[1] + w[2] * F[2];
}

/* -------------------------------------------------------------- Sod solver */

typedef struct {
    int QL, Q, NOm;
    const double *xi, *wx, *pb, *wl;
    double T0;
    int ng;
    const double *xg, *wg;
    int nz;
    double zlo, zhi;
    int tau_mode;          /* 0 CONST, 1 ETAS (eq. Sod:tau), 2 INF (collisionless) */
    double tau_r;          /* CONST */
    double tau_aw0;        /* ETAS: tau_{A-W;0} of eq. Sod:tau */
    double lambda_ref;     /* ETAS */
    int bc;                /* 0: ghosts fixed to f^eq_L/R (Sec. IV A); 1: zero-gradient outflow */
    int store_f32;         /* round f to binary32 after every RK stage */
    const double *feqL, *feqR;   /* [V] ghost states for bc = 0 */
} o_sod_t;

/* Relaxation time of one Sod cell (exported so that tests can pin it). */
double o_relax_time(const o_sod_t *S, double n, double T)
{
    if (S->tau_mode == 0) return S->tau_r;
    /* eq. Sod:tau with lambda_bar = n / T^3 (eq. lambda) */
    double lam = n / (T * T * T);
    return S->tau_aw0 / T * (1.0 - 0.25 * log(lam * S->lambda_ref));
}

/*
 * L_Sod[f] of eq. L_Sod for all interior cells:
 *   L = -(F_{s+1/2} - F_{s-1/2})/dz - gamma (1 - beta xi_j)/tau (f - f^eq).
 * f, L: [V][nz].  Ghost cells (3 per side, Sec. IV A) are filled from bc.
 */
int o_sod_L(const o_sod_t *S, const double *f, double *L)
{
    int Q = S->Q, V = S->QL * S->Q, nz = S->nz, ne = nz + 6;
    double dz = (S->zhi - S->zlo) / nz;
    double *fe = (double *)malloc(sizeof(double) * (size_t)V * ne);
    double *feq = (double *)malloc(sizeof(double) * V);
    double *col = (double *)malloc(sizeof(double) * V);
    double *Fl = (double *)malloc(sizeof(double) * (nz + 1));
    if (!fe || !feq || !col || !Fl) { free(fe); free(feq); free(col); free(Fl); return O_ENOMEM; }
    int rc = O_OK;
    /* extended array: fe[v][s+3], s = -3 .. nz+2 */
    for (int v = 0; v < V; ++v) {
        for (int s = 0; s < nz; ++s) fe[(long)v * ne + s + 3] = f[(long)v * nz + s];
        for (int g = 0; g < 3; ++g) {
            fe[(long)v * ne + g] = S->bc == 0 ? S->feqL[v] : f[(long)v * nz + 0];
            fe[(long)v * ne + nz + 3 + g] = S->bc == 0 ? S->feqR[v] : f[(long)v * nz + nz - 1];
        }
    }
    /* advection: fluxes at the nz+1 faces s+1/2, s = -1 .. nz-1 */
    for (int v = 0; v < V; ++v) {
        int j = v % Q;
        double x = S->xi[j];
        const double *J0 = fe + (long)v * ne + 3;   /* J0[s] = f at cell s */
        for (int s = -1; s < nz; ++s) {
            double F;
            if (x > 0.0)
                F = o_weno5(x * J0[s - 2], x * J0[s - 1], x * J0[s], x * J0[s + 1], x * J0[s + 2]);
            else if (x < 0.0)
                F = o_weno5(x * J0[s + 3], x * J0[s + 2], x * J0[s + 1], x * J0[s], x * J0[s - 1]);
            else
                F = 0.0;
            Fl[s + 1] = F;
        }
        for (int s = 0; s < nz; ++s)
            L[(long)v * nz + s] = -(Fl[s + 1] - Fl[s]) / dz;
    }
    /* collision term, cell by cell */
    if (S->tau_mode != 2) {
        for (int s = 0; s < nz; ++s) {
            double M[5], Ld[6];
            for (int v = 0; v < V; ++v) col[v] = f[(long)v * nz + s];
            o_cell_moments(S->QL, Q, S->xi, S->pb, S->T0, col, 1, M);
            if (o_landau(M, Ld) != O_OK) { rc = O_EBADSTATE; continue; }
            double beta = Ld[1], gam = Ld[2], n = Ld[3], T = Ld[5];
            double tau = o_relax_time(S, n, T);
            o_feq(S->QL, Q, S->NOm, S->xi, S->wx, S->pb, S->wl, S->T0, S->ng, S->xg, S->wg,
                  n, T, beta, feq);
            for (int v = 0; v < V; ++v) {
                int j = v % Q;
                L[(long)v * nz + s] += -gam * (1.0 - beta * S->xi[j]) / tau * (col[v] - feq[v]);
            }
        }
    }
    free(fe); free(feq); free(col); free(Fl);
    return rc;
}

static void o_round32(double *f, long n)
{
    for (long i = 0; i < n; ++i) f[i] = (double)(float)f[i];
}

/*
 * nsteps of the TVD RK3 scheme (Sec. III F, eq. rk3) on the Sod operator.
 * f [V][nz] is updated in place.
 */
int o_sod_run(const o_sod_t *S, double *f, double dt, int nsteps)
{
    long N = (long)S->QL * S->Q * S->nz;
    double *f1 = (double *)malloc(sizeof(double) * N);
    double *f2 = (double *)malloc(sizeof(double) * N);
    double *Lb = (double *)malloc(sizeof(double) * N);
    if (!f1 || !f2 || !Lb) { free(f1); free(f2); free(Lb); return O_ENOMEM; }
    int rc = O_OK;
    for (int it = 0; it < nsteps && rc == O_OK; ++it) {
        rc = o_sod_L(S, f, Lb);
        for (long i = 0; i < N; ++i) f1[i] = f[i] + dt * Lb[i];
        if (S->store_f32) o_round32(f1, N);
        if (rc == O_OK) rc = o_sod_L(S, f1, Lb);
        for (long i = 0; i < N; ++i) f2[i] = 0.75 * f[i] + 0.25 * f1[i] + 0.25 * dt * Lb[i];
        if (S->store_f32) o_round32(f2, N);
        if (rc == O_OK) rc = o_sod_L(S, f2, Lb);
        for (long i = 0; i < N; ++i) f[i] = f[i] / 3.0 + 2.0 * f2[i] / 3.0 + 2.0 * dt * Lb[i] / 3.0;
        if (S->store_f32) o_round32(f, N);
    }
    free(f1); free(f2); free(Lb);
    return rc;
}

/*
 * Sod initial state (Sec. IV A): f = f^eq_L for z_s < 0, f^eq_R for z_s > 0,
 * cell centres z_s = (s - 1/2) dz - L/2 (Sec. III F).  A cell centred exactly
 * on the membrane (odd nz) takes the average of the two states.
 */
void o_sod_init(const o_sod_t *S, double *f)
{
    int V = S->QL * S->Q, nz = S->nz;
    double dz = (S->zhi - S->zlo) / nz;
    double zm = 0.5 * (S->zlo + S->zhi);
    for (int s = 0; s < nz; ++s) {
        double z = S->zlo + (s + 0.5) * dz;
        for (int v = 0; v < V; ++v) {
            double val;
            if (z < zm && fabs(z - zm) > 0.25 * dz) val = S->feqL[v];
            else if (z > zm && fabs(z - zm) > 0.25 * dz) val = S->feqR[v];
            else val = 0.5 * (S->feqL[v] + S->feqR[v]);
            f[(long)v * nz + s] = val;
        }
    }
}

/* ----------------------------------------------------------- Bjorken flow */

typedef struct {
    int QL, Q, NOm;
    const double *xi, *wx, *pb, *wl;
    double T0;
    int ng;
    const double *xg, *wg;
    const double *KL;      /* [QL][QL]  eq. K_lag_disc */
    const double *KP;      /* [Q][Q]    eq. K_leg_disc */
    int gas;               /* 0 ideal (P = nT), 1 parton (n_eq = T^3, T = P^{1/4}) */
    int tau_mode;          /* 0 CONST, 1 ETAS, 2 INF */
    double tau_r;
    double tau_aw0;        /* eq. bjorken_tauAW */
    double lambda_ref;
    int store_f32;
} o_bj_t;

/* n = N^tau, E = T^{tau tau}, P_L = T^{eta eta} of one instance (eq. bjorken_SET). */
static void o_bj_moments(const o_bj_t *B, const double *f, double *n, double *E, double *PL)
{
    double M[5];
    o_cell_moments(B->QL, B->Q, B->xi, B->pb, B->T0, f, 1, M);
    *n = M[0]; *E = M[2]; *PL = M[4];
}

/*
 * L_Bjorken[f] at proper time tau (eq. L_Bjorken):
 *   -f/tau + xi_j^2/tau sum_k' K^L_{kk'} f_{jk'} + 1/tau sum_j' K^P_{jj'} f_{j'k}
 *   - (f - f^eq)/tau_AW,
 * with u = (1,0,0,0), P = E/3; ideal gas n_eq = n, T = P/n, tau_AW by eq.
 * bjorken_tauAW; parton gas T = P^{1/4}, n_eq = T^3, tau_AW = tau_AW0/T
 * (eqs. bjorken_mu0, bjorken_tauAW0).
 */
int o_bj_L(const o_bj_t *B, const double *f, double tau, double *L, double *feq)
{
    int Q = B->Q, QL = B->QL;
    double n, E, PL;
    o_bj_moments(B, f, &n, &E, &PL);
    double P = E / 3.0;
    for (int k = 0; k < QL; ++k)
        for (int j = 0; j < Q; ++j) {
            double acc = -f[k * Q + j] / tau;
            double sl = 0.0;
            for (int kp = 0; kp < QL; ++kp) sl += B->KL[k * QL + kp] * f[kp * Q + j];
            acc += B->xi[j] * B->xi[j] / tau * sl;
            double sp = 0.0;
            for (int jp = 0; jp < Q; ++jp) sp += B->KP[j * Q + jp] * f[k * Q + jp];
            acc += sp / tau;
            L[k * Q + j] = acc;
        }
    if (B->tau_mode == 2) return O_OK;
    double T, neq, taw;
    if (B->gas == 0) {
        if (!(n > 0.0) || !(P > 0.0)) return O_EBADSTATE;
        T = P / n; neq = n;
        if (B->tau_mode == 0) taw = B->tau_r;
        else taw = B->tau_aw0 / T * (1.0 - 0.25 * log(n / (T * T * T) * B->lambda_ref));
    } else {
        if (!(P > 0.0)) return O_EBADSTATE;
        T = pow(P, 0.25); neq = T * T * T;
        taw = B->tau_mode == 0 ? B->tau_r : B->tau_aw0 / T;
    }
    o_feq(QL, Q, B->NOm, B->xi, B->wx, B->pb, B->wl, B->T0, B->ng, B->xg, B->wg,
          neq, T, 0.0, feq);
    for (int v = 0; v < QL * Q; ++v) L[v] -= (f[v] - feq[v]) / taw;
    return O_OK;
}

/*
 * nsteps of RK3 (eq. rk3) for one Bjorken instance from proper time *tau;
 * stage times tau_n, tau_n + dtau, tau_n + dtau/2 (Butcher tableau, Table II).
 * hist (optional, [nsteps+1][3]) receives (n, E, P_L) before the first step and
 * after every step.
 */
int o_bj_run(const o_bj_t *B, double *f, double *tau, double dtau, int nsteps, double *hist)
{
    int V = B->QL * B->Q;
    double *f1 = (double *)malloc(sizeof(double) * V);
    double *f2 = (double *)malloc(sizeof(double) * V);
    double *Lb = (double *)malloc(sizeof(double) * V);
    double *feq = (double *)malloc(sizeof(double) * V);
    if (!f1 || !f2 || !Lb || !feq) { free(f1); free(f2); free(Lb); free(feq); return O_ENOMEM; }
    int rc = O_OK;
    double t = *tau;
    if (hist) o_bj_moments(B, f, &hist[0], &hist[1], &hist[2]);
    for (int it = 0; it < nsteps && rc == O_OK; ++it) {
        rc = o_bj_L(B, f, t, Lb, feq);
        for (int v = 0; v < V; ++v) f1[v] = f[v] + dtau * Lb[v];
        if (B->store_f32) o_round32(f1, V);
        if (rc == O_OK) rc = o_bj_L(B, f1, t + dtau, Lb, feq);
        for (int v = 0; v < V; ++v) f2[v] = 0.75 * f[v] + 0.25 * f1[v] + 0.25 * dtau * Lb[v];
        if (B->store_f32) o_round32(f2, V);
        if (rc == O_OK) rc = o_bj_L(B, f2, t + 0.5 * dtau, Lb, feq);
        for (int v = 0; v < V; ++v) f[v] = f[v] / 3.0 + 2.0 * f2[v] / 3.0 + 2.0 * dtau * Lb[v] / 3.0;
        if (B->store_f32) o_round32(f, V);
        t = *tau + (it + 1) * dtau;
        if (hist) o_bj_moments(B, f, &hist[3 * (it + 1)], &hist[3 * (it + 1) + 1], &hist[3 * (it + 1) + 2]);
    }
    *tau = t;
    free(f1); free(f2); free(Lb); free(feq);
    return rc;
}
