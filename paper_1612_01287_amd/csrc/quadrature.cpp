// Velocity-set construction for R-SLB(N_Omega; Q_xi) on the host (Sec. III).
//
// Gauss-Legendre nodes/weights (eq. quad_xi), generalised Gauss-Laguerre
// nodes/weights for the weight x^2 e^{-x} (eq. wL, Table I), the Legendre
// table P_m(xi_j), the discrete momentum-space kernels K^L (eq. K_lag_disc)
// and K^P (eq. K_leg_disc), and the Maclaurin tables used by the kernels for
// the equilibrium coefficients.  Everything is computed in x87 extended
// precision and rounded once to binary64.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "rsl_impl.h"

namespace rsl {

namespace {

using ld = long double;

// P_n(x) and P_{n-1}(x) by the Bonnet recurrence.
void legendre_pair(int n, ld x, ld* pn, ld* pnm1) {
    ld p0 = 1.0L, p1 = x;
    if (n == 0) { *pn = 1.0L; *pnm1 = 0.0L; return; }
    for (int m = 1; m < n; ++m) {
        ld p2 = ((2 * m + 1) * x * p1 - m * p0) / (m + 1);
        p0 = p1;
        p1 = p2;
    }
    *pn = p1;
    *pnm1 = p0;
}

// Ascending Gauss-Legendre nodes: Newton from the Tricomi-type initial guess,
// weights of eq. quad_xi; exact mirror symmetry imposed.
void gauss_legendre(int Q, std::vector<double>& xi, std::vector<double>& w) {
    std::vector<ld> x(Q), wt(Q);
    const ld pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < Q; ++i) {
        ld r = cosl(pi * (i + 0.75L) / (Q + 0.5L));   // descending in i
        for (int it = 0; it < 100; ++it) {
            ld p, pm1;
            legendre_pair(Q, r, &p, &pm1);
            ld dp = Q * (r * p - pm1) / (r * r - 1.0L);
            ld dr = p / dp;
            r -= dr;
            if (fabsl(dr) < 1e-21L * (1.0L + fabsl(r))) break;
        }
        // At a root of P_Q the weight of eq. quad_xi equals 2(1 - x^2)/[Q (P_{Q-1} - x P_Q)]^2;
        // (1 - x^2) P_Q' = Q (P_{Q-1} - x P_Q) is stationary at the root (Legendre's
        // equation), so this form does not amplify the last-bit error of the node.
        ld pq, pqm1;
        legendre_pair(Q, r, &pq, &pqm1);
        const ld g = Q * (pqm1 - r * pq);
        x[Q - 1 - i] = r;
        wt[Q - 1 - i] = 2.0L * (1.0L - r * r) / (g * g);
    }
    xi.assign(Q, 0.0);
    w.assign(Q, 0.0);
    for (int j = 0; j < Q; ++j) {
        ld a = 0.5L * (x[j] - x[Q - 1 - j]);
        ld b = 0.5L * (wt[j] + wt[Q - 1 - j]);
        xi[j] = (double)a;
        w[j] = (double)b;
    }
    if (Q % 2 == 1) xi[Q / 2] = 0.0;
}

// L_l^{(2)}(x) from its explicit sum (eq. lag_expl).
ld laguerre2(int l, ld x) {
    ld s = 0.0L, term;
    for (int k = 0; k <= l; ++k) {
        term = tgammal(l + 3) / (tgammal(k + 1) * tgammal(k + 3) * tgammal(l - k + 1));
        s += ((k % 2) ? -1.0L : 1.0L) * powl(x, k) * term;
    }
    return s;
}

// Roots of L_Q^{(2)} by sign-change scan and bisection; weights of eq. wL:
// w_k = x_k (Q+2) / ((Q+1) [L_{Q+1}^{(2)}(x_k)]^2).
int gauss_laguerre2(int QL, std::vector<double>& x, std::vector<double>& w) {
    std::vector<ld> roots;
    const ld hi = 4.0L * QL + 12.0L, h = 1.0L / 1024.0L;
    ld a = 1e-12L, fa = laguerre2(QL, a);
    for (ld b = a + h; b <= hi && (int)roots.size() < QL; b += h) {
        ld fb = laguerre2(QL, b);
        if ((fa < 0) != (fb < 0)) {
            ld lo = a, up = b, flo = fa;
            for (int it = 0; it < 200; ++it) {
                ld mid = 0.5L * (lo + up);
                ld fm = laguerre2(QL, mid);
                if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else { up = mid; }
                if (up - lo <= 1e-19L * up) break;
            }
            roots.push_back(0.5L * (lo + up));
        }
        a = b;
        fa = fb;
    }
    if ((int)roots.size() != QL) return -1;
    x.resize(QL);
    w.resize(QL);
    for (int k = 0; k < QL; ++k) {
        ld r = roots[k];
        // one Newton polish on the exact polynomial: d/dx L_l^(2) = -L_{l-1}^(3); use
        // a symmetric difference in extended precision instead
        ld hh = 1e-7L * (1.0L + r);
        ld d = (laguerre2(QL, r + hh) - laguerre2(QL, r - hh)) / (2 * hh);
        r -= laguerre2(QL, r) / d;
        ld l1 = laguerre2(QL + 1, r);
        x[k] = (double)r;
        w[k] = (double)(r * (QL + 2) / ((QL + 1) * l1 * l1));
    }
    return 0;
}

// Integral of c^n P_m(c) over [-1, 1] for n >= m, n - m even:
//   2^{m+1} n! ((n+m)/2)! / (((n-m)/2)! (n+m+1)!).
ld moment_cn_pm(int n, int m) {
    ld lg = (m + 1) * logl(2.0L) + lgammal(n + 1.0L) + lgammal((n + m) / 2 + 1.0L) -
            lgammal((n - m) / 2 + 1.0L) - lgammal(n + m + 2.0L);
    return expl(lg);
}

// Maclaurin coefficients of K_{k,m}(beta) = beta^m sum_i a_i beta^{2i}:
// (1 - beta c)^{-k} = sum_n C(n+k-1, k-1) beta^n c^n, so
// a_i = C(m+2i+k-1, k-1) int c^{m+2i} P_m.  thr[i] is the largest beta^2 for
// which the first i terms of every (k, m) series carry all but 2^-58 of it.
void series_tables(std::vector<double>& ser, std::vector<double>& thr) {
    const int NT = kSeriesTerms, NM = kMaxNOm + 1;
    static std::vector<double> cser, cthr;
    static std::once_flag once;
    std::call_once(once, [&] {
        std::vector<ld> A(2 * NM * 4 * NT);
        const int NA = 4 * NT;   // long tail for the threshold search
        auto coef = [&](int k, int m, int i) -> ld {
            int n = m + 2 * i;
            ld c = (k == 3) ? (ld)(n + 2) * (n + 1) / 2.0L : (ld)(n + 3) * (n + 2) * (n + 1) / 6.0L;
            return c * moment_cn_pm(n, m);
        };
        for (int kk = 0; kk < 2; ++kk)
            for (int m = 0; m < NM; ++m)
                for (int i = 0; i < NA; ++i) A[(kk * NM + m) * NA + i] = coef(3 + kk, m, i);
        cser.assign(2 * NM * NT, 0.0);
        for (int kk = 0; kk < 2; ++kk)
            for (int m = 0; m < NM; ++m)
                for (int i = 0; i < NT; ++i) cser[(size_t)i * 2 * NM + kk * NM + m] = (double)A[(kk * NM + m) * NA + i];
        auto ok = [&](int nt, ld x) {
            for (int s = 0; s < 2 * NM; ++s) {
                ld head = 0.0L, tail = 0.0L, p = 1.0L;
                for (int i = 0; i < NA; ++i) {
                    (i < nt ? head : tail) += A[s * NA + i] * p;
                    p *= x;
                    if (i >= nt && A[s * NA + i] * p < 1e-40L * head) break;
                }
                if (tail > ldexpl(head, -58)) return false;
            }
            return true;
        };
        cthr.assign(NT, 0.0);
        for (int nt = 1; nt < NT; ++nt) {
            ld lo = 0.0L, hi = 0.6L;
            if (ok(nt, hi)) { cthr[nt] = (double)hi; continue; }
            for (int it = 0; it < 60; ++it) {
                ld mid = 0.5L * (lo + hi);
                if (ok(nt, mid)) lo = mid; else hi = mid;
            }
            cthr[nt] = (double)lo;
        }
        // more terms never need a smaller beta^2: keep the table ascending
        for (int nt = 2; nt < NT; ++nt) cthr[nt] = std::max(cthr[nt], cthr[nt - 1]);
    });
    ser = cser;
    thr = cthr;
}

}  // namespace

int build_quadrature(int QL, int Q, int NOm, double T0, rsl_quad* q) {
    q->QL = QL;
    q->Q = Q;
    q->NOm = NOm;
    q->V = QL * Q;
    q->T0 = T0;
    // the recurrence branch loses ~1/beta per order m (see rsl_math.h): at
    // these switches its K_{k,m} stay within ~4e-14 of the defining integrals
    // (1e-14 for N_Omega <= 3 at 0.4, 3e-14 for N_Omega = 4 at 0.45, 8e-13 for
    // N_Omega = 6 at 0.5, hence 0.7 from N_Omega = 5 on)
    q->beta_series = NOm <= 3 ? 0.4 : (NOm == 4 ? 0.45 : 0.7);
    gauss_legendre(Q, q->xi, q->wxi);
    if (gauss_laguerre2(QL, q->pbar, q->wL) != 0) return set_error(RSL_EINVAL, "Laguerre root search failed");
    // Legendre table up to m = Q + 1 in extended precision
    const int MM = Q + 2;
    std::vector<ld> P((size_t)MM * Q);
    for (int j = 0; j < Q; ++j) {
        ld x = q->xi[j], p0 = 1.0L, p1 = x;
        P[j] = p0;
        if (MM > 1) P[(size_t)Q + j] = p1;
        for (int m = 1; m + 1 < MM; ++m) {
            ld p2 = ((2 * m + 1) * x * p1 - m * p0) / (m + 1);
            P[(size_t)(m + 1) * Q + j] = p2;
            p0 = p1;
            p1 = p2;
        }
    }
    q->Pm.assign((size_t)(NOm + 1) * Q, 0.0);
    for (int m = 0; m <= NOm; ++m)
        for (int j = 0; j < Q; ++j) q->Pm[(size_t)m * Q + j] = (double)P[(size_t)m * Q + j];
    // K^L (eq. K_lag_disc)
    q->KL.assign((size_t)QL * QL, 0.0);
    for (int k = 0; k < QL; ++k)
        for (int kp = 0; kp < QL; ++kp) {
            ld s = 0.0L;
            for (int l = 1; l < QL; ++l)
                s += laguerre2(l, q->pbar[k]) *
                     ((l + 2) * laguerre2(l - 1, q->pbar[kp]) - l * laguerre2(l, q->pbar[kp])) /
                     ((ld)(l + 1) * (l + 2));
            q->KL[(size_t)k * QL + kp] = (double)(q->wL[k] * s);
        }
    // K^P (eq. K_leg_disc): sum over m of outer products
    std::vector<ld> KP((size_t)Q * Q, 0.0L), colv(Q);
    for (int m = 1; m <= Q - 1; ++m) {
        const ld c1 = (m <= Q - 3) ? (ld)m * (m + 1) * (m + 2) / (2.0L * (2 * m + 3)) : 0.0L;
        const ld c2 = (ld)m * (m + 1) / 2.0L;
        for (int jp = 0; jp < Q; ++jp) {
            ld v = -c2 * (2 * m + 1) * P[(size_t)m * Q + jp] / ((ld)(2 * m - 1) * (2 * m + 3));
            if (m >= 2) v -= c2 * (m - 1) / (ld)(2 * m - 1) * P[(size_t)(m - 2) * Q + jp];
            if (c1 != 0.0L) v += c1 * P[(size_t)(m + 2) * Q + jp];
            colv[jp] = v;
        }
        for (int j = 0; j < Q; ++j) {
            const ld a = (ld)q->wxi[j] * P[(size_t)m * Q + j];
            ld* row = &KP[(size_t)j * Q];
            for (int jp = 0; jp < Q; ++jp) row[jp] += a * colv[jp];
        }
    }
    q->KP.resize((size_t)Q * Q);
    for (size_t i = 0; i < KP.size(); ++i) q->KP[i] = (double)KP[i];
    series_tables(q->ser, q->thr);
    if (!(q->thr[kSeriesTerms - 1] >= q->beta_series * q->beta_series))
        return set_error(RSL_EINVAL, "Maclaurin tables too short for the series switch");
    return RSL_OK;
}

}  // namespace rsl
