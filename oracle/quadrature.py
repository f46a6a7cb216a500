"""Oracle tables: quadratures, polynomial tables and the momentum-space kernels.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module;
only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use it.

Everything here is plain FP64 numpy (nodes refined in mpmath), written from the
paper's definitions, and shares no code with the HIP library:

* Gauss-Legendre nodes/weights on xi = cos(theta): roots of P_Q, weights
  w_j = 2(1 - xi_j^2) / [(Q+1) P_{Q+1}(xi_j)]^2            (Sec. III C, eq. quad_xi)
* Gauss-Laguerre nodes/weights for the weight e^{-x} x^2: roots of L^(2)_Q,
  w_k = x_k (Q+2) / ((Q+1) [L^(2)_{Q+1}(x_k)]^2)           (Sec. III B, eq. wL, Table I)
* generalised Laguerre polynomials from their explicit sum   (eq. lag_expl)
* K^L (Q_L x Q_L) and K^P (Q_xi x Q_xi)                     (Sec. III E, eqs. K_lag_disc, K_leg_disc)

Pins: tests/test_oracle_quadrature.py (exactness of the rules, Table I,
closed-form actions of K^L and K^P derived by calculus).
"""
from functools import lru_cache
from math import factorial

import mpmath
import numpy as np

_MP_DPS = 40


def _legendre_mp(n, x):
    """P_n(x) and P_{n-1}(x) by the three-term (Bonnet) recurrence, mpmath."""
    p0, p1 = mpmath.mpf(1), x
    if n == 0:
        return p0, mpmath.mpf(0)
    for m in range(1, n):
        p0, p1 = p1, ((2 * m + 1) * x * p1 - m * p0) / (m + 1)
    return p1, p0


@lru_cache(maxsize=None)
def gauss_legendre(Q):
    """Ascending Gauss-Legendre nodes xi_j and weights w_j (eq. quad_xi).

    The library routine numpy.polynomial.legendre.leggauss gives the starting
    points; each root is then polished by Newton's method on P_Q in 40-digit
    arithmetic and the weight is evaluated from the paper's formula.  Nodes are
    made exactly antisymmetric (xi_{Q+1-j} = -xi_j).
    """
    x0, _ = np.polynomial.legendre.leggauss(Q)
    xs, ws = [], []
    with mpmath.workdps(_MP_DPS):
        for guess in x0:
            x = mpmath.mpf(float(guess))
            for _ in range(6):
                p, pm1 = _legendre_mp(Q, x)
                # P_Q'(x) = Q (x P_Q - P_{Q-1}) / (x^2 - 1)
                dp = Q * (x * p - pm1) / (x * x - 1)
                x = x - p / dp
            pq1, _ = _legendre_mp(Q + 1, x)
            w = 2 * (1 - x * x) / ((Q + 1) * pq1) ** 2
            xs.append(x)
            ws.append(w)
    xi = np.array([float(v) for v in xs])
    w = np.array([float(v) for v in ws])
    # exact antisymmetry / symmetry
    xi = 0.5 * (xi - xi[::-1])
    w = 0.5 * (w + w[::-1])
    if Q % 2 == 1:
        xi[Q // 2] = 0.0
    return xi, w


def laguerre2_explicit(l, x):
    """Generalised Laguerre polynomial of type 2 from its explicit sum (eq. lag_expl):
    L_l^(2)(x) = sum_{s=0}^{l} (-x)^s (l+2)! / (s! (s+2)! (l-s)!)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    for s in range(l + 1):
        out = out + (-x) ** s * factorial(l + 2) / (factorial(s) * factorial(s + 2) * factorial(l - s))
    return out


def _laguerre2_mp(l, x):
    out = mpmath.mpf(0)
    for s in range(l + 1):
        out += (-x) ** s * mpmath.factorial(l + 2) / (
            mpmath.factorial(s) * mpmath.factorial(s + 2) * mpmath.factorial(l - s))
    return out


@lru_cache(maxsize=None)
def gauss_laguerre2(QL):
    """Nodes (roots of L^(2)_{Q_L}) and weights of eq. wL for the weight e^{-x} x^2.

    Starting points from scipy.special.roots_genlaguerre (library routine);
    roots polished by Newton in 40 digits on the explicit polynomial; weights
    from the paper's formula (eq. wL), not from the library."""
    from scipy.special import roots_genlaguerre
    x0, _ = roots_genlaguerre(QL, 2)
    xs, ws = [], []
    with mpmath.workdps(_MP_DPS):
        for guess in x0:
            x = mpmath.mpf(float(guess))
            for _ in range(8):
                p = _laguerre2_mp(QL, x)
                # d/dx L_l^(a) = -L_{l-1}^(a+1); evaluate derivative numerically exact via mp diff
                dp = mpmath.diff(lambda t: _laguerre2_mp(QL, t), x)
                x = x - p / dp
            lq1 = _laguerre2_mp(QL + 1, x)
            w = x * (QL + 2) / ((QL + 1) * lq1 ** 2)
            xs.append(x)
            ws.append(w)
    return np.array([float(v) for v in xs]), np.array([float(v) for v in ws])


def legendre_table(mmax, xi):
    """P_m(xi_j) for m = 0..mmax (rows), plain recurrence in FP64."""
    xi = np.asarray(xi, dtype=np.float64)
    P = np.zeros((mmax + 1, xi.size))
    P[0] = 1.0
    if mmax >= 1:
        P[1] = xi
    for m in range(1, mmax):
        P[m + 1] = ((2 * m + 1) * xi * P[m] - m * P[m - 1]) / (m + 1)
    return P


def kernel_KL(QL):
    """Discrete radial kernel K^L_{k,k'} of eq. K_lag_disc (Q_L x Q_L)."""
    pb, wL = gauss_laguerre2(QL)
    K = np.zeros((QL, QL))
    for l in range(1, QL):
        Lk = laguerre2_explicit(l, pb)
        Lkm1p = laguerre2_explicit(l - 1, pb)
        Lkp = laguerre2_explicit(l, pb)
        K += (wL * Lk)[:, None] * ((l + 2) * Lkm1p - l * Lkp)[None, :] / ((l + 1) * (l + 2))
    return K


def kernel_KP(Q):
    """Discrete angular kernel K^P_{j,j'} of eq. K_leg_disc (Q_xi x Q_xi).

    First sum: m = 1..Q-3 with the P_{m+2}(xi_j') term; second sum: m = 1..Q-1
    with the P_m and P_{m-2} terms (P_{-1} := 0 never occurs since the m=1 term
    of P_{m-2} carries the factor (m-1) = 0)."""
    xi, w = gauss_legendre(Q)
    P = legendre_table(Q + 1, xi)
    K = np.zeros((Q, Q))
    for m in range(1, Q - 2):
        K += (w * P[m])[:, None] * P[m + 2][None, :] * (m * (m + 1) * (m + 2) / (2.0 * (2 * m + 3)))
    for m in range(1, Q):
        c = m * (m + 1) / 2.0
        term = (2 * m + 1) * P[m] / ((2 * m - 1) * (2 * m + 3))
        if m >= 2:
            term = term + (m - 1) / (2 * m - 1) * P[m - 2]
        K -= c * (w * P[m])[:, None] * term[None, :]
    return K


class VelocitySet:
    """R-SLB(N_Omega; Q_xi) with Q_L radial nodes (Sec. III E): tables in FP64.

    Velocity plane index v = k * Q_xi + j (radial index outer), as in the
    grouping kappa = (k-1) Q_xi + j of App. B."""

    def __init__(self, QL, Q, NOm, T0=1.0, n_gauss=160):
        if not (Q > NOm >= 0):
            raise ValueError("need Q_xi > N_Omega >= 0")
        self.QL, self.Q, self.NOm, self.T0 = QL, Q, NOm, float(T0)
        self.xi, self.wxi = gauss_legendre(Q)
        self.pb, self.wL = gauss_laguerre2(QL)
        self.V = QL * Q
        # Gauss rule used only to evaluate the a~ integrals (eq. aeq_aux)
        self.xg, self.wg = gauss_legendre(n_gauss)
        self.KL = kernel_KL(QL)
        self.KP = kernel_KP(Q)
