"""Analytic and semi-analytic Bjorken-flow references (Sec. V).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* ideal fluid: n = 1/tau, P = tau^{-4/3}                 (eqs. bjorken_n, bjorken_inv)
* free streaming: P(tau), P_L(tau)                        (eq. bjorken_bal)
* first-order hydro, parton gas                           (eq. bjorken_mu0_hydro1)
* second-order hydro ODEs, parton and ideal gas           (eqs. bjorken_mu0_hydro2, milne_hydro2)
* Florkowski iterative solution for the parton gas        (eqs. flork_sol, flork_sol_aux)
"""
import numpy as np
from scipy.integrate import solve_ivp


def ideal(tau):
    tau = np.asarray(tau, dtype=np.float64)
    return 1.0 / tau, tau ** (-4.0 / 3.0)


def free_streaming(tau):
    """(P, P_L) of eq. bjorken_bal; the tau -> 1 limit is P = P_L = 1."""
    tau = np.asarray(tau, dtype=np.float64)
    s = np.sqrt(np.maximum(tau ** 2 - 1.0, 0.0))
    with np.errstate(invalid="ignore", divide="ignore"):
        A = np.where(s > 0, np.arctan(s) / np.where(s > 0, s, 1.0), 1.0)
        P = 0.5 * (A + 1.0 / tau ** 2)
        PL = np.where(s > 1e-4, 1.5 / np.where(s > 0, s * s, 1.0) * (A - 1.0 / tau ** 2), 1.0)
    return P, PL


def first_order_parton(tau, taw0):
    """P and Pi of eq. bjorken_mu0_hydro1."""
    tau = np.asarray(tau, dtype=np.float64)
    br = 1.0 + 2.0 * taw0 / 15.0 * (1.0 - tau ** (-2.0 / 3.0))
    return tau ** (-4.0 / 3.0) * br ** 4, -16.0 * taw0 / (15.0 * tau ** 2) * br ** 3


def second_order(tau_eval, taw0, gas="parton"):
    """Numerical solution of the second-order hydro system: eq. bjorken_mu0_hydro2
    (parton) or eq. milne_hydro2 (ideal gas), from P = 1, Pi = 0 at tau = 1."""
    def rhs(t, y):
        P, Pi = y
        if gas == "parton":
            inv_taw = P ** 0.25 / taw0
        else:
            inv_taw = t * P / (taw0 * (1.0 + np.log(t * P ** 0.75)))
        return [-4.0 * P / (3.0 * t) - Pi / (3.0 * t),
                -inv_taw * Pi - 38.0 / (21.0 * t) * Pi - 16.0 / (15.0 * t) * P]
    sol = solve_ivp(rhs, (1.0, float(np.max(tau_eval))), [1.0, 0.0], t_eval=tau_eval,
                    rtol=1e-11, atol=1e-13, method="LSODA")
    return sol.y[0], sol.y[1]


def _H(y):
    y = np.asarray(y, dtype=np.float64)
    out = np.empty_like(y)
    small = y >= 1.0 - 1e-12
    yy = np.where(small, 0.5, y)
    out = yy ** 2 + yy * np.arccos(yy) / np.sqrt(1.0 - yy ** 2)
    return np.where(small, 2.0, out)


def _HL(y):
    """H_L(y) = y^2 d/dy[H(y)/y] (eq. flork_sol_aux), written in closed form."""
    y = np.asarray(y, dtype=np.float64)
    near = y > 1.0 - 1e-4
    yy = np.where(near, 0.5, y)
    g = yy * np.arccos(yy) / np.sqrt(1.0 - yy ** 2)
    out = yy ** 2 * (1.0 + (g - 1.0) / (1.0 - yy ** 2))
    # series about y = 1: H_L = y^2 (2/3 + O(1 - y)); use it only in the last 1e-4
    d = 1.0 - y
    series = y ** 2 * (2.0 / 3.0 - 4.0 / 15.0 * d)
    return np.where(near, series, out)


def florkowski(taw0, tau_f=40.0, dtau=0.04, tol=1e-7, max_iter=2000):
    """Iterative semi-analytic solution of the parton-gas Bjorken flow, eq. flork_sol:
    returns tau grid, T, n, P_L.  Trapezoidal rule on an equidistant grid,
    started from T_(0) = tau^{-1/3}, stopped when the L2 change of T < tol."""
    nt = int(round((tau_f - 1.0) / dtau))
    tau = 1.0 + dtau * np.arange(nt + 1)
    T = tau ** (-1.0 / 3.0)
    H1 = 2.0
    for _ in range(max_iter):
        # cumulative integral of T for the damping function D(tau2, tau1)
        cum = np.concatenate([[0.0], np.cumsum(0.5 * dtau * (T[1:] + T[:-1]))])
        taw = taw0 / T
        T4 = np.empty_like(T)
        for i in range(nt + 1):
            D = np.exp(-(cum[i] - cum[: i + 1]) / taw0)
            integrand = T[: i + 1] ** 4 / (2.0 * taw[: i + 1]) * D * _H(tau[: i + 1] / tau[i])
            I = np.trapezoid(integrand, dx=dtau) if i > 0 else 0.0
            T4[i] = D[0] * _H(1.0 / tau[i]) / H1 + I
        Tn = T4 ** 0.25
        l2 = np.sqrt(np.trapezoid((Tn - T) ** 2, dx=dtau) / (tau_f - 1.0))
        T = Tn
        if l2 <= tol:
            break
    cum = np.concatenate([[0.0], np.cumsum(0.5 * dtau * (T[1:] + T[:-1]))])
    taw = taw0 / T
    n = np.empty_like(T)
    PL = np.empty_like(T)
    for i in range(nt + 1):
        D = np.exp(-(cum[i] - cum[: i + 1]) / taw0)
        In = np.trapezoid(T[: i + 1] ** 3 * tau[: i + 1] / taw[: i + 1] * D, dx=dtau) if i > 0 else 0.0
        n[i] = (D[0] + In) / tau[i]
        IL = np.trapezoid(T[: i + 1] ** 4 / (2.0 * taw[: i + 1]) * D * _HL(tau[: i + 1] / tau[i]),
                          dx=dtau) if i > 0 else 0.0
        PL[i] = 3.0 * (D[0] * _HL(1.0 / tau[i]) / H1 + IL)
    return tau, T, n, PL
