"""Oracle diagnostics of the macroscopic fields (plain numpy, test infrastructure).

TEST INFRASTRUCTURE ONLY: used by tests/ against the library's device
diagnostics, never by the product path.

* window_integral: dz times the sum of per-cell fields over a window of
  cells (the integrated q and Pi of Sec. IV B 3);
* sod_eps: the error measure of the Sod convergence test (Sec. IV E,
  eq. eps_def), read as max_z |d - d_ref| / (max_z d - min_z d) for
  d in {n, T, gamma};
* bjorken_l2: the L2 norm of the Bjorken convergence test (Sec. V E,
  eq. bjork_L2) for A in {n, T, P, Pi}, trapezoid rule over uniform samples;
* integrated_noneq: the analytic integrals of q and Pi over the contact and
  the shock in the near-inviscid limit (eqs. intq, intpi) with the
  Chapman-Enskog transport coefficients (eq. tcoeff_ce).

Rows are laid out as the oracle's sod_moments: (N0, Nz, T00, T0z, Tzz, n, E,
P, T, beta, lambda_bar, q, Pi).
"""
import numpy as np

from . import riemann

COL = dict(n=5, P=7, T=8, beta=9, lam=10, q=11, Pi=12)


def window_integral(M, dz, lo, hi):
    """dz * sum of rows lo..hi-1 of M, column by column."""
    M = np.asarray(M, dtype=np.float64)
    out = np.zeros(M.shape[1])
    for r in range(lo, hi):
        out += M[r]
    return dz * out


def _fields(M):
    M = np.asarray(M, dtype=np.float64)
    return {"n": M[:, COL["n"]], "T": M[:, COL["T"]], "gamma": 1.0 / np.sqrt(1.0 - M[:, COL["beta"]] ** 2),
            "P": M[:, COL["P"]], "Pi": M[:, COL["Pi"]]}


def sod_eps(M, Mref):
    """(eps_n, eps_T, eps_gamma, eps) of eq. eps_def."""
    d, r = _fields(M), _fields(Mref)
    out = []
    for k in ("n", "T", "gamma"):
        out.append(np.max(np.abs(d[k] - r[k])) / (np.max(d[k]) - np.min(d[k])))
    return np.array(out + [max(out)])


def bjorken_l2(H, Href, dtau):
    """(L2(n), L2(T), L2(P), L2(Pi), max) of eq. bjork_L2 from samples at
    tau = 1 + i dtau (trapezoid rule; tau_f - 1 = (N - 1) dtau)."""
    d, r = _fields(H), _fields(Href)
    n = len(H)
    w = np.ones(n)
    w[0] = w[-1] = 0.5
    out = []
    for k in ("n", "T", "P", "Pi"):
        out.append(np.sqrt(np.sum(w * (d[k] - r[k]) ** 2) * dtau / ((n - 1) * dtau)))
    return np.array(out + [max(out)])


def integrated_noneq(nL, PL, nR, PR, tau_of):
    """Integrals of q and Pi over the contact and the shock, near-inviscid
    limit (eqs. intq_c, intq_s, intpi_c, intpi_s), with eta = 4/5 P tau and
    lambda_heat = 4/3 P tau / T (eq. tcoeff_ce); tau_of(n, T) is the
    relaxation time of a state.  Returns dict(q_contact, q_shock, Pi_contact,
    Pi_shock)."""
    st = riemann.riemann_star(nL, PL, nR, PR)
    PC, bC, bS = st["PC"], st["beta_C"], st["beta_shock"]
    nI, nII = st["nI"], st["nII"]
    TI, TII, TR = PC / nI, PC / nII, PR / nR
    gC = 1.0 / np.sqrt(1.0 - bC * bC)
    lam = lambda n, T: n / T ** 3
    lheat = lambda n, P, T: 4.0 / 3.0 * P * tau_of(n, T) / T
    eta = lambda n, P, T: 4.0 / 5.0 * P * tau_of(n, T)
    lI, lII, lR = lheat(nI, PC, TI), lheat(nII, PC, TII), lheat(nR, PR, TR)
    q_c = (lI * TI + lII * TII) / 8.0 * np.log(lam(nII, TII) / lam(nI, TI))
    q_s = (lR * TR + lII * TII * gC * gC * (1.0 - bC * bS)) / 8.0 * np.log(lam(nR, TR) / lam(nII, TII))
    pi_s = 2.0 * bC * gC / 3.0 * (eta(nR, PR, TR) + eta(nII, PC, TII) * (1.0 - bC * bS))
    return dict(q_contact=q_c, q_shock=q_s, Pi_contact=0.0, Pi_shock=pi_s)
