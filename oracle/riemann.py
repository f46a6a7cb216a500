"""Exact inviscid Riemann solution for the massless ideal gas (P = E/3) and the
free-streaming (ballistic) Sod solution.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Inviscid: Sec. IV B 1 -- rarefaction invariants (eq. R_inv, eqs. betastar,
Pstar, nstar), Rankine-Hugoniot (eq. junction), plateau velocity and shock
speed (eq. Sod:uplateau), plateau pressure (eq. Sod:PC), rarefaction tail
(eq. Sod:xiT), densities (eqs. Sod:nI, Sod:nII).

Ballistic: Sec. IV C 1 -- N^mu (eq. Sod:bal:Nmu) and T^{mu nu}
(eq. Sod:bal:Tmunu) for |z/t| < 1.
"""
from math import sqrt

import numpy as np
from scipy.optimize import brentq

CS = 1.0 / sqrt(3.0)


def _plateau_residual(PC, PL, PR):
    r = (PL / PC) ** (sqrt(3.0) / 2.0)
    return (r - 1.0) / (r + 1.0) - sqrt(3.0 * (PC - PR) ** 2 / ((PC + 3.0 * PR) * (3.0 * PC + PR)))


def riemann_star(nL, PL, nR, PR):
    """Plateau pressure, velocities, tail position and densities (left state at rest
    on z < 0, right state at rest on z > 0, P_L > P_R)."""
    PC = brentq(_plateau_residual, PR * (1 + 1e-15), PL * (1 - 1e-15), args=(PL, PR), xtol=1e-17, rtol=1e-15,
                maxiter=500)
    beta_shock = sqrt((PR + 3.0 * PC) / (3.0 * (PC + 3.0 * PR)))
    beta_C = sqrt(3.0 * (PC - PR) ** 2 / ((PC + 3.0 * PR) * (3.0 * PC + PR)))
    q = (PC / PL) ** (sqrt(3.0) / 2.0)
    zeta_T = (sqrt(3.0) - 1.0 - (sqrt(3.0) + 1.0) * q) / (sqrt(3.0) - 1.0 + (sqrt(3.0) + 1.0) * q)
    nI = nL * (PC / PL) ** 0.75
    nII = nR * sqrt(PC * (PR + 3.0 * PC) / (PR * (PC + 3.0 * PR)))
    return dict(PC=PC, beta_C=beta_C, beta_shock=beta_shock, zeta_T=zeta_T, nI=nI, nII=nII,
                zeta_H=-CS)


def riemann_profile(zeta, nL, PL, nR, PR):
    """(n, P, beta) at similarity coordinate zeta = z/t (full solution, Sec. IV B 1)."""
    st = riemann_star(nL, PL, nR, PR)
    zeta = np.asarray(zeta, dtype=np.float64)
    n = np.empty_like(zeta)
    P = np.empty_like(zeta)
    b = np.empty_like(zeta)
    for i, x in np.ndenumerate(zeta):
        if x < -CS:
            n[i], P[i], b[i] = nL, PL, 0.0
        elif x < st["zeta_T"]:
            r = (1 - CS) * (1 - x) / ((1 + CS) * (1 + x))
            b[i] = (CS + x) / (1 + CS * x)
            P[i] = PL * r ** (2.0 / sqrt(3.0))
            n[i] = nL * r ** (sqrt(3.0) / 2.0)
        elif x < st["beta_C"]:
            n[i], P[i], b[i] = st["nI"], st["PC"], st["beta_C"]
        elif x < st["beta_shock"]:
            n[i], P[i], b[i] = st["nII"], st["PC"], st["beta_C"]
        else:
            n[i], P[i], b[i] = nR, PR, 0.0
    return n, P, b


def ballistic_sod(zeta, nL, PL, nR, PR):
    """Continuum free-streaming moments (N0, Nz, T00, T0z, Tzz) at zeta = z/t,
    eqs. Sod:bal:Nmu and Sod:bal:Tmunu for |zeta| < 1 (unperturbed outside)."""
    zeta = np.clip(np.asarray(zeta, dtype=np.float64), -1.0, 1.0)
    N0 = 0.5 * (nL + nR) - 0.5 * (nL - nR) * zeta
    Nz = 0.25 * (nL - nR) * (1 - zeta ** 2)
    T00 = 1.5 * (PL + PR) - 1.5 * (PL - PR) * zeta
    T0z = 0.75 * (PL - PR) * (1 - zeta ** 2)
    Tzz = 0.5 * (PL + PR) - 0.5 * (PL - PR) * zeta ** 3
    return np.stack([N0, Nz, T00, T0z, Tzz], axis=-1)
