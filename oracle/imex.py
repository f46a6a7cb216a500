"""Oracle of an implicit-explicit (IMEX) time step for the Sod operator, so that
the step is not bound by the relaxation time (the option Sec. I names in place
of dt < tau_AW; Sec. III F).

TEST INFRASTRUCTURE ONLY: used by tests/ against the library's rsl_step_imex,
never by the product path.  Plain FP64 numpy on top of the oracle's Sod pieces;
shares no code with the HIP library.

* Splitting of eq. L_Sod: A(f), the WENO5 advection with the instance's ghost
  rule (the oracle's L of the same tube without collisions), explicit;
  Q(f) = -gamma (1 - beta xi_j) / tau_AW (f - f^eq), the Anderson-Witting
  term with the Landau frame, tau and f^eq of f itself, implicit.
* IMEX-SSP2(2,2,2) (Pareschi & Russo): the SSP Heun method for A and an
  L-stable two-stage diagonally implicit rule for Q, with g = 1 - 1/sqrt(2):
      F1 = f + g dt Q(F1)
      F2 = f + dt A(F1) + (1 - 2 g) dt Q(F1) + g dt Q(F2)
      f' = f + dt/2 (A(F1) + A(F2)) + dt/2 (Q(F1) + Q(F2)).
* An implicit stage G = F + h Q(G) per cell: Q has zero N^0, T^00, T^0z
  (u_mu (N^mu - N^mu_eq) = 0 and u_mu (T^{mu nu} - T^{mu nu}_eq) = 0 in the
  Landau frame of G), so G keeps those of F and the unknowns are N^z(G),
  T^zz(G); for a guess of them G = (F + h c f^eq) / (1 + h c) with c, f^eq
  from the frame of the five moments, and the guess must reproduce itself.
  Solved with scipy.optimize.fsolve (MINPACK's hybrid method) to the last
  bits; Q(F1) = (F1 - f) / (g dt), Q(F2) = (F2 - F2*) / (g dt).

Pins: tests/test_oracle_imex.py.
"""
import warnings

import numpy as np
from scipy.optimize import fsolve

from . import TAU_INF, Sod, feq, landau

GAMMA = 1.0 - 1.0 / np.sqrt(2.0)


def _rows(vs):
    xi = np.tile(vs.xi, vs.QL)
    p = np.repeat(vs.pb * vs.T0, vs.Q)
    return xi, p, np.stack([np.ones_like(xi), xi, p, p * xi, p * xi * xi])


def _rate(S, L, xi):
    """gamma (1 - beta xi_j) / tau_AW of the frame L; zero for the
    collisionless law (tau_AW -> infinity, where the Anderson-Witting term of
    eq. AW vanishes)."""
    if S.s.tau_mode == TAU_INF:
        return np.zeros_like(xi)
    return L["gamma"] * (1.0 - L["beta"] * xi) / S.relax_time(L["n"], L["T"])


def relaxed(S, Fc, M, X, h):
    """G for one cell: F column Fc, its moments M (5,), guess X = (N^z, T^zz)."""
    vs = S.vs
    xi, _, _ = _rows(vs)
    L = landau(np.array([M[0], X[0], M[2], M[3], X[1]]))
    if L is None:
        return None
    c = _rate(S, L, xi)
    fe = feq(vs, L["n"], L["T"], L["beta"])
    return (Fc + h * c * fe) / (1.0 + h * c)


def implicit_stage(S, F, h):
    """G with G = F + h Q(G), cell by cell (F [V, nz])."""
    vs = S.vs
    xi, p, R = _rows(vs)
    F = np.asarray(F, dtype=np.float64)
    M = R @ F
    G = np.empty_like(F)
    for s in range(F.shape[1]):
        def res(X, s=s):
            g = relaxed(S, F[:, s], M[:, s], X, h)
            if g is None:
                return [1e300, 1e300]
            return [(xi @ g - X[0]) / M[0, s], (p * xi * xi @ g - X[1]) / M[2, s]]
        with warnings.catch_warnings():        # MINPACK reports when it is at the rounding floor
            warnings.simplefilter("ignore", RuntimeWarning)
            X = fsolve(res, [M[1, s], M[4, s]], xtol=1e-14)
        r = res(X)
        if not (abs(r[0]) < 1e-10 and abs(r[1]) < 1e-10):     # the stage's defining equation must hold
            raise FloatingPointError("oracle: implicit stage of cell %d did not converge (%r)" % (s, r))
        G[:, s] = relaxed(S, F[:, s], M[:, s], X, h)
    return G


def collision(S, G):
    """Q(G) with the frame of G itself (for checking the implicit stage)."""
    vs = S.vs
    xi, _, R = _rows(vs)
    M = R @ G
    out = np.empty_like(G)
    for s in range(G.shape[1]):
        L = landau(M[:, s])
        out[:, s] = -_rate(S, L, xi) * (G[:, s] - feq(vs, L["n"], L["T"], L["beta"]))
    return out


class ImexSod:
    """The oracle's Sod tube (same arguments as oracle.Sod) stepped with
    IMEX-SSP2(2,2,2).  store_f32: the state and the stored stages F1, F2*, F2
    are rounded to binary32 where they are stored; everything else, the
    advection of the rounded stages included, stays in binary64, and the
    final combination uses F2* before its rounding."""

    def __init__(self, vs, nz, store_f32=False, **kw):
        self.S = Sod(vs, nz, **kw)
        adv = dict(kw)
        adv["tau_mode"] = TAU_INF                 # collisionless: L is the advection alone
        self.A = Sod(vs, nz, **adv)
        self.vs, self.nz = vs, nz
        self.store = (lambda x: x.astype(np.float32).astype(np.float64)) if store_f32 else (lambda x: x)

    def init(self):
        return self.store(self.S.init())

    def step(self, f, dt):
        h = GAMMA * dt
        F1 = self.store(implicit_stage(self.S, f, h))
        Q1 = (F1 - f) / h
        A1 = self.A.L(F1)
        Fs2 = f + dt * A1 + (1.0 - 2.0 * GAMMA) * dt * Q1
        F2 = self.store(implicit_stage(self.S, self.store(Fs2), h))
        Q2 = (F2 - Fs2) / h
        A2 = self.A.L(F2)
        return self.store(f + 0.5 * dt * (A1 + A2) + 0.5 * dt * (Q1 + Q2))

    def run(self, f, dt, nsteps):
        for _ in range(nsteps):
            f = self.step(f, dt)
        return f

    def moments(self, f):
        return self.S.moments(f)
