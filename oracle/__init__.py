"""Plain FP64 CPU oracle for the R-SLB hot path (Ambrus & Blaga, arXiv:1612.01287).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library in ``paper_1612_01287_amd/`` and never imports it.

Layout: ``rslo.c`` holds the solver arithmetic (plain C, FP64, no FMA
contraction); ``quadrature.py`` the velocity-set tables; the analytic and
semi-analytic references the paper compares against live in ``riemann.py`` and
``bjorken_ref.py``; the field diagnostics (window integrals, the Sod error
measure, the Bjorken L2 norm) in ``diagnostics.py``; the reference network of
the learned correction and the moment-preserving feedback into f in
``mlp.py``; the velocity sets with azimuthal nodes in ``vel3d.py``; the
implicit-explicit step in ``imex.py``.  This module wraps ``rslo.c`` with
ctypes.

Parity status per function (pins in tests/test_oracle_*.py):
  quadrature, K^L, K^P ........ pinned (exactness, Table I, calculus identities)
  a~_{l,m}, f^eq .............. pinned (App. A closed forms and series, MJ moments)
  Landau frame ................ pinned (round trip, 2x2 eigenproblem)
  WENO5 ....................... pinned (constants, limiting cases, 5th order)
  relaxation-time laws ........ pinned (printed tau_{A-W;0}, tau_L/tau_R of eqs. tau_LR,
                                tau_LR2; Bjorken ideal gas against eq. bjorken_tauAW_mu)
  Sod step .................... pinned (conservation, uniform state, reflection,
                                ballistic staircase, inviscid Riemann plateau,
                                3rd order in dt, 5th order in dz for free streaming)
  Bjorken step ................ pinned (tau n = 1, energy identity, free streaming,
                                ideal-fluid limit, 3rd-order RK convergence)
  diagnostics ................. pinned (window integral, eps and L2 on profiles with
                                closed-form values; the analytic q and Pi integrals
                                against a near-inviscid kinetic solve)
  reference network ........... pinned (finite-difference gradients, Adam on a
                                quadratic, feature definitions)
  feedback into f, projection . pinned (only T^{mu nu} or only N^mu moved, equilibria
                                projected onto equilibria, conserved moments kept)
  azimuthal velocity sets ..... pinned (angular rule exact below its degree, ideal-gas
                                moments, the aligned set along z, rotation, isotropy
                                at rest, the 3D frame of boosted and noisy states)
  IMEX step ................... pinned (stage equation and conserved moments, uniform
                                state, exact Riemann plateau at dt >> tau, 2nd order,
                                collisionless = Heun, binary32 storage rounding)
"""
import ctypes
import os
import subprocess

import numpy as np

from .quadrature import VelocitySet  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rslo.c")
_SO = os.path.join(_HERE, "librslo.so")

_dp = ctypes.POINTER(ctypes.c_double)


def build(force=True):
    """Compile rslo.c with gcc (no FMA contraction, -O2)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-fPIC", "-shared",
           "-o", _SO, _SRC, "-lm"]
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        subprocess.check_call(cmd)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_SO)
        L.o_weno5.restype = ctypes.c_double
        L.o_weno5.argtypes = [ctypes.c_double] * 5
        L.o_atilde.restype = None
        L.o_atilde.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp, _dp, _dp]
        L.o_feq.restype = None
        L.o_feq.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp, ctypes.c_double,
                            ctypes.c_int, _dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp]
        L.o_landau.restype = ctypes.c_int
        L.o_landau.argtypes = [_dp, _dp]
        L.o_sod_moments.restype = ctypes.c_int
        L.o_sod_moments.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_double, ctypes.c_int, _dp, _dp]
        L.o_sod_L.restype = ctypes.c_int
        L.o_sod_L.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.o_sod_run.restype = ctypes.c_int
        L.o_sod_run.argtypes = [ctypes.c_void_p, _dp, ctypes.c_double, ctypes.c_int]
        L.o_relax_time.restype = ctypes.c_double
        L.o_relax_time.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double]
        L.o_sod_init.restype = None
        L.o_sod_init.argtypes = [ctypes.c_void_p, _dp]
        L.o_bj_L.restype = ctypes.c_int
        L.o_bj_L.argtypes = [ctypes.c_void_p, _dp, ctypes.c_double, _dp, _dp]
        L.o_bj_run.restype = ctypes.c_int
        L.o_bj_run.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_double, ctypes.c_int, _dp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_dp)


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class _SodStruct(ctypes.Structure):
    _fields_ = [("QL", ctypes.c_int), ("Q", ctypes.c_int), ("NOm", ctypes.c_int),
                ("xi", _dp), ("wx", _dp), ("pb", _dp), ("wl", _dp),
                ("T0", ctypes.c_double), ("ng", ctypes.c_int), ("xg", _dp), ("wg", _dp),
                ("nz", ctypes.c_int), ("zlo", ctypes.c_double), ("zhi", ctypes.c_double),
                ("tau_mode", ctypes.c_int), ("tau_r", ctypes.c_double), ("tau_aw0", ctypes.c_double),
                ("lambda_ref", ctypes.c_double), ("bc", ctypes.c_int), ("store_f32", ctypes.c_int),
                ("feqL", _dp), ("feqR", _dp)]


class _BjStruct(ctypes.Structure):
    _fields_ = [("QL", ctypes.c_int), ("Q", ctypes.c_int), ("NOm", ctypes.c_int),
                ("xi", _dp), ("wx", _dp), ("pb", _dp), ("wl", _dp),
                ("T0", ctypes.c_double), ("ng", ctypes.c_int), ("xg", _dp), ("wg", _dp),
                ("KL", _dp), ("KP", _dp),
                ("gas", ctypes.c_int), ("tau_mode", ctypes.c_int), ("tau_r", ctypes.c_double),
                ("tau_aw0", ctypes.c_double), ("lambda_ref", ctypes.c_double), ("store_f32", ctypes.c_int)]


TAU_CONST, TAU_ETAS, TAU_INF = 0, 1, 2
BC_EQ, BC_OUTFLOW = 0, 1
GAS_IDEAL, GAS_PARTON = 0, 1

# hbar c in GeV fm, used to turn eta/s into tau_{A-W;0} (eqs. Sod:tau, bjorken_tauAW)
HBARC_GEV_FM = 0.1973269804


def tau_aw0(eta_s, T_ref_GeV, L_ref_fm):
    """tau_{A-W;0} = 5 hbar c (eta/s) / (k_B T_ref L_ref)   (eq. Sod:tau, eq. bjorken_tauAW)."""
    return 5.0 * HBARC_GEV_FM * eta_s / (T_ref_GeV * L_ref_fm)


# ---------------------------------------------------------------- wrappers

def weno5(a, b, c, d, e):
    return lib().o_weno5(float(a), float(b), float(c), float(d), float(e))


def atilde(vs, beta, theta):
    """a~_{l,m} (l = 0,1; m = 0..N_Omega) from the integral definition, shape (2, N_Omega+1)."""
    out = np.zeros(2 * (vs.NOm + 1))
    lib().o_atilde(vs.NOm, float(beta), float(theta), vs.xg.size, _p(vs.xg), _p(vs.wg), _p(out))
    return out.reshape(2, vs.NOm + 1)


def feq(vs, n, T, beta):
    """Discrete equilibrium f^eq_{jk} of the truncated expansion, shape (V,), v = k*Q + j."""
    out = np.zeros(vs.V)
    lib().o_feq(vs.QL, vs.Q, vs.NOm, _p(vs.xi), _p(vs.wxi), _p(vs.pb), _p(vs.wL), vs.T0,
                vs.xg.size, _p(vs.xg), _p(vs.wg), float(n), float(T), float(beta), _p(out))
    return out


def landau(M):
    """Landau frame of raw moments (N0, Nz, T00, T0z, Tzz) -> dict or None if unphysical."""
    M = _c(M)
    out = np.zeros(6)
    rc = lib().o_landau(_p(M), _p(out))
    if rc != 0:
        return None
    return dict(E=out[0], beta=out[1], gamma=out[2], n=out[3], P=out[4], T=out[5])


MOMENT_FIELDS = ("N0", "Nz", "T00", "T0z", "Tzz", "n", "E", "P", "T", "beta", "lambda", "q", "Pi")


def sod_moments(vs, f):
    """Per-cell raw and derived fields, shape (nz, 13) in MOMENT_FIELDS order."""
    f = _c(f)
    V, nz = f.shape
    assert V == vs.V
    out = np.zeros((nz, 13))
    lib().o_sod_moments(vs.QL, vs.Q, _p(vs.xi), _p(vs.pb), vs.T0, nz, _p(f), _p(out))
    return out


class Sod:
    """Sod shock tube in the oracle (Sec. IV).

    Parameters mirror the paper's problem statement: states (n, T) left/right
    at rest, domain [zlo, zhi] with nz cells, relaxation-time law, ghost-cell
    rule and whether f is stored in binary32 between RK stages."""

    def __init__(self, vs, nz, nL=1.0, TL=1.0, nR=0.125, TR=0.5, zlo=-0.5, zhi=0.5,
                 tau_mode=TAU_CONST, tau_r=1e-3, tau_aw0=0.0, lambda_ref=1.0,
                 bc=BC_EQ, store_f32=False):
        self.vs, self.nz = vs, nz
        self.feqL = feq(vs, nL, TL, 0.0)
        self.feqR = feq(vs, nR, TR, 0.0)
        self.dz = (zhi - zlo) / nz
        self.s = _SodStruct(vs.QL, vs.Q, vs.NOm, _p(vs.xi), _p(vs.wxi), _p(vs.pb), _p(vs.wL),
                            vs.T0, vs.xg.size, _p(vs.xg), _p(vs.wg), nz, zlo, zhi,
                            tau_mode, tau_r, tau_aw0, lambda_ref, bc, int(store_f32),
                            _p(self.feqL), _p(self.feqR))

    def init(self):
        f = np.zeros((self.vs.V, self.nz))
        lib().o_sod_init(ctypes.byref(self.s), _p(f))
        return f

    def relax_time(self, n, T):
        """tau_AW of a cell with Landau-frame density n and temperature T."""
        return lib().o_relax_time(ctypes.byref(self.s), float(n), float(T))

    def L(self, f):
        f = _c(f)
        out = np.zeros_like(f)
        rc = lib().o_sod_L(ctypes.byref(self.s), _p(f), _p(out))
        if rc != 0:
            raise FloatingPointError("oracle: unphysical cell state (rc=%d)" % rc)
        return out

    def run(self, f, dt, nsteps):
        f = _c(f).copy()
        if self.s.store_f32:
            f = f.astype(np.float32).astype(np.float64)
        rc = lib().o_sod_run(ctypes.byref(self.s), _p(f), float(dt), int(nsteps))
        if rc != 0:
            raise FloatingPointError("oracle: unphysical cell state (rc=%d)" % rc)
        return f

    def moments(self, f):
        return sod_moments(self.vs, f)


class Bjorken:
    """One Bjorken-flow instance in Milne coordinates (Sec. V)."""

    def __init__(self, vs, gas=GAS_IDEAL, tau_mode=TAU_ETAS, tau_r=1.0, tau_aw0=1.0,
                 lambda_ref=1.0, store_f32=False):
        self.vs = vs
        self.KL = _c(vs.KL)
        self.KP = _c(vs.KP)
        self.s = _BjStruct(vs.QL, vs.Q, vs.NOm, _p(vs.xi), _p(vs.wxi), _p(vs.pb), _p(vs.wL),
                           vs.T0, vs.xg.size, _p(vs.xg), _p(vs.wg), _p(self.KL), _p(self.KP),
                           gas, tau_mode, tau_r, tau_aw0, lambda_ref, int(store_f32))

    def init(self):
        """f(tau = 1) = e^{-p}/(8 pi) at n = T = 1 (eq. bjorken_f0)."""
        return feq(self.vs, 1.0, 1.0, 0.0)

    def L(self, f, tau):
        f = _c(f)
        out = np.zeros_like(f)
        tmp = np.zeros_like(f)
        rc = lib().o_bj_L(ctypes.byref(self.s), _p(f), float(tau), _p(out), _p(tmp))
        if rc != 0:
            raise FloatingPointError("oracle: unphysical Bjorken state")
        return out

    def run(self, f, tau0, dtau, nsteps, history=False):
        f = _c(f).copy()
        if self.s.store_f32:
            f = f.astype(np.float32).astype(np.float64)
        tau = ctypes.c_double(tau0)
        hist = np.zeros((nsteps + 1, 3)) if history else None
        rc = lib().o_bj_run(ctypes.byref(self.s), _p(f), ctypes.byref(tau), float(dtau), int(nsteps),
                            _p(hist) if history else None)
        if rc != 0:
            raise FloatingPointError("oracle: unphysical Bjorken state")
        if history:
            return f, tau.value, hist
        return f, tau.value
