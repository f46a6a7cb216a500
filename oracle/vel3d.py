"""Oracle for velocity sets with azimuthal nodes, for flows not aligned with z.

TEST INFRASTRUCTURE ONLY: used by tests/ (and the CPU-baseline leg of
bench.py) against the library's rsl_quad3 calls, never by the product path.
Plain FP64 numpy written from the paper's definitions; shares no code with the
HIP library.

* Nodes (Sec. III E with the azimuthal rule of Sec. III D): the Q_L
  generalised Gauss-Laguerre radial nodes p_k = T0 pbar_k, the Q_xi
  Gauss-Legendre nodes xi_j = cos(theta_j), and Q_phi equally spaced azimuths
  phi_l = 2 pi l / Q_phi with equal weights 2 pi / Q_phi.  The equal-weight
  rule integrates trigonometric polynomials of degree below Q_phi exactly;
  Q_phi = 1 is the single point phi = 0 of eq. pjk.  Velocity index
  v = (k Q_phi + l) Q_xi + j, which is the index of the aligned set when
  Q_phi = 1.  Unit direction Omega_v = (sin theta_j cos phi_l,
  sin theta_j sin phi_l, xi_j).
* Equilibrium (Sec. III D, eqs. aeq_def, feq_trunc) for a fluid four-velocity
  u^mu = (u^0, u_vec) in any direction: the truncated expansion in
  L^(2)_l(pbar) and P_m(cos gamma_u) with cos gamma_u = Omega . u_vec / |u_vec|,
  evaluated directly at each node; the coefficients a_{l,m}(|u|, theta) are
  those of the aligned flow (eq. aeq_aux), since they depend on |u| only.
  The addition theorem (eq. leg_product) writes P_m(cos gamma_u) as a sum of
  P_m^q(xi) cos q(phi - phi_u), i.e. a trigonometric polynomial of degree m in
  phi: the azimuthal rule with Q_phi >= N_Omega + 3 points therefore
  integrates N^mu and T^{mu nu} of the truncated f^eq exactly.  Mapping to the
  discrete populations as eq. fjk with the azimuthal weight 2 pi / Q_phi:
      f_v = (2 pi / Q_phi) T0^3 e^{pbar_k} w_j w_k f^eq(p_k, Omega_v).
* Moments: N^mu = sum_v f_v Omega_v^mu, T^{mu nu} = sum_v f_v p_k Omega_v^mu
  Omega_v^nu (Omega^0 = 1), the discrete form of eq. macro_jk.
* Landau frame (Sec. II E): T^mu_nu u^nu = E u^mu with the metric
  (+, -, -, -), solved with numpy.linalg.eig (library routine) and the
  timelike eigenvector kept; n = u_mu N^mu, P = E / 3, T = P / n.

Parity pins: tests/test_oracle_vel3d.py.
"""
import numpy as np

from . import atilde
from .quadrature import VelocitySet, legendre_table

METRIC = np.diag([1.0, -1.0, -1.0, -1.0])


class VelocitySet3:
    """R-SLB(N_Omega; Q_xi) x Q_phi azimuths, Q_L radial nodes; FP64 tables in v order."""

    def __init__(self, QL, Q, Qphi, NOm, T0=1.0):
        if Qphi < 1:
            raise ValueError("need Q_phi >= 1")
        self.base = VelocitySet(QL, Q, NOm, T0)
        self.QL, self.Q, self.Qphi, self.NOm, self.T0 = QL, Q, Qphi, NOm, float(T0)
        self.V = QL * Qphi * Q
        self.phi = 2.0 * np.pi * np.arange(Qphi) / Qphi
        k, l, j = np.meshgrid(np.arange(QL), np.arange(Qphi), np.arange(Q), indexing="ij")
        self.k, self.l, self.j = k.ravel(), l.ravel(), j.ravel()
        xi = self.base.xi[self.j]
        s = np.sqrt(1.0 - xi * xi)
        self.Om = np.stack([s * np.cos(self.phi[self.l]), s * np.sin(self.phi[self.l]), xi], axis=1)
        self.pbar = self.base.pb[self.k]
        self.p = self.T0 * self.pbar
        self.w = (2.0 * np.pi / Qphi) * self.base.wxi[self.j] * self.base.wL[self.k]


def feq3(vs3, n, T, u_vec):
    """Discrete equilibrium f_v, shape (V,), for density n, temperature T and
    spatial four-velocity components u_vec = gamma v."""
    u_vec = np.asarray(u_vec, dtype=np.float64)
    u = float(np.sqrt(u_vec @ u_vec))
    gam = np.sqrt(1.0 + u * u)
    beta = u / gam
    at = atilde(vs3.base, beta, T / vs3.T0)                       # (2, N_Omega + 1)
    lidx = np.arange(2)[:, None]
    a = n * (lidx + 1.0) * (lidx + 2.0) * gam * at / (4.0 * np.pi)
    uhat = u_vec / u if u > 0.0 else np.array([0.0, 0.0, 1.0])
    c = vs3.Om @ uhat
    P = legendre_table(vs3.NOm, c)                                 # (N_Omega + 1, V)
    m = np.arange(vs3.NOm + 1)[:, None]
    S = ((2.0 * m + 1.0) / 2.0 * P)                                # (N_Omega + 1, V)
    x = vs3.pbar
    L = np.stack([np.ones_like(x), 3.0 - x])                       # L^(2)_0, L^(2)_1
    fc = np.zeros(vs3.V)
    for ell in range(2):
        fc += L[ell] / ((ell + 1.0) * (ell + 2.0)) * (a[ell] @ S)
    T03 = vs3.T0 ** 3
    fc *= np.exp(-x) / T03
    return vs3.w * T03 * np.exp(x) * fc


def moments3(vs3, f):
    """N^mu (4, ncell) and T^{mu nu} (4, 4, ncell) of f (V, ncell)."""
    f = np.asarray(f, dtype=np.float64)
    if f.ndim == 1:
        f = f[:, None]
    Om4 = np.concatenate([np.ones((vs3.V, 1)), vs3.Om], axis=1)   # (V, 4)
    N = Om4.T @ f
    T = np.einsum("vm,vn,vc->mnc", Om4, Om4 * vs3.p[:, None], f)
    return N, T


def landau3(N, T):
    """Landau frame of one cell: dict(E, n, P, T, u (4,)) or None when no
    timelike eigenvector with positive energy exists."""
    A = T @ METRIC                                                 # T^mu_nu
    ev, vec = np.linalg.eig(A)
    best = None
    for i in range(4):
        if abs(ev[i].imag) > 1e-12 * max(1.0, abs(ev[i].real)):
            continue
        u = vec[:, i].real
        norm2 = u[0] ** 2 - u[1:] @ u[1:]
        if norm2 <= 0.0:
            continue
        u = u / np.sqrt(norm2)
        if u[0] < 0.0:
            u = -u
        best = (ev[i].real, u)
    if best is None or best[0] <= 0.0:
        return None
    E, u = best
    n = u[0] * N[0] - u[1:] @ N[1:]
    if n <= 0.0:
        return None
    P = E / 3.0
    return dict(E=E, n=n, P=P, T=P / n, u=u)


def equilibrium_moments(n, T, u_vec):
    """Closed forms for a massless ideal gas: N^mu = n u^mu,
    T^{mu nu} = (E + P) u^mu u^nu - P g^{mu nu}, E = 3 P, P = n T."""
    u_vec = np.asarray(u_vec, dtype=np.float64)
    u = np.concatenate([[np.sqrt(1.0 + u_vec @ u_vec)], u_vec])
    P = n * T
    return n * u, 4.0 * P * np.outer(u, u) - P * METRIC
