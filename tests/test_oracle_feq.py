"""Pins of the oracle's equilibrium, Landau frame and collision term.

* a~_{l,m}: the oracle integrates the definition (eq. aeq_aux); here it is
  checked against the closed forms of App. A where they are well conditioned
  (|u| >= 0.5) and against the App. A Maclaurin series at small u, with the two
  misprints of App. A read as listed in the design doc (a stray bracket in a~_{1,3},
  a doubled minus sign in its series).
* f^eq moments reproduce the Maxwell-Juttner N^mu = n u^mu and
  T^{mu nu} = (E+P) u^mu u^nu + P eta^{mu nu} exactly for Q_xi > N_Omega >= 2
  (quadrature exactness, Secs. III B-C).
* Landau frame: round trip and the 2x2 eigenproblem (eqs. EL_def, E_landau, u_landau).
* Collision invariants (eq. collinv): sum_jk C_jk {1, p, p xi} = 0.
"""
import numpy as np
import pytest

import oracle
from oracle import quadrature as oq


def app_a_closed(u, th):
    """a~_{l,m} for m = 0..6 from the closed forms printed in App. A."""
    u0 = np.sqrt(1 + u * u)
    A = np.arcsinh(u)
    a0 = [1.0,
          u / u0,
          3 / (2 * u ** 3 * u0) * A + 1 - 3 / (2 * u ** 2),
          15 / (2 * u ** 4) * A - (15 + 5 * u ** 2 - 2 * u ** 4) / (2 * u ** 3 * u0),
          15 / (4 * u ** 5 * u0) * (7 + 6 * u ** 2) * A - (105 + 20 * u ** 2 - 4 * u ** 4) / (4 * u ** 4),
          105 / (4 * u ** 6) * (3 + 2 * u ** 2) * A - (315 + 315 * u ** 2 + 28 * u ** 4 - 4 * u ** 6) / (4 * u ** 5 * u0),
          105 / (16 * u ** 7 * u0) * (33 + 48 * u ** 2 + 16 * u ** 4) * A
          - (3465 + 2730 * u ** 2 + 168 * u ** 4 - 16 * u ** 6) / (16 * u ** 6)]
    a1 = [a0[0] - th / (3 * u0) * (3 + 4 * u ** 2),
          a0[1] - 4 * u * th / 3,
          a0[2] - 4 * th * u ** 2 / (3 * u0),
          a0[3] + 5 * th / (2 * u ** 4 * u0) * A - th / (6 * u ** 3) * (15 - 10 * u ** 2 + 8 * u ** 4),
          a0[4] + 35 * th / (2 * u ** 5) * A - th / (6 * u ** 4 * u0) * (105 + 35 * u ** 2 - 14 * u ** 4 + 8 * u ** 6),
          a0[5] + 35 * th / (4 * u ** 6 * u0) * (9 + 8 * u ** 2) * A
          - th / (12 * u ** 5) * (945 + 210 * u ** 2 - 56 * u ** 4 + 16 * u ** 6),
          a0[6] + 105 * th / (4 * u ** 7) * (11 + 8 * u ** 2) * A
          - th / (12 * u ** 6 * u0) * (3465 + 3675 * u ** 2 + 378 * u ** 4 - 72 * u ** 6 + 16 * u ** 8)]
    return np.array([a0, a1])


def app_a_series(u, th):
    """Maclaurin series of App. A (to u^11) for m = 2..6; m = 0, 1 exact forms."""
    u0 = np.sqrt(1 + u * u)
    a0 = [1.0, u / u0,
          4 * u ** 2 / 5 - 24 * u ** 4 / 35 + 64 * u ** 6 / 105 - 128 * u ** 8 / 231 + 512 * u ** 10 / 1001,
          4 * u ** 3 / 7 - 2 * u ** 5 / 3 + 15 * u ** 7 / 22 - 35 * u ** 9 / 52 + 21 * u ** 11 / 32,
          8 * u ** 4 / 21 - 128 * u ** 6 / 231 + 640 * u ** 8 / 1001 - 2048 * u ** 10 / 3003,
          8 * u ** 5 / 33 - 60 * u ** 7 / 143 + 7 * u ** 9 / 13 - 21 * u ** 11 / 34,
          64 * u ** 6 / 429 - 128 * u ** 8 / 429 + 1024 * u ** 10 / 2431]
    a1 = [1.0 - th / (3 * u0) * (3 + 4 * u ** 2), u / u0 - 4 * u * th / 3,
          a0[2] - 4 * th / 3 * u ** 2 + 2 * th / 3 * u ** 4 - th / 2 * u ** 6 + 5 * th / 12 * u ** 8 - 35 * th / 96 * u ** 10,
          a0[3] - 8 * th / 7 * u ** 3 + 64 * th / 63 * u ** 5 - 640 * th / 693 * u ** 7 + 2560 * th / 3003 * u ** 9
          - 1024 * th / 1287 * u ** 11,
          a0[4] - 8 * th / 9 * u ** 4 + 12 * th / 11 * u ** 6 - 15 * th / 13 * u ** 8 + 7 * th / 6 * u ** 10,
          a0[5] - 64 * th / 99 * u ** 5 + 1280 * th / 1287 * u ** 7 - 512 * th / 429 * u ** 9 + 28672 * th / 21879 * u ** 11,
          a0[6] - 64 * th / 143 * u ** 6 + 32 * th / 39 * u ** 8 - 56 * th / 51 * u ** 10]
    return np.array([a0, a1])


VS6 = oracle.VelocitySet(2, 8, 6)


@pytest.mark.parametrize("u", [0.5, 0.8, 1.0, 1.7, 3.0, -1.2])
@pytest.mark.parametrize("th", [0.3, 1.0, 1.6])
def test_atilde_closed_forms(u, th):
    beta = u / np.sqrt(1 + u * u)
    got = oracle.atilde(VS6, beta, th)
    ref = app_a_closed(abs(u), th)
    if u < 0:
        ref = ref * np.array([(-1) ** m for m in range(7)])[None, :]
    # closed forms lose ~ eps * (u^-2m) digits by cancellation; tolerance scaled accordingly
    tol = 1e-14 * np.array([max(1.0, abs(u) ** (-2 * m)) for m in range(7)]) * 200
    assert np.all(np.abs(got - ref) <= tol[None, :]), (got - ref)


@pytest.mark.parametrize("u", [0.003, 0.01, 0.03, -0.02])
@pytest.mark.parametrize("th", [0.5, 1.0, 1.3])
def test_atilde_series(u, th):
    beta = u / np.sqrt(1 + u * u)
    got = oracle.atilde(VS6, beta, th)
    ref = app_a_series(abs(u), th)
    if u < 0:
        ref = ref * np.array([(-1) ** m for m in range(7)])[None, :]
    # the quadrature of the definition carries ~eps*sqrt(ng) absolute rounding
    assert np.max(np.abs(got - ref)) < 1e-14 + 2 * abs(u) ** 12


def test_atilde_misprint_readings():
    """Reading of the doubled minus in the a~_{1,3} series: the alternating sign
    (-640 theta/693 u^7) matches the integral; '+' does not."""
    u, th = 0.04, 1.0
    beta = u / np.sqrt(1 + u * u)
    got = oracle.atilde(VS6, beta, th)[1, 3]
    s = app_a_series(u, th)[1, 3]
    flipped = s + 2 * 640 * th / 693 * u ** 7
    assert abs(got - s) < 1e-14
    assert abs(got - flipped) > 1e-10


def test_atilde_rest_frame():
    at = oracle.atilde(VS6, 0.0, 0.7)
    assert at[0, 0] == pytest.approx(1.0, abs=1e-15)
    assert at[1, 0] == pytest.approx(0.3, abs=1e-15)       # 1 - theta
    assert np.max(np.abs(at[:, 1:])) < 1e-16


def _mj_moments(n, T, beta):
    g = 1.0 / np.sqrt(1 - beta ** 2)
    u = beta * g
    P = n * T
    return np.array([n * g, n * u, P * (3 + 4 * u * u), 4 * P * g * u, P * (1 + 4 * u * u)])


@pytest.mark.parametrize("QL,Q,NOm", [(2, 3, 2), (2, 8, 3), (3, 8, 3), (3, 16, 4), (3, 40, 4), (2, 100, 6)])
@pytest.mark.parametrize("state", [(1.0, 1.0, 0.0), (0.4, 0.8, 0.0), (0.7, 0.9, 0.3), (1.3, 1.7, -0.6),
                                   (0.2, 0.35, 0.85)])
def test_feq_moments_exact(QL, Q, NOm, state):
    vs = oracle.VelocitySet(QL, Q, NOm)
    n, T, beta = state
    fe = oracle.feq(vs, n, T, beta)
    M = oracle.sod_moments(vs, fe[:, None])[0]
    ref = _mj_moments(n, T, beta)
    assert np.max(np.abs(M[:5] - ref) / np.abs(ref).max()) < 2e-14
    # derived fields of an equilibrium: Landau state recovered, q = Pi = 0
    assert M[5] == pytest.approx(n, rel=1e-13)
    assert M[8] == pytest.approx(T, rel=1e-13)
    assert M[9] == pytest.approx(beta, abs=1e-13)
    assert abs(M[11]) < 1e-13 and abs(M[12]) < 1e-13


def test_feq_rest_frame_closed_form():
    """At u = 0 the expansion gives f_jk = (n/4) w_j w_k [1 + (1 - theta)(3 - pb_k)]."""
    vs = oracle.VelocitySet(3, 8, 3)
    n, T = 0.4, 0.8
    fe = oracle.feq(vs, n, T, 0.0).reshape(vs.QL, vs.Q)
    ref = n / 4 * np.outer(vs.wL * (1 + (1 - T) * (3 - vs.pb)), vs.wxi)
    assert np.max(np.abs(fe - ref)) < 1e-16


def test_landau_eigenproblem():
    rng = np.random.default_rng(1)
    for _ in range(50):
        # moments of a random positive distribution are always physical
        vs = VS6
        f = rng.uniform(0.0, 1.0, vs.V) ** 3 * np.outer(vs.wL, vs.wxi).ravel()
        M = oracle.sod_moments(vs, f[:, None])[0, :5]
        L = oracle.landau(M)
        assert L is not None
        T00, T0z, Tzz = M[2], M[3], M[4]
        # T^a_g u^g = -E u^a with eta = diag(-1, 1): T^a_g = T^{ab} eta_{bg}
        Tmix = np.array([[-T00, T0z], [-T0z, Tzz]])
        uvec = L["gamma"] * np.array([1.0, L["beta"]])
        res = Tmix @ uvec + L["E"] * uvec
        assert np.max(np.abs(res)) < 1e-13 * L["E"] * L["gamma"]
        # the same eigenvalue from the library eigen-solver
        ev = np.linalg.eigvals(Tmix)
        assert np.min(np.abs(ev + L["E"])) < 1e-12 * L["E"]
        assert L["E"] > 0 and L["gamma"] >= 1


def test_landau_round_trip():
    for n, T, beta in [(1.0, 1.0, 0.0), (0.3, 0.5, 0.7), (2.0, 0.4, -0.99)]:
        L = oracle.landau(_mj_moments(n, T, beta))
        assert L["n"] == pytest.approx(n, rel=1e-13)
        assert L["T"] == pytest.approx(T, rel=1e-13)
        assert L["beta"] == pytest.approx(beta, rel=1e-12, abs=1e-15)


def test_landau_rejects_unphysical():
    assert oracle.landau([1.0, 0.0, 1.0, 2.0, 0.2]) is None      # |T0z| > T00


def test_collision_invariants():
    """A random non-equilibrium cell: the AW collision term conserves N^0, T^00,
    T^0z (eq. collinv) when f^eq is built from the Landau frame."""
    rng = np.random.default_rng(2)
    for QL, Q, NOm in [(2, 8, 3), (3, 16, 4), (3, 40, 2)]:
        vs = oracle.VelocitySet(QL, Q, NOm)
        f = rng.uniform(0.2, 1.0, vs.V) * np.outer(vs.wL, vs.wxi).ravel()
        M = oracle.sod_moments(vs, f[:, None])[0]
        n, T, beta = M[5], M[8], M[9]
        g = 1 / np.sqrt(1 - beta ** 2)
        fe = oracle.feq(vs, n, T, beta)
        xi = np.tile(vs.xi, QL)
        p = np.repeat(vs.pb * vs.T0, Q)
        C = -g * (1 - beta * xi) * (f - fe)
        scale = np.abs(C).sum() * p.max()
        for wgt in (np.ones_like(p), p, p * xi):
            assert abs(np.sum(C * wgt)) < 1e-14 * scale


def test_mj_exact_nodes_vs_expansion_rest():
    """At T = T0 and u = 0 the truncated expansion equals the exact MJ value at the
    nodes: f_jk = 2 pi e^{pb_k} w_j w_k n/(8 pi) e^{-pb_k} = n w_j w_k / 4 (eqs. MJ, fjk)."""
    vs = oracle.VelocitySet(2, 6, 5)
    fe = oracle.feq(vs, 1.0, 1.0, 0.0)
    ref = np.outer(vs.wL, vs.wxi).ravel() / 4.0
    assert np.max(np.abs(fe - ref)) < 1e-16
