"""Pins of the oracle's Sod time step (Secs. III F, IV) against what the paper and
the structure of the scheme fix, independently of the oracle's own code:

* a uniform equilibrium (at rest or moving) is a fixed point of L_Sod: WENO5
  reproduces a constant flux and the AW term vanishes at f = f^eq;
* global conservation before any signal reaches the ghost cells: the cell sums
  of N^0 and T^00 stay fixed, and the sum of T^0z grows at exactly P_L - P_R
  (flux telescoping, eq. L_Sod + collision invariants eq. collinv);
* mirror symmetry z -> -z, xi -> -xi with the two states swapped;
* free streaming (tau -> infinity): each population moves at xi_j, so between
  the fronts the moments are the exact discrete sums; as Q_xi grows they
  approach the continuum ballistic profiles (eqs. Sod:bal:Nmu, Sod:bal:Tmunu);
* near-inviscid flow reproduces the exact Riemann plateau of Sec. IV B 1.
"""
import numpy as np
import pytest

import oracle
from oracle import riemann


def _uniform_run(vs, n, T, beta, nz=40, steps=5, tau_r=0.05):
    S = oracle.Sod(vs, nz, nL=n, TL=T, nR=n, TR=T, tau_mode=oracle.TAU_CONST, tau_r=tau_r,
                   bc=oracle.BC_OUTFLOW)
    f0 = np.repeat(oracle.feq(vs, n, T, beta)[:, None], nz, axis=1)
    f = S.run(f0, 0.4 / nz, steps)
    return f0, f


@pytest.mark.parametrize("beta", [0.0, 0.35, -0.6])
def test_uniform_equilibrium_is_fixed_point(beta):
    vs = oracle.VelocitySet(3, 8, 3)
    f0, f = _uniform_run(vs, 0.7, 0.9, beta)
    assert np.max(np.abs(f - f0)) < 5e-15 * np.max(np.abs(f0))


def test_global_conservation_before_boundary():
    vs = oracle.VelocitySet(3, 8, 3)
    nz, steps = 200, 12                       # 9 cells per step << 100 cells to the ghosts
    dt = 0.5 / nz
    S = oracle.Sod(vs, nz, nL=1.0, TL=1.0, nR=0.4, TR=0.8, tau_r=2e-3)
    f0 = S.init()
    f = S.run(f0, dt, steps)
    M0 = S.moments(f0)[:, :5].sum(axis=0) * S.dz
    M1 = S.moments(f)[:, :5].sum(axis=0) * S.dz
    assert M1[0] == pytest.approx(M0[0], rel=1e-13)          # N^0
    assert M1[2] == pytest.approx(M0[2], rel=1e-13)          # T^00
    PL, PR = 1.0 * 1.0, 0.4 * 0.8
    assert M1[3] - M0[3] == pytest.approx(steps * dt * (PL - PR), rel=1e-11)
    # particles flow from left to right: N^z total grows from 0
    assert M1[1] > 0


def test_mirror_symmetry():
    vs = oracle.VelocitySet(2, 6, 4)
    nz, steps, dt = 64, 10, 0.4 / 64
    A = oracle.Sod(vs, nz, nL=1.0, TL=1.0, nR=0.3, TR=0.7, tau_r=0.01)
    B = oracle.Sod(vs, nz, nL=0.3, TL=0.7, nR=1.0, TR=1.0, tau_r=0.01)
    fA = A.run(A.init(), dt, steps).reshape(vs.QL, vs.Q, nz)
    fB = B.run(B.init(), dt, steps).reshape(vs.QL, vs.Q, nz)
    mirrored = fA[:, ::-1, ::-1]
    assert np.max(np.abs(fB - mirrored)) < 1e-13 * np.max(np.abs(fA))


def test_free_streaming_between_fronts():
    """tau = infinity: population (j,k) is f_L for z < xi_j t and f_R beyond."""
    vs = oracle.VelocitySet(2, 8, 3)
    nz, steps = 400, 60
    dt = 0.5 / nz
    S = oracle.Sod(vs, nz, nL=1.0, TL=1.0, nR=0.125, TR=0.5, tau_mode=oracle.TAU_INF)
    f = S.run(S.init(), dt, steps)
    t = steps * dt
    z = -0.5 + (np.arange(nz) + 0.5) * S.dz
    xi = np.tile(vs.xi, vs.QL)
    exact = np.where(z[None, :] < xi[:, None] * t, S.feqL[:, None], S.feqR[:, None])
    # WENO5 smears each front over a few cells; 25 cells away the profile is exact
    far = np.abs(z[None, :] - xi[:, None] * t) > 25 * S.dz
    assert far.sum() > 0.7 * far.size
    err = np.max(np.abs(f - exact)[far])
    assert err < 1e-15 * np.max(np.abs(f)) * 10, err
    # and near the fronts the solution is monotone between the two states
    lo = np.minimum(S.feqL, S.feqR)[:, None] - 1e-15
    hi = np.maximum(S.feqL, S.feqR)[:, None] + 1e-15
    assert np.all((f >= lo) & (f <= hi))


def test_free_streaming_approaches_continuum():
    """Discrete staircase -> continuum ballistic moments as Q_xi grows (O(1/Q_xi))."""
    nz, steps = 200, 80
    dt = 0.5 / nz
    t = steps * dt
    errs = []
    for Q in (10, 40):
        vs = oracle.VelocitySet(2, Q, 3)
        S = oracle.Sod(vs, nz, nL=1.0, TL=1.0, nR=0.125, TR=0.5, tau_mode=oracle.TAU_INF)
        f = S.run(S.init(), dt, steps)
        M = S.moments(f)[:, :5]
        zeta = (-0.5 + (np.arange(nz) + 0.5) * S.dz) / t
        ref = riemann.ballistic_sod(zeta, 1.0, 1.0, 0.125, 0.0625)
        inner = np.abs(zeta) < 0.9
        errs.append(np.max(np.abs(M - ref)[inner]) / np.max(np.abs(ref)))
    assert errs[1] < 0.5 * errs[0]
    assert errs[1] < 0.05


def test_ballistic_reference_conservation():
    """The continuum ballistic profiles conserve N^0 and T^00 (integral over z of
    the deviation from the initial state vanishes) and carry the momentum
    injected at the rate P_L - P_R."""
    # the profiles are polynomials in zeta on [-1, 1]: a 10-point Gauss rule is exact
    zeta, w = np.polynomial.legendre.leggauss(10)
    nL, PL, nR, PR = 1.0, 1.0, 0.125, 0.0625
    M = riemann.ballistic_sod(zeta, nL, PL, nR, PR)
    init_int = np.array([nL + nR, 0.0, 3 * (PL + PR), 0.0, PL + PR])   # step function, exact
    d = w @ M - init_int
    assert abs(d[0]) < 1e-14 and abs(d[2]) < 1e-14
    assert d[3] == pytest.approx(PL - PR, rel=1e-14)


def test_riemann_printed_values():
    """Exact solution of Sec. IV B 1 reproduces the printed numbers (Sec. IV B 2)."""
    from conftest import load_golden
    g = load_golden()
    st = riemann.riemann_star(1.0, 1.0, 0.125, 0.0625)
    for key, name in [("riemann_beta_shock", "beta_shock"), ("riemann_beta_C", "beta_C"),
                      ("riemann_P_C", "PC"), ("riemann_n_I", "nI"), ("riemann_n_II", "nII"),
                      ("riemann_zeta_T", "zeta_T"), ("riemann_zeta_H", "zeta_H")]:
        val, tol, _ = g[key]
        assert st[name] == pytest.approx(val, abs=tol), key


def test_riemann_jump_conditions():
    """Rankine-Hugoniot across the shock for P = E/3: continuity of T^{zz} and T^{0z}
    fluxes in the shock frame, and of the particle flux."""
    nL, PL, nR, PR = 1.0, 1.0, 0.4, 0.32
    st = riemann.riemann_star(nL, PL, nR, PR)
    vs_, b, P = st["beta_shock"], st["beta_C"], st["PC"]
    g2 = 1 / (1 - b * b)
    # plateau II (moving, P_C, n_II) vs right state at rest; T^{0z} = 4 P g^2 b, T^{zz} = P(1 + 4 g^2 b^2)
    T0z, Tzz, T00 = 4 * P * g2 * b, P * (1 + 4 * g2 * b * b), P * (3 + 4 * g2 * b * b)
    # shock-frame flux continuity: [T^{0z}] = v_s [T^{00}], [T^{zz}] = v_s [T^{0z}], [N^z] = v_s [N^0]
    assert T0z - 0 == pytest.approx(vs_ * (T00 - 3 * PR), rel=1e-9)
    assert Tzz - PR == pytest.approx(vs_ * (T0z - 0), rel=1e-9)
    g = np.sqrt(g2)
    assert st["nII"] * g * b == pytest.approx(vs_ * (st["nII"] * g - nR), rel=1e-9)


@pytest.mark.slow
def test_near_inviscid_sod_plateau():
    """The Sod tube at N_z = 400, R-SLB(3;8) with Q_L = 3, tau = 1e-3, CFL 0.5,
    200 steps reproduces the exact inviscid plateau within a few per cent."""
    vs = oracle.VelocitySet(3, 8, 3)
    nz = 400
    S = oracle.Sod(vs, nz, nL=1.0, TL=1.0, nR=0.4, TR=0.8, tau_r=1e-3, bc=oracle.BC_OUTFLOW)
    f = S.run(S.init(), 0.5 / nz, 200)
    t = 200 * 0.5 / nz
    M = S.moments(f)
    zeta = (-0.5 + (np.arange(nz) + 0.5) * S.dz) / t
    st = riemann.riemann_star(1.0, 1.0, 0.4, 0.32)
    # plateau between the rarefaction tail and the shock, away from the contact
    sel = (zeta > st["zeta_T"] + 0.08) & (zeta < st["beta_shock"] - 0.08)
    P, beta = M[sel, 7], M[sel, 9]
    assert np.median(P) == pytest.approx(st["PC"], rel=0.02)
    assert np.median(beta) == pytest.approx(st["beta_C"], rel=0.05)
    left_plateau = (zeta > st["zeta_T"] + 0.08) & (zeta < st["beta_C"] - 0.08)
    right_plateau = (zeta > st["beta_C"] + 0.08) & (zeta < st["beta_shock"] - 0.08)
    assert np.median(M[left_plateau, 5]) == pytest.approx(st["nI"], rel=0.03)
    assert np.median(M[right_plateau, 5]) == pytest.approx(st["nII"], rel=0.03)
