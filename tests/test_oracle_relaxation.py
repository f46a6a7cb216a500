"""Pins of the oracle's relaxation-time laws and of its time integration.

Relaxation time (Sec. IV B 2 and IV D; Sec. V C):
* tau_{A-W;0} = 5 hbar c (eta/s) / (T_ref L_ref) reproduces the printed
  0.3854 (T_ref = 0.4 GeV) and 0.4405 (T_ref = 0.35 GeV) per unit eta/s
  (eqs. Sod:tau1, Sod:tau2, L_ref = 6.4 fm);
* the reference fugacity of eq. lambda (g_s = 16) at the printed reference
  states is ~1 and ~1.715;
* the oracle's relaxation law at the printed initial states gives the printed
  left/right relaxation times 0.3854 / 0.7708 (eq. tau_LR, lambda_ref = 1) and
  0.3811 / 0.4795 (eq. tau_LR2, lambda_ref = 1.715), both through the exported
  law and as it acts inside L_Sod (the AW term of a state whose Landau frame
  is known);
* the Bjorken ideal-gas law as it acts inside L_Bjorken equals the reduced form
  the paper prints in terms of tau and P (eq. bjorken_tauAW_mu), away from
  lambda_bar = 1 where its log term matters.

Time integration (eq. rk3, Table II; Sec. III F):
* the Sod solver converges at third order in dt on a smooth non-equilibrium
  state (same grid, so only the time error changes);
* WENO5 + RK3 free streaming of a smooth profile converges at ~fifth order in
  dz towards the exact translated profile (time step shrinking faster).
"""
import numpy as np
import pytest

import oracle
from conftest import load_golden

G_S = 16                      # gluon degrees of freedom (eq. lambda_def)


def _golden(key):
    return load_golden()[key]


def _lambda_ref(n_ref_fm3, T_ref_GeV):
    """eq. lambda: lambda_ref = n_ref pi^2 / g_s (hbar c / k_B T_ref)^3."""
    return n_ref_fm3 * np.pi ** 2 / G_S * (oracle.HBARC_GEV_FM / T_ref_GeV) ** 3


def test_tau_aw0_printed_values():
    v, tol, _ = _golden("tau_aw0_per_etas")
    assert oracle.tau_aw0(1.0, 0.4, 6.4) == pytest.approx(v, abs=tol)
    v, tol, _ = _golden("tau_aw0_per_etas_2")
    assert oracle.tau_aw0(1.0, 0.35, 6.4) == pytest.approx(v, abs=tol)


def test_reference_fugacities():
    # eq. Sod:left: n_ref = 13.57 fm^-3 at 0.4 GeV -> lambda_ref ~ 1
    assert _lambda_ref(13.57, 0.4) == pytest.approx(1.0, abs=0.01)
    # eq. Sod:left2: n_ref = 15.514 fm^-3 at 0.35 GeV -> 1.715 (printed)
    v, tol, _ = _golden("lambda_ref_2")
    assert _lambda_ref(15.514, 0.35) == pytest.approx(v, abs=tol)


def _sod_etas(T_ref, lam_ref, vs=None):
    vs = vs or oracle.VelocitySet(2, 8, 3)
    return oracle.Sod(vs, 16, tau_mode=oracle.TAU_ETAS, tau_aw0=oracle.tau_aw0(1.0, T_ref, 6.4),
                      lambda_ref=lam_ref, bc=oracle.BC_OUTFLOW)


def test_relaxation_law_printed_first_setup():
    """eq. tau_LR: (n, T) = (1, 1) left and (0.125, 0.5) right (eq. Sod:right_adim)."""
    S = _sod_etas(0.4, 1.0)
    for key, (n, T) in (("tau_L_per_etas", (1.0, 1.0)), ("tau_R_per_etas", (0.125, 0.5))):
        v, tol, _ = _golden(key)
        assert S.relax_time(n, T) == pytest.approx(v, abs=tol), key


def test_relaxation_law_printed_second_setup():
    """eq. tau_LR2: (n, T) = (1, 1) left and (0.409, 1) right (eq. Sod:right2_adim),
    lambda_ref = 1.715 (eq. Sod:tau2)."""
    S = _sod_etas(0.35, _golden("lambda_ref_2")[0])
    for key, (n, T) in (("tau_L2_per_etas", (1.0, 1.0)), ("tau_R2_per_etas", (0.409, 1.0))):
        v, tol, _ = _golden(key)
        assert S.relax_time(n, T) == pytest.approx(v, abs=tol), key


def _p2_perturbed(vs, n, T, eps=1e-3):
    """f^eq(n, T, 0) (1 + eps P_2(xi_j)): at rest the populations of f^eq are
    w_j times a function of k, and sum_j w_j P_2(xi_j) = sum_j w_j xi_j P_2(xi_j) = 0,
    so N^0, N^z, T^00, T^0z keep their equilibrium values; T^0z = 0 makes
    E = T^00 and beta = 0, so the Landau frame is still (n, T, 0) while f
    differs from f^eq by eps f^eq P_2."""
    f0 = oracle.feq(vs, n, T, 0.0)
    P2 = 0.5 * (3 * np.tile(vs.xi, vs.QL) ** 2 - 1)
    return f0 * (1 + eps * P2), f0 * eps * P2


@pytest.mark.parametrize("setup,states", [
    ((0.4, 1.0), (("tau_L_per_etas", 1.0, 1.0), ("tau_R_per_etas", 0.125, 0.5))),
    ((0.35, None), (("tau_L2_per_etas", 1.0, 1.0), ("tau_R2_per_etas", 0.409, 1.0))),
])
def test_relaxation_time_inside_L_sod(setup, states):
    """L_Sod of a z-uniform state is its AW term alone (constant planes carry
    equal fluxes through every face), -(f - f^eq)/tau at rest (eq. L_Sod): the
    tau it implies equals the printed relaxation times."""
    T_ref, lam = setup
    lam = lam if lam is not None else _golden("lambda_ref_2")[0]
    vs = oracle.VelocitySet(2, 8, 3)
    S = _sod_etas(T_ref, lam, vs)
    for key, n, T in states:
        f, df = _p2_perturbed(vs, n, T)
        L = S.L(np.repeat(f[:, None], 16, axis=1))
        sel = np.abs(df) > 0.1 * np.max(np.abs(df))
        taus = -df[sel][:, None] / L[sel, :]
        v, tol, _ = _golden(key)
        assert np.all(np.abs(taus - v) < tol), (key, taus.min(), taus.max())


@pytest.mark.parametrize("tau,T", [(2.0, 0.5), (5.0, 0.2), (1.5, 1.2)])
def test_bjorken_ideal_gas_relaxation_time(tau, T):
    """Inside L_Bjorken the AW term of an ideal gas with tau n = 1 relaxes at
    tau_AW = tau_AW0 / (tau P) [1 + ln(tau P^{3/4})]  (eq. bjorken_tauAW_mu),
    here at states with tau P^{3/4} far from 1."""
    vs = oracle.VelocitySet(3, 12, 4)
    taw0 = 0.37
    n = 1.0 / tau
    f, df = _p2_perturbed(vs, n, T)
    Bc = oracle.Bjorken(vs, gas=oracle.GAS_IDEAL, tau_mode=oracle.TAU_ETAS, tau_aw0=taw0)
    Bf = oracle.Bjorken(vs, gas=oracle.GAS_IDEAL, tau_mode=oracle.TAU_INF)
    coll = Bc.L(f, tau) - Bf.L(f, tau)
    P = n * T
    expect = taw0 / (tau * P) * (1.0 + np.log(tau * P ** 0.75))
    assert abs(np.log(tau * P ** 0.75)) > 0.1
    sel = np.abs(df) > 0.1 * np.max(np.abs(df))
    got = -df[sel] / coll[sel]
    assert np.max(np.abs(got / expect - 1)) < 1e-10


def test_sod_rk3_third_order():
    """Smooth moving non-equilibrium state, t = 0.06, dt halved three times on
    one grid: successive differences shrink by 2^3 (eq. rk3 is third order)."""
    vs = oracle.VelocitySet(2, 6, 4)
    nz = 32
    S = oracle.Sod(vs, nz, nL=1.0, TL=1.0, nR=1.0, TR=1.0, tau_r=0.05, bc=oracle.BC_OUTFLOW)
    z = -0.5 + (np.arange(nz) + 0.5) / nz
    bump = np.exp(-(z / 0.18) ** 2)
    base = np.stack([oracle.feq(vs, 1.0 + 0.3 * b, 1.0 + 0.2 * b, 0.25 * b) for b in bump], axis=1)
    f0 = base * (1 + 0.1 * np.cos(np.pi * z)[None, :] * np.tile(vs.xi, vs.QL)[:, None])
    t_end = 0.06
    sols = [S.run(f0, t_end / m, m) for m in (3, 6, 12, 24)]
    d = [np.max(np.abs(sols[i] - sols[i + 1])) for i in range(3)]
    orders = np.log2(np.array(d[:-1]) / np.array(d[1:]))
    assert d[-1] > 1e-12 * np.max(np.abs(f0))
    assert np.all(np.abs(orders - 3.0) < 0.2), orders


def test_weno5_rk3_free_streaming_order():
    """Ballistic limit (tau -> infinity): each population translates at xi_j.
    A smooth bump away from the ghosts is carried by WENO5 + RK3 with an error
    that falls at ~fifth order in dz (dt ~ dz^{5/3}, so the RK3 error falls as
    fast)."""
    vs = oracle.VelocitySet(2, 4, 3)
    xi = np.tile(vs.xi, vs.QL)
    feq = oracle.feq(vs, 1.0, 1.0, 0.0)
    t_end = 0.1
    prof = lambda z: 1.0 + 0.5 * np.exp(-(z / 0.1) ** 2)
    errs = []
    for nz in (80, 160, 320):
        S = oracle.Sod(vs, nz, nL=1.0, TL=1.0, nR=1.0, TR=1.0, tau_mode=oracle.TAU_INF, bc=oracle.BC_OUTFLOW)
        dz = 1.0 / nz
        z = -0.5 + (np.arange(nz) + 0.5) * dz
        # cell averages of the profile (5-point Gauss rule per cell)
        g, w = np.polynomial.legendre.leggauss(5)
        avg = lambda shift: sum(wi / 2 * prof(z[None, :] + gi * dz / 2 - shift) for gi, wi in zip(g, w))
        f0 = feq[:, None] * avg(0.0 * xi[:, None])
        m = int(np.ceil(t_end / (0.8 * dz ** (5 / 3))))
        f = S.run(f0, t_end / m, m)
        exact = feq[:, None] * avg(xi[:, None] * t_end)
        errs.append(np.max(np.abs(f - exact)))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 4.3), (errs, orders)
