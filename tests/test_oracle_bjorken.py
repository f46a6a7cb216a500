"""Pins of the oracle's Bjorken-flow step (Sec. V; operator eq. L_Bjorken) against
what the paper and the structure of the equations fix:

* the momentum-space terms conserve particle number and give the Bjorken
  energy equation d(tau E)/dtau = -P_L exactly at the semi-discrete level
  (eqs. bjorken_macro; column identities of K^L and K^P);
* ideal gas: tau n = 1 to rounding at any step (eq. bjorken_n: the RK3 stages
  integrate the number equation exactly), energy converging at third order (eq. rk3);
* free streaming follows the closed forms of eq. bjorken_bal, which are
  themselves checked against direct quadrature of eq. milne_bal_f;
* small eta/s approaches the ideal fluid, P tau^{4/3} -> 1 (eq. bjorken_inv),
  and agrees with second-order hydrodynamics (eq. milne_hydro2);
* the parton gas in the transition regime agrees with the Florkowski
  semi-analytic solution (eq. flork_sol).
"""
import numpy as np
import pytest
from scipy import integrate

import oracle
from oracle import bjorken_ref


def test_energy_identity_and_number_semi_discrete():
    rng = np.random.default_rng(7)
    for QL, Q in [(2, 8), (3, 20), (3, 41)]:
        vs = oracle.VelocitySet(QL, Q, min(Q - 1, 5))
        B = oracle.Bjorken(vs, tau_mode=oracle.TAU_CONST, tau_r=0.3)
        f = rng.uniform(0.3, 1.0, vs.V) * np.outer(vs.wL, vs.wxi).ravel()
        tau = 1.7
        L = B.L(f, tau)
        p = np.repeat(vs.pb * vs.T0, Q)
        xi = np.tile(vs.xi, QL)
        E, PL, N = np.sum(p * f), np.sum(p * xi * xi * f), np.sum(f)
        assert tau * np.sum(p * L) + E + PL == pytest.approx(0.0, abs=1e-13 * E)
        assert tau * np.sum(L) + N == pytest.approx(0.0, abs=1e-13 * N)


def _ideal_run(dtau, tau_f=2.0, Q=12):
    vs = oracle.VelocitySet(2, Q, 5)
    B = oracle.Bjorken(vs, gas=oracle.GAS_IDEAL, tau_mode=oracle.TAU_ETAS, tau_aw0=0.2)
    nsteps = int(round((tau_f - 1.0) / dtau))
    f, tau = B.run(B.init(), 1.0, dtau, nsteps)
    return vs, f, tau


def test_number_density_exact():
    """tau n = 1 is recovered to rounding at any step size: the number equation
    d(tau N)/dtau = 0 is integrated exactly by the RK3 stages (eq. rk3, Table II)."""
    for dtau in (8e-2, 2e-2, 1e-3):
        vs, f, tau = _ideal_run(dtau, tau_f=1.4)
        assert abs(tau * np.sum(f) - 1.0) < 4e-15


def test_energy_rk3_third_order():
    """The energy density converges at third order in dtau (eq. rk3)."""
    ref = np.sum(np.repeat(_ideal_run(2.5e-3)[0].pb, 12) * _ideal_run(2.5e-3)[1])
    errs = []
    for dtau in (4e-2, 2e-2, 1e-2):
        vs, f, tau = _ideal_run(dtau)
        E = np.sum(np.repeat(vs.pb * vs.T0, vs.Q) * f)
        errs.append(abs(E - ref))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(orders - 3.0) < 0.2), orders


def test_free_streaming_closed_form_vs_quadrature():
    """eq. bjorken_bal against direct integration of the moments of eq. milne_bal_f:
    P = (1/3) int d^3p p f, P_L = int d^3p p xi^2 f with f = e^{-p s}/(8 pi),
    s = sqrt(1 + (tau^2 - 1) xi^2); the p-integral gives 3!/s^4."""
    for tau in (1.0, 1.5, 3.0, 10.0):
        s = lambda x: np.sqrt(1 + (tau ** 2 - 1) * x ** 2)
        E = integrate.quad(lambda x: 2 * np.pi * 6.0 / s(x) ** 4 / (8 * np.pi), -1, 1, epsabs=1e-14)[0]
        PLq = integrate.quad(lambda x: 2 * np.pi * 6.0 * x * x / s(x) ** 4 / (8 * np.pi), -1, 1,
                             epsabs=1e-14)[0]
        P, PL = bjorken_ref.free_streaming(tau)
        assert P == pytest.approx(E / 3, rel=1e-12)
        assert PL == pytest.approx(PLq, rel=1e-10, abs=1e-14)


def test_free_streaming_asymptote():
    from conftest import load_golden
    val = load_golden()["bjorken_tauP_asymptote"][0]
    P, _ = bjorken_ref.free_streaming(1e7)
    assert 1e7 * P == pytest.approx(val, rel=1e-6)


def test_free_streaming_oracle():
    """tau_AW = infinity: the oracle follows eq. bjorken_bal (Q_xi = 40, N_Omega = 5)."""
    vs = oracle.VelocitySet(2, 40, 5)
    B = oracle.Bjorken(vs, tau_mode=oracle.TAU_INF)
    f, tau, hist = B.run(B.init(), 1.0, 1e-3, 4000, history=True)
    taus = 1.0 + 1e-3 * np.arange(4001)
    P, PL = bjorken_ref.free_streaming(taus)
    assert np.max(np.abs(hist[:, 1] / 3 - P) / P) < 2e-3
    assert np.max(np.abs(hist[:, 2] - PL) / P) < 2e-3
    # and the number density is conserved exactly in tau n
    assert np.max(np.abs(taus * hist[:, 0] - 1.0)) < 1e-10


def test_ideal_fluid_limit():
    """eta/s -> 0: P tau^{4/3} -> 1 (eq. bjorken_inv); at small tau_AW0 the
    second-order equations (eq. milne_hydro2) agree with the kinetic solution."""
    vs = oracle.VelocitySet(2, 20, 5)
    res = []
    for taw0 in (0.02, 0.005):
        B = oracle.Bjorken(vs, gas=oracle.GAS_IDEAL, tau_mode=oracle.TAU_ETAS, tau_aw0=taw0)
        f, tau, hist = B.run(B.init(), 1.0, 1e-3, 2000, history=True)
        taus = 1.0 + 1e-3 * np.arange(2001)
        P = hist[:, 1] / 3
        res.append(abs(P[-1] * tau ** (4.0 / 3.0) - 1.0))
        P2, Pi2 = bjorken_ref.second_order(taus[::100], taw0, gas="ideal")
        assert np.max(np.abs(P[::100] - P2) / P2) < 5 * taw0 ** 2 + 1e-4
    # deviation from the ideal fluid shrinks ~ linearly with tau_AW0
    assert res[1] < 0.4 * res[0]


@pytest.mark.slow
def test_parton_gas_florkowski():
    """Transition regime, parton gas (T = P^{1/4}, n_eq = T^3, tau_AW = tau_AW0/T):
    the kinetic solution follows the Florkowski iteration (eq. flork_sol)."""
    taw0 = 0.5
    tau_f = 6.0
    tg, T, n, PL = bjorken_ref.florkowski(taw0, tau_f=tau_f, dtau=0.01, tol=1e-9)
    vs = oracle.VelocitySet(2, 40, 5)
    B = oracle.Bjorken(vs, gas=oracle.GAS_PARTON, tau_mode=oracle.TAU_ETAS, tau_aw0=taw0)
    nsteps = int(round((tau_f - 1) / 1e-3))
    f, tau, hist = B.run(B.init(), 1.0, 1e-3, nsteps, history=True)
    taus = 1.0 + 1e-3 * np.arange(nsteps + 1)
    Tk = (hist[:, 1] / 3) ** 0.25
    Ti = np.interp(tg, taus, Tk)
    assert np.max(np.abs(Ti - T) / T) < 2e-4
    nk = np.interp(tg, taus, hist[:, 0])
    assert np.max(np.abs(nk - n) / n) < 5e-4
