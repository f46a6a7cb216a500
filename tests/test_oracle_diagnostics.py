"""Pins of the oracle's diagnostics (Sec. IV B 3, IV E, V E):

* the window integral is exact (to rounding) for cell averages of a linear
  field and equals a brute-force sum;
* the Sod error measure (eq. eps_def) of hand-built profiles with known
  deviations and ranges, including gamma from beta;
* the Bjorken L2 norm (eq. bjork_L2) of power laws against its closed form;
* physics: in a near-inviscid Sod run (the paper's states, eta/s = 5e-3, in
  the oracle) the integrated heat flux over the contact and the shock and the
  integrated shear pressure over the shock agree with the analytic values of
  eqs. intq, intpi with the Chapman-Enskog coefficients (eq. tcoeff_ce), and
  the shear pressure integrates to ~0 over the contact.
"""
import numpy as np
import pytest

import oracle
from oracle import diagnostics as dg, riemann


def _rows(n=None, T=None, beta=None, P=None, Pi=None, size=10):
    M = np.zeros((size, 13))
    for key, col in (("n", 5), ("T", 8), ("beta", 9), ("P", 7), ("Pi", 12)):
        v = locals()[key]
        if v is not None:
            M[:, col] = v
    return M


def test_window_integral_linear_field():
    nz, dz = 50, 0.02
    z = (np.arange(nz) + 0.5) * dz
    M = np.stack([3.0 + 2.0 * z, -z], axis=1)       # cell averages of linear fields = centre values
    got = dg.window_integral(M, dz, 10, 30)
    a, b = 10 * dz, 30 * dz
    assert got[0] == pytest.approx(3.0 * (b - a) + (b * b - a * a), rel=1e-14)
    assert got[1] == pytest.approx(-(b * b - a * a) / 2, rel=1e-14)
    assert np.array_equal(dg.window_integral(M, dz, 7, 7), np.zeros(2))


def test_sod_eps_known_profiles():
    z = np.linspace(0, 1, 11)
    n = 1 + z                                  # range 1
    T = 2 * z                                  # range 2
    beta = 0.6 * z                             # gamma from 1 to 1.25
    M = _rows(n=n, T=T, beta=beta, size=11)
    R = M.copy()
    R[4, 5] += 0.03                            # n off by 0.03 at one cell -> eps_n = 0.03
    R[7, 8] -= 0.1                             # T off by 0.1 -> eps_T = 0.05
    e = dg.sod_eps(M, R)
    assert e[0] == pytest.approx(0.03, rel=1e-12)
    assert e[1] == pytest.approx(0.05, rel=1e-12)
    assert e[2] == 0.0 and e[3] == pytest.approx(0.05, rel=1e-12)
    R2 = M.copy()
    R2[10, 9] = 0.0                            # gamma 1 instead of 1.25 at the end
    assert dg.sod_eps(M, R2)[2] == pytest.approx(1.0, rel=1e-12)


def test_bjorken_l2_closed_form():
    """A(tau) = a tau^{-4/3} vs a_ref tau^{-4/3}: L2 = |a - a_ref| sqrt(int_1^tf
    tau^{-8/3} dtau / (tf - 1)); the trapezoid rule converges to it."""
    tf, N = 40.0, 39001
    tau = np.linspace(1.0, tf, N)
    dtau = tau[1] - tau[0]
    H = _rows(n=1.1 * tau ** (-4 / 3), T=0.5 * tau ** (-1 / 3), P=tau ** (-4 / 3), Pi=0.0 * tau, size=N)
    R = _rows(n=tau ** (-4 / 3), T=0.5 * tau ** (-1 / 3), P=tau ** (-4 / 3), Pi=-0.01 / tau, size=N)
    got = dg.bjorken_l2(H, R, dtau)
    exact_n = 0.1 * np.sqrt((1 - tf ** (-5 / 3)) * 3 / 5 / (tf - 1))
    exact_pi = 0.01 * np.sqrt((1 - 1 / tf) / (tf - 1))
    assert got[0] == pytest.approx(exact_n, rel=1e-6)
    assert got[1] == 0.0 and got[2] == 0.0
    assert got[3] == pytest.approx(exact_pi, rel=1e-6)
    assert got[4] == pytest.approx(max(exact_n, exact_pi), rel=1e-6)


@pytest.mark.slow
def test_integrated_noneq_matches_analytic():
    es = 5e-3
    taw0 = oracle.tau_aw0(es, 0.4, 6.4)
    tau_of = lambda n, T: taw0 / T * (1 - 0.25 * np.log(n / T ** 3))
    pred = dg.integrated_noneq(1.0, 1.0, 0.125, 0.0625, tau_of)
    nz, t_end = 1600, 0.3
    vs = oracle.VelocitySet(2, 16, 4)
    S = oracle.Sod(vs, nz, nL=1, TL=1, nR=0.125, TR=0.5, tau_mode=oracle.TAU_ETAS, tau_aw0=taw0, bc=oracle.BC_EQ)
    dt = 0.5 / nz
    f = S.run(S.init(), dt, int(round(t_end / dt)))
    M, dz = S.moments(f), 1.0 / nz
    st = riemann.riemann_star(1, 1, 0.125, 0.0625)
    z = -0.5 + (np.arange(nz) + 0.5) * dz
    mid = 0.5 * (st["beta_C"] + st["beta_shock"]) * t_end
    a, b, c = np.searchsorted(z, st["zeta_T"] * t_end + 0.02), np.searchsorted(z, mid), np.searchsorted(z, 0.49)
    Ic, Is = dg.window_integral(M, dz, a, b), dg.window_integral(M, dz, b, c)
    assert Ic[11] == pytest.approx(pred["q_contact"], rel=0.12)
    assert Is[11] == pytest.approx(pred["q_shock"], rel=0.08)
    assert Is[12] == pytest.approx(pred["Pi_shock"], rel=0.03)
    assert abs(Ic[12]) < 0.12 * pred["Pi_shock"]
