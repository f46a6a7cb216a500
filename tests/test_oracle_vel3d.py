"""Pins of the oracle for velocity sets with azimuthal nodes (oracle/vel3d.py):
the azimuthal rule against closed-form integrals, the truncated equilibrium's
N^mu and T^{mu nu} against the ideal-gas closed forms (Sec. II, Sec. III D:
N_Omega >= 2 keeps them exact), reduction to the aligned velocity set of the
paper when u is along z, the rotation symmetry of the node set, and the
Landau frame against its defining eigen-equation and a boosted equilibrium."""
import numpy as np
import pytest

import oracle
from oracle import vel3d

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _random_u(rng, beta_max):
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    beta = rng.uniform(0.0, beta_max)
    return d * beta / np.sqrt(1.0 - beta * beta)


@pytest.mark.parametrize("Qphi", [1, 3, 7, 12])
def test_azimuthal_rule_exact_below_its_degree(Qphi):
    """sum_l (2 pi / Q) cos(a phi_l) sin(b phi_l)^e equals the integral over
    [0, 2 pi) for every trigonometric polynomial of degree < Q."""
    vs = vel3d.VelocitySet3(2, 4, Qphi, 1)
    wphi = 2.0 * np.pi / Qphi
    for q in range(Qphi):
        c = wphi * np.sum(np.cos(q * vs.phi))
        s = wphi * np.sum(np.sin(q * vs.phi))
        assert c == pytest.approx(2.0 * np.pi if q == 0 else 0.0, abs=1e-12)
        assert s == pytest.approx(0.0, abs=1e-12)
    # and it is not exact at degree Q (the rule aliases cos(Q phi) onto 1)
    assert wphi * np.sum(np.cos(Qphi * vs.phi)) == pytest.approx(2.0 * np.pi)


@pytest.mark.parametrize("QL,Q,Qphi,NOm", [(2, 6, 5, 2), (3, 8, 6, 3), (3, 16, 8, 4), (3, 12, 9, 6)])
def test_feq3_moments_are_the_ideal_gas_closed_forms(QL, Q, Qphi, NOm):
    vs = vel3d.VelocitySet3(QL, Q, Qphi, NOm)
    rng = np.random.default_rng(11)
    for _ in range(6):
        n, T = rng.uniform(0.3, 2.0), rng.uniform(0.4, 2.0)
        u = _random_u(rng, 0.6 if NOm < 4 else 0.8)
        f = vel3d.feq3(vs, n, T, u)
        N, Tm = vel3d.moments3(vs, f)
        Nw, Tw = vel3d.equilibrium_moments(n, T, u)
        assert _rel(N[:, 0], Nw) < 1e-12
        assert _rel(Tm[:, :, 0], Tw) < 1e-12


def test_feq3_temperature_scale_T0():
    vs = vel3d.VelocitySet3(3, 10, 6, 3, T0=0.7)
    u = np.array([0.2, -0.1, 0.3])
    N, Tm = vel3d.moments3(vs, vel3d.feq3(vs, 1.3, 0.9, u))
    Nw, Tw = vel3d.equilibrium_moments(1.3, 0.9, u)
    assert _rel(N[:, 0], Nw) < 1e-12 and _rel(Tm[:, :, 0], Tw) < 1e-12


@pytest.mark.parametrize("Qphi", [1, 4, 7])
@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_feq3_along_z_is_the_aligned_set(Qphi, sign):
    """u along +-z: every azimuth carries 1/Q_phi of the aligned set's f^eq_{jk}
    (eq. fjk with the single point phi = 0) at the same (j, k)."""
    vs = vel3d.VelocitySet3(3, 12, Qphi, 4)
    beta = 0.55
    u = np.array([0.0, 0.0, sign * beta / np.sqrt(1.0 - beta * beta)])
    f = vel3d.feq3(vs, 0.8, 1.2, u).reshape(3, Qphi, 12)
    f1 = oracle.feq(vs.base, 0.8, 1.2, sign * beta).reshape(3, 12)
    for l in range(Qphi):
        assert _rel(f[:, l, :] * Qphi, f1) < 1e-13


def test_feq3_rotation_by_one_azimuthal_step():
    Qphi = 6
    vs = vel3d.VelocitySet3(2, 10, Qphi, 4)
    u = np.array([0.35, 0.1, -0.2])
    a = 2.0 * np.pi / Qphi
    R = np.array([[np.cos(a), -np.sin(a), 0.0], [np.sin(a), np.cos(a), 0.0], [0.0, 0.0, 1.0]])
    f = vel3d.feq3(vs, 1.0, 1.0, u).reshape(2, Qphi, 10)
    g = vel3d.feq3(vs, 1.0, 1.0, R @ u).reshape(2, Qphi, 10)
    assert _rel(np.roll(f, 1, axis=1), g) < 1e-13


def test_feq3_at_rest_is_isotropic():
    vs = vel3d.VelocitySet3(3, 8, 5, 4)
    f = vel3d.feq3(vs, 1.0, 1.0, np.zeros(3)).reshape(3, 5, 8)
    per_dir = f / vs.base.wxi[None, None, :]
    assert np.allclose(per_dir, per_dir[:, :1, :1], rtol=1e-13, atol=0.0)


def test_landau3_recovers_a_boosted_equilibrium():
    rng = np.random.default_rng(5)
    for _ in range(20):
        n, T = rng.uniform(0.2, 3.0), rng.uniform(0.2, 3.0)
        u = _random_u(rng, 0.95)
        N, Tm = vel3d.equilibrium_moments(n, T, u)
        L = vel3d.landau3(N, Tm)
        assert L is not None
        assert L["n"] == pytest.approx(n, rel=1e-12)
        assert L["T"] == pytest.approx(T, rel=1e-12)
        assert _rel(L["u"][1:], u) < 1e-11


def test_landau3_solves_its_eigen_equation_off_equilibrium():
    vs = vel3d.VelocitySet3(3, 12, 7, 4)
    rng = np.random.default_rng(9)
    for _ in range(10):
        f = vel3d.feq3(vs, 1.0, 1.0, _random_u(rng, 0.7)) * (1.0 + 0.2 * rng.uniform(-1, 1, vs.V))
        N, Tm = vel3d.moments3(vs, f)
        L = vel3d.landau3(N[:, 0], Tm[:, :, 0])
        u, E = L["u"], L["E"]
        res = Tm[:, :, 0] @ vel3d.METRIC @ u - E * u
        assert np.max(np.abs(res)) < 1e-12 * np.max(np.abs(Tm))
        assert u[0] ** 2 - u[1:] @ u[1:] == pytest.approx(1.0, abs=1e-12)


def test_landau3_along_z_matches_the_aligned_closed_form():
    """T^{mu nu} with u along z and T^xx = T^yy: the 2x2 problem of eqs.
    E_landau, u_landau (the aligned oracle) gives the same frame."""
    vs = vel3d.VelocitySet3(3, 12, 6, 4)
    f = vel3d.feq3(vs, 1.1, 0.9, np.array([0.0, 0.0, 0.4]))
    f = f * (1.0 + 0.1 * np.cos(np.pi * vs.Om[:, 2]))      # off equilibrium, still azimuthally symmetric
    N, Tm = vel3d.moments3(vs, f)
    L3 = vel3d.landau3(N[:, 0], Tm[:, :, 0])
    L1 = oracle.landau(np.array([N[0, 0], N[3, 0], Tm[0, 0, 0], Tm[0, 3, 0], Tm[3, 3, 0]]))
    assert L3["E"] == pytest.approx(L1["E"], rel=1e-12)
    assert L3["n"] == pytest.approx(L1["n"], rel=1e-12)
    assert L3["u"][3] == pytest.approx(L1["beta"] * L1["gamma"], rel=1e-11)
    assert abs(L3["u"][1]) < 1e-13 and abs(L3["u"][2]) < 1e-13


def test_landau3_rejects_spacelike_flux():
    N = np.array([1.0, 0.0, 0.0, 0.0])
    T = np.diag([1.0, 2.0, 2.0, 2.0])        # pressure above energy density
    T[0, 1] = T[1, 0] = 1.5
    assert vel3d.landau3(N, T) is None
