"""Pins of the oracle's in-loop feedback pieces (oracle/mlp.py inject,
project): the moments they must move or keep, by their definitions, and the
projection of an equilibrium, which must be the low-order equilibrium of the
same state (the pinned f^eq of Sec. III D)."""
import numpy as np
import pytest

import oracle
from oracle import mlp
from tests import inputs


def _moments(vs, f):
    return mlp._moment_rows(vs) @ f


@pytest.mark.parametrize("QL,Q,NOm", [(3, 8, 4), (2, 3, 2), (4, 16, 5)])
def test_inject_moves_only_the_energy_momentum_tensor(QL, Q, NOm):
    vs = oracle.VelocitySet(QL, Q, NOm)
    rng = inputs.rng(1)
    f = rng.uniform(0.1, 1.0, (vs.V, 7)) * np.outer(vs.wL, vs.wxi).ravel()[:, None]
    dT = rng.normal(size=(7, 3)) * 0.01
    g = mlp.inject(vs, f, dT)
    d = _moments(vs, g) - _moments(vs, f)
    scale = np.max(np.abs(_moments(vs, f)))
    assert np.max(np.abs(d[:2])) < 1e-14 * scale
    assert np.allclose(d[2:].T, dT, rtol=1e-12, atol=1e-14 * scale)
    # the change has the radial shape L_1(pbar_k) and is quadratic in xi_j
    dd = (g - f).reshape(QL, Q, 7) / (np.outer(vs.wL * (3.0 - vs.pb), vs.wxi)[:, :, None])
    for s in range(7):
        c = np.polyfit(vs.xi, dd[0, :, s], 2)
        assert np.allclose(np.polyval(c, vs.xi), dd[0, :, s], rtol=1e-10, atol=1e-12)
        assert np.allclose(dd[:, :, s], dd[:1, :, s], rtol=1e-10, atol=1e-12)


def test_inject_moves_the_particle_current_alone():
    vs = oracle.VelocitySet(3, 8, 4)
    f = np.outer(vs.wL, vs.wxi).ravel()[:, None] * np.ones((1, 2))
    dN = np.array([[0.01, -0.02], [0.0, 0.03]])
    d = _moments(vs, mlp.inject(vs, f, np.zeros((2, 3)), dN)) - _moments(vs, f)
    assert np.allclose(d[:2].T, dN, rtol=1e-12, atol=1e-15)
    assert np.max(np.abs(d[2:])) < 1e-14


def test_project_of_an_equilibrium_is_the_low_order_equilibrium():
    hi, lo = oracle.VelocitySet(3, 64, 4), oracle.VelocitySet(3, 8, 4)
    states = [(1.0, 1.0, 0.0), (0.4, 0.8, 0.3), (1.3, 0.6, -0.45)]
    f_hi = np.stack([oracle.feq(hi, n, T, b) for n, T, b in states], axis=1)
    g = mlp.project(hi, f_hi, lo)
    want = np.stack([oracle.feq(lo, n, T, b) for n, T, b in states], axis=1)
    assert np.max(np.abs(g - want)) < 1e-13 * np.max(np.abs(want))


def test_project_keeps_every_conserved_moment():
    hi, lo = oracle.VelocitySet(3, 40, 4), oracle.VelocitySet(3, 8, 4)
    rng = inputs.rng(4)
    f_hi = np.stack([oracle.feq(hi, 1.0, 1.0, b) for b in (0.1, -0.3, 0.5)], axis=1)
    f_hi *= 1.0 + 0.1 * rng.uniform(-1, 1, f_hi.shape)
    g = mlp.project(hi, f_hi, lo)
    assert np.allclose(_moments(lo, g), _moments(hi, f_hi), rtol=1e-12, atol=1e-14)
