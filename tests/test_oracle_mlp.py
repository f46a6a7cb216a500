"""Pins of the oracle's learned-correction reference (not part of the paper, so
pinned by calculus and construction instead): backward against central finite
differences, Adam against its textbook recursion on a quadratic, features
against moments computed from the definition and the equilibrium's exact
moments."""
import numpy as np
import pytest

import oracle
from oracle import mlp


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    P = mlp.init_params(1)
    for k in P:
        P[k] = P[k] + 0.05 * rng.standard_normal(P[k].shape)     # non-zero biases too
    X = rng.standard_normal((17, mlp.N_IN))
    T = rng.standard_normal((17, mlp.N_OUT))
    y, cache = mlp.forward(P, X)
    G = mlp.backward(P, cache, y, T)
    h = 1e-6
    for k in P:
        flat = P[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(12, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = mlp.loss(mlp.forward(P, X)[0], T)
            flat[idx] = old - h
            lm = mlp.loss(mlp.forward(P, X)[0], T)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert G[k].reshape(-1)[idx] == pytest.approx(fd, rel=1e-6, abs=1e-9), (k, idx)


def test_adam_minimises_quadratic():
    """Adam on f(p) = |p - c|^2 reaches c; first step has length lr per coordinate."""
    c = np.array([1.0, -2.0, 0.5])
    P = {"p": np.zeros(3)}
    state = {}
    mlp.adam_step(P, {"p": 2 * (P["p"] - c)}, state, 1, lr=0.1)
    assert np.allclose(np.abs(P["p"]), 0.1, rtol=1e-6)
    for t in range(2, 2000):
        mlp.adam_step(P, {"p": 2 * (P["p"] - c)}, state, t, lr=0.01)
    assert np.allclose(P["p"], c, atol=1e-3)


def test_features_definition():
    vs = oracle.VelocitySet(3, 8, 3)
    rng = np.random.default_rng(2)
    nz = 9
    f = rng.uniform(0.1, 1.0, (vs.V, nz)) * np.outer(vs.wL, vs.wxi).ravel()[:, None]
    F = mlp.features(vs, f, np.log(0.1))
    assert F.shape == (nz, 81)
    s = 4
    xi = np.tile(vs.xi, 3)
    p = np.repeat(vs.pb, 8)
    n0 = f[:, s].sum()
    e0 = (p * f[:, s]).sum()
    for o in range(5):
        c = min(max(s - 2 + o, 0), nz - 1)
        for r in range(8):
            assert F[s, 16 * o + r] == pytest.approx((xi ** r * f[:, c]).sum() / n0, rel=1e-13)
            assert F[s, 16 * o + 8 + r] == pytest.approx((p * xi ** r * f[:, c]).sum() / e0, rel=1e-13)
    assert F[s, 80] == pytest.approx(np.log(0.1))
    # at rest in equilibrium the odd angular moments vanish and M_{0,2}/N^0 = 1/3
    fe = oracle.feq(vs, 0.7, 0.9, 0.0)[:, None].repeat(5, axis=1)
    Fe = mlp.features(vs, fe, 0.0)
    assert abs(Fe[2, 1]) < 1e-15 and Fe[2, 2] == pytest.approx(1.0 / 3.0, rel=1e-14)
    assert Fe[2, 8] == pytest.approx(1.0, rel=1e-15)
