"""Pins of the oracle's velocity-set tables against what the paper and calculus fix.

Gauss-Legendre exactness (eq. quad_xi: exact for polynomial degree < 2 Q_xi),
Gauss-Laguerre alpha=2 exactness (eq. quadL) and Table I, and the actions of the
discrete kernels K^L (eq. K_lag_disc) and K^P (eq. K_leg_disc) on functions
whose p- or xi-derivative terms are known in closed form.
"""
from fractions import Fraction
from math import factorial

import numpy as np
import pytest

from conftest import load_golden
from oracle import quadrature as oq


@pytest.mark.parametrize("Q", [2, 3, 8, 16, 21, 40, 100, 200])
def test_gauss_legendre_exactness(Q):
    xi, w = oq.gauss_legendre(Q)
    assert np.all(np.diff(xi) > 0)
    assert np.array_equal(xi, -xi[::-1])             # exact antisymmetry
    for r in range(0, 2 * Q):
        exact = 2.0 / (r + 1) if r % 2 == 0 else 0.0
        got = np.sum(w * xi ** r)
        assert abs(got - exact) <= 2e-15 * max(1.0, abs(exact)) + 1e-15, (Q, r, got, exact)
    # degree 2Q is not integrated exactly: the rule really has Q nodes.  The
    # Gauss error term is 2^{2Q+1} (Q!)^4 / ((2Q+1) ((2Q)!)^2) for x^{2Q}.
    err = np.sum(w * xi ** (2 * Q)) - 2.0 / (2 * Q + 1)
    expect = float(Fraction(2 ** (2 * Q + 1) * factorial(Q) ** 4, (2 * Q + 1) * factorial(2 * Q) ** 2))
    if expect > 1e-12:
        assert err == pytest.approx(-expect, rel=1e-6)


def test_gauss_legendre_matches_library():
    for Q in (5, 40, 200):
        xi, w = oq.gauss_legendre(Q)
        xl, wl = np.polynomial.legendre.leggauss(Q)
        assert np.max(np.abs(xi - xl)) < 1e-13
        assert np.max(np.abs(w - wl)) < 1e-13


def test_laguerre_table_I():
    g = load_golden()
    pb, w = oq.gauss_laguerre2(2)
    assert pb[0] == pytest.approx(g["laguerre_Q2_node_1"][0], abs=1e-15)
    assert pb[1] == pytest.approx(g["laguerre_Q2_node_2"][0], abs=1e-14)
    assert w[0] == pytest.approx(g["laguerre_Q2_weight_1"][0], abs=1e-15)
    assert w[1] == pytest.approx(g["laguerre_Q2_weight_2"][0], abs=1e-15)


@pytest.mark.parametrize("QL", [2, 3, 4, 5])
def test_laguerre_exactness(QL):
    """sum_k w_k x_k^s = (s+2)! for s <= 2 Q_L - 1 (eq. quadL)."""
    pb, w = oq.gauss_laguerre2(QL)
    for s in range(2 * QL):
        assert np.sum(w * pb ** s) == pytest.approx(factorial(s + 2), rel=1e-13)
    assert abs(np.sum(w * pb ** (2 * QL)) / factorial(2 * QL + 2) - 1.0) > 1e-10


def test_laguerre_explicit_polynomials():
    # L_0 = 1, L_1 = 3 - x, L_2 = 6 - 4x + x^2/2 (the equation printed before Table I)
    x = np.linspace(0, 10, 7)
    assert np.allclose(oq.laguerre2_explicit(0, x), 1.0)
    assert np.allclose(oq.laguerre2_explicit(1, x), 3.0 - x)
    assert np.allclose(oq.laguerre2_explicit(2, x), 6.0 - 4.0 * x + 0.5 * x ** 2)
    # orthogonality, eq. lag_ortho: int e^{-x} x^2 L_l L_l' = (l+1)(l+2) delta
    pb, w = oq.gauss_laguerre2(6)
    for l in range(4):
        for lp in range(4):
            val = np.sum(w * oq.laguerre2_explicit(l, pb) * oq.laguerre2_explicit(lp, pb))
            assert val == pytest.approx((l + 1) * (l + 2) if l == lp else 0.0, abs=1e-11)


@pytest.mark.parametrize("QL", [2, 3, 4])
def test_KL_identities(QL):
    K = oq.kernel_KL(QL)
    pb, w = oq.gauss_laguerre2(QL)
    # particle number: sum_k K_{kk'} = 0
    assert np.max(np.abs(K.sum(axis=0))) < 4e-15 * np.max(np.abs(K))
    # energy: sum_k pb_k K_{kk'} = -pb_k'  (drives d(tau T^tautau)/dtau = -T^etaeta)
    assert np.max(np.abs(pb @ K + pb)) < 4e-15 * np.max(np.abs(K)) * pb.max()
    # f(p) = e^{-p}: p^-2 d(p^3 e^{-p})/dp = (3 - p) e^{-p}; in f_jk scaling f_k = w_k
    assert np.max(np.abs(K @ w - w * (3.0 - pb))) < 4e-15 * np.max(np.abs(K)) * pb.max()


def test_KL_Q2_closed_form():
    K = oq.kernel_KL(2)
    pb, w = oq.gauss_laguerre2(2)
    ref = np.outer(w * (3.0 - pb), pb) / 6.0           # eq. K_lag_disc1
    assert np.max(np.abs(K - ref)) < 1e-15


@pytest.mark.parametrize("Q", [3, 8, 20, 40, 101, 200])
def test_KP_identities(Q):
    K = oq.kernel_KP(Q)
    xi, w = oq.gauss_legendre(Q)
    # particle number conservation: column sums vanish
    assert np.max(np.abs(K.sum(axis=0))) < 1e-12 * Q
    # f(xi) = xi^a: d/dxi[xi (1 - xi^2) xi^a] = (a+1) xi^a - (a+3) xi^{a+2}
    for a in range(0, Q - 2):
        f = w * xi ** a
        ref = w * ((a + 1) * xi ** a - (a + 3) * xi ** (a + 2))
        err = np.max(np.abs(K @ f - ref))
        assert err < 5e-14 * max(1, Q / 8) * (1 + a), (Q, a, err)
    # parity: the operator commutes with xi -> -xi
    R = np.eye(Q)[::-1]
    assert np.max(np.abs(R @ K @ R - K)) < 1e-12 * Q


def test_KP_dense_not_banded():
    """K^P couples every node to every node (it is the dense projection)."""
    K = oq.kernel_KP(12)
    assert np.count_nonzero(np.abs(K) > 1e-12) > 0.5 * K.size
