"""Pins of the oracle's WENO5 flux (Sec. III F, eqs. flux_weno, weno5_omega).

* a constant state is reproduced exactly (limiting case (i));
* any stencil with a vanishing smoothness indicator returns the upwind value
  (cases (ii), (iii): a zero indicator means a constant 3-point stencil, and
  all candidate stencils share the upwind cell);
* on smooth monotone data the weights approach the ideal ones and the flux is
  the fifth-order upwind reconstruction: convergence order ~5 on cell averages;
* at a discontinuity the flux uses the smooth side only (no overshoot).
"""
import numpy as np
import pytest

import oracle


def test_constant_state():
    for c in (0.0, 1.0, -3.7, 1e-300, 7.25e10):
        assert oracle.weno5(c, c, c, c, c) == pytest.approx(c, rel=4e-16, abs=0)


@pytest.mark.parametrize("vals", [
    (1.0, 1.0, 1.0, 2.0, 5.0),      # stencil 1 constant -> case (iii)
    (3.0, 1.0, 1.0, 1.0, 4.0),      # stencil 2 constant -> case (iii)
    (3.0, 0.5, 1.0, 1.0, 1.0),      # stencil 3 constant -> case (iii)
    (1.0, 1.0, 1.0, 1.0, 4.0),      # stencils 1, 2 constant -> case (ii)
    (2.0, 1.0, 1.0, 1.0, 1.0),      # stencils 2, 3 constant -> case (ii)
])
def test_limiting_cases_return_upwind_value(vals):
    assert oracle.weno5(*vals) == pytest.approx(vals[2], abs=1e-15)


def test_ideal_weights_on_polynomial_data():
    """Cell averages of a quadratic have equal smoothness indicators of the
    first-difference part; for data with sigma_1 = sigma_2 = sigma_3 the flux is
    the ideal-weight (fifth-order) combination (2a - 13b + 47c + 27d - 3e)/60."""
    a, b, c, d, e = (1.0, 2.0, 3.0, 4.0, 5.0)          # linear data: all sigma equal
    lin = (2 * a - 13 * b + 47 * c + 27 * d - 3 * e) / 60.0
    assert oracle.weno5(a, b, c, d, e) == pytest.approx(lin, abs=1e-14)
    assert lin == pytest.approx(3.5, abs=1e-14)         # exact interface value


def _cell_avg_exp(z0, dz, k):
    # cell averages of exp(k z) over [z0 - dz/2, z0 + dz/2]
    return np.exp(k * z0) * (np.exp(k * dz / 2) - np.exp(-k * dz / 2)) / (k * dz)


def test_fifth_order_convergence():
    errs = []
    for N in (20, 40, 80):
        dz = 1.0 / N
        zc = (np.arange(-3, N + 3) + 0.5) * dz
        J = _cell_avg_exp(zc, dz, 1.3)
        err = 0.0
        for s in range(3, N + 3 - 3):
            F = oracle.weno5(J[s - 2], J[s - 1], J[s], J[s + 1], J[s + 2])
            exact = np.exp(1.3 * (zc[s] + dz / 2))
            err = max(err, abs(F - exact))
        errs.append(err)
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 4.6), orders


def test_discontinuity_non_oscillatory():
    # upwind side smooth (constant 1), jump to 0 downwind: flux stays in [0, 1]
    F = oracle.weno5(1.0, 1.0, 1.0, 0.0, 0.0)
    assert F == pytest.approx(1.0, abs=1e-15)
    F = oracle.weno5(1.0, 1.0, 0.0, 0.0, 0.0)
    assert 0.0 <= F <= 1.0
