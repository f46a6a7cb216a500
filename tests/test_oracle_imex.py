"""Pins of the oracle's IMEX step (oracle/imex.py): the implicit stage against
its defining equation and the moments the collision conserves, a uniform
equilibrium kept, the near-inviscid tube at dt >> tau_AW against the exact
Riemann plateau (Sec. IV B 2; the explicit RK3 diverges there), and second
order in dt against a fine explicit RK3 reference, and the collisionless law
reducing the scheme to Heun's method on the advection."""
import numpy as np
import pytest

import oracle
from oracle import imex, riemann
from tests import inputs


def test_implicit_stage_solves_its_equation_and_conserves():
    vs = oracle.VelocitySet(3, 8, 4)
    S = oracle.Sod(vs, 12, tau_mode=oracle.TAU_CONST, tau_r=1e-3)
    rng = inputs.rng(2)
    F = np.stack([oracle.feq(vs, 1.0, 1.0, b) for b in np.linspace(-0.5, 0.5, 12)], axis=1)
    F *= 1.0 + 0.1 * rng.uniform(-1.0, 1.0, F.shape)
    for h in (1e-5, 1e-3, 0.1):
        G = imex.implicit_stage(S, F, h)
        res = G - F - h * imex.collision(S, G)
        assert np.max(np.abs(res)) < 1e-12 * np.max(np.abs(F))
        _, _, R = imex._rows(vs)
        d = R @ G - R @ F
        assert np.max(np.abs(d[[0, 2, 3]])) < 1e-13 * np.max(np.abs(R @ F))
    # stiff: G is the equilibrium with F's N^0, T^00, T^0z (|G - f^eq(G)| = tau |Q(G)| / (gamma (1 - beta xi)))
    G = imex.implicit_stage(S, F, 1e6)
    assert np.max(np.abs(imex.collision(S, G))) * 1e-3 < 1e-9 * np.max(np.abs(G))


def test_imex_keeps_a_uniform_equilibrium():
    vs = oracle.VelocitySet(3, 8, 4)
    T = imex.ImexSod(vs, 20, nL=0.7, TL=1.2, nR=0.7, TR=1.2, tau_mode=oracle.TAU_CONST, tau_r=1e-4,
                     bc=oracle.BC_OUTFLOW)
    f0 = T.init()
    f1 = T.run(f0, 0.5 / 20, 3)
    assert np.max(np.abs(f1 - f0)) < 1e-14 * np.max(np.abs(f0))


def test_imex_near_inviscid_tube_at_dt_far_above_tau():
    """tau_r = 1e-7 with dt = 0.5 dz = 5e-3: dt/tau = 5e4.  The plateau
    between contact and shock carries the exact Riemann pressure and velocity
    (Sec. IV B 2) to the accuracy of the grid."""
    nz, t_end = 100, 0.4
    vs = oracle.VelocitySet(3, 8, 4)
    T = imex.ImexSod(vs, nz, nL=1.0, TL=1.0, nR=0.125, TR=0.5, tau_mode=oracle.TAU_CONST, tau_r=1e-7,
                     bc=oracle.BC_EQ)
    dt = 0.5 / nz
    f = T.run(T.init(), dt, int(round(t_end / dt)))
    M = T.moments(f)
    st = riemann.riemann_star(1.0, 1.0, 0.125, 0.0625)
    z = -0.5 + (np.arange(nz) + 0.5) / nz
    plateau = (z > (st["beta_C"] * t_end + 0.02)) & (z < (st["beta_shock"] * t_end - 0.02))
    assert plateau.sum() >= 5
    P, beta = M[plateau, 7], M[plateau, 9]
    assert np.mean(P) == pytest.approx(st["PC"], rel=0.02)
    assert np.mean(beta) == pytest.approx(st["beta_C"], rel=0.03)
    assert np.all(np.isfinite(M))


def test_imex_second_order_in_dt():
    """A smooth, collisional state (tau = 0.02): the IMEX solution at t = 0.1
    against explicit RK3 with dt / 16 on the same grid; halving dt divides the
    error by ~4."""
    nz = 64
    vs = oracle.VelocitySet(3, 8, 4)
    kw = dict(nL=1.0, TL=1.0, nR=1.0, TR=1.0, tau_mode=oracle.TAU_CONST, tau_r=0.02, bc=oracle.BC_OUTFLOW)
    T = imex.ImexSod(vs, nz, **kw)
    z = -0.5 + (np.arange(nz) + 0.5) / nz
    bump = np.exp(-(z / 0.15) ** 2)
    f0 = np.stack([oracle.feq(vs, 1.0 + 0.2 * b, 1.0 + 0.1 * b, 0.2 * b) for b in bump], axis=1)
    f0 *= 1.0 + 0.05 * np.outer(np.tile(vs.xi, vs.QL), bump)        # off equilibrium
    t_end, dt0 = 0.1, 0.1 / 8
    ref = oracle.Sod(vs, nz, **kw).run(f0, dt0 / 16, 8 * 16)
    errs = []
    for r in (1, 2, 4):
        f = T.run(f0, dt0 / r, 8 * r)
        errs.append(np.max(np.abs(f - ref)))
    p1, p2 = np.log2(errs[0] / errs[1]), np.log2(errs[1] / errs[2])
    assert 1.7 < p1 < 2.5 and 1.7 < p2 < 2.5, (errs, p1, p2)


def test_collisionless_imex_is_heun_on_the_advection():
    """tau_AW -> infinity: Q = 0, so F1 = f, F2 = f + dt A(f) and the step is
    the SSP Heun method f + dt/2 (A(f) + A(f + dt A(f))) on the oracle's
    collisionless L."""
    nz = 40
    vs = oracle.VelocitySet(2, 6, 2)
    kw = dict(nL=1.0, TL=1.0, nR=0.4, TR=0.8, tau_mode=oracle.TAU_INF, bc=oracle.BC_EQ)
    T = imex.ImexSod(vs, nz, **kw)
    A = oracle.Sod(vs, nz, **kw)
    f = T.init() * inputs.smooth_perturbation(vs.V, nz, seed=3, amp=0.2)
    dt = 0.5 / nz
    a1 = A.L(f)
    want = f + 0.5 * dt * (a1 + A.L(f + dt * a1))
    got = T.step(f, dt)
    assert np.max(np.abs(got - want)) < 1e-14 * np.max(np.abs(want))


def test_binary32_storage_rounds_only_what_is_stored():
    """store_f32: every stored value is a binary32 number, the step stays
    within binary32 rounding of the binary64 step from the same (rounded)
    state, and the unrounded mode is untouched by the option."""
    nz = 30
    vs = oracle.VelocitySet(3, 8, 4)
    kw = dict(nL=1.0, TL=1.0, nR=0.4, TR=0.8, tau_mode=oracle.TAU_CONST, tau_r=1e-3, bc=oracle.BC_OUTFLOW)
    T32 = imex.ImexSod(vs, nz, store_f32=True, **kw)
    T64 = imex.ImexSod(vs, nz, **kw)
    f = T32.init() * inputs.smooth_perturbation(vs.V, nz, seed=9, amp=0.1)
    f = f.astype(np.float32).astype(np.float64)
    g32, g64 = T32.step(f, 0.5 / nz), T64.step(f, 0.5 / nz)
    assert np.array_equal(g32, g32.astype(np.float32).astype(np.float64))
    assert 0.0 < np.max(np.abs(g32 - g64)) < 1e-6 * np.max(np.abs(g64))
    assert np.array_equal(T64.init(), oracle.Sod(vs, nz, **kw).init())
