"""GPU parity of the implicit-explicit step (rsl_step_imex) against the
oracle's IMEX-SSP2(2,2,2) step (oracle/imex.py): WENO5 advection explicit,
the Anderson-Witting term implicit, each implicit stage solved per cell.
Sec. I (a time step not bound by tau_AW), Sec. III F, Sec. IV B 2.

Bar: max |f_gpu - f_oracle| / max |f_oracle| <= 1e-12 (binary64 storage).
Cases: several blocks with a ragged tail and a single short block, 4 to 64
lanes per cell and two angular nodes per lane, both ghost rules, the three relaxation-time laws, an odd Q_xi (a node at
xi = 0), moving off-equilibrium states, and dt / tau_AW from 0.06 to 4e4."""
import numpy as np
import pytest
import torch

import oracle
from oracle import imex, riemann
from tests import inputs

pytestmark = pytest.mark.gpu

TAU = {"const": oracle.TAU_CONST, "etas": oracle.TAU_ETAS, "inf": oracle.TAU_INF}


@pytest.fixture(scope="module")
def rsl():
    from paper_1612_01287_amd import rsl as mod
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return mod


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _pair(rsl, QL, Q, NOm, nz, bc, tau_mode, tau_r, tau_aw0, states):
    quad = rsl.Quadrature(QL, Q, NOm)
    p = rsl.make_problem(nz=nz, bc=bc, tau_mode=tau_mode, tau_r=tau_r, tau_aw0=tau_aw0, **states)
    inst = rsl.Instance(quad, p)
    vs = oracle.VelocitySet(QL, Q, NOm)
    T = imex.ImexSod(vs, nz, tau_mode=TAU[tau_mode], tau_r=tau_r, tau_aw0=tau_aw0, lambda_ref=1.0,
                     bc=oracle.BC_OUTFLOW if bc == "outflow" else oracle.BC_EQ, **states)
    return quad, inst, vs, T


CASES = [
    # QL, Q, NOm, nz, bc, tau law, tau_r, tau_aw0, dt dz^-1, steps, start
    (3, 8, 4, 150, "eq", "const", 1e-3, 0.0, 0.5, 4, "sod"),          # dt / tau = 3.3
    (3, 8, 4, 130, "eq", "const", 1e-7, 0.0, 0.5, 4, "sod"),          # dt / tau = 3.8e4
    (3, 8, 3, 5, "outflow", "const", 1e-2, 0.0, 0.5, 3, "sod"),       # one short block
    (2, 9, 3, 203, "outflow", "etas", 0.0, 0.03, 0.4, 3, "moving"),   # xi = 0 node
    (3, 16, 5, 64, "outflow", "const", 0.05, 0.0, 0.9, 3, "moving"),  # dt / tau = 0.28
    (2, 6, 2, 70, "eq", "inf", 0.0, 0.0, 0.5, 3, "moving"),           # collisionless
    (3, 20, 5, 97, "eq", "const", 1e-4, 0.0, 0.5, 3, "sod"),          # 32 lanes per cell
    (2, 100, 4, 70, "outflow", "const", 0.01, 0.0, 0.5, 2, "moving"), # two nodes per lane
    (2, 200, 4, 20, "eq", "const", 1e-5, 0.0, 0.5, 2, "sod"),         # four nodes per lane
]


@pytest.mark.parametrize("QL,Q,NOm,nz,bc,law,tau_r,tau_aw0,cfl,steps,start", CASES)
def test_imex_matches_oracle(rsl, QL, Q, NOm, nz, bc, law, tau_r, tau_aw0, cfl, steps, start):
    states = inputs.SOD_PAPER if start == "sod" else inputs.SOD_C1
    quad, inst, vs, T = _pair(rsl, QL, Q, NOm, nz, bc, law, tau_r, tau_aw0, states)
    inst.init()                                   # ghost states and status word
    f0 = T.init()
    if start == "moving":
        z = -0.5 + (np.arange(nz) + 0.5) / nz
        beta = 0.4 * np.sin(2.0 * np.pi * z)
        f0 = np.stack([oracle.feq(vs, 1.0 + 0.3 * np.cos(np.pi * z[s]), 0.9 + 0.2 * z[s] ** 2, beta[s])
                       for s in range(nz)], axis=1)
        f0 = f0 * inputs.smooth_perturbation(vs.V, nz, seed=nz, amp=0.2)
    inst.set_f(f0)
    dt = cfl / (nz * np.max(np.abs(vs.xi)))
    f = f0
    for k in range(steps):                        # each step against the oracle's step of the same state
        inst.step_imex(dt, 1)
        got = inst.f().cpu().numpy()
        want = T.step(f, dt)
        assert _rel(got, want) < 1e-12, k
        f = got
    assert inst.status() == 0
    assert inst.t == pytest.approx(steps * dt, rel=1e-15)


def test_imex_keeps_a_uniform_equilibrium(rsl):
    st = dict(nL=0.7, TL=1.2, nR=0.7, TR=1.2)
    quad, inst, vs, T = _pair(rsl, 3, 8, 4, 100, "outflow", "const", 1e-4, 0.0, st)
    inst.init()
    f0 = inst.f().cpu().numpy()
    inst.step_imex(0.5 / 100, 5)
    assert np.max(np.abs(inst.f().cpu().numpy() - f0)) < 1e-14 * np.max(np.abs(f0))


def test_imex_near_inviscid_plateau_at_size(rsl):
    """The stiff tube the benchmark times (N_z = 4096, R-SLB(4;8), Q_L = 3,
    tau_r = 1e-7, dt = 0.5 dz: dt / tau = 1.2e3) to t = 0.4: the plateau
    between contact and shock at the exact Riemann pressure and velocity
    (Sec. IV B 2), the particle number kept (the waves have not reached the
    ghosts), and sampled cells of one more step against the oracle's step of
    the same state (the step of a cell needs only its 7-cell neighbourhood)."""
    nz = 4096
    quad, inst, vs, T = _pair(rsl, 3, 8, 4, nz, "eq", "const", 1e-7, 0.0, inputs.SOD_PAPER)
    inst.init()
    dt = 0.5 / nz
    n0 = inst.moments().cpu().numpy()[:, 0].sum()
    inst.step_imex(dt, int(round(0.4 / dt)))
    assert inst.status() == 0
    M = inst.moments().cpu().numpy()
    assert np.all(np.isfinite(M))
    assert abs(M[:, 0].sum() - n0) < 1e-11 * n0
    st = riemann.riemann_star(1.0, 1.0, 0.125, 0.0625)
    z = -0.5 + (np.arange(nz) + 0.5) / nz
    t = inst.t
    plateau = (z > st["beta_C"] * t + 0.01) & (z < st["beta_shock"] * t - 0.01)
    assert plateau.sum() > 100
    assert np.mean(M[plateau, 7]) == pytest.approx(st["PC"], rel=2e-3)
    assert np.mean(M[plateau, 9]) == pytest.approx(st["beta_C"], rel=2e-3)
    # sampled cells of one more step: the oracle steps a 20-cell window around each
    f = inst.f().cpu().numpy()
    inst.step_imex(dt, 1)
    g = inst.f().cpu().numpy()
    for c in inputs.rng(5).choice(np.arange(20, nz - 20), 12, replace=False):
        W = imex.ImexSod(vs, 41, zlo=0.0, zhi=41.0 / nz, tau_mode=oracle.TAU_CONST, tau_r=1e-7,
                         bc=oracle.BC_OUTFLOW, **inputs.SOD_PAPER)      # the tube's dz
        want = W.step(f[:, c - 20:c + 21], dt)[:, 20]     # cell c, 20 cells from either window edge
        assert _rel(g[:, c], want) < 1e-12, c


def test_imex_argument_errors(rsl):
    q = rsl.Quadrature(3, 8, 4)
    bj = rsl.Instance(rsl.Quadrature(3, 20, 2), rsl.make_problem(kind="bjorken", tau_mode="const", tau_r=0.3))
    with pytest.raises(rsl.RslError) as e:
        bj.step_imex(0.01, 1)
    assert e.value.code == rsl.RSL_EUNSUPPORTED
    inst = rsl.Instance(q, rsl.make_problem(nz=16))
    inst.init()
    with pytest.raises(rsl.RslError) as e:                      # dt max|xi| / dz >= 1
        inst.step_imex(1.1 / 16, 1)
    assert e.value.code == rsl.RSL_EUNSTABLE
    with pytest.raises(rsl.RslError) as e:
        inst.step_imex(0.01, -1)
    assert e.value.code == rsl.RSL_EINVAL
    f0 = inst.f().cpu().numpy()
    inst.step_imex(0.01, 0)
    assert inst.t == 0.0 and np.array_equal(inst.f().cpu().numpy(), f0)


def test_imex_c1_tube_without_the_guard(rsl):
    """The near-inviscid tube C1 (N_z = 400, R-SLB(3;8), tau_r = 1e-3,
    dt = 1.25e-3 > tau_r) with no stiffness guard or override: the first three
    steps against the oracle's, then 200 steps (t = 0.25) keeping N^0 and
    T^00 to 1e-12 and within the schemes' truncation difference of the
    explicit RK3 run (the oracle's two solvers differ there by 0.47 % in N^0,
    0.49 % in T^00, 0.61 % in P at most)."""
    nz, dt = 400, 1.25e-3
    quad, inst, vs, T = _pair(rsl, 3, 8, 3, nz, "outflow", "const", 1e-3, 0.0, inputs.SOD_C1)
    inst.init()
    f = T.init()
    n0 = inst.moments().cpu().numpy()[:, [0, 2]].sum(axis=0)
    for k in range(3):
        inst.step_imex(dt, 1)
        got = inst.f().cpu().numpy()
        assert _rel(got, T.step(f, dt)) < 1e-12, k
        f = got
    inst.step_imex(dt, 197)
    assert inst.status() == 0
    Mi = inst.moments().cpu().numpy()
    assert np.allclose(Mi[:, [0, 2]].sum(axis=0), n0, rtol=1e-12, atol=0)
    ex = rsl.Instance(quad, rsl.make_problem(nz=nz, tau_r=1e-3, **inputs.SOD_C1))
    ex.init()
    ex.step(dt, 200)
    Me = ex.moments().cpu().numpy()
    for c, tol in ((0, 0.01), (2, 0.01), (7, 0.0125)):
        assert np.max(np.abs(Mi[:, c] - Me[:, c])) < tol * np.max(np.abs(Me[:, c])), c


@pytest.mark.parametrize("QL,Q,NOm,nz,bc,law,tau_r,cfl,start", [
    (3, 8, 4, 150, "eq", "const", 1e-3, 0.5, "sod"),
    (3, 16, 4, 203, "outflow", "const", 1e-6, 0.5, "moving"),
    (2, 100, 4, 70, "outflow", "const", 0.01, 0.5, "moving"),
])
def test_imex_binary32_matches_oracle(rsl, QL, Q, NOm, nz, bc, law, tau_r, cfl, start):
    """Binary32 storage: the oracle rounds f and the stored stages F1, F2*,
    F2 to binary32 where the kernels store them; bar 1e-5 per step."""
    states = inputs.SOD_PAPER if start == "sod" else inputs.SOD_C1
    quad = rsl.Quadrature(QL, Q, NOm)
    inst = rsl.Instance(quad, rsl.make_problem(nz=nz, dtype="f32", bc=bc, tau_mode=law, tau_r=tau_r, **states))
    vs = oracle.VelocitySet(QL, Q, NOm)
    T = imex.ImexSod(vs, nz, store_f32=True, tau_mode=TAU[law], tau_r=tau_r,
                     bc=oracle.BC_OUTFLOW if bc == "outflow" else oracle.BC_EQ, **states)
    inst.init()
    f = T.init()
    if start == "moving":
        z = -0.5 + (np.arange(nz) + 0.5) / nz
        f = np.stack([oracle.feq(vs, 1.0 + 0.3 * np.cos(np.pi * z[s]), 0.9 + 0.2 * z[s] ** 2,
                                 0.4 * np.sin(2.0 * np.pi * z[s])) for s in range(nz)], axis=1)
        f = (f * inputs.smooth_perturbation(vs.V, nz, seed=nz, amp=0.2)).astype(np.float32).astype(np.float64)
        inst.set_f(f)
    dt = cfl / (nz * np.max(np.abs(vs.xi)))
    for k in range(3):
        inst.step_imex(dt, 1)
        got = inst.f().double().cpu().numpy()
        assert _rel(got, T.step(f, dt)) < 1e-5, k
        f = got
    assert inst.status() == 0


BATCH = [  # QL, Q, NOm, nz, bc, tau_r, dtype
    (3, 8, 4, 150, "eq", 1e-7, "f64"),
    (3, 16, 4, 70, "outflow", 1e-3, "f64"),
    (2, 3, 2, 5, "outflow", 0.05, "f64"),
    (3, 20, 5, 97, "eq", 1e-4, "f64"),
    (2, 100, 4, 64, "outflow", 0.01, "f64"),
    (3, 64, 4, 203, "outflow", 1e-5, "f64"),
    (2, 200, 4, 20, "eq", 1e-3, "f64"),
]


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_batch_imex_matches_oracle(rsl, dtype, tol):
    """An uneven batch (6 velocity-set classes, ragged tails, a 5-cell tube,
    dt / tau up to 3e4) created with RSL_FLAG_IMEX at dt = 0.5 dz for every
    instance: each instance after two batch steps against two oracle steps,
    and against the single-instance call."""
    quads, probs, dts, pairs = [], [], [], []
    for QL, Q, NOm, nz, bc, tau_r, _ in BATCH:
        q = rsl.Quadrature(QL, Q, NOm)
        quads.append(q)
        probs.append(rsl.make_problem(nz=nz, dtype=dtype, bc=bc, tau_r=tau_r, imex=True, **inputs.SOD_PAPER))
        dts.append(0.5 / nz)
        vs = oracle.VelocitySet(QL, Q, NOm)
        pairs.append(imex.ImexSod(vs, nz, store_f32=(dtype == "f32"), tau_mode=oracle.TAU_CONST, tau_r=tau_r,
                                  bc=oracle.BC_OUTFLOW if bc == "outflow" else oracle.BC_EQ, **inputs.SOD_PAPER))
    B = rsl.Batch(quads, probs, dts)
    B.init()
    B.step_imex(2)
    for i, T in enumerate(pairs):
        got = B.f(i).double().cpu().numpy()
        want = T.run(T.init(), dts[i], 2)
        assert _rel(got, want) < tol, i
        single = rsl.Instance(quads[i], probs[i])
        single.init()
        single.step_imex(dts[i], 2)
        assert _rel(got, single.f().double().cpu().numpy()) < 1e-14, i
    assert B.status()[0] == 0


def test_batch_imex_refuses_explicit_steps_and_checks_cfl(rsl):
    q = rsl.Quadrature(3, 8, 4)
    p = rsl.make_problem(nz=64, tau_r=1e-6, imex=True)
    B = rsl.Batch([q], [p], [0.5 / 64])
    B.init()
    for call in (lambda: B.step(1), lambda: B.stage(1)):
        with pytest.raises(rsl.RslError) as e:
            call()
        assert e.value.code == rsl.RSL_EUNSTABLE
    with pytest.raises(rsl.RslError) as e:                      # CFL still applies
        rsl.Batch([q], [p], [1.1 / 64])
    assert e.value.code == rsl.RSL_EUNSTABLE
    with pytest.raises(rsl.RslError) as e:                      # without the flag the guard applies
        rsl.Batch([q], [rsl.make_problem(nz=64, tau_r=1e-6)], [0.5 / 64])
    assert e.value.code == rsl.RSL_EUNSTABLE
    bj = rsl.Batch([rsl.Quadrature(3, 20, 2)], [rsl.make_problem(kind="bjorken", tau_mode="const", tau_r=0.3)],
                   [1e-3])
    with pytest.raises(rsl.RslError) as e:
        bj.step_imex(1)
    assert e.value.code == rsl.RSL_EUNSUPPORTED


def test_batch_imex_full_ensemble_sampled(rsl):
    """The benchmark's 1024-instance binary32 ensemble created with
    RSL_FLAG_IMEX at dt = 0.5/N_z for every instance, in the launch form the
    benchmark times: 30 steps with no unphysical or non-finite cell, then
    sampled cells of one more step against the oracle's binary32-storage step
    of a 41-cell window of the tube (a cell's step needs 6 cells either side)."""
    import bench
    params = bench.ensemble_params()
    B, quads, probs = bench.ensemble_batch(rsl, params, imex=True)
    B.init()
    B.step_imex(30)
    assert all(s == 0 for s in B.instance_status())
    rng = inputs.rng(11)
    picks = [int(i) for i in rng.choice(len(params), 6, replace=False)]
    before = {i: B.f(i).double().cpu().numpy() for i in picks}
    B.step_imex(1)
    for i in picks:
        nz, Q, TR, tau, _ = params[i]
        vs = oracle.VelocitySet(3, Q, min(Q - 1, 4))
        W = imex.ImexSod(vs, 41, store_f32=True, zlo=0.0, zhi=41.0 / nz, nL=1.0, TL=1.0, nR=TR ** 3, TR=TR,
                         tau_mode=oracle.TAU_CONST, tau_r=tau, bc=oracle.BC_OUTFLOW)
        got = B.f(i).double().cpu().numpy()
        for c in (nz // 2, int(rng.integers(20, nz - 20))):       # the membrane and a random cell
            want = W.step(before[i][:, c - 20:c + 21], 0.5 / nz)[:, 20]
            assert _rel(got[:, c], want) < 1e-5, (i, c)


def test_imex_second_order_at_size(rsl):
    """A smooth off-equilibrium state on N_z = 1024 (tau_r = 0.02): the GPU's
    IMEX solution at t = 0.05 against the GPU's explicit RK3 with dt / 16;
    halving dt divides the error by about four (the scheme's second order, a
    property of any size)."""
    nz = 1024
    quad = rsl.Quadrature(3, 8, 4)
    vs = oracle.VelocitySet(3, 8, 4)
    z = -0.5 + (np.arange(nz) + 0.5) / nz
    bump = np.exp(-(z / 0.15) ** 2)
    f0 = np.stack([oracle.feq(vs, 1.0 + 0.2 * b, 1.0 + 0.1 * b, 0.2 * b) for b in bump], axis=1)
    f0 *= 1.0 + 0.05 * np.outer(np.tile(vs.xi, vs.QL), bump)
    p = rsl.make_problem(nz=nz, tau_r=0.02, nL=1.0, TL=1.0, nR=1.0, TR=1.0)
    dt0 = 0.5 / nz
    ref = rsl.Instance(quad, p)
    ref.init()
    ref.set_f(f0)
    ref.step(dt0 / 16, 100 * 16)
    want = ref.f().cpu().numpy()
    errs = []
    for r in (1, 2, 4):
        inst = rsl.Instance(quad, p)
        inst.init()
        inst.set_f(f0)
        inst.step_imex(dt0 / r, 100 * r)
        errs.append(np.max(np.abs(inst.f().cpu().numpy() - want)))
    p1, p2 = np.log2(errs[0] / errs[1]), np.log2(errs[1] / errs[2])
    assert 1.7 < p1 < 2.5 and 1.7 < p2 < 2.5, (errs, p1, p2)


@pytest.mark.parametrize("tau_r,bc", [(1e-7, "eq"), (2e-3, "outflow")])
def test_imex_steps_in_one_call_match_single_steps(rsl, tau_r, bc):
    """Within one call the implicit solves start from each cell's previous
    Jacobian; the first solve of a call starts from finite differences.  The
    converged stages are the same: eight steps in one call against eight
    calls of one step, and against the oracle's eight steps."""
    nz = 150
    quad, inst, vs, T = _pair(rsl, 3, 8, 4, nz, bc, "const", tau_r, 0.0, inputs.SOD_PAPER)
    one = rsl.Instance(quad, inst.p)
    inst.init()
    one.init()
    dt = 0.5 / nz
    inst.step_imex(dt, 8)
    for _ in range(8):
        one.step_imex(dt, 1)
    a, b = inst.f().cpu().numpy(), one.f().cpu().numpy()
    assert _rel(a, b) < 1e-12
    assert _rel(a, T.run(T.init(), dt, 8)) < 1e-11


def test_explicit_and_imex_steps_alternate(rsl):
    """rsl_step and rsl_step_imex share the work buffer's per-cell rows (the
    explicit stages' coefficients, the implicit solves' carried Jacobians);
    each call sets the rows it reads, so the two alternate freely: explicit,
    IMEX and explicit steps against the oracle's same sequence."""
    nz = 130
    quad, inst, vs, T = _pair(rsl, 3, 8, 4, nz, "outflow", "const", 0.05, 0.0, inputs.SOD_C1)
    S = oracle.Sod(vs, nz, tau_mode=oracle.TAU_CONST, tau_r=0.05, bc=oracle.BC_OUTFLOW, **inputs.SOD_C1)
    inst.init()
    dt = 0.5 / nz
    f = S.init()
    for kind in ("rk3", "imex", "imex", "rk3", "imex"):
        if kind == "rk3":
            inst.step(dt, 2)
            f = S.run(f, dt, 2)
        else:
            inst.step_imex(dt, 2)
            f = T.run(f, dt, 2)
        assert _rel(inst.f().cpu().numpy(), f) < 1e-11, kind
