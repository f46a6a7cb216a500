"""GPU parity of the Sod step (librsl through its C ABI) against the oracle.

Bar: max |f_gpu - f_oracle| / max |f_oracle| <= 1e-12 with f stored in FP64,
<= 1e-5 with f stored in FP32 (the oracle then rounds f to binary32 after each
RK stage as the kernels do).  Cases cover several tiles and a ragged last tile,
both ghost-cell rules, the three relaxation-time laws, odd Q_xi (a node at
xi = 0), velocity sets too large for the LDS window, moving states, the
full C2 size (N_z = 4096, R-SLB(4;100), Q_L = 3), and the whole 16-instance
sweep at that size in the launch configuration the benchmark times.
"""
import numpy as np
import pytest
import torch

import oracle
from tests import inputs

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


@pytest.fixture(scope="module")
def rsl():
    from paper_1612_01287_amd import rsl as mod
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return mod


def _pair(rsl, QL, Q, NOm, nz, dtype="f64", bc="outflow", tau_mode="const", tau_r=1e-2, tau_aw0=0.0,
          states=inputs.SOD_C1):
    quad = rsl.Quadrature(QL, Q, NOm)
    p = rsl.make_problem(nz=nz, dtype=dtype, bc=bc, tau_mode=tau_mode, tau_r=tau_r, tau_aw0=tau_aw0,
                         **states)
    inst = rsl.Instance(quad, p)
    vs = oracle.VelocitySet(QL, Q, NOm)
    S = oracle.Sod(vs, nz, nL=states["nL"], TL=states["TL"], nR=states["nR"], TR=states["TR"],
                   tau_mode={"const": oracle.TAU_CONST, "etas": oracle.TAU_ETAS, "inf": oracle.TAU_INF}[tau_mode],
                   tau_r=tau_r, tau_aw0=tau_aw0, lambda_ref=1.0,
                   bc=oracle.BC_OUTFLOW if bc == "outflow" else oracle.BC_EQ, store_f32=(dtype == "f32"))
    return quad, inst, vs, S


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def test_init_and_moments(rsl):
    quad, inst, vs, S = _pair(rsl, 3, 8, 3, 400, bc="eq")
    inst.init()
    f = inst.f().cpu().numpy()
    f0 = S.init()
    assert _rel(f, f0) < 1e-15
    M = inst.moments().cpu().numpy()
    Mo = S.moments(f0)
    assert np.max(np.abs(M - Mo)) < 1e-14


@pytest.mark.parametrize("nz", [5, 63, 64, 130, 400])
@pytest.mark.parametrize("bc", ["outflow", "eq"])
def test_step_c1_family(rsl, nz, bc):
    """R-SLB(3;8), Q_L = 3 (C1's set) from the Sod initial state, 4 steps."""
    quad, inst, vs, S = _pair(rsl, 3, 8, 3, nz, bc=bc, tau_r=1e-3)
    inst.init()
    dt = 0.5 / max(nz, 400)
    inst.step(dt, 4)
    got = inst.f().cpu().numpy()
    ref = S.run(S.init(), dt, 4)
    assert _rel(got, ref) < TOL["f64"]
    assert inst.status() == 0


@pytest.mark.parametrize("tau_mode,tau_r,tau_aw0", [("const", 0.05, 0.0), ("etas", 0.0, 0.03), ("inf", 0.0, 0.0)])
@pytest.mark.parametrize("QL,Q,NOm", [(2, 6, 5), (3, 9, 4), (2, 16, 6), (3, 40, 4)])
def test_random_state(rsl, tau_mode, tau_r, tau_aw0, QL, Q, NOm):
    """Random smooth non-equilibrium state (moving cells) through 3 steps."""
    nz = 200
    quad, inst, vs, S = _pair(rsl, QL, Q, NOm, nz, tau_mode=tau_mode, tau_r=tau_r, tau_aw0=tau_aw0)
    base = S.init()
    f0 = base * inputs.smooth_perturbation(vs.V, nz, seed=11, amp=0.3)
    inst.set_f(f0)
    dt = 0.4 / nz
    inst.step(dt, 3)
    got = inst.f().cpu().numpy()
    ref = S.run(f0, dt, 3)
    assert _rel(got, ref) < TOL["f64"]


def _envelope(S, f0, dt, nsteps, seed=0, store_f32=False):
    """Spread of the oracle itself when its input is perturbed at the last bit:
    WENO5 without a regulariser (Sec. III F) amplifies rounding differences
    near the fronts, so long runs are compared against this envelope."""
    rng = np.random.default_rng(seed)
    eps = 6e-8 if store_f32 else 1.1e-16
    a = S.run(f0, dt, nsteps)
    b = S.run(f0 * (1 + eps * rng.standard_normal(f0.shape)), dt, nsteps)
    return a, float(np.max(np.abs(a - b)) / np.max(np.abs(a)))


def _trajectory_parity(inst, S, dt, nsteps, every, tol, dtype=np.float64):
    """Along the GPU trajectory, every `every` steps one GPU step is compared
    with one oracle step taken from the identical (GPU) state."""
    worst = 0.0
    for it in range(nsteps):
        if it % every == 0:
            x = inst.f().cpu().numpy().astype(np.float64)
            inst.step(dt, 1)
            y = inst.f().cpu().numpy().astype(np.float64)
            worst = max(worst, _rel(y, S.run(x, dt, 1)))
        else:
            inst.step(dt, 1)
    assert worst < tol, worst
    return worst


def test_c1_full_run(rsl):
    """C1: N_z = 400, R-SLB(3;8), Q_L = 3, tau_r = 1e-3, CFL 0.5, 200 steps, FP64.
    Every step of the GPU trajectory matches the oracle's step to 1e-12; the
    end state lies within the oracle's own last-bit sensitivity envelope."""
    quad, inst, vs, S = _pair(rsl, 3, 8, 3, 400, tau_r=1e-3)
    inst.init()
    dt = 0.5 / 400
    _trajectory_parity(inst, S, dt, 200, 1, TOL["f64"])
    got = inst.f().cpu().numpy()
    ref, env = _envelope(S, S.init(), dt, 200)
    assert _rel(got, ref) < 10 * max(env, TOL["f64"]), (_rel(got, ref), env)
    Mg = inst.moments().cpu().numpy()
    Mo = S.moments(ref)
    # conserved totals agree to rounding (no signal reached the boundary)
    for q in (0, 2):
        assert abs(Mg[:, q].sum() - Mo[:, q].sum()) < 1e-12 * abs(Mo[:, q].sum())


def test_large_velocity_set_without_lds_window(rsl):
    """V = 300 in FP64 does not fit the LDS window: stencil from global memory."""
    quad, inst, vs, S = _pair(rsl, 3, 100, 4, 300, tau_mode="etas", tau_aw0=0.3854 * 0.1)
    inst.init()
    dt = 0.5 / 300
    inst.step(dt, 3)
    assert _rel(inst.f().cpu().numpy(), S.run(S.init(), dt, 3)) < TOL["f64"]


@pytest.mark.parametrize("QL,Q", [(2, 150), (3, 107), (3, 128)])
def test_velocity_classes_above_256(rsl, QL, Q):
    """Velocity sets handled by the 32-lane kernel classes (V in (256, 384])."""
    quad, inst, vs, S = _pair(rsl, QL, Q, 4, 100, bc="eq", tau_mode="etas", tau_aw0=0.3854 * 0.1)
    inst.init()
    dt = 0.5 / 100
    inst.step(dt, 2)
    assert _rel(inst.f().cpu().numpy(), S.run(S.init(), dt, 2)) < TOL["f64"]


@pytest.mark.parametrize("QL,Q,nz,bc", [(3, 200, 150, "eq"), (4, 256, 64, "outflow"), (3, 129, 70, "eq")])
def test_velocity_sets_above_384(rsl, QL, Q, nz, bc):
    """Large velocity sets (V > 384) run in the two-kernel stage form."""
    quad, inst, vs, S = _pair(rsl, QL, Q, 4, nz, bc=bc, tau_mode="etas", tau_aw0=0.3854 * 0.1)
    inst.init()
    dt = 0.5 / nz
    inst.step(dt, 2)
    assert _rel(inst.f().cpu().numpy(), S.run(S.init(), dt, 2)) < TOL["f64"]


def test_c2_full_size(rsl):
    """C2 size: N_z = 4096, R-SLB(4;100), Q_L = 3, eta/s = 0.01, 2 steps."""
    quad, inst, vs, S = _pair(rsl, 3, 100, 4, 4096, tau_mode="etas", tau_aw0=0.3854 * 0.01)
    inst.init()
    dt = 0.5 / 4096
    inst.step(dt, 2)
    assert _rel(inst.f().cpu().numpy(), S.run(S.init(), dt, 2)) < TOL["f64"]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_sweep_full_size_as_one_class(rsl, dtype):
    """The sweep at full size in the launch configuration the benchmark times:
    16 instances (N_z = 4096, Q_xi in {8, 16, 40, 100}, eta/s in {0.01, 0.1,
    1, 10}) as one class in the loop form, 2 steps; the R-SLB(4;100) and
    R-SLB(3;8)-sized instances at eta/s = 0.01 and 10 against the oracle."""
    from tests.test_gpu_batch import _loop_variant
    nz, dt = 4096, 0.5 / 4096
    QXI, ETAS = (8, 16, 40, 100), (0.01, 0.1, 1.0, 10.0)
    quads, probs, keys = [], [], []
    for Q in QXI:
        q = rsl.Quadrature(3, Q, 4)
        for es in ETAS:
            quads.append(q)
            probs.append(rsl.make_problem(nz=nz, dtype=dtype, bc="outflow", tau_mode="etas", tau_aw0=0.3854 * es,
                                          **inputs.SOD_C1))
            keys.append((Q, es))
    B = rsl.Batch(quads, probs, [dt] * len(probs))
    B.set_variant(7, _loop_variant(rsl))
    B.init()
    B.step(2)
    assert B.status()[0] == 0
    for (Q, es) in ((100, 0.01), (100, 10.0), (8, 0.01), (8, 10.0)):
        i = keys.index((Q, es))
        S = oracle.Sod(oracle.VelocitySet(3, Q, 4), nz, tau_mode=oracle.TAU_ETAS, tau_aw0=0.3854 * es,
                       lambda_ref=1.0, bc=oracle.BC_OUTFLOW, store_f32=(dtype == "f32"), **inputs.SOD_C1)
        ref = S.run(S.init(), dt, 2)
        assert _rel(B.f(i).double().cpu().numpy(), ref) < TOL[dtype], (Q, es)


@pytest.mark.parametrize("QL,Q,NOm,nz", [(3, 8, 3, 130), (3, 16, 4, 257), (3, 64, 4, 100), (3, 128, 4, 90),
                                        (3, 160, 4, 70)])
def test_fp32_storage(rsl, QL, Q, NOm, nz):
    """f in binary32, per-cell work in binary64: one-step parity at 1e-5 along
    a 20-step trajectory, end state within the oracle's binary32 envelope."""
    quad, inst, vs, S = _pair(rsl, QL, Q, NOm, nz, dtype="f32", tau_r=5e-3)
    inst.init()
    dt = 0.5 / nz
    _trajectory_parity(inst, S, dt, 20, 5, TOL["f32"])
    got = inst.f().cpu().numpy().astype(np.float64)
    ref, env = _envelope(S, S.init(), dt, 20, store_f32=True)
    assert _rel(got, ref) < max(10 * env, TOL["f32"])


def test_unstable_step_rejected(rsl):
    quad, inst, vs, S = _pair(rsl, 3, 8, 3, 400, tau_r=1e-4)
    inst.init()
    with pytest.raises(rsl.RslError) as e:
        inst.step(1.25e-3, 1)            # dt > 2 tau_r: stiff
    assert e.value.code == rsl.RSL_EUNSTABLE
    with pytest.raises(rsl.RslError) as e:
        inst.step(0.01, 1)               # CFL > 1
    assert e.value.code == rsl.RSL_EUNSTABLE


def test_nonfinite_reported(rsl):
    quad, inst, vs, S = _pair(rsl, 3, 8, 3, 100)
    inst.init()
    assert inst.status() == 0
    f = inst.f()
    f[5, 50] = float("nan")
    inst.step(1e-3, 1)
    assert inst.status() == rsl.RSL_ENONFINITE
