"""GPU parity of the Bjorken-flow step against the oracle (FP64: 1e-12, FP32: 1e-5)."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rsl():
    from paper_1612_01287_amd import rsl as mod
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return mod


@pytest.mark.parametrize("gas,tau_mode,taw", [("ideal", "etas", 0.2), ("ideal", "const", 0.5),
                                              ("parton", "etas", 0.4), ("ideal", "inf", 0.0)])
@pytest.mark.parametrize("QL,Q,NOm", [(2, 6, 5), (3, 20, 4), (3, 77, 4), (3, 200, 4)])
def test_bjorken_parity(rsl, gas, tau_mode, taw, QL, Q, NOm):
    quad = rsl.Quadrature(QL, Q, NOm)
    p = rsl.make_problem(kind="bjorken", gas=gas, tau_mode=tau_mode, tau_r=taw, tau_aw0=taw, nL=1.0, TL=1.0)
    inst = rsl.Instance(quad, p)
    inst.init(t0=1.0)
    inst.step(1e-3, 300)
    assert abs(inst.t - 1.3) < 1e-12
    vs = oracle.VelocitySet(QL, Q, NOm)
    B = oracle.Bjorken(vs, gas=oracle.GAS_IDEAL if gas == "ideal" else oracle.GAS_PARTON,
                       tau_mode={"const": oracle.TAU_CONST, "etas": oracle.TAU_ETAS, "inf": oracle.TAU_INF}[tau_mode],
                       tau_r=taw, tau_aw0=taw)
    ref, _ = B.run(B.init(), 1.0, 1e-3, 300)
    got = inst.f().cpu().numpy().reshape(-1)
    assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) < 1e-12
    if gas == "ideal":
        M = inst.moments().cpu().numpy()[0]
        assert M[0] * 1.3 == pytest.approx(1.0, abs=1e-12)      # tau n = 1 (eq. bjorken_n)


def test_bjorken_fp32(rsl):
    quad = rsl.Quadrature(3, 40, 4)
    p = rsl.make_problem(kind="bjorken", dtype="f32", tau_mode="etas", tau_aw0=0.1)
    inst = rsl.Instance(quad, p)
    inst.init(t0=1.0)
    inst.step(1e-3, 500)
    vs = oracle.VelocitySet(3, 40, 4)
    B = oracle.Bjorken(vs, tau_mode=oracle.TAU_ETAS, tau_aw0=0.1, store_f32=True)
    ref, _ = B.run(B.init(), 1.0, 1e-3, 500)
    got = inst.f().cpu().numpy().reshape(-1).astype(np.float64)
    assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) < 1e-5
