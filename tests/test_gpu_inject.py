"""GPU parity of the in-loop feedback calls (rsl_mlp_inject, rsl_project)
against the oracle's plain versions (oracle/mlp.py inject, project), and the
moments they must keep or move on a developed high-order state.

Bar: max |gpu - oracle| / max |oracle| <= 1e-12 (binary64 populations),
2e-6 (binary32: the stored values are rounded once more than the oracle's)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import mlp
from tests import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rsl():
    from paper_1612_01287_amd import rsl as mod
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return mod


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _moments(vs, f):
    return mlp._moment_rows(vs) @ np.asarray(f, dtype=np.float64)


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 2e-6)])
@pytest.mark.parametrize("Q,NOm", [(8, 4), (3, 2), (16, 5)])
def test_inject_matches_oracle(rsl, dtype, tol, Q, NOm):
    nz = 203
    q = rsl.Quadrature(3, Q, NOm)
    vs = oracle.VelocitySet(3, Q, NOm)
    p = rsl.make_problem(nz=nz, dtype=dtype)
    inst = rsl.Instance(q, p)
    rng = inputs.rng(Q)
    f0 = rng.uniform(0.2, 1.0, (vs.V, nz)) * np.outer(vs.wL, vs.wxi).ravel()[:, None]
    inst.set_f(f0)
    f_stored = inst.f().double().cpu().numpy()
    y = (0.02 * rng.uniform(-1.0, 1.0, (nz, 3))).astype(np.float32)
    rsl.inject(q, p, inst.f_buf, torch.tensor(y, device="cuda"))
    got = inst.f().double().cpu().numpy()
    e = _moments(vs, f_stored)[2]
    want = mlp.inject(vs, f_stored, y.astype(np.float64) * e[:, None])
    assert _rel(got, want) < tol
    d = _moments(vs, got) - _moments(vs, f_stored)
    assert np.max(np.abs(d[:2])) < 10 * tol * np.max(np.abs(e))
    assert np.allclose(d[2:].T, y * e[:, None], rtol=0, atol=10 * tol * np.max(np.abs(e)))


@pytest.mark.parametrize("dh,dl,tol", [("f64", "f64", 1e-12), ("f32", "f32", 2e-6), ("f64", "f32", 2e-6)])
def test_project_matches_oracle(rsl, dh, dl, tol):
    """A high-order state off equilibrium (moving equilibria times noise, some
    cells at beta ~ 0.6) onto R-SLB(4;8)."""
    nz = 150
    qh, ql = rsl.Quadrature(3, 64, 4), rsl.Quadrature(3, 8, 4)
    vh, vl = oracle.VelocitySet(3, 64, 4), oracle.VelocitySet(3, 8, 4)
    rng = inputs.rng(8)
    betas = rng.uniform(-0.6, 0.6, nz)
    fh = np.stack([oracle.feq(vh, rng.uniform(0.3, 1.5), rng.uniform(0.5, 1.2), b) for b in betas], axis=1)
    fh *= 1.0 + 0.05 * rng.uniform(-1.0, 1.0, fh.shape)
    ph, pl = rsl.make_problem(nz=nz, dtype=dh), rsl.make_problem(nz=nz, dtype=dl)
    ih, il = rsl.Instance(qh, ph), rsl.Instance(ql, pl)
    ih.set_f(fh)
    fh_stored = ih.f().double().cpu().numpy()
    rsl.project(qh, ph, ih.f_buf, ql, pl, il.f_buf)
    got = il.f().double().cpu().numpy()
    want = mlp.project(vh, fh_stored, vl)
    assert _rel(got, want) < tol
    assert np.allclose(_moments(vl, got), _moments(vh, fh_stored), rtol=10 * tol, atol=10 * tol)


def test_project_keeps_the_moments_of_a_developed_flow(rsl):
    """R-SLB(4;128) tube of the learned-correction workload (N_z = 8192,
    binary32) run to t = 0.1, projected onto R-SLB(4;8): every cell's N^0, N^z,
    T^00, T^0z, T^zz kept (a property at any size)."""
    nz = 8192
    qh, ql = rsl.Quadrature(3, 128, 4), rsl.Quadrature(3, 8, 4)
    ph = rsl.make_problem(nz=nz, dtype="f32", tau_r=0.05, nL=1.0, TL=1.0, nR=0.125, TR=0.5)
    pl = rsl.make_problem(nz=nz, dtype="f32", tau_r=0.05, nL=1.0, TL=1.0, nR=0.125, TR=0.5)
    ih, il = rsl.Instance(qh, ph), rsl.Instance(ql, pl)
    ih.init()
    ih.step(0.5 / nz, int(0.1 * nz / 0.5))
    rsl.project(qh, ph, ih.f_buf, ql, pl, il.f_buf)
    mh = ih.moments().cpu().numpy()[:, :5]
    ml = il.moments().cpu().numpy()[:, :5]
    assert np.all(np.isfinite(ml))
    assert np.max(np.abs(ml - mh)) < 2e-6 * np.max(np.abs(mh))


def test_feedback_argument_errors(rsl):
    q2 = rsl.Quadrature(3, 2, 1)
    p = rsl.make_problem(nz=8)
    inst = rsl.Instance(q2, p)
    y = torch.zeros((8, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(rsl.RslError) as e:
        rsl.inject(q2, p, inst.f_buf, y)
    assert e.value.code == rsl.RSL_EUNSUPPORTED
    q = rsl.Quadrature(3, 8, 4)
    pa, pb = rsl.make_problem(nz=8), rsl.make_problem(nz=9)
    ia, ib = rsl.Instance(q, pa), rsl.Instance(q, pb)
    with pytest.raises(rsl.RslError) as e:
        rsl.project(q, pa, ia.f_buf, q, pb, ib.f_buf)
    assert e.value.code == rsl.RSL_EINVAL
