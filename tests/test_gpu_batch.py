"""Batched launches equal the single-instance path bitwise (same tile function,
same arithmetic), for ragged Sod ensembles (uneven N_z, velocity sets, tau and
dt, instances with and without an LDS window) and Bjorken ensembles."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rsl():
    from paper_1612_01287_amd import rsl as mod
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return mod


def _sod_ensemble(rsl, dtype, seed=4, n=12):
    rng = np.random.default_rng(seed)
    quads, probs, dts = [], [], []
    cache = {}
    for i in range(n):
        Q = int(rng.choice([8, 16, 32, 64, 100]))
        nz = int(round(np.exp(rng.uniform(np.log(5), np.log(3000)))))
        TR = 1.0 / rng.uniform(1.1, 3.0)
        tau_r = float(np.exp(rng.uniform(np.log(1e-3), np.log(1.0))))
        key = Q
        if key not in cache:
            cache[key] = rsl.Quadrature(3, Q, min(Q - 1, 4))
        quads.append(cache[key])
        probs.append(rsl.make_problem(nz=nz, dtype=dtype, bc="outflow" if i % 2 else "eq", tau_r=tau_r,
                                      nL=1.0, TL=1.0, nR=TR ** 3, TR=TR))
        dts.append(min(0.5 / nz, 0.5 * tau_r))
    return quads, probs, dts


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_sod_batch_equals_single(rsl, dtype):
    quads, probs, dts = _sod_ensemble(rsl, dtype)
    B = rsl.Batch(quads, probs, dts)
    B.init()
    B.step(5)
    singles = []
    for q, p, dt in zip(quads, probs, dts):
        inst = rsl.Instance(q, p)
        inst.init()
        inst.step(dt, 5)
        singles.append(inst)
    torch.cuda.synchronize()
    for i, inst in enumerate(singles):
        a = B.f(i).cpu().numpy()
        b = inst.f().cpu().numpy()
        assert np.array_equal(a, b), (i, np.max(np.abs(a - b)))
        assert B.time(i) == pytest.approx(5 * dts[i], rel=1e-15)
    rc, bad = B.status()
    assert rc == 0 and bad == -1
    M = B.moments().cpu().numpy()
    row = 0
    for inst in singles:
        Mi = inst.moments().cpu().numpy()
        assert np.array_equal(M[row:row + inst.nz], Mi)
        row += inst.nz


def test_sod_batch_stage_by_stage(rsl):
    quads, probs, dts = _sod_ensemble(rsl, "f64", seed=9, n=5)
    A = rsl.Batch(quads, probs, dts)
    B = rsl.Batch(quads, probs, dts)
    A.init()
    B.init()
    A.step(2)
    for _ in range(2):
        for s in (1, 2, 3):
            B.stage(s)
    torch.cuda.synchronize()
    for i in range(len(probs)):
        assert torch.equal(A.f(i), B.f(i))


def test_bjorken_batch_equals_single(rsl):
    rng = np.random.default_rng(3)
    quads, probs, dts = [], [], []
    for i in range(6):
        Q = int(rng.integers(20, 201))
        q = rsl.Quadrature(3, Q, 4)
        quads.append(q)
        es = float(np.exp(rng.uniform(np.log(0.01), np.log(10.0))))
        T0 = float(np.exp(rng.uniform(np.log(0.5), np.log(2.0))))
        taw0 = 5 * 0.1973269804 * es / (0.25 * T0)
        probs.append(rsl.make_problem(kind="bjorken", tau_mode="etas", tau_aw0=taw0))
        dts.append(1e-3)
    B = rsl.Batch(quads, probs, dts)
    B.init()
    B.step(200)
    for i, (q, p) in enumerate(zip(quads, probs)):
        inst = rsl.Instance(q, p)
        inst.init(t0=1.0)
        inst.step(1e-3, 200)
        assert torch.equal(B.f(i), inst.f()), i
        assert B.time(i) == pytest.approx(1.2, abs=1e-12)
    B.step(100)   # the device clocks continue from tau = 1.2
    inst = rsl.Instance(quads[0], probs[0])
    inst.init(t0=1.0)
    inst.step(1e-3, 200)
    inst.step(1e-3, 100)
    assert torch.equal(B.f(0), inst.f())


def test_graph_replay_equals_eager(rsl):
    """Steps replayed from the captured HIP graph equal eager steps bitwise, on
    every replay, with eager work and synchronisations between replays."""
    quads, probs, dts = _sod_ensemble(rsl, "f64", seed=21, n=7)
    A = rsl.Batch(quads, probs, dts)
    B = rsl.Batch(quads, probs, dts)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        A.init()
        B.init()
        for rep in range(4):
            A.step(3)
            B.graph_step(3)
            junk = torch.randn(1000, device="cuda").sum()     # unrelated eager work
            torch.cuda.synchronize()
            for i in range(len(probs)):
                assert torch.equal(A.f(i), B.f(i)), (rep, i)
            assert float(junk) == float(junk)
        assert B.time(0) == pytest.approx(12 * dts[0], rel=1e-14)
