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


def _fits(rsl, cap_needed):
    return [v for v, sh in enumerate(rsl.stage_variants()) if sh[3] >= cap_needed]


def _ragged_all_classes(rsl, dtype):
    """Instances in all seven velocity classes (V = 24, 48, 120, 192, 300, 384, 450)."""
    quads, probs, dts = [], [], []
    for i, (Q, nz) in enumerate([(8, 200), (16, 77), (40, 130), (64, 64), (100, 95), (128, 33), (8, 5),
                                 (150, 70)]):
        quads.append(rsl.Quadrature(3, Q, min(Q - 1, 4)))
        TR = 1.0 / (1.2 + 0.2 * i)
        probs.append(rsl.make_problem(nz=nz, dtype=dtype, bc="eq" if i % 2 else "outflow", tau_r=0.02 + 0.01 * i,
                                      nL=1.0, TL=1.0, nR=TR ** 3, TR=TR))
        dts.append(min(0.4 / nz, 0.5 * (0.02 + 0.01 * i)))
    return quads, probs, dts


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_every_stage_variant_matches_default(rsl, dtype, tol):
    """Variants change only the order of the per-cell moment sums."""
    quads, probs, dts = _ragged_all_classes(rsl, dtype)
    ref = rsl.Batch(quads, probs, dts)
    ref.init()
    ref.step(2)
    torch.cuda.synchronize()
    want = [ref.f(i).double().cpu().numpy() for i in range(ref.n)]
    B = rsl.Batch(quads, probs, dts)
    tried = 0
    for cls in range(rsl.N_CLASSES):
        var0, maxv = B.variant(cls)
        assert var0 >= 0 and maxv > 0
        for v in _fits(rsl, maxv):
            B.set_variant(cls, v)
            assert B.variant(cls)[0] == v
            B.init()
            B.step(2)
            torch.cuda.synchronize()
            for i in range(B.n):
                got = B.f(i).double().cpu().numpy()
                err = np.max(np.abs(got - want[i])) / np.max(np.abs(want[i]))
                assert err < tol, (cls, v, i, err)
            tried += 1
        B.set_variant(cls, -1)
        assert B.variant(cls)[0] == var0
    assert tried >= 20
    rc, bad = B.status()
    assert rc == 0 and bad == -1


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_single_class_launches_match_default(rsl, dtype, tol):
    """Every instance in one class (class index 7: one launch per kernel and
    stage on the caller's stream), in the two-kernel and the loop form, agrees
    with the per-class launches to rounding; index -1 goes back to them."""
    quads, probs, dts = _ragged_all_classes(rsl, dtype)
    ref = rsl.Batch(quads, probs, dts)
    ref.init()
    ref.step(3)
    torch.cuda.synchronize()
    want = [ref.f(i).double().cpu().numpy() for i in range(ref.n)]
    shapes = rsl.stage_variants()
    B = rsl.Batch(quads, probs, dts)
    assert B.variant(7)[0] == -1
    for form in (1, 2):
        v = next(k for k, sh in enumerate(shapes) if sh[5] == form)
        B.set_variant(7, v)
        assert B.variant(7)[0] == v
        B.init()
        B.step(3)
        torch.cuda.synchronize()
        for i in range(B.n):
            got = B.f(i).double().cpu().numpy()
            assert np.max(np.abs(got - want[i])) / np.max(np.abs(want[i])) < tol, (v, i)
    B.set_variant(7, -1)
    assert B.variant(7)[0] == -1
    B.init()
    B.step(3)
    for i in range(B.n):
        assert torch.equal(B.f(i).double().cpu(), torch.from_numpy(want[i]))
    assert B.status()[0] == 0


def test_set_variant_rejects_small_variants(rsl):
    quads, probs, dts = _ragged_all_classes(rsl, "f64")
    B = rsl.Batch(quads, probs, dts)
    caps = [sh[3] for sh in rsl.stage_variants()]
    small = int(np.argmin(caps))
    with pytest.raises(RuntimeError):
        B.set_variant(5, small)        # class of V = 384
    with pytest.raises(RuntimeError):
        B.set_variant(0, len(caps))    # no such variant


def test_autotune_keeps_state_and_results(rsl):
    quads, probs, dts = _ragged_all_classes(rsl, "f64")
    B = rsl.Batch(quads, probs, dts)
    B.init()
    B.step(1)
    torch.cuda.synchronize()
    before = [B.f(i).clone() for i in range(B.n)]
    chosen = B.autotune(reps=2)
    torch.cuda.synchronize()
    caps = [sh[3] for sh in rsl.stage_variants()]
    for cls, v in enumerate(chosen):
        var, maxv = B.variant(cls)
        assert v == var and caps[v] >= maxv
    for i in range(B.n):
        assert torch.equal(before[i], B.f(i))
    A = rsl.Batch(quads, probs, dts)
    A.init()
    A.step(3)
    B.step(2)
    torch.cuda.synchronize()
    for i in range(B.n):
        a, b = A.f(i).cpu().numpy(), B.f(i).cpu().numpy()
        assert np.max(np.abs(a - b)) / np.max(np.abs(a)) < 1e-12


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
    B.set_path(0)          # the per-instance kernel shares the single-instance code
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


def _loop_variant(rsl):
    return next(k for k, sh in enumerate(rsl.stage_variants()) if sh[5] == 2)


def test_loop_form_graph_and_stages(rsl):
    """The whole batch as one class in the loop form: graph replays equal eager
    steps bitwise (each call starts with the per-cell kernel, later stages take
    the coefficients the previous stage left); single stages (each computing
    its coefficients afresh) agree with whole steps to rounding."""
    quads, probs, dts = _sod_ensemble(rsl, "f64", seed=23, n=7)
    v = _loop_variant(rsl)
    A, B, C = (rsl.Batch(quads, probs, dts) for _ in range(3))
    for X in (A, B, C):
        X.set_variant(7, v)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        A.init()
        B.init()
        C.init()
        for rep in range(3):
            A.step(4)
            B.graph_step(4)
            for _ in range(4):
                for st in (1, 2, 3):
                    C.stage(st)
            torch.cuda.synchronize()
            for i in range(len(probs)):
                assert torch.equal(A.f(i), B.f(i)), (rep, i)
                a, c = A.f(i).cpu().numpy(), C.f(i).cpu().numpy()
                assert np.max(np.abs(a - c)) / np.max(np.abs(a)) < 1e-12, (rep, i)
    assert B.status()[0] == 0


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_loop_form_every_relaxation_law(rsl, dtype, tol):
    """Constant tau, the eta/s law and free streaming (no collision term: the
    loop form then skips the coefficients and the closing chain) in one batch
    as one class, against single-instance steps (two-kernel form)."""
    cases = [(8, 130, "const"), (16, 70, "etas"), (40, 200, "inf"), (100, 64, "etas"), (8, 5, "inf"),
             (64, 90, "const")]
    quads, probs, dts = [], [], []
    for Q, nz, mode in cases:
        quads.append(rsl.Quadrature(3, Q, min(Q - 1, 4)))
        probs.append(rsl.make_problem(nz=nz, dtype=dtype, bc="eq" if nz % 2 else "outflow", tau_mode=mode,
                                      tau_r=0.02, tau_aw0=0.3854 * 0.5, nL=1.0, TL=1.0, nR=0.4, TR=0.8))
        dts.append(0.4 / nz)
    B = rsl.Batch(quads, probs, dts)
    B.set_variant(7, _loop_variant(rsl))
    B.init()
    B.step(6)
    torch.cuda.synchronize()
    for i, (q, p) in enumerate(zip(quads, probs)):
        inst = rsl.Instance(q, p)
        inst.init()
        inst.step(dts[i], 6)
        a, b = inst.f().double().cpu().numpy(), B.f(i).double().cpu().numpy()
        assert np.max(np.abs(a - b)) / np.max(np.abs(a)) < tol, (i, cases[i])
    assert B.status()[0] == 0


def _bj_ensemble(rsl, n, seed, dtype="f64", Qs=(20, 37, 64, 200)):
    rng = np.random.default_rng(seed)
    quads = {Q: rsl.Quadrature(3, Q, 4) for Q in Qs}
    qs, probs, dts = [], [], []
    for i in range(n):
        Q = int(rng.choice(Qs))
        es = float(np.exp(rng.uniform(np.log(0.01), np.log(10.0))))
        T0 = float(np.exp(rng.uniform(np.log(0.5), np.log(2.0))))
        taw0 = 5 * 0.1973269804 * es / (0.25 * T0)
        gas, mode = [("ideal", "etas"), ("parton", "etas"), ("ideal", "inf"), ("ideal", "const")][i % 4]
        qs.append(quads[Q])
        probs.append(rsl.make_problem(kind="bjorken", gas=gas, tau_mode=mode, tau_aw0=taw0, tau_r=0.3, dtype=dtype))
        dts.append(1e-3)
    return qs, probs, dts


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_bjorken_matrix_cores_match_vector_path(rsl, dtype, tol):
    """The matrix-core group kernel (K^P F by MFMA f64 16x16x4) agrees with the
    per-instance vector kernel (itself at 1e-12 of the oracle) to rounding;
    groups are ragged (fewer than 16 instances, Q_xi not a multiple of 16)."""
    qs, probs, dts = _bj_ensemble(rsl, 37, seed=5, dtype=dtype)
    A = rsl.Batch(qs, probs, dts)
    B = rsl.Batch(qs, probs, dts)
    A.set_path(0)
    B.set_path(1)
    A.init()
    B.init()
    A.step(150)
    B.step(150)
    B.step(50)
    A.step(50)
    torch.cuda.synchronize()
    for i in range(len(probs)):
        a = A.f(i).double().cpu().numpy()
        b = B.f(i).double().cpu().numpy()
        assert np.max(np.abs(a - b)) / np.max(np.abs(a)) < tol, i
        assert B.time(i) == pytest.approx(1.2, abs=1e-12)
    rc, bad = B.status()
    assert rc == 0


def test_bjorken_matrix_cores_mixed_radial_sets(rsl):
    """One batch holding Q_L = 2, 3 and 4 velocity sets: one matrix-core launch
    per Q_L, each group against the vector path to rounding."""
    rng = np.random.default_rng(12)
    qs, probs, dts = [], [], []
    cache = {}
    for i in range(40):
        QL = int(rng.choice([2, 3, 4]))
        Q = int(rng.choice([20, 33, 64, 150]))
        if (QL, Q) not in cache:
            cache[(QL, Q)] = rsl.Quadrature(QL, Q, 4)
        es = float(np.exp(rng.uniform(np.log(0.01), np.log(10.0))))
        qs.append(cache[(QL, Q)])
        probs.append(rsl.make_problem(kind="bjorken", tau_mode="etas", tau_aw0=5 * 0.1973269804 * es / 0.25))
        dts.append(1e-3)
    A = rsl.Batch(qs, probs, dts)
    B = rsl.Batch(qs, probs, dts)
    A.set_path(0)
    B.set_path(1)
    A.init()
    B.init()
    A.step(120)
    B.step(120)
    torch.cuda.synchronize()
    for i in range(len(probs)):
        a = A.f(i).cpu().numpy()
        b = B.f(i).cpu().numpy()
        assert np.max(np.abs(a - b)) / np.max(np.abs(a)) < 1e-12, (i, qs[i].QL, qs[i].Q)
    assert B.status()[0] == 0


def test_bjorken_groups_of_every_tile_count(rsl):
    """Velocity sets of very different sizes: the batch spreads the large sets
    over groups of fewer instances (1, 2 or 3 of the 16-column tiles at
    Q_L = 3) to balance the compute units; every instance still agrees with
    the vector path to rounding, whatever the size of its group."""
    rng = np.random.default_rng(21)
    quads, qs, probs, dts = {}, [], [], []
    for _ in range(1500):
        Q = int(rng.integers(20, 201))
        if Q not in quads:
            quads[Q] = rsl.Quadrature(3, Q, 4)
        es = float(np.exp(rng.uniform(np.log(0.01), np.log(10.0))))
        qs.append(quads[Q])
        probs.append(rsl.make_problem(kind="bjorken", tau_mode="etas", tau_aw0=5 * 0.1973269804 * es / 0.25))
        dts.append(1e-3)
    A = rsl.Batch(qs, probs, dts)
    B = rsl.Batch(qs, probs, dts)
    A.set_path(0)
    B.set_path(1)
    sizes = B.groups()
    assert sum(sizes) == len(probs) and all(1 <= n <= 16 for n in sizes)
    assert {(3 * n + 15) // 16 for n in sizes} == {1, 2, 3}
    A.init()
    B.init()
    A.step(30)
    B.step(30)
    a = torch.cat([A.f(i).reshape(-1) for i in range(len(probs))]).cpu().numpy()
    b = torch.cat([B.f(i).reshape(-1) for i in range(len(probs))]).cpu().numpy()
    amax = torch.stack([A.f(i).abs().max() for i in range(len(probs))]).cpu().numpy()
    scale = np.repeat(amax, [q.V for q in qs])
    assert np.max(np.abs(a - b) / scale) < 1e-12
    assert B.status()[0] == 0


def test_bjorken_matrix_cores_vs_oracle(rsl):
    import oracle
    qs, probs, dts = _bj_ensemble(rsl, 5, seed=8, Qs=(40, 101))
    B = rsl.Batch(qs, probs, dts)
    B.set_path(1)
    B.init()
    B.step(400)
    for i in range(len(probs)):
        q, p = qs[i], probs[i]
        vs = oracle.VelocitySet(3, q.Q, 4)
        Bo = oracle.Bjorken(vs, gas=oracle.GAS_IDEAL if p.gas == 0 else oracle.GAS_PARTON,
                            tau_mode=p.tau_mode, tau_r=p.tau_r, tau_aw0=p.tau_aw0)
        ref, _ = Bo.run(Bo.init(), 1.0, 1e-3, 400)
        got = B.f(i).cpu().numpy().reshape(-1)
        assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) < 1e-12, i


def test_batch_rejects_unstable_steps(rsl):
    """rsl_batch_create applies the CFL and stiffness guards of rsl_step to every instance."""
    quad = rsl.Quadrature(3, 8, 3)
    ok = rsl.make_problem(nz=100, tau_r=0.01)
    stiff = rsl.make_problem(nz=100, tau_r=1e-4)
    with pytest.raises(RuntimeError, match="instance 1"):
        rsl.Batch([quad, quad], [ok, stiff], [0.004, 0.004])
    with pytest.raises(RuntimeError, match="CFL"):
        rsl.Batch([quad], [ok], [0.02])
    forced = rsl.make_problem(nz=100, tau_r=1e-4, force=True)
    rsl.Batch([quad, quad], [ok, forced], [0.004, 0.004])
