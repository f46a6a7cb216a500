"""Throughput of the R-SLB Sod step on one MI355X.

Workload (the finite-viscosity shock-tube sweep): N_z = 4096 cells on
z in [-0.5, 0.5], (T, n)_L = (1, 1), (T, n)_R = (0.8, 0.4), outflow ghosts,
Q_L = 3 radial nodes, Q_xi in {8, 16, 40, 100}, N_Omega = 4, eta/s in
{0.01, 0.1, 1, 10} with tau_AW0 = 0.3854 eta/s (relaxation-time law of
eq. Sod:tau), dt = 0.5 / N_z, f in binary64 -- sixteen instances.  One step =
one TVD-RK3 step (three fused stage kernels) of all sixteen instances.
Metric: distribution updates per second, one update = one (cell, velocity,
RK stage).

Prints one JSON line (see the repository's measurement contract).  Its "aux"
object carries five further measurements on seeded synthetic inputs:
  c1       the near-inviscid tube (N_z = 400, R-SLB(3;8), tau_r = 1e-3,
           dt = 1.25e-3, 200 steps), launch-bound: updates/s and the last
           step against the oracle;
  bjorken  4096 Bjorken runs (T0 log-uniform in [0.5, 2] GeV, eta/s
           log-uniform in [0.01, 10], Q_xi uniform in {20..200}, Q_L = 3,
           ideal gas), a 1000-step window at dtau = 1e-3 in one launch; the
           K^P F product on the matrix cores against the FP64 MFMA peak;
  ensemble 1024 uneven Sod instances (N_z log-uniform in [256, 16384],
           Q_xi in {8, 16, 32, 64}, T_L/T_R uniform in [1.1, 3], tau_r
           log-uniform in [1e-4, 1], dt = min(0.5/N_z, tau_r/2)), f in
           binary32, 200 steps in graph replays of 100; 1.4 GB per field,
           so HBM-bound;
  scaled   the sweep's 16 instances x 128 copies (8.3 GB per field, FP64),
           out of the last-level cache: 20 steps timed after 1000;
  learned  the learned T^{mu nu} correction, scaled down (2048 paired
           training runs x 5 snapshots x 2048 cells = 2.1e7 samples, 100
           epochs, and 64 evaluation instances, at N_z = 2048 instead of 8192):
           R-SLB(4;8) + features + network against the plain R-SLB(4;128)
           solve, wall time and relative T^{mu nu} error at t = 0.25.
The first three carry a "cpu_baseline" of the oracle on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

QXI = (8, 16, 40, 100)
ETAS = (0.01, 0.1, 1.0, 10.0)
NZ = 4096
QL = 3
NOM = 4
BYTES_PER_CELL_VEL_STEP = {"f64": 64, "f32": 32}   # f_n read 3x, stage fields read 2x, written 3x
HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6
HBARC = 0.1973269804      # GeV fm
CHUNK = 10          # RK3 steps per captured HIP graph
STEPS = 2000        # RK3 steps of the sweep (t = 0.244 at dt = 0.5 / N_z)
# HBM bytes per stage launch group read from rocprofv3 FETCH_SIZE / WRITE_SIZE
# counters (scaled by a plain copy kernel's readings); valid only for the
# kernel sources and variants they were taken with
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sod_stage_c2_traffic.txt")
KERNEL_SOURCES = ("sod_stage.h", "sod_split.h", "sod_stage_f64.hip", "sod_stage_f32.hip", "rsl_math.h", "rsl_impl.h")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--dtype", default="f64", choices=("f64", "f32"))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default stage-kernel variants")
    ap.add_argument("--variants", default=None,
                    help="comma-separated stage-kernel variant per velocity class (-1: empty), and an eighth "
                         "for the whole batch as one class (-1: per class); skips the autotuner")
    ap.add_argument("--aux", default="all", choices=("none", "all", "c1", "bjorken", "ensemble", "scaled",
                                                           "learned"),
                    help="also measure the near-inviscid tube, the Bjorken batch, the uneven Sod ensemble, the "
                         "sweep scaled out of the cache and the learned correction (all), or one of them")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy five times (the reference kernel for "
                         "scaling FETCH_SIZE / WRITE_SIZE counters to bytes)")
    return ap.parse_args()


def build_batch(rsl, dtype):
    quads, probs, dts = [], [], []
    for Q in QXI:
        quad = rsl.Quadrature(QL, Q, NOM)
        for es in ETAS:
            quads.append(quad)
            probs.append(rsl.make_problem(nz=NZ, dtype=dtype, bc="outflow", tau_mode="etas",
                                          tau_aw0=0.3854 * es, nL=1.0, TL=1.0, nR=0.4, TR=0.8))
            dts.append(0.5 / NZ)
    B = rsl.Batch(quads, probs, dts)
    B.init()
    return B


def kernel_source_hash():
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1612_01287_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(dtype, variants):
    """HBM bytes per stage launch group from the committed counter summary, or
    None when it was taken on other kernel sources or variants."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    rec = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    key = "bytes_per_stage_group_" + dtype
    if rec.get("kernel_source_hash") != kernel_source_hash() or key not in rec:
        return None
    if rec.get("kernel_forms_" + dtype) != kernel_forms(variants):
        return None
    return float(rec[key])


def kernel_forms(variants):
    """Per class: 's' for the two-kernel form, 'l' for the loop form (their HBM
    traffic does not depend on the launch shape), else the fused variant id;
    '-' for an empty class; "all:<form>" when the whole batch runs as one
    class (an eighth entry >= 0)."""
    from paper_1612_01287_amd import rsl
    shapes = rsl.stage_variants()
    form = lambda v: "-" if v < 0 else {1: "s", 2: "l"}.get(shapes[v][5], str(v))
    if len(variants) > rsl.N_CLASSES and variants[rsl.N_CLASSES] >= 0:
        return "all:" + form(variants[rsl.N_CLASSES])
    return ",".join(form(v) for v in variants[:rsl.N_CLASSES])


def kernel_roofline(torch, B, dtype, updates_per_step, variants, chunk, stream, reps=10):
    """Average duration of one RK stage of the whole batch (a stage launch
    group: the stage kernels of every velocity class, launched concurrently
    from one stream), from HIP events on that stream around graph replays of
    `chunk` steps (3 chunk stage groups each)."""
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * reps)]
    for r in range(reps):
        ev[2 * r].record(stream)
        B.graph_step(chunk, stream=stream)
        ev[2 * r + 1].record(stream)
    ev[-1].synchronize()
    ms = sum(ev[i].elapsed_time(ev[i + 1]) for i in range(0, len(ev), 2)) / (3 * chunk * reps)
    cell_vel = updates_per_step / 3
    bytes_per_launch = BYTES_PER_CELL_VEL_STEP[dtype] / 3.0 * cell_vel
    gbs = bytes_per_launch / (ms * 1e-3) / 1e9
    return dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(gbs / HBM_PEAK_GBS, 4), traffic=measured_traffic(dtype, variants),
                kernel="Sod stage launch group (one RK stage of all velocity classes; mean over %d graph-replayed "
                       "stages)" % (3 * chunk * reps), avg_launch_us=round(ms * 1e3, 2),
                bytes_per_launch=bytes_per_launch, variants=variants, kernel_forms=kernel_forms(variants),
                kernel_source_hash=kernel_source_hash(),
                residency="the sweep's three fields (%.0f MB) fit in the 256 MB last-level cache, so part of the "
                          "traffic is served there; the HBM-resident cases are the scaled and ensemble aux legs"
                          % (3 * BYTES_PER_CELL_VEL_STEP[dtype] / 8 * cell_vel / 1e6))


def _events(torch, stream, fn, reps=1):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e-3


def _progress(msg):
    """One line per finished part of the run, on stderr (the JSON line is stdout's only line)."""
    print("bench: " + msg, file=sys.stderr, flush=True)


def _oracle_rate(fn, updates, sample):
    """Single-threaded oracle on a bounded sample: updates/s and what was run."""
    t0 = time.perf_counter()
    fn()
    return dict(value=updates / (time.perf_counter() - t0), unit="updates/s", cores=1, kind="oracle",
                sample=sample)


def c1_leg(torch, rsl, stream, cpu=True):
    """The near-inviscid tube: N_z = 400, R-SLB(3;8), tau_r = 1e-3, dt = 1.25e-3,
    200 steps (launch-bound, not HBM-bound): updates/s of the whole run as a
    one-instance batch (autotuned on a developed state) replayed from graphs
    of 10 steps, and as eager single-instance steps.  Parity: one more batch step from the final state
    against one oracle step from that same state; and the final state against
    the oracle's 200-step run (the CPU baseline's sample), beside the spread
    of the oracle itself under a one-ulp perturbation of its input (WENO5
    without a regulariser amplifies rounding differences near the fronts)."""
    import numpy as np
    import oracle
    nz, dt, steps = 400, 1.25e-3, 200
    quad = rsl.Quadrature(QL, 8, 3)
    prob = rsl.make_problem(nz=nz, tau_r=1e-3, nL=1.0, TL=1.0, nR=0.4, TR=0.8)
    B = rsl.Batch([quad], [prob], [dt])
    B.init(stream=stream)
    B.step(20, stream=stream)
    B.autotune(reps=3, stream=stream)
    B.init(stream=stream)
    B.graph_step(10, stream=stream)
    B.init(stream=stream)
    sec = _events(torch, stream, lambda: B.graph_step(10, stream=stream), reps=steps // 10)
    got = B.f(0).cpu().numpy()
    B.step(1, stream=stream)
    one = B.f(0).cpu().numpy()
    inst = rsl.Instance(quad, prob)
    inst.init(stream=stream)
    inst.step(dt, 10, stream=stream)
    sec_eager = _events(torch, stream, lambda: inst.step(dt, steps, stream=stream))
    S = oracle.Sod(oracle.VelocitySet(QL, 8, 3), nz, nL=1.0, TL=1.0, nR=0.4, TR=0.8, tau_r=1e-3,
                   bc=oracle.BC_OUTFLOW)
    f0 = S.init()
    t0 = time.perf_counter()
    ref = S.run(f0, dt, steps)
    cpu_s = time.perf_counter() - t0
    rel = lambda x, y: float(np.max(np.abs(x - y)) / np.max(np.abs(y)))
    pert = S.run(f0 * (1 + 1.1e-16 * np.random.default_rng(0).standard_normal(f0.shape)), dt, steps)
    updates = 3.0 * nz * quad.V * steps
    out = {"workload": "Sod near-inviscid: N_z = 400, Q_L = 3, Q_xi = 8, N_Omega = 3, tau_r = 1e-3, "
                       "dt = 1.25e-3, 200 steps, f64",
           "value": updates / sec, "unit": "updates/s", "seconds": sec,
           "eager_single_instance_updates_per_s": updates / sec_eager,
           "variants": [B.variant(c)[0] for c in range(rsl.N_CLASSES + 1)],
           "one_step_rel_err_vs_oracle": rel(one, S.run(got, dt, 1)),
           "run_rel_err_vs_oracle": rel(got, ref), "oracle_one_ulp_envelope": rel(pert, ref)}
    if cpu:
        out["cpu_baseline"] = dict(value=updates / cpu_s, unit="updates/s", cores=1, kind="oracle",
                                   sample="the whole 200-step run (single-threaded plain C)")
    return out


def scaled_leg(torch, rsl, stream, copies=128, dev_steps=1000, steps=20, chunk=10):
    """The sweep scaled out of the last-level cache: 128 copies of each of its
    16 instances (2048 instances, 24.8 GB in the three f fields, FP64), run
    for 1000 steps (the state the headline's variants are tuned on), tuned,
    then 20 steps timed in graph replays of 10."""
    quads, probs, dts = [], [], []
    for Q in QXI:
        quad = rsl.Quadrature(QL, Q, NOM)
        for es in ETAS:
            for _ in range(copies):
                quads.append(quad)
                probs.append(rsl.make_problem(nz=NZ, bc="outflow", tau_mode="etas", tau_aw0=0.3854 * es,
                                              nL=1.0, TL=1.0, nR=0.4, TR=0.8))
                dts.append(0.5 / NZ)
    B = rsl.Batch(quads, probs, dts)
    B.init(stream=stream)
    B.step(dev_steps, stream=stream)
    B.autotune(reps=3, stream=stream)
    B.graph_step(chunk, stream=stream)
    sec = _events(torch, stream, lambda: B.graph_step(chunk, stream=stream), reps=steps // chunk)
    rc, bad = B.status(stream)
    assert rc == 0, "non-finite scaled-sweep instance %d" % bad
    cellvel = sum(p.nz * q.V for p, q in zip(probs, quads))
    updates = 3.0 * cellvel * steps
    gbs = BYTES_PER_CELL_VEL_STEP["f64"] * cellvel * steps / sec / 1e9
    return {"workload": "the sweep x %d copies: %d Sod instances, N_z = 4096, Q_xi in {8,16,40,100}, "
                        "eta/s in {0.01,0.1,1,10}, f64, steps %d-%d"
                        % (copies, 16 * copies, dev_steps, dev_steps + steps),
            "value": updates / sec, "unit": "updates/s", "ms_per_step": sec / steps * 1e3,
            "f_bytes_per_field": 8 * cellvel,
            "variants": [B.variant(c)[0] for c in range(rsl.N_CLASSES + 1)],
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "kernel": "Sod stage kernels of the whole batch, 64 B per cell-velocity and step"}}


def bjorken_leg(torch, rsl, stream, n=4096, window=1000, seed=3, cpu=True):
    import numpy as np
    rng = np.random.default_rng(seed)
    quads, qs, probs = {}, [], []
    flop_stage = 0.0
    for _ in range(n):
        Q = int(rng.integers(20, 201))
        T0 = float(np.exp(rng.uniform(np.log(0.5), np.log(2.0))))
        es = float(np.exp(rng.uniform(np.log(0.01), np.log(10.0))))
        if Q not in quads:
            quads[Q] = rsl.Quadrature(QL, Q, 4)
        qs.append(quads[Q])
        probs.append(rsl.make_problem(kind="bjorken", gas="ideal", tau_mode="etas",
                                      tau_aw0=5 * HBARC * es / (0.25 * T0)))
        flop_stage += 2.0 * Q * Q * QL
    B = rsl.Batch(qs, probs, [1e-3] * n)
    B.init(stream=stream)
    B.step(10, stream=stream)
    sec = _events(torch, stream, lambda: B.step(window, stream=stream))
    rc, bad = B.status(stream)
    assert rc == 0, "non-finite Bjorken instance %d" % bad
    updates = 3.0 * window * sum(q.V for q in qs)
    tflops = 3.0 * window * flop_stage / sec / 1e12
    out = {"workload": "4096 Bjorken runs, Q_xi uniform in {20..200}, Q_L = 3, 1000 steps of dtau = 1e-3, f64",
           "value": updates / sec, "unit": "updates/s", "seconds": sec,
           "roofline": {"bound": "mfma", "achieved": round(tflops, 3), "peak": FP64_MFMA_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(tflops / FP64_MFMA_PEAK_TFLOPS, 4),
                        "kernel": "bj_mfma_kernel (K^P F, 2 Q_xi^2 Q_L flop per instance and stage)"}}
    if cpu:
        import oracle
        sample = [(int(q.Q), p.tau_aw0) for q, p in zip(qs[:8], probs[:8])]
        runs = [oracle.Bjorken(oracle.VelocitySet(QL, Q, 4), tau_mode=oracle.TAU_ETAS, tau_aw0=taw)
                for Q, taw in sample]
        out["cpu_baseline"] = _oracle_rate(lambda: [R.run(R.init(), 1.0, 1e-3, window) for R in runs],
                                           3.0 * window * sum(QL * Q for Q, _ in sample),
                                           "the first 8 runs of the batch, the same %d-step window each "
                                           "(single-threaded plain C)" % window)
    return out


def ensemble_leg(torch, rsl, stream, n=1024, steps=200, chunk=100, seed=4, cpu=True):
    import numpy as np
    rng = np.random.default_rng(seed)
    quads = {Q: rsl.Quadrature(QL, Q, min(Q - 1, 4)) for Q in (8, 16, 32, 64)}
    qs, probs, dts = [], [], []
    for _ in range(n):
        nz = int(round(np.exp(rng.uniform(np.log(256), np.log(16384)))))
        Q = int(rng.choice((8, 16, 32, 64)))
        TR = 1.0 / rng.uniform(1.1, 3.0)
        tau = float(np.exp(rng.uniform(np.log(1e-4), np.log(1.0))))
        qs.append(quads[Q])
        probs.append(rsl.make_problem(nz=nz, dtype="f32", bc="outflow", tau_r=tau, nL=1.0, TL=1.0,
                                      nR=TR ** 3, TR=TR))
        dts.append(min(0.5 / nz, 0.5 * tau))
    B = rsl.Batch(qs, probs, dts)
    B.init(stream=stream)
    B.autotune(reps=3, stream=stream)
    B.graph_step(chunk, stream=stream)
    sec = _events(torch, stream, lambda: B.graph_step(chunk, stream=stream), reps=steps // chunk)
    rc, bad = B.status(stream)
    assert rc == 0, "non-finite ensemble instance %d" % bad
    cellvel = sum(p.nz * q.V for p, q in zip(probs, qs))
    updates = 3.0 * cellvel * steps
    gbs = 32.0 * cellvel * steps / sec / 1e9
    out = {"workload": "1024 uneven Sod instances, N_z log-uniform in [256, 16384], Q_xi in {8,16,32,64}, f32, "
                       "graph replays of 100 steps, 200 steps",
            "value": updates / sec, "unit": "updates/s", "ms_per_step": sec / steps * 1e3,
            "f_bytes_per_field": 4 * cellvel,
            "variants": [B.variant(c)[0] for c in range(rsl.N_CLASSES + 1)],
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "kernel": "Sod stage kernels of all classes, 32 B per cell-velocity and step"}}
    if cpu:
        import oracle
        p0, q0 = probs[0], qs[0]
        S = oracle.Sod(oracle.VelocitySet(QL, q0.Q, min(q0.Q - 1, 4)), p0.nz, nL=1.0, TL=1.0, nR=p0.n_R, TR=p0.T_R,
                       tau_r=p0.tau_r, bc=oracle.BC_OUTFLOW, store_f32=True)
        out["cpu_baseline"] = _oracle_rate(lambda: S.run(S.init(), dts[0], 5), 3.0 * 5 * p0.nz * q0.V,
                                           "5 steps of the batch's first instance (N_z = %d, V = %d), "
                                           "single-threaded plain C" % (p0.nz, q0.V))
    return out


def learned_leg(torch, stream):
    from paper_1612_01287_amd import learned
    t0 = time.perf_counter()
    X, T = learned.generate(n_runs=2048, nz=2048, t_snaps=(0.05, 0.1, 0.15, 0.2, 0.25), seed=5, q_lo=8, q_hi=128)
    _progress("learned: %d training samples generated (%.1f s)" % (X.shape[0], time.perf_counter() - t0))
    corr, hist = learned.train(X, T, epochs=100, batch=8192, lr=2e-3, seed=1, margin=0.25)
    torch.cuda.synchronize()
    prep = time.perf_counter() - t0
    res = learned.evaluate(corr, n_inst=64, nz=2048, t_end=0.25, seed=6, q_lo=8, q_hi=128)
    out = {"workload": "learned T^{mu nu} correction: R-SLB(4;8) + network vs R-SLB(4;128), 64 instances, "
                       "N_z = 2048, t = 0.25 (scaled from 512 x 8192)",
           "samples": int(X.shape[0]), "train_and_data_s": prep, "final_loss_scaled": hist[-1]}
    out.update(res)
    if res["err_corrected"] is not None:
        out["speedup_vs_plain"] = res["t_high_order_s"] / res["t_learned_s"]
    return out


def cpu_baseline(dtype, budget_s=15.0):
    """The oracle (plain C, one thread) on a bounded sample of the same workload:
    whole RK3 steps of the R-SLB(4;100) eta/s = 0.1 instance."""
    import numpy as np
    import oracle
    vs = oracle.VelocitySet(QL, 100, NOM)
    S = oracle.Sod(vs, NZ, nL=1.0, TL=1.0, nR=0.4, TR=0.8, tau_mode=oracle.TAU_ETAS,
                   tau_aw0=0.3854 * 0.1, bc=oracle.BC_OUTFLOW, store_f32=(dtype == "f32"))
    f = S.init()
    dt = 0.5 / NZ
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        f = S.run(f, dt, 1)
        steps += 1
    el = time.perf_counter() - t0
    ups = steps * 3 * NZ * vs.V / el
    assert np.isfinite(f).all()
    return dict(value=ups, unit="updates/s", cores=1, kind="oracle",
                sample="%d RK3 steps of the R-SLB(4;100), Q_L = 3, N_z = 4096, eta/s = 0.1 instance "
                       "(single-threaded plain C)" % steps)


def copy_calibration(torch):
    n = 256 * 1024 * 1024 // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_per_copy": n * 8, "copies": 5}))


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the multi-GPU path is not built (one GPU per box)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    if a.copy_calibration:
        copy_calibration(torch)
        return
    from paper_1612_01287_amd import rsl
    B = build_batch(rsl, a.dtype)
    stream = torch.cuda.Stream()          # graph replay needs an explicit stream
    chunk = max(1, min(CHUNK, a.steps))
    with torch.cuda.stream(stream):
        if a.variants:
            for c, v in enumerate(int(x) for x in a.variants.split(",")):
                if v >= 0 and (c == rsl.N_CLASSES or B.variant(c)[0] >= 0):
                    B.set_variant(c, v)
        elif not a.no_autotune:
            # tuned on the state halfway through the run (the cost of a step
            # grows as the flows develop), then back to the initial state
            B.step(STEPS // 2, stream=stream)
            B.autotune(reps=5, stream=stream)
            B.init(stream=stream)
        variants = [B.variant(c)[0] for c in range(rsl.N_CLASSES + 1)]
        for _ in range(max(1, a.warmup // chunk)):
            B.graph_step(chunk)           # first call captures the graph of `chunk` steps
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        while done < a.steps:
            B.graph_step(chunk)
            done += chunk
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    a.steps = done
    rc, bad = B.status()
    assert rc == 0, "non-finite state in instance %d of the benchmark run" % bad
    updates_per_step = sum(3 * NZ * q.V for q in B.quads)
    value = updates_per_step * a.steps / el
    with torch.cuda.stream(stream):
        roof = kernel_roofline(torch, B, a.dtype, updates_per_step, variants, chunk, stream)
    _progress("sweep: %d steps in %.3f s" % (a.steps, el))
    out = {
        "metric": "distribution updates/s (cells x velocities x RK stages)",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": el / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": a.dtype,
        "data": "synthetic (Sod initial states, seeded parameters)",
        "config": {"workload": "Sod shock tube at finite viscosity, N_z = 4096, Q_L = 3, "
                               "Q_xi in {8,16,40,100}, eta/s in {0.01,0.1,1,10}, N_Omega = 4, 16 instances",
                   "updates_per_step": updates_per_step, "graph_steps": chunk,
                   "parallelism": "single GPU"},
        "roofline": roof,
    }
    if a.aux != "none":
        cpu = not a.no_cpu_baseline
        legs = {"c1": lambda: c1_leg(torch, rsl, stream, cpu),
                "bjorken": lambda: bjorken_leg(torch, rsl, stream, cpu=cpu),
                "ensemble": lambda: ensemble_leg(torch, rsl, stream, cpu=cpu),
                "scaled": lambda: scaled_leg(torch, rsl, stream),
                "learned": lambda: learned_leg(torch, stream)}
        out["aux"] = {}
        with torch.cuda.stream(stream):
            for k, fn in legs.items():
                if a.aux in ("all", k):
                    t0 = time.perf_counter()
                    out["aux"][k] = fn()
                    _progress("aux leg %s done (%.1f s)" % (k, time.perf_counter() - t0))
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a.dtype)
        _progress("oracle baseline done")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
