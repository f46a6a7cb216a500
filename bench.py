"""Throughput of the R-SLB Sod step on one MI355X.

Headline workload (the uneven shock-tube ensemble, HBM-resident): 1024 Sod
instances drawn with numpy's default_rng(4): N_z log-uniform in [256, 16384]
(rounded), Q_xi uniform in {8, 16, 32, 64} with Q_L = 3 and
N_Omega = min(Q_xi - 1, 4), (T, n)_L = (1, 1), T_R = T_L / r with r uniform in
[1.1, 3] and n_R = T_R^3, tau_r log-uniform in [1e-4, 1] (constant),
dt_i = min(0.5 / N_z, tau_r / 2), zero-gradient ghosts; f stored in binary32,
per-cell work (moments, Landau frame, tau, f^eq coefficients) in binary64.
The whole batch runs as one class in the loop form, in captured graphs of
`chunk` RK3 steps.  Before timing, the ensemble is advanced by --dev-steps
steps (so the flows have developed) and the stage-kernel shapes are tuned on
that state; timing continues from there.  One step = one TVD-RK3 step of
every instance.  Metric: distribution updates per second, one update = one
(cell, velocity, RK stage); the roofline is the HBM one, with 32 B per
cell-velocity and step (f_n read by the three stages, stage fields read
twice, three stores) over the mean duration of one RK stage of the whole
batch, from HIP events on the launching stream around the timed replays.

Prints one JSON line.  Its "aux" object carries further measurements:
  sweep    the finite-viscosity tube sweep (16 instances, N_z = 4096,
           Q_xi in {8, 16, 40, 100}, eta/s in {0.01, 0.1, 1, 10}), binary64;
           its three fields (193 MB) fit in the 256 MB last-level cache;
  c1       the near-inviscid tube (N_z = 400, R-SLB(3;8), tau_r = 1e-3,
           dt = 1.25e-3, 200 steps), launch-bound;
  bjorken  4096 Bjorken runs (T0 log-uniform in [0.5, 2] GeV, eta/s
           log-uniform in [0.01, 10], Q_xi uniform in {20..200}, Q_L = 3,
           ideal gas), a 1000-step window on the matrix cores;
  scaled   the sweep's 16 instances x 128 copies (24.8 GB in the three
           binary64 fields), out of the last-level cache;
  learned  the learned T^{mu nu} correction (training on 2.1e7 samples from
           2048 paired runs at N_z = 2048, evaluation on 64 instances);
  learned_c5 (only on request) the learned correction evaluated at full
           size: 512 instances x N_z = 8192 against R-SLB(4;128);
  learned_inloop (only on request) the correction fed back into the
           low-order populations every 0.05 (rsl_mlp_inject), trained on
           teacher-forced runs, measured against R-SLB(4;128);
  imex     the near-inviscid tube (N_z = 4096, R-SLB(4;8), tau_r = 1e-7)
           stepped implicit-explicit at dt = 0.5 dz = 1.2e3 tau_r to t = 0.4;
  ensemble_imex the headline's 1024 instances stepped implicit-explicit at
           dt = 0.5/N_z for every instance;
  vel3d    a velocity set with azimuthal nodes (Q_L = 3, Q_xi = 16, Q_phi = 8,
           N_Omega = 4: 384 nodes) over 2^20 cells of seeded states moving in
           any direction: the equilibrium written (rsl_feq3) and the moments
           with the Landau frame read back (rsl_moments3), binary32.
The oracle (plain C) is timed on the host's cores on a bounded sample of the
headline workload ("cpu_baseline"), and single-threaded beside each aux leg.
"""
import argparse
import concurrent.futures
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

QL = 3
HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6
HBARC = 0.1973269804                       # GeV fm
TAU_AW0_PER_ETAS = 5 * HBARC / (0.4 * 6.4)  # eq. Sod:tau at T_ref = 0.4 GeV, L_ref = 6.4 fm
BYTES_PER_CELL_VEL_STEP = {"f64": 64, "f32": 32}   # f_n read 3x, stage fields read 2x, written 3x
# sweep workload
SWEEP_QXI = (8, 16, 40, 100)
SWEEP_ETAS = (0.01, 0.1, 1.0, 10.0)
SWEEP_NZ = 4096
# uneven ensemble workload
ENS_N, ENS_SEED = 1024, 4
KERNEL_SOURCES = ("sod_stage.h", "sod_split.h", "sod_stage_f64.hip", "sod_stage_f32.hip", "rsl_math.h", "rsl_impl.h")
# HBM bytes per RK stage of the whole batch from rocprofv3 FETCH_SIZE / WRITE_SIZE
# counters (scaled by a plain copy's readings); valid only for the kernel
# sources and launch forms they were taken with
TRAFFIC_FILES = {"ensemble": os.path.join(ROOT, "profiles", "sod_loop_ensemble_f32_traffic.txt"),
                 "sweep": os.path.join(ROOT, "profiles", "sod_loop_sweep_f64_traffic.txt"),
                 "scaled": os.path.join(ROOT, "profiles", "sod_loop_scaled_f64_traffic.txt")}


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--dev-steps", type=int, default=1000,
                    help="steps taken before tuning and timing, so that the flows have developed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default stage-kernel variants")
    ap.add_argument("--variants", default=None,
                    help="comma-separated stage-kernel variant per velocity class (-1: empty), and an eighth "
                         "for the whole batch as one class (-1: per class); skips the autotuner")
    ap.add_argument("--aux", default="all",
                    choices=("none", "all", "sweep", "c1", "bjorken", "scaled", "learned", "learned_c5", "vel3d", "imex",
                             "ensemble_imex",
                             "learned_inloop"),
                    help="also measure the aux legs (all: every one but learned_c5 and learned_inloop), or one of them")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy five times (the reference kernel for "
                         "scaling FETCH_SIZE / WRITE_SIZE counters to bytes)")
    return ap.parse_args(argv)


def _progress(msg):
    """One line per finished part of the run, on stderr (the JSON line is stdout's only line)."""
    print("bench: " + msg, file=sys.stderr, flush=True)


# ------------------------------------------------------------------ workloads

def ensemble_params(n=ENS_N, seed=ENS_SEED):
    """(nz, Q_xi, T_R, tau_r, dt) of every instance of the uneven ensemble."""
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        nz = int(round(np.exp(rng.uniform(np.log(256), np.log(16384)))))
        Q = int(rng.choice((8, 16, 32, 64)))
        TR = 1.0 / rng.uniform(1.1, 3.0)
        tau = float(np.exp(rng.uniform(np.log(1e-4), np.log(1.0))))
        out.append((nz, Q, TR, tau, min(0.5 / nz, 0.5 * tau)))
    return out


def ensemble_batch(rsl, params, imex=False):
    """The uneven ensemble as a batch; imex: every instance at dt = 0.5/N_z,
    created for implicit-explicit steps (CFL bound only)."""
    quads = {Q: rsl.Quadrature(QL, Q, min(Q - 1, 4)) for Q in (8, 16, 32, 64)}
    qs, probs, dts = [], [], []
    for nz, Q, TR, tau, dt in params:
        qs.append(quads[Q])
        probs.append(rsl.make_problem(nz=nz, dtype="f32", bc="outflow", tau_r=tau, nL=1.0, TL=1.0,
                                      nR=TR ** 3, TR=TR, imex=imex))
        dts.append(0.5 / nz if imex else dt)
    return rsl.Batch(qs, probs, dts), qs, probs


def sweep_batch(rsl, dtype="f64", copies=1):
    quads, probs, dts = [], [], []
    for Q in SWEEP_QXI:
        quad = rsl.Quadrature(QL, Q, 4)
        for es in SWEEP_ETAS:
            for _ in range(copies):
                quads.append(quad)
                probs.append(rsl.make_problem(nz=SWEEP_NZ, dtype=dtype, bc="outflow", tau_mode="etas",
                                              tau_aw0=TAU_AW0_PER_ETAS * es, nL=1.0, TL=1.0, nR=0.4, TR=0.8))
                dts.append(0.5 / SWEEP_NZ)
    return rsl.Batch(quads, probs, dts), quads, probs


# ------------------------------------------------------------ roofline record

def kernel_source_hash():
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1612_01287_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


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


def read_record(path):
    rec = {}
    if os.path.exists(path):
        with open(path) as fh:
            for line in fh:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    rec[k.strip()] = v.strip()
    return rec


def measured_traffic(workload, variants):
    """HBM bytes per RK stage of the whole batch from the committed counter
    record of `workload`, or None when it was taken on other kernel sources
    or launch forms."""
    rec = read_record(TRAFFIC_FILES[workload])
    if not rec or rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    if rec.get("kernel_forms") != kernel_forms(variants):
        return None
    return float(rec["bytes_per_stage"])


def roofline(seconds, stages, cell_vel, dtype, workload, variants, label):
    """HBM roofline of one RK stage of the whole batch: algorithmic bytes
    (BYTES_PER_CELL_VEL_STEP / 3 per cell-velocity) over the mean stage time."""
    us = seconds / stages * 1e6
    bytes_per_launch = BYTES_PER_CELL_VEL_STEP[dtype] / 3.0 * cell_vel
    gbs = bytes_per_launch / (us * 1e-6) / 1e9
    return dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(gbs / HBM_PEAK_GBS, 4), traffic=measured_traffic(workload, variants),
                kernel=label, avg_launch_us=round(us, 2), bytes_per_launch=bytes_per_launch,
                variants=variants, kernel_forms=kernel_forms(variants), kernel_source_hash=kernel_source_hash())


def timed_replays(torch, B, chunk, nsteps, stream):
    """Wall time and HIP-event time (launching stream) of graph replays
    covering nsteps steps; returns (steps done, wall s, event s)."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    done = 0
    while done < nsteps:
        B.graph_step(chunk, stream=stream)
        done += chunk
    e1.record(stream)
    e1.synchronize()
    return done, time.perf_counter() - t0, e0.elapsed_time(e1) * 1e-3


def _events(torch, stream, fn, reps=1):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e-3


def _variants(rsl, B):
    return [B.variant(c)[0] for c in range(rsl.N_CLASSES + 1)]


def _apply_variants(rsl, B, spec):
    for c, v in enumerate(int(x) for x in spec.split(",")):
        if v >= 0 and (c == rsl.N_CLASSES or B.variant(c)[0] >= 0):
            B.set_variant(c, v)


# --------------------------------------------------------------- CPU oracle

def _host_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline_all_cores(params, budget_s=15.0):
    """The oracle (plain C, one instance per thread; ctypes releases the GIL
    during each call) on the host's cores, over the first instances of the
    ensemble, 2 RK3 steps each from the initial state, until the budget is
    spent: updates/s of the whole pool."""
    import oracle
    cores = _host_cores()
    sets = {}

    def one(i):
        nz, Q, TR, tau, dt = params[i]
        S = oracle.Sod(sets[Q], nz, nL=1.0, TL=1.0, nR=TR ** 3, TR=TR, tau_r=tau, bc=oracle.BC_OUTFLOW,
                       store_f32=True)
        S.run(S.init(), dt, 2)
        return 3.0 * 2 * nz * 3 * Q

    for Q in (8, 16, 32, 64):
        sets[Q] = oracle.VelocitySet(QL, Q, min(Q - 1, 4))
    t0 = time.perf_counter()
    updates, done = 0.0, 0
    with concurrent.futures.ThreadPoolExecutor(max_workers=cores) as pool:
        while time.perf_counter() - t0 < budget_s and done < len(params):
            n = min(cores, len(params) - done)
            updates += sum(pool.map(one, range(done, done + n)))
            done += n
    el = time.perf_counter() - t0
    return dict(value=updates / el, unit="updates/s", cores=cores, kind="oracle",
                sample="2 RK3 steps from the initial state of each of the ensemble's first %d instances, one "
                       "instance per thread on %d host threads (plain C, binary32 storage mode), %.1f s"
                       % (done, cores, el))


def cpu_baseline_one_core(params, budget_s=8.0):
    import oracle
    nz, Q, TR, tau, dt = params[0]
    S = oracle.Sod(oracle.VelocitySet(QL, Q, min(Q - 1, 4)), nz, nL=1.0, TL=1.0, nR=TR ** 3, TR=TR, tau_r=tau,
                   bc=oracle.BC_OUTFLOW, store_f32=True)
    f = S.init()
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        f = S.run(f, dt, 1)
        steps += 1
    return dict(value=3.0 * steps * nz * 3 * Q / (time.perf_counter() - t0), unit="updates/s", cores=1,
                kind="oracle", sample="%d RK3 steps of the ensemble's first instance (N_z = %d, V = %d), "
                                      "single-threaded" % (steps, nz, 3 * Q))


def _oracle_rate(fn, updates, sample):
    """Single-threaded oracle on a bounded sample: updates/s and what was run."""
    t0 = time.perf_counter()
    fn()
    return dict(value=updates / (time.perf_counter() - t0), unit="updates/s", cores=1, kind="oracle",
                sample=sample)


# ------------------------------------------------------------------ aux legs

def sweep_leg(torch, rsl, stream, cpu=True, steps=2000, chunk=10):
    """The finite-viscosity sweep, whole 2000-step run, tuned halfway through."""
    B, quads, probs = sweep_batch(rsl, "f64")
    B.init(stream=stream)
    B.step(steps // 2, stream=stream)
    B.autotune(reps=5, stream=stream)
    B.init(stream=stream)
    B.graph_step(chunk, stream=stream)
    B.init(stream=stream)
    done, wall, ev = timed_replays(torch, B, chunk, steps, stream)
    rc, bad = B.status(stream)
    assert rc == 0, "non-finite sweep instance %d" % bad
    cell_vel = sum(SWEEP_NZ * q.V for q in quads)
    variants = _variants(rsl, B)
    roof = roofline(ev, 3 * done, cell_vel, "f64", "sweep", variants,
                    "Sod loop-form stage kernel, whole batch, mean over %d graph-replayed stages" % (3 * done))
    roof["residency"] = ("the three fields (%.0f MB) fit in the 256 MB last-level cache: part of the traffic is "
                         "served there, so this is not an HBM figure" % (3 * 8 * cell_vel / 1e6))
    out = {"workload": "Sod finite-viscosity sweep: 16 instances, N_z = 4096, Q_L = 3, Q_xi in {8,16,40,100}, "
                       "eta/s in {0.01,0.1,1,10}, N_Omega = 4, f64, the whole 2000-step run",
           "value": 3.0 * cell_vel * done / wall, "unit": "updates/s", "ms_per_step": wall / done * 1e3,
           "roofline": roof}
    if cpu:
        import oracle
        S = oracle.Sod(oracle.VelocitySet(QL, 100, 4), SWEEP_NZ, nL=1.0, TL=1.0, nR=0.4, TR=0.8,
                       tau_mode=oracle.TAU_ETAS, tau_aw0=TAU_AW0_PER_ETAS * 0.1, bc=oracle.BC_OUTFLOW)
        out["cpu_baseline"] = _oracle_rate(lambda: S.run(S.init(), 0.5 / SWEEP_NZ, 10), 3.0 * 10 * SWEEP_NZ * 300,
                                           "10 RK3 steps of the R-SLB(4;100), eta/s = 0.1 instance "
                                           "(single-threaded plain C)")
    return out


def c1_leg(torch, rsl, stream, cpu=True):
    """The near-inviscid tube: N_z = 400, R-SLB(3;8), tau_r = 1e-3, dt = 1.25e-3,
    200 steps (launch-bound): updates/s of the whole run as a one-instance
    batch replayed from graphs of 10 steps (autotuned on a developed state),
    and as eager single-instance steps.  Parity: one more batch step from the
    final state against one oracle step from that state; and the final state
    against the oracle's 200-step run, beside the spread of the oracle itself
    under a one-ulp perturbation of its input (WENO5 without a regulariser
    amplifies rounding differences near the fronts)."""
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
           "variants": _variants(rsl, B),
           "one_step_rel_err_vs_oracle": rel(one, S.run(got, dt, 1)),
           "run_rel_err_vs_oracle": rel(got, ref), "oracle_one_ulp_envelope": rel(pert, ref)}
    if cpu:
        out["cpu_baseline"] = dict(value=updates / cpu_s, unit="updates/s", cores=1, kind="oracle",
                                   sample="the whole 200-step run (single-threaded plain C)")
    return out


def imex_leg(torch, rsl, stream, nz=4096, cpu=True):
    """The stiff tube stepped implicit-explicit (rsl_step_imex): N_z = 4096,
    R-SLB(4;8), Q_L = 3, tau_r = 1e-7, the paper's Sod states, equilibrium
    ghosts, dt = 0.5 dz (dt / tau = 1.2e3) to t = 0.4: updates/s (cell-velocity
    pairs per step) over the whole run, beside the step the explicit scheme's
    stiffness guard would allow.  Parity: one more step on sampled cells
    against the oracle's step of a 41-cell window around each; the plateau
    against the exact Riemann solution."""
    import numpy as np
    import oracle
    from oracle import imex, riemann
    quad = rsl.Quadrature(QL, 8, 4)
    prob = rsl.make_problem(nz=nz, bc="eq", tau_r=1e-7, nL=1.0, TL=1.0, nR=0.125, TR=0.5)
    inst = rsl.Instance(quad, prob)
    dt = 0.5 / nz
    steps = int(round(0.4 / dt))
    inst.init(stream=stream)
    inst.step_imex(dt, 10, stream=stream)
    inst.init(stream=stream)
    inst.t = 0.0
    sec = _events(torch, stream, lambda: inst.step_imex(dt, steps, stream=stream))
    M = inst.moments(stream=stream).cpu().numpy()
    st = riemann.riemann_star(1.0, 1.0, 0.125, 0.0625)
    z = -0.5 + (np.arange(nz) + 0.5) / nz
    t = inst.t
    pl = (z > st["beta_C"] * t + 0.01) & (z < st["beta_shock"] * t - 0.01)
    f = inst.f().cpu().numpy()
    inst.step_imex(dt, 1, stream=stream)
    g = inst.f().cpu().numpy()
    vs = oracle.VelocitySet(QL, 8, 4)
    err = 0.0
    for c in np.random.default_rng(5).choice(np.arange(20, nz - 20), 8, replace=False):
        W = imex.ImexSod(vs, 41, zlo=0.0, zhi=41.0 / nz, nL=1.0, TL=1.0, nR=0.125, TR=0.5,
                         tau_mode=oracle.TAU_CONST, tau_r=1e-7, bc=oracle.BC_OUTFLOW)
        want = W.step(f[:, c - 20:c + 21], dt)[:, 20]
        err = max(err, float(np.max(np.abs(g[:, c] - want)) / np.max(np.abs(want))))
    updates = float(nz) * quad.V * steps
    # C1 (N_z = 400, R-SLB(3;8), tau_r = 1e-3, dt = 1.25e-3 > tau_r) without
    # the stiffness guard, against the explicit RK3 run of the same tube
    q1 = rsl.Quadrature(QL, 8, 3)
    p1 = rsl.make_problem(nz=400, tau_r=1e-3, nL=1.0, TL=1.0, nR=0.4, TR=0.8)
    c1 = rsl.Instance(q1, p1)
    c1.init(stream=stream)
    c1.step_imex(1.25e-3, 10, stream=stream)
    c1.init(stream=stream)
    sec1 = _events(torch, stream, lambda: c1.step_imex(1.25e-3, 200, stream=stream))
    ex = rsl.Instance(q1, p1)
    ex.init(stream=stream)
    ex.step(1.25e-3, 200, stream=stream)
    Mi, Me = c1.moments(stream=stream).cpu().numpy(), ex.moments(stream=stream).cpu().numpy()
    c1_out = {"us_per_step": sec1 / 200 * 1e6, "updates_per_s": 400.0 * q1.V * 200 / sec1,
              "max_rel_diff_vs_rk3": {k: float(np.max(np.abs(Mi[:, c] - Me[:, c])) / np.max(np.abs(Me[:, c])))
                                      for k, c in (("N0", 0), ("T00", 2), ("P", 7))},
              "status": c1.status(stream=stream)}
    out = {"workload": "Sod near-inviscid, implicit-explicit: N_z = 4096, Q_L = 3, Q_xi = 8, N_Omega = 4, "
                       "tau_r = 1e-7, dt = 0.5 dz to t = 0.4 (%d steps), equilibrium ghosts, f64" % steps,
           "value": updates / sec, "unit": "updates/s", "seconds": sec, "us_per_step": sec / steps * 1e6,
           "dt_over_tau": dt / 1e-7, "explicit_dt_bound": rsl.max_dt(quad, prob)[1],
           "sampled_step_rel_err_vs_oracle": err,
           "plateau_P_rel_err": float(np.mean(M[pl, 7]) / st["PC"] - 1.0),
           "plateau_beta_rel_err": float(np.mean(M[pl, 9]) / st["beta_C"] - 1.0),
           "status": inst.status(stream=stream), "c1_tube": c1_out}
    if cpu:
        T = imex.ImexSod(vs, nz, nL=1.0, TL=1.0, nR=0.125, TR=0.5, tau_mode=oracle.TAU_CONST, tau_r=1e-7,
                         bc=oracle.BC_EQ)
        f0 = T.init()
        out["cpu_baseline"] = _oracle_rate(lambda: T.run(f0, dt, 3), 3.0 * nz * quad.V,
                                           "3 oracle IMEX steps of the whole tube from the initial state "
                                           "(numpy + scipy fsolve per cell, one core)")
    return out


def ensemble_imex_leg(torch, rsl, stream, params, dev_steps=80, steps=20, cpu=True):
    """The uneven ensemble stepped implicit-explicit at dt = 0.5/N_z for every
    instance (the explicit stage's guard takes dt = tau_r/2 below that on 169
    of them): updates/s over `steps` batch steps after `dev_steps`, instances whose status
    reports an unphysical or non-finite cell, and sampled cells of one more
    step against the oracle's step (binary32 storage) of a 41-cell window."""
    import numpy as np
    import oracle
    from oracle import imex
    B, quads, probs = ensemble_batch(rsl, params, imex=True)
    B.init(stream=stream)
    B.step_imex(dev_steps, stream=stream)
    sec = _events(torch, stream, lambda: B.step_imex(steps, stream=stream))
    bad = sum(1 for s in B.instance_status(stream=stream) if s != 0)
    rng = np.random.default_rng(7)
    picks = [int(i) for i in rng.choice(len(params), 4, replace=False)]
    before = {i: B.f(i).double().cpu().numpy() for i in picks}
    B.step_imex(1, stream=stream)
    err = 0.0
    for i in picks:
        nz, Q, TR, tau, _ = params[i]
        c = int(rng.integers(20, nz - 20))
        vs = oracle.VelocitySet(QL, Q, min(Q - 1, 4))
        W = imex.ImexSod(vs, 41, store_f32=True, zlo=0.0, zhi=41.0 / nz, nL=1.0, TL=1.0, nR=TR ** 3, TR=TR,
                         tau_mode=oracle.TAU_CONST, tau_r=tau, bc=oracle.BC_OUTFLOW)
        want = W.step(before[i][:, c - 20:c + 21], 0.5 / nz)[:, 20]
        got = B.f(i).double().cpu().numpy()[:, c]
        err = max(err, float(np.max(np.abs(got - want)) / np.max(np.abs(want))))
    updates = float(sum(nz * quads[i].V for i, (nz, *_rest) in enumerate(params))) * steps
    n_small_tau = sum(1 for nz, Q, TR, tau, dt in params if dt < 0.5 / nz)
    out = {"workload": "the uneven ensemble (same 1024 instances, f32) at dt = 0.5/N_z for every instance, "
                       "implicit-explicit (%d of them have tau_r/2 < 0.5/N_z)" % n_small_tau,
           "value": updates / sec, "unit": "updates/s", "ms_per_step": sec / steps * 1e3,
           "timed_from_step": dev_steps, "instances_with_unphysical_cells": bad, "sampled_step_rel_err_vs_oracle": err}
    del B
    return out


def scaled_leg(torch, rsl, stream, copies=128, dev_steps=1000, steps=20, chunk=10):
    """The sweep scaled out of the last-level cache: 128 copies of each of its
    16 instances (2048 instances, 24.8 GB in the three f fields, FP64), run
    for 1000 steps, tuned on that state, then 20 steps timed in graph replays
    of 10."""
    B, quads, probs = sweep_batch(rsl, "f64", copies=copies)
    B.init(stream=stream)
    B.step(dev_steps, stream=stream)
    B.autotune(reps=3, stream=stream)
    B.graph_step(chunk, stream=stream)
    done, wall, ev = timed_replays(torch, B, chunk, steps, stream)
    rc, bad = B.status(stream)
    assert rc == 0, "non-finite scaled-sweep instance %d" % bad
    cell_vel = sum(p.nz * q.V for p, q in zip(probs, quads))
    variants = _variants(rsl, B)
    roof = roofline(ev, 3 * done, cell_vel, "f64", "scaled", variants,
                    "Sod loop-form stage kernel, whole batch, mean over %d graph-replayed stages" % (3 * done))
    return {"workload": "the sweep x %d copies: %d Sod instances, N_z = 4096, Q_xi in {8,16,40,100}, "
                        "eta/s in {0.01,0.1,1,10}, f64, steps %d-%d"
                        % (copies, 16 * copies, dev_steps, dev_steps + done),
            "value": 3.0 * cell_vel * done / wall, "unit": "updates/s", "ms_per_step": wall / done * 1e3,
            "f_bytes_per_field": 8 * cell_vel, "roofline": roof}


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
                        "kernel": "bj_mfma_kernel (K^P F, 2 Q_xi^2 Q_L flop per instance and stage)",
                        "avg_launch_us": round(sec * 1e6, 1)}}
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


def vel3d_states(ncell, seed=7):
    """(ncell, 5) rows (n, T, u^x, u^y, u^z): n, T uniform in [0.3, 2], fluid
    directions uniform on the sphere, |beta| uniform in [0, 0.9]."""
    import numpy as np
    rng = np.random.default_rng(seed)
    n, T = rng.uniform(0.3, 2.0, ncell), rng.uniform(0.3, 2.0, ncell)
    d = rng.normal(size=(ncell, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    beta = rng.uniform(0.0, 0.9, ncell)
    return np.column_stack([n, T, d * (beta / np.sqrt(1.0 - beta * beta))[:, None]])


def vel3d_leg(torch, rsl, stream, ncell=1 << 20, reps=20, cpu=True):
    """rsl_feq3 (bytes: V binary32 values written and 40 B of state read per
    cell) and rsl_moments3 (V values read, 176 B written per cell), HIP events
    over `reps` launches each."""
    QL, Q, Qphi, NOm = 3, 16, 8, 4
    q3 = rsl.Quadrature3(QL, Q, Qphi, NOm)
    S = vel3d_states(ncell)
    st = torch.tensor(S, device="cuda")
    f = torch.empty((q3.V, ncell), dtype=torch.float32, device="cuda")
    rsl.feq3(q3, st, "f32", out=f, stream=stream)
    m = rsl.moments3(q3, f, ncell, stream=stream)
    stream.synchronize()
    t_feq = _events(torch, stream, lambda: rsl.feq3(q3, st, "f32", out=f, stream=stream), reps) / reps
    out_m = torch.empty_like(m)
    t_mom = _events(torch, stream, lambda: _lib_moments3(rsl, q3, f, ncell, out_m, stream), reps) / reps
    mh = out_m.cpu().numpy()
    import numpy as np
    rec_err = float(np.max(np.abs(mh[:, 14] - S[:, 0]) / S[:, 0]))
    b_feq = ncell * (q3.V * 4.0 + 40.0)
    b_mom = ncell * (q3.V * 4.0 + 8.0 * rsl.C["RSL_NMOM3"])
    gf, gm = b_feq / t_feq / 1e9, b_mom / t_mom / 1e9
    out = {"workload": "velocity set with azimuthal nodes: Q_L = 3, Q_xi = 16, Q_phi = 8, N_Omega = 4 (384 nodes), "
                       "2^20 cells, fluid directions uniform on the sphere, |beta| <= 0.9, f32",
           "value": ncell * q3.V / t_feq, "unit": "equilibrium populations/s",
           "feq3_us": round(t_feq * 1e6, 1), "moments3_us": round(t_mom * 1e6, 1),
           "moments3_values_per_s": ncell * q3.V / t_mom,
           "density_round_trip_rel_err": rec_err,
           "roofline": {"bound": "hbm", "achieved": round(gf, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(gf / HBM_PEAK_GBS, 4),
                        "kernel": "feq3_kernel<float> (384 x 4 B written + 40 B read per cell)",
                        "moments3": {"achieved": round(gm, 1), "frac": round(gm / HBM_PEAK_GBS, 4),
                                     "kernel": "moments3_kernel<float> (384 x 4 B read + 176 B written per cell)"}}}
    if cpu:
        from oracle import vel3d
        vs = vel3d.VelocitySet3(QL, Q, Qphi, NOm)
        nsamp = 2000
        out["cpu_baseline"] = _oracle_rate(lambda: [vel3d.feq3(vs, *S[c, :2], S[c, 2:]) for c in range(nsamp)],
                                           nsamp * q3.V,
                                           "the oracle's equilibrium for the first %d cells (numpy, one core)"
                                           % nsamp)
        out["cpu_baseline"]["unit"] = "equilibrium populations/s"
    return out


def learned_inloop_leg(torch, stream, n_runs=2048, nz=2048, n_inst=64, interval=0.05, n_intervals=5, epochs=100):
    from paper_1612_01287_amd import learned
    t0 = time.perf_counter()
    prog = lambda msg: _progress("learned_inloop: " + msg)
    X, T = learned.generate_inloop(n_runs=n_runs, nz=nz, interval=interval, n_intervals=n_intervals, seed=5, q_lo=8,
                                   q_hi=128, chunk=512)
    _progress("learned_inloop: %d training samples generated (%.1f s)" % (X.shape[0], time.perf_counter() - t0))
    corr, hist = learned.train(X, T, epochs=epochs, batch=8192, lr=2e-3, seed=1, margin=0.25, progress=prog)
    del X, T
    torch.cuda.empty_cache()
    res = learned.evaluate_inloop(corr, n_inst=n_inst, nz=nz, interval=interval, n_intervals=n_intervals, seed=6,
                                  q_lo=8, q_hi=128, progress=prog)
    out = {"workload": "learned T^{mu nu} correction fed back into f every %g (%d times): R-SLB(4;8) + network vs "
                       "R-SLB(4;128), %d instances, N_z = %d, t = %g; trained on %d teacher-forced runs at N_z = %d"
                       % (interval, n_intervals, n_inst, nz, interval * n_intervals, n_runs, nz),
           "train_and_data_s": time.perf_counter() - t0, "final_loss_scaled": hist[-1]}
    out.update(res)
    out["speedup_vs_plain"] = res["t_high_order_s"] / res["t_learned_s"]
    return out


def _lib_moments3(rsl, q3, f, ncell, out, stream):
    import ctypes
    rsl.check(rsl.lib().rsl_moments3(q3.handle, ctypes.c_void_p(f.data_ptr()), rsl.C["RSL_F32"], ncell,
                                     f.shape[1], ctypes.c_void_p(out.data_ptr()),
                                     ctypes.c_void_p(stream.cuda_stream)))


def learned_leg(torch, stream, n_runs=2048, nz_train=2048, n_inst=64, nz_eval=2048, epochs=100, chunk=None):
    from paper_1612_01287_amd import learned
    t0 = time.perf_counter()
    prog = lambda msg: _progress("learned: " + msg)
    X, T = learned.generate(n_runs=n_runs, nz=nz_train, t_snaps=(0.05, 0.1, 0.15, 0.2, 0.25), seed=5, q_lo=8,
                            q_hi=128, progress=prog, chunk=chunk)
    _progress("learned: %d training samples generated (%.1f s)" % (X.shape[0], time.perf_counter() - t0))
    corr, hist = learned.train(X, T, epochs=epochs, batch=8192, lr=2e-3, seed=1, margin=0.25, progress=prog)
    torch.cuda.synchronize()
    prep = time.perf_counter() - t0
    del X, T
    res = learned.evaluate(corr, n_inst=n_inst, nz=nz_eval, t_end=0.25, seed=6, q_lo=8, q_hi=128, progress=prog)
    out = {"workload": "learned T^{mu nu} correction: R-SLB(4;8) + network vs R-SLB(4;128), %d instances, "
                       "N_z = %d, t = 0.25; trained on %d paired runs at N_z = %d" % (n_inst, nz_eval, n_runs,
                                                                                      nz_train),
           "train_and_data_s": prep, "final_loss_scaled": hist[-1]}
    out.update(res)
    out["speedup_vs_plain"] = res["t_high_order_s"] / res["t_learned_s"]
    return out


def copy_calibration(torch):
    n = 256 * 1024 * 1024 // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_per_copy": n * 8, "copies": 5}))


# --------------------------------------------------------------------- main

def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the multi-GPU path (z slabs or instances per GPU) is not built",
              file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    if a.copy_calibration:
        copy_calibration(torch)
        return
    from paper_1612_01287_amd import rsl
    params = ensemble_params()
    B, qs, probs = ensemble_batch(rsl, params)
    stream = torch.cuda.Stream()          # graph replay needs an explicit stream
    chunk = max(1, min(100, a.steps))
    with torch.cuda.stream(stream):
        if a.variants:
            _apply_variants(rsl, B, a.variants)      # fixed shapes: the whole run uses them
        B.init(stream=stream)
        done_dev = 0
        while done_dev < a.dev_steps:                 # in pieces, with a progress line each
            k = min(250, a.dev_steps - done_dev)
            B.step(k, stream=stream)
            stream.synchronize()
            done_dev += k
            _progress("ensemble: %d of %d development steps" % (done_dev, a.dev_steps))
        if not a.variants and not a.no_autotune:
            B.autotune(reps=3, stream=stream)      # on the developed state; f is restored after
        variants = _variants(rsl, B)
        for _ in range(max(1, -(-a.warmup // chunk))):
            B.graph_step(chunk, stream=stream)     # the first call captures the graph of `chunk` steps
        done, wall, ev = timed_replays(torch, B, chunk, a.steps, stream)
    # instances whose flow met an unphysical cell (the scheme's own limit for
    # strong shocks at small tau_r / dz, which the oracle reaches as well);
    # they are counted, not hidden: every instance still does its full work
    unphysical = sum(1 for st in B.instance_status(stream) if st != 0)
    cell_vel = sum(p.nz * q.V for p, q in zip(probs, qs))
    updates_per_step = 3 * cell_vel
    roof = roofline(ev, 3 * done, cell_vel, "f32", "ensemble", variants,
                    "Sod loop-form stage kernel over the whole batch (one launch per RK stage, plus the "
                    "per-cell kernel at the first stage of each replay); mean over the %d timed stages"
                    % (3 * done))
    roof["residency"] = "the three binary32 fields (%.2f GB) are HBM-resident" % (3 * 4 * cell_vel / 1e9)
    _progress("ensemble: %d steps in %.3f s (%.3f s on the stream's events)" % (done, wall, ev))
    out = {
        "metric": "distribution updates/s (cells x velocities x RK stages)",
        "value": updates_per_step * done / wall,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": done,
        "warmup": a.warmup,
        "ms_per_step": wall / done * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "dtype_note": "f stored in binary32 with binary32 stencil, relaxation and RK arithmetic; moments, "
                      "Landau frame, tau and f^eq coefficients in binary64",
        "data": "synthetic (Sod initial states, seeded parameters)",
        "config": {"workload": "uneven Sod ensemble: 1024 instances (seed 4), N_z log-uniform in [256, 16384], "
                               "Q_xi in {8,16,32,64}, Q_L = 3, N_Omega = min(Q_xi - 1, 4), T_L/T_R uniform in "
                               "[1.1, 3], n_R = T_R^3, tau_r log-uniform in [1e-4, 1], dt = min(0.5/N_z, tau_r/2), "
                               "outflow ghosts, f32",
                   "updates_per_step": updates_per_step, "graph_steps": chunk,
                   "timed_from_step": a.dev_steps + max(1, -(-a.warmup // chunk)) * chunk,
                   "instances_with_unphysical_cells": unphysical,
                   "parallelism": "single GPU"},
        "roofline": roof,
    }
    if a.aux != "none":
        cpu = not a.no_cpu_baseline
        legs = {"sweep": lambda: sweep_leg(torch, rsl, stream, cpu),
                "c1": lambda: c1_leg(torch, rsl, stream, cpu),
                "bjorken": lambda: bjorken_leg(torch, rsl, stream, cpu=cpu),
                "scaled": lambda: scaled_leg(torch, rsl, stream),
                "learned": lambda: learned_leg(torch, stream),
                "vel3d": lambda: vel3d_leg(torch, rsl, stream, cpu=cpu),
                "imex": lambda: imex_leg(torch, rsl, stream, cpu=cpu),
                "ensemble_imex": lambda: ensemble_imex_leg(torch, rsl, stream, params, cpu=cpu),
                "learned_inloop": lambda: learned_inloop_leg(torch, stream),
                "learned_c5": lambda: learned_leg(torch, stream, n_runs=512, nz_train=8192, n_inst=512,
                                                  nz_eval=8192, epochs=100, chunk=128)}
        del B
        torch.cuda.empty_cache()
        out["aux"] = {}
        with torch.cuda.stream(stream):
            for k, fn in legs.items():
                if a.aux == k or (a.aux == "all" and k not in ("learned_c5", "learned_inloop")):
                    t0 = time.perf_counter()
                    out["aux"][k] = fn()
                    torch.cuda.empty_cache()
                    _progress("aux leg %s done (%.1f s)" % (k, time.perf_counter() - t0))
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_all_cores(params)
        out["cpu_baseline_one_core"] = cpu_baseline_one_core(params)
        _progress("oracle baselines done")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
