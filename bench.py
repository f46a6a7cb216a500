"""Throughput of the R-SLB Sod step on one MI355X.

Workload (the finite-viscosity shock-tube sweep): N_z = 4096 cells on
z in [-0.5, 0.5], (T, n)_L = (1, 1), (T, n)_R = (0.8, 0.4), outflow ghosts,
Q_L = 3 radial nodes, Q_xi in {8, 16, 40, 100}, N_Omega = 4, eta/s in
{0.01, 0.1, 1, 10} with tau_AW0 = 0.3854 eta/s (relaxation-time law of
eq. Sod:tau), dt = 0.5 / N_z, f in binary64 -- sixteen instances.  One step =
one TVD-RK3 step (three fused stage kernels) of all sixteen instances.
Metric: distribution updates per second, one update = one (cell, velocity,
RK stage).

Prints one JSON line (see the repository's measurement contract).
"""
import argparse
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
CHUNK = 10          # RK3 steps per captured HIP graph


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--dtype", default="f64", choices=("f64", "f32"))
    ap.add_argument("--no-cpu-baseline", action="store_true")
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


def kernel_roofline(torch, B, dtype, updates_per_step, reps=20):
    """Average duration of the batched stage kernel (all three RK stages),
    measured with HIP events on the stream the kernels are launched on."""
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * 3 * reps)]
    k = 0
    for _ in range(reps):
        for s in (1, 2, 3):
            ev[k].record(stream)
            B.stage(s)
            ev[k + 1].record(stream)
            k += 2
    ev[-1].synchronize()
    ms = sum(ev[i].elapsed_time(ev[i + 1]) for i in range(0, len(ev), 2)) / (3 * reps)
    cell_vel = updates_per_step / 3
    bytes_per_launch = BYTES_PER_CELL_VEL_STEP[dtype] / 3.0 * cell_vel
    gbs = bytes_per_launch / (ms * 1e-3) / 1e9
    return dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(gbs / HBM_PEAK_GBS, 4), traffic=None,
                kernel="sod_batch_stage_kernel (mean of the three RK stages)", avg_launch_us=round(ms * 1e3, 2),
                bytes_per_launch=bytes_per_launch)


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


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the multi-GPU path is not built (one GPU per box)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1612_01287_amd import rsl
    torch.cuda.set_device(0)
    B = build_batch(rsl, a.dtype)
    stream = torch.cuda.Stream()          # graph replay needs an explicit stream
    chunk = max(1, min(CHUNK, a.steps))
    with torch.cuda.stream(stream):
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
        roof = kernel_roofline(torch, B, a.dtype, updates_per_step)
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
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a.dtype)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
