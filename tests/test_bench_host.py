"""Host logic of bench.py, without a GPU: the one-GPU guard, the kernel-form
labels and the traffic record they select, and the roofline arithmetic
(HIP events replaced by a fixed clock)."""
import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1612_01287_amd", "librsl.so")


@pytest.fixture(scope="module")
def bench():
    if not os.path.exists(LIB):
        from paper_1612_01287_amd import build
        build.build()
    import bench as mod
    return mod


def _loop_and_split(rsl):
    shapes = rsl.stage_variants()
    loop = [v for v, s in enumerate(shapes) if s[5] == 2]
    split = [v for v, s in enumerate(shapes) if s[5] == 1]
    fused = [v for v, s in enumerate(shapes) if s[5] == 0]
    return loop, split, fused


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_kernel_form_labels(bench):
    from paper_1612_01287_amd import rsl
    loop, split, fused = _loop_and_split(rsl)
    n = rsl.N_CLASSES
    per_class = [split[0], loop[0], fused[0], -1] + [-1] * (n - 4)
    assert bench.kernel_forms(per_class + [-1]) == ",".join(["s", "l", str(fused[0]), "-"] + ["-"] * (n - 4))
    assert bench.kernel_forms(per_class) == bench.kernel_forms(per_class + [-1])
    assert bench.kernel_forms(per_class + [loop[-1]]) == "all:l"
    assert bench.kernel_forms(per_class + [split[-1]]) == "all:s"


def test_traffic_record_selected_by_sources_and_forms(bench):
    """The committed counter record is used only for the kernel sources and
    launch forms it was taken with."""
    from paper_1612_01287_amd import rsl
    rec = {}
    with open(bench.TRAFFIC_FILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    loop, split, _ = _loop_and_split(rsl)
    n = rsl.N_CLASSES
    merged_loop = [split[0]] * 4 + [-1] * (n - 4) + [loop[0]]
    per_class_split = [split[0]] * 4 + [-1] * (n - 4) + [-1]
    for dt in ("f64", "f32"):
        got = bench.measured_traffic(dt, merged_loop)
        if rec.get("kernel_source_hash") == bench.kernel_source_hash() and rec.get("kernel_forms_" + dt) == "all:l":
            assert got == pytest.approx(float(rec["bytes_per_stage_group_" + dt]))
        else:
            assert got is None
        assert bench.measured_traffic(dt, per_class_split) is None


def test_roofline_arithmetic(bench):
    class Ev:
        def __init__(self, enable_timing=True):
            pass

        def record(self, stream=None):
            pass

        def synchronize(self):
            pass

        def elapsed_time(self, other):
            return 1.0                      # ms per replay of `chunk` steps

    torch = types.SimpleNamespace(cuda=types.SimpleNamespace(Event=Ev))
    replays = []

    class B:
        def graph_step(self, n, stream=None):
            replays.append(n)

    cell_vel = bench.NZ * 4 * (24 + 48 + 120 + 300)
    ups = 3 * cell_vel
    for dt, bpc in (("f64", 64), ("f32", 32)):
        replays.clear()
        r = bench.kernel_roofline(torch, B(), dt, ups, [-1] * 8, 10, None, reps=10)
        assert replays == [10] * 10
        ms = 10 * 1.0 / (3 * 10 * 10)      # one RK stage of the whole batch
        assert r["avg_launch_us"] == pytest.approx(ms * 1e3, abs=0.01)
        assert r["bytes_per_launch"] == pytest.approx(bpc / 3.0 * cell_vel)
        gbs = bpc / 3.0 * cell_vel / (ms * 1e-3) / 1e9
        assert r["achieved"] == pytest.approx(gbs, abs=0.1)
        assert r["frac"] == pytest.approx(gbs / bench.HBM_PEAK_GBS, abs=1e-4)
        assert r["peak"] == 8000.0 and r["unit"] == "GB/s" and r["bound"] == "hbm"
        assert r["traffic"] is None         # no counter record for per-class empty variants
        assert "%.0f MB" % (3 * bpc / 8 * cell_vel / 1e6) in r["residency"]
