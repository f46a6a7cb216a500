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


def test_traffic_record_selected_by_sources_and_forms(bench, tmp_path, monkeypatch):
    """A counter record is used only for the kernel sources and launch forms
    it was taken with."""
    from paper_1612_01287_amd import rsl
    loop, split, _ = _loop_and_split(rsl)
    n = rsl.N_CLASSES
    merged_loop = [split[0]] * 4 + [-1] * (n - 4) + [loop[0]]
    per_class_split = [split[0]] * 4 + [-1] * (n - 4) + [-1]
    rec = tmp_path / "rec.txt"
    monkeypatch.setitem(bench.TRAFFIC_FILES, "ensemble", str(rec))
    assert bench.measured_traffic("ensemble", merged_loop) is None            # no record
    rec.write_text("# comment\nbytes_per_stage: 1.5e9\nkernel_forms: all:l\nkernel_source_hash: %s\n"
                   % bench.kernel_source_hash())
    assert bench.measured_traffic("ensemble", merged_loop) == pytest.approx(1.5e9)
    assert bench.measured_traffic("ensemble", per_class_split) is None        # other launch forms
    rec.write_text("bytes_per_stage: 1.5e9\nkernel_forms: all:l\nkernel_source_hash: 0000\n")
    assert bench.measured_traffic("ensemble", merged_loop) is None            # other kernel sources


def test_committed_traffic_records_parse(bench):
    for path in bench.TRAFFIC_FILES.values():
        rec = bench.read_record(path)
        if rec:
            assert float(rec["bytes_per_stage"]) > 0 and rec["kernel_forms"] and rec["kernel_source_hash"]


def test_roofline_arithmetic(bench):
    cell_vel = 1024 * 3878 * 90
    for dt, bpc in (("f64", 64), ("f32", 32)):
        r = bench.roofline(0.3, 600, cell_vel, dt, "ensemble", [-1] * 8, "k")
        us = 0.3 / 600 * 1e6
        assert r["avg_launch_us"] == pytest.approx(us, abs=0.01)
        assert r["bytes_per_launch"] == pytest.approx(bpc / 3.0 * cell_vel)
        gbs = bpc / 3.0 * cell_vel / (us * 1e-6) / 1e9
        assert r["achieved"] == pytest.approx(gbs, abs=0.1)
        assert r["frac"] == pytest.approx(gbs / bench.HBM_PEAK_GBS, abs=1e-4)
        assert r["peak"] == 8000.0 and r["unit"] == "GB/s" and r["bound"] == "hbm"
        assert r["traffic"] is None         # no counter record for per-class empty variants


def test_timed_replays_use_stream_events(bench):
    """The headline's time comes from HIP events recorded on the launching
    stream around exactly the timed graph replays."""
    recorded = []

    class Ev:
        def __init__(self, enable_timing=True):
            pass

        def record(self, stream=None):
            recorded.append(stream)

        def synchronize(self):
            pass

        def elapsed_time(self, other):
            return 250.0

    class S:
        def synchronize(self):
            pass

    torch = types.SimpleNamespace(cuda=types.SimpleNamespace(Event=Ev))
    replays = []

    class B:
        def graph_step(self, n, stream=None):
            replays.append((n, stream))

    st = S()
    done, wall, ev = bench.timed_replays(torch, B(), 20, 50, st)
    assert done == 60 and replays == [(20, st)] * 3
    assert recorded == [st, st] and ev == pytest.approx(0.25)


def test_ensemble_recipe(bench):
    p = bench.ensemble_params()
    assert len(p) == 1024
    import numpy as np
    nz = np.array([x[0] for x in p])
    assert nz.min() >= 256 and nz.max() <= 16384 and 3000 < nz.mean() < 4800
    assert {x[1] for x in p} == {8, 16, 32, 64}
    assert all(1 / 3 - 1e-12 <= x[2] <= 1 / 1.1 + 1e-12 for x in p)
    assert all(1e-4 <= x[3] <= 1 and x[4] == min(0.5 / x[0], 0.5 * x[3]) for x in p)
