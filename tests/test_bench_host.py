"""Host logic of bench.py (no GPU): the one-GPU guard, the recorded-traffic
lookup, the CPU-baseline thread count, the LDS roofline and the training-loss
summary."""
import json
import os
import subprocess
import sys
from types import SimpleNamespace

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _args(**kw):
    a = dict(colouring=3, variant=0, packing=0, block=0, group=0, tool_shape="sphere",
             tool_lift=0.0)
    a.update(kw)
    return SimpleNamespace(**a)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr


def test_recorded_traffic_only_for_the_recorded_run():
    with open(os.path.join(ROOT, "profiles", "xpbd_step_traffic.json")) as f:
        rec = json.load(f)
    wl = rec["workload"]
    same = bench.measured_traffic(wl, 1, _args(colouring=rec["colouring"]))
    if (rec["kernel_source_sha256"] == bench.source_sha("xpbd_kernels.hip")
            and rec["runtime_source_sha256"] == bench.source_sha("xpbd_runtime.hip")):
        assert same == rec["traffic_bytes_per_launch"]
    else:
        assert same is None   # taken on other sources: not reported
    for changed in (dict(tool_shape="capsule"), dict(tool_lift=1.0), dict(block=512),
                    dict(variant=2), dict(colouring=rec["colouring"] + 1)):
        assert bench.measured_traffic(wl, 1, _args(**{"colouring": rec["colouring"],
                                                      **changed})) is None
    assert bench.measured_traffic(wl, 2, _args(colouring=rec["colouring"])) is None
    assert bench.measured_traffic("another-workload", 1, _args(colouring=rec["colouring"])) is None


def test_host_threads_follow_the_share(monkeypatch):
    monkeypatch.setenv("OMP_NUM_THREADS", "3")
    n, host = bench.host_threads(64)
    assert 1 <= n <= 3 and host["threads"] == n
    assert bench.host_threads(1)[0] == 1
    monkeypatch.delenv("OMP_NUM_THREADS")
    n, host = bench.host_threads(10 ** 6)
    assert n == host["cpus_allowed"]


def test_lds_roofline_is_the_mix_of_the_two_rates():
    rd, wr, _ = bench.lds_peaks()
    total, written = 3.0e9, 1.0e9
    t_min = (total - written) / (rd * bench.CUS * bench.CLOCK) + written / (wr * bench.CUS * bench.CLOCK)
    r = bench.lds_roofline(total, written, 2 * t_min)
    assert r["frac"] == pytest.approx(0.5)
    assert r["achieved"] == pytest.approx(total / (2 * t_min) / 1e9)
    assert r["peak"] == pytest.approx(total / t_min / 1e9)


def test_loss_summary_over_equal_windows():
    losses = [4.0] * 50 + [2.0] * 100 + [1.0, 3.0] * 25
    s = bench.loss_summary(losses)
    assert s["loss_first"] == 4.0 and s["loss_first_median"] == 4.0
    assert s["loss_last"] == 2.0 and s["loss_last_median"] == 2.0
    assert s["loss_window"] == 50
