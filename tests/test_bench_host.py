"""Host-side logic of bench.py (no GPU): the roofline line's arithmetic,
the counter traffic it reports only for the kernel source the counters were
taken from, and the refusal of more than one GPU."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def result(plain=True):
    # 16 whole-cycle steps of 2 species with 40 ms of push in all (1.25 ms a
    # launch); 7 steps without a sort with 28 ms (2.0 ms a launch)
    r = {"phases": [1.0, 2.0, 40.0, 3.0], "phase_steps": 16,
         "alive0": 4.0e8, "alive1": 3.8e8}
    if plain:
        r["plain"] = {"push_ms": 28.0, "steps": 7, "alive": 3.9e8}
    return r


def test_roofline_uses_the_plain_push_when_timed(bench):
    out = bench.roofline(1, result(), 40, 2, 5000.0)
    # 48 B x 1.95e8 particles per launch over 2.0 ms
    achieved = 48.0 * 3.9e8 / 2 / 2.0e-3 / 1e9
    assert out["avg_launch_ms"] == pytest.approx(2.0)
    assert out["avg_launch_ms_cycle"] == pytest.approx(1.25)
    assert out["achieved"] == pytest.approx(achieved, abs=0.1)
    assert out["frac"] == pytest.approx(achieved / 8000.0, abs=1e-4)
    assert out["frac_of_copy"] == pytest.approx(achieved / 5000.0, abs=1e-4)
    assert out["bound"] == "hbm" and out["peak"] == 8000.0 and out["unit"] == "GB/s"
    assert out["kernel"] == "k_push32" and "without a sort" in out["launch_timing"]


def test_roofline_falls_back_to_whole_cycles(bench):
    out = bench.roofline(0, result(plain=False), 40, 2, 5000.0)
    # FP64: 80 B x 1.95e8 particles per launch over 1.25 ms
    achieved = 80.0 * 3.9e8 / 2 / 1.25e-3 / 1e9
    assert out["avg_launch_ms"] == pytest.approx(1.25)
    assert out["achieved"] == pytest.approx(achieved, abs=0.1)
    assert out["kernel"] == "k_push64" and "whole sort cycles" in out["launch_timing"]


def test_traffic_only_for_the_profiled_source(bench, tmp_path, monkeypatch):
    for prec in (0, 1):
        path = os.path.join(ROOT, bench.COUNTER_FILE[prec])
        text = open(path).read()
        # the committed summary was taken from the committed kernel source
        assert bench.measured_traffic(prec) is not None, bench.COUNTER_FILE[prec]
        # a summary whose hash names another source gives no traffic
        stale = tmp_path / f"stale{prec}.txt"
        stale.write_text(text.replace("source_sha256: ", "source_sha256: 0"))
        monkeypatch.setitem(bench.COUNTER_FILE, prec, str(stale))
        assert bench.measured_traffic(prec) is None
        # no summary: no traffic
        monkeypatch.setitem(bench.COUNTER_FILE, prec, str(tmp_path / "absent.txt"))
        assert bench.measured_traffic(prec) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr
