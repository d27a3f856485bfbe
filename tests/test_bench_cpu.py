"""CPU-side checks of bench.py's reporting: the roofline picks the class with the largest
device time, measured traffic is attached only to the workload and sources it was taken on,
and the script refuses more than one GPU.  No GPU is used."""

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


def _profile(bench, **classes):
    prof = {c: {"ms": 0.0, "launches": 0, "flops": 0.0, "bytes": 0.0} for c in bench.KERNELS}
    for c, (ms, launches, flops, nbytes) in classes.items():
        prof[c] = {"ms": ms, "launches": launches, "flops": flops, "bytes": nbytes}
    return prof


def test_roofline_ranks_classes_by_device_time(bench):
    prof = _profile(bench, contour_solve=(60.0, 5, 5 * 1.2885e12, 0.0), rr_gemm=(30.0, 95, 1.4e12, 0.0))
    r0 = bench.roofline_of(prof, workload="pencil")
    r1 = bench.roofline_of(prof, 1, workload="pencil")
    assert r0["kernel_class"] == "contour_solve" and r1["kernel_class"] == "rr_gemm"
    # 1.2885e12 flops per launch over 12 ms per launch
    assert r0["achieved"] == pytest.approx(1.2885e12 / 12e-3 / 1e12)
    assert r0["frac"] == pytest.approx(r0["achieved"] / 157.3)
    assert bench.roofline_of(prof, 2) is None


def test_traffic_only_for_the_measured_workload(bench):
    prof = _profile(bench, reduced_eig=(29.0, 9, 9 * 4e9, 0.0))
    tr = bench.TRAFFIC["reduced_eig"]
    on_pencil = bench.roofline_of(prof, workload="pencil")
    elsewhere = bench.roofline_of(prof, workload="batched")
    unnamed = bench.roofline_of(prof)
    assert elsewhere["traffic"] is None and unnamed["traffic"] is None
    # attached on the pencil exactly when the profiled sources are unchanged
    assert on_pencil["traffic"] == (tr["bytes"] if bench._source_unchanged(tr) else None)


def test_traffic_dropped_when_sources_change(bench, monkeypatch):
    prof = _profile(bench, contour_solve=(60.0, 5, 5 * 1.2885e12, 0.0))
    stale = dict(bench.TRAFFIC["contour_solve"], sha256_16="0000000000000000")
    monkeypatch.setitem(bench.TRAFFIC, "contour_solve", stale)
    assert bench.roofline_of(prof, workload="pencil")["traffic"] is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert p.returncode != 0
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""
