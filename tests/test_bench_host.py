"""Host-side logic of bench.py that needs no GPU: the one-GPU guard and the lookup of
the recorded HBM traffic of the A.D kernel."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_recorded_traffic_covers_the_default_workload_or_is_null():
    b = _bench()
    t = b.recorded_traffic(8192, 8, "fp64")
    alg = 8192 * 8192 * 8 + 2 * 8192 * 8 * 8      # A once, plus the D and R rows
    # null when the kernel source changed since the counters were taken; otherwise the
    # measured bytes can only exceed the algorithmic bytes, and by little
    assert t is None or alg <= t <= 1.1 * alg


def test_recorded_traffic_is_null_for_other_workloads_and_stale_sources(monkeypatch):
    b = _bench()
    assert b.recorded_traffic(1000, 3, "fp64") is None
    monkeypatch.setattr(b, "kernel_source_sha", lambda prec: "0" * 64)
    assert b.recorded_traffic(8192, 8, "fp64") is None


def test_kernel_source_sha_depends_on_precision():
    b = _bench()
    shas = {p: b.kernel_source_sha(p) for p in ("fp64", "fp32", "bf16x2")}
    assert len(set(shas.values())) == 3
    assert all(len(s) == 64 for s in shas.values())
