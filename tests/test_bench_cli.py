"""bench.py on the CPU: a request for more than one GPU is refused with a JSON
message and exit status 2, before any device is touched; and the committed HBM
traffic table is self-consistent and reported only where it applies."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_entries_are_consistent_and_matched_by_source_and_config(monkeypatch):
    # Each committed HBM-traffic entry is the calibrated FETCH_SIZE + WRITE_SIZE (KiB per dispatch), and
    # the benchmark reports it only for the kernel source and launch configuration it was measured on.
    bench = _bench_module()
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        table = json.load(f)
    for kernel, by_workload in table.items():
        for workload, entries in by_workload.items():
            for e in entries:
                expect = 1024.0 * (e["fetch_kib_per_dispatch"] * e["fetch_scale"]
                                   + e["write_kib_per_dispatch"] * e["write_scale"])
                assert abs(e["hbm_bytes_per_launch"] - expect) <= 1e-9 * expect
                assert os.path.exists(os.path.join(ROOT, e["source"]))
                monkeypatch.setattr(bench, "kernel_source_hash", lambda h=e["m2l_hip_sha256_16"]: h)
                assert bench.load_traffic(workload, kernel, e["config"]) == e["hbm_bytes_per_launch"]
                other = dict(e["config"], m2l_rank=e["config"]["m2l_rank"] + 1)
                assert bench.load_traffic(workload, kernel, other) is None
                assert bench.load_traffic(workload + "_other", kernel, e["config"]) is None
                monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
                assert bench.load_traffic(workload, kernel, e["config"]) is None
