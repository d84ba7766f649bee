"""Host-side parts of bench.py, without a GPU: the one-GPU guard, the CPU
oracle baselines and the traffic figure's validity check."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_cpu_baselines_report_their_sample():
    one = bench.cpu_baseline(4, 1024, 42)
    assert one["cores"] == 1 and one["kind"] == "oracle" and one["value"] > 0
    assert "4096 outputs" in one["sample"]
    many = bench.cpu_baseline_all_cores(8, 1024, 42, max_threads=4)
    assert 1 <= many["cores"] <= 4 and many["value"] > 0
    assert many["nproc"] >= many["cores"]
    assert "8192 outputs" in many["sample"]
    single = bench.cpu_baseline_single(2048, 42)
    assert single["cores"] == 1 and "2048 outputs" in single["sample"]
    for gen in ("mrg32k3a", "mixed"):
        assert bench.cpu_baseline_single(2048, 42, gen)["value"] > 0


def test_all_core_tasks_fill_what_one_thread_fills():
    # the threads share the oracle library; each substream must still come
    # out as it does alone
    import numpy as np
    import oracle as O
    from concurrent.futures import ThreadPoolExecutor

    def one(s):
        return O.PRNGD(O.GEN_PHILOX, 32, seed=42, stream=s).fill(4096)

    with ThreadPoolExecutor(max_workers=4) as pool:
        together = list(pool.map(one, range(16)))
    for s in range(16):
        assert np.array_equal(together[s].view(np.uint64), one(s).view(np.uint64))


@pytest.mark.parametrize("path", [bench.TRAFFIC_FILE, bench.TRAFFIC_FILE_SINGLE])
def test_traffic_is_used_only_for_the_kernel_it_was_taken_on(path, tmp_path, monkeypatch):
    with open(path) as f:
        t = json.load(f)
    stale = dict(t, kernel_sha256_16="0" * 16)
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps(stale))
    assert bench.measured_traffic(str(p)) is None
    monkeypatch.setattr(bench, "kernel_hash", lambda: t["kernel_sha256_16"])
    assert bench.measured_traffic(path) == t["bytes_per_launch"]
    assert bench.measured_traffic(str(tmp_path / "missing.json")) is None
