"""Host-side logic of bench.py, on the CPU: the HBM traffic of the committed
rocprofv3 counter summary is reported only for the kernel source it was taken
on, the summary's figures are consistent with the algorithmic bytes, and a
request for more than one GPU is refused before anything touches a device."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")

# algorithmic bytes per launch, 2 Q s N: D3Q19 on 256^3 and on 384x192x192
ALGORITHMIC = {
    "k_step_d3q19_fp64_c3": 2 * 19 * 8 * 256 ** 3,
    "k_step_d3q19_fp32_c3": 2 * 19 * 4 * 256 ** 3,
    "k_step_d3q19_fp16_c3": 2 * 19 * 2 * 256 ** 3,
    "k_step_d3q19_fp16_c5": 2 * 19 * 2 * 384 * 192 * 192,
}


def test_kernel_digest_is_a_stable_hex_prefix():
    a = bench.kernel_digest()
    assert a == bench.kernel_digest()
    assert len(a) == 16 and int(a, 16) >= 0


def test_traffic_only_for_the_profiled_source(monkeypatch):
    data = json.load(open(TRAFFIC))
    key = "k_step_d3q19_fp32_c3"
    ent = data[key]
    monkeypatch.setattr(bench, "kernel_digest", lambda: ent["source_sha256_16"])
    assert bench._traffic(key) == ent["bytes_per_launch"]
    monkeypatch.setattr(bench, "kernel_digest", lambda: "0" * 16)
    assert bench._traffic(key) is None
    assert bench._traffic("no_such_kernel") is None


def test_committed_traffic_is_near_the_algorithmic_bytes():
    data = json.load(open(TRAFFIC))
    # the copy kernel reads and writes what it moves: FETCH_SIZE counts half
    # of the bytes read, WRITE_SIZE all of those written
    assert abs(data["_scale"]["fetch"] - 2.0) < 0.01
    assert abs(data["_scale"]["write"] - 1.0) < 0.01
    for key, alg in ALGORITHMIC.items():
        ratio = data[key]["bytes_per_launch"] / alg
        assert 1.0 <= ratio <= 1.3, (key, ratio)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stdout + r.stderr
    assert r.stdout.strip() == "" or not r.stdout.strip().startswith("{")
