"""The benchmark's contract, checked on the CPU: a request for more than one
GPU ends with a JSON message and a non-zero status before anything touches a
GPU; the algorithmic bytes of the K.v headline follow their definition
(49 B per node, 8 B per element); and the counter traffic is reported only
while the fine-product source is the one the counters were taken on."""

import hashlib
import json
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode != 0
    line = [l for l in out.stdout.splitlines() if l.startswith("{")][-1]
    msg = json.loads(line)
    assert "one GPU" in msg["error"]


def test_headline_bytes_definition():
    import bench

    b, nn = bench.ebe_bytes(256, 128, 128)
    assert nn == 257 * 129 * 129
    assert b == 49 * nn + 8 * 256 * 128 * 128 == 243114545


def test_counter_traffic_tracks_the_kernel_source():
    import bench

    text = open(os.path.join(ROOT, "profiles", "ebe_kv_pmc_traffic.txt")).read()
    src = os.path.join(ROOT, "paper_2205_00385_amd", "csrc", "kernels_ebe.hip")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    recorded = re.search(r"sha256\[:16\]=([0-9a-f]{16})", text).group(1)
    t = bench.pmc_traffic("256x128x128")
    if recorded == h:
        want = int(re.search(r"kv grid=256x128x128 .*traffic_bytes=(\d+)", text).group(1))
        assert t == want
        # within 10% of the algorithmic bytes: the halo re-reads of the tile
        assert 1.0 <= t / bench.ebe_bytes(256, 128, 128)[0] < 1.1
    else:
        assert t is None
    assert bench.pmc_traffic("1x1x1") is None
