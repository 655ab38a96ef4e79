"""Host-side parts of the benchmark, on the CPU: it refuses more than one GPU
with a message, finds no profiler clock when none is loaded, and ties the
stored traffic figure to the library sources by their digest."""
from __future__ import annotations

import hashlib
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_no_profiler_clock_outside_the_profiler():
    sys.path.insert(0, ROOT)
    import bench
    assert bench._profiler_ns() is None


def test_sources_digest_covers_the_library_sources_in_order():
    sys.path.insert(0, ROOT)
    import bench
    h = hashlib.sha256()
    for name in ("ck_kernels.hip", "ck_api.hip", "ck_internal.h"):
        with open(os.path.join(ROOT, "paper_1605_05236_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    assert bench._sources_sha256() == h.hexdigest()
    # the stored traffic figure names its profile, which is committed
    assert os.path.isfile(os.path.join(ROOT, bench.MEASURED_EVICT_TRAFFIC["profile"]))
