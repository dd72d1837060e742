"""Host-side checks of bench.py: the counter record parses, the digest is
stable, and more than one GPU is refused with a message."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_traffic_record_parses():
    rec = bench.traffic_record()
    assert rec is not None
    for key in ("digest", "params", "fetch_kib_per_launch", "write_kib_per_launch",
                "fetch_factor", "write_factor", "bytes_per_launch"):
        assert key in rec
    # bytes per launch is the scaled sum of the two counters (KiB -> bytes)
    want = (rec["fetch_kib_per_launch"] * rec["fetch_factor"]
            + rec["write_kib_per_launch"] * rec["write_factor"]) * 1024
    assert abs(rec["bytes_per_launch"] - want) <= 0.001 * want + 2048
    from paper_2208_04514_amd import dawn as D
    assert set(rec["params"]) <= {f for f, _ in D.Params._fields_}


def test_digest_is_stable():
    assert bench.kernel_digest() == bench.kernel_digest()
    assert len(bench.kernel_digest()) == 16


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
