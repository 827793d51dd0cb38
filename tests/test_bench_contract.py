"""The bench's command-line contract and its HBM traffic figure (CPU only).

The traffic reported beside the roofline comes from committed rocprofv3
counter runs; it is valid only for the kernel sources and launch shape the
counters were taken on, and the bench must report null otherwise."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

# the row pass with the fused sum reads u and the sum weights and writes q:
# 3 float32 words per point of the 4096^2 field
ALGORITHMIC_BYTES = 3 * 4 * 4096 * 4096


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""   # no JSON line


def test_committed_counter_run_is_used_only_for_the_kernel_it_measured():
    """The committed counter run is consistent (its bytes are within 10% of the
    algorithmic bytes), and the bench reports it exactly when the hashed
    kernel sources are the ones it was taken on; after a source change the
    traffic figure is null until the counters are taken again."""
    with open(bench.TRAFFIC_FILE) as f:
        t = json.load(f)
    assert 0.99 <= t["hbm_bytes_per_launch"] / ALGORITHMIC_BYTES <= 1.10
    assert t["algorithmic_bytes_per_launch"] == ALGORITHMIC_BYTES
    v = bench.measured_traffic(t["kernel"], t["launch_shape"])
    if t["source_sha256"] == bench.kernel_source_hash():
        assert v == t["hbm_bytes_per_launch"]
    else:
        assert v is None


def test_traffic_is_null_for_another_kernel_shape_or_source(tmp_path, monkeypatch):
    with open(bench.TRAFFIC_FILE) as f:
        t = json.load(f)
    assert bench.measured_traffic("another_kernel", t["launch_shape"]) is None
    other_shape = [[8, 4, 2], [16, 0, 2]]
    assert other_shape != [list(x) for x in t["launch_shape"]]
    assert bench.measured_traffic(t["kernel"], other_shape) is None
    stale = tmp_path / "traffic.json"
    stale.write_text(json.dumps(dict(t, source_sha256="0" * 64)))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(stale))
    assert bench.measured_traffic(t["kernel"], t["launch_shape"]) is None
