"""Host-side logic of bench.py (no GPU): the one-GPU refusal, the rules under which the
committed counter record supplies `roofline.traffic`, and the algorithmic byte count."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from workloads import config  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "error" in json.loads(r.stdout.strip().splitlines()[-1])


def _record(tmp_path, **over):
    rec = {"kernel_sources_sha256": bench.kernel_sources_sha256(), "config": "c2", "precision": "f64",
           "m": 48, "k": 4, "workgroups": 80, "traffic_bytes_per_launch": 1.25e9}
    rec.update(over)
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps(rec))
    return str(p)


def test_traffic_only_for_the_profiled_kernel_and_launch(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _record(tmp_path))
    assert bench.measured_traffic("c2", "f64", 48, 4, 80) == 1.25e9
    for args in (("c3", "f64", 48, 4, 80), ("c2", "mixed_f32", 48, 4, 80), ("c2", "f64", 40, 4, 80),
                 ("c2", "f64", 48, 2, 80), ("c2", "f64", 48, 4, 96)):
        assert bench.measured_traffic(*args) is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _record(tmp_path, kernel_sources_sha256="0" * 64))
    assert bench.measured_traffic("c2", "f64", 48, 4, 80) is None      # kernel changed since
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic("c2", "f64", 48, 4, 80) is None


def test_committed_record_describes_the_headline_launch():
    with open(bench.TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    assert (rec["config"], rec["precision"]) == ("c2", "f64")
    assert rec["traffic_bytes_per_launch"] > 0 and len(rec["kernel_sources_sha256"]) == 64


@pytest.mark.parametrize("m", [1, 5, 48])
def test_algorithmic_bytes_counts_each_vector_pass(m):
    """Basis traffic counted by walking the projection: the initial read of w and write of
    v_1, then per Arnoldi step j one operator apply, reads of v_1..v_j and one write, then the
    combination (m reads, one write)."""
    p = config("c1")
    n3 = 3 * p.n_nodes
    L = 2 * n3 + 1
    apply_bytes = (2 * n3 + 2 * n3 + n3 + n3) * 8 + 32 * p.n_elems   # x, y, M^-1/2, load, conn
    total = 2 * L * 8                                                 # w read, v_1 written
    for j in range(1, m + 1):
        total += apply_bytes + j * L * 8 + L * 8
    total += m * L * 8 + L * 8
    assert bench.algorithmic_bytes(p, m, 1) == total
    assert bench.algorithmic_bytes(p, m, 3, projections=2) == 6 * total
