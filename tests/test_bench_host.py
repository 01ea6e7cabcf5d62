"""Host-side logic of bench.py (no GPU): the one-GPU refusal, the rules under which the
committed counter record supplies `roofline.traffic`, and the algorithmic byte counts."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_2405_05213_amd.profsum import batch_kernel_sha256  # noqa: E402
from workloads import batch_instances, config  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "error" in json.loads(r.stdout.strip().splitlines()[-1])


def _record(tmp_path, **over):
    rec = {"kernel_sources_sha256": batch_kernel_sha256(), "workload": "W", "precision": "mixed_f32",
           "traffic_bytes_per_launch": 1.25e9}
    rec.update(over)
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps(rec))
    return str(p)


def test_traffic_only_for_the_profiled_kernel_and_workload(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _record(tmp_path))
    assert bench.measured_traffic("W", "mixed_f32") == 1.25e9
    assert bench.measured_traffic("W2", "mixed_f32") is None
    assert bench.measured_traffic("W", "f64") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _record(tmp_path, kernel_sources_sha256="0" * 64))
    assert bench.measured_traffic("W", "mixed_f32") is None            # kernel changed since
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic("W", "mixed_f32") is None


def test_committed_record_describes_the_headline_launch():
    if not os.path.exists(bench.TRAFFIC_FILE):
        pytest.skip("no counter record of the batch kernel committed")
    with open(bench.TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    probs = batch_instances(256, seed=5, dt=6.25e-6)
    assert rec["workload"] == bench.batch_workload(probs, 6.25e-6, 32, bench.CHECK_EVERY)
    assert rec["precision"] == "mixed_f32"
    assert rec["traffic_bytes_per_launch"] > 0 and len(rec["kernel_sources_sha256"]) == 64


def _walk_projection(p, m, s_x, sets):
    """Bytes of one projection of size m walked pass by pass: v_1 written, then per Arnoldi
    step j one operator apply (x, y, M^-1/2 and `sets` linearisation fields of 3n values,
    connectivity), reads of v_1..v_j and one write, then the combination (m reads)."""
    n3 = 3 * p.n_nodes
    L = 2 * p.n_free + 1
    apply_bytes = (2 * n3 + n3 + sets * n3) * s_x + 32 * p.n_elems
    total = L * 8
    for j in range(1, m + 1):
        total += apply_bytes + j * L * 8 + L * 8
    return total + m * L * 8


@pytest.mark.parametrize("m", [1, 5, 48])
def test_algorithmic_bytes_counts_each_vector_pass(m):
    p = config("c1")
    total = _walk_projection(p, m, 8, 0)
    assert bench.algorithmic_bytes(p, m, 1) == total
    assert bench.algorithmic_bytes(p, m, 3, projections=2) == 6 * total


def test_batch_bytes_sum_both_projections_of_every_instance():
    probs = batch_instances(3, seed=5, dt=2.5e-5)
    per = [(10, 1, 8, 1), (12, 2, 9, 1), (11, 1, 7, 2)]
    ref = sum(kc * _walk_projection(p, mc, 4, 1) + kp * _walk_projection(p, mp, 4, 2)
              for p, (mc, kc, mp, kp) in zip(probs, per))
    assert bench.batch_algorithmic_bytes(probs, per, 4) == ref
