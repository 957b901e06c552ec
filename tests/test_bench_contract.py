"""Host-side parts of bench.py: the refusal of several GPUs, the issue-slot
models behind the roofline, and the reading of the committed HBM-traffic
profile (it is taken only while the kernel source still matches its hash)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_several_gpus_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)


@pytest.mark.parametrize("D", [1, 3, 16])
def test_issue_slot_models(D):
    flops, slots = bench.base_tile_model(D)
    assert flops == 3 * D + 5 and slots == 2 * D + 2 + bench.EXP_SLOTS
    f2, s2 = bench.fused_base_model(D, 10.0, 25.0)
    assert f2 == 10.0 * 3 * D + 25.0 * 5
    assert s2 == 10.0 * 2 * D + 25.0 * (2 + bench.EXP_SLOTS)
    assert bench.alu_peak_pairs_per_s(D) == bench.LANE_SLOTS_PER_S / slots


def test_traffic_profile_needs_matching_source(tmp_path):
    import hashlib
    src = tmp_path / "k.hip"
    src.write_bytes(b"kernel source")
    h = hashlib.sha256(b"kernel source").hexdigest()[:16]
    prof = tmp_path / "p.txt"
    prof.write_text("k_base.hip sha256 prefix: %s\ntraffic_bytes_per_launch base_fused_kernel<3> = 1234\n" % h)
    assert bench.measured_traffic(str(src), str(prof)) == 1234.0
    src.write_bytes(b"changed kernel source")
    assert bench.measured_traffic(str(src), str(prof)) is None
    assert bench.measured_traffic(str(src), str(tmp_path / "missing.txt")) is None
