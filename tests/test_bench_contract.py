"""Host-side parts of bench.py: the refusal of several GPUs, the issue-slot
models behind the roofline, the reading of the committed HBM-traffic
profile (it is taken only while the kernel source still matches its hash),
and the CPU dual-tree baseline's report."""
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


def test_work_models_against_hand_counts():
    """The roofline's work model, checked against counts made by hand: a D=3
    launch with 14.65e9 kernel evaluations and 5.60e9 squared distances is
    3*3*5.60e9 + 4*14.65e9 = 1.090e11 flops; its non-packed issue slots are
    6*5.60e9 + (2 + 1.65)*14.65e9 = 8.7073e10 at the measured exp2 cost."""
    assert abs(bench.method_flops(3, 5.60e9, 14.65e9) - 1.090e11) < 1e6
    assert bench.EXP_SLOTS == 1.65
    assert abs(bench.issue_slots(3, 5.60e9, 14.65e9) - 8.70725e10) < 1e6
    # the split-float exhaustive tiles: 4 slots per dimension of a distance
    assert bench.issue_slots(16, 1.0, 0.0, 4.0) == 64.0
    # the published FP32 peak and the non-packed issue rate: 256 CU x 64 lanes x 2.4 GHz
    assert bench.LANE_SLOTS_PER_S == 256 * 64 * 2.4e9
    assert abs(2 * 2 * bench.LANE_SLOTS_PER_S / 1e12 - bench.FP32_PEAK_TFLOPS) < 0.1


def test_traffic_profile_needs_matching_source(tmp_path):
    import hashlib
    src = tmp_path / "k.hip"
    src.write_bytes(b"kernel source")
    h = hashlib.sha256(b"kernel source").hexdigest()[:16]
    prof = tmp_path / "p.txt"
    prof.write_text("k_base.hip sha256 prefix: %s\ntraffic_bytes_per_launch base_fused_kernel<3> = 1234\n"
                    "traffic_bytes_per_launch base_fused_kernel<5> = 99\n" % h)
    assert bench.measured_traffic(str(src), str(prof), "base_fused_kernel<3>") == 1234.0
    assert bench.measured_traffic(str(src), str(prof), "base_fused_kernel<5>") == 99.0
    assert bench.measured_traffic(str(src), str(prof), "base_fused_kernel<8>") is None
    src.write_bytes(b"changed kernel source")
    assert bench.measured_traffic(str(src), str(prof), "base_fused_kernel<3>") is None
    assert bench.measured_traffic(str(src), str(tmp_path / "missing.txt"), "base_fused_kernel<3>") is None


def test_cpu_dualtree_baseline_shape():
    """The CPU baseline's dual-tree leg times the oracle in both traversal
    modes on one core and reports pair-evals/s equivalent of the draw it ran
    (here a 500-point draw of the D = 3 recipe)."""
    from paper_1206_6857_amd.datagen import workload
    r = bench.cpu_dualtree_baseline(workload, D=3, scale=0.0005, leaf=32)
    wl = workload(4, D=3, scale=0.0005)
    n = wl.refs.shape[0]
    assert r["cores"] == 1 and r["kind"] == "oracle" and wl.name in r["sample"]
    for mode in ("frontier", "paper"):
        leg = r[mode]
        assert leg["unit"] == "pair-evals/s" and leg["seconds"] > 0
        assert abs(leg["value"] * leg["seconds"] - float(n) * n * len(wl.bandwidths)) < 1e-6 * n * n * 64
