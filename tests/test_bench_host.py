"""Host-side logic of bench.py: the one-GPU guard, the algorithmic byte model
the roofline figures are priced with, the per-kernel fractions and the lookup
of the committed traffic summary. No GPU is used."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _unit(kernel, **one):
    args = dict(I=0, nvis=0, N=0, A=0, P=0)
    args.update(one)
    return bench.algorithmic_bytes(**args)[kernel]


def test_blend_byte_model_per_unit():
    """Per intersection one record: u, v, the conic and opacity (6 floats) and
    the 20 channels (rgb, depth, 16 features) = 104 B; per pixel the 20
    channel gradients, the opacity-sum gradient, T and the last index = 92 B;
    per visible Gaussian one gradient record of the same 104 B. The forward
    also writes a 4-byte index per intersection and, with the fused L1 term,
    reads 21 targets and writes 21 gradients per pixel."""
    assert _unit("blend_bwd", I=1) == 104
    assert _unit("blend_bwd", P=1) == 92
    assert _unit("blend_bwd", nvis=1) == 104
    assert _unit("blend_fwd", I=1) == 108
    assert _unit("blend_fwd", P=1) == 92 + 2 * 21 * 4
    assert bench.algorithmic_bytes(1, 0, 0, 0, 1, l1=False)["blend_fwd"] == 108 + 92
    # the headline launch: 153 103 intersections, 56 268 visible Gaussians, 640 x 480
    assert bench.algorithmic_bytes(153_103, 56_268, 200_000, 20_000, 307_200)["blend_bwd"] == 50_036_984


def test_byte_model_is_linear_in_the_counts():
    a = bench.algorithmic_bytes(7, 3, 11, 2, 5)
    b = bench.algorithmic_bytes(14, 6, 22, 4, 10)
    for k in a:
        assert b[k] == 2 * a[k], k


def test_roofline_entry_picks_the_binding_bound():
    # 8 kB at 8 TB/s is 1 ns; measured 2 ns -> half of HBM, HBM binds
    e = bench.roofline_entry(2e-6, 8000, {})
    assert e["bound"] == "hbm" and e["pct_hbm"] == pytest.approx(50.0) and e["pct_bound"] == pytest.approx(50.0)
    # the vector-ALU time exceeds the HBM time: the ALU bound binds
    ops = {"valu": bench.VALU_PEAK_OPS * 1e-9}  # 1 ns of vector-ALU work
    e = bench.roofline_entry(4e-6, 800, ops)  # 0.1 ns of HBM, 4 ns measured
    assert e["bound"] == "valu" and e["pct_bound"] == pytest.approx(25.0) and e["pct_hbm"] == pytest.approx(2.5)
    e = bench.roofline_entry(1e-6, 0, {"mfma": bench.MFMA_PEAK["bf16"] * 1e-9, "mfma_type": "bf16"})
    assert e["bound"] == "mfma" and e["pct_bound"] == pytest.approx(100.0)


def test_measured_traffic_only_for_the_profiled_source(tmp_path):
    src = tmp_path / "kernel.hip"
    src.write_text("// kernel source\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    prof = tmp_path / "summary.md"
    prof.write_text(f"source: {src}\nsource_sha256: {sha}\ntraffic_bytes_per_launch: 12345.0\n")
    assert bench.measured_traffic(str(prof)) == 12345.0
    src.write_text("// kernel source, changed\n")
    assert bench.measured_traffic(str(prof)) is None
    assert bench.measured_traffic(str(tmp_path / "missing.md")) is None
