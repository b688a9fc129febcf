"""Host logic of bench.py (no GPU): the one-GPU guard, the algorithmic byte model of the hop
and the lookup of the committed hardware-counter summary."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


@pytest.mark.parametrize("prec,Ls,want", [
    ("fp64", 16, 456.0), ("fp64", 32, 420.0),   # (48 + 144/Ls) words of 8 bytes
    ("fp32", 16, 228.0), ("fp32", 32, 210.0),
    ("fp16", 32, 105.0 + 8.0),                  # 2-byte words plus the FP32 norms of in and out
])
def test_hop_bytes_per_site(prec, Ls, want):
    """Input and output spinor once, the 8 links of a 4D site shared by its Ls slices."""
    assert bench.hop_bytes_per_site(prec, Ls) == pytest.approx(want)


def test_measured_traffic_needs_the_current_kernel_source(tmp_path, monkeypatch):
    kern = "hop_kernel<dwf::P16, 32, 1, false, false, 3, false, false, false>"
    f = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic(kern) is None  # no summary
    d = {"kernel_source_sha256_16": bench.kernel_source_hash(), "kernels": {kern: {"hbm_bytes_per_launch": 4.0e9}}}
    f.write_text(json.dumps(d))
    assert bench.measured_traffic(kern) == 4.0e9
    assert bench.measured_traffic("hop_kernel<dwf::P64, 32>") is None  # kernel not in the summary
    d["kernel_source_sha256_16"] = "0" * 16
    f.write_text(json.dumps(d))
    assert bench.measured_traffic(kern) is None  # taken on another kernel source
