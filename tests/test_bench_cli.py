"""bench.py's contract on the host: more than one GPU is refused with a
message, and the byte model of one projected Krylov vector adds up."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_byte_model_and_fusion_switch(monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    b = bench.algorithmic_bytes_per_cell_fp64()
    # stencil with the divergence fused: read x and X0 (64), write y (32) and
    # the divergence (8); six transform passes of 16; correction 56
    assert b["stencil"] == 104 and b["stencil_io"] == 96 and b["fd"] == 6 * 16 and b["correction"] == 56
    assert b["stencil"] + b["fd"] + b["correction"] == 256
    monkeypatch.delenv("KV_FUSED_DIV", raising=False)
    assert bench.divergence_fused()
    monkeypatch.setenv("KV_FUSED_DIV", "0")
    assert not bench.divergence_fused()
