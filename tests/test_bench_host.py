"""Host logic of bench.py that needs no GPU: the one-GPU refusal, the counter summary's validity check,
and the byte models the roofline figures rest on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    # the refusal comes before anything touches a device
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in p.stdout + p.stderr


def test_traffic_is_reported_only_for_the_current_kernel_sources(tmp_path, monkeypatch):
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps({"kernel_hash": bench.kernel_hash(), "hbm_bytes_per_launch": {"spmv": 123}}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.load_traffic("spmv", 1.0) == 123
    assert bench.load_traffic("dots", 1.0) is None
    f.write_text(json.dumps({"kernel_hash": "0" * 16, "hbm_bytes_per_launch": {"spmv": 123}}))
    assert bench.load_traffic("spmv", 1.0) is None  # counters taken on other sources
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "absent.json"))
    assert bench.load_traffic("spmv", 1.0) is None


@pytest.mark.parametrize("has_val", [False, True])
def test_spmv_byte_model_counts_each_array_once(has_val):
    # a 3-node path 0-1-2 (z = 4 stored entries), FP32: row pointers 4 x 4 B, the columns 4 x 4 B,
    # the values 4 x 4 B when present, the gathered vector read once (3 x 4 B) and w written (3 x 4 B)
    want = 16 + 16 + (16 if has_val else 0) + 12 + 12
    assert bench.spmv_bytes(3, 4, 4, has_val) == want


def test_gram_schmidt_byte_models():
    # step j: the dots read w and v_0..v_j; the update reads them again and writes v~_{j+1}
    n, es = 1000, 4
    for j in (0, 5, 29):
        assert bench.dots_bytes(n, j, es) == (j + 2) * n * es
        assert bench.update_bytes(n, j, es) == (j + 3) * n * es
    assert bench.combine_bytes(n, 30, es) == 31 * n * es
