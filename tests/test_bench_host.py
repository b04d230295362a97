"""Host-side pieces of bench.py, without a GPU: the algorithmic bytes the
roofline divides by, the counter lookup that reports HBM traffic only for the
kernel build the counters were taken on, and the refusal of more than one GPU.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("dbl,nrow,expect", [
    (True, 3, 1248), (True, 2, 864), (True, 1, 608),      # FP64 18-, 12-, 8-real
    (False, 3, 624), (False, 2, 432), (False, 1, 304),    # FP32
    (True, 13, 1248), (True, 12, 864),                    # float pairs read whole in FP64
    (False, 13, 624), (False, 12, 432),                   # and their single precision half
])
def test_dslash_bytes_per_site(dbl, nrow, expect):
    # 8 links of 18, 12 or 8 reals, the input and the output colour vector
    assert bench.dslash_bytes_per_site(dbl, nrow) == expect
    # the normal operator's epilogue reads p once more
    assert bench.dslash_bytes_per_site(dbl, nrow, "epilogue") == expect + (48 if dbl else 24)


def test_link_field_bytes_at_32_4():
    vh = 32 ** 4 // 2
    assert bench.link_field_bytes(True, 1, vh) == 4 * 2 * vh * 8 * 8       # 268 MB: 4 V links of 8 doubles
    assert bench.link_field_bytes(True, 3, vh) == 4 * 2 * vh * 18 * 8      # 604 MB
    assert bench.link_field_bytes(False, 2, vh) == 4 * 2 * vh * 12 * 4     # 201 MB
    assert bench.link_field_bytes(False, 13, vh) == 4 * 2 * vh * 18 * 4    # the pairs' single half


def test_traffic_reported_only_for_the_counted_build(tmp_path, monkeypatch):
    (tmp_path / "t.txt").write_text(
        "# counters\n"
        "kernel_isa_hash[k_dslash<double,1,PLAIN>]: 0123abcd\n"
        "traffic_bytes_per_launch[k_dslash<double,1,PLAIN>]: 352151360\n")
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    monkeypatch.setattr(bench, "built_kernel_hash", lambda k: "0123abcd")
    assert bench.read_traffic("k_dslash<double,1,PLAIN>", "t.txt") == 352151360.0
    # no counters for another kernel
    assert bench.read_traffic("k_dslash<double,3,PLAIN>", "t.txt") is None
    # the kernel changed since the counters were taken
    monkeypatch.setattr(bench, "built_kernel_hash", lambda k: "fedc3210")
    assert bench.read_traffic("k_dslash<double,1,PLAIN>", "t.txt") is None
    # no build
    monkeypatch.setattr(bench, "built_kernel_hash", lambda k: None)
    assert bench.read_traffic("k_dslash<double,1,PLAIN>", "t.txt") is None
    assert bench.read_traffic("k_dslash<double,1,PLAIN>", "missing.txt") is None


def test_committed_summary_names_the_roofline_kernel():
    path = os.path.join(bench.PROFILES, "dslash_traffic_32x32x32x32.txt")
    keys = [line.split(":", 1)[0].strip() for line in open(path) if ":" in line and not line.startswith("#")]
    assert "kernel_isa_hash[k_dslash<double,1,PLAIN>]" in keys
    assert "traffic_bytes_per_launch[k_dslash<double,1,PLAIN>]" in keys


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""
