"""bench.py's host-side contract: one GPU only, and the issued-work count of
the Gram kernel against the useful flops."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_issued_flops_cover_whole_tiles():
    # N = 1024, T = 60000: 36 upper tiles of 128 x 128 over K padded to 32
    useful = bench.FLOP_PER_PAIR_SAMPLE["split_bf16"] * (1024 * 1023 // 2) * 60000
    issued = bench.issued_flops("split_bf16", 1024, 60000)
    assert issued == bench.FLOP_PER_PAIR_SAMPLE["split_bf16"] * 36 * 128 * 128 * 60000
    assert 1.12 < issued / useful < 1.13
    # a single row still issues one whole tile; F64 tiles are 64 wide
    assert bench.issued_flops("f64", 1, 1) == bench.FLOP_PER_PAIR_SAMPLE["f64"] * 64 * 64 * 32
