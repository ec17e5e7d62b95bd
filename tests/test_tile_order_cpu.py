"""The blocked launch order of a single problem's tiles (csrc/tile_order.h),
decoded on the device from a position, against a plain enumeration of the
order it is meant to follow: blocks of 4 x 8 tiles row-major, and row-major
over the upper-triangle tiles inside each block."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1710_08037_amd", "csrc")

HARNESS = r"""
#include <cstdio>
#include "tile_order.h"
int main(int argc, char **argv) {
    for (int k = 1; k < argc; ++k) {
        int nt = atoi(argv[k]);
        int n = nt * (nt + 1) / 2;
        for (int p = 0; p < n; ++p) {
            int I = -1, J = -1;
            plv::blocked_tile(p, nt, I, J);
            printf("%d %d\n", I, J);
        }
    }
    return 0;
}
"""


def enumerate_order(nt, br=4, bc=8):
    out = []
    for bi in range(0, nt, br):
        for bj in range(0, nt, bc):
            for i in range(bi, min(nt, bi + br)):
                for j in range(bj, min(nt, bj + bc)):
                    if i <= j:
                        out.append((i, j))
    return out


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_blocked_tile_matches_the_enumerated_order():
    sizes = list(range(1, 41)) + [118, 133]
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "h.cpp")
        exe = os.path.join(d, "h")
        with open(src, "w") as fh:
            fh.write("#include <cstdlib>\n" + HARNESS)
        subprocess.run(["g++", "-O1", "-std=c++17", "-I" + CSRC, src, "-o", exe], check=True)
        out = subprocess.run([exe] + [str(s) for s in sizes], check=True, capture_output=True, text=True).stdout
    got = [tuple(map(int, line.split())) for line in out.splitlines()]
    want = [ij for nt in sizes for ij in enumerate_order(nt)]
    assert got == want
    # every upper tile exactly once per size
    k = 0
    for nt in sizes:
        n = nt * (nt + 1) // 2
        assert sorted(got[k:k + n]) == sorted((i, j) for i in range(nt) for j in range(i, nt))
        k += n
