"""The GEMM's buffer-resource load path is taken only when every 32-bit byte
offset of a tile load fits (host only).

A small C++ program built with g++ against csrc/gemm_limits.hpp evaluates
the predicate on shapes the library meets: the Coulomb product reads B_ia
with a row stride of N = no*nv elements, so a 128-row tile spans 127 N
elements.  Below the limit the fast path is kept; above it (N around 2.1 M
in FP64, 4.2 M in FP32, both accepted by the problem's shape check) the
predicate must send the launch to the 64-bit-address path instead of letting
offsets wrap.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2404_17133_amd", "csrc")

# (lda, ldb, K, esize) -> expected
CASES = [
    ((160000, 160000, 800, 8), True),      # no=200 Coulomb, FP64
    ((160000, 160000, 800, 4), True),      # FP32
    ((800, 800, 208, 4), True),            # exchange W: K = nv_a padded
    ((2_100_000, 2_100_000, 800, 8), True),   # 127 * 2.1e6 * 8 = 2.13e9 < 2^31 - 1 - K
    ((2_200_000, 2_200_000, 800, 8), False),  # 127 * 2.2e6 * 8 = 2.24e9: offsets would wrap
    ((4_300_000, 64, 800, 4), False),      # the larger of the two strides decides
    ((64, 4_300_000, 800, 4), False),
    ((1 << 28, 1 << 28, 4, 2), False),     # the largest no*nv the problem accepts, BF16
    ((16, 16, (1 << 31) // 8, 8), False),  # K alone past the range
    ((-1, 16, 16, 8), False),
]


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_offset_predicate(tmp_path):
    lines = ["#include <cstdio>", '#include "gemm_limits.hpp"', "int main() {"]
    for (lda, ldb, k, es), _ in CASES:
        lines.append('  std::printf("%%d\\n", (int)rid::gemm_offsets_fit(%dLL, %dLL, %dLL, %dLL));' % (lda, ldb, k, es))
    lines += ["  return 0;", "}"]
    src = tmp_path / "lim.cpp"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "lim"
    subprocess.run(["g++", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    for (args, want), g in zip(CASES, got):
        assert bool(g) == want, args
    # boundary: the worst offset of the last accepted stride is below 2^31 - 1
    esize, k = 8, 800
    kbytes = (k * esize + 127) // 128 * 128
    ld_max = (0x7fffffff - 1 - kbytes - 128) // (127 * esize)
    assert 127 * ld_max * esize + kbytes + 128 < 0x7fffffff
