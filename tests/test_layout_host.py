"""The FP8 operand placement and the FP4 J nibble map of the FP8 product (csrc/gsb_device.h),
compiled for the host from the kernels' own header and checked without a GPU: the placement
is a bijection onto each fragment's bytes; four consecutive spins are one word; the sixteen
spins a 16x16 MFMA result lane holds for one replica (its four row tiles) are 16 contiguous
bytes; and every FP4 nibble p pairs with the spin the placement puts at MFMA k index p
(byte p mod 16 of lane group (p / 16) mod 4 in half p / 64 of the B operand, the lane
layout of the 16x16x128 MFMA).  The GPU parity tests check the same maps end to end."""
import os
import shutil
import subprocess
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2508_17655_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

PROGRAM = textwrap.dedent(r"""
    #include "gsb_device.h"
    #include <cstdio>
    #include <vector>
    using namespace gsb;
    static int fail(const char* what, int a, int b, int c) {
      std::printf("FAIL %s %d %d %d\n", what, a, b, c);
      return 1;
    }
    int main() {
      for (int nks : {1, 2, 3, 16, 32}) {
        const int blocks = 3;  // 16-replica blocks
        std::vector<int> seen((size_t)blocks * nks * 2048, 0);
        for (int r = 0; r < 16 * blocks; ++r)
          for (int k = 0; k < 128 * nks; ++k) {
            const size_t o = fp8_elem_offset(nks, r, k);
            if (o >= seen.size()) return fail("out of range", nks, r, k);
            if (seen[o]++) return fail("two spins on one byte", nks, r, k);
            if (k % 4 && o != fp8_elem_offset(nks, r, k - (k % 4)) + (size_t)(k % 4))
              return fail("four spins not one word", nks, r, k);
          }
        // lane L of a 16x16 MFMA result holds rows 16 t + 4 L + v of replica lane % 16
        for (int row0 = 0; row0 < 128 * nks; row0 += 64)
          for (int lane = 0; lane < 64; ++lane)
            for (int t = 0; t < 4; ++t) {
              const size_t base = fp8_operand_offset(nks, row0, 16, lane);
              if (base % 16) return fail("lane bytes not aligned", nks, row0, lane);
              if (fp8_operand_offset(nks, row0 + 16 * t, 16, lane) != base + 4 * (size_t)t)
                return fail("row tiles not contiguous", nks, row0, lane);
            }
      }
      for (int p = 0; p < 128; ++p) {
        const int kk = fp4_pair_kk(p);
        const size_t want = (size_t)(p >> 6) * 1024 + (size_t)(16 * ((p >> 4) & 3)) * 16 + (size_t)(p & 15);
        if (fp8_elem_offset(1, 0, kk) != want) return fail("nibble pairs with another spin", p, kk, 0);
      }
      std::printf("OK\n");
      return 0;
    }
""")


def test_fp8_placement_and_fp4_pairing(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    src = tmp_path / "layout_check.hip"
    src.write_text(PROGRAM)
    exe = tmp_path / "layout_check"
    r = subprocess.run([HIPCC, "-O1", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                        "-packed-fp32-ops", "-I", CSRC, str(src), "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "OK", out.stdout + out.stderr
