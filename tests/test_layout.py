"""The layout of a length class's codes (csrc/layout.h), checked on the host with
g++: for every stride and tile size, code_index maps (slot, code) one to one onto
the class's array, a tile's codes fill one block of T * S, and each group of four
codes, and each group of a whole tile, is one contiguous run."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROGRAM = r"""
#include "layout.h"
#include <cstdio>
#include <vector>
using namespace gss;
int main() {
    for (uint32_t s = 2; s <= 9; ++s)
        for (uint32_t t = 0; t <= 6; ++t) {
            const uint64_t S = 1ull << s, T = 1ull << t, cap = 3 * T;
            std::vector<int> seen(cap * S, 0);
            for (uint64_t slot = 0; slot < cap; ++slot)
                for (uint32_t k = 0; k < S; ++k) {
                    const uint64_t x = code_index(slot, k, s, t);
                    if (x >= cap * S || seen[x]++) { std::printf("not one to one s=%u t=%u\n", s, t); return 1; }
                    const uint64_t tile = slot / T;  // the tile's block
                    if (x / (T * S) != tile) { std::printf("outside its tile s=%u t=%u\n", s, t); return 1; }
                    // a group of four: consecutive codes
                    if (code_index(slot, k, s, t) != code_index(slot, k & ~3u, s, t) + (k & 3)) {
                        std::printf("group not contiguous s=%u t=%u\n", s, t); return 1;
                    }
                    // group g of the tile's clauses side by side: clause j at offset 4 j
                    if (code_index(slot, k & ~3u, s, t) != code_index(tile * T, k & ~3u, s, t) + 4 * (slot % T)) {
                        std::printf("tile group not contiguous s=%u t=%u\n", s, t); return 1;
                    }
                }
        }
    std::printf("ok\n");
    return 0;
}
"""


def test_code_layout_is_a_tiled_bijection(tmp_path):
    src = tmp_path / "layout_check.cpp"
    exe = tmp_path / "layout_check"
    src.write_text(PROGRAM)
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", os.path.join(ROOT, "paper_2012_03119_amd", "csrc"), str(src),
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout
