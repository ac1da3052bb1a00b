"""The camera-batch take-up order (tile_order_pixel, a host/device function of
the library's internal header) built for the host with g++: a bijection of
the pixels for every remainder of width and height modulo 8, whose first
positions are whole 8 x 8 tiles along bands of 8 rows."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2207_05009_amd", "csrc")

PROGRAM = r"""
#include "lq_internal.h"
#include <cstdio>
#include <vector>
int main() {
    for (unsigned w = 1; w <= 41; ++w)
        for (unsigned h = 1; h <= 27; h += (h < 17 ? 1 : 5)) {
            std::vector<unsigned char> seen((size_t)w * h, 0);
            for (unsigned v = 0; v < w * h; ++v) {
                const unsigned p = lq::tile_order_pixel(v, w, h);
                if (p >= w * h || seen[p]) { std::printf("not a bijection at %u x %u, v = %u\n", w, h, v); return 1; }
                seen[p] = 1;
            }
            // whole tiles first: positions 64 t .. 64 t + 63 cover one 8 x 8 tile,
            // tiles in order along each band of 8 rows
            const unsigned tw = w / 8, th = h / 8;
            for (unsigned t = 0; t < tw * th; ++t)
                for (unsigned k = 0; k < 64; ++k) {
                    const unsigned p = lq::tile_order_pixel(64 * t + k, w, h);
                    const unsigned x = p % w, y = p / w;
                    if (x != (t % tw) * 8 + k % 8 || y != (t / tw) * 8 + k / 8) {
                        std::printf("tile layout at %u x %u, t = %u, k = %u\n", w, h, t, k);
                        return 1;
                    }
                }
        }
    const unsigned big = 2048;
    std::vector<unsigned char> seen((size_t)big * big, 0);
    for (unsigned v = 0; v < big * big; ++v) {
        const unsigned p = lq::tile_order_pixel(v, big, big);
        if (p >= big * big || seen[p]) { std::printf("not a bijection at 2048 x 2048\n"); return 1; }
        seen[p] = 1;
    }
    std::printf("ok\n");
    return 0;
}
"""


def test_tile_order_is_a_bijection_with_whole_tiles_first(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs g++ and the ROCm headers")
    src = tmp_path / "tile_order.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "tile_order"
    subprocess.run([gxx, "-std=c++17", "-O2", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", f"-I{CSRC}",
                    str(src), "-o", str(exe)], check=True, capture_output=True, timeout=120)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout
