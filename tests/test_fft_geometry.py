"""Host logic of the full-box spectrum kernels (gmf_fft.hpp), compiled for the
CPU: the shell of a wave vector from a single-precision root that is a few
units of the last place off, against the integer definition
s = floor((floor(sqrt(4 n2)) + 1) / 2) (the rounding of |n| = sqrt(n2), with
no ties since 4 n2 is never an odd square); the stage radices of every line
length; the exact quotients of the small-divisor division; and the tiles of
the y and z passes, which must hold every column of a half spectrum exactly
once, with every tile of at most kFftTilePts points and every pass within
one compute unit's LDS, for all 2-3-5-smooth boxes the library accepts."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2601_03806_amd", "csrc")

DRIVER = r"""
#include "gmf_fft.hpp"
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>
using namespace gmf;
static int fail(const char* what, long a, long b, long c) {
    printf("FAIL %s %ld %ld %ld\n", what, a, b, c);
    return 1;
}
static uint64_t isqrt(uint64_t v) {
    uint64_t r = (uint64_t)std::sqrt((double)v);
    while (r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return r;
}
int main() {
    // shells from perturbed roots
    for (uint32_t n2 = 0; n2 <= 3u * 512u * 512u; ++n2) {
        const uint32_t want = (uint32_t)((isqrt(4ull * n2) + 1) / 2);
        if (shell_of(n2) != want) return fail("shell_of", n2, shell_of(n2), want);
        const float r = sqrtf((float)n2);
        for (int k = -3; k <= 3; ++k) {
            float rr = r;
            for (int i = 0; i < (k < 0 ? -k : k); ++i) rr = nextafterf(rr, k < 0 ? 0.0f : 1e30f);
            if (shell_from_root(n2, rr) != want) return fail("shell_from_root", n2, k, want);
        }
    }
    // stage radices: the run-time plan of every accepted length, the fixed plans of 2^6 .. 2^10
    std::vector<uint32_t> smooth;
    for (uint32_t L = 1; L <= kFftMaxLen; ++L) {
        FftPlan pl;
        if (!fft_plan(L, pl)) continue;
        smooth.push_back(L);
        uint32_t m = L, prod = 1;
        while (m > 1) {
            const uint32_t R = fft_next_radix(m);
            if (!(R == 16 || R == 8 || R == 4 || R == 2 || R == 3 || R == 5)) return fail("radix", L, R, 0);
            prod *= R;
            m /= R;
        }
        if (prod != L) return fail("plan product", L, prod, 0);
        const int c = fft_class(L);
        if (c != 0) {
            if (L != (1u << c) || L < 64) return fail("class", L, c, 0);
            uint32_t p = 1;
            for (int i = 0; i < 3 && p2_radix(c, i) != 0; ++i) p *= (uint32_t)p2_radix(c, i);
            if (p != L) return fail("fixed plan", L, p, 0);
        } else if ((L & (L - 1)) == 0 && L >= 64) {
            return fail("class missing", L, 0, 0);
        }
    }
    for (uint32_t d = 1; d <= 4096; ++d) {
        const SmallDiv q(d);
        for (uint32_t x = 0; x < 70000; x += (d % 7) + 1)
            if (q.div(x) != x / d) return fail("divide", x, d, q.div(x));
    }
    // tiles of random accepted boxes and of the named ones
    std::mt19937 rng(2601);
    std::vector<std::vector<uint32_t>> boxes = {{256, 256, 256}, {1024, 6, 5}, {2, 3, 1024}, {1, 1, 1}, {1, 8, 4},
                                                {16, 4, 2}, {1024, 1024, 2}, {128, 512, 64}, {96, 64, 80}, {5, 6, 3}};
    for (int i = 0; i < 600; ++i) {
        const uint32_t a = smooth[rng() % smooth.size()], b = smooth[rng() % smooth.size()];
        const uint32_t c = smooth[rng() % (i % 3 == 0 ? smooth.size() : 40)];
        boxes.push_back({a, b, c});
    }
    long checked = 0;
    for (const auto& bx : boxes) {
        const uint32_t nx = bx[0], ny = bx[1], nz = bx[2];
        if ((uint64_t)nx * ny * nz >= (1ull << 31)) continue;
        const uint32_t H = half_len(nx), Hp = half_stride(nx);
        for (uint32_t cb : {8u, 16u}) {
            for (int axis = 0; axis < 3; ++axis) {
                const uint32_t L = fft_axis_len(axis, nx, ny, nz), W = fft_tile_lines(axis, nx, ny, nz);
                if (W * L > kFftTilePts) return fail("tile points", nx, ny, nz);
                if (fft_ld(axis, nx, ny, nz, cb) < fft_phys(L - 1) + 1) return fail("ld", nx, ny, nz);
                if (fft_lds_bytes(axis, nx, ny, nz, cb, box_shells(nx, ny, nz)) > kLdsBytes) return fail("lds", nx, ny, nz);
            }
        }
        {
            const uint32_t RT = fft_x_rows(nx), T = fft_x_tiles(nx, ny, nz), rows = ny * nz;
            if ((uint64_t)T * RT < rows || (uint64_t)(T - 1) * RT >= rows) return fail("x tiles", nx, ny, nz);
            if (fft_tile_lines(0, nx, ny, nz) != kFftXKinds * RT || T != fft_pass_tiles(0, nx, ny, nz))
                return fail("x grid", nx, ny, nz);
        }
        for (int axis = 0; axis < 3; ++axis) {
            // workgroups: kFftTilesPerWG tiles each for the fixed-stage kernels, one for the others
            const uint32_t k = fft_tiles_per_wg(axis, nx, ny, nz), T = fft_pass_tiles(axis, nx, ny, nz);
            if (k != (fft_class(fft_axis_len(axis, nx, ny, nz)) ? kFftTilesPerWG[axis] : 1u)) return fail("per wg", nx, ny, axis);
            const uint32_t G = fft_tiles(axis, nx, ny, nz, 8);
            if ((uint64_t)G * k < T || (uint64_t)(G - 1) * k >= T) return fail("workgroups", nx, ny, axis);
        }
        for (int axis = 1; axis <= 2; ++axis) {
            const FftCols cols = fft_cols(axis, nx, ny, nz);
            if (cols.tiles() != fft_pass_tiles(axis, nx, ny, nz)) return fail("y z tiles", nx, ny, axis);
            const uint32_t planes = axis == 1 ? nz : ny, pstride = axis == 1 ? ny * Hp : Hp;
            std::vector<unsigned char> seen((size_t)planes * H, 0);
            for (uint32_t tile = 0; tile < cols.tiles(); ++tile) {
                const ColTile t = col_tile(cols, tile);
                const SmallDiv dcw(t.cw);
                for (uint32_t w = 0; w < cols.W; ++w) {
                    uint32_t off, plane, kx;
                    const bool ok = col_offset(t, dcw, pstride, w, off, plane, kx);
                    if (plane >= planes || kx >= H || off != plane * pstride + kx) return fail("column", nx, ny, nz);
                    if (!ok) continue;
                    if (seen[(size_t)plane * H + kx]++) return fail("twice", nx, ny, nz);
                }
            }
            for (unsigned char s : seen)
                if (s != 1) return fail("missed", nx, ny, nz);
        }
        ++checked;
    }
    printf("ok %ld\n", checked);
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc is needed to build the host driver")
def test_fft_geometry(tmp_path):
    src = tmp_path / "geom.hip"
    src.write_text(DRIVER)
    exe = tmp_path / "geom"
    # host code only: nothing here runs on a GPU
    subprocess.run(["hipcc", "-x", "hip", "--cuda-host-only", "-O2", "-std=c++17", f"-I{CSRC}", str(src), "-o",
                    str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout
