// gmf_fft.hpp -- definitions shared by the host runtime and the kernels of the
// full-box shell spectra (Results section: structure factors from a normalised
// FFT of the whole box, averaged over shells of equal |k|).
//
// On a sampling step the six sampled fields (drho, jx, jy, jz, pdiag, poff)
// and jsum = jx + jy + jz are transformed by batched line FFTs (Stockham,
// radices 16, 8, 4, 2, 3, 5; the first stage reads its line from global
// memory into registers, the last one hands its outputs on from registers):
//   x pass   two real fields packed as one complex line, transformed, and
//            separated into the half spectra kx = 0 .. floor(nx / 2) of both
//            (a real field has F(-k) = conj F(k), so the other half is
//            redundant): each row as drho + i pdiag, poff + i jx, jy + i jz,
//            every field read once, and jsum = jx + jy + jz from the half
//            spectra of its three parts;
//   y pass   in place on each half spectrum, tiles of W consecutive columns;
//   z pass   the same tiles along z, followed in the same workgroup by the
//            power at every wave vector, summed into the shells
//            s = round(|n|) of that field's spectrum.
// The columns kx of a half spectrum that do not fill a whole tile of W (the
// kx = nx / 2 column for even nx, mostly) are gathered from several planes
// into tiles of their own, so every tile has W columns of work.
// The transforms run in the kernel precision (complex FP32 for the FP32
// path, FP64 for FP64); the shell sums are integer fixed-point sums.  Box
// lengths must have no prime factor above 5 and be at most kFftMaxLen.
#pragma once

#include <math.h>
#include <stdint.h>

#include "gmf_device.hpp"

namespace gmf {

constexpr uint32_t kFftMaxLen = 1024;     // longest line
constexpr uint32_t kFftTilePts = 4096;    // points of a tile: sixteen per thread
constexpr uint32_t kLdsBytes = 160u * 1024u;   // LDS of a gfx950 compute unit
constexpr int kFftMaxStages = 12;
constexpr uint32_t kFftXKinds = 3;        // x-pass lines per row: drho + i pdiag, poff + i jx, jy + i jz
constexpr int kFftFields = 7;             // half spectra: drho, jx, jy, jz, pdiag, poff, jsum = jx + jy + jz
constexpr uint32_t kFftPad = 16;          // half-spectrum rows are padded to a multiple of 16 columns
constexpr uint32_t kBinCopies = 64;       // copies of the integer shell bins (workgroup b adds to copy b mod 64)
// tiles of a workgroup of the kernels with fixed stages, per pass (x, y, z)
constexpr uint32_t kFftTilesPerWG[3] = {4, 1, 4};

struct FftPlan {
    int nst;
    int radix[kFftMaxStages];
};

// Prime factorisation check of a line length L: true when L has no prime
// factor above 5 and 1 <= L <= kFftMaxLen (radices 4, 2, 3, 5 listed).
__host__ __device__ inline bool fft_plan(uint32_t L, FftPlan& p)
{
    p.nst = 0;
    if (L < 1 || L > kFftMaxLen) return false;
    uint32_t m = L;
    const int radices[4] = {4, 2, 3, 5};
    for (int q = 0; q < 4; ++q) {
        const uint32_t R = (uint32_t)radices[q];
        while (m % R == 0 && p.nst < kFftMaxStages) {
            p.radix[p.nst++] = (int)R;
            m /= R;
        }
    }
    return m == 1;
}

// Radix of the next stage of a line whose untransformed part has length m:
// 16, 8, 4, 2, 3 or 5 (m itself when m is 1).
__host__ __device__ inline uint32_t fft_next_radix(uint32_t m)
{
    if (m % 16 == 0) return 16;
    if (m % 8 == 0) return 8;
    if (m % 4 == 0) return 4;
    if (m % 2 == 0) return 2;
    if (m % 3 == 0) return 3;
    if (m % 5 == 0) return 5;
    return m;
}

// Columns kx = 0 .. floor(nx / 2) of the half spectra, and the padded row
// length (whole 128-byte segments of FP32 complex values).
__host__ __device__ inline uint32_t half_len(uint32_t nx) { return nx / 2 + 1; }
__host__ __device__ inline uint32_t half_stride(uint32_t nx) { return (half_len(nx) + kFftPad - 1) / kFftPad * kFftPad; }

__host__ __device__ inline uint32_t fft_axis_len(int axis, uint32_t nx, uint32_t ny, uint32_t nz)
{
    return axis == 0 ? nx : (axis == 1 ? ny : nz);
}

// LDS slot of point p of a line: one pad slot after every 16 points, so the
// first stage's radix-16 outputs (16 consecutive points per thread) spread
// over the banks.
__host__ __device__ inline uint32_t fft_phys(uint32_t p) { return p + (p >> 4); }

// Lines of a tile: x pass kFftXKinds lines for each of its rows; y and z
// passes W columns of the half spectra (W <= H).
__host__ __device__ inline uint32_t fft_x_rows(uint32_t nx);
__host__ __device__ inline uint32_t fft_tile_lines(int axis, uint32_t nx, uint32_t ny, uint32_t nz)
{
    if (axis == 0) return kFftXKinds * fft_x_rows(nx);
    const uint32_t L = fft_axis_len(axis, nx, ny, nz);
    uint32_t W = kFftTilePts / L;
    if (W < 1u) W = 1u;
    if (W > half_len(nx)) W = half_len(nx);
    return W;
}

// LDS row length of a tile's lines (complex values of cbytes bytes): the
// padded line, rounded for lines of at least 64 points so that the lanes of a
// stage meet different banks.  The y and z passes give consecutive lanes
// consecutive lines, the x pass consecutive butterflies of one line.
__host__ __device__ inline uint32_t fft_ld(int axis, uint32_t nx, uint32_t ny, uint32_t nz, uint32_t cbytes)
{
    const uint32_t L = fft_axis_len(axis, nx, ny, nz);
    const uint32_t len = fft_phys(L - 1) + 1;
    if (L < 64) return len;
    const uint32_t S = 256u / cbytes;   // values of one pass over the 64 banks
    const uint32_t W = fft_tile_lines(axis, nx, ny, nz);
    uint32_t target = 1;
    if (axis == 0) {
        const uint32_t nb = L / fft_next_radix(L);   // lanes of one line in the first stage
        if (fft_next_radix(L) == 16 && nb < S && S % nb == 0) target = nb;
    } else if (W < S && S % W == 0) {
        target = S / W;
    }
    return len + (target + S - len % S) % S;
}

// Tiling of the half-spectrum columns of one field for the y (axis 1) and z
// (axis 2) passes: `full` whole tiles of W columns in each plane (z planes for
// the y pass, y rows for the z pass), then the last `rem` columns of every
// plane, `group` planes to a tile.
struct FftCols {
    uint32_t W, full, rem, group, planes;
    __host__ __device__ uint32_t tiles() const
    {
        return full * planes + (rem ? (planes + group - 1) / group : 0u);
    }
};

__host__ __device__ inline FftCols fft_cols(int axis, uint32_t nx, uint32_t ny, uint32_t nz)
{
    FftCols c;
    c.W = fft_tile_lines(axis, nx, ny, nz);
    const uint32_t H = half_len(nx);
    c.full = H / c.W;
    c.rem = H - c.full * c.W;
    c.group = c.rem ? c.W / c.rem : 1u;
    c.planes = axis == 1 ? nz : ny;
    return c;
}

// x pass: rows per tile (kFftXKinds lines each) and tiles of a box.
__host__ __device__ inline uint32_t fft_x_rows(uint32_t nx)
{
    const uint32_t NL = kFftTilePts / nx;
    return NL >= kFftXKinds ? NL / kFftXKinds : 1u;
}
__host__ __device__ inline uint32_t fft_x_tiles(uint32_t nx, uint32_t ny, uint32_t nz)
{
    const uint32_t RT = fft_x_rows(nx);
    return (ny * nz + RT - 1) / RT;
}

// Kernel class of a line of length L: log2 L for a power of two 64 .. 1024
// (kernels with fixed stages), else 0 (stages chosen at run time).  Each
// replica's lines always go through the kernels of their own class, so a
// replica's spectra do not depend on the other replicas of its context.
__host__ __device__ inline int fft_class(uint32_t L)
{
    for (int p = 6; p <= 10; ++p)
        if (L == (1u << p)) return p;
    return 0;
}

// Tiles of one pass over one field (the x pass: over the box), and the
// workgroups that take them: for the kernels with fixed stages up to
// kFftTilesPerWG[axis] tiles each, G apart (G the number of workgroups; the
// next tile's inputs are loaded while one is transformed), else one each.
__host__ __device__ inline uint32_t fft_pass_tiles(int axis, uint32_t nx, uint32_t ny, uint32_t nz)
{
    return axis == 0 ? fft_x_tiles(nx, ny, nz) : fft_cols(axis, nx, ny, nz).tiles();
}
__host__ __device__ inline uint32_t fft_tiles_per_wg(int axis, uint32_t nx, uint32_t ny, uint32_t nz)
{
    return fft_class(fft_axis_len(axis, nx, ny, nz)) > 0 ? kFftTilesPerWG[axis] : 1u;
}
// Workgroups of one pass over one replica (y and z passes: per field, grid.y
// runs over the fields).
__host__ __device__ inline uint32_t fft_tiles(int axis, uint32_t nx, uint32_t ny, uint32_t nz, uint32_t cbytes)
{
    (void)cbytes;
    const uint32_t k = fft_tiles_per_wg(axis, nx, ny, nz);
    return (fft_pass_tiles(axis, nx, ny, nz) + k - 1) / k;
}

// Dynamic LDS of a pass with complex values of cbytes bytes: the tile's
// lines as rows of fft_ld values, then the L twiddles; the z pass adds,
// 8-byte aligned, its integer shell bins.
__host__ __device__ inline uint32_t fft_lds_bytes(int axis, uint32_t nx, uint32_t ny, uint32_t nz, uint32_t cbytes,
                                                  uint32_t nshell)
{
    const uint32_t L = fft_axis_len(axis, nx, ny, nz);
    const uint32_t W = fft_tile_lines(axis, nx, ny, nz);
    uint32_t b = cbytes * (W * fft_ld(axis, nx, ny, nz, cbytes) + L);
    if (axis == 2) b = (b + 7u) / 8u * 8u + 8u * nshell;
    return b;
}

// Shell of a wave vector with |n|^2 = n2 > 0: s = round(|n|), i.e.
// (2s - 1)^2 <= 4 n2 < (2s + 1)^2 (4 n2 is even, so there are no ties).
__host__ __device__ inline uint32_t shell_of(uint64_t n2)
{
    uint64_t s = (uint64_t)(sqrt((double)n2) + 0.5);
    while ((2 * s + 1) * (2 * s + 1) <= 4 * n2) ++s;
    while (s > 0 && (2 * s - 1) * (2 * s - 1) > 4 * n2) --s;
    return (uint32_t)s;
}

// The same for n2 < 2^24 from an approximate root r of n2, within a few
// units of the last place of sqrt(n2) in single precision: rounding r is off
// by at most one shell, which one comparison either way corrects.
__host__ __device__ inline uint32_t shell_from_root(uint32_t n2, float r)
{
    uint32_t s = (uint32_t)(r + 0.5f);
    const uint32_t n4 = 4u * n2;
    if ((2u * s + 1u) * (2u * s + 1u) <= n4) ++s;
    else if (s > 0u && (2u * s - 1u) * (2u * s - 1u) > n4) --s;
    return s;
}

// Quotients of small non-negative integers by a divisor known only at run
// time: with m = ceil(2^32 / d) = floor((2^32 - 1) / d) + 1,
// floor(x m / 2^32) = floor(x / d) whenever x d < 2^32 (here x, d < 2^16).
struct SmallDiv {
    uint32_t d, m;
    __host__ __device__ explicit SmallDiv(uint32_t dd) : d(dd), m(dd > 1u ? 0xffffffffu / dd + 1u : 0u) {}
    __host__ __device__ uint32_t div(uint32_t x) const
    {
#ifdef __HIP_DEVICE_COMPILE__
        return d > 1u ? __umulhi(x, m) : x;
#else
        return d > 1u ? (uint32_t)(((uint64_t)x * m) >> 32) : x;
#endif
    }
};

// Columns of a y- or z-pass tile.  A whole tile holds W consecutive columns
// kx0 .. kx0 + W - 1 of one plane; a remainder tile holds the last `rem`
// columns of up to `group` consecutive planes.  Column w is at plane
// plane0 + w / cw, kx = kx0 + w mod cw; columns of planes past gcount are
// empty (loads read the tile's first column, nothing is stored).
struct ColTile {
    uint32_t plane0, kx0, cw, gcount;
};

__host__ __device__ inline ColTile col_tile(const FftCols& c, uint32_t tile)
{
    ColTile t;
    const uint32_t nfull = c.full * c.planes;
    if (tile < nfull) {
        t.plane0 = tile / c.full;
        t.kx0 = (tile - t.plane0 * c.full) * c.W;
        t.cw = c.W;
        t.gcount = 1;
    } else {
        t.plane0 = (tile - nfull) * c.group;
        t.kx0 = c.full * c.W;
        t.cw = c.rem;
        t.gcount = c.planes - t.plane0 < c.group ? c.planes - t.plane0 : c.group;
    }
    return t;
}

// Column w of a tile in a half spectrum whose planes are pstride values
// apart: its plane, kx and offset (the tile's first column for an empty one);
// false for an empty column.
__host__ __device__ inline bool col_offset(const ColTile& t, const SmallDiv& dcw, uint32_t pstride, uint32_t w,
                                           uint32_t& off, uint32_t& plane, uint32_t& kx)
{
    const uint32_t g = dcw.div(w);
    const bool ok = g < t.gcount;
    plane = t.plane0 + (ok ? g : 0u);
    kx = t.kx0 + (ok ? w - g * t.cw : 0u);
    off = plane * pstride + kx;
    return ok;
}

// Stage radices of a line of 2^P points, P = 6 .. 10 (0 past the last stage)
__host__ __device__ constexpr int p2_radix(int P, int i)
{
    return i == 0 ? 16 : P == 6 ? (i == 1 ? 4 : 0) : P == 7 ? (i == 1 ? 8 : 0) : P == 8 ? (i == 1 ? 16 : 0)
         : P == 9 ? (i == 1 ? 8 : i == 2 ? 4 : 0) : (i == 1 ? 16 : i == 2 ? 4 : 0);
}

// Signed integer frequency of FFT output index i of a line of length L: n in [-L/2, L/2).
__host__ __device__ inline int32_t signed_freq(uint32_t i, uint32_t L)
{
    return 2 * i < L ? (int32_t)i : (int32_t)i - (int32_t)L;
}

// Shells 0 .. smax of a box, smax = round(sqrt(sum_a floor(L_a / 2)^2)).
__host__ __device__ inline uint32_t box_shells(uint32_t nx, uint32_t ny, uint32_t nz)
{
    const uint64_t a = nx / 2, b = ny / 2, c = nz / 2;
    const uint64_t n2 = a * a + b * b + c * c;
    return (n2 == 0 ? 0u : shell_of(n2)) + 1u;
}


// Read-bandwidth reference (gmf_read_probe): one plain read of `bytes` (a
// multiple of 16) from src; *flag is set if a thread's sum is not finite.
hipError_t launch_read_probe(const void* src, uint64_t bytes, uint32_t* flag, hipStream_t s);

}  // namespace gmf
