// gmf_fft.hpp -- definitions shared by the host runtime and the kernels of the
// full-box shell spectra (Results section: structure factors from a normalised
// FFT of the whole box, averaged over shells of equal |k|).
//
// On a sampling step the six sampled fields are packed into three complex
// arrays (drho + i jx, jy + i jz, pdiag + i poff), transformed along x, y and
// z by batched line FFTs (mixed-radix Stockham, radices 4, 2, 3, 5, one line
// per LDS row), unpacked per wave vector with the symmetry of real fields, and
// binned into shells s = round(|n|).  Box lengths must have no prime factor
// above 5 and be at most kFftMaxLen.
#pragma once

#include <stdint.h>

#include "gmf_device.hpp"

namespace gmf {

constexpr uint32_t kFftMaxLen = 1024;   // longest line
constexpr uint32_t kFftPoints = 2048;   // complex points of one workgroup tile
constexpr int kFftMaxStages = 12;
constexpr int kFftArrays = 3;           // packed field pairs
constexpr uint32_t kBinPoints = 16 * kBlock;   // wave vectors per workgroup of the binning kernel

struct FftPlan {
    int nst;
    int radix[kFftMaxStages];
};

// Stage radices of a line of length L: 4s, then 2, 3s, 5s (the Stockham
// stages accept them in any order).  False when L has another prime factor or
// is out of range.
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

// Lines per workgroup tile of the pass along `axis` (0: x, 1: y, 2: z).  The
// y and z passes take W consecutive x columns, so W <= nx.
__host__ __device__ inline uint32_t fft_tile_lines(int axis, uint32_t L, uint32_t nx)
{
    uint32_t W = kFftPoints / (L < 2u ? 2u : L);   // L = 1: keep the padded rows within the LDS
    if (axis != 0 && W > nx) W = nx;
    return W;
}

__host__ __device__ inline uint32_t fft_axis_len(int axis, uint32_t nx, uint32_t ny, uint32_t nz)
{
    return axis == 0 ? nx : (axis == 1 ? ny : nz);
}

// Workgroups of one pass over one packed array of a replica.
__host__ __device__ inline uint32_t fft_tiles(int axis, uint32_t nx, uint32_t ny, uint32_t nz)
{
    const uint32_t L = fft_axis_len(axis, nx, ny, nz);
    const uint32_t W = fft_tile_lines(axis, L, nx);
    if (axis == 0) return (ny * nz + W - 1) / W;
    const uint32_t per = (nx + W - 1) / W;
    return per * (axis == 1 ? nz : ny);
}

// Dynamic LDS of a pass: W padded rows of L + 1 values, then L twiddles.
__host__ __device__ inline uint32_t fft_lds_bytes(int axis, uint32_t nx, uint32_t ny, uint32_t nz)
{
    const uint32_t L = fft_axis_len(axis, nx, ny, nz);
    const uint32_t W = fft_tile_lines(axis, L, nx);
    return 16u * (W * (L + 1) + L);
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

// Signed integer frequency of FFT output index i of a line of length L: n in [-L/2, L/2).
__host__ __device__ inline int32_t signed_freq(uint32_t i, uint32_t L)
{
    return 2 * i < L ? (int32_t)i : (int32_t)i - (int32_t)L;
}

// Wave vectors the binning kernel visits: the planes n_z = 0 .. floor(nz / 2)
// of the FFT output (index order x fastest).  Every pair {k, -k} has a member
// there; a pair whose members both lie there (n_z = 0 or nz / 2) is taken at
// its lower index.
__host__ __device__ inline uint64_t bin_nodes(uint32_t nx, uint32_t ny, uint32_t nz)
{
    return (uint64_t)(nz / 2 + 1) * nx * ny;
}

// Shells 0 .. smax of a box, smax = round(sqrt(sum_a floor(L_a / 2)^2)).
__host__ __device__ inline uint32_t box_shells(uint32_t nx, uint32_t ny, uint32_t nz)
{
    const uint64_t a = nx / 2, b = ny / 2, c = nz / 2;
    const uint64_t n2 = a * a + b * b + c * c;
    return (n2 == 0 ? 0u : shell_of(n2)) + 1u;
}

}  // namespace gmf
