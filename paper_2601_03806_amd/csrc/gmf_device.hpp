// gmf_device.hpp -- device-side building blocks of the GMF-FLBM step on gfx950:
// lattice constants in the library's internal population order, the per-replica
// parameter record, fast integer division, Philox4x32-10 and the normal
// transforms.
//
// Internal population order ("tensor order"): p = 9 (cx+1) + 3 (cy+1) + (cz+1)
// for c = (cx, cy, cz) in {-1,0,1}^3.  With this order the D3Q27 weights and the
// full-Hermite basis of Table II factorise over the three axes, which is what
// the separable moment transforms in the step kernel use.  The host interface
// converts to and from the documented canonical order (see gmf.h).
//
// Storage layout of one replica ("row-interleaved"): the 27 populations are
// split into 27/G groups of G (G in {27, 9, 3, 1}, the largest for which a
// group fits 32-bit byte offsets); inside a group, each x-row of the box keeps
// its G population rows next to each other:
//     element(p, x, y, z) = g N G + ((z ny + y) G + q) nx + x,
// with slot s = 3 (3 (cy+1) + (cz+1)) + (cx+1), g = s / G, q = s % G.  The
// populations that a node pulls from one neighbouring row then sit in one
// contiguous block, and a wavefront's 27 stores land in a few DRAM pages
// instead of 27 separate arrays.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gmf_math.hpp"

namespace gmf {

constexpr int Q = 27;
constexpr int kBlock = 256;          // threads per workgroup of the lattice kernels
constexpr int kObs = 10;             // sampled observables (see gmf.h)
constexpr int kPartialStride = 24;   // doubles per partial record of the observables (2*kObs + 1, padded)
constexpr uint32_t kObsNodes = 16 * kBlock;   // nodes per workgroup of the observables kernel (FP64 path; 16 per thread)
constexpr int kFields = 6;           // fields kept for the spectra: drho, jx, jy, jz, pdiag, poff
constexpr int kDftNx = 4;            // n_x = 0..3 in the first DFT stage
constexpr int kDftNy = 7;            // n_y = -3..3
constexpr int kDftPlane = kDftNx * kDftNy;
constexpr int kShells = 8;
constexpr int kSpec = 5;
constexpr int kAccStride = 3 * kObs + kSpec * kShells + 8;  // doubles per replica accumulator

__host__ __device__ constexpr int tcx(int p) { return p / 9 - 1; }
__host__ __device__ constexpr int tcy(int p) { return (p / 3) % 3 - 1; }
__host__ __device__ constexpr int tcz(int p) { return p % 3 - 1; }
__host__ __device__ constexpr int tindex(int cx, int cy, int cz) { return 9 * (cx + 1) + 3 * (cy + 1) + (cz + 1); }
// storage slot of tensor-order population p: x-velocity fastest, so that the
// three populations pulled from the same neighbouring row are adjacent
__host__ __device__ constexpr int slot_of(int p) { return 3 * (p % 9) + p / 9; }

// D1Q3 weight factor: w(c) = w1(cx) w1(cy) w1(cz), w1(0) = 2/3, w1(+-1) = 1/6
__host__ __device__ constexpr double w1(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
__host__ __device__ constexpr double tweight(int p) { return w1(tcx(p)) * w1(tcy(p)) * w1(tcz(p)); }

// Round-up magic-number division for 0 <= n < 2^31 and 1 <= d < 2^31
// (Granlund & Montgomery, PLDI'94): q = (mulhi(n, m) + n) >> s with
// s = ceil(log2 d), m = floor(2^32 (2^s - d) / d) + 1.
struct FastDiv {
    uint32_t d, m, s;
};

inline FastDiv make_fastdiv(uint32_t d)
{
    uint32_t s = 0;
    while ((1ull << s) < d) ++s;
    uint64_t m = ((((1ull << s) - d) << 32) / d) + 1;
    return FastDiv{d, (uint32_t)m, s};
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f)
{
    return (__umulhi(n, f.m) + n) >> f.s;
}

// Per-replica record read by every lattice kernel (uniform across a workgroup).
struct RepDev {
    uint64_t pop_offset;      // element offset of the replica's 27*N block in a population buffer
    uint64_t field_offset;    // element offset of the replica's kFields*N block in the field buffer
    uint32_t nx, ny, nz, n;   // box and node count
    FastDiv divx, divy;
    uint32_t block_begin;     // first workgroup of this replica in the lattice grid
    uint32_t nblocks;         // workgroups of this replica in the lattice grid
    uint32_t key0, key1;      // Philox key
    uint32_t dft_offset;      // offset (in complex values) of the replica's DFT partials
    uint32_t noise_on;        // 0 when k_BT = 0
    uint32_t noise_rho0;      // 1: rho0 instead of the local rho in the noise amplitudes
    uint32_t grp;             // populations per storage group (27, 3 or 1)
    uint64_t grp_elems;       // elements per storage group (n * grp)
    uint32_t row_stride;      // elements between consecutive rows of a group (grp * nx)
    uint32_t tw_offset;       // offset (complex values) of the replica's twiddle tables (nx, ny, nz entries)
    uint32_t slice_first;     // first slice record of the replica in the statistics reduction
    uint32_t obs_first;       // first observables record of the replica (obs_records)
    uint32_t obs_blocks;      // its records (obs_records)
    uint32_t pad2;
    double rho0;
    double omega;             // 1 / tau
    double one_m_omega;       // 1 - omega
    double amp[8];            // noise amplitudes / sqrt(rho): groups of equal b_k (see host)
    // the same parameters rounded to binary32 once, for the FP32 kernels
    float rho0f, omegaf, one_m_omegaf, padf;
    float ampf[8];
    // full-box spectra (only when they are switched on)
    uint64_t spec_offset;     // offset (complex values of the kernel precision) of the replica's seven half spectra
    uint32_t shell_offset;    // first shell record of the replica
    uint32_t nshell;          // shells 0 .. nshell - 1 (shell 0 holds k = 0 only and stays empty)
};

// A replica parameter in the kernel's precision: the double field for FP64,
// its binary32 copy for FP32 (no per-thread conversion).
template <typename T>
__host__ __device__ inline T rep_param(double d, float f);
template <>
__host__ __device__ inline double rep_param<double>(double d, float) { return d; }
template <>
__host__ __device__ inline float rep_param<float>(double, float f) { return f; }

// Work units ("chunks") of the first shell-spectrum DFT stage: 64 columns
// (x, z) of the box, one per lane of a wavefront.  nx >= 64: a block of 64
// columns of one z plane, ceil(nx / 64) blocks per plane; nx < 64: floor(64 / nx)
// whole planes (one block per plane).  Partial records are kept per plane and
// column block.
constexpr uint32_t kDftCols = 64;
__host__ __device__ inline uint32_t dft_col_blocks(uint32_t nx) { return nx >= kDftCols ? (nx + kDftCols - 1) / kDftCols : 1u; }
__host__ __device__ inline uint32_t dft_planes_per_chunk(uint32_t nx) { return nx >= kDftCols ? 1u : kDftCols / nx; }
__host__ __device__ inline uint64_t dft_chunks(uint32_t nx, uint32_t nz)
{
    return nx >= kDftCols ? (uint64_t)nz * dft_col_blocks(nx) : ((uint64_t)nz + dft_planes_per_chunk(nx) - 1) / dft_planes_per_chunk(nx);
}

// Partial observables records of a replica per sample: the FP32 path sums them
// in the first DFT stage (one record per chunk), the FP64 path in
// observables_kernel (one per kObsNodes nodes).
__host__ __device__ inline uint64_t obs_records(bool fp32, uint32_t nx, uint32_t ny, uint32_t nz)
{
    return fp32 ? dft_chunks(nx, nz) : ((uint64_t)nx * ny * nz + kObsNodes - 1) / kObsNodes;
}

// Replica of workgroup b of a grid laid out by the prefix array first
// (first[r] <= b < first[r + 1], first[0] = 0).
__device__ __forceinline__ int replica_of_block(const uint32_t* first, int32_t nrep, uint32_t b)
{
    int lo = 0, hi = nrep - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (first[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Element offset (inside the replica block) of the start of population p's
// row at (y, z) = (0, 0).
__host__ __device__ inline uint64_t pop_base_offset(const RepDev& R, int p)
{
    const uint32_t s = (uint32_t)slot_of(p);
    return (uint64_t)(s / R.grp) * R.grp_elems + (uint64_t)(s % R.grp) * R.nx;
}
// Element offset of row (y, z) inside a group (valid for every population),
// in 32 bits: only for the per-node addressing modes, where a whole group
// fits 32-bit byte offsets.
__host__ __device__ inline uint32_t row_offset32(const RepDev& R, uint32_t y, uint32_t z)
{
    return (z * R.ny + y) * R.row_stride;
}
// Full element offset of population p at node (x, y, z), any box.
__host__ __device__ inline uint64_t pop_index(const RepDev& R, int p, uint32_t x, uint32_t y, uint32_t z)
{
    return pop_base_offset(R, p) + (uint64_t)(z * R.ny + y) * R.row_stride + x;
}

// Streaming patterns of the step kernel.  Tensor order makes the opposite
// velocity of p the population 26 - p (and its storage slot 26 - slot_of(p)).
//   kAB       two buffers; read f_p at x - c_p in the source buffer, write f*_p
//             at x in the other one;
//   kAAPull   one buffer, steps with even index: read f_p at x - c_p, write
//             f*_p where f_(26-p) was read (population 26 - p at x + c_p);
//   kAALocal  one buffer, steps with odd index: read f_p as population 26 - p
//             at x, write f*_p as population p at x.
// Each node writes exactly the locations it read, so the in-place update
// needs no synchronisation between nodes.
constexpr int kAB = 0, kAAPull = 1, kAALocal = 2;
__host__ __device__ constexpr int opposite(int p) { return Q - 1 - p; }

// Element offset of the canonical pre-collision value f_p(x, y, z): after a
// two-buffer step or an even number of AA steps it is population p at x - c_p;
// after an odd number of AA steps (aa_odd) it is population 26 - p at x.
__host__ __device__ inline uint64_t canon_index(const RepDev& R, int p, uint32_t x, uint32_t y, uint32_t z,
                                                int aa_odd)
{
    if (aa_odd) return pop_index(R, opposite(p), x, y, z);
    const uint32_t xs = (x + R.nx - (uint32_t)(tcx(p) + 1) + 1) % R.nx;
    const uint32_t ys = (y + R.ny - (uint32_t)(tcy(p) + 1) + 1) % R.ny;
    const uint32_t zs = (z + R.nz - (uint32_t)(tcz(p) + 1) + 1) % R.nz;
    return pop_index(R, p, xs, ys, zs);
}

// ---------------------------------------------------------------------------
// Philox4x32-10: ten rounds of two 32x32->64 multiplies and xors, key bumped by
// the Weyl constants between rounds (Salmon et al., SC'11).
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

// three-input xor in one VALU op (gfx950 v_bitop3_b32, truth table 0x96)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        U4 o;
        o.x = xor3((uint32_t)(p1 >> 32), c.y, k0);
        o.y = (uint32_t)p1;
        o.z = xor3((uint32_t)(p0 >> 32), c.w, k1);
        o.w = (uint32_t)p0;
        c = o;
    }
    return c;
}

// Block j of the noise of node n at step t.
__device__ __forceinline__ U4 noise_block(uint32_t n, uint64_t t, uint32_t j, uint32_t k0, uint32_t k1)
{
    return philox4x32_10(U4{n, (uint32_t)t, j, (uint32_t)(t >> 32)}, k0, k1);
}

// Box-Muller pair from two words.
template <typename T>
struct Normal;

template <>
struct Normal<double> {
    __device__ __forceinline__ static void pair(uint32_t a, uint32_t b, double& r0, double& r1)
    {
        const double u1 = ((double)a + 0.5) * 0x1p-32;
        const double u2 = ((double)b + 0.5) * 0x1p-32;
        // logarithm and sine/cosine specialised to these arguments (gmf_math.hpp)
        const double rad = fp64::sqrt_pos(-2.0 * fp64::log_unit(u1));
        double s, c;
        fp64::sincos_2pi(u2, &s, &c);
        r0 = rad * c;
        r1 = rad * s;
    }
};

template <>
struct Normal<float> {
    __device__ __forceinline__ static void pair(uint32_t a, uint32_t b, float& r0, float& r1)
    {
        // top 23 bits: (m + 1/2) 2^-23 is exact in binary32
        const float u1 = __builtin_fmaf((float)(a >> 9), 0x1p-23f, 0x1p-24f);
        const float u2 = __builtin_fmaf((float)(b >> 9), 0x1p-23f, 0x1p-24f);
        // -2 ln u1 = -2 ln(2) log2(u1); v_log_f32 is log2, v_sin/v_cos take revolutions
        const float rad = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));
        r0 = rad * __builtin_amdgcn_cosf(u2);
        r1 = rad * __builtin_amdgcn_sinf(u2);
    }
};

// The 23 standard normals r_4..r_26 of one node and step, r[k-4].
template <typename T>
__device__ __forceinline__ void node_normals(uint32_t n, uint64_t t, uint32_t k0, uint32_t k1, T r[23])
{
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const U4 w = noise_block(n, t, (uint32_t)j, k0, k1);
        T a, b, c, d;
        Normal<T>::pair(w.x, w.y, a, b);
        r[4 * j + 0] = a;
        r[4 * j + 1] = b;
        if (j < 5) {
            Normal<T>::pair(w.z, w.w, c, d);
            r[4 * j + 2] = c;
            r[4 * j + 3] = d;
        } else {
            // k = 26 is the last mode; the sine of the last pair is unused
            Normal<T>::pair(w.z, w.w, c, d);
            r[22] = c;
        }
    }
}

}  // namespace gmf
