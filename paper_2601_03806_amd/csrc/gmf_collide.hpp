// gmf_collide.hpp -- device building blocks shared by the two step kernels
// (population storage in gmf_kernels.hip, moment storage in gmf_mstep.hip):
// the separable moment transforms over the D3Q27 tensor order, the Table II
// ghost slots, the scalar-register copy of a replica record, and the FP32/FP64
// reciprocal and square root.
#pragma once

#include <hip/hip_runtime.h>

#include "gmf_device.hpp"
#include "gmf_internal.hpp"

namespace gmf {

// ---------------------------------------------------------------------------
// Separable transforms
// ---------------------------------------------------------------------------

// One axis of the back-projection f*(c) = sum_abc T[cx][a] T[cy][b] T[cz][c] M_abc,
// T[c][a] = w1(c) h_a(c) / |h_a|^2 with |h|^2 = (1, 1/3, 2/9):
//   T[-1] = (1/6, -1/2, 1/2),  T[0] = (2/3, 0, -1),  T[+1] = (1/6, 1/2, 1/2).
template <typename T>
__device__ __forceinline__ void tr3(T a0, T a1, T a2, T& om, T& oz, T& op)
{
    const T s = a0 * T(1.0 / 6.0) + a2 * T(0.5);
    const T h = a1 * T(0.5);
    oz = a0 * T(2.0 / 3.0) - a2;
    om = s - h;
    op = s + h;
}

// M[9a + 3b + c] (Hermite coefficient of order (a,b,c)) -> F[p] (tensor order)
template <typename T>
__device__ __forceinline__ void back_project(const T M[Q], T F[Q])
{
    T N[Q], P[Q];
#pragma unroll
    for (int ab = 0; ab < 9; ++ab)
        tr3(M[3 * ab + 0], M[3 * ab + 1], M[3 * ab + 2], N[3 * ab + 0], N[3 * ab + 1], N[3 * ab + 2]);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int cz = 0; cz < 3; ++cz)
            tr3(N[9 * a + 0 + cz], N[9 * a + 3 + cz], N[9 * a + 6 + cz],
                P[9 * a + 0 + cz], P[9 * a + 3 + cz], P[9 * a + 6 + cz]);
#pragma unroll
    for (int q = 0; q < 9; ++q)
        tr3(P[q], P[9 + q], P[18 + q], F[q], F[9 + q], F[18 + q]);
}

// Raw moments of order <= 2: s0 = sum f, j = sum f c, pi = sum f c c.
template <typename T>
struct Hydro {
    T s0, jx, jy, jz, pxx, pyy, pzz, pxy, pxz, pyz;
};

template <typename T>
__device__ __forceinline__ Hydro<T> forward_moments(const T f[Q])
{
    T X0[9], X1[9], X2[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const T a = f[q], b = f[9 + q], c = f[18 + q];   // cx = -1, 0, +1
        X2[q] = a + c;
        X0[q] = X2[q] + b;
        X1[q] = c - a;
    }
    T Y00[3], Y01[3], Y02[3], Y10[3], Y11[3], Y20[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {                      // cz index; cy lines q = 3*cyi + r
        Y02[r] = X0[r] + X0[6 + r];
        Y00[r] = Y02[r] + X0[3 + r];
        Y01[r] = X0[6 + r] - X0[r];
        Y10[r] = X1[r] + X1[3 + r] + X1[6 + r];
        Y11[r] = X1[6 + r] - X1[r];
        Y20[r] = X2[r] + X2[3 + r] + X2[6 + r];
    }
    Hydro<T> h;
    h.pzz = Y00[0] + Y00[2];
    h.s0 = h.pzz + Y00[1];
    h.jz = Y00[2] - Y00[0];
    h.jy = Y01[0] + Y01[1] + Y01[2];
    h.pyz = Y01[2] - Y01[0];
    h.pyy = Y02[0] + Y02[1] + Y02[2];
    h.jx = Y10[0] + Y10[1] + Y10[2];
    h.pxz = Y10[2] - Y10[0];
    h.pxy = Y11[0] + Y11[1] + Y11[2];
    h.pxx = Y20[0] + Y20[1] + Y20[2];
    return h;
}

// (a,b,c) Hermite orders of the Table II ghost vectors k = 10..26, as 9a+3b+c
__device__ constexpr int kGhostSlot[17] = {
    21, 19, 15, 11, 7, 5,   // x^2y, x^2z, y^2x, z^2x, y^2z, z^2y
    13,                     // xyz
    24, 20, 8,              // x^2y^2, x^2z^2, y^2z^2
    14, 16, 22,             // xyz^2, xzy^2, yzx^2
    23, 25, 17,             // x^2yz^2, x^2zy^2, y^2xz^2
    26};                    // x^2y^2z^2
// amplitude group of each ghost (index into RepDev::amp)
__device__ constexpr int kGhostGroup[17] = {2, 2, 2, 2, 2, 2, 3, 4, 4, 4, 5, 5, 5, 6, 6, 6, 7};

// Raw buffer access: a uniform 64-bit base in a buffer resource plus a 32-bit
// vector offset (and a scalar one), so that no per-access 64-bit address
// arithmetic is spent on the vector ALUs.  POLICY: cache-policy bits,
// kNontemporal for data touched once per step, 0 for cached accesses.
constexpr int kNontemporal = 2;   // cache-policy bits of the buffer builtins on gfx950

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base)
{
    // raw buffer: stride 0, 2^32 - 1 bytes addressable, gfx9 resource word 3
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, -1, 0x00020000);
}

template <typename T, int POLICY = kNontemporal>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    if constexpr (sizeof(T) == 4)
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, POLICY));
    else
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, POLICY));
}

template <int POLICY = kNontemporal>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, POLICY);
}
template <int POLICY = kNontemporal>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, double v)
{
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, POLICY);
}

// The replica record is read once per workgroup and pinned in scalar
// registers: the compiler cannot otherwise prove that fields re-read after
// the first stores are uniform, and buffer offsets must be scalar.
__device__ __forceinline__ uint32_t sgpr(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t sgpr64(uint64_t v)
{
    return ((uint64_t)sgpr((uint32_t)(v >> 32)) << 32) | sgpr((uint32_t)v);
}
__device__ __forceinline__ double sgprf(double v) { return __builtin_bit_cast(double, sgpr64(__builtin_bit_cast(uint64_t, v))); }

__device__ __forceinline__ RepDev uniform_rep(const RepDev& in)
{
    RepDev R;
    R.pop_offset = sgpr64(in.pop_offset);
    R.field_offset = sgpr64(in.field_offset);
    R.nx = sgpr(in.nx);
    R.ny = sgpr(in.ny);
    R.nz = sgpr(in.nz);
    R.n = sgpr(in.n);
    R.divx = FastDiv{sgpr(in.divx.d), sgpr(in.divx.m), sgpr(in.divx.s)};
    R.divy = FastDiv{sgpr(in.divy.d), sgpr(in.divy.m), sgpr(in.divy.s)};
    R.block_begin = sgpr(in.block_begin);
    R.nblocks = sgpr(in.nblocks);
    R.key0 = sgpr(in.key0);
    R.key1 = sgpr(in.key1);
    R.dft_offset = sgpr(in.dft_offset);
    R.noise_on = sgpr(in.noise_on);
    R.noise_rho0 = sgpr(in.noise_rho0);
    R.grp = sgpr(in.grp);
    R.grp_elems = sgpr64(in.grp_elems);
    R.row_stride = sgpr(in.row_stride);
    R.tw_offset = sgpr(in.tw_offset);
    R.slice_first = sgpr(in.slice_first);
    R.obs_first = sgpr(in.obs_first);
    R.obs_blocks = sgpr(in.obs_blocks);
    R.pad2 = 0;
    R.rho0 = sgprf(in.rho0);
    R.omega = sgprf(in.omega);
    R.one_m_omega = sgprf(in.one_m_omega);
#pragma unroll
    for (int g = 0; g < 8; ++g) R.amp[g] = sgprf(in.amp[g]);
    auto sgprf32 = [](float v) { return __builtin_bit_cast(float, sgpr(__builtin_bit_cast(uint32_t, v))); };
    R.rho0f = sgprf32(in.rho0f);
    R.omegaf = sgprf32(in.omegaf);
    R.one_m_omegaf = sgprf32(in.one_m_omegaf);
    R.padf = 0.0f;
#pragma unroll
    for (int g = 0; g < 8; ++g) R.ampf[g] = sgprf32(in.ampf[g]);
    R.spec_offset = sgpr64(in.spec_offset);
    R.shell_offset = sgpr(in.shell_offset);
    R.nshell = sgpr(in.nshell);
    return R;
}

// 1/x and sqrt(x) of a positive density: correctly rounded in FP64; the
// hardware reciprocal and square root (about 1 ulp) in FP32, whose parity
// tolerance covers them
__device__ __forceinline__ double recip(double v) { return 1.0 / v; }
__device__ __forceinline__ float recip(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double sqroot(double v) { return sqrt(v); }
__device__ __forceinline__ float sqroot(float v) { return __builtin_amdgcn_sqrtf(v); }


// Hermite coefficients M[9a + 3b + c] of f* before the noise, from the raw
// moments h of f (of g = f - w rho0 in shifted storage, where the rho0 parts of
// a2 cancel): GMF keeps rho and j, relaxes the non-equilibrium stress by
// (1 - omega) around rho u u and drops every ghost (Eqs. (10)-(13)); BGK is
// f* = (1 - omega) f + omega f^eq (Eq. (1)), of which this is the omega f^eq
// part (the caller adds (1 - omega) f).
template <typename T, int COLL>
__device__ __forceinline__ void relaxed_coefficients(const Hydro<T>& h, T irho, T om, T omm, T M[Q])
{
    const T cs2 = T(1.0 / 3.0);
    // equilibrium second-order Hermite coefficient rho u u = j j / rho
    const T exx = h.jx * h.jx * irho, eyy = h.jy * h.jy * irho, ezz = h.jz * h.jz * irho;
    const T exy = h.jx * h.jy * irho, exz = h.jx * h.jz * irho, eyz = h.jy * h.jz * irho;
    if (COLL == kGMF) {
        // Hermite coefficient of f: a2 = Pi - rho cs2 I
        const T a2xx = h.pxx - cs2 * h.s0, a2yy = h.pyy - cs2 * h.s0, a2zz = h.pzz - cs2 * h.s0;
        M[0] = h.s0;
        M[9] = h.jx; M[3] = h.jy; M[1] = h.jz;
        M[18] = om * exx + omm * a2xx;
        M[6] = om * eyy + omm * a2yy;
        M[2] = om * ezz + omm * a2zz;
        M[12] = om * exy + omm * h.pxy;
        M[10] = om * exz + omm * h.pxz;
        M[4] = om * eyz + omm * h.pyz;
    } else {
        M[0] = om * h.s0;
        M[9] = om * h.jx; M[3] = om * h.jy; M[1] = om * h.jz;
        M[18] = om * exx; M[6] = om * eyy; M[2] = om * ezz;
        M[12] = om * exy; M[10] = om * exz; M[4] = om * eyz;
    }
#pragma unroll
    for (int g = 0; g < 17; ++g) M[kGhostSlot[g]] = T(0);
}

// Noise of Eqs. (2) and (9) added to the coefficients: r[k - 4] = r_k, sr the
// square root of the density in the amplitudes (local rho, or rho0 when the
// replica asks for it); RepDev::amp holds phi_k / sqrt(rho) for each group of
// equal b_k (the back-projection divides by b_k).
template <typename T>
__device__ __forceinline__ void add_noise(const RepDev& R, T sr, const T r[23], T M[Q])
{
    const T sh0 = rep_param<T>(R.amp[0], R.ampf[0]) * sr, sh1 = rep_param<T>(R.amp[1], R.ampf[1]) * sr;
    M[18] += sh0 * r[0]; M[6] += sh0 * r[1]; M[2] += sh0 * r[2];
    M[12] += sh1 * r[3]; M[10] += sh1 * r[4]; M[4] += sh1 * r[5];
#pragma unroll
    for (int g = 0; g < 17; ++g)
        M[kGhostSlot[g]] = (rep_param<T>(R.amp[kGhostGroup[g]], R.ampf[kGhostGroup[g]]) * sr) * r[6 + g];
}

// Workgroup sums of NV doubles (kBlock threads), written by threads 0..NV-1.
// Sums of NV doubles over the NT threads of a workgroup (NT a multiple of 64),
// in a fixed order (butterfly within each wave, then the waves in turn):
// threads 0 .. NV - 1 store them to out.  Every thread must call it.
template <int NV, int NT>
__device__ __forceinline__ void block_sum_store_nt(double (&v)[NV], double* out)
{
    static_assert(NT % 64 == 0, "whole wavefronts");
    __shared__ double red[NT / 64][NV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double s = v[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        v[q] = s;
    }
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) red[wave][q] = v[q];
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) s += red[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// Observables of one sampled node, from the six sampled fields in the kernel
// precision (rho - rho0, j, sum_a Pi_aa - 3 rho0 cs2, sum_{a<b} Pi_ab; the
// order of gmf.h's GMF_OBS_*), added in FP64 to a partial record: the sums of
// o and o^2 and the count of non-finite densities.  u = j / rho is formed in
// the kernel precision (the fields carry no more), everything after in FP64.
constexpr int kObsVals = 2 * kObs + 1;
template <typename T>
__device__ __forceinline__ void add_observables(double (&acc)[kObsVals], T rho0, T drho, T jx, T jy, T jz,
                                                T pdiag, T poff, double w = 1.0)
{
    const T irho = recip(rho0 + drho);
    double o[kObs];
    o[0] = (double)drho;
    o[1] = (double)jx;
    o[2] = (double)jy;
    o[3] = (double)jz;
    o[4] = o[1] + o[2] + o[3];
    o[5] = (double)pdiag;
    o[6] = (double)poff;
    o[7] = (double)(jx * irho);
    o[8] = (double)(jy * irho);
    o[9] = (double)(jz * irho);
    // w = 0 leaves the record as it is (a node repeated past the box end)
#pragma unroll
    for (int q = 0; q < kObs; ++q) {
        const double wo = w * o[q];
        acc[2 * q] += wo;
        acc[2 * q + 1] = fma(wo, o[q], acc[2 * q + 1]);
    }
    acc[2 * kObs] += isfinite(o[0]) ? 0.0 : w;
}

template <int NV>
__device__ __forceinline__ void block_sum_store(double (&v)[NV], double* out)
{
    block_sum_store_nt<NV, kBlock>(v, out);
}

}  // namespace gmf
