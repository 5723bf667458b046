// gmf_sample.hip -- gfx950 kernels of the sampling steps (Results section:
// the equilibrium ratios of the sampled observables and the shell spectra
// S_m(|k|) of the eight smallest shells), run after a sampling step of the
// step kernel has written the six fields drho, jx, jy, jz, pdiag, poff of the
// pre-collision state.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "gmf_collide.hpp"
#include "gmf_device.hpp"
#include "gmf_internal.hpp"

namespace gmf {

// ---------------------------------------------------------------------------
// Sampling: the observables of the sampled state, from the six fields the step
// kernel wrote, summed in FP64 into the accumulators in a fixed order (so that
// a state always gives the same bits):
//   observables_kernel       kObsNodes consecutive nodes of one replica per
//                            workgroup, 16 per thread, into one partial record;
//   stats_slice_kernel       kBlock consecutive records of a replica per slice;
//   stats_accumulate_kernel  one workgroup per replica adds its slices.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void observables_kernel(const RepDev* reps, const uint32_t* first, int32_t nrep,
                                                             const T* __restrict__ fields, double* partials)
{
    const int r = replica_of_block(first, nrep, blockIdx.x);
    const RepDev R = uniform_rep(reps[r]);
    const uint64_t N = R.n;
    const T* fl = fields + R.field_offset;
    const T rho0 = rep_param<T>(R.rho0, R.rho0f);
    double acc[kObsVals];
#pragma unroll
    for (int q = 0; q < kObsVals; ++q) acc[q] = 0.0;
    const uint32_t n0 = (blockIdx.x - first[r]) * kObsNodes + threadIdx.x;
    // batches of four nodes, two in flight: a batch's 24 loads are issued
    // unconditionally (past the box end they read the last node again, which
    // then adds with weight 0) while the previous batch is being summed
    constexpr int kBatch = 4, kBatches = kObsNodes / kBlock / kBatch;
    auto load = [&](T (&v)[kBatch][kFields], int k) {
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const uint32_t n = min(n0 + (uint32_t)(k * kBatch + u) * kBlock, R.n - 1);
#pragma unroll
            for (int f = 0; f < kFields; ++f) v[u][f] = fl[(uint64_t)f * N + n];
        }
    };
    auto add = [&](T (&v)[kBatch][kFields], int k) {
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const double w = n0 + (uint32_t)(k * kBatch + u) * kBlock < R.n ? 1.0 : 0.0;
            add_observables<T>(acc, rho0, v[u][0], v[u][1], v[u][2], v[u][3], v[u][4], v[u][5], w);
        }
    };
    T va[kBatch][kFields], vb[kBatch][kFields];
    load(va, 0);
#pragma unroll
    for (int k = 0; k < kBatches; ++k) {
        // two register sets in turn (a copy between them would wait for the loads)
        if (k % 2 == 0) {
            if (k + 1 < kBatches) load(vb, k + 1);
            add(va, k);
        } else {
            if (k + 1 < kBatches) load(va, k + 1);
            add(vb, k);
        }
    }
    block_sum_store<kObsVals>(acc, partials + (size_t)blockIdx.x * kPartialStride);
}

hipError_t launch_observables(int precision, const RepDev* reps, int32_t nrep, const uint32_t* first,
                              uint32_t nblocks, const void* fields, double* partials, hipStream_t s)
{
    if (precision == kFP64)
        observables_kernel<double><<<nblocks, kBlock, 0, s>>>(reps, first, nrep, (const double*)fields, partials);
    else
        observables_kernel<float><<<nblocks, kBlock, 0, s>>>(reps, first, nrep, (const float*)fields, partials);
    return hipGetLastError();
}

// Stage 1 of the reduction: each workgroup sums kBlock consecutive partial
// records of one replica (blockIdx.y) into a slice record; slices past the
// replica's count exit.
__global__ __launch_bounds__(kBlock) void stats_slice_kernel(const RepDev* reps, const double* partials,
                                                             double* slices)
{
    const RepDev R = uniform_rep(reps[blockIdx.y]);
    const uint32_t nsl = (R.obs_blocks + kBlock - 1) / kBlock;
    if (blockIdx.x >= nsl) return;
    const uint32_t b = blockIdx.x * kBlock + threadIdx.x;
    double v[kObsVals];
#pragma unroll
    for (int q = 0; q < kObsVals; ++q)
        v[q] = b < R.obs_blocks ? partials[(size_t)(R.obs_first + b) * kPartialStride + q] : 0.0;
    block_sum_store<kObsVals>(v, slices + (size_t)(R.slice_first + blockIdx.x) * kPartialStride);
}

// Stage 2: the slices of each replica, summed in a fixed order, update the
// accumulators (spatial mean, mean square and variance of each observable).
__global__ __launch_bounds__(kBlock) void stats_accumulate_kernel(const RepDev* reps, const double* slices,
                                                                  double* acc, double* sample_sq)
{
    const RepDev& R = reps[blockIdx.x];
    const uint32_t nsl = (R.obs_blocks + kBlock - 1) / kBlock;
    double v[kObsVals];
    for (int q = 0; q < kObsVals; ++q) v[q] = 0.0;
    for (uint32_t c = threadIdx.x; c < nsl; c += kBlock) {
        const double* p = slices + (size_t)(R.slice_first + c) * kPartialStride;
#pragma unroll
        for (int q = 0; q < kObsVals; ++q) v[q] += p[q];
    }
    __shared__ double tot[kObsVals];
    block_sum_store<kObsVals>(v, tot);
    __syncthreads();
    if (threadIdx.x == 0) {
        double* A = acc + (size_t)blockIdx.x * kAccStride;
        const double invn = 1.0 / (double)R.n;
        A[kAccNsamp] += 1.0;
        A[kAccNonfinite] += tot[2 * kObs];
        for (int q = 0; q < kObs; ++q) {
            const double m = tot[2 * q] * invn, m2 = tot[2 * q + 1] * invn;
            A[kAccMean + q] += m;
            A[kAccMeanSq + q] += m2;
            A[kAccVar + q] += m2 - m * m;
        }
        // this sample's sums of squares (they bound the full-box spectra, see gmf_fft.hip)
        if (sample_sq)
            for (int q = 0; q < kObs; ++q) sample_sq[(size_t)blockIdx.x * kObs + q] = tot[2 * q + 1];
    }
}

hipError_t launch_stats_reduce(const RepDev* reps, int32_t nrep, uint32_t max_slices, const double* partials,
                               double* slices, double* acc, double* sample_sq, hipStream_t s)
{
    stats_slice_kernel<<<dim3(max_slices, nrep), kBlock, 0, s>>>(reps, partials, slices);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    stats_accumulate_kernel<<<nrep, kBlock, 0, s>>>(reps, slices, acc, sample_sq);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Shell spectra (normalised DFT at the vectors of the shells |n|^2 in
// {1,2,3,4,5,6,8,9}).  A real field has |m(-k)| = |m(k)|, so only n_x >= 0 is
// computed and n_x > 0 counts twice.  Twiddles e^{2 pi i m / L} for the three
// box lengths of each replica are tabulated once (twiddle_kernel).
//   Stage 1 (workgroups of 64 columns (x, z), per field): DFT along y at
//     n_y = 0..3 (Y(-n_y) = conj Y(n_y)), then along x at n_x = 0..3 from the
//     columns kept in LDS, one partial record per plane and column block.
//   Stage 2 (per replica, field and z chunk): the column blocks of each plane
//     summed, then the DFT along z at n_z = -3..3.
//   Stage 3 (one workgroup per replica): powers of the five spectra, shell
//     averages into the accumulators (fixed summation order).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void twiddle_kernel(const RepDev* reps, double2* tw)
{
    const RepDev& R = reps[blockIdx.x];
    const uint32_t lens[3] = {R.nx, R.ny, R.nz};
    uint32_t off = R.tw_offset;
    for (int a = 0; a < 3; ++a) {
        for (uint32_t m = threadIdx.x; m < lens[a]; m += kBlock) {
            double sn, cs;
            sincospi(2.0 * (double)m / (double)lens[a], &sn, &cs);
            tw[off + m] = make_double2(cs, sn);
        }
        off += lens[a];
    }
}

hipError_t launch_twiddles(const RepDev* reps, int32_t nrep, double2* tw, hipStream_t s)
{
    twiddle_kernel<<<nrep, kBlock, 0, s>>>(reps, tw);
    return hipGetLastError();
}

// Stage 1, one workgroup per (chunk, field): the y-transform at n_y = 0..3 of
// the chunk's 64 columns (lane = column), the y range split over the four
// wavefronts so that each thread issues ny / 4 loads of its column, eight at a
// time; the wavefronts' sums meet in LDS; then the x-transform at n_x = 0..3 of
// each plane's columns in the chunk: the 28 items (n_x, n_y = -3..3, using
// Y(-n_y) = conj(Y(n_y)) of a real column) of each plane, eight threads per item
// with a fixed-order shuffle sum, into the partial record of (plane, column
// block).  twx[m] = e^{2 pi i m / nx}, twy[m] = e^{2 pi i m / ny} in memory:
// the y loop's twiddle indices are uniform, so its twiddles come through
// scalar loads.
// A first-stage chunk as one lane sees it: lane = column (plane z0 + p,
// x), the y range split over the four wavefronts; a lane without a column
// reads the chunk's first column (the loads stay unconditional) and adds zero.
struct DftLane {
    uint32_t z0, cb, CB, P, lane, wave, ylo, yhi;
    bool wide;
    uint64_t off;   // node of the lane's column at y = 0
    double keep;
};

__device__ __forceinline__ DftLane dft_lane(const RepDev& R, uint32_t chunk)
{
    DftLane g;
    const uint32_t nx = R.nx, ny = R.ny, nz = R.nz;
    g.CB = dft_col_blocks(nx);
    g.P = dft_planes_per_chunk(nx);
    g.wide = nx >= kDftCols;
    g.z0 = g.wide ? chunk / g.CB : chunk * g.P;
    g.cb = g.wide ? chunk - g.z0 * g.CB : 0u;
    // the wavefront index is uniform: the y loop, its twiddle indices and loads stay scalar
    g.lane = threadIdx.x & 63u;
    g.wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t p = g.wide ? 0u : g.lane / nx;
    const uint32_t x = g.wide ? g.cb * kDftCols + g.lane : g.lane - p * nx;
    const bool valid = g.wide ? x < nx : (p < g.P && g.z0 + p < nz);
    g.off = valid ? (uint64_t)(g.z0 + p) * nx * ny + x : (uint64_t)g.z0 * nx * ny + g.cb * kDftCols;
    g.keep = valid ? 1.0 : 0.0;
    const uint32_t yq = (ny + 3) / 4;
    g.ylo = min(ny, g.wave * yq);
    g.yhi = min(ny, g.ylo + yq);
    return g;
}

// the x twiddles e^{2 pi i q x / nx} (q = 1..3) of the chunk's columns, for
// the x-transform; their loads overlap the y loop
__device__ __forceinline__ void dft_load_tx(const RepDev& R, const DftLane& g, const double2* __restrict__ twx,
                                            double2 (*Tx)[kDftCols])
{
    const uint32_t nx = R.nx;
    if (threadIdx.x < 3 * kDftCols) {
        const uint32_t q = threadIdx.x / kDftCols + 1, c = threadIdx.x % kDftCols;
        const uint32_t xc = g.wide ? min(g.cb * kDftCols + c, nx - 1) : c % nx;
        Tx[q - 1][c] = twx[(uint32_t)(((uint64_t)q * xc) % nx)];
    }
}

// A lane's y-transform of one field at n_y = 0..3 (twy[m] = e^{2 pi i m / ny}).
struct YSum {
    double y0 = 0.0, y1r = 0.0, y1i = 0.0, y2r = 0.0, y2i = 0.0, y3r = 0.0, y3i = 0.0;
    __device__ __forceinline__ void add(double v, uint32_t y, uint32_t ny, const double2* __restrict__ twy)
    {
        // 2y mod ny and 3y mod ny for y < ny, without loop-carried state
        const uint32_t m2 = 2 * y - (2 * y >= ny ? ny : 0u);
        const uint32_t m3 = 3 * y - ny * ((3 * y >= ny ? 1u : 0u) + (3 * y >= 2 * ny ? 1u : 0u));
        const double2 t1 = twy[y], t2 = twy[m2], t3 = twy[m3];
        y0 += v;
        y1r = fma(v, t1.x, y1r);
        y1i = fma(-v, t1.y, y1i);
        y2r = fma(v, t2.x, y2r);
        y2i = fma(-v, t2.y, y2i);
        y3r = fma(v, t3.x, y3r);
        y3i = fma(-v, t3.y, y3i);
    }
};

// The four wavefronts' y sums of one field meet in LDS (in wavefront order);
// then the x-transform at n_x = 0..3 of each plane's columns in the chunk:
// the 28 items (n_x, n_y = -3..3, using Y(-n_y) = conj(Y(n_y)) of a real
// column) of each plane, eight threads per item with a fixed-order shuffle
// sum, into the partial record of (plane, column block).  Ends with the LDS
// free again.
__device__ __forceinline__ void dft_plane_finish(const RepDev& R, const DftLane& g, const YSum& a, int fld,
                                                 double2 (*Ys)[kDftCols][4], double2 (*Tx)[kDftCols], double2* dft)
{
    const uint32_t nx = R.nx, nz = R.nz;
    Ys[g.wave][g.lane][0] = make_double2(a.y0, 0.0);
    Ys[g.wave][g.lane][1] = make_double2(a.y1r, a.y1i);
    Ys[g.wave][g.lane][2] = make_double2(a.y2r, a.y2i);
    Ys[g.wave][g.lane][3] = make_double2(a.y3r, a.y3i);
    __syncthreads();
    {
        const uint32_t c = threadIdx.x & 63u, k = threadIdx.x >> 6;
        double2 s = Ys[0][c][k];
#pragma unroll
        for (int w = 1; w < 4; ++w) s = make_double2(s.x + Ys[w][c][k].x, s.y + Ys[w][c][k].y);
        Ys[0][c][k] = s;
    }
    __syncthreads();
    // item it = (plane pp, n_x, n_y); group of eight threads per item
    const uint32_t grp = threadIdx.x >> 3, sub = threadIdx.x & 7u;
    const uint32_t nitems = (g.wide ? 1u : g.P) * (uint32_t)kDftPlane;
    const uint32_t ncols = g.wide ? min(kDftCols, nx - g.cb * kDftCols) : nx;
    for (uint32_t base = 0; base < nitems; base += kBlock / 8) {
        const uint32_t it = base + grp;
        const bool act = it < nitems;
        const uint32_t pp = act ? it / kDftPlane : 0u, o = act ? it % kDftPlane : 0u;
        const uint32_t q = o / kDftNy;
        const int sy = (int)(o % kDftNy) - 3;
        const uint32_t ay = (uint32_t)(sy < 0 ? -sy : sy);
        const double sg = sy < 0 ? -1.0 : 1.0;          // conjugate for negative n_y
        double re = 0.0, im = 0.0;
        if (act) {
            for (uint32_t c = sub; c < ncols; c += 8) {
                const double2 yv = Ys[0][g.wide ? c : pp * nx + c][ay];
                const double yr = yv.x, yi = sg * yv.y;
                const double2 t = q == 0 ? make_double2(1.0, 0.0) : Tx[q - 1][c];
                // (yr + i yi)(c - i s)
                re += yr * t.x + yi * t.y;
                im += yi * t.x - yr * t.y;
            }
        }
#pragma unroll
        for (int off = 4; off > 0; off >>= 1) {
            re += __shfl_xor(re, off, 64);
            im += __shfl_xor(im, off, 64);
        }
        if (act && sub == 0 && g.z0 + pp < nz)
            dft[R.dft_offset + (((uint64_t)fld * nz + g.z0 + pp) * g.CB + g.cb) * kDftPlane + o] = make_double2(re, im);
    }
    __syncthreads();
}

// Stage 1, one workgroup per (chunk, field): the y-transform at n_y = 0..3 of
// the chunk's 64 columns, each thread taking ny / 4 rows of its column in
// batches of eight, two in flight; then dft_plane_finish.  The y loop's
// twiddle indices are uniform, so its twiddles come through scalar loads.
template <typename T>
__device__ __forceinline__ void dft_plane_body(const RepDev& R, uint32_t chunk, int fld, const T* __restrict__ fields,
                                               const double2* __restrict__ twx, const double2* __restrict__ twy,
                                               double2 (*Ys)[kDftCols][4], double2 (*Tx)[kDftCols], double2* dft)
{
    const uint32_t nx = R.nx, ny = R.ny;
    const DftLane g = dft_lane(R, chunk);
    const T* col = fields + R.field_offset + (uint64_t)fld * R.n + g.off;
    dft_load_tx(R, g, twx, Tx);
    YSum a;
    // batches of eight rows, two in flight: the next batch is loaded while one
    // is summed (past the last whole batch the load repeats it, unused)
    const uint32_t ylo = g.ylo, yhi = g.yhi, nfull = (yhi - ylo) / 8;
    auto load8 = [&](T (&v)[8], uint32_t k) {
        const uint32_t y0 = ylo + 8 * (k < nfull ? k : nfull - 1);
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = col[(uint64_t)(y0 + u) * nx];
    };
    auto add8 = [&](T (&v)[8], uint32_t k) {
#pragma unroll
        for (int u = 0; u < 8; ++u) a.add(g.keep * (double)v[u], ylo + 8 * k + u, ny, twy);
    };
    if (nfull > 0) {
        T va[8], vb[8];
        load8(va, 0);
        uint32_t k = 0;
        for (; k + 1 < nfull; k += 2) {
            load8(vb, k + 1);
            add8(va, k);
            load8(va, k + 2);
            add8(vb, k + 1);
        }
        if (k < nfull) add8(va, k);
    }
    for (uint32_t y = ylo + 8 * nfull; y < yhi; ++y) a.add(g.keep * (double)col[(uint64_t)y * nx], y, ny, twy);
    dft_plane_finish(R, g, a, fld, Ys, Tx, dft);
}

// The observables of add_observables (gmf_collide.hpp) in two parts, with the
// same operations in the same order on each accumulator: first those of drho
// and j (drho, jx, jy, jz, their sum, u = j / rho, and the non-finite count),
// then those of pdiag and poff.
template <typename T>
__device__ __forceinline__ void add_observables_rho_j(double (&acc)[kObsVals], T rho0, T drho, T jx, T jy, T jz,
                                                      double w)
{
    const T irho = recip(rho0 + drho);
    double o[kObs];
    o[0] = (double)drho;
    o[1] = (double)jx;
    o[2] = (double)jy;
    o[3] = (double)jz;
    o[4] = o[1] + o[2] + o[3];
    o[7] = (double)(jx * irho);
    o[8] = (double)(jy * irho);
    o[9] = (double)(jz * irho);
#pragma unroll
    for (int q = 0; q < kObs; ++q) {
        if (q == 5 || q == 6) continue;
        const double wo = w * o[q];
        acc[2 * q] += wo;
        acc[2 * q + 1] = fma(wo, o[q], acc[2 * q + 1]);
    }
    acc[2 * kObs] += isfinite(o[0]) ? 0.0 : w;
}
template <typename T>
__device__ __forceinline__ void add_observables_stress(double (&acc)[kObsVals], T pdiag, T poff, double w)
{
    const double o5 = (double)pdiag, o6 = (double)poff;
    const double w5 = w * o5, w6 = w * o6;
    acc[10] += w5;
    acc[11] = fma(w5, o5, acc[11]);
    acc[12] += w6;
    acc[13] = fma(w6, o6, acc[13]);
}

// Stage 1 with the observables (the FP32 path): one workgroup per chunk and
// all six fields, in two groups so that one group's accumulators and loads
// fit the registers of four waves per SIMD: each thread reads drho, jx, jy, jz
// of its column's rows (batches of four rows) into their y-transforms and the
// observables of drho and j, finishes those four fields (dft_plane_finish),
// then reads pdiag and poff the same way.  A lane without a column adds with
// weight 0.  The observables record of the chunk goes to partials[blockIdx.x].
// Every sum takes the same values in the same order as with one group.
template <typename T>
__device__ __forceinline__ void dft_plane_obs_body(const RepDev& R, uint32_t chunk, const T* __restrict__ fields,
                                                   const double2* __restrict__ twx, const double2* __restrict__ twy,
                                                   double2 (*Ys)[kDftCols][4], double2 (*Tx)[kDftCols],
                                                   double2* dft, double* partials)
{
    const uint32_t nx = R.nx, ny = R.ny;
    const uint64_t N = R.n;
    const DftLane g = dft_lane(R, chunk);
    const T* col = fields + R.field_offset + g.off;
    const T rho0 = rep_param<T>(R.rho0, R.rho0f);
    dft_load_tx(R, g, twx, Tx);
    double acc[kObsVals];
#pragma unroll
    for (int q = 0; q < kObsVals; ++q) acc[q] = 0.0;
    // fields F0 .. F0 + NF - 1, rows in increasing y
    auto group = [&](auto nf_tag, auto f0_tag, auto&& add_obs) {
        constexpr int NF = decltype(nf_tag)::value, F0 = decltype(f0_tag)::value;
        YSum a[NF];
        auto add_row = [&](const T (&v)[NF], uint32_t y) {
#pragma unroll
            for (int f = 0; f < NF; ++f) a[f].add(g.keep * (double)v[f], y, ny, twy);
            add_obs(v);
        };
        uint32_t y = g.ylo;
        for (; y + 4 <= g.yhi; y += 4) {
            T v[4][NF];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int f = 0; f < NF; ++f) v[u][f] = col[(uint64_t)(F0 + f) * N + (uint64_t)(y + u) * nx];
#pragma unroll
            for (int u = 0; u < 4; ++u) add_row(v[u], y + u);
        }
        for (; y < g.yhi; ++y) {
            T v[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) v[f] = col[(uint64_t)(F0 + f) * N + (uint64_t)y * nx];
            add_row(v, y);
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) dft_plane_finish(R, g, a[f], F0 + f, Ys, Tx, dft);
    };
    group(std::integral_constant<int, 4>{}, std::integral_constant<int, 0>{},
          [&](const T (&v)[4]) { add_observables_rho_j<T>(acc, rho0, v[0], v[1], v[2], v[3], g.keep); });
    group(std::integral_constant<int, 2>{}, std::integral_constant<int, 4>{},
          [&](const T (&v)[2]) { add_observables_stress<T>(acc, v[0], v[1], g.keep); });
    block_sum_store<kObsVals>(acc, partials + (size_t)blockIdx.x * kPartialStride);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void dft_plane_obs_kernel(const RepDev* reps, const uint32_t* first,
                                                               int32_t nrep, const T* __restrict__ fields,
                                                               const double2* __restrict__ tw, double2* dft,
                                                               double* partials)
{
    __shared__ double2 Ys[4][kDftCols][4];
    __shared__ double2 Tx[3][kDftCols];
    const int r = replica_of_block(first, nrep, blockIdx.x);
    const RepDev R = uniform_rep(reps[r]);
    const double2* twg = tw + R.tw_offset;            // e^{2 pi i m / nx}, then e^{2 pi i m / ny}
    dft_plane_obs_body<T>(R, blockIdx.x - first[r], fields, twg, twg + R.nx, Ys, Tx, dft, partials);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void dft_plane_kernel(const RepDev* reps, const uint32_t* first, int32_t nrep,
                                                           const T* __restrict__ fields,
                                                           const double2* __restrict__ tw, double2* dft)
{
    // Y[wavefront][column][n_y = 0..3] (16 KiB) and the x twiddles of the chunk (3 KiB)
    __shared__ double2 Ys[4][kDftCols][4];
    __shared__ double2 Tx[3][kDftCols];
    const int r = replica_of_block(first, nrep, blockIdx.x);
    const RepDev R = uniform_rep(reps[r]);
    const uint32_t chunk = blockIdx.x - first[r];
    const int fld = blockIdx.y;
    const double2* twg = tw + R.tw_offset;            // e^{2 pi i m / nx}, then e^{2 pi i m / ny}
    dft_plane_body<T>(R, chunk, fld, fields, twg, twg + R.nx, Ys, Tx, dft);
}

__device__ __forceinline__ int shell_of(int n2)
{
    switch (n2) {
    case 1: return 0;
    case 2: return 1;
    case 3: return 2;
    case 4: return 3;
    case 5: return 4;
    case 6: return 5;
    case 8: return 6;
    case 9: return 7;
    default: return -1;
    }
}

__device__ constexpr int kShellCount[kShells] = {6, 12, 8, 6, 24, 24, 12, 30};
constexpr int kDftVec = kDftNx * kDftNy * 7;   // n_x 0..3, n_y -3..3, n_z -3..3

// Stage 2: Z[f][v] = sum_z P[f][z][n_x, n_y] e^{-2 pi i n_z z / nz}, one
// wavefront per wave vector v (grid.z: groups of four): lane l takes the
// planes z = l, l + 64, ... (each plane's column-block records summed in
// block order), and the 64 lane sums are added in a fixed tree order.
__global__ __launch_bounds__(kBlock) void dft_z_kernel(const RepDev* reps, const double2* __restrict__ tw,
                                                       const double2* __restrict__ dft, double2* zout)
{
    const RepDev& R = reps[blockIdx.x];
    const int fld = blockIdx.y;
    const int lane = (int)(threadIdx.x & 63u);
    const int v = (int)blockIdx.z * (kBlock / 64) + (int)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (v >= kDftVec) return;
    const int q = v / (kDftNy * 7);
    const int u = v % 7 - 3;
    const int col = q * kDftNy + ((v / 7) % kDftNy);
    const uint32_t nz = R.nz;
    const double2* twz = tw + R.tw_offset + R.nx + R.ny;
    const uint32_t step = (uint32_t)((u % (int)nz + (int)nz) % (int)nz);
    const uint32_t CB = dft_col_blocks(R.nx);
    const double2* P = dft + R.dft_offset + (uint64_t)fld * nz * CB * kDftPlane + col;
    double zr = 0.0, zi = 0.0;
    for (uint32_t z = (uint32_t)lane; z < nz; z += 64u) {
        double2 p = P[(uint64_t)z * CB * kDftPlane];
        for (uint32_t cb = 1; cb < CB; ++cb) {
            const double2 pc = P[((uint64_t)z * CB + cb) * kDftPlane];
            p = make_double2(p.x + pc.x, p.y + pc.y);
        }
        const double2 t = twz[(uint32_t)(((uint64_t)step * z) % nz)];
        zr += p.x * t.x + p.y * t.y;
        zi += p.y * t.x - p.x * t.y;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        zr += __shfl_xor(zr, off, 64);
        zi += __shfl_xor(zi, off, 64);
    }
    if (lane == 0) zout[((size_t)blockIdx.x * kFields + fld) * kDftVec + v] = make_double2(zr, zi);
}

// Stage 3: shell averages of the five spectra
__global__ __launch_bounds__(kBlock) void dft_shell_kernel(const RepDev* reps, const double2* zin, double* acc)
{
    const RepDev& R = reps[blockIdx.x];
    __shared__ double contrib[kDftVec][kSpec];
    __shared__ int shell[kDftVec];
    const int v = threadIdx.x;
    if (v < kDftVec) {
        const int q = v / (kDftNy * 7);
        const int s = (v / 7) % kDftNy - 3;
        const int u = v % 7 - 3;
        const int sh = shell_of(q * q + s * s + u * u);
        shell[v] = sh;
        double pw[kSpec] = {0, 0, 0, 0, 0};
        if (sh >= 0) {
            double zr[kFields], zi[kFields];
#pragma unroll
            for (int f = 0; f < kFields; ++f) {
                const double2 zz = zin[((size_t)blockIdx.x * kFields + f) * kDftVec + v];
                zr[f] = zz.x;
                zi[f] = zz.y;
            }
            const double w = (q > 0 ? 2.0 : 1.0) / (double)R.n;
            auto pow2 = [](double a, double b) { return a * a + b * b; };
            pw[0] = w * pow2(zr[0], zi[0]);
            pw[1] = w * (pow2(zr[1], zi[1]) + pow2(zr[2], zi[2]) + pow2(zr[3], zi[3])) / 3.0;
            pw[2] = w * pow2(zr[1] + zr[2] + zr[3], zi[1] + zi[2] + zi[3]);
            pw[3] = w * pow2(zr[4], zi[4]);
            pw[4] = w * pow2(zr[5], zi[5]);
        }
#pragma unroll
        for (int m = 0; m < kSpec; ++m) contrib[v][m] = pw[m];
    }
    __syncthreads();
    if (threadIdx.x < kSpec * kShells) {
        const int m = threadIdx.x / kShells, sh = threadIdx.x % kShells;
        double s = 0.0;
        for (int j = 0; j < kDftVec; ++j)
            if (shell[j] == sh) s += contrib[j][m];
        acc[(size_t)blockIdx.x * kAccStride + kAccSpec + m * kShells + sh] += s / (double)kShellCount[sh];
    }
}

hipError_t launch_dft(int precision, const RepDev* reps, int32_t nrep, const uint32_t* first, uint32_t nchunks,
                      const void* fields, const double2* tw, double2* dft, double2* zbuf, double* acc,
                      double* partials, hipStream_t s)
{
    if (precision == kFP64)
        dft_plane_kernel<double><<<dim3(nchunks, kFields), kBlock, 0, s>>>(reps, first, nrep, (const double*)fields,
                                                                           tw, dft);
    else
        dft_plane_obs_kernel<float><<<nchunks, kBlock, 0, s>>>(reps, first, nrep, (const float*)fields, tw, dft,
                                                               partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dft_z_kernel<<<dim3(nrep, kFields, (kDftVec + kBlock / 64 - 1) / (kBlock / 64)), kBlock, 0, s>>>(reps, tw, dft,
                                                                                                  zbuf);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    dft_shell_kernel<<<nrep, kBlock, 0, s>>>(reps, zbuf, acc);
    return hipGetLastError();
}

}  // namespace gmf
