// gmf_fft.hip -- full-box shell spectra (Results section: the structure
// factors S_m(|k|) of the density, momentum and stress fields from a
// normalised FFT of the whole box, averaged over shells of equal |k|).
//
// Per sampling step, after the step kernel has written the six fields:
//   fft_pass_kernel<x>   packs (drho + i jx, jy + i jz, pdiag + i poff) in FP64
//                        and transforms along x;
//   fft_pass_kernel<y>, fft_pass_kernel<z>  transform in place along y and z;
//   spectrum_bin_kernel  unpacks the two real fields of each array at k and -k,
//                        forms the five spectra and sums them into shells
//                        s = round(|n|);
//   spectrum_finalize_kernel  adds each shell average to the accumulators.
// The shell sums are exact integer sums of fixed-point values, so they do not
// depend on the order in which workgroups finish: the same state always gives
// the same bits.  The fixed-point scale of each spectrum is 2^62 divided by
// the sample's sum of squares of that field, which by Parseval's identity
// bounds every partial sum of |m(k)|^2.
#include <hip/hip_runtime.h>

#include "gmf_fft.hpp"
#include "gmf_internal.hpp"

namespace gmf {

// ---------------------------------------------------------------------------
// Line FFTs in LDS: mixed-radix Stockham, forward sign e^{-2 pi i / L}.
// A stage of radix R with Ns = product of the earlier radices maps, for each
// butterfly j < L/R with k = j mod Ns,
//   v_r = in[j + r L/R] e^{-2 pi i k r / (Ns R)},  r < R,
//   out[(j / Ns) Ns R + k + q Ns] = sum_r v_r e^{-2 pi i r q / R}.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
// a * conj(t)
__device__ __forceinline__ double2 cmulc(double2 a, double2 t)
{
    return make_double2(a.x * t.x + a.y * t.y, a.y * t.x - a.x * t.y);
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// -i a and +i a
__device__ __forceinline__ double2 cmi(double2 a) { return make_double2(a.y, -a.x); }
__device__ __forceinline__ double2 cpi(double2 a) { return make_double2(-a.y, a.x); }

template <int R>
__device__ __forceinline__ void small_dft(double2 (&v)[R]);

template <>
__device__ __forceinline__ void small_dft<2>(double2 (&v)[2])
{
    const double2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <>
__device__ __forceinline__ void small_dft<3>(double2 (&v)[3])
{
    // w = e^{-2 pi i / 3} = -1/2 - i sqrt(3)/2
    const double h = 0.86602540378443864676;   // sqrt(3) / 2
    const double2 t1 = cadd(v[1], v[2]);
    const double2 t2 = csub(v[0], cscale(t1, 0.5));
    const double2 t3 = cscale(csub(v[1], v[2]), h);
    v[0] = cadd(v[0], t1);
    v[1] = cadd(t2, cmi(t3));
    v[2] = cadd(t2, cpi(t3));
}

template <>
__device__ __forceinline__ void small_dft<4>(double2 (&v)[4])
{
    // w = -i
    const double2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    const double2 s13 = cadd(v[1], v[3]), d13 = csub(v[1], v[3]);
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, cmi(d13));
    v[3] = cadd(d02, cpi(d13));
}

template <>
__device__ __forceinline__ void small_dft<5>(double2 (&v)[5])
{
    // cos and sin of 2 pi / 5 and 4 pi / 5
    const double c1 = 0.30901699437494742410, c2 = -0.80901699437494742410;
    const double s1 = 0.95105651629515357212, s2 = 0.58778525229247312917;
    const double2 b1 = cadd(v[1], v[4]), b2 = cadd(v[2], v[3]);
    const double2 d1 = csub(v[1], v[4]), d2 = csub(v[2], v[3]);
    const double2 a1 = cadd(v[0], cadd(cscale(b1, c1), cscale(b2, c2)));
    const double2 a2 = cadd(v[0], cadd(cscale(b1, c2), cscale(b2, c1)));
    const double2 e1 = cadd(cscale(d1, s1), cscale(d2, s2));
    const double2 e2 = csub(cscale(d1, s2), cscale(d2, s1));
    v[0] = cadd(v[0], cadd(b1, b2));
    v[1] = cadd(a1, cmi(e1));
    v[4] = cadd(a1, cpi(e1));
    v[2] = cadd(a2, cmi(e2));
    v[3] = cadd(a2, cpi(e2));
}

// One stage over W lines of length L (rows of `ld` values in buf).  twl[m] =
// e^{+2 pi i m / L}.  Every thread reads all its butterflies before the
// barrier and writes them after it, so the stage works in place.  P2: L is a
// power of two (then so are L / R and Ns, and the index arithmetic is shifts
// and masks; lnb = log2(L / R)).
template <int R, bool P2>
__device__ __forceinline__ void fft_stage(double2* buf, const double2* twl, uint32_t L, uint32_t W, uint32_t ld,
                                          uint32_t Ns, uint32_t lnb)
{
    constexpr uint32_t kMaxB = (kFftPoints / R + kBlock - 1) / kBlock;
    const uint32_t nb = L / R, total = W * nb, span = L / (Ns * (uint32_t)R);
    double2 v[kMaxB][R];
    uint32_t dst[kMaxB];
#pragma unroll
    for (uint32_t q = 0; q < kMaxB; ++q) {
        const uint32_t b = threadIdx.x + q * kBlock;
        dst[q] = 0;
        if (b < total) {
            const uint32_t w = P2 ? b >> lnb : b / nb;
            const uint32_t j = b - w * nb;
            const uint32_t k = P2 ? j & (Ns - 1) : j % Ns;
            const double2* line = buf + w * ld;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double2 a = line[j + (uint32_t)r * nb];
                v[q][r] = r == 0 ? a : cmulc(a, twl[k * (uint32_t)r * span]);
            }
            dst[q] = w * ld + (j - k) * (uint32_t)R + k;   // (j / Ns) Ns R + k
        }
    }
    __syncthreads();
#pragma unroll
    for (uint32_t q = 0; q < kMaxB; ++q) {
        const uint32_t b = threadIdx.x + q * kBlock;
        if (b < total) {
            small_dft<R>(v[q]);
#pragma unroll
            for (int r = 0; r < R; ++r) buf[dst[q] + (uint32_t)r * Ns] = v[q][r];
        }
    }
    __syncthreads();
}

template <bool P2>
__device__ __forceinline__ void fft_lines(double2* buf, const double2* twl, uint32_t L, uint32_t W, uint32_t ld)
{
    // the stages of fft_plan, taken from the part of L not yet transformed (no
    // indexed array, which would live in scratch memory)
    uint32_t Ns = 1, m = L;
    while (m > 1) {
        const uint32_t R = m % 4 == 0 ? 4u : (m % 2 == 0 ? 2u : (m % 3 == 0 ? 3u : 5u));
        const uint32_t lnb = P2 ? (uint32_t)__builtin_ctz(L / R) : 0u;
        if (P2) {
            if (R == 4) fft_stage<4, true>(buf, twl, L, W, ld, Ns, lnb);
            else fft_stage<2, true>(buf, twl, L, W, ld, Ns, lnb);
        } else {
            switch (R) {
            case 4: fft_stage<4, false>(buf, twl, L, W, ld, Ns, 0); break;
            case 2: fft_stage<2, false>(buf, twl, L, W, ld, Ns, 0); break;
            case 3: fft_stage<3, false>(buf, twl, L, W, ld, Ns, 0); break;
            default: fft_stage<5, false>(buf, twl, L, W, ld, Ns, 0); break;
            }
        }
        Ns *= R;
        m /= R;
    }
}

// Replica of workgroup b: first[r] <= b < first[r + 1] (first[0] = 0).
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

// One pass of the 3D transform along AXIS for packed array `arr`, tile `tile`
// of replica R.  AXIS 0 builds the packed values from the sampled fields.
// P2: the line length L and the lines per tile W are powers of two (the
// index arithmetic is then shifts and masks).
template <typename T, int AXIS, bool P2>
__device__ __forceinline__ void fft_pass_body(const RepDev& R, uint32_t tile, uint32_t arr, uint32_t L, uint32_t W,
                                              const T* __restrict__ fields, const double2* __restrict__ tw,
                                              double2* spec, double2* lds)
{
    const uint32_t nx = R.nx, ny = R.ny, nz = R.nz;
    const uint32_t ld = L + 1;
    const uint32_t lL = P2 ? (uint32_t)__builtin_ctz(L) : 0u, lW = P2 ? (uint32_t)__builtin_ctz(W) : 0u;
    double2* buf = lds;
    double2* twl = lds + W * ld;
    const uint32_t toff = R.tw_offset + (AXIS == 0 ? 0u : (AXIS == 1 ? nx : nx + ny));
    for (uint32_t m = threadIdx.x; m < L; m += kBlock) twl[m] = tw[toff + m];

    // tile origin: AXIS 0: rows tile*W ..; AXIS 1/2: columns x0 .. x0+W-1 of plane z (AXIS 1) or row y (AXIS 2)
    uint32_t row0 = 0, x0 = 0, fixed = 0;
    if (AXIS == 0) {
        row0 = tile * W;
    } else {
        const uint32_t per = (nx + W - 1) / W;
        fixed = tile / per;
        x0 = (tile - fixed * per) * W;
    }
    const uint64_t N = R.n;
    double2* S = spec + R.spec_offset + (uint64_t)arr * N;
    const uint32_t tot = W * L;
    auto node_of = [&](uint32_t i, uint32_t& w, uint32_t& j, uint32_t& node) -> bool {
        if (AXIS == 0) {
            w = P2 ? i >> lL : i / L;
            j = i - w * L;
            const uint32_t row = row0 + w;
            node = row * nx + j;
            return row < ny * nz;
        }
        j = P2 ? i >> lW : i / W;
        w = i - j * W;
        const uint32_t x = x0 + w;
        node = AXIS == 1 ? x + nx * (j + ny * fixed) : x + nx * (fixed + ny * j);
        return x < nx;
    };
    // all global loads of the thread are issued before the first LDS store
    constexpr uint32_t kPer = kFftPoints / kBlock;
    double2 v[kPer];
    uint32_t at[kPer];
#pragma unroll
    for (uint32_t q = 0; q < kPer; ++q) {
        const uint32_t i = threadIdx.x + q * kBlock;
        uint32_t w = 0, j = 0, node = 0;
        v[q] = make_double2(0.0, 0.0);
        at[q] = ~0u;
        if (i < tot) {
            if (node_of(i, w, j, node)) {
                if (AXIS == 0) {
                    const T* F = fields + R.field_offset + (uint64_t)(2 * arr) * N;
                    v[q] = make_double2((double)F[node], (double)F[N + node]);
                } else {
                    v[q] = S[node];
                }
            }
            at[q] = w * ld + j;
        }
    }
#pragma unroll
    for (uint32_t q = 0; q < kPer; ++q)
        if (at[q] != ~0u) buf[at[q]] = v[q];
    __syncthreads();
    fft_lines<P2>(buf, twl, L, W, ld);
#pragma unroll
    for (uint32_t q = 0; q < kPer; ++q) {
        const uint32_t i = threadIdx.x + q * kBlock;
        uint32_t w, j, node;
        if (i < tot && node_of(i, w, j, node)) S[node] = buf[w * ld + j];
    }
}

template <typename T, int AXIS>
__global__ __launch_bounds__(kBlock) void fft_pass_kernel(const RepDev* reps, const uint32_t* first, int32_t nrep,
                                                          const T* __restrict__ fields,
                                                          const double2* __restrict__ tw, double2* spec)
{
    extern __shared__ double2 lds[];
    const int r = replica_of_block(first, nrep, blockIdx.x);
    const RepDev& R = reps[r];
    const uint32_t tile = blockIdx.x - first[r];
    const uint32_t L = fft_axis_len(AXIS, R.nx, R.ny, R.nz);
    const uint32_t W = fft_tile_lines(AXIS, L, R.nx);
    if ((L & (L - 1)) == 0 && (W & (W - 1)) == 0)
        fft_pass_body<T, AXIS, true>(R, tile, blockIdx.y, L, W, fields, tw, spec, lds);
    else
        fft_pass_body<T, AXIS, false>(R, tile, blockIdx.y, L, W, fields, tw, spec, lds);
}

// Fixed-point scale of each spectrum for the current sample: 2^62 / bound,
// bound = sum over the box of the field squared (for j: the mean over the
// three components); 0 when the field is identically zero.
__device__ __forceinline__ void spectrum_scales(const double* ssq, double (&scale)[kSpec])
{
    const double bound[kSpec] = {ssq[0], (ssq[1] + ssq[2] + ssq[3]) / 3.0, ssq[4], ssq[5], ssq[6]};
#pragma unroll
    for (int m = 0; m < kSpec; ++m) scale[m] = bound[m] > 0.0 ? 0x1p62 / bound[m] : 0.0;
}

// Each wavefront takes kBinPoints / 4 consecutive wave vectors of the half
// space that bin_nodes() describes, 64 at a time (one per lane, so the loads
// of k and of -k are contiguous).  The spectra of real fields take equal
// values at k and -k, so a wave vector whose partner -k lies outside that
// range counts twice, one that is its own partner once, and the upper member
// of a pair inside the range not at all: every wave vector of the box is
// counted once, with half the loads.  Neighbouring
// lanes mostly share a shell: a segmented scan over the lanes, keyed by the
// shell, sums the five powers of each run of equal shell in FP64, and the last
// lane of each run adds its rounded fixed-point value to the workgroup's shell
// bins in LDS.
__global__ __launch_bounds__(kBlock) void spectrum_bin_kernel(const RepDev* reps, const uint32_t* first, int32_t nrep,
                                                              const double2* __restrict__ spec,
                                                              const double* __restrict__ sample_sq,
                                                              unsigned long long* bins)
{
    extern __shared__ unsigned long long lbin[];
    const int r = replica_of_block(first, nrep, blockIdx.x);
    const RepDev& R = reps[r];
    const uint32_t ns = R.nshell;
    for (uint32_t i = threadIdx.x; i < ns * kSpec; i += kBlock) lbin[i] = 0ull;
    double scale[kSpec];
    spectrum_scales(sample_sq + (size_t)r * kObs, scale);
    __syncthreads();

    const uint32_t nx = R.nx, ny = R.ny, nz = R.nz;
    const uint64_t N = R.n;
    const double invn = 1.0 / (double)N;
    const double2* Z = spec + R.spec_offset;
    const int lane = (int)(threadIdx.x & 63u);
    const uint32_t wave = threadIdx.x >> 6;
    const uint64_t Nh = bin_nodes(nx, ny, nz);
    const uint32_t base = (blockIdx.x - first[r]) * kBinPoints + wave * (kBinPoints / (kBlock / 64));
    for (uint32_t it = 0; it < kBinPoints / kBlock; ++it) {
        const uint32_t n = base + it * 64u + (uint32_t)lane;
        double v[kSpec] = {0.0, 0.0, 0.0, 0.0, 0.0};
        uint32_t s = 0;   // 0: no contribution (k = 0, past the half space, or counted at -k)
        if (n < Nh) {
            const uint32_t yz = fdiv(n, R.divx);
            const uint32_t x = n - yz * nx;
            const uint32_t z = fdiv(yz, R.divy);
            const uint32_t y = yz - z * ny;
            // -k
            const uint32_t mx = x == 0 ? 0 : nx - x, my = y == 0 ? 0 : ny - y, mz = z == 0 ? 0 : nz - z;
            const uint32_t mn = mx + nx * (my + ny * mz);
            const int64_t fx = signed_freq(x, nx), fy = signed_freq(y, ny), fz = signed_freq(z, nz);
            const uint64_t n2 = (uint64_t)(fx * fx + fy * fy + fz * fz);
            if (n2 > 0 && (mn >= Nh || n <= mn)) {
                s = shell_of(n2);
                const double wk = n == mn ? invn : 2.0 * invn;   // 1/N per wave vector counted
                double2 X[2 * kFftArrays];
#pragma unroll
                for (int c = 0; c < kFftArrays; ++c) {
                    const double2 A = Z[(uint64_t)c * N + n], B = Z[(uint64_t)c * N + mn];
                    // A = F(k) + i G(k), B = F(-k) + i G(-k) for transforms F, G of real fields:
                    // F(k) = (A + conj B) / 2, G(k) = (A - conj B) / (2 i)
                    X[2 * c] = make_double2(0.5 * (A.x + B.x), 0.5 * (A.y - B.y));
                    X[2 * c + 1] = make_double2(0.5 * (A.y + B.y), -0.5 * (A.x - B.x));
                }
                // X: drho, jx, jy, jz, pdiag, poff
                const double2 js = make_double2(X[1].x + X[2].x + X[3].x, X[1].y + X[2].y + X[3].y);
                auto pw = [](double2 a) { return a.x * a.x + a.y * a.y; };
                v[0] = pw(X[0]) * wk;
                v[1] = (pw(X[1]) + pw(X[2]) + pw(X[3])) * (wk / 3.0);
                v[2] = pw(js) * wk;
                v[3] = pw(X[4]) * wk;
                v[4] = pw(X[5]) * wk;
            }
        }
        // segmented inclusive scan over the lanes; a run starts where the shell changes
        const uint32_t s_prev = (uint32_t)__shfl_up((int)s, 1, 64);
        const uint32_t s_next = (uint32_t)__shfl_down((int)s, 1, 64);
        int flag = (lane == 0 || s_prev != s) ? 1 : 0;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            double pv[kSpec];
#pragma unroll
            for (int m = 0; m < kSpec; ++m) pv[m] = __shfl_up(v[m], d, 64);
            const int pf = __shfl_up(flag, d, 64);
            if (lane >= d && !flag) {
#pragma unroll
                for (int m = 0; m < kSpec; ++m) v[m] += pv[m];
                flag = pf;
            }
        }
        const bool tail = lane == 63 || s_next != s;
        if (tail && s > 0) {
#pragma unroll
            for (int m = 0; m < kSpec; ++m) {
                const unsigned long long q = (unsigned long long)(v[m] * scale[m] + 0.5);
                if (q) atomicAdd(&lbin[s * kSpec + m], q);
            }
        }
    }
    __syncthreads();
    unsigned long long* gb = bins + (size_t)R.shell_offset * kSpec;
    for (uint32_t i = threadIdx.x; i < ns * kSpec; i += kBlock)
        if (lbin[i]) atomicAdd(&gb[i], lbin[i]);
}

// Shell averages of the sample into the FP64 accumulators; the integer bins
// are cleared for the next sample.
__global__ __launch_bounds__(kBlock) void spectrum_finalize_kernel(const RepDev* reps, const double* sample_sq,
                                                                   const int64_t* counts,
                                                                   unsigned long long* bins, double* sacc)
{
    const RepDev& R = reps[blockIdx.x];
    double scale[kSpec];
    spectrum_scales(sample_sq + (size_t)blockIdx.x * kObs, scale);
    const uint32_t base = R.shell_offset;
    for (uint32_t i = threadIdx.x; i < R.nshell * kSpec; i += kBlock) {
        const uint32_t s = i / kSpec, m = i - s * kSpec;
        const unsigned long long q = bins[(size_t)base * kSpec + i];
        const int64_t c = counts[base + s];
        if (c > 0 && scale[m] > 0.0) sacc[(size_t)base * kSpec + i] += ((double)q / scale[m]) / (double)c;
        bins[(size_t)base * kSpec + i] = 0ull;
    }
}

hipError_t launch_spectrum(int precision, const RepDev* reps, int32_t nrep, const uint32_t* first, const uint32_t* nblk,
                           const void* fields, const double2* tw, double2* spec, const double* sample_sq,
                           const int64_t* counts, unsigned long long* bins, double* sacc, const size_t* lds,
                           hipStream_t s)
{
    // first: 4 prefix arrays of nrep + 1 entries (passes x, y, z, binning); nblk: their totals
    for (int axis = 0; axis < 3; ++axis) {
        const dim3 grid(nblk[axis], kFftArrays);
        const uint32_t* f = first + (size_t)axis * (nrep + 1);
        if (precision == kFP64) {
            const double* fl = (const double*)fields;
            if (axis == 0) fft_pass_kernel<double, 0><<<grid, kBlock, lds[0], s>>>(reps, f, nrep, fl, tw, spec);
            else if (axis == 1) fft_pass_kernel<double, 1><<<grid, kBlock, lds[1], s>>>(reps, f, nrep, fl, tw, spec);
            else fft_pass_kernel<double, 2><<<grid, kBlock, lds[2], s>>>(reps, f, nrep, fl, tw, spec);
        } else {
            const float* fl = (const float*)fields;
            if (axis == 0) fft_pass_kernel<float, 0><<<grid, kBlock, lds[0], s>>>(reps, f, nrep, fl, tw, spec);
            else if (axis == 1) fft_pass_kernel<float, 1><<<grid, kBlock, lds[1], s>>>(reps, f, nrep, fl, tw, spec);
            else fft_pass_kernel<float, 2><<<grid, kBlock, lds[2], s>>>(reps, f, nrep, fl, tw, spec);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    spectrum_bin_kernel<<<nblk[3], kBlock, lds[3], s>>>(reps, first + 3 * (size_t)(nrep + 1), nrep, spec, sample_sq,
                                                        bins);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    spectrum_finalize_kernel<<<nrep, kBlock, 0, s>>>(reps, sample_sq, counts, bins, sacc);
    return hipGetLastError();
}

}  // namespace gmf
