// gmf_fft.hip -- full-box shell spectra (Results section: the structure
// factors S_m(|k|) of the density, momentum and stress fields from a
// normalised FFT of the whole box, averaged over shells of equal |k|).
//
// Per sampling step, after the step kernel has written the six fields:
//   fft_x_kernel     packs two real fields as one complex line (drho + i pdiag,
//                    poff + i jx, jy + i jz, and jsum = jx + jy + jz of rows
//                    2m + i 2m + 1), transforms along x and writes the half
//                    spectra kx = 0 .. floor(nx / 2) of the seven fields;
//   fft_y_kernel     transforms each half spectrum in place along y;
//   fft_zbin_kernel  transforms each half spectrum's columns along z and sums
//                    the power of every wave vector into the shells
//                    s = round(|n|) of that field's spectrum;
//   spectrum_finalize_kernel  adds each shell average to the accumulators.
// The passes run either pass by pass over all seven fields, or group by group
// (x pass of one group, then y and z passes of its half spectra), which keeps
// a group's half spectra in the memory-side cache between the passes.
// Every wave vector with kx = 0 (or kx = nx / 2 for even nx) is counted once;
// every other one stands also for its mirror -k (same shell, same power, a
// column the half spectra do not hold) and is counted twice.  The transforms
// run in the kernel precision, complex FP32 for the FP32 path and FP64 for the
// FP64 path.  The shell sums are exact integer sums of fixed-point values, so
// they do not depend on the order in which workgroups finish: the same state
// always gives the same bits.  The fixed-point scale of each spectrum is 2^62
// divided by the sample's sum of squares of that field, which by Parseval's
// identity bounds every partial sum of |m(k)|^2.
#include <hip/hip_runtime.h>

#include "gmf_fft.hpp"
#include "gmf_internal.hpp"

namespace gmf {

// ---------------------------------------------------------------------------
// Complex values of the transform precision Rt
// ---------------------------------------------------------------------------
template <typename Rt>
struct CxOf;
template <>
struct CxOf<float> {
    using type = float2;
};
template <>
struct CxOf<double> {
    using type = double2;
};

__device__ __forceinline__ float2 cmake(float a, float b) { return make_float2(a, b); }
__device__ __forceinline__ double2 cmake(double a, double b) { return make_double2(a, b); }

template <typename C>
__device__ __forceinline__ C cadd(C a, C b)
{
    return cmake(a.x + b.x, a.y + b.y);
}
template <typename C>
__device__ __forceinline__ C csub(C a, C b)
{
    return cmake(a.x - b.x, a.y - b.y);
}
// a * conj(t)
template <typename C>
__device__ __forceinline__ C cmulc(C a, C t)
{
    return cmake(a.x * t.x + a.y * t.y, a.y * t.x - a.x * t.y);
}
template <typename C, typename Rt>
__device__ __forceinline__ C cscale(C a, Rt s)
{
    return cmake(a.x * s, a.y * s);
}
// -i a and +i a
template <typename C>
__device__ __forceinline__ C cmi(C a)
{
    return cmake(a.y, -a.x);
}
template <typename C>
__device__ __forceinline__ C cpi(C a)
{
    return cmake(-a.y, a.x);
}

// ---------------------------------------------------------------------------
// Workgroup barrier ordering LDS accesses only: global loads stay in flight
// across it (a full barrier would wait for every outstanding load, the next
// tile's too).  No thread of these kernels reads global memory that another
// thread of its workgroup writes.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------------------
// DFTs of R points in registers, forward sign: v_q <- sum_r v_r e^{-2 pi i r q / R}.
// ---------------------------------------------------------------------------
template <typename Rt, typename C>
__device__ __forceinline__ void small_dft(C (&)[1])
{
}

template <typename Rt, typename C>
__device__ __forceinline__ void small_dft(C (&v)[2])
{
    const C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <typename Rt, typename C>
__device__ __forceinline__ void small_dft(C (&v)[3])
{
    // w = e^{-2 pi i / 3} = -1/2 - i sqrt(3)/2
    const Rt h = (Rt)0.86602540378443864676;   // sqrt(3) / 2
    const C t1 = cadd(v[1], v[2]);
    const C t2 = csub(v[0], cscale(t1, (Rt)0.5));
    const C t3 = cscale(csub(v[1], v[2]), h);
    v[0] = cadd(v[0], t1);
    v[1] = cadd(t2, cmi(t3));
    v[2] = cadd(t2, cpi(t3));
}

template <typename Rt, typename C>
__device__ __forceinline__ void small_dft(C (&v)[4])
{
    // w = -i
    const C s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    const C s13 = cadd(v[1], v[3]), d13 = csub(v[1], v[3]);
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, cmi(d13));
    v[3] = cadd(d02, cpi(d13));
}

template <typename Rt, typename C>
__device__ __forceinline__ void small_dft(C (&v)[5])
{
    // cos and sin of 2 pi / 5 and 4 pi / 5
    const Rt c1 = (Rt)0.30901699437494742410, c2 = (Rt)-0.80901699437494742410;
    const Rt s1 = (Rt)0.95105651629515357212, s2 = (Rt)0.58778525229247312917;
    const C b1 = cadd(v[1], v[4]), b2 = cadd(v[2], v[3]);
    const C d1 = csub(v[1], v[4]), d2 = csub(v[2], v[3]);
    const C a1 = cadd(v[0], cadd(cscale(b1, c1), cscale(b2, c2)));
    const C a2 = cadd(v[0], cadd(cscale(b1, c2), cscale(b2, c1)));
    const C e1 = cadd(cscale(d1, s1), cscale(d2, s2));
    const C e2 = csub(cscale(d1, s2), cscale(d2, s1));
    v[0] = cadd(v[0], cadd(b1, b2));
    v[1] = cadd(a1, cmi(e1));
    v[4] = cadd(a1, cpi(e1));
    v[2] = cadd(a2, cmi(e2));
    v[3] = cadd(a2, cpi(e2));
}

// cos and sin of 2 pi e / 16
constexpr double kC1 = 0.92387953251128675613;   // cos(pi / 8)
constexpr double kS1 = 0.38268343236508977173;   // sin(pi / 8)
constexpr double kH = 0.70710678118654752440;    // sqrt(2) / 2
constexpr double cos16(int e)
{
    return e == 0 ? 1.0 : e == 1 ? kC1 : e == 2 ? kH : e == 3 ? kS1 : e == 4 ? 0.0 : e == 5 ? -kS1 : e == 6 ? -kH
         : e == 7 ? -kC1 : e == 8 ? -1.0 : e == 9 ? -kC1 : e == 10 ? -kH : e == 11 ? -kS1 : e == 12 ? 0.0
         : e == 13 ? kS1 : e == 14 ? kH : kC1;
}
constexpr double sin16(int e) { return cos16((e + 12) & 15); }

// a e^{-2 pi i e / 16}; e is a constant once the callers' loops are unrolled
template <typename Rt, typename C>
__device__ __forceinline__ C rot16(C a, int e)
{
    e &= 15;
    if (e == 0) return a;
    if (e == 4) return cmi(a);
    if (e == 8) return cmake(-a.x, -a.y);
    if (e == 12) return cpi(a);
    const Rt c = (Rt)cos16(e), s = (Rt)sin16(e);
    return cmake(a.x * c + a.y * s, a.y * c - a.x * s);
}

// R = 8 as 4 x 2: n = 2 n1 + n2, q = q1 + 4 q2
template <typename Rt, typename C>
__device__ __forceinline__ void small_dft(C (&v)[8])
{
    C y[2][4];
#pragma unroll
    for (int n2 = 0; n2 < 2; ++n2) {
        C t[4] = {v[n2], v[n2 + 2], v[n2 + 4], v[n2 + 6]};
        small_dft<Rt>(t);
#pragma unroll
        for (int q1 = 0; q1 < 4; ++q1) y[n2][q1] = rot16<Rt>(t[q1], 2 * n2 * q1);
    }
#pragma unroll
    for (int q1 = 0; q1 < 4; ++q1) {
        C t[2] = {y[0][q1], y[1][q1]};
        small_dft<Rt>(t);
        v[q1] = t[0];
        v[q1 + 4] = t[1];
    }
}

// R = 16 as 4 x 4: n = 4 n1 + n2, q = q1 + 4 q2
template <typename Rt, typename C>
__device__ __forceinline__ void small_dft(C (&v)[16])
{
    C y[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        C t[4] = {v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]};
        small_dft<Rt>(t);
#pragma unroll
        for (int q1 = 0; q1 < 4; ++q1) y[n2][q1] = rot16<Rt>(t[q1], n2 * q1);
    }
#pragma unroll
    for (int q1 = 0; q1 < 4; ++q1) {
        C t[4] = {y[0][q1], y[1][q1], y[2][q1], y[3][q1]};
        small_dft<Rt>(t);
#pragma unroll
        for (int q2 = 0; q2 < 4; ++q2) v[q1 + 4 * q2] = t[q2];
    }
}

// ---------------------------------------------------------------------------
// Line FFTs of a tile: W lines of length L, mixed-radix Stockham.  A stage of
// radix R with Ns = product of the earlier radices maps, for each butterfly
// j < L/R with k = j mod Ns,
//   v_r = in[j + r L/R] e^{-2 pi i k r / (Ns R)},  r < R,
//   out[(j / Ns) Ns R + k + q Ns] = sum_r v_r e^{-2 pi i r q / R},
// so the outputs come in natural order.  The first stage takes its inputs
// from load.get(h, p) with h = load.col(w) (line w, global memory) and the
// last one hands point p of line w to out.put(h, p, value), h = out.col(w, ok)
// (nothing for a line with ok false); the stages between work in place on LDS
// rows of `ld` values (point p in slot fft_phys(p)), reading every butterfly
// of the thread before a barrier and writing after it.  WF: consecutive butterflies belong
// to consecutive lines (the y and z passes, whose lines are the columns of a
// half spectrum), else to one line (the x pass, whose lines are contiguous).
// Butterflies past the tile repeat butterfly 0's loads and store nothing.
// ---------------------------------------------------------------------------
template <bool WF>
__device__ __forceinline__ void butterfly(uint32_t b, const SmallDiv& dW, const SmallDiv& dnb, uint32_t& w, uint32_t& j)
{
    if (WF) {
        j = dW.div(b);
        w = b - j * dW.d;
    } else {
        w = dnb.div(b);
        j = b - w * dnb.d;
    }
}

template <int R>
constexpr uint32_t stage_slots()
{
    return (kFftTilePts / R + kBlock - 1) / kBlock;
}

template <int R, bool WF, typename Rt, class Load>
__device__ __forceinline__ void stage_first(typename CxOf<Rt>::type* buf, uint32_t L, uint32_t W, uint32_t ld,
                                            const SmallDiv& dW, const Load& load)
{
    using C = typename CxOf<Rt>::type;
    constexpr uint32_t kB = stage_slots<R>();
    const uint32_t nb = L / R, total = W * nb;
    const SmallDiv dnb(nb);
    C v[kB][R];
#pragma unroll
    for (uint32_t q = 0; q < kB; ++q) {
        const uint32_t b0 = threadIdx.x + q * kBlock;
        uint32_t w, j;
        butterfly<WF>(b0 < total ? b0 : 0u, dW, dnb, w, j);
        const auto h = load.col(w);
#pragma unroll
        for (int r = 0; r < R; ++r) v[q][r] = load.get(h, j + (uint32_t)r * nb);
    }
#pragma unroll
    for (uint32_t q = 0; q < kB; ++q) {
        const uint32_t b = threadIdx.x + q * kBlock;
        if (b < total) {
            uint32_t w, j;
            butterfly<WF>(b, dW, dnb, w, j);
            small_dft<Rt>(v[q]);
#pragma unroll
            for (int r = 0; r < R; ++r) buf[w * ld + fft_phys(j * (uint32_t)R + (uint32_t)r)] = v[q][r];
        }
    }
}

// the inputs of a stage after the first, twiddled
template <int R, bool WF, typename Rt>
__device__ __forceinline__ void stage_read(const typename CxOf<Rt>::type* buf, const typename CxOf<Rt>::type* twl,
                                           uint32_t L, uint32_t W, uint32_t ld, uint32_t Ns, const SmallDiv& dW,
                                           const SmallDiv& dnb, const SmallDiv& dNs,
                                           typename CxOf<Rt>::type (&v)[stage_slots<R>()][R])
{
    constexpr uint32_t kB = stage_slots<R>();
    const uint32_t nb = L / R, total = W * nb, span = L / (Ns * (uint32_t)R);
#pragma unroll
    for (uint32_t q = 0; q < kB; ++q) {
        const uint32_t b0 = threadIdx.x + q * kBlock;
        uint32_t w, j;
        butterfly<WF>(b0 < total ? b0 : 0u, dW, dnb, w, j);
        const uint32_t k = j - dNs.div(j) * Ns;
        const auto* line = buf + w * ld;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const auto a = line[fft_phys(j + (uint32_t)r * nb)];
            v[q][r] = r == 0 ? a : cmulc(a, twl[k * (uint32_t)r * span]);
        }
    }
}

template <int R, bool WF, typename Rt>
__device__ __forceinline__ void stage_mid(typename CxOf<Rt>::type* buf, const typename CxOf<Rt>::type* twl,
                                          uint32_t L, uint32_t W, uint32_t ld, uint32_t Ns, const SmallDiv& dW)
{
    using C = typename CxOf<Rt>::type;
    constexpr uint32_t kB = stage_slots<R>();
    const uint32_t nb = L / R, total = W * nb;
    const SmallDiv dnb(nb), dNs(Ns);
    C v[kB][R];
    stage_read<R, WF, Rt>(buf, twl, L, W, ld, Ns, dW, dnb, dNs, v);
    lds_barrier();
#pragma unroll
    for (uint32_t q = 0; q < kB; ++q) {
        const uint32_t b = threadIdx.x + q * kBlock;
        if (b < total) {
            uint32_t w, j;
            butterfly<WF>(b, dW, dnb, w, j);
            const uint32_t k = j - dNs.div(j) * Ns;
            small_dft<Rt>(v[q]);
#pragma unroll
            for (int r = 0; r < R; ++r)
                buf[w * ld + fft_phys((j - k) * (uint32_t)R + k + (uint32_t)r * Ns)] = v[q][r];
        }
    }
    lds_barrier();
}

// kSync: a barrier between the reads and the outputs (out writes the LDS
// rows in place, or must follow work of other threads)
template <int R, bool WF, bool kSync, typename Rt, class Out>
__device__ __forceinline__ void stage_last(const typename CxOf<Rt>::type* buf, const typename CxOf<Rt>::type* twl,
                                           uint32_t L, uint32_t W, uint32_t ld, uint32_t Ns, const SmallDiv& dW,
                                           const Out& out)
{
    using C = typename CxOf<Rt>::type;
    constexpr uint32_t kB = stage_slots<R>();
    const uint32_t nb = L / R, total = W * nb;
    const SmallDiv dnb(nb), dNs(Ns);
    C v[kB][R];
    stage_read<R, WF, Rt>(buf, twl, L, W, ld, Ns, dW, dnb, dNs, v);
    if (kSync) lds_barrier();
#pragma unroll
    for (uint32_t q = 0; q < kB; ++q) {
        const uint32_t b = threadIdx.x + q * kBlock;
        if (b < total) {
            uint32_t w, j;
            butterfly<WF>(b, dW, dnb, w, j);   // here j < Ns, so k = j
            bool ok;
            const auto h = out.col(w, ok);
            small_dft<Rt>(v[q]);
            if (ok) {
#pragma unroll
                for (int r = 0; r < R; ++r) out.put(h, j + (uint32_t)r * Ns, v[q][r]);
            }
        }
    }
}

// lines of one stage (R = L): load, transform, hand on
template <int R, bool WF, bool kSync, typename Rt, class Load, class Out>
__device__ __forceinline__ void stage_only(uint32_t W, const SmallDiv& dW, const Load& load, const Out& out)
{
    using C = typename CxOf<Rt>::type;
    constexpr uint32_t kB = stage_slots<R>();
    const SmallDiv d1(1u);
    C v[kB][R];
#pragma unroll
    for (uint32_t q = 0; q < kB; ++q) {
        const uint32_t b0 = threadIdx.x + q * kBlock;
        uint32_t w, j;
        butterfly<WF>(b0 < W ? b0 : 0u, dW, d1, w, j);
        const auto h = load.col(w);
#pragma unroll
        for (int r = 0; r < R; ++r) v[q][r] = load.get(h, (uint32_t)r);
    }
    if (kSync) lds_barrier();
#pragma unroll
    for (uint32_t q = 0; q < kB; ++q) {
        const uint32_t b = threadIdx.x + q * kBlock;
        if (b < W) {
            uint32_t w, j;
            butterfly<WF>(b, dW, d1, w, j);
            bool ok;
            const auto h = out.col(w, ok);
            small_dft<Rt>(v[q]);
            if (ok) {
#pragma unroll
                for (int r = 0; r < R; ++r) out.put(h, (uint32_t)r, v[q][r]);
            }
        }
    }
}

// Lines of 2^PL points (PL = 6 .. 10) in fixed stages p2_radix(PL, i), the
// first of radix 16 with one butterfly per thread: p2_load takes a tile's
// sixteen inputs per thread into registers (the loads can be issued while an
// earlier tile is still being transformed), p2_run transforms them.
template <bool WF, int PL, typename Rt, class Load>
__device__ __forceinline__ void p2_load(typename CxOf<Rt>::type (&v)[16], uint32_t W, const SmallDiv& dW,
                                        const Load& load)
{
    constexpr uint32_t nb = (1u << PL) / 16u;
    const uint32_t b = threadIdx.x < W * nb ? threadIdx.x : 0u;
    uint32_t w, j;
    butterfly<WF>(b, dW, SmallDiv(nb), w, j);
    const auto h = load.col(w);
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = load.get(h, j + (uint32_t)r * nb);
}

template <bool WF, bool kSync, int PL, typename Rt, class Out>
__device__ __forceinline__ void p2_run(typename CxOf<Rt>::type (&v)[16], typename CxOf<Rt>::type* buf,
                                       const typename CxOf<Rt>::type* twl, uint32_t W, uint32_t ld,
                                       const SmallDiv& dW, const Out& out)
{
    constexpr uint32_t kL = 1u << PL, nb = kL / 16u;
    constexpr int R1 = p2_radix(PL, 1), R2 = p2_radix(PL, 2);
    if (threadIdx.x < W * nb) {
        uint32_t w, j;
        butterfly<WF>(threadIdx.x, dW, SmallDiv(nb), w, j);
        small_dft<Rt>(v);
#pragma unroll
        for (int r = 0; r < 16; ++r) buf[w * ld + fft_phys(j * 16u + (uint32_t)r)] = v[r];
    }
    lds_barrier();
    if constexpr (R2 == 0) {
        stage_last<R1, WF, kSync, Rt>(buf, twl, kL, W, ld, 16u, dW, out);
    } else {
        stage_mid<R1, WF, Rt>(buf, twl, kL, W, ld, 16u, dW);
        stage_last<R2, WF, kSync, Rt>(buf, twl, kL, W, ld, 16u * (uint32_t)R1, dW, out);
    }
}

// The transform of a tile.  PL = 6 .. 10: every line has 2^PL points and the
// stages are fixed at compile time; PL = 0: any length, the radices chosen at
// run time (fft_next_radix).
template <bool WF, bool kSync, int PL, typename Rt, class Load, class Out>
__device__ __forceinline__ void fft_tile(typename CxOf<Rt>::type* buf, const typename CxOf<Rt>::type* twl, uint32_t L,
                                         uint32_t W, uint32_t ld, const Load& load, const Out& out)
{
    const SmallDiv dW(W);
    if constexpr (PL > 0) {
        typename CxOf<Rt>::type v[16];
        p2_load<WF, PL, Rt>(v, W, dW, load);
        p2_run<WF, kSync, PL, Rt>(v, buf, twl, W, ld, dW, out);
        (void)L;
        return;
    }
    uint32_t R = fft_next_radix(L);
    if (R == L) {
        switch (R) {
        case 16: stage_only<16, WF, kSync, Rt>(W, dW, load, out); break;
        case 8: stage_only<8, WF, kSync, Rt>(W, dW, load, out); break;
        case 5: stage_only<5, WF, kSync, Rt>(W, dW, load, out); break;
        case 4: stage_only<4, WF, kSync, Rt>(W, dW, load, out); break;
        case 3: stage_only<3, WF, kSync, Rt>(W, dW, load, out); break;
        case 2: stage_only<2, WF, kSync, Rt>(W, dW, load, out); break;
        default: stage_only<1, WF, kSync, Rt>(W, dW, load, out); break;
        }
        return;
    }
    switch (R) {
    case 16: stage_first<16, WF, Rt>(buf, L, W, ld, dW, load); break;
    case 8: stage_first<8, WF, Rt>(buf, L, W, ld, dW, load); break;
    case 4: stage_first<4, WF, Rt>(buf, L, W, ld, dW, load); break;
    case 2: stage_first<2, WF, Rt>(buf, L, W, ld, dW, load); break;
    case 3: stage_first<3, WF, Rt>(buf, L, W, ld, dW, load); break;
    default: stage_first<5, WF, Rt>(buf, L, W, ld, dW, load); break;
    }
    lds_barrier();
    uint32_t Ns = R, m = L / R;
    for (;;) {
        R = fft_next_radix(m);
        if (R == m) {
            switch (R) {
            case 16: stage_last<16, WF, kSync, Rt>(buf, twl, L, W, ld, Ns, dW, out); break;
            case 8: stage_last<8, WF, kSync, Rt>(buf, twl, L, W, ld, Ns, dW, out); break;
            case 4: stage_last<4, WF, kSync, Rt>(buf, twl, L, W, ld, Ns, dW, out); break;
            case 2: stage_last<2, WF, kSync, Rt>(buf, twl, L, W, ld, Ns, dW, out); break;
            case 3: stage_last<3, WF, kSync, Rt>(buf, twl, L, W, ld, Ns, dW, out); break;
            default: stage_last<5, WF, kSync, Rt>(buf, twl, L, W, ld, Ns, dW, out); break;
            }
            return;
        }
        switch (R) {
        case 16: stage_mid<16, WF, Rt>(buf, twl, L, W, ld, Ns, dW); break;
        case 8: stage_mid<8, WF, Rt>(buf, twl, L, W, ld, Ns, dW); break;
        case 4: stage_mid<4, WF, Rt>(buf, twl, L, W, ld, Ns, dW); break;
        case 2: stage_mid<2, WF, Rt>(buf, twl, L, W, ld, Ns, dW); break;
        case 3: stage_mid<3, WF, Rt>(buf, twl, L, W, ld, Ns, dW); break;
        default: stage_mid<5, WF, Rt>(buf, twl, L, W, ld, Ns, dW); break;
        }
        Ns *= R;
        m /= R;
    }
}

// twl[m] = e^{+2 pi i m / L} in the transform precision, from the FP64 table
template <typename Rt>
__device__ __forceinline__ void load_twiddles(typename CxOf<Rt>::type* twl, const double2* __restrict__ tw, uint32_t L)
{
    for (uint32_t m = threadIdx.x; m < L; m += kBlock) twl[m] = cmake((Rt)tw[m].x, (Rt)tw[m].y);
}

// ---------------------------------------------------------------------------
// Line sources and sinks of the passes (see fft_tile).
// ---------------------------------------------------------------------------
// x pass: the tile's 3 RT lines are RT rows in three kinds (kind-major, line
// w = kind RT + row), each two real rows packed as a + i b: kind 0
// drho + i pdiag, 1 poff + i jx, 2 jy + i jz.  A row past the box reads row 0
// and is never stored.
template <typename T, typename Rt>
struct XSrc {
    using C = typename CxOf<Rt>::type;
    const T* F;   // the six fields, N values apart
    uint64_t N;
    uint32_t nx, row0, RT, rows;
    SmallDiv dRT;
    struct H {
        const T* a;
        const T* b;
    };
    __device__ __forceinline__ H col(uint32_t w) const
    {
        const uint32_t kind = dRT.div(w), r = row0 + (w - kind * RT);
        const uint64_t base = (uint64_t)(r < rows ? r : 0u) * nx;
        // fields of each kind: (0, 4), (5, 1), (2, 3)
        const uint32_t fa = kind == 0 ? 0u : (kind == 1 ? 5u : 2u), fb = kind == 0 ? 4u : (kind == 1 ? 1u : 3u);
        return H{F + fa * N + base, F + fb * N + base};
    }
    __device__ __forceinline__ C get(const H& h, uint32_t p) const { return cmake((Rt)h.a[p], (Rt)h.b[p]); }
};

// rows of ld values in LDS, point p in slot fft_phys(p)
template <typename C>
struct LdsRows {
    C* buf;
    uint32_t ld;
    __device__ __forceinline__ C* col(uint32_t w, bool& ok) const
    {
        ok = true;
        return buf + w * ld;
    }
    __device__ __forceinline__ void put(C* h, uint32_t p, C v) const { h[fft_phys(p)] = v; }
};

// the columns of a tile as lines of points lstride values apart
template <typename C>
struct ColLines {
    C* S;
    ColTile t;
    SmallDiv dcw;
    uint32_t pstride, lstride;
    __device__ __forceinline__ C* col(uint32_t w, bool& ok) const
    {
        uint32_t off, plane, kx;
        ok = col_offset(t, dcw, pstride, w, off, plane, kx);
        return S + off;
    }
    __device__ __forceinline__ const C* col(uint32_t w) const
    {
        bool ok;
        return col(w, ok);
    }
    __device__ __forceinline__ C get(const C* h, uint32_t p) const { return h[p * lstride]; }
    __device__ __forceinline__ void put(C* h, uint32_t p, C v) const { h[p * lstride] = v; }
};

// ---------------------------------------------------------------------------
// The tiles of workgroup wg: one (the generic kernels), or up to
// kFftTilesPerWG (the kernels with fixed stages), whose first-stage inputs
// are loaded while the previous tile is transformed.  run(tile, v) transforms
// a tile from its inputs v and uses the result; the LDS rows are free again
// after it.
// ---------------------------------------------------------------------------
template <uint32_t TPW, bool WF, int PL, typename Rt, class Make, class Run>
__device__ __forceinline__ void pipelined_tiles(uint32_t wg, uint32_t ntiles, uint32_t W, const SmallDiv& dW,
                                                const Make& make, const Run& run)
{
    using C = typename CxOf<Rt>::type;
    // tiles wg, wg + G, wg + 2 G, ... (G workgroups): the workgroups resident at
    // one time work on neighbouring tiles, which share DRAM pages
    const uint32_t G = (ntiles + TPW - 1) / TPW;
    auto tile_of = [&](uint32_t k) { return wg + k * G < ntiles ? wg + k * G : wg; };
    // two register buffers in turn (a copy between them would wait for the loads)
    C va[16], vb[16];
    p2_load<WF, PL, Rt>(va, W, dW, make(tile_of(0)));
#pragma unroll
    for (uint32_t k = 0; k < TPW; ++k) {
        const bool live = wg + k * G < ntiles;
        if (k % 2 == 0) {
            if (k + 1 < TPW) p2_load<WF, PL, Rt>(vb, W, dW, make(tile_of(k + 1)));
            if (live) run(tile_of(k), va);
        } else {
            if (k + 1 < TPW) p2_load<WF, PL, Rt>(va, W, dW, make(tile_of(k + 1)));
            if (live) run(tile_of(k), vb);
        }
        if (k + 1 < TPW) lds_barrier();
    }
}

// ---------------------------------------------------------------------------
// x pass: RT rows of the box per tile, each as three complex lines (XSrc)
// transformed along x; the half spectra of a and b of a line follow from
// A(k) = (Z(k) + conj Z(-k)) / 2 and B(k) = (Z(k) - conj Z(-k)) / (2 i), with
// Z(-k) in the same LDS row, and that of jsum = jx + jy + jz from theirs.
// ---------------------------------------------------------------------------
template <typename T, typename Rt, int PL>
__device__ __forceinline__ void fft_x_body(const RepDev& R, uint32_t wg, const T* __restrict__ fields,
                                           const double2* __restrict__ tw, typename CxOf<Rt>::type* spec,
                                           typename CxOf<Rt>::type* lds)
{
    using C = typename CxOf<Rt>::type;
    const uint32_t nx = R.nx, ny = R.ny, nz = R.nz, L = nx;
    const uint32_t RT = fft_x_rows(nx), NL = kFftXKinds * RT, ld = fft_ld(0, nx, ny, nz, sizeof(C));
    const uint32_t H = half_len(nx), Hp = half_stride(nx), rows = ny * nz;
    C* buf = lds;
    C* twl = lds + NL * ld;
    load_twiddles<Rt>(twl, tw + R.tw_offset, L);
    const T* F = fields + R.field_offset;
    const uint64_t N = R.n;
    const SmallDiv dH(H), dRT(RT), dW(NL);
    auto make = [&](uint32_t tile) { return XSrc<T, Rt>{F, N, nx, tile * RT, RT, rows, dRT}; };
    const LdsRows<C> out{buf, ld};
    C* S = spec + R.spec_offset;
    const uint64_t HN = (uint64_t)Hp * rows;
    // the seven half spectra of the tile's rows from its transformed lines in LDS
    auto separate = [&](uint32_t tile) {
        const uint32_t row0 = tile * RT;
        for (uint32_t i = threadIdx.x; i < RT * H; i += kBlock) {
            const uint32_t w = dH.div(i), kx = i - w * H, row = row0 + w;
            if (row >= rows) continue;
            const uint32_t km = kx == 0 ? 0u : L - kx;
            const uint64_t o = (uint64_t)row * Hp + kx;
            C js = cmake((Rt)0, (Rt)0);
#pragma unroll
            for (uint32_t kind = 0; kind < kFftXKinds; ++kind) {
                const C* line = buf + (kind * RT + w) * ld;
                const C Z = line[fft_phys(kx)], Zm = line[fft_phys(km)];
                const C A = cmake((Rt)0.5 * (Z.x + Zm.x), (Rt)0.5 * (Z.y - Zm.y));
                const C B = cmake((Rt)0.5 * (Z.y + Zm.y), (Rt)-0.5 * (Z.x - Zm.x));
                const uint32_t fa = kind == 0 ? 0u : (kind == 1 ? 5u : 2u), fb = kind == 0 ? 4u : (kind == 1 ? 1u : 3u);
                S[(uint64_t)fa * HN + o] = A;
                S[(uint64_t)fb * HN + o] = B;
                // jx is kind 1's second field, jy and jz kind 2's
                if (kind == 1) js = B;
                if (kind == 2) js = cadd(js, cadd(A, B));
            }
            S[(uint64_t)6 * HN + o] = js;
        }
    };
    if constexpr (PL > 0) {
        auto run = [&](uint32_t tile, C (&v)[16]) {
            p2_run<false, true, PL, Rt>(v, buf, twl, NL, ld, dW, out);
            lds_barrier();
            separate(tile);
        };
        pipelined_tiles<kFftTilesPerWG[0], false, PL, Rt>(wg, fft_x_tiles(nx, ny, nz), NL, dW, make, run);
    } else {
        fft_tile<false, true, 0, Rt>(buf, twl, L, NL, ld, make(wg), out);
        lds_barrier();
        separate(wg);
    }
}

template <typename T, typename Rt, int PL>
__global__ __launch_bounds__(kBlock) void fft_x_kernel(const RepDev* reps, const uint32_t* first, int32_t nrep,
                                                       const T* __restrict__ fields, const double2* __restrict__ tw,
                                                       typename CxOf<Rt>::type* spec)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    using C = typename CxOf<Rt>::type;
    const int r = replica_of_block(first, nrep, blockIdx.x);
    const RepDev& R = reps[r];
    if (fft_class(R.nx) != PL) return;
    fft_x_body<T, Rt, PL>(R, blockIdx.x - first[r], fields, tw, spec, reinterpret_cast<C*>(lds_raw));
}

// ---------------------------------------------------------------------------
// y pass: tiles of columns of half spectrum `fld`, transformed along y in place.
// ---------------------------------------------------------------------------
template <typename Rt, int PL>
__device__ __forceinline__ void fft_y_body(const RepDev& R, uint32_t wg, uint32_t fld, const double2* __restrict__ tw,
                                           typename CxOf<Rt>::type* spec, typename CxOf<Rt>::type* lds)
{
    using C = typename CxOf<Rt>::type;
    const uint32_t nx = R.nx, ny = R.ny, nz = R.nz, L = ny;
    const FftCols cols = fft_cols(1, nx, ny, nz);
    const uint32_t W = cols.W, ld = fft_ld(1, nx, ny, nz, sizeof(C)), Hp = half_stride(nx);
    C* buf = lds;
    C* twl = lds + W * ld;
    load_twiddles<Rt>(twl, tw + R.tw_offset + nx, L);
    C* Sf = spec + R.spec_offset + (uint64_t)fld * Hp * ny * nz;
    auto make = [&](uint32_t tile) {
        const ColTile t = col_tile(cols, tile);
        return ColLines<C>{Sf, t, SmallDiv(t.cw), ny * Hp, Hp};
    };
    const SmallDiv dW(W);
    if constexpr (PL > 0) {
        auto run = [&](uint32_t tile, C (&v)[16]) { p2_run<true, false, PL, Rt>(v, buf, twl, W, ld, dW, make(tile)); };
        pipelined_tiles<kFftTilesPerWG[1], true, PL, Rt>(wg, cols.tiles(), W, dW, make, run);
    } else {
        const auto io = make(wg);
        fft_tile<true, false, 0, Rt>(buf, twl, L, W, ld, io, io);
    }
}

// grid.y runs over the fields of flist (four bits per field)
template <typename Rt, int PL>
__global__ __launch_bounds__(kBlock) void fft_y_kernel(const RepDev* reps, const uint32_t* first, int32_t nrep,
                                                       uint32_t flist, const double2* __restrict__ tw,
                                                       typename CxOf<Rt>::type* spec)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    using C = typename CxOf<Rt>::type;
    const int r = replica_of_block(first, nrep, blockIdx.x);
    if (fft_class(reps[r].ny) != PL) return;
    fft_y_body<Rt, PL>(reps[r], blockIdx.x - first[r], (flist >> (4u * blockIdx.y)) & 15u, tw, spec,
                       reinterpret_cast<C*>(lds_raw));
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

// Spectrum of half spectrum f (drho, jx, jy, jz, pdiag, poff, jsum): rho, j
// (the mean over three fields), jsum, pdiag, poff.
__device__ __forceinline__ int spectrum_of_field(uint32_t f) { return f == 0 ? 0 : (f <= 3 ? 1 : (f == 6 ? 2 : (int)f - 1)); }

// floor(|x|^2 sc + 1/2) for 0 <= |x|^2 sc < 2^63: the power in the transform
// precision, scaled in FP64, converted as two exact 32-bit halves
__device__ __forceinline__ double power_of(float2 x) { return (double)fmaf(x.x, x.x, x.y * x.y); }
__device__ __forceinline__ double power_of(double2 x) { return fma(x.x, x.x, x.y * x.y); }
template <typename C>
__device__ __forceinline__ unsigned long long fixed_power(C x, double sc)
{
    const double q = fma(power_of(x), sc, 0.5);
    const uint32_t hi = (uint32_t)(q * 0x1p-32);
    const uint32_t lo = (uint32_t)fma((double)hi, -0x1p32, q);
    return ((unsigned long long)hi << 32) | lo;
}

// ---------------------------------------------------------------------------
// z pass and shell sums: tiles of columns of half spectrum `fld`, transformed
// along z into LDS; then each column's wave vectors in runs of |fz| (fz and
// -fz together): the power of each in FP64 times its weight (1/N, twice for a
// wave vector that stands also for its mirror -k), rounded to the spectrum's
// fixed point and summed while the shell stays the same (it grows with |fz|,
// by at most one per step), each run's sum added to the workgroup's shell
// bins in LDS by one integer atomic (exact, so the order does not matter);
// after the workgroup's tiles the bins go to copy `copy` of the replica's bins.
// ---------------------------------------------------------------------------
template <typename Rt, int PL>
__device__ __forceinline__ void fft_zbin_body(const RepDev& R, uint32_t wg, uint32_t fld,
                                              const double2* __restrict__ tw,
                                              const typename CxOf<Rt>::type* __restrict__ spec,
                                              const double* __restrict__ ssq, unsigned long long* bins,
                                              uint32_t copy, uint32_t bin_stride, unsigned char* lds_raw)
{
    using C = typename CxOf<Rt>::type;
    const uint32_t nx = R.nx, ny = R.ny, nz = R.nz, L = nz;
    const FftCols cols = fft_cols(2, nx, ny, nz);
    const uint32_t W = cols.W, ld = fft_ld(2, nx, ny, nz, sizeof(C)), Hp = half_stride(nx);
    C* buf = reinterpret_cast<C*>(lds_raw);
    C* twl = buf + W * ld;
    const uint32_t bin_off = ((uint32_t)sizeof(C) * (W * ld + L) + 7u) / 8u * 8u;
    unsigned long long* lbin = reinterpret_cast<unsigned long long*>(lds_raw + bin_off);
    const uint32_t ns = R.nshell;
    for (uint32_t i = threadIdx.x; i < ns; i += kBlock) lbin[i] = 0ull;
    load_twiddles<Rt>(twl, tw + R.tw_offset + nx + ny, L);
    C* Sf = const_cast<C*>(spec) + R.spec_offset + (uint64_t)fld * Hp * ny * nz;
    auto make = [&](uint32_t tile) {
        const ColTile t = col_tile(cols, tile);
        return ColLines<C>{Sf, t, SmallDiv(t.cw), Hp, ny * Hp};
    };
    const LdsRows<C> out{buf, ld};

    double scale[kSpec];
    spectrum_scales(ssq, scale);
    const int m = spectrum_of_field(fld);
    const double sc1 = scale[m] * (fld >= 1 && fld <= 3 ? 1.0 / 3.0 : 1.0) / (double)R.n, sc2 = 2.0 * sc1;
    // items: (column w, run c of CH values a = |fz|, a = 0 .. L/2)
    const uint32_t na = L / 2 + 1;
    const uint32_t CH = (na * W + kBlock - 1) / kBlock, nch = (na + CH - 1) / CH;
    const SmallDiv dW(W);
    auto bin = [&](uint32_t tile) {
        const ColTile t = col_tile(cols, tile);
        const SmallDiv dcw(t.cw);
        for (uint32_t i = threadIdx.x; i < nch * W; i += kBlock) {
            const uint32_t c = dW.div(i), w = i - c * W;
            uint32_t off, plane, kx;
            if (!col_offset(t, dcw, Hp, w, off, plane, kx)) continue;
            const C* line = buf + w * ld;
            const int32_t fy = signed_freq(plane, ny);
            const uint32_t c0 = kx * kx + (uint32_t)(fy * fy);
            const double sc = (kx == 0u || 2u * kx == nx) ? sc1 : sc2;
            const uint32_t a0 = c * CH, a1 = a0 + CH < na ? a0 + CH : na;
            const uint32_t n20 = c0 + a0 * a0;
            uint32_t s = shell_from_root(n20, __builtin_amdgcn_sqrtf((float)n20));
            unsigned long long acc = 0ull;
            for (uint32_t a = a0; a < a1; ++a) {
                const uint32_t n2 = c0 + a * a;
                if (n2 == 0u) continue;   // k = 0
                if ((2u * s + 1u) * (2u * s + 1u) <= 4u * n2) {
                    if (acc) atomicAdd(&lbin[s], acc);
                    acc = 0ull;
                    ++s;
                }
                acc += fixed_power(line[fft_phys(a)], sc);
                const uint32_t zm = L - a;   // fz = -a
                if (a != 0u && zm != a) acc += fixed_power(line[fft_phys(zm)], sc);
            }
            if (acc) atomicAdd(&lbin[s], acc);
        }
    };
    if constexpr (PL > 0) {
        auto run = [&](uint32_t tile, C (&v)[16]) {
            p2_run<true, true, PL, Rt>(v, buf, twl, W, ld, dW, out);
            lds_barrier();
            bin(tile);
        };
        pipelined_tiles<kFftTilesPerWG[2], true, PL, Rt>(wg, cols.tiles(), W, dW, make, run);
    } else {
        fft_tile<true, true, 0, Rt>(buf, twl, L, W, ld, make(wg), out);
        lds_barrier();
        bin(wg);
    }
    lds_barrier();
    unsigned long long* gb = bins + (size_t)copy * bin_stride + (size_t)R.shell_offset * kSpec;
    for (uint32_t i = threadIdx.x; i < ns; i += kBlock)
        if (lbin[i]) atomicAdd(&gb[(size_t)i * kSpec + m], lbin[i]);
}

template <typename Rt, int PL>
__global__ __launch_bounds__(kBlock) void fft_zbin_kernel(const RepDev* reps, const uint32_t* first, int32_t nrep,
                                                          uint32_t flist, const double2* __restrict__ tw,
                                                          const typename CxOf<Rt>::type* __restrict__ spec,
                                                          const double* __restrict__ sample_sq,
                                                          unsigned long long* bins, uint32_t bin_stride)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int r = replica_of_block(first, nrep, blockIdx.x);
    if (fft_class(reps[r].nz) != PL) return;
    fft_zbin_body<Rt, PL>(reps[r], blockIdx.x - first[r], (flist >> (4u * blockIdx.y)) & 15u, tw, spec,
                          sample_sq + (size_t)r * kObs, bins, (blockIdx.x + blockIdx.y) % kBinCopies, bin_stride,
                          lds_raw);
}

// Shell averages of the sample into the FP64 accumulators: each bin is the
// sum of its kBinCopies copies (bin_stride values apart), one thread per bin
// (grid.y: replica); the copies are cleared for the next sample.
__global__ __launch_bounds__(kBlock) void spectrum_finalize_kernel(const RepDev* reps, const double* sample_sq,
                                                                   const int64_t* counts,
                                                                   unsigned long long* bins, uint32_t bin_stride,
                                                                   double* sacc)
{
    const RepDev& R = reps[blockIdx.y];
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= R.nshell * kSpec) return;
    double scale[kSpec];
    spectrum_scales(sample_sq + (size_t)blockIdx.y * kObs, scale);
    const uint32_t s = i / kSpec, m = i - s * kSpec;
    unsigned long long* b = bins + (size_t)R.shell_offset * kSpec + i;
    unsigned long long v[kBinCopies];
#pragma unroll
    for (uint32_t k = 0; k < kBinCopies; ++k) v[k] = b[(size_t)k * bin_stride];
    unsigned long long q = 0;
#pragma unroll
    for (uint32_t k = 0; k < kBinCopies; ++k) {
        q += v[k];
        b[(size_t)k * bin_stride] = 0ull;
    }
    const int64_t c = counts[R.shell_offset + s];
    if (c > 0 && scale[m] > 0.0) sacc[(size_t)R.shell_offset * kSpec + i] += ((double)q / scale[m]) / (double)c;
}

// y- and z-pass field groups of order 1 (four bits per field)
constexpr int kFieldGroups = 4;
constexpr uint32_t kGroupFields[kFieldGroups] = {0x40u, 0x15u, 0x32u, 0x6u};
constexpr uint32_t kGroupFieldCount[kFieldGroups] = {2u, 2u, 2u, 1u};

// One pass's kernel for the plan PL of its lines (see fft_tile).
template <typename T, typename Rt, int PL>
static void launch_pass(int axis, dim3 grid, size_t lds, hipStream_t s, const RepDev* reps, const uint32_t* first,
                        int32_t nrep, uint32_t list, const T* fields, const double2* tw,
                        typename CxOf<Rt>::type* sp, const double* sample_sq, unsigned long long* bins,
                        uint32_t bin_stride)
{
    if (axis == 0)
        fft_x_kernel<T, Rt, PL><<<grid, kBlock, lds, s>>>(reps, first, nrep, fields, tw, sp);
    else if (axis == 1)
        fft_y_kernel<Rt, PL><<<grid, kBlock, lds, s>>>(reps, first, nrep, list, tw, sp);
    else
        fft_zbin_kernel<Rt, PL><<<grid, kBlock, lds, s>>>(reps, first, nrep, list, tw, sp, sample_sq, bins, bin_stride);
}

template <typename T, typename Rt>
static hipError_t launch_spectrum_t(const RepDev* reps, int32_t nrep, const uint32_t* first, const uint32_t* nblk,
                                    const T* fields, const double2* tw, void* spec, const double* sample_sq,
                                    const int64_t* counts, unsigned long long* bins, uint32_t bin_stride, double* sacc,
                                    uint32_t max_nshell, const size_t* lds, const uint32_t* classes, int order,
                                    hipStream_t s)
{
    using C = typename CxOf<Rt>::type;
    C* sp = static_cast<C*>(spec);
    const size_t stride = (size_t)nrep + 1;
    // one launch per kernel class present along the axis (bit c of classes[axis])
    auto pass = [&](int axis, uint32_t list, uint32_t ny) -> hipError_t {
        const dim3 grid(nblk[axis], ny);
        const uint32_t* f = first + (size_t)axis * stride;
        for (int c = 0; c <= 10; ++c) {
            if (!((classes[axis] >> c) & 1u)) continue;
            switch (c) {
            case 6: launch_pass<T, Rt, 6>(axis, grid, lds[axis], s, reps, f, nrep, list, fields, tw, sp, sample_sq, bins, bin_stride); break;
            case 7: launch_pass<T, Rt, 7>(axis, grid, lds[axis], s, reps, f, nrep, list, fields, tw, sp, sample_sq, bins, bin_stride); break;
            case 8: launch_pass<T, Rt, 8>(axis, grid, lds[axis], s, reps, f, nrep, list, fields, tw, sp, sample_sq, bins, bin_stride); break;
            case 9: launch_pass<T, Rt, 9>(axis, grid, lds[axis], s, reps, f, nrep, list, fields, tw, sp, sample_sq, bins, bin_stride); break;
            case 10: launch_pass<T, Rt, 10>(axis, grid, lds[axis], s, reps, f, nrep, list, fields, tw, sp, sample_sq, bins, bin_stride); break;
            default: launch_pass<T, Rt, 0>(axis, grid, lds[axis], s, reps, f, nrep, list, fields, tw, sp, sample_sq, bins, bin_stride); break;
            }
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    hipError_t e = pass(0, 0u, 1u);
    if (order == 0) {
        if (e == hipSuccess) e = pass(1, 0x6543210u, kFftFields);
        if (e == hipSuccess) e = pass(2, 0x6543210u, kFftFields);
    } else {
        for (int g = 0; g < kFieldGroups && e == hipSuccess; ++g) {
            e = pass(1, kGroupFields[g], kGroupFieldCount[g]);
            if (e == hipSuccess) e = pass(2, kGroupFields[g], kGroupFieldCount[g]);
        }
    }
    if (e != hipSuccess) return e;
    spectrum_finalize_kernel<<<dim3((max_nshell * kSpec + kBlock - 1) / kBlock, nrep), kBlock, 0, s>>>(
        reps, sample_sq, counts, bins, bin_stride, sacc);
    return hipGetLastError();
}

hipError_t launch_spectrum(int precision, const RepDev* reps, int32_t nrep, const uint32_t* first, const uint32_t* nblk,
                           const void* fields, const double2* tw, void* spec, const double* sample_sq,
                           const int64_t* counts, unsigned long long* bins, uint32_t bin_stride, double* sacc,
                           uint32_t max_nshell, const size_t* lds, const uint32_t* classes, int order,
                           hipStream_t s)
{
    // first: 3 prefix arrays of nrep + 1 workgroup counts (passes x, y, z); nblk: their totals
    if (precision == kFP64)
        return launch_spectrum_t<double, double>(reps, nrep, first, nblk, (const double*)fields, tw, spec, sample_sq,
                                                 counts, bins, bin_stride, sacc, max_nshell, lds, classes, order, s);
    return launch_spectrum_t<float, float>(reps, nrep, first, nblk, (const float*)fields, tw, spec, sample_sq, counts,
                                           bins, bin_stride, sacc, max_nshell, lds, classes, order, s);
}


// ---------------------------------------------------------------------------
// Read-bandwidth reference of the spectrum passes, each of which reads what
// the kernel before it has just written: one 16-byte load per thread
// (grid-stride beyond 2^28 threads), summed per thread; a thread whose sum is
// not finite sets *flag, so the loads are not dead.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void read_probe_kernel(const float4* __restrict__ src, uint64_t n4,
                                                            uint32_t* flag)
{
    float acc = 0.0f;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += stride) {
        const float4 v = src[i];
        acc += (v.x + v.y) + (v.z + v.w);
    }
    if (!(fabsf(acc) <= 3.4e38f)) *flag = 1u;
}

hipError_t launch_read_probe(const void* src, uint64_t bytes, uint32_t* flag, hipStream_t s)
{
    const uint64_t n4 = bytes / 16;
    const uint64_t want = (n4 + kBlock - 1) / kBlock;
    const uint32_t g = (uint32_t)(want < (1u << 20) ? want : (1u << 20));
    read_probe_kernel<<<g, kBlock, 0, s>>>(reinterpret_cast<const float4*>(src), n4, flag);
    return hipGetLastError();
}

}  // namespace gmf
