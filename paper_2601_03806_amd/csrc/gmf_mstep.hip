// gmf_mstep.hip -- the moment-storage step on gfx950 (GMF collision only).
//
// The thread-safe reading of Sec. II: the GMF collision (Eq. (10)) uses only
// the ten hydrodynamic moments of f at a node (Eqs. (3), (4), (13)) and keeps
// no deterministic ghost content, so the lattice state can be those moments.
// A step rebuilds, at every node, the post-collision populations that stream
// into it from its neighbours' moments (with the neighbours' noise drawn
// again from their Philox counters) and writes the node's new moments: ten
// values read and ten written per node, against 27 and 27 for populations.
//
// Stored state (kMom fields of N values per replica, gmf_internal.hpp): the
// raw moments of g = f - w rho0 of the pre-collision state f(x, t), i.e.
// rho - rho0, j, Pi_aa - rho0 cs2 and the off-diagonal Pi.  The shift keeps
// the small thermal fluctuations at full relative precision in FP32.
//
// Kernel: a workgroup owns a TX x TY x TZ tile and marches through it in z.
// For each source plane s it runs the collision of every column of the tile
// plus a one-node halo in x and y ((TX+2)(TY+2) columns, one per thread, or
// two rounds of columns per thread for the largest tile) and keeps the 27
// post-collision populations in LDS; then each tile column adds the 27
// populations that stream into it to the moment accumulators of the planes
// s-1, s, s+1 (by c_z), and writes plane s-1, now complete.  The planes z0-1
// and z0+TZ are computed as halo.  The next plane's moments are loaded while
// the current one is processed, and where two LDS buffers fit, consecutive
// planes alternate between them so that one barrier per plane suffices.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gmf_collide.hpp"
#include "gmf_device.hpp"
#include "gmf_internal.hpp"

namespace gmf {

// Post-collision shifted populations g*(p) (tensor order) of a node with
// stored moments h, node index n, step t: Eq. (10) with the noise of
// Eqs. (2) and (9).
template <typename T>
__device__ __forceinline__ void post_collision(const Hydro<T>& h, const RepDev& R, uint32_t n, uint64_t t, T F[Q])
{
    const T rho0 = rep_param<T>(R.rho0, R.rho0f);
    const T rho = rho0 + h.s0;
    const T om = rep_param<T>(R.omega, R.omegaf), omm = rep_param<T>(R.one_m_omega, R.one_m_omegaf);
    T M[Q];
    relaxed_coefficients<T, kGMF>(h, recip(rho), om, omm, M);
    if (R.noise_on) {
        T r[23];
        node_normals<T>(n, t, R.key0, R.key1, r);
        add_noise<T>(R, sqroot(R.noise_rho0 ? rho0 : rho), r, M);
    }
    back_project(M, F);
}

// Adds to A the raw moments of the nine populations with z velocity CZ that
// streamed into a node, g[3 (cx+1) + (cy+1)]: separable sums over cx, then cy.
// FIRST (CZ = +1 only, the first contribution a destination receives): A is
// assigned instead.
template <typename T, int CZ, bool FIRST = false>
__device__ __forceinline__ void add_slice(Hydro<T>& A, const T g[9])
{
    static_assert(!FIRST || CZ == 1, "only the c_z = +1 slice comes first");
    T X0[3], X1[3], X2[3];
#pragma unroll
    for (int cy = 0; cy < 3; ++cy) {
        const T m = g[cy], z = g[3 + cy], p = g[6 + cy];   // cx = -1, 0, +1
        X2[cy] = m + p;
        X0[cy] = X2[cy] + z;
        X1[cy] = p - m;
    }
    const T syy = X0[0] + X0[2];
    const T s = syy + X0[1];
    const T sy = X0[2] - X0[0];
    const T sx = X1[0] + X1[1] + X1[2];
    const T sxy = X1[2] - X1[0];
    const T sxx = X2[0] + X2[1] + X2[2];
    if (FIRST) {
        A = Hydro<T>{s, sx, sy, s, sxx, syy, s, sxy, sx, sy};
        return;
    }
    A.s0 += s;
    A.jx += sx;
    A.jy += sy;
    A.pxx += sxx;
    A.pyy += syy;
    A.pxy += sxy;
    if (CZ != 0) {
        A.pzz += s;
        if (CZ > 0) {
            A.jz += s;
            A.pxz += sx;
            A.pyz += sy;
        } else {
            A.jz -= s;
            A.pxz -= sx;
            A.pyz -= sy;
        }
    }
}

template <typename T>
__device__ __forceinline__ Hydro<T> zero_hydro()
{
    return Hydro<T>{T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
}

template <typename T, bool SAMPLE, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void mstep_kernel(const StepArgs a)
{
    constexpr int EX = TX + 2, EY = TY + 2, NE = EX * EY;
    constexpr int NR = (NE + NT - 1) / NT;   // haloed columns per thread
    static_assert(TX * TY <= NT, "one tile column per thread in the gather");
    // two LDS buffers when they fit: consecutive planes alternate between them,
    // so one barrier per plane suffices (a wave rewrites a buffer only after
    // the next plane's barrier, which every wave reaches after its reads)
    constexpr int NB = 2 * Q * NE * sizeof(T) <= 160 * 1024 ? 2 : 1;
    __shared__ T lds[NB * Q * NE];

    // workgroup -> tile, with the same XCD mappings as the population step
    uint32_t blk = blockIdx.x;
    if (a.xcd) {
        const uint32_t x = blockIdx.x % a.xcd, j = blockIdx.x / a.xcd;
        blk = (x + a.xcd * (j / a.chunk)) * a.chunk + j % a.chunk;
        if (blk >= a.nblocks) return;
    }
    const int r = a.blk2rep ? (int)sgpr(a.blk2rep[blk]) : 0;
    const RepDev R = uniform_rep(a.reps[r]);
    const uint64_t t = sgpr64((uint64_t)(a.step_base + (a.d_step ? *a.d_step : 0)));
    const uint32_t nx = R.nx, ny = R.ny, nz = R.nz;
    const uint32_t plane = nx * ny;
    const uint64_t N = R.n;
    // tiles of a replica: x fastest, then y, then z
    const uint32_t b = blk - R.block_begin;
    const uint32_t ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY;
    const uint32_t x0 = (b % ntx) * TX, y0 = ((b / ntx) % nty) * TY, z0 = (b / ntx / nty) * a.tz;
    const uint32_t z1 = min(z0 + a.tz, nz);
    const int nplanes = (int)(z1 - z0) + 2;

    // the columns this thread collides: e = threadIdx.x + q NT = ey EX + ex of
    // the haloed tile, at (x0 + ex - 1, y0 + ey - 1) mod the box; moments move
    // through buffer resources (per field and plane a uniform base, per column
    // a fixed 32-bit offset; loads cached, so that the halo columns that
    // neighbouring tiles read again come from the L2)
    uint32_t col[NR], vcol[NR];
    bool inner[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const uint32_t e = threadIdx.x + (uint32_t)(q * NT);
        const uint32_t ex = e % EX, ey = e / EX;
        col[q] = ((y0 + ey + ny - 1) % ny) * nx + (x0 + ex + nx - 1) % nx;   // in the box for any e
        vcol[q] = col[q] * (uint32_t)sizeof(T);
        inner[q] = SAMPLE && e < (uint32_t)NE && ex >= 1 && ex <= (uint32_t)TX && ey >= 1 && ey <= (uint32_t)TY &&
                   x0 + ex - 1 < nx && y0 + ey - 1 < ny;
    }
    // the tile column this thread gathers into (threads 0 .. TX TY - 1)
    const uint32_t ix = threadIdx.x % TX, iy = threadIdx.x / TX;
    const bool gatherer = threadIdx.x < (uint32_t)(TX * TY);
    const bool owner = gatherer && x0 + ix < nx && y0 + iy < ny;
    const uint32_t vown = ((y0 + iy) * nx + (x0 + ix)) * (uint32_t)sizeof(T);
    const uint32_t e0 = (iy + 1) * EX + ix + 1;

    const T* src = reinterpret_cast<const T*>(a.src) + R.pop_offset;
    T* dst = reinterpret_cast<T*>(a.dst) + R.pop_offset;
    // source plane k of the march is z0 - 1 + k (periodic)
    auto src_plane = [&](int k) { return (z0 + (uint32_t)k + nz - 1) % nz; };
    auto load = [&](int k, T (&m)[NR][kMom]) {
        const T* base = src + (uint64_t)src_plane(k) * plane;
#pragma unroll
        for (int f = 0; f < kMom; ++f) {
            const __amdgpu_buffer_rsrc_t rs = make_rsrc(base + (uint64_t)f * N);
#pragma unroll
            for (int q = 0; q < NR; ++q)
                if (q == 0 || threadIdx.x + (uint32_t)(q * NT) < (uint32_t)NE) m[q][f] = bload<T, 0>(rs, vcol[q], 0);
        }
    };

    // accumulators of the destination planes s-1 (am), s (a0), s+1 (ap)
    Hydro<T> am = zero_hydro<T>(), a0 = zero_hydro<T>(), ap = zero_hydro<T>();
    T mn[NR][kMom];
    load(0, mn);
    for (int k = 0; k < nplanes; ++k) {
        T* buf = lds + (NB == 2 ? (k & 1) * Q * NE : 0);
        T mc[NR][kMom];
#pragma unroll
        for (int q = 0; q < NR; ++q)
#pragma unroll
            for (int f = 0; f < kMom; ++f) mc[q][f] = mn[q][f];
        if (k + 1 < nplanes) load(k + 1, mn);
        const uint32_t sz = src_plane(k);
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const uint32_t e = threadIdx.x + (uint32_t)(q * NT);
            if (e >= (uint32_t)NE) continue;
            const Hydro<T> h{mc[q][0], mc[q][1], mc[q][2], mc[q][3], mc[q][4],
                             mc[q][5], mc[q][6], mc[q][7], mc[q][8], mc[q][9]};
            const uint32_t n = sz * plane + col[q];
            T F[Q];
            post_collision<T>(h, R, n, t, F);
#pragma unroll
            for (int p = 0; p < Q; ++p) buf[p * NE + e] = F[p];
            if (SAMPLE && inner[q] && k >= 1 && k <= nplanes - 2) {
                // fields of the sampled state f(., t) at a node of the tile
                T* fl = reinterpret_cast<T*>(a.fields) + R.field_offset + n;
                fl[0] = h.s0;
                fl[N] = h.jx;
                fl[2 * N] = h.jy;
                fl[3 * N] = h.jz;
                fl[4 * N] = h.pxx + h.pyy + h.pzz;
                fl[5 * N] = h.pxy + h.pxz + h.pyz;
            }
        }
        __syncthreads();
        if (gatherer) {
            // population p = (cx, cy, cz) reaching this column left column (ix - cx, iy - cy);
            // the c_z = +1 slice is the first that plane s+1 receives
            T g[9];
#pragma unroll
            for (int cz = 0; cz < 3; ++cz) {
#pragma unroll
                for (int cx = 0; cx < 3; ++cx)
#pragma unroll
                    for (int cy = 0; cy < 3; ++cy)
                        g[3 * cx + cy] = buf[(9 * cx + 3 * cy + cz) * NE + e0 - (cy - 1) * EX - (cx - 1)];
                if (cz == 0) add_slice<T, -1>(am, g);
                if (cz == 1) add_slice<T, 0>(a0, g);
                if (cz == 2) add_slice<T, 1, true>(ap, g);
            }
            if (k >= 2 && owner) {
                T* base = dst + (uint64_t)(z0 + (uint32_t)k - 2) * plane;
                const T v[kMom] = {am.s0, am.jx, am.jy, am.jz, am.pxx, am.pyy, am.pzz, am.pxy, am.pxz, am.pyz};
#pragma unroll
                for (int f = 0; f < kMom; ++f) bstore(make_rsrc(base + (uint64_t)f * N), vown, 0, v[f]);
            }
            am = a0;
            a0 = ap;
        }
        if (NB == 1) __syncthreads();
    }
}

template <typename T, bool SAMPLE, int TILE>
static hipError_t launch_mstep_tile(const StepArgs& a, uint32_t nblocks, hipStream_t s)
{
    if constexpr (!mtile_fits(TILE, sizeof(T))) {
        return hipErrorInvalidValue;
    } else {
    StepArgs b = a;
    b.nblocks = nblocks;
    uint32_t g = nblocks;
    if (a.xcd) {
        b.chunk = a.chunk ? a.chunk : (nblocks + a.xcd - 1u) / a.xcd;
        g = (nblocks + a.xcd * b.chunk - 1u) / (a.xcd * b.chunk) * b.chunk * a.xcd;
    }
    mstep_kernel<T, SAMPLE, kMTileX[TILE], kMTileY[TILE], mtile_threads(TILE)><<<g, mtile_threads(TILE), 0, s>>>(b);
    return hipGetLastError();
    }
}

template <typename T, bool SAMPLE>
static hipError_t launch_mstep_t(int tile, const StepArgs& a, uint32_t nblocks, hipStream_t s)
{
    switch (tile) {
    case 0: return launch_mstep_tile<T, SAMPLE, 0>(a, nblocks, s);
    case 1: return launch_mstep_tile<T, SAMPLE, 1>(a, nblocks, s);
    case 2: return launch_mstep_tile<T, SAMPLE, 2>(a, nblocks, s);
    case 3: return launch_mstep_tile<T, SAMPLE, 3>(a, nblocks, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_mstep(int precision, bool sample, int tile, const StepArgs& a, uint32_t nblocks, hipStream_t s)
{
    if (a.tz < 1) return hipErrorInvalidValue;
    if (precision == kFP64)
        return sample ? launch_mstep_t<double, true>(tile, a, nblocks, s) : launch_mstep_t<double, false>(tile, a, nblocks, s);
    return sample ? launch_mstep_t<float, true>(tile, a, nblocks, s) : launch_mstep_t<float, false>(tile, a, nblocks, s);
}

// ---------------------------------------------------------------------------
// Host-interface helpers.  Populations handed out are the second-order
// Hermite populations of the stored moments,
//   f_i = w_i (rho + c_i . j / cs2 + (c_i c_i - cs2 I) : a2 / (2 cs2^2)),
//   a2 = Pi - rho cs2 I,
// which carry exactly the moments the GMF dynamics depends on; populations
// handed in are reduced to their moments.
// ---------------------------------------------------------------------------
struct MCanon {
    int8_t cx[Q], cy[Q], cz[Q];   // velocity of canonical population i
};

static MCanon make_mcanon()
{
    int t[Q];
    canonical_to_tensor(t);
    MCanon m;
    for (int i = 0; i < Q; ++i) {
        m.cx[i] = (int8_t)tcx(t[i]);
        m.cy[i] = (int8_t)tcy(t[i]);
        m.cz[i] = (int8_t)tcz(t[i]);
    }
    return m;
}

template <typename T>
__device__ __forceinline__ void load_moments(const T* s, uint64_t N, uint64_t n, double m[kMom])
{
#pragma unroll
    for (int f = 0; f < kMom; ++f) m[f] = (double)s[(uint64_t)f * N + n];
}

// canonical populations of node n from its moments (FP64)
__device__ __forceinline__ void hermite_populations(const double m[kMom], double rho0, const MCanon& cm,
                                                    double* out, uint64_t stride)
{
    const double cs2 = 1.0 / 3.0;
    const double rho = rho0 + m[0];
    // a2 = Pi - rho cs2 I from the shifted moments: Pi_aa - rho0 cs2 - (rho - rho0) cs2
    const double axx = m[4] - cs2 * m[0], ayy = m[5] - cs2 * m[0], azz = m[6] - cs2 * m[0];
    for (int i = 0; i < Q; ++i) {
        const int cx = cm.cx[i], cy = cm.cy[i], cz = cm.cz[i];
        const double w = w1(cx) * w1(cy) * w1(cz);
        const double cj = cx * m[1] + cy * m[2] + cz * m[3];
        const double ha = (cx * cx - cs2) * axx + (cy * cy - cs2) * ayy + (cz * cz - cs2) * azz +
                          2.0 * (cx * cy * m[7] + cx * cz * m[8] + cy * cz * m[9]);
        out[(uint64_t)i * stride] = w * (rho + cj / cs2 + ha / (2.0 * cs2 * cs2));
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void mgather_kernel(const T* src, const RepDev* rep, uint32_t z0, uint32_t z1,
                                                         double* out, MCanon cm)
{
    const RepDev& R = *rep;
    const uint64_t plane = (uint64_t)R.nx * R.ny;
    const uint64_t cnt = plane * (z1 - z0);
    const uint64_t idx = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= cnt) return;
    double m[kMom];
    load_moments(src + R.pop_offset, R.n, z0 * plane + idx, m);
    hermite_populations(m, R.rho0, cm, out + idx, cnt);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void mscatter_kernel(T* dst, const RepDev* rep, uint32_t z0, uint32_t z1,
                                                          const double* in, MCanon cm)
{
    const RepDev& R = *rep;
    const uint64_t plane = (uint64_t)R.nx * R.ny;
    const uint64_t cnt = plane * (z1 - z0);
    const uint64_t idx = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= cnt) return;
    double m[kMom] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = 0; i < Q; ++i) {
        const int cx = cm.cx[i], cy = cm.cy[i], cz = cm.cz[i];
        const double g = in[(uint64_t)i * cnt + idx] - w1(cx) * w1(cy) * w1(cz) * R.rho0;
        m[0] += g;
        m[1] += cx * g;
        m[2] += cy * g;
        m[3] += cz * g;
        m[4] += cx * cx * g;
        m[5] += cy * cy * g;
        m[6] += cz * cz * g;
        m[7] += cx * cy * g;
        m[8] += cx * cz * g;
        m[9] += cy * cz * g;
    }
    T* d = dst + R.pop_offset + z0 * plane + idx;
    for (int f = 0; f < kMom; ++f) d[(uint64_t)f * R.n] = (T)m[f];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void mmoments_kernel(const T* src, const RepDev* rep, uint32_t z0, uint32_t z1,
                                                          double* rho_out, double* u_out, double* partials)
{
    const RepDev& R = *rep;
    const uint64_t plane = (uint64_t)R.nx * R.ny;
    const uint64_t cnt = plane * (z1 - z0);
    const uint64_t idx = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (idx < cnt) {
        double m[kMom];
        load_moments(src + R.pop_offset, R.n, z0 * plane + idx, m);
        const double rho = R.rho0 + m[0];
        if (rho_out) rho_out[idx] = rho;
        if (u_out) {
            u_out[idx] = m[1] / rho;
            u_out[cnt + idx] = m[2] / rho;
            u_out[2 * cnt + idx] = m[3] / rho;
        }
        v[0] = rho; v[1] = m[1]; v[2] = m[2]; v[3] = m[3];
    }
    block_sum_store<4>(v, partials + (size_t)blockIdx.x * 4);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void mnodes_kernel(const T* src, const RepDev* rep, const int64_t* nodes,
                                                        int32_t count, double* out, MCanon cm)
{
    const RepDev& R = *rep;
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= count) return;
    double m[kMom];
    load_moments(src + R.pop_offset, R.n, (uint64_t)nodes[j], m);
    hermite_populations(m, R.rho0, cm, out + (size_t)j * Q, 1);
}

static inline uint32_t mgrid(uint64_t cnt) { return (uint32_t)((cnt + kBlock - 1) / kBlock); }

hipError_t launch_mgather(int precision, const void* src, const RepDev* rep_dev, const RepDev& rep, uint32_t z0,
                          uint32_t z1, double* out, hipStream_t s)
{
    static const MCanon cm = make_mcanon();
    const uint32_t g = mgrid((uint64_t)rep.nx * rep.ny * (z1 - z0));
    if (precision == kFP64)
        mgather_kernel<double><<<g, kBlock, 0, s>>>((const double*)src, rep_dev, z0, z1, out, cm);
    else
        mgather_kernel<float><<<g, kBlock, 0, s>>>((const float*)src, rep_dev, z0, z1, out, cm);
    return hipGetLastError();
}

hipError_t launch_mscatter(int precision, void* dst, const RepDev* rep_dev, const RepDev& rep, uint32_t z0,
                           uint32_t z1, const double* in, hipStream_t s)
{
    static const MCanon cm = make_mcanon();
    const uint32_t g = mgrid((uint64_t)rep.nx * rep.ny * (z1 - z0));
    if (precision == kFP64)
        mscatter_kernel<double><<<g, kBlock, 0, s>>>((double*)dst, rep_dev, z0, z1, in, cm);
    else
        mscatter_kernel<float><<<g, kBlock, 0, s>>>((float*)dst, rep_dev, z0, z1, in, cm);
    return hipGetLastError();
}

hipError_t launch_mmoments(int precision, const void* src, const RepDev* rep_dev, const RepDev& rep, uint32_t z0,
                           uint32_t z1, double* rho, double* u, double* partials, hipStream_t s)
{
    const uint32_t g = mgrid((uint64_t)rep.nx * rep.ny * (z1 - z0));
    if (precision == kFP64)
        mmoments_kernel<double><<<g, kBlock, 0, s>>>((const double*)src, rep_dev, z0, z1, rho, u, partials);
    else
        mmoments_kernel<float><<<g, kBlock, 0, s>>>((const float*)src, rep_dev, z0, z1, rho, u, partials);
    return hipGetLastError();
}

hipError_t launch_mnodes(int precision, const void* src, const RepDev* rep_dev, const int64_t* nodes, int32_t count,
                         double* out, hipStream_t s)
{
    static const MCanon cm = make_mcanon();
    const uint32_t g = mgrid((uint64_t)count);
    if (precision == kFP64)
        mnodes_kernel<double><<<g, kBlock, 0, s>>>((const double*)src, rep_dev, nodes, count, out, cm);
    else
        mnodes_kernel<float><<<g, kBlock, 0, s>>>((const float*)src, rep_dev, nodes, count, out, cm);
    return hipGetLastError();
}

}  // namespace gmf
