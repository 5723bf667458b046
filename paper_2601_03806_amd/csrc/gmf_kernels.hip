// gmf_kernels.hip -- gfx950 kernels of the GMF-FLBM library.
//
// The step kernel fuses, per lattice node (Sec. II):
//   pull of the 27 populations from the neighbours (periodic box),
//   the ten hydrodynamic moments rho, j, Pi (Eqs. (3), (4), (13)),
//   the second-order equilibrium and the relaxation of the stress by
//   (1 - omega) (Eqs. (10)-(12)),
//   the Philox4x32-10 normals and the noise amplitudes of Eqs. (2) and (9),
//   the projection back to populations (Eq. (10)), and the write.
// The ghost moments of f are never formed: Eq. (10) keeps none of their
// deterministic content.  Moments and the back-projection are separable
// 3-point transforms along x, y, z in the internal tensor order, because the
// D3Q27 weights and the Table II basis factorise over the axes
// (w_i = w1(cx) w1(cy) w1(cz), e_k = h_a(cx) h_b(cy) h_c(cz) with
// h0 = 1, h1 = c, h2 = c^2 - 1/3).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gmf_collide.hpp"
#include "gmf_device.hpp"
#include "gmf_internal.hpp"

namespace gmf {

// ---------------------------------------------------------------------------
// The fused stream + collide step
// ---------------------------------------------------------------------------
// Population traffic goes through raw buffer instructions (gmf_collide.hpp):
// one resource per storage group (uniform), the population's row start as
// scalar offset and the node's row/x offset as 32-bit vector offset, so no
// per-access 64-bit address arithmetic is spent on the vector ALUs.  Every
// population value is read and written exactly once per step: the accesses
// are marked nontemporal.

// resource of the storage group holding population p, and p's row-start offset in it (bytes)
template <typename T, int G>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t group_rsrc(const void* rep_base, const RepDev& R, int p)
{
    const int g = slot_of(p) / G;
    return make_rsrc(reinterpret_cast<const char*>(rep_base) + (uint64_t)g * R.grp_elems * sizeof(T));
}
template <typename T, int G>
__device__ __forceinline__ uint32_t slot_soff(const RepDev& R, int p)
{
    return (uint32_t)(slot_of(p) % G) * R.nx * (uint32_t)sizeof(T);
}

// Plain (cached) store of a sampled field value; 64-bit offsets, since a field
// of a large FP64 box exceeds 4 GiB.
template <typename T>
__device__ __forceinline__ void stg_cached(T* base, uint32_t idx, T v)
{
    base[(uint64_t)idx] = v;
}

// Addressing modes of the step kernel:
//   G = 27, 3, 1  per-node addressing; population groups of G (see gmf_device.hpp),
//                 byte offsets inside a group must fit 32 bits;
//   G = kPlane    every workgroup lies in one z plane (n_x n_y a multiple of the
//                 nodes per workgroup); storage groups of 27, the three source
//                 planes are uniform and get their own 64-bit scalar base, so only
//                 a plane (n_y 27 n_x values) must fit 32-bit offsets.
constexpr int kPlane = 0;

template <typename T, bool SHIFTED, int COLL, bool SAMPLE, int G, int SM>
__device__ __forceinline__ void node_update(const StepArgs& a, const RepDev& R, uint32_t n, uint32_t zplane,
                                            uint64_t t)
{
    const uint32_t nx = R.nx, ny = R.ny, nz = R.nz, N = R.n;
    uint32_t x, y, z;
    if constexpr (G == kPlane) {
        z = zplane;
        const uint32_t local = n - z * (nx * ny);
        y = fdiv(local, R.divx);
        x = local - y * nx;
    } else {
        const uint32_t yz = fdiv(n, R.divx);
        x = n - yz * nx;
        z = fdiv(yz, R.divy);
        y = yz - z * ny;
    }

    // pull: f_p(x) = f*_p(x - c_p); index 0/1/2 <-> c = -1/0/+1
    uint32_t xs[3], yv[3], zv[3];
    xs[0] = (x + 1 == nx) ? 0u : x + 1;
    xs[1] = x;
    xs[2] = (x == 0) ? nx - 1 : x - 1;
    yv[0] = (y + 1 == ny) ? 0u : y + 1;
    yv[1] = y;
    yv[2] = (y == 0) ? ny - 1 : y - 1;
    zv[0] = (z + 1 == nz) ? 0u : z + 1;
    zv[1] = z;
    zv[2] = (z == 0) ? nz - 1 : z - 1;
    uint32_t xb[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) xb[q] = xs[q] * (uint32_t)sizeof(T);

    const T* src = reinterpret_cast<const T*>(a.src) + R.pop_offset;
    T* dst = reinterpret_cast<T*>(a.dst) + R.pop_offset;
    T f[Q];
    // kAALocal reads population 26 - p at the node itself
    constexpr bool kLocal = SM == kAALocal;
    uint32_t self;
    __amdgpu_buffer_rsrc_t wr;   // plane mode: resource of the node's own plane
    __amdgpu_buffer_rsrc_t rp[3];
    uint32_t ry[3];
    uint32_t rows[9];
    if constexpr (G == kPlane) {
        // uniform source planes z - cz, per-node source rows y - cy (bytes inside a plane)
        const uint64_t plane_elems = (uint64_t)ny * R.row_stride;
#pragma unroll
        for (int q = 0; q < 3; ++q) rp[q] = make_rsrc(src + (uint64_t)zv[q] * plane_elems);
#pragma unroll
        for (int q = 0; q < 3; ++q) ry[q] = yv[q] * R.row_stride * (uint32_t)sizeof(T);
        self = ry[1] + xb[1];
#pragma unroll
        for (int p = 0; p < Q; ++p) {
            if (kLocal)
                f[p] = bload<T>(rp[1], self, slot_soff<T, 27>(R, opposite(p)));
            else
                f[p] = bload<T>(rp[p % 3], ry[(p / 3) % 3] + xb[p / 9], slot_soff<T, 27>(R, p));
        }
        wr = SM == kAB ? make_rsrc(dst + (uint64_t)z * plane_elems) : rp[1];
    } else {
        // byte offsets: source row (y - cy, z - cz) at index 3*cyi + czi
#pragma unroll
        for (int q = 0; q < 9; ++q) rows[q] = row_offset32(R, yv[q / 3], zv[q % 3]) * (uint32_t)sizeof(T);
        self = rows[4] + xb[1];
#pragma unroll
        for (int p = 0; p < Q; ++p) {
            if (kLocal)
                f[p] = bload<T>(group_rsrc<T, G>(src, R, opposite(p)), self, slot_soff<T, G>(R, opposite(p)));
            else
                f[p] = bload<T>(group_rsrc<T, G>(src, R, p), rows[p % 9] + xb[p / 9], slot_soff<T, G>(R, p));
        }
    }

    // noise words do not depend on the populations: issue them while the loads fly
    T r[23];
    // FP64 draws even without noise (the amplitudes are then 0): with the
    // draw in the same basic block as the loads, the compiler overlaps the
    // generator's arithmetic with them, which measured 3-4% faster.  FP32
    // measured faster with the branch (fewer live registers).
    if (sizeof(T) == 8 || R.noise_on) node_normals<T>(n, t, R.key0, R.key1, r);

    const Hydro<T> h = forward_moments(f);
    const T rho0 = rep_param<T>(R.rho0, R.rho0f);
    const T rho = SHIFTED ? rho0 + h.s0 : h.s0;
    const T irho = recip(rho);
    const T cs2 = T(1.0 / 3.0);
    const T om = rep_param<T>(R.omega, R.omegaf), omm = rep_param<T>(R.one_m_omega, R.one_m_omegaf);

    T M[Q];
    relaxed_coefficients<T, COLL>(h, irho, om, omm, M);
    if (sizeof(T) == 8 || R.noise_on) add_noise<T>(R, sqroot(R.noise_rho0 ? rho0 : rho), r, M);

    T F[Q];
    back_project(M, F);
    if (COLL == kBGK) {
#pragma unroll
        for (int p = 0; p < Q; ++p) F[p] += omm * f[p];
    }

    if constexpr (SM == kAAPull) {
        // f*_p goes where f_(26-p) came from: population 26 - p at x + c_p
        // (rows shifted by one node in x are written through the cache, policy 0:
        // the L2 completes their partly covered lines before writing them back)
        if constexpr (G == kPlane) {
#pragma unroll
            for (int p = 0; p < Q; ++p) {
                const int o = opposite(p);
                const uint32_t off = ry[(o / 3) % 3] + xb[o / 9], so = slot_soff<T, 27>(R, o);
                if (o / 9 == 1) bstore(rp[o % 3], off, so, F[p]);
                else bstore<0>(rp[o % 3], off, so, F[p]);
            }
        } else {
#pragma unroll
            for (int p = 0; p < Q; ++p) {
                const int o = opposite(p);
                const uint32_t off = rows[o % 9] + xb[o / 9], so = slot_soff<T, G>(R, o);
                if (o / 9 == 1) bstore(group_rsrc<T, G>(dst, R, o), off, so, F[p]);
                else bstore<0>(group_rsrc<T, G>(dst, R, o), off, so, F[p]);
            }
        }
    } else if constexpr (G == kPlane) {
#pragma unroll
        for (int p = 0; p < Q; ++p) bstore(wr, self, slot_soff<T, 27>(R, p), F[p]);
    } else {
#pragma unroll
        for (int p = 0; p < Q; ++p) bstore(group_rsrc<T, G>(dst, R, p), self, slot_soff<T, G>(R, p), F[p]);
    }

    if (SAMPLE) {
        const T drho = SHIFTED ? h.s0 : h.s0 - rho0;
        const T pdiag = SHIFTED ? (h.pxx + h.pyy + h.pzz) : (h.pxx + h.pyy + h.pzz - T(3) * cs2 * rho0);
        const T poff = h.pxy + h.pxz + h.pyz;
        T* fl = reinterpret_cast<T*>(a.fields) + R.field_offset;
        stg_cached(fl + 0ull * N, n, drho);
        stg_cached(fl + 1ull * N, n, h.jx);
        stg_cached(fl + 2ull * N, n, h.jy);
        stg_cached(fl + 3ull * N, n, h.jz);
        stg_cached(fl + 4ull * N, n, pdiag);
        stg_cached(fl + 5ull * N, n, poff);
    }
}

template <typename T, bool SHIFTED, int COLL, bool SAMPLE, int NPT, int G, int SM>
__global__ __launch_bounds__(kBlock) void step_kernel(const StepArgs a)
{
    // Workgroups are dealt to the XCDs in turn (workgroup i to XCD i mod X).
    // With a.xcd = X each XCD instead takes runs of a.chunk consecutive lattice
    // blocks (chunk k of the lattice to XCD k mod X), so the neighbouring rows
    // that a block pulls from are mostly read through the same L2; the
    // autotuner picks the mapping.  The grid covers whole chunks on every XCD;
    // the workgroups past the last block exit at once.
    uint32_t blk = blockIdx.x;
    if (a.xcd) {
        const uint32_t x = blockIdx.x % a.xcd, j = blockIdx.x / a.xcd;
        blk = (x + a.xcd * (j / a.chunk)) * a.chunk + j % a.chunk;
        if (blk >= a.nblocks) return;
    }
    const int r = a.blk2rep ? (int)sgpr(a.blk2rep[blk]) : 0;
    const RepDev R = uniform_rep(a.reps[r]);
    const uint64_t t = sgpr64((uint64_t)(a.step_base + (a.d_step ? *a.d_step : 0)));
    const uint32_t first = (blk - R.block_begin) * (uint32_t)(kBlock * NPT);
    const uint32_t base = first + threadIdx.x;
    // plane mode: the whole workgroup lies in z plane first / (nx ny)
    const uint32_t zplane = G == kPlane ? fdiv(fdiv(first, R.divx), R.divy) : 0u;
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const uint32_t n = base + (uint32_t)(k * kBlock);
        if (n < R.n) node_update<T, SHIFTED, COLL, SAMPLE, G, SM>(a, R, n, zplane, t);
    }
}

template <typename T, bool SHIFTED, int COLL, bool SAMPLE, int G, int SM>
static hipError_t launch_step_npt(int npt, const StepArgs& a, uint32_t nblocks, hipStream_t s)
{
    StepArgs b = a;
    b.nblocks = nblocks;
    uint32_t g = nblocks;
    if (a.xcd) {
        // chunk 0: one contiguous range per XCD
        b.chunk = a.chunk ? a.chunk : (nblocks + a.xcd - 1u) / a.xcd;
        g = (nblocks + a.xcd * b.chunk - 1u) / (a.xcd * b.chunk) * b.chunk * a.xcd;
    }
    // LDS the kernel does not touch, reserved only to cap the workgroups per CU
    const uint32_t lds = occ_lds_bytes(a.occ);
    switch (npt) {
    case 1: step_kernel<T, SHIFTED, COLL, SAMPLE, 1, G, SM><<<g, kBlock, lds, s>>>(b); break;
    case 2: step_kernel<T, SHIFTED, COLL, SAMPLE, 2, G, SM><<<g, kBlock, lds, s>>>(b); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, bool SHIFTED, int COLL, bool SAMPLE, int SM>
static hipError_t launch_step_grp(int grp, int npt, const StepArgs& a, uint32_t nb, hipStream_t s)
{
    switch (grp) {
    case kPlane: return launch_step_npt<T, SHIFTED, COLL, SAMPLE, kPlane, SM>(npt, a, nb, s);
    case 27: return launch_step_npt<T, SHIFTED, COLL, SAMPLE, 27, SM>(npt, a, nb, s);
    case 3: return launch_step_npt<T, SHIFTED, COLL, SAMPLE, 3, SM>(npt, a, nb, s);
    case 1: return launch_step_npt<T, SHIFTED, COLL, SAMPLE, 1, SM>(npt, a, nb, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, bool SHIFTED, int COLL, bool SAMPLE>
static hipError_t launch_step_sm(int sm, int grp, int npt, const StepArgs& a, uint32_t nb, hipStream_t s)
{
    switch (sm) {
    case kAB: return launch_step_grp<T, SHIFTED, COLL, SAMPLE, kAB>(grp, npt, a, nb, s);
    case kAAPull: return launch_step_grp<T, SHIFTED, COLL, SAMPLE, kAAPull>(grp, npt, a, nb, s);
    case kAALocal: return launch_step_grp<T, SHIFTED, COLL, SAMPLE, kAALocal>(grp, npt, a, nb, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, bool SHIFTED>
static hipError_t launch_step_t(int collision, bool sample, int sm, int grp, int npt, const StepArgs& a,
                                uint32_t nb, hipStream_t s)
{
    if (collision == kGMF)
        return sample ? launch_step_sm<T, SHIFTED, kGMF, true>(sm, grp, npt, a, nb, s)
                      : launch_step_sm<T, SHIFTED, kGMF, false>(sm, grp, npt, a, nb, s);
    return sample ? launch_step_sm<T, SHIFTED, kBGK, true>(sm, grp, npt, a, nb, s)
                  : launch_step_sm<T, SHIFTED, kBGK, false>(sm, grp, npt, a, nb, s);
}

hipError_t launch_step(int precision, int collision, bool sample, int sm, int grp, int npt, const StepArgs& a,
                       uint32_t nblocks, hipStream_t s)
{
    // the AA patterns update one buffer in place
    if (sm != kAB && a.src != a.dst) return hipErrorInvalidValue;
    bool occ_known = false;
    for (uint32_t k : kOccCap) occ_known = occ_known || a.occ == k;
    if (!occ_known) return hipErrorInvalidValue;
    if (precision == kFP64) return launch_step_t<double, false>(collision, sample, sm, grp, npt, a, nblocks, s);
    return launch_step_t<float, true>(collision, sample, sm, grp, npt, a, nblocks, s);
}

// ---------------------------------------------------------------------------
// Initial state: rest equilibrium f = w rho0 (shifted: g = 0)
// ---------------------------------------------------------------------------
template <typename T, bool SHIFTED>
__global__ __launch_bounds__(kBlock) void init_kernel(T* buf, const RepDev* rep)
{
    const RepDev& R = *rep;
    const uint32_t n = blockIdx.x * (uint32_t)kBlock + threadIdx.x;
    if (n >= R.n) return;
    const uint32_t x = n % R.nx, y = (n / R.nx) % R.ny, z = n / (R.nx * R.ny);
    T* b = buf + R.pop_offset;
#pragma unroll
    for (int p = 0; p < Q; ++p) b[pop_index(R, p, x, y, z)] = SHIFTED ? T(0) : (T)(tweight(p) * R.rho0);
}

hipError_t launch_init(int precision, void* buf, const RepDev* rep_dev, const RepDev& rep, hipStream_t s)
{
    const uint32_t g = (rep.n + kBlock - 1) / kBlock;
    if (precision == kFP64)
        init_kernel<double, false><<<g, kBlock, 0, s>>>((double*)buf, rep_dev);
    else
        init_kernel<float, true><<<g, kBlock, 0, s>>>((float*)buf, rep_dev);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Step counter kept on the device so that captured graphs can be replayed
// ---------------------------------------------------------------------------
__global__ void set_step_kernel(int64_t* d, int64_t v)
{
    if (threadIdx.x == 0) *d = v;
}
__global__ void advance_step_kernel(int64_t* d, int64_t by)
{
    if (threadIdx.x == 0) *d += by;
}

hipError_t launch_set_step(int64_t* d_step, int64_t value, hipStream_t s)
{
    set_step_kernel<<<1, 64, 0, s>>>(d_step, value);
    return hipGetLastError();
}

hipError_t launch_advance_step(int64_t* d_step, int64_t by, hipStream_t s)
{
    advance_step_kernel<<<1, 64, 0, s>>>(d_step, by);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Canonical order of the interface: rest; faces +x,-x,+y,-y,+z,-z; edges and
// corners in lexicographic order of (cx, cy, cz).
// ---------------------------------------------------------------------------
void canonical_to_tensor(int out[Q])
{
    int i = 0;
    out[i++] = tindex(0, 0, 0);
    const int faces[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
    for (auto& c : faces) out[i++] = tindex(c[0], c[1], c[2]);
    for (int nnz = 2; nnz <= 3; ++nnz)
        for (int cx = -1; cx <= 1; ++cx)
            for (int cy = -1; cy <= 1; ++cy)
                for (int cz = -1; cz <= 1; ++cz)
                    if ((cx != 0) + (cy != 0) + (cz != 0) == nnz) out[i++] = tindex(cx, cy, cz);
}

struct CanonMap {
    int8_t tensor_of[Q];   // canonical i -> tensor p
};

static CanonMap make_canon_map()
{
    CanonMap m;
    int t[Q];
    canonical_to_tensor(t);
    for (int i = 0; i < Q; ++i) m.tensor_of[i] = (int8_t)t[i];
    return m;
}

// canonical f(x) (+ w_p rho0 when shifted, see canon_index), planes z0 <= z < z1
template <typename T, bool SHIFTED>
__global__ __launch_bounds__(kBlock) void gather_kernel(const T* src, const RepDev* rep, uint32_t z0, uint32_t z1,
                                                        double* out, CanonMap cm, int aa_odd)
{
    const RepDev& R = *rep;
    const uint64_t plane = (uint64_t)R.nx * R.ny;
    const uint64_t cnt = plane * (z1 - z0);
    const uint64_t idx = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= cnt) return;
    const uint32_t x = (uint32_t)(idx % R.nx);
    const uint32_t y = (uint32_t)((idx / R.nx) % R.ny);
    const uint32_t z = z0 + (uint32_t)(idx / plane);
    const T* s = src + R.pop_offset;
    for (int i = 0; i < Q; ++i) {
        const int p = cm.tensor_of[i];
        double v = (double)s[canon_index(R, p, x, y, z, aa_odd)];
        if (SHIFTED) v += tweight(p) * R.rho0;
        out[(uint64_t)i * cnt + idx] = v;
    }
}

template <typename T, bool SHIFTED>
__global__ __launch_bounds__(kBlock) void scatter_kernel(T* dst, const RepDev* rep, uint32_t z0, uint32_t z1,
                                                         const double* in, CanonMap cm, int aa_odd)
{
    const RepDev& R = *rep;
    const uint64_t plane = (uint64_t)R.nx * R.ny;
    const uint64_t cnt = plane * (z1 - z0);
    const uint64_t idx = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= cnt) return;
    const uint32_t x = (uint32_t)(idx % R.nx);
    const uint32_t y = (uint32_t)((idx / R.nx) % R.ny);
    const uint32_t z = z0 + (uint32_t)(idx / plane);
    T* d = dst + R.pop_offset;
    for (int i = 0; i < Q; ++i) {
        const int p = cm.tensor_of[i];
        double v = in[(uint64_t)i * cnt + idx];
        if (SHIFTED) v -= tweight(p) * R.rho0;
        d[canon_index(R, p, x, y, z, aa_odd)] = (T)v;
    }
}

// density and velocity of the canonical state plus FP64 workgroup sums of rho, j
template <typename T, bool SHIFTED>
__global__ __launch_bounds__(kBlock) void moments_kernel(const T* src, const RepDev* rep, uint32_t z0, uint32_t z1,
                                                         double* rho_out, double* u_out, double* partials,
                                                         int aa_odd)
{
    const RepDev& R = *rep;
    const uint64_t plane = (uint64_t)R.nx * R.ny;
    const uint64_t cnt = plane * (z1 - z0);
    const uint64_t idx = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (idx < cnt) {
        const uint32_t x = (uint32_t)(idx % R.nx);
        const uint32_t y = (uint32_t)((idx / R.nx) % R.ny);
        const uint32_t z = z0 + (uint32_t)(idx / plane);
        const T* s = src + R.pop_offset;
        double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
        for (int p = 0; p < Q; ++p) {
            double fv = (double)s[canon_index(R, p, x, y, z, aa_odd)];
            if (SHIFTED) fv += tweight(p) * R.rho0;
            rho += fv;
            jx += fv * tcx(p);
            jy += fv * tcy(p);
            jz += fv * tcz(p);
        }
        if (rho_out) rho_out[idx] = rho;
        if (u_out) {
            u_out[idx] = jx / rho;
            u_out[cnt + idx] = jy / rho;
            u_out[2 * cnt + idx] = jz / rho;
        }
        v[0] = rho; v[1] = jx; v[2] = jy; v[3] = jz;
    }
    block_sum_store<4>(v, partials + (size_t)blockIdx.x * 4);
}

__global__ __launch_bounds__(kBlock) void sum_partials_kernel(const double* partials, uint32_t nb, double* out4,
                                                              int accumulate)
{
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (uint32_t b = threadIdx.x; b < nb; b += kBlock)
        for (int q = 0; q < 4; ++q) v[q] += partials[(size_t)b * 4 + q];
    __shared__ double tot[4];
    block_sum_store<4>(v, tot);
    __syncthreads();
    if (threadIdx.x < 4) out4[threadIdx.x] = (accumulate ? out4[threadIdx.x] : 0.0) + tot[threadIdx.x];
}

template <typename T, bool SHIFTED>
__global__ __launch_bounds__(kBlock) void nodes_kernel(const T* src, const RepDev* rep, const int64_t* nodes,
                                                       int32_t count, double* out, CanonMap cm, int aa_odd)
{
    const RepDev& R = *rep;
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= count) return;
    const uint64_t n = (uint64_t)nodes[j];
    const uint32_t x = (uint32_t)(n % R.nx);
    const uint32_t y = (uint32_t)((n / R.nx) % R.ny);
    const uint32_t z = (uint32_t)(n / ((uint64_t)R.nx * R.ny));
    const T* s = src + R.pop_offset;
    for (int i = 0; i < Q; ++i) {
        const int p = cm.tensor_of[i];
        double v = (double)s[canon_index(R, p, x, y, z, aa_odd)];
        if (SHIFTED) v += tweight(p) * R.rho0;
        out[(size_t)j * Q + i] = v;
    }
}

static inline uint32_t grid_for(uint64_t cnt) { return (uint32_t)((cnt + kBlock - 1) / kBlock); }

hipError_t launch_gather(int precision, const void* src, const RepDev* rep_dev, const RepDev& rep, uint32_t z0,
                         uint32_t z1, double* out, int aa_odd, hipStream_t s)
{
    const uint32_t g = grid_for((uint64_t)rep.nx * rep.ny * (z1 - z0));
    static const CanonMap cm = make_canon_map();
    if (precision == kFP64)
        gather_kernel<double, false><<<g, kBlock, 0, s>>>((const double*)src, rep_dev, z0, z1, out, cm, aa_odd);
    else
        gather_kernel<float, true><<<g, kBlock, 0, s>>>((const float*)src, rep_dev, z0, z1, out, cm, aa_odd);
    return hipGetLastError();
}

hipError_t launch_scatter(int precision, void* dst, const RepDev* rep_dev, const RepDev& rep, uint32_t z0,
                          uint32_t z1, const double* in, int aa_odd, hipStream_t s)
{
    const uint32_t g = grid_for((uint64_t)rep.nx * rep.ny * (z1 - z0));
    static const CanonMap cm = make_canon_map();
    if (precision == kFP64)
        scatter_kernel<double, false><<<g, kBlock, 0, s>>>((double*)dst, rep_dev, z0, z1, in, cm, aa_odd);
    else
        scatter_kernel<float, true><<<g, kBlock, 0, s>>>((float*)dst, rep_dev, z0, z1, in, cm, aa_odd);
    return hipGetLastError();
}

hipError_t launch_moments(int precision, const void* src, const RepDev* rep_dev, const RepDev& rep, uint32_t z0,
                          uint32_t z1, double* rho, double* u, double* partials, int aa_odd, hipStream_t s)
{
    const uint32_t g = grid_for((uint64_t)rep.nx * rep.ny * (z1 - z0));
    if (precision == kFP64)
        moments_kernel<double, false><<<g, kBlock, 0, s>>>((const double*)src, rep_dev, z0, z1, rho, u, partials, aa_odd);
    else
        moments_kernel<float, true><<<g, kBlock, 0, s>>>((const float*)src, rep_dev, z0, z1, rho, u, partials, aa_odd);
    return hipGetLastError();
}

hipError_t launch_sum_partials(const double* partials, uint32_t nblocks, double* out4, int accumulate, hipStream_t s)
{
    sum_partials_kernel<<<1, kBlock, 0, s>>>(partials, nblocks, out4, accumulate);
    return hipGetLastError();
}

hipError_t launch_nodes(int precision, const void* src, const RepDev* rep_dev, const int64_t* nodes, int32_t count,
                        double* out, int aa_odd, hipStream_t s)
{
    static const CanonMap cm = make_canon_map();
    const uint32_t g = grid_for((uint64_t)count);
    if (precision == kFP64)
        nodes_kernel<double, false><<<g, kBlock, 0, s>>>((const double*)src, rep_dev, nodes, count, out, cm, aa_odd);
    else
        nodes_kernel<float, true><<<g, kBlock, 0, s>>>((const float*)src, rep_dev, nodes, count, out, cm, aa_odd);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The step kernels' noise generator, exposed for inspection.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void noise_probe_kernel(uint32_t k0, uint32_t k1, int64_t t, uint32_t node0,
                                                             int32_t count, uint32_t* words, double* normals)
{
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= count) return;
    const uint32_t n = node0 + (uint32_t)j;
    if (words) {
        for (int b = 0; b < 6; ++b) {
            const U4 w = noise_block(n, (uint64_t)t, (uint32_t)b, k0, k1);
            words[(size_t)j * 24 + 4 * b + 0] = w.x;
            words[(size_t)j * 24 + 4 * b + 1] = w.y;
            words[(size_t)j * 24 + 4 * b + 2] = w.z;
            words[(size_t)j * 24 + 4 * b + 3] = w.w;
        }
    }
    if (normals) {
        T r[23];
        node_normals<T>(n, (uint64_t)t, k0, k1, r);
        for (int k = 0; k < 23; ++k) normals[(size_t)j * 23 + k] = (double)r[k];
    }
}

// Staging of the allocation-free noise probe (gmf_noise_probe_noalloc): a
// file-scope device array, so that the probe needs no device allocation.  Host
// code never names it except to look up its address per device.
static __device__ __align__(256) unsigned char scratch[kProbeScratchBytes];

hipError_t probe_scratch_address(void** out)
{
    return hipGetSymbolAddress(out, HIP_SYMBOL(scratch));
}

hipError_t launch_noise_probe(int precision, uint64_t seed, int64_t t, uint32_t node0, int32_t count,
                              uint32_t* words, double* normals, hipStream_t s)
{
    const uint32_t g = grid_for((uint64_t)count);
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    if (precision == kFP64)
        noise_probe_kernel<double><<<g, kBlock, 0, s>>>(k0, k1, t, node0, count, words, normals);
    else
        noise_probe_kernel<float><<<g, kBlock, 0, s>>>(k0, k1, t, node0, count, words, normals);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Streaming copy (16-byte nontemporal accesses, one per thread up to 2^28
// threads, grid-stride beyond): the practical bandwidth reference the step
// kernel is compared with.  Of the copy forms measured on MI355X (cached or
// nontemporal, 1 to 8 vectors per thread, grid-stride), this one was fastest.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void copy_kernel(const float4* __restrict__ src, float4* __restrict__ dst,
                                                      uint64_t n4)
{
    typedef float v4f __attribute__((ext_vector_type(4)));
    const v4f* s = reinterpret_cast<const v4f*>(src);
    v4f* d = reinterpret_cast<v4f*>(dst);
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(s + i), d + i);
}

hipError_t launch_copy(const void* src, void* dst, uint64_t bytes, hipStream_t s)
{
    const uint64_t n4 = bytes / 16;
    const uint64_t want = (n4 + kBlock - 1) / kBlock;
    const uint32_t g = (uint32_t)std::min<uint64_t>(want, 1u << 20);
    copy_kernel<<<g, kBlock, 0, s>>>(reinterpret_cast<const float4*>(src), reinterpret_cast<float4*>(dst), n4);
    return hipGetLastError();
}

}  // namespace gmf
