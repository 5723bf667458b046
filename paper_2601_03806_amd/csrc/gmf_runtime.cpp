// gmf_runtime.cpp -- host runtime and C ABI of the GMF-FLBM library (see gmf.h).
//
// A context owns: the replica table, the population buffers (two for the A/B
// pull scheme, where the step with index t reads buffer t%2 and writes the
// other; one for the in-place AA scheme), the sampling buffers and FP64
// accumulators, a staging area for host transfers, the device step counter
// and the captured step-loop graphs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/gmf.h"
#include "gmf_device.hpp"
#include "gmf_fft.hpp"
#include "gmf_graphplan.hpp"
#include "gmf_internal.hpp"

using namespace gmf;

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kStageCap = 64ull << 20;   // staging for host transfers (per chunk of z planes)
constexpr int kDefaultGraphSteps = 64;
// Conservation guard of gmf_stats: relative drift of mass and momentum from the
// replica's reference (see conservation_drift) above which the call reports
// GMF_EUNSTABLE, by precision (GMF_FP64, GMF_FP32_SHIFTED).  The update
// conserves both exactly; rounding moves them by about 1e-16 (FP64) or 3e-9
// (FP32, O(1e-2) shifted populations) per node and step, a random walk far
// below these bounds for any run length a box can afford.
constexpr double kDriftBound[2] = {1e-10, 1e-4};
constexpr int kDefaultNpt = 1;
constexpr float kTuneMargin = 0.01f;   // relative gain a later tuning candidate needs to win
// workgroup mappings: linear, one contiguous range per XCD, runs of 16 blocks per XCD
constexpr int kXcdMaps = 3;
constexpr uint32_t kXcdChunks[kXcdMaps] = {0u, 0u, 16u};
// moment storage: z planes per tile tried by the autotuner, and the default tile
constexpr int kMTzCount = 4;
constexpr uint32_t kMTz[kMTzCount] = {16u, 32u, 64u, 128u};
constexpr int kDefaultMTile = 1;
constexpr uint32_t kDefaultMTz = 64u;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

const double kCs2 = 1.0 / 3.0;
// b_k of the Table II groups feeding RepDev::amp: k=4..6, 7..9, 10..15, 16, 17..19, 20..22, 23..25, 26
const double kGroupB[8] = {2.0 / 9, 1.0 / 9, 2.0 / 27, 1.0 / 27, 4.0 / 81, 2.0 / 81, 4.0 / 243, 8.0 / 729};
const int kShellN2[kShells] = {1, 2, 3, 4, 5, 6, 8, 9};
const int kShellCnt[kShells] = {6, 12, 8, 6, 24, 24, 12, 30};

struct Layout {
    size_t pop_bytes = 0, popA = 0, popB = 0;   // popB == popA: one buffer (AA only)
    size_t reps = 0, blk2rep = 0, step = 0, acc = 0, tot = 0, mpart = 0;
    size_t fields = 0, partials = 0, slices = 0, obs_first = 0, dft = 0, chunks = 0, stage = 0, stage_bytes = 0,
           total = 0;
    uint64_t obs_blocks = 0, obs_slices = 0;   // observables workgroups and their slices (sampling)
    uint32_t total_chunks = 0;     // workgroups of the first DFT stage of the shell spectra
    size_t twiddles = 0, zbuf = 0;
    size_t sample_sq = 0;          // per-sample sums of squares (sampling)
    // full-box spectra (spectrum option)
    bool spectrum = false;
    size_t spec = 0, sbins = 0, sacc = 0, scounts = 0, sfirst = 0;
    uint64_t nshell_total = 0;
    uint32_t max_nshell = 0;        // most shells of one replica
    uint32_t spec_blocks[3] = {0, 0, 0};   // workgroups of the x, y and z (with shell sums) passes
    size_t spec_lds[3] = {0, 0, 0};
    uint32_t tw_complex = 0;
    uint64_t total_nodes = 0;
    uint32_t max_blocks = 0;     // lattice grid at one node per thread
    uint32_t total_planes = 0;
    uint32_t dft_complex = 0;
    uint32_t max_chunk_blocks = 0;
    int max_nx = 0, max_ny = 0;
    bool sampling = false;
};

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Addressing modes of the step kernel (see gmf_kernels.hip) that fit a set of
// replicas: per-node addressing with storage groups of 27, 3 or 1 populations
// when the group's byte offsets fit 32 bits in every replica, and plane-uniform
// addressing (0) when every z plane is a whole number of workgroups of
// kBlock * npt nodes.
bool mode_fits(const gmf_replica* reps, int32_t nrep, uint64_t es, int mode, int npt)
{
    for (int r = 0; r < nrep; ++r) {
        const uint64_t pl = (uint64_t)reps[r].nx * reps[r].ny;
        if (mode == 0) {
            if (pl % ((uint64_t)kBlock * npt) != 0) return false;
        } else if (pl * reps[r].nz * (uint64_t)mode * es >= (1ull << 32)) {
            return false;
        }
    }
    return true;
}

// Default mode: groups of 27 when they fit, else plane-uniform, else 3, else 1;
// -1 when none fits.
int choose_mode(const gmf_replica* reps, int32_t nrep, uint64_t es, int npt)
{
    for (int m : {27, 0, 3, 1})
        if (mode_fits(reps, nrep, es, m, npt)) return m;
    return -1;
}

// Integer wave vectors of an nx x ny x nz box in each shell s = round(|n|)
// (s = 0 holds k = 0 only and is left empty); appends nshell counts.
void count_shells(uint32_t nx, uint32_t ny, uint32_t nz, uint32_t nshell, std::vector<int64_t>& out)
{
    std::vector<int64_t> cnt(nshell, 0);
    for (uint32_t z = 0; z < nz; ++z) {
        const int64_t fz = signed_freq(z, nz);
        for (uint32_t y = 0; y < ny; ++y) {
            const int64_t fy = signed_freq(y, ny);
            const int64_t c = fy * fy + fz * fz;
            for (uint32_t x = 0; x < nx; ++x) {
                const int64_t fx = signed_freq(x, nx);
                const uint64_t n2 = (uint64_t)(fx * fx + c);
                if (n2 > 0) cnt[shell_of(n2)] += 1;
            }
        }
    }
    out.insert(out.end(), cnt.begin(), cnt.end());
}

int validate(const gmf_replica* reps, int32_t nrep, const gmf_options* opt)
{
    if (!reps || nrep < 1 || nrep > 65535) return GMF_EINVAL;
    if (opt) {
        if (opt->precision != GMF_FP64 && opt->precision != GMF_FP32_SHIFTED) return GMF_EINVAL;
        if (opt->collision != GMF_COLLISION_GMF && opt->collision != GMF_COLLISION_BGK) return GMF_EINVAL;
        if (opt->noise_rho != 0 && opt->noise_rho != 1) return GMF_EINVAL;
        if (opt->sample_every < 0 || opt->tune < 0 || opt->tune > 1) return GMF_EINVAL;
        if (opt->streaming < GMF_STREAM_AUTO || opt->streaming > GMF_STREAM_AA) return GMF_EINVAL;
        if (opt->spectrum != 0 && (opt->spectrum != 1 || opt->sample_every <= 0)) return GMF_EINVAL;
        if (opt->storage != GMF_STORE_POPULATIONS && opt->storage != GMF_STORE_MOMENTS) return GMF_EINVAL;
        if (opt->storage == GMF_STORE_MOMENTS &&
            (opt->collision != GMF_COLLISION_GMF || opt->streaming == GMF_STREAM_AA))
            return GMF_EINVAL;
    }
    const size_t es = (opt && opt->precision == GMF_FP32_SHIFTED) ? 4 : 8;
    for (int r = 0; r < nrep; ++r) {
        const gmf_replica& R = reps[r];
        if (R.nx < 1 || R.ny < 1 || R.nz < 1 || R.reserved != 0) return GMF_EINVAL;
        const uint64_t n = (uint64_t)R.nx * R.ny * R.nz;
        // 32-bit node indices; one z plane of 27 population rows within 32-bit byte offsets
        if (n >= (1ull << 31) || (uint64_t)R.nx * R.ny * Q * es >= (1ull << 32)) return GMF_EINVAL;
        if (!finite_pos(R.rho0) || !std::isfinite(R.tau) || !(R.tau > 0.5)) return GMF_EINVAL;
        if (!std::isfinite(R.kbt) || R.kbt < 0.0) return GMF_EINVAL;
        // full-box spectra: line lengths with prime factors 2, 3, 5 only, at most kFftMaxLen
        if (opt && opt->spectrum) {
            FftPlan pl;
            if (!fft_plan((uint32_t)R.nx, pl) || !fft_plan((uint32_t)R.ny, pl) || !fft_plan((uint32_t)R.nz, pl))
                return GMF_EINVAL;
            // every pass's tile (with the z pass's shell bins) within one CU's LDS
            const uint32_t cb = 2u * (uint32_t)es, ns = box_shells((uint32_t)R.nx, (uint32_t)R.ny, (uint32_t)R.nz);
            for (int a = 0; a < 3; ++a)
                if (fft_lds_bytes(a, (uint32_t)R.nx, (uint32_t)R.ny, (uint32_t)R.nz, cb, ns) > kLdsBytes)
                    return GMF_EINVAL;
        }
    }
    if (choose_mode(reps, nrep, es, 1) < 0) return GMF_EINVAL;
    // sampling: the first DFT stage's workgroups of all replicas form one
    // 32-bit grid, and the plane sums of all replicas sit at 32-bit offsets
    if (opt && opt->sample_every > 0) {
        uint64_t dft = 0, chunks = 0;
        for (int r = 0; r < nrep; ++r) {
            dft += (uint64_t)kFields * reps[r].nz * dft_col_blocks((uint32_t)reps[r].nx) * kDftPlane;
            chunks += dft_chunks((uint32_t)reps[r].nx, (uint32_t)reps[r].nz);
        }
        if (dft >= (1ull << 32) || chunks >= (1ull << 31)) return GMF_EINVAL;
    }
    // workgroup and tile counts of the whole context are 32-bit: fewer than
    // 2^32 nodes in all (far beyond any device memory) keeps every one in range
    uint64_t total = 0;
    for (int r = 0; r < nrep; ++r) total += (uint64_t)reps[r].nx * reps[r].ny * reps[r].nz;
    if (total >= (1ull << 32)) return GMF_EINVAL;
    return GMF_OK;
}

Layout plan(const gmf_replica* reps, int32_t nrep, const gmf_options* opt)
{
    Layout L;
    const size_t es = (opt && opt->precision == GMF_FP32_SHIFTED) ? 4 : 8;
    L.sampling = opt && opt->sample_every > 0;
    uint64_t stage_nodes = 0;
    for (int r = 0; r < nrep; ++r) {
        const uint64_t n = (uint64_t)reps[r].nx * reps[r].ny * reps[r].nz;
        const uint64_t plane = (uint64_t)reps[r].nx * reps[r].ny;
        L.total_nodes += n;
        L.max_blocks += (uint32_t)((n + kBlock - 1) / kBlock);
        L.total_planes += (uint32_t)reps[r].nz;
        L.total_chunks += (uint32_t)dft_chunks((uint32_t)reps[r].nx, (uint32_t)reps[r].nz);
        L.dft_complex += (uint32_t)(kFields * reps[r].nz * dft_col_blocks((uint32_t)reps[r].nx) * kDftPlane);
        {
            const uint64_t ob = obs_records(es == 4, reps[r].nx, reps[r].ny, reps[r].nz);
            L.obs_blocks += ob;
            L.obs_slices += (ob + kBlock - 1) / kBlock;
        }
        L.tw_complex += (uint32_t)(reps[r].nx + reps[r].ny + reps[r].nz);
        L.max_nx = std::max(L.max_nx, (int)reps[r].nx);
        L.max_ny = std::max(L.max_ny, (int)reps[r].ny);
        // a chunk holds whole z planes: at least one plane, at most kStageCap bytes of FP64 populations
        uint64_t planes = std::max<uint64_t>(1, kStageCap / (Q * 8 * plane));
        planes = std::min<uint64_t>(planes, (uint64_t)reps[r].nz);
        stage_nodes = std::max(stage_nodes, planes * plane);
    }
    // at least 64 KiB so that node lists (gmf_get_nodes) always have room
    L.stage_bytes = std::max<uint64_t>(stage_nodes * Q * 8, 64u << 10);
    // chunk_planes() never puts more than stage_bytes / (27 * 8) nodes in a chunk
    const uint64_t chunk_nodes_max = L.stage_bytes / (Q * 8);
    L.max_chunk_blocks = (uint32_t)((chunk_nodes_max + kBlock - 1) / kBlock);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + std::max<size_t>(bytes, 1));
        return o;
    };
    const bool mom = opt && opt->storage == GMF_STORE_MOMENTS;
    if (mom) {
        // tiles of the moment-storage step at the shortest tile depth, for the block table
        uint64_t most = 0;
        for (int t = 0; t < kMTiles; ++t) {
            uint64_t tiles = 0;
            for (int r = 0; r < nrep; ++r)
                tiles += (uint64_t)((reps[r].nx + kMTileX[t] - 1) / kMTileX[t]) *
                         ((reps[r].ny + kMTileY[t] - 1) / kMTileY[t]) * ((reps[r].nz + kMTz[0] - 1) / kMTz[0]);
            most = std::max(most, tiles);
        }
        L.max_blocks = (uint32_t)std::max<uint64_t>(L.max_blocks, most);
    }
    L.pop_bytes = (size_t)L.total_nodes * (mom ? kMom : Q) * es;
    L.popA = take(L.pop_bytes);
    L.popB = (opt && opt->streaming == GMF_STREAM_AA) ? L.popA : take(L.pop_bytes);
    L.reps = take(sizeof(RepDev) * nrep);
    L.blk2rep = take(sizeof(uint16_t) * L.max_blocks);
    L.step = take(sizeof(int64_t));
    L.acc = take(sizeof(double) * kAccStride * nrep);
    L.tot = take(sizeof(double) * 4);
    L.mpart = take(sizeof(double) * 4 * L.max_chunk_blocks);
    if (L.sampling) {
        L.fields = take((size_t)L.total_nodes * kFields * es);
        // one record per workgroup of observables_kernel, and their slices of kBlock records
        L.partials = take(sizeof(double) * kPartialStride * L.obs_blocks);
        L.slices = take(sizeof(double) * kPartialStride * L.obs_slices);
        L.obs_first = take(sizeof(uint32_t) * ((size_t)nrep + 1));
        L.dft = take(sizeof(double) * 2 * L.dft_complex);
        L.chunks = take(sizeof(uint32_t) * ((size_t)nrep + 1));   // prefix sums of the first-stage workgroups
        L.twiddles = take(sizeof(double) * 2 * L.tw_complex);
        L.zbuf = take(sizeof(double) * 2 * kFields * 196 * nrep);
        L.sample_sq = take(sizeof(double) * kObs * nrep);
    }
    L.spectrum = L.sampling && opt->spectrum;
    if (L.spectrum) {
        // half spectra of the six fields and of jsum in the kernel precision: complex of 2 es bytes
        const uint32_t cb = 2u * (uint32_t)es;
        uint64_t half_values = 0;
        for (int r = 0; r < nrep; ++r) {
            const uint32_t nx = (uint32_t)reps[r].nx, ny = (uint32_t)reps[r].ny, nz = (uint32_t)reps[r].nz;
            const uint32_t ns = box_shells(nx, ny, nz);
            L.nshell_total += ns;
            L.max_nshell = std::max(L.max_nshell, ns);
            for (int a = 0; a < 3; ++a) {
                L.spec_blocks[a] += fft_tiles(a, nx, ny, nz, cb);
                L.spec_lds[a] = std::max<size_t>(L.spec_lds[a], fft_lds_bytes(a, nx, ny, nz, cb, ns));
            }
            half_values += (uint64_t)kFftFields * half_stride(nx) * ny * nz;
        }
        L.spec = take((size_t)cb * half_values);
        L.sbins = take(sizeof(unsigned long long) * kSpec * kBinCopies * L.nshell_total);
        L.sacc = take(sizeof(double) * kSpec * L.nshell_total);
        L.scounts = take(sizeof(int64_t) * L.nshell_total);
        L.sfirst = take(sizeof(uint32_t) * 3 * (nrep + 1));
    }
    L.stage = take(L.stage_bytes);
    L.total = off;
    return L;
}

gmf_options default_options()
{
    gmf_options o;
    std::memset(&o, 0, sizeof(o));
    o.precision = GMF_FP64;
    o.collision = GMF_COLLISION_GMF;
    o.graph_steps = -1;
    o.storage = GMF_STORE_POPULATIONS;
    return o;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace

struct gmf_ctx {
    gmf_options opt;
    int32_t nrep = 0;
    std::vector<gmf_replica> reps;
    std::vector<RepDev> rdev;
    Layout L;
    int device = 0;
    char* ws = nullptr;
    bool own_ws = false;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // the sampling kernels of a sampling step run on a second stream of the
    // library's own, forked after the step kernel and joined before the next
    // sampling step writes the fields again (or at the end of gmf_step), so
    // they overlap the plain steps in between; in the graph step loop they are
    // a graph of their own (sampler_graph) launched on that stream.  Without
    // the side stream (population storage, or GMF_SAMPLE_OVERLAP=0) they run
    // on the main stream, in the step's graph.
    hipStream_t side = nullptr;
    hipEvent_t side_fork = nullptr, side_join = nullptr;
    bool side_open = false;        // sampling work forked and not yet joined
    hipGraphExec_t sampler_graph = nullptr;
    int npt = kDefaultNpt;
    int grp = 27;                  // storage group size (see gmf_device.hpp)
    int mode = 0;                  // step-kernel addressing mode (choose_mode)
    bool aa = false;               // in-place AA streaming (else A/B)
    bool mom = false;              // moment storage (gmf_mstep.hip); the two buffers alternate like A/B
    int mtile = kDefaultMTile;     // moment storage: tile shape (index into kMTileX/Y)
    uint32_t mtz = kDefaultMTz;    // moment storage: z planes per tile
    uint32_t xcd_count = 1;        // XCDs of the device
    int fft_order = 0;             // spectrum passes pass by pass (0, measured faster) or group by group (1)
    uint32_t fft_classes[3] = {0, 0, 0};   // per axis: bit c set when a replica's lines are of kernel class c
    int xcd_map = 0;               // workgroup mapping: 0 linear, else an index into kXcdChunks
    uint32_t occ = 0;              // population step: workgroups per CU cap (kOccCap; 0: none)
    uint32_t nblocks = 0;          // lattice grid for the current npt
    uint32_t obs_total = 0;        // workgroups of observables_kernel (sampling)
    uint32_t max_slices = 0;       // most statistics slices of one replica (sampling)
    int graph_steps = 0;           // longest captured step loop; 0: direct launches
    int64_t step = 0;
    bool dev_step_valid = false;   // device counter == step
    std::map<int64_t, hipGraphExec_t> graphs;   // keyed by graph_key()
    int64_t graph_launches = 0, graph_steps_run = 0, direct_steps = 0;
    // conservation reference of each replica: mass and momentum[3] (FP64)
    std::vector<std::array<double, 4>> ref;
    bool poisoned = false;

    void* pop(int which) { return ws + (which ? L.popB : L.popA); }
    // buffer holding the state f(., step) and how it is stored there (canon_index)
    void* cur_pop() { return aa ? pop(0) : pop((int)(step & 1)); }
    int aa_odd() const { return aa && (step & 1) ? 1 : 0; }
    RepDev* d_reps() { return reinterpret_cast<RepDev*>(ws + L.reps); }
    uint16_t* d_blk2rep() { return nrep > 1 ? reinterpret_cast<uint16_t*>(ws + L.blk2rep) : nullptr; }
    int64_t* d_step() { return reinterpret_cast<int64_t*>(ws + L.step); }
    double* d_acc() { return reinterpret_cast<double*>(ws + L.acc); }
    double* d_tot() { return reinterpret_cast<double*>(ws + L.tot); }
    double* d_mpart() { return reinterpret_cast<double*>(ws + L.mpart); }
    void* d_fields() { return L.sampling ? ws + L.fields : nullptr; }
    double* d_partials() { return L.sampling ? reinterpret_cast<double*>(ws + L.partials) : nullptr; }
    double* d_slices() { return L.sampling ? reinterpret_cast<double*>(ws + L.slices) : nullptr; }
    uint32_t* d_obs_first() { return L.sampling ? reinterpret_cast<uint32_t*>(ws + L.obs_first) : nullptr; }
    double* d_dft() { return L.sampling ? reinterpret_cast<double*>(ws + L.dft) : nullptr; }
    uint32_t* d_chunks() { return L.sampling ? reinterpret_cast<uint32_t*>(ws + L.chunks) : nullptr; }
    double2* d_twiddles() { return L.sampling ? reinterpret_cast<double2*>(ws + L.twiddles) : nullptr; }
    double2* d_zbuf() { return L.sampling ? reinterpret_cast<double2*>(ws + L.zbuf) : nullptr; }
    double* d_sample_sq() { return L.sampling ? reinterpret_cast<double*>(ws + L.sample_sq) : nullptr; }
    void* d_spec() { return ws + L.spec; }
    unsigned long long* d_sbins() { return reinterpret_cast<unsigned long long*>(ws + L.sbins); }
    double* d_sacc() { return reinterpret_cast<double*>(ws + L.sacc); }
    int64_t* d_scounts() { return reinterpret_cast<int64_t*>(ws + L.scounts); }
    uint32_t* d_sfirst() { return reinterpret_cast<uint32_t*>(ws + L.sfirst); }
    char* d_stage() { return ws + L.stage; }
};

#define CK(expr)                                                                                 \
    do {                                                                                         \
        hipError_t _e = (expr);                                                                  \
        if (_e != hipSuccess) {                                                                  \
            if (getenv("GMF_DEBUG")) fprintf(stderr, "gmf: %s failed: %s\n", #expr, hipGetErrorString(_e)); \
            ctx->poisoned = true;                                                                \
            return GMF_EDEVICE;                                                                  \
        }                                                                                        \
    } while (0)

namespace {

// Workgroup -> replica map and per-replica grid ranges for `npt` nodes per thread.
int build_grid(gmf_ctx* ctx, int npt)
{
    std::vector<uint16_t> map;
    uint32_t b = 0;
    for (int r = 0; r < ctx->nrep; ++r) {
        RepDev& R = ctx->rdev[r];
        const uint32_t per = (uint32_t)kBlock * (uint32_t)npt;
        R.block_begin = b;
        if (ctx->mom)
            R.nblocks = ((R.nx + kMTileX[ctx->mtile] - 1) / kMTileX[ctx->mtile]) *
                        ((R.ny + kMTileY[ctx->mtile] - 1) / kMTileY[ctx->mtile]) * ((R.nz + ctx->mtz - 1) / ctx->mtz);
        else
            R.nblocks = (R.n + per - 1) / per;
        b += R.nblocks;
        if (ctx->nrep > 1) map.insert(map.end(), R.nblocks, (uint16_t)r);
    }
    ctx->nblocks = b;
    ctx->npt = npt;
    CK(hipMemcpyAsync(ctx->d_reps(), ctx->rdev.data(), sizeof(RepDev) * ctx->nrep, hipMemcpyHostToDevice,
                      ctx->stream));
    if (ctx->nrep > 1)
        CK(hipMemcpyAsync(ctx->d_blk2rep(), map.data(), sizeof(uint16_t) * map.size(), hipMemcpyHostToDevice,
                          ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    if (ctx->side) CK(hipStreamSynchronize(ctx->side));
    for (auto& g : ctx->graphs) (void)hipGraphExecDestroy(g.second);
    ctx->graphs.clear();
    if (ctx->sampler_graph) (void)hipGraphExecDestroy(ctx->sampler_graph);
    ctx->sampler_graph = nullptr;
    return GMF_OK;
}

bool sampling_step(const gmf_ctx* ctx, int64_t t)
{
    return ctx->opt.sample_every > 0 && t % ctx->opt.sample_every == 0;
}

// Enqueue the step with index t.  In a graph (in_graph) the kernels read the
// step from the device counter plus offset j.
int step_pattern(const gmf_ctx* ctx, int64_t t) { return ctx->aa ? ((t & 1) ? kAALocal : kAAPull) : kAB; }

// Order the main stream after the sampling work forked last (no-op if none).
int join_side(gmf_ctx* ctx)
{
    if (ctx->side_open) {
        CK(hipStreamWaitEvent(ctx->stream, ctx->side_join, 0));
        ctx->side_open = false;
    }
    return GMF_OK;
}

// The sampling kernels of the sample the step kernel has just written on
// stream s: observables, the DFT stages of the eight smallest shells, the
// statistics, and the full-box spectra when they are on.
int enqueue_sampler(gmf_ctx* ctx, hipStream_t s)
{
    // the observables records come from observables_kernel (FP64) or from the
    // first DFT stage (FP32); the statistics reduction follows both
    if (ctx->opt.precision == GMF_FP64)
        CK(launch_observables(ctx->opt.precision, ctx->d_reps(), ctx->nrep, ctx->d_obs_first(), ctx->obs_total,
                              ctx->d_fields(), ctx->d_partials(), s));
    CK(launch_dft(ctx->opt.precision, ctx->d_reps(), ctx->nrep, ctx->d_chunks(), ctx->L.total_chunks,
                  ctx->d_fields(), ctx->d_twiddles(), reinterpret_cast<double2*>(ctx->d_dft()), ctx->d_zbuf(),
                  ctx->d_acc(), ctx->d_partials(), s));
    CK(launch_stats_reduce(ctx->d_reps(), ctx->nrep, ctx->max_slices, ctx->d_partials(), ctx->d_slices(),
                           ctx->d_acc(), ctx->d_sample_sq(), s));
    if (ctx->L.spectrum)
        CK(launch_spectrum(ctx->opt.precision, ctx->d_reps(), ctx->nrep, ctx->d_sfirst(), ctx->L.spec_blocks,
                           ctx->d_fields(), ctx->d_twiddles(), ctx->d_spec(), ctx->d_sample_sq(), ctx->d_scounts(),
                           ctx->d_sbins(), (uint32_t)(kSpec * ctx->L.nshell_total), ctx->d_sacc(), ctx->L.max_nshell,
                           ctx->L.spec_lds, ctx->fft_classes, ctx->fft_order, s));
    return GMF_OK;
}

// The sampling kernels on the side stream, after the work enqueued so far on
// the main stream: as the captured sampler graph (graph step loop) or as
// direct launches.
int fork_sampler(gmf_ctx* ctx, bool graph)
{
    CK(hipEventRecord(ctx->side_fork, ctx->stream));
    CK(hipStreamWaitEvent(ctx->side, ctx->side_fork, 0));
    if (graph) {
        CK(hipGraphLaunch(ctx->sampler_graph, ctx->side));
    } else {
        const int rc = enqueue_sampler(ctx, ctx->side);
        if (rc != GMF_OK) return rc;
    }
    CK(hipEventRecord(ctx->side_join, ctx->side));
    ctx->side_open = true;
    return GMF_OK;
}

// Capture the sampler graph on the side stream (once per grid).
int capture_sampler(gmf_ctx* ctx)
{
    if (ctx->sampler_graph) return GMF_OK;
    hipGraph_t g = nullptr;
    CK(hipStreamBeginCapture(ctx->side, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_sampler(ctx, ctx->side);
    hipError_t e = hipStreamEndCapture(ctx->side, &g);
    if (rc != GMF_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        ctx->poisoned = true;
        return GMF_EDEVICE;
    }
    e = hipGraphInstantiate(&ctx->sampler_graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        ctx->sampler_graph = nullptr;
        ctx->poisoned = true;
        return GMF_EDEVICE;
    }
    return GMF_OK;
}

// Enqueue the step with index t.  In a graph (in_graph) the kernels read the
// step from the device counter plus offset j, and a sampling step's kernels
// on the side stream are left to the caller (run_steps).
int enqueue_step(gmf_ctx* ctx, int64_t t, bool in_graph, int j)
{
    const int par = ctx->aa ? 0 : (int)(t & 1);
    StepArgs a;
    a.src = ctx->pop(par);
    a.dst = ctx->pop(ctx->aa ? 0 : par ^ 1);
    a.reps = ctx->d_reps();
    a.blk2rep = ctx->d_blk2rep();
    a.d_step = in_graph ? ctx->d_step() : nullptr;
    a.step_base = in_graph ? (int64_t)j : t;
    a.fields = ctx->d_fields();
    a.partials = ctx->d_partials();
    a.nblocks = ctx->nblocks;
    a.xcd = ctx->xcd_map ? ctx->xcd_count : 0u;
    a.chunk = kXcdChunks[ctx->xcd_map];
    a.tz = ctx->mtz;
    a.occ = ctx->mom ? 0u : ctx->occ;
    const bool sample = sampling_step(ctx, t);
    // a sampling step writes the fields that the previous sample's kernels read
    if (sample && !in_graph) {
        const int rc = join_side(ctx);
        if (rc != GMF_OK) return rc;
    }
    if (ctx->mom)
        CK(launch_mstep(ctx->opt.precision, sample, ctx->mtile, a, ctx->nblocks, ctx->stream));
    else
        CK(launch_step(ctx->opt.precision, ctx->opt.collision, sample, step_pattern(ctx, t), ctx->mode, ctx->npt, a,
                       ctx->nblocks, ctx->stream));
    if (sample) {
        if (!ctx->side) return enqueue_sampler(ctx, ctx->stream);
        if (!in_graph) return fork_sampler(ctx, false);
    }
    return GMF_OK;
}

// Step loop in captured HIP graphs: which steps go into which graph is
// decided by gmf_graphplan.hpp.
GraphPlan graph_plan(const gmf_ctx* ctx) { return GraphPlan{ctx->opt.sample_every, ctx->graph_steps}; }

int capture_graph(gmf_ctx* ctx, int64_t t, int64_t len, hipGraphExec_t* out)
{
    hipGraph_t g = nullptr;
    CK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    int rc = GMF_OK;
    for (int j = 0; j < (int)len && rc == GMF_OK; ++j) rc = enqueue_step(ctx, t + j, true, j);
    if (rc == GMF_OK) {
        hipError_t e = launch_advance_step(ctx->d_step(), len, ctx->stream);
        if (e != hipSuccess) rc = GMF_EDEVICE;
    }
    hipError_t e = hipStreamEndCapture(ctx->stream, &g);
    if (rc != GMF_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        ctx->poisoned = true;
        return GMF_EDEVICE;
    }
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        ctx->poisoned = true;
        return GMF_EDEVICE;
    }
    *out = ex;
    return GMF_OK;
}

// The graph for the unit at step t, captured on first use.
int find_graph(gmf_ctx* ctx, int64_t t, int64_t len, bool sample, hipGraphExec_t* out)
{
    const int64_t key = graph_key(t, len, sample);
    if (sample && ctx->side) {
        const int rc = capture_sampler(ctx);
        if (rc != GMF_OK) return rc;
    }
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
        hipGraphExec_t ex;
        const int rc = capture_graph(ctx, t, len, &ex);
        if (rc != GMF_OK) return rc;
        it = ctx->graphs.emplace(key, ex).first;
    }
    *out = it->second;
    return GMF_OK;
}

int run_steps(gmf_ctx* ctx, int64_t n)
{
    while (n > 0) {
        bool sample = false;
        const int64_t len = plan_unit(graph_plan(ctx), ctx->step, n, &sample);
        if (len > 0) {
            hipGraphExec_t ex;
            int rc = find_graph(ctx, ctx->step, len, sample, &ex);
            if (rc != GMF_OK) return rc;
            if (!ctx->dev_step_valid) {
                CK(launch_set_step(ctx->d_step(), ctx->step, ctx->stream));
                ctx->dev_step_valid = true;
            }
            // a sampling step's graph writes the fields the previous sample's kernels read
            if (sample) {
                rc = join_side(ctx);
                if (rc != GMF_OK) return rc;
            }
            CK(hipGraphLaunch(ex, ctx->stream));
            if (sample && ctx->side) {
                rc = fork_sampler(ctx, true);
                if (rc != GMF_OK) return rc;
            }
            ctx->step += len;
            n -= len;
            ctx->graph_launches += 1;
            ctx->graph_steps_run += len;
        } else {
            int rc = enqueue_step(ctx, ctx->step, false, 0);
            if (rc != GMF_OK) return rc;
            ctx->step += 1;
            n -= 1;
            ctx->direct_steps += 1;
            ctx->dev_step_valid = false;
        }
    }
    // the caller's stream orders everything gmf_step enqueued
    return join_side(ctx);
}

// Capture every graph that run_steps(n) from the current step would launch.
int prepare_steps(gmf_ctx* ctx, int64_t n)
{
    return walk_graph_units(graph_plan(ctx), ctx->step, n, [&](int64_t t, int64_t len, bool sample) {
        hipGraphExec_t ex;
        return find_graph(ctx, t, len, sample, &ex);
    });
}

// Storage layout of every replica for addressing mode m (0: plane-uniform with
// groups of 27).  Only the host records change; the caller re-uploads them.
void set_layout(gmf_ctx* ctx, int m)
{
    ctx->mode = m;
    ctx->grp = m == 0 ? 27 : m;
    for (auto& R : ctx->rdev) {
        R.grp = (uint32_t)ctx->grp;
        R.grp_elems = (uint64_t)R.n * R.grp;
        R.row_stride = R.grp * R.nx;
    }
}

// Rest equilibrium in the buffer that the next step reads.
int init_state(gmf_ctx* ctx)
{
    // moment storage: the rest state has zero shifted moments
    if (ctx->mom) {
        CK(hipMemsetAsync(ctx->cur_pop(), 0, ctx->L.pop_bytes, ctx->stream));
        CK(hipStreamSynchronize(ctx->stream));
        return GMF_OK;
    }
    for (int r = 0; r < ctx->nrep; ++r)
        CK(launch_init(ctx->opt.precision, ctx->cur_pop(), ctx->d_reps() + r, ctx->rdev[r],
                       ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    return GMF_OK;
}

// Autotuner support shared by both storages.  A candidate is up to five
// integer parameters.  The file named by GMF_TUNE_CACHE caches choices as
// lines "key v0 v1 v2 v3 v4"; the last line for a key whose parameters still
// fit the context is used, and lines of any other form are skipped.
using TuneParams = std::array<int, 5>;

bool tune_cache_read(const std::string& key, const std::function<bool(const TuneParams&)>& valid, TuneParams* out)
{
    const char* path = getenv("GMF_TUNE_CACHE");
    FILE* fh = path ? fopen(path, "r") : nullptr;
    if (!fh) return false;
    char line[8192], k[4096], extra[2];
    TuneParams v;
    bool found = false;
    while (fgets(line, sizeof(line), fh))
        if (sscanf(line, "%4095s %d %d %d %d %d %1s", k, &v[0], &v[1], &v[2], &v[3], &v[4], extra) == 6 && key == k &&
            valid(v)) {
            *out = v;
            found = true;
        }
    fclose(fh);
    return found;
}

void tune_cache_append(const std::string& key, const TuneParams& v)
{
    const char* path = getenv("GMF_TUNE_CACHE");
    if (FILE* fh = path ? fopen(path, "a") : nullptr) {
        fprintf(fh, "%s %d %d %d %d %d\n", key.c_str(), v[0], v[1], v[2], v[3], v[4]);
        fclose(fh);
    }
}

struct EventPair {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~EventPair()
    {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

// Time every candidate on the context's stream in two rounds, so that a
// transient slowdown does not decide the choice (the faster round counts):
// `configure` sets the context up for a candidate, `launch(c, i)` enqueues its
// step number i; two steps warm up, eight are timed (an even count, so that
// AA runs whole pull/local pairs).  *best receives the fastest candidate,
// where a candidate displaces an earlier one only when it is faster by more
// than kTuneMargin: near-ties go to the earlier candidate, so the choice does
// not follow timing noise from one context to the next.
int tune_time(gmf_ctx* ctx, const std::vector<TuneParams>& cands, const std::function<int(const TuneParams&)>& configure,
              const std::function<hipError_t(const TuneParams&, int)>& launch, TuneParams* best)
{
    if (cands.empty()) return GMF_OK;
    EventPair ev;
    CK(hipEventCreate(&ev.e0));
    CK(hipEventCreate(&ev.e1));
    std::vector<float> ms(cands.size(), 1e30f);
    const int reps = 8;
    for (int round = 0; round < 2; ++round)
        for (size_t c = 0; c < cands.size(); ++c) {
            const int rc = configure(cands[c]);
            if (rc != GMF_OK) return rc;
            CK(launch(cands[c], 0));
            CK(launch(cands[c], 1));
            CK(hipEventRecord(ev.e0, ctx->stream));
            for (int i = 0; i < reps; ++i) CK(launch(cands[c], i));
            CK(hipEventRecord(ev.e1, ctx->stream));
            CK(hipEventSynchronize(ev.e1));
            float t = 0.f;
            CK(hipEventElapsedTime(&t, ev.e0, ev.e1));
            ms[c] = std::min(ms[c], t);
        }
    size_t bi = 0;
    for (size_t c = 1; c < cands.size(); ++c)
        if (ms[c] < ms[bi] * (1.0f - kTuneMargin)) bi = c;
    *best = cands[bi];
    return GMF_OK;
}

std::string boxes_key(const gmf_ctx* ctx)
{
    std::string key;
    for (auto& r : ctx->reps) key += "_" + std::to_string(r.nx) + "x" + std::to_string(r.ny) + "x" + std::to_string(r.nz);
    return key;
}

bool contains(const std::vector<int>& v, int x) { return std::find(v.begin(), v.end(), x) != v.end(); }

// Population storage: time every fitting (addressing mode, nodes per thread,
// streaming pattern, workgroup-to-XCD mapping) combination on the initial
// state without an occupancy cap; then, for the fastest addressing mode and
// nodes per thread, every (streaming pattern, mapping, occupancy cap
// (kOccCap)); keep the fastest and restore the initial state in its layout.  A/B re-runs the same step from the same source buffer; AA
// alternates its two step kinds in place (the state then changes, which does
// not matter for the timing and is undone by the re-initialisation).  AA is a
// candidate only when the options leave the pattern open; A/B only when the
// workspace has its second buffer.
int autotune(gmf_ctx* ctx)
{
    const uint64_t es = ctx->opt.precision == GMF_FP32_SHIFTED ? 4 : 8;
    std::vector<int> patterns;
    if (ctx->opt.streaming != GMF_STREAM_AA) patterns.push_back(GMF_STREAM_AB);
    if (ctx->opt.streaming != GMF_STREAM_AB) patterns.push_back(GMF_STREAM_AA);
    const std::string key = "v4p" + std::to_string(ctx->opt.precision) + "c" + std::to_string(ctx->opt.collision) +
                            "s" + std::to_string(ctx->opt.streaming) + boxes_key(ctx);
    std::vector<int> maps = {0};
    if (ctx->xcd_count > 1)
        for (int xm = 1; xm < kXcdMaps; ++xm) maps.push_back(xm);
    std::vector<int> caps(kOccCap, kOccCap + kOccCaps);
    // parameters: addressing mode, nodes per thread, streaming pattern, mapping, occupancy cap
    auto fits = [&](const TuneParams& v) {
        return contains({27, 0, 3, 1}, v[0]) && (v[1] == 1 || v[1] == 2) &&
               mode_fits(ctx->reps.data(), ctx->nrep, es, v[0], v[1]) && contains(patterns, v[2]) &&
               contains(maps, v[3]) && contains(caps, v[4]);
    };
    TuneParams best = {ctx->mode, ctx->npt, ctx->aa ? GMF_STREAM_AA : GMF_STREAM_AB, ctx->xcd_map, (int)ctx->occ};
    if (!tune_cache_read(key, fits, &best)) {
        std::vector<TuneParams> cands;
        for (int pat : patterns)
            for (int m : {27, 0, 3, 1})
                for (int c : {1, 2})
                    for (int xm : maps)
                        if (fits({m, c, pat, xm, 0})) cands.push_back({m, c, pat, xm, 0});
        StepArgs a;
        auto configure = [&](const TuneParams& v) {
            set_layout(ctx, v[0]);
            const int rc = build_grid(ctx, v[1]);
            std::memset(&a, 0, sizeof(a));
            a.src = ctx->pop(0);
            a.dst = ctx->pop(v[2] == GMF_STREAM_AA ? 0 : 1);
            a.reps = ctx->d_reps();
            a.blk2rep = ctx->d_blk2rep();
            a.step_base = ctx->step;
            a.nblocks = ctx->nblocks;
            a.xcd = v[3] ? ctx->xcd_count : 0u;
            a.chunk = kXcdChunks[v[3]];
            a.occ = (uint32_t)v[4];
            return rc;
        };
        auto launch = [&](const TuneParams& v, int i) {
            const int sm = v[2] == GMF_STREAM_AA ? ((i & 1) ? kAALocal : kAAPull) : kAB;
            return launch_step(ctx->opt.precision, ctx->opt.collision, false, sm, v[0], v[1], a, ctx->nblocks,
                               ctx->stream);
        };
        int rc = tune_time(ctx, cands, configure, launch, &best);
        if (rc != GMF_OK) return rc;
        // second stage: the chosen addressing mode and nodes per thread with
        // every streaming pattern, mapping and occupancy cap (the mapping that
        // wins without a cap need not win with one)
        std::vector<TuneParams> occs;
        for (int pat : patterns)
            for (int xm : maps)
                for (uint32_t k : kOccCap) occs.push_back({best[0], best[1], pat, xm, (int)k});
        rc = tune_time(ctx, occs, configure, launch, &best);
        if (rc != GMF_OK) return rc;
        tune_cache_append(key, best);
    }
    ctx->aa = best[2] == GMF_STREAM_AA;
    ctx->xcd_map = best[3];
    ctx->occ = (uint32_t)best[4];
    set_layout(ctx, best[0]);
    const int rc = build_grid(ctx, best[1]);
    if (rc != GMF_OK) return rc;
    return init_state(ctx);
}

// Moment storage: time every fitting (tile shape, tile depth, workgroup
// mapping) on the initial state in the same way, keep the fastest, and
// restore the initial state.
int autotune_moments(gmf_ctx* ctx)
{
    const size_t es = ctx->opt.precision == GMF_FP32_SHIFTED ? 4 : 8;
    const std::string key = "m3p" + std::to_string(ctx->opt.precision) + boxes_key(ctx);
    // the halo columns a tile reads again are L2 hits only when neighbouring
    // tiles run on the same XCD: with several XCDs only the XCD mappings are
    // tried (the linear one measured 1.66x the algorithmic reads at 256^3)
    std::vector<int> maps;
    if (ctx->xcd_count > 1)
        for (int xm = 1; xm < kXcdMaps; ++xm) maps.push_back(xm);
    else
        maps.push_back(0);
    // parameters: tile shape, tile depth, mapping, two unused
    auto fits = [&](const TuneParams& v) {
        return v[0] >= 0 && v[0] < kMTiles && mtile_fits(v[0], es) && v[1] >= (int)kMTz[0] && contains(maps, v[2]) &&
               v[3] == 0 && v[4] == 0;
    };
    TuneParams best = {ctx->mtile, (int)ctx->mtz, maps.front(), 0, 0};
    if (!tune_cache_read(key, fits, &best)) {
        std::vector<TuneParams> cands;
        for (int tl = 0; tl < kMTiles; ++tl)
            for (uint32_t tz : kMTz)
                for (int xm : maps)
                    if (fits({tl, (int)tz, xm, 0, 0})) cands.push_back({tl, (int)tz, xm, 0, 0});
        StepArgs a;
        auto configure = [&](const TuneParams& v) {
            ctx->mtile = v[0];
            ctx->mtz = (uint32_t)v[1];
            const int rc = build_grid(ctx, 1);
            std::memset(&a, 0, sizeof(a));
            a.src = ctx->pop(0);
            a.dst = ctx->pop(1);
            a.reps = ctx->d_reps();
            a.blk2rep = ctx->d_blk2rep();
            a.step_base = ctx->step;
            a.nblocks = ctx->nblocks;
            a.xcd = v[2] ? ctx->xcd_count : 0u;
            a.chunk = kXcdChunks[v[2]];
            a.tz = (uint32_t)v[1];
            return rc;
        };
        auto launch = [&](const TuneParams& v, int) {
            return launch_mstep(ctx->opt.precision, false, v[0], a, ctx->nblocks, ctx->stream);
        };
        const int rc = tune_time(ctx, cands, configure, launch, &best);
        if (rc != GMF_OK) return rc;
        tune_cache_append(key, best);
    }
    ctx->mtile = best[0];
    ctx->mtz = (uint32_t)best[1];
    ctx->xcd_map = best[2];
    const int rc = build_grid(ctx, 1);
    if (rc != GMF_OK) return rc;
    return init_state(ctx);
}

uint32_t chunk_planes(const gmf_ctx* ctx, int r)
{
    const uint64_t plane = (uint64_t)ctx->reps[r].nx * ctx->reps[r].ny;
    uint64_t p = std::max<uint64_t>(1, ctx->L.stage_bytes / (Q * 8 * plane));
    return (uint32_t)std::min<uint64_t>(p, (uint64_t)ctx->reps[r].nz);
}

// FP64 mass and momentum of the current state of replica r (tot[0] = sum_x rho,
// tot[1..3] = sum_x rho u), summed on the device over chunks of z planes.
int device_totals(gmf_ctx* ctx, int r, double tot[4])
{
    const RepDev& R = ctx->rdev[r];
    const uint64_t plane = (uint64_t)R.nx * R.ny;
    const uint32_t cp = chunk_planes(ctx, r);
    bool first = true;
    for (uint32_t z0 = 0; z0 < R.nz; z0 += cp) {
        const uint32_t z1 = std::min(R.nz, z0 + cp);
        const uint64_t cnt = plane * (z1 - z0);
        const uint32_t nb = (uint32_t)((cnt + kBlock - 1) / kBlock);
        if (ctx->mom)
            CK(launch_mmoments(ctx->opt.precision, ctx->cur_pop(), ctx->d_reps() + r, R, z0, z1, nullptr, nullptr,
                               ctx->d_mpart(), ctx->stream));
        else
            CK(launch_moments(ctx->opt.precision, ctx->cur_pop(), ctx->d_reps() + r, R, z0, z1, nullptr, nullptr,
                              ctx->d_mpart(), ctx->aa_odd(), ctx->stream));
        CK(launch_sum_partials(ctx->d_mpart(), nb, ctx->d_tot(), first ? 0 : 1, ctx->stream));
        first = false;
    }
    CK(hipMemcpyAsync(tot, ctx->d_tot(), sizeof(double) * 4, hipMemcpyDeviceToHost, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    return GMF_OK;
}

// Relative drift of mass and momentum from the reference:
// max(|M - M_ref|, max_a |J_a - J_ref,a|) / |M_ref| (momentum per unit mass, a velocity).
double conservation_drift(const double tot[4], const std::array<double, 4>& ref)
{
    double d = std::fabs(tot[0] - ref[0]);
    for (int a = 1; a < 4; ++a) d = std::max(d, std::fabs(tot[a] - ref[a]));
    return d / std::fabs(ref[0]);
}

int check_ctx(gmf_ctx* ctx)
{
    if (!ctx) return GMF_ESTATE;
    if (ctx->poisoned) return GMF_EDEVICE;
    return GMF_OK;
}

}  // namespace

extern "C" {

size_t gmf_workspace_bytes(const gmf_replica* reps, int32_t nrep, const gmf_options* opt)
{
    if (validate(reps, nrep, opt) != GMF_OK) return 0;
    return plan(reps, nrep, opt).total;
}

int gmf_init(const gmf_replica* reps, int32_t nrep, const gmf_options* opt_in, void* dev_workspace,
             size_t ws_bytes, void* hip_stream, gmf_ctx** out)
{
    if (!out) return GMF_EINVAL;
    *out = nullptr;
    int rc = validate(reps, nrep, opt_in);
    if (rc != GMF_OK) return rc;
    gmf_options opt = opt_in ? *opt_in : default_options();
    Layout L = plan(reps, nrep, &opt);
    if (dev_workspace && (ws_bytes < L.total || ((uintptr_t)dev_workspace % kAlign) != 0)) return GMF_EINVAL;

    gmf_ctx* ctx = new (std::nothrow) gmf_ctx();
    if (!ctx) return GMF_ENOMEM;
    ctx->opt = opt;
    ctx->nrep = nrep;
    ctx->reps.assign(reps, reps + nrep);
    ctx->L = L;
    if (hipGetDevice(&ctx->device) != hipSuccess) {
        delete ctx;
        return GMF_EDEVICE;
    }
    if (dev_workspace) {
        ctx->ws = static_cast<char*>(dev_workspace);
    } else {
        if (hipMalloc((void**)&ctx->ws, L.total) != hipSuccess) {
            (void)hipGetLastError();
            delete ctx;
            return GMF_ENOMEM;
        }
        ctx->own_ws = true;
    }
    if (hip_stream) {
        ctx->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            gmf_destroy(ctx);
            return GMF_EDEVICE;
        }
        ctx->own_stream = true;
    }
    if (L.sampling) {
        // the side stream pays where the step kernel leaves HBM bandwidth unused:
        // moment storage (bound by its vector ALU work) gains 1-2% per sampled
        // step; the population step streams HBM near the copy rate and loses 2%
        // when the sampling kernels compete with it.  GMF_SAMPLE_OVERLAP = 0 | 1
        // forces either.
        const char* ov = getenv("GMF_SAMPLE_OVERLAP");
        const bool overlap = ov ? strcmp(ov, "0") != 0 : opt.storage == GMF_STORE_MOMENTS;
        if (overlap) {
            if (hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&ctx->side_fork, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&ctx->side_join, hipEventDisableTiming) != hipSuccess) {
                (void)hipGetLastError();
                gmf_destroy(ctx);
                return GMF_EDEVICE;
            }
        }
    }

    // addressing mode (one per context: the step kernel is instantiated for it)
    ctx->mode = choose_mode(reps, nrep, opt.precision == GMF_FP32_SHIFTED ? 4 : 8, 1);
    // GMF_ADDRESSING = plane | 27 | 3 | 1 forces an addressing mode (used by the
    // tests to run every mode on the same problem; ignored when it does not fit)
    if (const char* forced = getenv("GMF_ADDRESSING")) {
        const int m = strcmp(forced, "plane") == 0 ? 0 : atoi(forced);
        const bool known = strcmp(forced, "plane") == 0 || m == 27 || m == 3 || m == 1;
        if (known && mode_fits(reps, nrep, opt.precision == GMF_FP32_SHIFTED ? 4 : 8, m, 1)) ctx->mode = m;
    }
    ctx->grp = ctx->mode == 0 ? 27 : ctx->mode;
    ctx->aa = opt.streaming == GMF_STREAM_AA;
    ctx->mom = opt.storage == GMF_STORE_MOMENTS;
    // GMF_MTILE = "tile,depth" forces the moment-storage tile (tests)
    if (const char* forced = getenv("GMF_MTILE")) {
        int tl = -1, tz = 0;
        if (sscanf(forced, "%d,%d", &tl, &tz) == 2 && tl >= 0 && tl < kMTiles && tz >= (int)kMTz[0] &&
            mtile_fits(tl, opt.precision == GMF_FP32_SHIFTED ? 4 : 8)) {
            ctx->mtile = tl;
            ctx->mtz = (uint32_t)tz;
        }
    }
    {
        int nx = 0;
        if (hipDeviceGetAttribute(&nx, hipDeviceAttributeNumberOfXccs, ctx->device) == hipSuccess && nx > 1)
            ctx->xcd_count = (uint32_t)nx;
        else
            (void)hipGetLastError();
    }
    // moment storage reads the halo columns of a tile again: by default each
    // XCD takes runs of neighbouring tiles, so that those reads hit its L2
    if (ctx->mom && ctx->xcd_count > 1) ctx->xcd_map = 2;
    // GMF_OCCUPANCY = k forces an occupancy cap of the population step (tests;
    // k in kOccCap, 0: none)
    if (const char* forced = getenv("GMF_OCCUPANCY")) {
        const int k = atoi(forced);
        for (uint32_t c : kOccCap)
            if ((int)c == k) ctx->occ = c;
    }
    // GMF_BLOCK_MAP = linear | xcd | xcd16 forces the workgroup-to-block mapping (tests)
    if (const char* forced = getenv("GMF_BLOCK_MAP")) {
        ctx->xcd_map = 0;
        if (ctx->xcd_count > 1 && strcmp(forced, "xcd") == 0) ctx->xcd_map = 1;
        if (ctx->xcd_count > 1 && strcmp(forced, "xcd16") == 0) ctx->xcd_map = 2;
    }
    // spectrum kernel classes present along each axis
    for (int r = 0; r < nrep; ++r) {
        ctx->fft_classes[0] |= 1u << fft_class((uint32_t)reps[r].nx);
        ctx->fft_classes[1] |= 1u << fft_class((uint32_t)reps[r].ny);
        ctx->fft_classes[2] |= 1u << fft_class((uint32_t)reps[r].nz);
    }
    // GMF_FFT_ORDER = 0 | 1 forces the order of the spectrum passes (tests)
    if (const char* forced = getenv("GMF_FFT_ORDER")) {
        const int k = atoi(forced);
        if (k == 0 || k == 1) ctx->fft_order = k;
    }
    // replica records
    uint64_t pop_off = 0, field_off = 0, spec_off = 0;
    uint32_t dft_off = 0, tw_off = 0, shell_off = 0, slice_off = 0;
    std::vector<uint32_t> obs_first(1, 0u);   // prefix sums of the observables workgroups
    std::vector<uint32_t> chunks(1, 0u);   // prefix sums of the first DFT stage's workgroups
    std::vector<int64_t> shell_counts;
    std::vector<uint32_t> spec_first(L.spectrum ? 3 * (size_t)(nrep + 1) : 0, 0u);
    for (int r = 0; r < nrep; ++r) {
        const gmf_replica& in = reps[r];
        RepDev R;
        std::memset(&R, 0, sizeof(R));
        R.nx = (uint32_t)in.nx;
        R.ny = (uint32_t)in.ny;
        R.nz = (uint32_t)in.nz;
        R.n = R.nx * R.ny * R.nz;
        R.divx = make_fastdiv(R.nx);
        R.divy = make_fastdiv(R.ny);
        R.pop_offset = pop_off;
        R.field_offset = field_off;
        R.dft_offset = dft_off;
        R.tw_offset = tw_off;
        // observables reduction: obs_records partial records, slices of kBlock of them
        R.obs_first = ctx->obs_total;
        R.obs_blocks = (uint32_t)obs_records(opt.precision == GMF_FP32_SHIFTED, R.nx, R.ny, R.nz);
        R.slice_first = slice_off;
        ctx->obs_total += R.obs_blocks;
        slice_off += (R.obs_blocks + kBlock - 1) / kBlock;
        ctx->max_slices = std::max(ctx->max_slices, (R.obs_blocks + kBlock - 1) / kBlock);
        obs_first.push_back(ctx->obs_total);
        tw_off += R.nx + R.ny + R.nz;
        pop_off += (uint64_t)(ctx->mom ? kMom : Q) * R.n;
        field_off += (uint64_t)kFields * R.n;
        dft_off += (uint32_t)(kFields * R.nz * dft_col_blocks(R.nx) * kDftPlane);
        R.key0 = (uint32_t)in.seed;
        R.key1 = (uint32_t)(in.seed >> 32);
        R.noise_on = in.kbt > 0.0 ? 1u : 0u;
        R.noise_rho0 = (uint32_t)opt.noise_rho;
        R.rho0 = in.rho0;
        R.omega = 1.0 / in.tau;
        R.one_m_omega = 1.0 - R.omega;
        // phi_k / sqrt(rho): Eq. (2) for k = 4..9 (and every k under BGK), Eq. (9) for GMF ghosts
        const double relax = R.omega * (2.0 - R.omega);
        for (int g = 0; g < 8; ++g) {
            const bool hydro = g < 2 || opt.collision == GMF_COLLISION_BGK;
            R.amp[g] = std::sqrt(in.kbt * (hydro ? relax : 1.0) * kGroupB[g] / kCs2);
            R.ampf[g] = (float)R.amp[g];
        }
        R.rho0f = (float)R.rho0;
        R.omegaf = (float)R.omega;
        R.one_m_omegaf = (float)R.one_m_omega;
        if (L.spectrum) {
            const uint32_t cb = opt.precision == GMF_FP32_SHIFTED ? 8u : 16u;   // complex value of the kernels
            R.spec_offset = spec_off;
            R.shell_offset = shell_off;
            R.nshell = box_shells(R.nx, R.ny, R.nz);
            spec_off += (uint64_t)kFftFields * half_stride(R.nx) * R.ny * R.nz;
            shell_off += R.nshell;
            count_shells(R.nx, R.ny, R.nz, R.nshell, shell_counts);
            for (int a = 0; a < 3; ++a)
                spec_first[(size_t)a * (nrep + 1) + r + 1] =
                    spec_first[(size_t)a * (nrep + 1) + r] + fft_tiles(a, R.nx, R.ny, R.nz, cb);
        }
        ctx->rdev.push_back(R);
        if (L.sampling) chunks.push_back(chunks.back() + (uint32_t)dft_chunks(R.nx, R.nz));
    }
    if (L.sampling) {
        hipError_t e = hipMemcpy(ctx->d_chunks(), chunks.data(), sizeof(uint32_t) * chunks.size(),
                                 hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(ctx->d_obs_first(), obs_first.data(), sizeof(uint32_t) * obs_first.size(),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess && L.spectrum) {
            e = hipMemcpy(ctx->d_scounts(), shell_counts.data(), sizeof(int64_t) * shell_counts.size(),
                          hipMemcpyHostToDevice);
            if (e == hipSuccess)
                e = hipMemcpy(ctx->d_sfirst(), spec_first.data(), sizeof(uint32_t) * spec_first.size(),
                              hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) {
            gmf_destroy(ctx);
            return GMF_EDEVICE;
        }
    }
    ctx->graph_steps = opt.graph_steps < 0 ? kDefaultGraphSteps : opt.graph_steps;

    set_layout(ctx, ctx->mode);
    rc = build_grid(ctx, kDefaultNpt);
    if (rc == GMF_OK) rc = init_state(ctx);
    if (rc == GMF_OK && L.sampling) {
        if (launch_twiddles(ctx->d_reps(), nrep, ctx->d_twiddles(), ctx->stream) != hipSuccess) rc = GMF_EDEVICE;
    }
    if (rc != GMF_OK) {
        gmf_destroy(ctx);
        return rc;
    }
    if (hipMemsetAsync(ctx->d_acc(), 0, sizeof(double) * kAccStride * nrep, ctx->stream) != hipSuccess ||
        (L.spectrum &&
         (hipMemsetAsync(ctx->d_sbins(), 0, sizeof(unsigned long long) * kSpec * kBinCopies * L.nshell_total, ctx->stream) !=
              hipSuccess ||
          hipMemsetAsync(ctx->d_sacc(), 0, sizeof(double) * kSpec * L.nshell_total, ctx->stream) != hipSuccess)) ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
        gmf_destroy(ctx);
        return GMF_EDEVICE;
    }
    if (opt.tune) {
        rc = ctx->mom ? autotune_moments(ctx) : autotune(ctx);
        if (rc != GMF_OK) {
            gmf_destroy(ctx);
            return rc;
        }
    }
    // conservation references of the rest state, as stored
    ctx->ref.assign(nrep, std::array<double, 4>{0.0, 0.0, 0.0, 0.0});
    for (int r = 0; r < nrep && rc == GMF_OK; ++r) rc = gmf_set_reference(ctx, r, nullptr);
    if (rc != GMF_OK) {
        gmf_destroy(ctx);
        return rc;
    }
    *out = ctx;
    return GMF_OK;
}

int gmf_step(gmf_ctx* ctx, int64_t n)
{
    int rc = check_ctx(ctx);
    if (rc != GMF_OK) return rc;
    if (n < 0) return GMF_EINVAL;
    DeviceGuard g(ctx->device);
    return run_steps(ctx, n);
}

int gmf_prepare(gmf_ctx* ctx, int64_t n)
{
    int rc = check_ctx(ctx);
    if (rc != GMF_OK) return rc;
    if (n < 0) return GMF_EINVAL;
    DeviceGuard g(ctx->device);
    return prepare_steps(ctx, n);
}

int gmf_get_launch_counts(gmf_ctx* ctx, int64_t* graph_launches, int64_t* graph_steps, int64_t* direct_steps,
                          int32_t* graphs_captured)
{
    if (!ctx) return GMF_ESTATE;
    if (graph_launches) *graph_launches = ctx->graph_launches;
    if (graph_steps) *graph_steps = ctx->graph_steps_run;
    if (direct_steps) *direct_steps = ctx->direct_steps;
    if (graphs_captured) *graphs_captured = (int32_t)ctx->graphs.size();
    return GMF_OK;
}

int gmf_moments(gmf_ctx* ctx, int32_t r, double* rho, double* u)
{
    int rc = check_ctx(ctx);
    if (rc != GMF_OK) return rc;
    if (r < 0 || r >= ctx->nrep) return GMF_EINVAL;
    DeviceGuard g(ctx->device);
    const RepDev& R = ctx->rdev[r];
    const uint64_t plane = (uint64_t)R.nx * R.ny;
    const uint32_t cp = chunk_planes(ctx, r);
    double* srho = reinterpret_cast<double*>(ctx->d_stage());
    for (uint32_t z0 = 0; z0 < R.nz; z0 += cp) {
        const uint32_t z1 = std::min(R.nz, z0 + cp);
        const uint64_t cnt = plane * (z1 - z0);
        double* su = srho + cnt;
        if (ctx->mom)
            CK(launch_mmoments(ctx->opt.precision, ctx->cur_pop(), ctx->d_reps() + r, R, z0, z1, srho, su,
                               ctx->d_mpart(), ctx->stream));
        else
            CK(launch_moments(ctx->opt.precision, ctx->cur_pop(), ctx->d_reps() + r, R, z0, z1, srho, su,
                              ctx->d_mpart(), ctx->aa_odd(), ctx->stream));
        CK(hipStreamSynchronize(ctx->stream));
        if (rho) CK(hipMemcpy(rho + plane * z0, srho, sizeof(double) * cnt, hipMemcpyDeviceToHost));
        if (u)
            for (int a = 0; a < 3; ++a)
                CK(hipMemcpy(u + (uint64_t)a * R.n + plane * z0, su + a * cnt, sizeof(double) * cnt,
                             hipMemcpyDeviceToHost));
    }
    return GMF_OK;
}

int gmf_stats(gmf_ctx* ctx, int32_t r, gmf_stats_t* out)
{
    int rc = check_ctx(ctx);
    if (rc != GMF_OK) return rc;
    if (r < 0 || r >= ctx->nrep || !out) return GMF_EINVAL;
    DeviceGuard g(ctx->device);
    double tot[4];
    rc = device_totals(ctx, r, tot);
    if (rc != GMF_OK) return rc;
    std::vector<double> acc(kAccStride);
    CK(hipMemcpyAsync(acc.data(), ctx->d_acc() + (size_t)r * kAccStride, sizeof(double) * kAccStride,
                      hipMemcpyDeviceToHost, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    std::memset(out, 0, sizeof(*out));
    out->step = ctx->step;
    out->nsamples = (int64_t)acc[kAccNsamp];
    out->nonfinite = (int64_t)acc[kAccNonfinite];
    out->mass = tot[0];
    for (int a = 0; a < 3; ++a) out->momentum[a] = tot[1 + a];
    for (int q = 0; q < kObs; ++q) {
        out->sum_mean[q] = acc[kAccMean + q];
        out->sum_meansq[q] = acc[kAccMeanSq + q];
        out->sum_var[q] = acc[kAccVar + q];
    }
    for (int m = 0; m < kSpec; ++m)
        for (int s = 0; s < kShells; ++s) out->spectrum[m][s] = acc[kAccSpec + m * kShells + s];
    for (int s = 0; s < kShells; ++s) {
        out->shell_n2[s] = kShellN2[s];
        out->shell_count[s] = kShellCnt[s];
    }
    const std::array<double, 4>& ref = ctx->ref[r];
    out->mass_ref = ref[0];
    for (int a = 0; a < 3; ++a) out->momentum_ref[a] = ref[1 + a];
    out->drift = conservation_drift(tot, ref);
    out->drift_bound = kDriftBound[ctx->opt.precision];
    // NaN drift (a non-finite total) fails the comparison and is caught below too
    if (out->nonfinite > 0 || !std::isfinite(out->mass) || !(out->drift <= out->drift_bound)) return GMF_EUNSTABLE;
    return GMF_OK;
}

int gmf_set_reference(gmf_ctx* ctx, int32_t r, const double* ref)
{
    int rc = check_ctx(ctx);
    if (rc != GMF_OK) return rc;
    if (r < 0 || r >= ctx->nrep) return GMF_EINVAL;
    if (ref) {
        if (!std::isfinite(ref[0]) || !(ref[0] != 0.0) || !std::isfinite(ref[1]) || !std::isfinite(ref[2]) ||
            !std::isfinite(ref[3]))
            return GMF_EINVAL;
        for (int a = 0; a < 4; ++a) ctx->ref[r][a] = ref[a];
        return GMF_OK;
    }
    DeviceGuard g(ctx->device);
    double tot[4];
    rc = device_totals(ctx, r, tot);
    if (rc != GMF_OK) return rc;
    for (int a = 0; a < 4; ++a) ctx->ref[r][a] = tot[a];
    return GMF_OK;
}

int gmf_reset_stats(gmf_ctx* ctx)
{
    int rc = check_ctx(ctx);
    if (rc != GMF_OK) return rc;
    DeviceGuard g(ctx->device);
    CK(hipMemsetAsync(ctx->d_acc(), 0, sizeof(double) * kAccStride * ctx->nrep, ctx->stream));
    if (ctx->L.spectrum) {
        CK(hipMemsetAsync(ctx->d_sacc(), 0, sizeof(double) * kSpec * ctx->L.nshell_total, ctx->stream));
        CK(hipMemsetAsync(ctx->d_sbins(), 0, sizeof(unsigned long long) * kSpec * kBinCopies * ctx->L.nshell_total, ctx->stream));
    }
    CK(hipStreamSynchronize(ctx->stream));
    return GMF_OK;
}

int gmf_spectrum(gmf_ctx* ctx, int32_t r, int32_t max_shells, double* sums, int64_t* counts, int32_t* nshell)
{
    int rc = check_ctx(ctx);
    if (rc != GMF_OK) return rc;
    if (r < 0 || r >= ctx->nrep || max_shells < 0 || !ctx->L.spectrum) return GMF_EINVAL;
    DeviceGuard g(ctx->device);
    const RepDev& R = ctx->rdev[r];
    if (nshell) *nshell = (int32_t)R.nshell;
    const uint32_t ns = std::min<uint32_t>(R.nshell, (uint32_t)max_shells);
    CK(hipStreamSynchronize(ctx->stream));
    if (sums && ns > 0) {
        std::vector<double> rec((size_t)kSpec * R.nshell);
        CK(hipMemcpy(rec.data(), ctx->d_sacc() + (size_t)R.shell_offset * kSpec, sizeof(double) * rec.size(),
                     hipMemcpyDeviceToHost));
        for (int m = 0; m < kSpec; ++m)
            for (uint32_t s2 = 0; s2 < ns; ++s2) sums[(size_t)m * max_shells + s2] = rec[(size_t)s2 * kSpec + m];
    }
    if (counts && ns > 0)
        CK(hipMemcpy(counts, ctx->d_scounts() + R.shell_offset, sizeof(int64_t) * ns, hipMemcpyDeviceToHost));
    return GMF_OK;
}

int gmf_get_populations(gmf_ctx* ctx, int32_t r, double* f)
{
    int rc = check_ctx(ctx);
    if (rc != GMF_OK) return rc;
    if (r < 0 || r >= ctx->nrep || !f) return GMF_EINVAL;
    DeviceGuard g(ctx->device);
    const RepDev& R = ctx->rdev[r];
    const uint64_t plane = (uint64_t)R.nx * R.ny;
    const uint32_t cp = chunk_planes(ctx, r);
    double* st = reinterpret_cast<double*>(ctx->d_stage());
    for (uint32_t z0 = 0; z0 < R.nz; z0 += cp) {
        const uint32_t z1 = std::min(R.nz, z0 + cp);
        const uint64_t cnt = plane * (z1 - z0);
        if (ctx->mom)
            CK(launch_mgather(ctx->opt.precision, ctx->cur_pop(), ctx->d_reps() + r, R, z0, z1, st, ctx->stream));
        else
            CK(launch_gather(ctx->opt.precision, ctx->cur_pop(), ctx->d_reps() + r, R, z0, z1, st, ctx->aa_odd(),
                             ctx->stream));
        CK(hipStreamSynchronize(ctx->stream));
        for (int i = 0; i < Q; ++i)
            CK(hipMemcpy(f + (uint64_t)i * R.n + plane * z0, st + (uint64_t)i * cnt, sizeof(double) * cnt,
                         hipMemcpyDeviceToHost));
    }
    return GMF_OK;
}

int gmf_set_populations(gmf_ctx* ctx, int32_t r, const double* f)
{
    int rc = check_ctx(ctx);
    if (rc != GMF_OK) return rc;
    if (r < 0 || r >= ctx->nrep || !f) return GMF_EINVAL;
    DeviceGuard g(ctx->device);
    const RepDev& R = ctx->rdev[r];
    const uint64_t plane = (uint64_t)R.nx * R.ny;
    const uint32_t cp = chunk_planes(ctx, r);
    double* st = reinterpret_cast<double*>(ctx->d_stage());
    CK(hipStreamSynchronize(ctx->stream));
    for (uint32_t z0 = 0; z0 < R.nz; z0 += cp) {
        const uint32_t z1 = std::min(R.nz, z0 + cp);
        const uint64_t cnt = plane * (z1 - z0);
        for (int i = 0; i < Q; ++i)
            CK(hipMemcpy(st + (uint64_t)i * cnt, f + (uint64_t)i * R.n + plane * z0, sizeof(double) * cnt,
                         hipMemcpyHostToDevice));
        if (ctx->mom)
            CK(launch_mscatter(ctx->opt.precision, ctx->cur_pop(), ctx->d_reps() + r, R, z0, z1, st, ctx->stream));
        else
            CK(launch_scatter(ctx->opt.precision, ctx->cur_pop(), ctx->d_reps() + r, R, z0, z1, st, ctx->aa_odd(),
                              ctx->stream));
        CK(hipStreamSynchronize(ctx->stream));
    }
    // the state as stored (rounded to the device precision) is the new conservation reference
    return gmf_set_reference(ctx, r, nullptr);
}

int gmf_get_nodes(gmf_ctx* ctx, int32_t r, const int64_t* nodes, int32_t count, double* f)
{
    int rc = check_ctx(ctx);
    if (rc != GMF_OK) return rc;
    if (r < 0 || r >= ctx->nrep || count < 0 || (count > 0 && (!nodes || !f))) return GMF_EINVAL;
    const RepDev& R = ctx->rdev[r];
    for (int32_t j = 0; j < count; ++j)
        if (nodes[j] < 0 || (uint64_t)nodes[j] >= R.n) return GMF_EINVAL;
    DeviceGuard g(ctx->device);
    const size_t per = sizeof(int64_t) + sizeof(double) * Q;
    // node list, alignment gap (< kAlign) and outputs must fit the staging area
    const int32_t batch = (int32_t)std::min<size_t>((ctx->L.stage_bytes - kAlign) / per, 1u << 20);
    char* st = ctx->d_stage();
    for (int32_t j0 = 0; j0 < count; j0 += batch) {
        const int32_t c = std::min(batch, count - j0);
        int64_t* dn = reinterpret_cast<int64_t*>(st);
        double* dout = reinterpret_cast<double*>(st + align_up(sizeof(int64_t) * (size_t)c));
        CK(hipStreamSynchronize(ctx->stream));
        CK(hipMemcpy(dn, nodes + j0, sizeof(int64_t) * c, hipMemcpyHostToDevice));
        if (ctx->mom)
            CK(launch_mnodes(ctx->opt.precision, ctx->cur_pop(), ctx->d_reps() + r, dn, c, dout, ctx->stream));
        else
            CK(launch_nodes(ctx->opt.precision, ctx->cur_pop(), ctx->d_reps() + r, dn, c, dout, ctx->aa_odd(),
                            ctx->stream));
        CK(hipStreamSynchronize(ctx->stream));
        CK(hipMemcpy(f + (size_t)j0 * Q, dout, sizeof(double) * Q * c, hipMemcpyDeviceToHost));
    }
    return GMF_OK;
}

int gmf_get_step(gmf_ctx* ctx, int64_t* t)
{
    if (!ctx) return GMF_ESTATE;
    if (!t) return GMF_EINVAL;
    *t = ctx->step;
    return GMF_OK;
}

int gmf_get_config(gmf_ctx* ctx, int32_t* nodes_per_thread, int32_t* block, int32_t* graphs, int32_t* addressing,
                   int32_t* streaming, int32_t* xcd_map)
{
    if (!ctx) return GMF_ESTATE;
    if (xcd_map) {
        // blocks each XCD takes at a time (0: linear mapping)
        const uint32_t c = kXcdChunks[ctx->xcd_map];
        *xcd_map = ctx->xcd_map == 0 ? 0 : (int32_t)(c ? c : (ctx->nblocks + ctx->xcd_count - 1) / ctx->xcd_count);
    }
    if (streaming) *streaming = ctx->aa ? GMF_STREAM_AA : GMF_STREAM_AB;
    if (nodes_per_thread) *nodes_per_thread = ctx->npt;
    if (block) *block = ctx->mom ? mtile_threads(ctx->mtile) : kBlock;
    if (graphs) *graphs = ctx->graph_steps;
    if (addressing) *addressing = ctx->mom ? -1 : ctx->mode;
    return GMF_OK;
}

int gmf_get_occupancy(gmf_ctx* ctx, int32_t* workgroups_per_cu)
{
    if (!ctx) return GMF_ESTATE;
    if (!workgroups_per_cu) return GMF_EINVAL;
    *workgroups_per_cu = ctx->mom ? 0 : (int32_t)ctx->occ;
    return GMF_OK;
}

int gmf_get_tiling(gmf_ctx* ctx, int32_t* storage, int32_t* tile_x, int32_t* tile_y, int32_t* tile_z)
{
    if (!ctx) return GMF_ESTATE;
    if (storage) *storage = ctx->mom ? GMF_STORE_MOMENTS : GMF_STORE_POPULATIONS;
    if (tile_x) *tile_x = ctx->mom ? kMTileX[ctx->mtile] : 0;
    if (tile_y) *tile_y = ctx->mom ? kMTileY[ctx->mtile] : 0;
    if (tile_z) *tile_z = ctx->mom ? (int32_t)ctx->mtz : 0;
    return GMF_OK;
}

int gmf_noise_probe(uint64_t seed, int64_t t, uint32_t node0, int32_t count, int32_t precision, uint32_t* words,
                    double* normals)
{
    if (count < 0 || (precision != GMF_FP64 && precision != GMF_FP32_SHIFTED)) return GMF_EINVAL;
    if (count == 0) return GMF_OK;
    if ((uint64_t)node0 + (uint64_t)count > (1ull << 32)) return GMF_EINVAL;
    hipStream_t s = nullptr;
    uint32_t* dw = nullptr;
    double* dn = nullptr;
    int rc = GMF_OK;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return GMF_EDEVICE;
    if ((words && hipMalloc((void**)&dw, sizeof(uint32_t) * 24 * (size_t)count) != hipSuccess) ||
        (normals && hipMalloc((void**)&dn, sizeof(double) * 23 * (size_t)count) != hipSuccess)) {
        rc = GMF_ENOMEM;
    } else if (launch_noise_probe(precision, seed, t, node0, count, dw, dn, s) != hipSuccess ||
               hipStreamSynchronize(s) != hipSuccess) {
        rc = GMF_EDEVICE;
    } else {
        if (words && hipMemcpy(words, dw, sizeof(uint32_t) * 24 * (size_t)count, hipMemcpyDeviceToHost) != hipSuccess)
            rc = GMF_EDEVICE;
        if (normals && hipMemcpy(normals, dn, sizeof(double) * 23 * (size_t)count, hipMemcpyDeviceToHost) != hipSuccess)
            rc = GMF_EDEVICE;
    }
    if (dw) (void)hipFree(dw);
    if (dn) (void)hipFree(dn);
    (void)hipStreamDestroy(s);
    return rc;
}

}  // extern "C"

namespace {

// Address of the allocation-free probe's device scratch, looked up once per
// device (with that device current) and kept for the life of the process.
constexpr int kMaxProbeDevices = 64;
std::mutex g_probe_mu;
void* g_probe_scratch[kMaxProbeDevices] = {};

int probe_scratch(int dev, char** out)
{
    if (dev < 0 || dev >= kMaxProbeDevices) return GMF_EDEVICE;
    std::lock_guard<std::mutex> lock(g_probe_mu);
    if (!g_probe_scratch[dev]) {
        void* p = nullptr;
        if (probe_scratch_address(&p) != hipSuccess || !p) {
            (void)hipGetLastError();
            return GMF_EDEVICE;
        }
        g_probe_scratch[dev] = p;
    }
    *out = static_cast<char*>(g_probe_scratch[dev]);
    return GMF_OK;
}

}  // namespace

extern "C" {

int gmf_noise_probe_noalloc(uint64_t seed, int64_t t, uint32_t node0, int32_t count, int32_t precision,
                            uint32_t* words, double* normals, void* hip_stream)
{
    if (count < 0 || count > kProbeMaxNodes || (precision != GMF_FP64 && precision != GMF_FP32_SHIFTED))
        return GMF_EINVAL;
    if ((uint64_t)node0 + (uint64_t)count > (1ull << 32)) return GMF_EINVAL;
    if (count == 0 || (!words && !normals)) return GMF_OK;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return GMF_EDEVICE;
    char* base = nullptr;
    const int rc = probe_scratch(dev, &base);
    if (rc != GMF_OK) return rc;
    uint32_t* dw = words ? reinterpret_cast<uint32_t*>(base) : nullptr;
    double* dn = normals ? reinterpret_cast<double*>(base + kProbeNormalsOffset) : nullptr;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (launch_noise_probe(precision, seed, t, node0, count, dw, dn, s) != hipSuccess) return GMF_EDEVICE;
    if (words && hipMemcpyAsync(words, dw, sizeof(uint32_t) * 24 * (size_t)count, hipMemcpyDeviceToHost, s) !=
                     hipSuccess)
        return GMF_EDEVICE;
    if (normals && hipMemcpyAsync(normals, dn, sizeof(double) * 23 * (size_t)count, hipMemcpyDeviceToHost, s) !=
                       hipSuccess)
        return GMF_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return GMF_EDEVICE;
    return GMF_OK;
}

int gmf_copy_probe(const void* src, void* dst, size_t bytes, void* hip_stream)
{
    if (!src || !dst || bytes == 0 || bytes % 16 != 0 || ((uintptr_t)src % 16) != 0 || ((uintptr_t)dst % 16) != 0)
        return GMF_EINVAL;
    if (launch_copy(src, dst, bytes, static_cast<hipStream_t>(hip_stream)) != hipSuccess) return GMF_EDEVICE;
    return GMF_OK;
}

int gmf_read_probe(const void* src, size_t bytes, uint32_t* flag, void* hip_stream)
{
    if (!src || !flag || bytes == 0 || bytes % 16 != 0 || ((uintptr_t)src % 16) != 0 || ((uintptr_t)flag % 4) != 0)
        return GMF_EINVAL;
    if (launch_read_probe(src, bytes, flag, static_cast<hipStream_t>(hip_stream)) != hipSuccess) return GMF_EDEVICE;
    return GMF_OK;
}

void gmf_destroy(gmf_ctx* ctx)
{
    if (!ctx) return;
    DeviceGuard g(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->side) (void)hipStreamSynchronize(ctx->side);
    for (auto& gr : ctx->graphs) (void)hipGraphExecDestroy(gr.second);
    if (ctx->sampler_graph) (void)hipGraphExecDestroy(ctx->sampler_graph);
    if (ctx->own_ws && ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->side_fork) (void)hipEventDestroy(ctx->side_fork);
    if (ctx->side_join) (void)hipEventDestroy(ctx->side_join);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

const char* gmf_strerror(int code)
{
    switch (code) {
    case GMF_OK: return "success";
    case GMF_EINVAL: return "invalid argument";
    case GMF_ENOMEM: return "out of memory";
    case GMF_EDEVICE: return "HIP device error (context poisoned)";
    case GMF_ESTATE: return "invalid context";
    case GMF_EUNSTABLE: return "non-finite density (numerical instability)";
    default: return "unknown error";
    }
}

}  // extern "C"
