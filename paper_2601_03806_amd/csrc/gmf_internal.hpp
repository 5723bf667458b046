// gmf_internal.hpp -- interface between the host runtime (gmf_runtime.cpp) and
// the kernels (gmf_kernels.hip).  Not installed, not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gmf_device.hpp"

namespace gmf {

enum Precision { kFP64 = 0, kFP32Shifted = 1 };
enum Collision { kGMF = 0, kBGK = 1 };

// accumulator record of one replica (doubles)
constexpr int kAccNsamp = 0;
constexpr int kAccNonfinite = 1;
constexpr int kAccMean = 2;
constexpr int kAccMeanSq = kAccMean + kObs;
constexpr int kAccVar = kAccMeanSq + kObs;
constexpr int kAccSpec = kAccVar + kObs;
static_assert(kAccSpec + kSpec * kShells <= kAccStride, "accumulator record too small");

struct StepArgs {
    const void* src;              // population buffer read at this step
    void* dst;                    // population buffer written at this step
    const RepDev* reps;
    const uint16_t* blk2rep;      // workgroup -> replica (NULL when nrep == 1)
    const int64_t* d_step;        // device step counter (NULL: step_base is the step)
    int64_t step_base;            // step = step_base + (d_step ? *d_step : 0)
    void* fields;                 // sampled fields (SAMPLE variants)
    double* partials;             // sampling steps: one record of kPartialStride doubles per lattice
                                  // block (FP64 sums of the observables of its nodes)
    uint32_t nblocks;             // lattice blocks (set by launch_step)
    uint32_t xcd;                 // 0: workgroup b takes lattice block b; else the number of XCDs,
                                  // each taking runs of `chunk` consecutive blocks
    uint32_t chunk;               // blocks per run (0: one contiguous range per XCD)
    uint32_t tz;                  // moment storage: z planes per tile
    uint32_t occ;                 // population step: at most occ workgroups per CU (0: no cap);
                                  // a launch parameter only (see occ_lds_bytes)
};

// Occupancy caps of the population step kernel that the autotuner tries: at
// most k workgroups per CU, k in kOccCap (0: no cap).  The kernel uses no LDS;
// a cap is enforced by reserving LDS at launch, midway between what k + 1 and
// k workgroups fill of the 160 KiB of a gfx950 CU (always under the 64 KiB a
// workgroup may take).
constexpr int kOccCaps = 4;
constexpr uint32_t kOccCap[kOccCaps] = {0u, 5u, 4u, 3u};
constexpr uint32_t occ_lds_bytes(uint32_t k)
{
    return k == 0 ? 0u : ((160u * 1024u / (k + 1u) + 160u * 1024u / k) / 2u) / 256u * 256u;
}
static_assert(occ_lds_bytes(3) < 64u * 1024u && occ_lds_bytes(3) * 3u <= 160u * 1024u &&
                  occ_lds_bytes(3) * 4u > 160u * 1024u,
              "three workgroups per CU");
static_assert(occ_lds_bytes(5) * 5u <= 160u * 1024u && occ_lds_bytes(5) * 6u > 160u * 1024u, "five workgroups per CU");

// Moment storage (gmf_mstep.hip): the state is kMom fields of N values per
// replica, the raw moments of g = f - w rho0 of the pre-collision state:
//   0: rho - rho0, 1-3: j_x, j_y, j_z, 4-6: Pi_aa - rho0 cs2 (a = x, y, z),
//   7: Pi_xy, 8: Pi_xz, 9: Pi_yz.
constexpr int kMom = 10;
// tile shapes (x, y) of the moment-storage step kernel and threads per
// workgroup: one per column of the tile plus its one-node halo rounded up to
// whole wavefronts, at most 1024 (larger haloed tiles take two rounds of
// columns per thread)
constexpr int kMTiles = 4;
constexpr int kMTileX[kMTiles] = {64, 32, 32, 64};
constexpr int kMTileY[kMTiles] = {8, 16, 8, 16};
// LDS of one workgroup (the 27 post-collision populations of the haloed tile)
// and whether it fits the 160 KiB of a gfx950 CU, for values of es bytes
constexpr size_t mtile_lds_bytes(int t, size_t es) { return (size_t)Q * (kMTileX[t] + 2) * (kMTileY[t] + 2) * es; }
constexpr bool mtile_fits(int t, size_t es) { return mtile_lds_bytes(t, es) <= 160u * 1024u; }
constexpr int mtile_threads(int t)
{
    return ((kMTileX[t] + 2) * (kMTileY[t] + 2) + 63) / 64 * 64 > 1024 ? 1024
                                                                      : ((kMTileX[t] + 2) * (kMTileY[t] + 2) + 63) / 64 * 64;
}

// lattice kernels
// sm: streaming pattern kAB, kAAPull or kAALocal (gmf_device.hpp); the AA
// patterns need a.src == a.dst.
// grp: addressing mode shared by every replica of the context: 0 (plane-uniform,
// storage groups of 27) or the storage group size 27, 3 or 1 (per-node addressing)
// a.xcd > 0: the grid is rounded up to whole chunks on every XCD (see step_kernel)
// a.occ > 0: at most a.occ workgroups per CU (occ_lds_bytes)
hipError_t launch_step(int precision, int collision, bool sample, int sm, int grp, int npt, const StepArgs& a,
                       uint32_t nblocks, hipStream_t s);
hipError_t launch_init(int precision, void* buf, const RepDev* rep_dev, const RepDev& rep, hipStream_t s);
// FP64 partial records of the observables from the sampled fields: one per workgroup of kObsNodes
// nodes (RepDev::obs_first, obs_blocks; first: nrep + 1 prefix sums, nblocks their total)
hipError_t launch_observables(int precision, const RepDev* reps, int32_t nrep, const uint32_t* first,
                              uint32_t nblocks, const void* fields, double* partials, hipStream_t s);
// Those records summed in two fixed-order stages: slices of kBlock records (RepDev::slice_first;
// max_slices the most slices of a replica), then one workgroup per replica updating its accumulators.
// sample_sq (nullable): nrep * kObs sums over the box of each observable squared, for this sample
hipError_t launch_stats_reduce(const RepDev* reps, int32_t nrep, uint32_t max_slices, const double* partials,
                               double* slices, double* acc, double* sample_sq, hipStream_t s);
hipError_t launch_twiddles(const RepDev* reps, int32_t nrep, double2* tw, hipStream_t s);
// dft: per replica kFields * nz * dft_col_blocks(nx) * kDftPlane complex; zbuf: nrep * kFields * 196
// complex; first: nrep + 1 prefix sums of the replicas' first-stage workgroups (dft_chunks), nchunks their total;
// partials: the FP32 path's first stage also writes the observables record of each chunk there
hipError_t launch_dft(int precision, const RepDev* reps, int32_t nrep, const uint32_t* first, uint32_t nchunks,
                      const void* fields, const double2* tw, double2* dft, double2* zbuf, double* acc,
                      double* partials, hipStream_t s);
// full-box shell spectra of one sample (gmf_fft.hip): first = 3 prefix arrays of
// nrep + 1 workgroup counts (passes x, y and z with the shell sums), nblk their
// totals, lds the dynamic LDS bytes of each of the three kernels; spec holds the
// seven half spectra of every replica in the kernel precision (RepDev::spec_offset);
// bins: kBinCopies copies, bin_stride = kSpec * (shells of all replicas) values apart;
// max_nshell: the most shells of one replica;
// classes[a]: bit c set when a replica's lines along axis a are of kernel class c
// (fft_class: log2 of a power-of-two length 64 .. 1024, else 0);
// order 0 runs the passes one after the other over all fields, order 1 group by
// group (x pass of a field pair, then y and z passes of its half spectra)
hipError_t launch_spectrum(int precision, const RepDev* reps, int32_t nrep, const uint32_t* first, const uint32_t* nblk,
                           const void* fields, const double2* tw, void* spec, const double* sample_sq,
                           const int64_t* counts, unsigned long long* bins, uint32_t bin_stride, double* sacc,
                           uint32_t max_nshell, const size_t* lds, const uint32_t* classes, int order,
                           hipStream_t s);
hipError_t launch_set_step(int64_t* d_step, int64_t value, hipStream_t s);
hipError_t launch_advance_step(int64_t* d_step, int64_t by, hipStream_t s);

// host-interface helpers (chunks of z planes of one replica); aa_odd: the buffer
// holds the state after an odd number of AA steps (see canon_index)
hipError_t launch_gather(int precision, const void* src, const RepDev* rep_dev, const RepDev& rep,
                         uint32_t z0, uint32_t z1, double* out, int aa_odd, hipStream_t s);
hipError_t launch_scatter(int precision, void* dst, const RepDev* rep_dev, const RepDev& rep,
                          uint32_t z0, uint32_t z1, const double* in, int aa_odd, hipStream_t s);
hipError_t launch_moments(int precision, const void* src, const RepDev* rep_dev, const RepDev& rep,
                          uint32_t z0, uint32_t z1, double* rho, double* u, double* partials,
                          int aa_odd, hipStream_t s);
hipError_t launch_sum_partials(const double* partials, uint32_t nblocks, double* out4, int accumulate,
                               hipStream_t s);
hipError_t launch_nodes(int precision, const void* src, const RepDev* rep_dev, const int64_t* nodes,
                        int32_t count, double* out, int aa_odd, hipStream_t s);
hipError_t launch_noise_probe(int precision, uint64_t seed, int64_t t, uint32_t node0, int32_t count,
                              uint32_t* words, double* normals, hipStream_t s);
// Fixed device scratch of the allocation-free noise probe (gmf_kernels.hip):
// the words (24 per node) from offset 0 and the normals (23 doubles per node)
// from kProbeNormalsOffset, for at most kProbeMaxNodes nodes per call.
constexpr int32_t kProbeMaxNodes = 16384;
constexpr size_t kProbeNormalsOffset = ((size_t)kProbeMaxNodes * 24 * sizeof(uint32_t) + 255) / 256 * 256;
constexpr size_t kProbeScratchBytes = kProbeNormalsOffset + (size_t)kProbeMaxNodes * 23 * sizeof(double);
// Device address of that scratch on the current device (each device holds its
// own copy of the array at its own address).
hipError_t probe_scratch_address(void** out);

// moment storage: one step (tile: index into kMTileX/Y; a.tz planes per tile;
// nblocks tiles in all, RepDev::block_begin/nblocks per replica), the rest state
// (zeros), and the host-interface helpers in the same conventions as the
// population ones above (populations are the second-order Hermite
// populations of the stored moments)
hipError_t launch_mstep(int precision, bool sample, int tile, const StepArgs& a, uint32_t nblocks, hipStream_t s);
hipError_t launch_mgather(int precision, const void* src, const RepDev* rep_dev, const RepDev& rep,
                          uint32_t z0, uint32_t z1, double* out, hipStream_t s);
hipError_t launch_mscatter(int precision, void* dst, const RepDev* rep_dev, const RepDev& rep,
                           uint32_t z0, uint32_t z1, const double* in, hipStream_t s);
hipError_t launch_mmoments(int precision, const void* src, const RepDev* rep_dev, const RepDev& rep,
                           uint32_t z0, uint32_t z1, double* rho, double* u, double* partials, hipStream_t s);
hipError_t launch_mnodes(int precision, const void* src, const RepDev* rep_dev, const int64_t* nodes,
                         int32_t count, double* out, hipStream_t s);

hipError_t launch_copy(const void* src, void* dst, uint64_t bytes, hipStream_t s);

// canonical velocity order of the interface -> internal tensor order
void canonical_to_tensor(int out[Q]);

}  // namespace gmf
