/*
 * gmf.h -- C ABI of the MI355X (gfx950) library for the ghost-mode filtered
 * fluctuating lattice Boltzmann method (GMF-FLBM) on the D3Q27 lattice
 * (Lauricella, Montessori, Tiribocchi, Succi, arXiv:2601.03806).
 *
 * The library advances one or more independent periodic boxes ("replicas")
 * with the fused stream+collide update of Sec. II, Eq. (10):
 *
 *   f_i(x + c_i, t + 1) = f^eq_i + (1 - omega) f^neq_i
 *                         + w_i sum_{k=4..9}   e_ki phi_k   r_k / b_k
 *                         + w_i sum_{k=10..26} e_ki phi^g_k r_k / b_k
 *
 * with the second-order equilibrium (Eq. (11)), the filtered non-equilibrium
 * part rebuilt from its second-order Hermite coefficient (Eqs. (12)-(13)),
 * omega = 1/tau (Sec. II), and the noise amplitudes of Eqs. (2) and (9).
 * The BGK-FLBM update of Eq. (1) is available as an option.
 *
 * Conventions (the paper leaves them open; the test oracle uses the same):
 *   - Velocity order i = 0..26 (Table I groups): rest; faces +x,-x,+y,-y,+z,-z;
 *     the 12 edges, then the 8 corners, each in lexicographic order of
 *     (cx, cy, cz) with -1 < 0 < +1.
 *   - Moment order k = 0..26 as printed in Table II.
 *   - Node index n = x + nx*(y + ny*z); host population arrays are FP64,
 *     laid out f[i*N + n] (N = nx*ny*nz) and hold the pre-collision state
 *     f(x, t), i.e. the left-hand side of Eq. (10) after streaming.
 *   - The collision that produces f(., t+1) from f(., t) has step index t.
 *   - The standard normals r_k come from Philox4x32-10 (Salmon et al., SC'11),
 *     key = (seed & 0xffffffff, seed >> 32), counter =
 *     (n, t & 0xffffffff, j, t >> 32) for blocks j = 0..5; block j feeds
 *     r_{4+4j} .. r_{7+4j} through the Box-Muller transform on the word pairs
 *     (x0, x1) and (x2, x3): radius sqrt(-2 ln U1), angle 2 pi U2.  FP64 uses
 *     U = (x + 1/2) 2^-32; FP32 uses U = ((x >> 9) + 1/2) 2^-23 (exact in binary32).
 *   - Initial state: rest equilibrium f_i = w_i rho0 in every replica.
 *
 * Threading and synchronisation: a context is not thread-safe; distinct
 * contexts are independent.  gmf_step only enqueues work on the context's
 * stream; every other call that returns data synchronises that stream.
 * No C++ exception crosses this interface; every function returns one of the
 * GMF_* codes below.  After a HIP error a context is poisoned: every later
 * call on it returns GMF_EDEVICE.
 *
 * Environment variables, read by gmf_init (none changes a trajectory's bits):
 *   GMF_TUNE_CACHE   file that caches the autotuner's choices (tune = 1),
 *                    one line per box set and options; appended to
 *   GMF_ADDRESSING   plane | 27 | 3 | 1: force the population addressing mode
 *                    (ignored where it does not fit the boxes)
 *   GMF_BLOCK_MAP    linear | xcd | xcd16: force the workgroup-to-XCD mapping
 *   GMF_MTILE        "tile,depth": force the moment-storage tiling (tile 0..3
 *                    = 64x8, 32x16, 32x8, 64x16; depth >= 16 planes)
 *   GMF_OCCUPANCY    0 | 5 | 4 | 3: force the occupancy cap of the population
 *                    step (workgroups per CU; 0: none)
 *   GMF_DEBUG        print each failing HIP call to stderr
 * The autotuner (tune = 1) overrides the forced choices it searches.
 */
#ifndef GMF_H
#define GMF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GMF_ABI_VERSION 2

/* return codes */
#define GMF_OK 0
#define GMF_EINVAL (-1)     /* an argument is out of range (see each call)  */
#define GMF_ENOMEM (-2)     /* device or host allocation failed             */
#define GMF_EDEVICE (-3)    /* a HIP call failed; the context is poisoned   */
#define GMF_ESTATE (-4)     /* NULL context                                 */
#define GMF_EUNSTABLE (-5)  /* a sampled density was NaN or infinite, or mass
                               and momentum drifted past the bound (gmf_stats) */

/* gmf_options.precision */
#define GMF_FP64 0          /* populations f stored and stepped in FP64     */
#define GMF_FP32_SHIFTED 1  /* g = f - w rho0 stored and stepped in FP32    */
/* gmf_options.collision */
#define GMF_COLLISION_GMF 0 /* Eq. (10): ghost-mode filtered               */
#define GMF_COLLISION_BGK 1 /* Eq. (1): BGK-FLBM, noise on k = 4..26 with omega(2-omega) */
/* gmf_options.streaming: how the populations move between steps.  Both
 * patterns give bit-identical trajectories; they differ in memory and speed. */
#define GMF_STREAM_AUTO 0   /* A/B; with tune = 1 the faster of A/B and AA   */
#define GMF_STREAM_AB 1     /* two population buffers, pull from one into the other */
#define GMF_STREAM_AA 2     /* one buffer updated in place (even steps pull from the
                               neighbours and write back where they read, odd steps
                               read and write the node's own values): half the
                               population memory */
/* gmf_options.storage: what the lattice keeps between steps. */
#define GMF_STORE_POPULATIONS 0 /* the 27 populations of every node            */
#define GMF_STORE_MOMENTS 1 /* the thread-safe formulation of Sec. II: the ten
                               hydrodynamic moments of f(x, t) (Eqs. (3), (4),
                               (13)), from which every node rebuilds the
                               post-collision populations of its neighbours
                               (their noise drawn again from the same Philox
                               counters) and sums its new moments; 10 values
                               read and written per node instead of 27.  GMF
                               collision only (Eq. (10) keeps no ghost content,
                               so the moments are the whole state that matters),
                               two moment buffers (streaming AUTO or AB).  The
                               populations that gmf_get_populations and
                               gmf_get_nodes return are then the second-order
                               Hermite populations of the stored moments, and
                               gmf_set_populations keeps the moments of f. */

/* observables accumulated by the sampler (index into gmf_stats_t arrays) */
#define GMF_NOBS 10
#define GMF_OBS_DRHO 0      /* rho - rho0, rho of Eq. (3)                   */
#define GMF_OBS_JX 1        /* rho u_x, Eq. (4)                             */
#define GMF_OBS_JY 2
#define GMF_OBS_JZ 3
#define GMF_OBS_JSUM 4      /* sum_a rho u_a                                */
#define GMF_OBS_PDIAG 5     /* sum_a (Pi_aa - rho0 cs^2), Pi = sum_i f_i c_i c_i */
#define GMF_OBS_POFF 6      /* sum_{a<b} Pi_ab                              */
#define GMF_OBS_UX 7        /* u_x = j_x / rho                              */
#define GMF_OBS_UY 8
#define GMF_OBS_UZ 9
/* shell spectra S_m(|k|) (Results section), normalised DFT
 * m(k) = N^-1/2 sum_x m(x) exp(-i k.x), k_a = 2 pi n_a / L_a, averaged over all
 * integer vectors n of the shell |n|^2 = 1,2,3,4,5,6,8,9 */
#define GMF_NSPEC 5
#define GMF_SPEC_RHO 0
#define GMF_SPEC_J 1        /* mean over the three components of j          */
#define GMF_SPEC_JSUM 2
#define GMF_SPEC_PDIAG 3
#define GMF_SPEC_POFF 4
#define GMF_NSHELL 8

typedef struct gmf_ctx gmf_ctx;   /* opaque, owned by the library */

/* One periodic box.  Lattice size and periodic box, rho0 ("rho = 1" in the
 * Results section), tau = 1/omega (Sec. II), k_B T (Eqs. (2), (9)), seed of
 * the noise stream. */
typedef struct {
    int32_t nx, ny, nz;   /* >= 1 each; nx*ny*nz < 2^31                     */
    int32_t reserved;     /* must be 0                                      */
    double rho0;          /* > 0                                            */
    double tau;           /* > 0.5                                          */
    double kbt;           /* >= 0; 0 switches the noise off                 */
    uint64_t seed;        /* Philox key                                     */
} gmf_replica;

typedef struct {
    int32_t precision;    /* GMF_FP64 or GMF_FP32_SHIFTED                   */
    int32_t collision;    /* GMF_COLLISION_GMF or GMF_COLLISION_BGK         */
    int32_t noise_rho;    /* 0: local rho in Eqs. (2)/(9); 1: rho0         */
    int32_t sample_every; /* > 0: sample f(., t) at every step with t % sample_every == 0; 0: off */
    int32_t graph_steps;  /* longest run of steps captured in one HIP graph; 0: direct
                             launches; < 0: the default (64).  A graph holds one
                             sampling step or up to graph_steps non-sampling steps
                             (between two samples closer than that, the run from one
                             sample to the next); steps that fit no graph (the tail
                             of a gmf_step call) are launched directly.  With moment
                             storage a sampling step's sampling kernels are a graph
                             of their own on the library's second stream (gmf_step).
                             Graphs are captured on first use or by gmf_prepare;
                             every choice gives the same bits. */
    int32_t tune;         /* 0: built-in kernel configuration; 1: time the variants at init */
    int32_t streaming;    /* GMF_STREAM_AUTO, GMF_STREAM_AB or GMF_STREAM_AA */
    int32_t spectrum;     /* 1: also accumulate the full-box shell spectra on every
                             sampling step (needs sample_every > 0 and box lengths
                             whose prime factors are 2, 3, 5, at most 1024 each;
                             see gmf_spectrum); 0: off */
    int32_t storage;      /* GMF_STORE_POPULATIONS or GMF_STORE_MOMENTS      */
} gmf_options;

typedef struct {
    int64_t step;                           /* current step index t         */
    int64_t nsamples;                       /* samples accumulated          */
    int64_t nonfinite;                      /* non-finite densities seen    */
    double mass;                            /* sum_x rho(x, t), FP64        */
    double momentum[3];                     /* sum_x rho u(x, t), FP64      */
    double sum_mean[GMF_NOBS];              /* sum over samples of the spatial mean          */
    double sum_meansq[GMF_NOBS];            /* sum over samples of the spatial mean of o^2   */
    double sum_var[GMF_NOBS];               /* sum over samples of the spatial variance      */
    double spectrum[GMF_NSPEC][GMF_NSHELL]; /* sum over samples of the shell average |m(k)|^2 */
    int32_t shell_n2[GMF_NSHELL];           /* |n|^2 of each shell          */
    int32_t shell_count[GMF_NSHELL];        /* integer vectors per shell    */
    /* conservation guard (mass and momentum are invariants of Eqs. (1)/(10):
     * the conserved modes k = 0..3 are neither relaxed nor noised) */
    double mass_ref;                        /* reference mass (gmf_set_reference) */
    double momentum_ref[3];                 /* reference momentum           */
    double drift;                           /* max(|mass - mass_ref|, max_a |momentum_a -
                                               momentum_ref_a|) / |mass_ref|  */
    double drift_bound;                     /* 1e-10 (FP64), 1e-4 (FP32 shifted): above it
                                               gmf_stats returns GMF_EUNSTABLE */
} gmf_stats_t;

/* Device bytes gmf_init needs when the caller provides the workspace.
 * Returns 0 when the arguments are invalid.  Size limits (each one an
 * argument error):
 *   1 <= nrep <= 65535; fewer than 2^32 nodes over all replicas;
 *   per replica nx*ny*nz < 2^31 and one z plane of 27 populations
 *   (nx*ny*27*element bytes) under 4 GiB;
 *   some addressing mode of the step kernel fits every replica: either a
 *   storage group of 27, 3 or 1 populations over the whole replica within
 *   32-bit byte offsets (at the least nx*ny*nz*element bytes < 4 GiB), or
 *   every z plane a whole number of 256-node workgroups;
 *   with sampling: 6 * 28 * nz * ceil(nx / 64) summed over the replicas
 *   (the partial sums of the first DFT stage, per plane and block of 64
 *   columns; one block for nx < 64) below 2^32;
 *   with full-box spectra: nx, ny, nz <= 1024 with prime factors 2, 3, 5. */
size_t gmf_workspace_bytes(const gmf_replica* reps, int32_t nrep, const gmf_options* opt);

/* Create a context for nrep replicas and set each to rest equilibrium.
 *   reps, opt       host pointers, read during the call only (opt may be NULL
 *                   for the defaults: FP64, GMF, local rho, no sampling).
 *   dev_workspace   device pointer of at least ws_bytes >= gmf_workspace_bytes
 *                   bytes, caller-owned, must outlive the context; NULL lets
 *                   the library allocate (and free at gmf_destroy).
 *   hip_stream      hipStream_t to enqueue on (caller-owned, must outlive the
 *                   context and must not be the legacy NULL stream when
 *                   graph_steps != 0); NULL: the library creates its own.
 * Errors: GMF_EINVAL for any out-of-range field (including a workspace that is
 * too small or misaligned to 256 bytes), GMF_ENOMEM, GMF_EDEVICE. */
int gmf_init(const gmf_replica* reps, int32_t nrep, const gmf_options* opt,
             void* dev_workspace, size_t ws_bytes, void* hip_stream, gmf_ctx** out);

/* Enqueue n >= 0 steps of Eq. (10) (or Eq. (1)) on every replica.  Asynchronous.
 * Everything is ordered on the context's stream when the call returns.  With
 * moment storage the sampling kernels of each sampling step run on a second
 * stream of the library's own, which waits for the step and which the
 * context's stream waits for before the next sampling step and before this
 * call returns; the results are the same bits as on one stream. */
int gmf_step(gmf_ctx* ctx, int64_t n);

/* Capture (without running anything) every HIP graph that gmf_step(ctx, n)
 * from the current step would launch, so that the following gmf_step calls
 * capture nothing: for timed regions and latency-bound loops.  n >= 0; a no-op
 * with graph_steps = 0.  Capturing uses the context's stream; the graphs stay
 * valid until gmf_destroy. */
int gmf_prepare(gmf_ctx* ctx, int64_t n);

/* What the step loop has launched since gmf_init: graph replays, the steps
 * they covered, steps launched directly, and graphs captured so far.  Any
 * output pointer may be NULL. */
int gmf_get_launch_counts(gmf_ctx* ctx, int64_t* graph_launches, int64_t* graph_steps, int64_t* direct_steps,
                          int32_t* graphs_captured);

/* Density rho (N values) and velocity u = j/rho (3N values, ux | uy | uz) of
 * the current state of replica r, Eqs. (3)-(4), into caller-owned host
 * buffers (either may be NULL).  Synchronises. */
int gmf_moments(gmf_ctx* ctx, int32_t r, double* rho, double* u);

/* Statistics of replica r: current FP64 mass and momentum, and the sums of the
 * sampled observables (see gmf_stats_t).  Synchronises.  Returns
 * GMF_EUNSTABLE (after filling *out) when a sampled density was not finite,
 * the mass is not finite, or drift exceeds drift_bound. */
int gmf_stats(gmf_ctx* ctx, int32_t r, gmf_stats_t* out);

/* Conservation reference of replica r that gmf_stats measures drift from.
 * gmf_init takes the rest state's mass and momentum and gmf_set_populations
 * the new state's, both as stored on the device.  ref = NULL: take the
 * current state's (synchronises); else ref[0] = mass (finite, nonzero),
 * ref[1..3] = momentum (finite), host array read during the call, e.g. the
 * reference of the run a checkpoint was taken from, so that drift keeps
 * counting across a resume.  GMF_EINVAL for r out of range or a bad ref. */
int gmf_set_reference(gmf_ctx* ctx, int32_t r, const double* ref);

/* Zero the sample accumulators of every replica (the full-box spectra too). */
int gmf_reset_stats(gmf_ctx* ctx);

/* Full-box shell spectra of replica r (Results section: structure factors
 * from a normalised FFT of the whole box, averaged over shells of equal |k|).
 * Needs options.spectrum = 1.  Shell s >= 1 holds the integer wave vectors n
 * (k_a = 2 pi n_a / L_a, n_a in [-L_a/2, L_a/2)) with s - 1/2 <= |n| < s + 1/2;
 * shell 0 (k = 0) stays empty.  On return:
 *   sums[m * max_shells + s]  sum over the samples of the average of |m(k)|^2
 *                             over shell s, m = GMF_SPEC_* (the same fields and
 *                             normalisation as gmf_stats_t.spectrum);
 *   counts[s]                 wave vectors in shell s;
 *   *nshell                   shells of this replica (round(|n_max|) + 1).
 * At most max_shells shells are written; any output pointer may be NULL
 * (host memory, caller-owned).  The shell sums are exact integer sums of
 * fixed-point terms, so a run reproduces its spectra bit for bit.
 * Synchronises.  GMF_EINVAL if the option is off or r is out of range. */
int gmf_spectrum(gmf_ctx* ctx, int32_t r, int32_t max_shells, double* sums, int64_t* counts, int32_t* nshell);

/* Canonical populations f(x, t) of replica r (27*N FP64 values, host). */
int gmf_get_populations(gmf_ctx* ctx, int32_t r, double* f);
/* Overwrite the state of replica r with f(x, t) (27*N FP64 values, host), and
 * take its mass and momentum as the new conservation reference. */
int gmf_set_populations(gmf_ctx* ctx, int32_t r, const double* f);
/* Canonical populations at `count` listed nodes (node indices 0 <= n < N, host
 * array) of replica r into f[27*j + i] (host).  Synchronises. */
int gmf_get_nodes(gmf_ctx* ctx, int32_t r, const int64_t* nodes, int32_t count, double* f);

/* Current step index t. */
int gmf_get_step(gmf_ctx* ctx, int64_t* t);

/* Run the device noise generator that the step kernels use for `count`
 * consecutive nodes node0.. at step t: words[24*j + 4*b + q] is word q of
 * Philox block b for node node0+j; normals[23*j + (k-4)] is r_k, k = 4..26.
 * precision selects the FP64 or FP32 normal transform (FP32 results are
 * widened to double).  Host output arrays; either may be NULL.  Uses a
 * private stream and synchronises. */
int gmf_noise_probe(uint64_t seed, int64_t t, uint32_t node0, int32_t count, int32_t precision,
                    uint32_t* words, double* normals);

/* gmf_noise_probe without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, latency-bound loops, harnesses that
 * forbid hipMalloc).  Same outputs as gmf_noise_probe, bit for bit, staged in a
 * fixed device array that the library holds on every device it runs on until
 * the process ends (4.4 MiB per device; its address is looked up on the first
 * call on each device).  The kernel and the copies to the host arrays run on
 * hip_stream (NULL: the legacy stream), which is synchronised before return.
 *   count  0 <= count <= GMF_PROBE_MAX_NODES, else GMF_EINVAL (nothing runs).
 * Every call on one device shares that device's array: calls that overlap in
 * time on one device (other threads or streams) race and must be serialised
 * by the caller.  Nothing in the array needs clearing: each call writes every
 * value it copies out. */
#define GMF_PROBE_MAX_NODES 16384
int gmf_noise_probe_noalloc(uint64_t seed, int64_t t, uint32_t node0, int32_t count, int32_t precision,
                            uint32_t* words, double* normals, void* hip_stream);

/* Kernel configuration in use (for reports): nodes per thread, threads per
 * workgroup, steps per captured HIP graph (0: direct launches), the
 * addressing mode of the step kernel (0: plane-uniform rows of 27 populations;
 * 27, 3, 1: per-node addressing with storage groups of that many populations;
 * -1 with moment storage), the streaming pattern (GMF_STREAM_AB or
 * GMF_STREAM_AA; moment storage alternates two buffers like GMF_STREAM_AB), and
 * the workgroup mapping (0: workgroup b updates lattice block b, so consecutive
 * blocks go to different XCDs; C > 0: each XCD updates runs of C consecutive
 * blocks, of 256 or 512 nodes, or tiles with moment storage).  Any output
 * pointer may be NULL. */
int gmf_get_config(gmf_ctx* ctx, int32_t* nodes_per_thread, int32_t* block, int32_t* graphs, int32_t* addressing,
                   int32_t* streaming, int32_t* xcd_map);
/* Storage kind in use (GMF_STORE_*) and, for moment storage, the tile of one
 * workgroup of the step kernel: tile_x x tile_y nodes (plus a one-node halo)
 * marched over tile_z z planes (0, 0, 0 for population storage).  Any output
 * pointer may be NULL. */
int gmf_get_tiling(gmf_ctx* ctx, int32_t* storage, int32_t* tile_x, int32_t* tile_y, int32_t* tile_z);
/* Occupancy cap of the population step kernel: at most *workgroups_per_cu
 * workgroups of it run on one compute unit at a time (5, 4 or 3), or 0 for no
 * cap (also with moment storage).  The autotuner (tune = 1) times the caps
 * for the variant it chose: fewer concurrent workgroups can stream HBM
 * faster.  GMF_EINVAL if the pointer is NULL. */
int gmf_get_occupancy(gmf_ctx* ctx, int32_t* workgroups_per_cu);

/* Bandwidth reference: enqueue one plain streaming copy of `bytes` (a positive
 * multiple of 16) from device buffer src to device buffer dst (both 16-byte
 * aligned, caller-owned, not overlapping) on hip_stream (NULL: the legacy
 * stream).  Asynchronous.  The measured rate of this copy is the practical HBM
 * ceiling that the step kernel's bandwidth is compared with. */
int gmf_copy_probe(const void* src, void* dst, size_t bytes, void* hip_stream);

/* Read-bandwidth reference: enqueue one plain read of `bytes` (a positive
 * multiple of 16) from device buffer src (16-byte aligned, caller-owned) on
 * hip_stream (NULL: the legacy stream).  Asynchronous.  flag is one device
 * uint32_t (4-byte aligned, caller-owned, not cleared here) that is set to 1
 * if a value read is not finite, which keeps every load live.  Timed right
 * after a kernel has written the same buffer, this is the ceiling of the
 * spectrum passes, each of which reads what the pass before it wrote.
 * GMF_EINVAL on a NULL pointer, a misaligned pointer or a bad size. */
int gmf_read_probe(const void* src, size_t bytes, uint32_t* flag, void* hip_stream);

/* Release the context and everything the library allocated for it. */
void gmf_destroy(gmf_ctx* ctx);

/* Static description of a return code. */
const char* gmf_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* GMF_H */
