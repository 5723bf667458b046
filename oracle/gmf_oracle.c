/*
 * gmf_oracle.c -- FP64 CPU oracle for the ghost-mode filtered fluctuating
 * lattice Boltzmann method (GMF-FLBM) on the D3Q27 lattice
 * (Lauricella, Montessori, Tiribocchi, Succi, arXiv:2601.03806).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, literal reading of
 * the paper that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark load it.  It shares
 * no code, header, table or constant with the HIP library: every table below
 * is written out from the paper's Table I and Table II.
 *
 * Arithmetic is IEEE double, built with -O2 -ffp-contract=off (no FMA
 * contraction), so each expression rounds exactly as written.
 *
 * Conventions the paper leaves open (the GPU library takes the same ones):
 *   - velocity order inside each Table I group: rest; the six faces
 *     (+x,-x,+y,-y,+z,-z); the twelve edges and then the eight corners, each in
 *     lexicographic order of (cx,cy,cz) with -1 < 0 < +1;
 *   - moment order k = 0..26 exactly as printed in Table II;
 *   - periodic box, node index n = x + nx*(y + ny*z), populations stored
 *     f[i*N + n] and holding the pre-collision state f(x,t) (left-hand side of
 *     Eq. (10) after streaming);
 *   - the collision that maps f(.,t) to f(.,t+1) has step index t;
 *   - the standard normals r_k of Eqs. (1) and (10) come from Philox4x32-10
 *     (Salmon et al., SC'11) keyed by the seed, with counter
 *     (node, step_lo32, block, step_hi32), block j = 0..5 giving r_{4+4j..7+4j}
 *     through the Box-Muller transform; the 24th normal (k = 27) is unused;
 *   - the density in the noise amplitudes of Eqs. (2) and (9) is the local
 *     density rho of Eq. (3) unless noise_rho = 1, which uses rho0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 27

/* Sec. II: c_s^2 = 1/3 in lattice units. */
static const double CS2 = 1.0 / 3.0;

/* ----------------------------------------------------------------------- */
/* Table I: D3Q27 velocities and weights.                                   */
/* ----------------------------------------------------------------------- */
static const int VEL[Q][3] = {
    {0, 0, 0},
    /* faces, |c|^2 = 1 */
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    /* edges, |c|^2 = 2, lexicographic */
    {-1, -1, 0}, {-1, 0, -1}, {-1, 0, 1}, {-1, 1, 0},
    {0, -1, -1}, {0, -1, 1}, {0, 1, -1}, {0, 1, 1},
    {1, -1, 0}, {1, 0, -1}, {1, 0, 1}, {1, 1, 0},
    /* corners, |c|^2 = 3, lexicographic */
    {-1, -1, -1}, {-1, -1, 1}, {-1, 1, -1}, {-1, 1, 1},
    {1, -1, -1}, {1, -1, 1}, {1, 1, -1}, {1, 1, 1},
};

static double weight_of(int i)
{
    int c2 = VEL[i][0] * VEL[i][0] + VEL[i][1] * VEL[i][1] + VEL[i][2] * VEL[i][2];
    switch (c2) {
    case 0: return 8.0 / 27.0;
    case 1: return 2.0 / 27.0;
    case 2: return 1.0 / 54.0;
    default: return 1.0 / 216.0;
    }
}

/* ----------------------------------------------------------------------- */
/* Table II: the 27 full-Hermite basis vectors e_ki, order n_k,             */
/* multiplicity mu_k and norm b_k = n_k! c_s^(2 n_k) / mu_k.               */
/* Each vector is written from the printed formula of its group with the    */
/* Cartesian indices of its Hermite symbol substituted.                     */
/* ----------------------------------------------------------------------- */
static const int NK[Q] = {0, 1, 1, 1, 2, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3,
                          4, 4, 4, 4, 4, 4, 5, 5, 5, 6};
static const int MUK[Q] = {1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 3, 3, 3, 3, 3, 3, 6,
                           6, 6, 6, 12, 12, 12, 30, 30, 30, 90};

enum { X = 0, Y = 1, Z = 2 };

static double herm3_a2b(const int *c, int a, int b)
{   /* c_a^2 c_b - c_s^2 c_b  (Table II, k = 10..15) */
    return (double)(c[a] * c[a] * c[b]) - CS2 * c[b];
}

static double herm4_a2b2(const int *c, int a, int b)
{   /* c_a^2 c_b^2 - c_s^2 (c_a^2 + c_b^2) + c_s^4  (Table II, k = 17..19) */
    return (double)(c[a] * c[a] * c[b] * c[b]) - CS2 * (double)(c[a] * c[a] + c[b] * c[b]) + CS2 * CS2;
}

static double herm4_abg2(const int *c, int a, int b, int g)
{   /* c_a c_b c_g^2 - c_s^2 c_a c_b  (Table II, k = 20..22) */
    return (double)(c[a] * c[b] * c[g] * c[g]) - CS2 * (double)(c[a] * c[b]);
}

static double herm5(const int *c, int a, int b, int g)
{   /* c_a^2 c_b c_g^2 - c_s^2 (c_a^2 c_b + c_b c_g^2) + c_s^4 c_b  (k = 23..25) */
    return (double)(c[a] * c[a] * c[b] * c[g] * c[g])
         - CS2 * (double)(c[a] * c[a] * c[b] + c[b] * c[g] * c[g])
         + CS2 * CS2 * c[b];
}

static double herm6(const int *c)
{   /* k = 26 */
    double x2 = c[X] * c[X], y2 = c[Y] * c[Y], z2 = c[Z] * c[Z];
    return x2 * y2 * z2 - CS2 * (x2 * y2 + x2 * z2 + y2 * z2) + CS2 * CS2 * (x2 + y2 + z2)
         - CS2 * CS2 * CS2;
}

static double basis_e(int k, int i)
{
    const int *c = VEL[i];
    switch (k) {
    case 0: return 1.0;
    case 1: return c[X];
    case 2: return c[Y];
    case 3: return c[Z];
    case 4: return (double)(c[X] * c[X]) - CS2;
    case 5: return (double)(c[Y] * c[Y]) - CS2;
    case 6: return (double)(c[Z] * c[Z]) - CS2;
    case 7: return (double)(c[X] * c[Y]);
    case 8: return (double)(c[X] * c[Z]);
    case 9: return (double)(c[Y] * c[Z]);
    case 10: return herm3_a2b(c, X, Y);        /* x^2 y */
    case 11: return herm3_a2b(c, X, Z);        /* x^2 z */
    case 12: return herm3_a2b(c, Y, X);        /* y^2 x */
    case 13: return herm3_a2b(c, Z, X);        /* z^2 x */
    case 14: return herm3_a2b(c, Y, Z);        /* y^2 z */
    case 15: return herm3_a2b(c, Z, Y);        /* z^2 y */
    case 16: return (double)(c[X] * c[Y] * c[Z]);
    case 17: return herm4_a2b2(c, X, Y);       /* x^2 y^2 */
    case 18: return herm4_a2b2(c, X, Z);       /* x^2 z^2 */
    case 19: return herm4_a2b2(c, Y, Z);       /* y^2 z^2 */
    case 20: return herm4_abg2(c, X, Y, Z);    /* x y z^2 */
    case 21: return herm4_abg2(c, X, Z, Y);    /* x z y^2 */
    case 22: return herm4_abg2(c, Y, Z, X);    /* y z x^2 */
    case 23: return herm5(c, X, Y, Z);         /* x^2 y z^2 */
    case 24: return herm5(c, X, Z, Y);         /* x^2 z y^2 */
    case 25: return herm5(c, Y, X, Z);         /* y^2 x z^2 */
    default: return herm6(c);                  /* x^2 y^2 z^2 */
    }
}

static double factorial(int n)
{
    double r = 1.0;
    for (int m = 2; m <= n; ++m) r *= m;
    return r;
}

static double basis_b(int k)
{   /* Sec. II: b_k = n_k! c_s^(2 n_k) / mu_k */
    return factorial(NK[k]) * pow(CS2, NK[k]) / MUK[k];
}

static double W[Q];
static double E[Q][Q];   /* E[k][i] = e_ki */
static double B[Q];
static int tables_ready = 0;

static void init_tables(void)
{
    if (tables_ready) return;
    for (int i = 0; i < Q; ++i) W[i] = weight_of(i);
    for (int k = 0; k < Q; ++k) {
        B[k] = basis_b(k);
        for (int i = 0; i < Q; ++i) E[k][i] = basis_e(k, i);
    }
    tables_ready = 1;
}

/* ----------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the     */
/* multiply-xor S-box on a 4-word counter with a 2-word key that is bumped  */
/* by the Weyl constants between rounds.                                    */
/* ----------------------------------------------------------------------- */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* The four raw words of block j for (seed, node, step). */
void oracle_noise_words(uint64_t seed, uint32_t node, int64_t step, uint32_t block, uint32_t out[4])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint64_t t = (uint64_t)step;
    uint32_t ctr[4] = {node, (uint32_t)t, block, (uint32_t)(t >> 32)};
    oracle_philox4x32_10(ctr, key, out);
}

/* Uniform on (0,1) from a 32-bit word.  bits = 32: (x + 1/2) 2^-32.  bits = 23:
 * the top 23 bits, ((x >> 9) + 1/2) 2^-23, the single-precision variant (the
 * largest width for which every such value is exact in binary32).  Both are
 * exact in double. */
static double uniform_of(uint32_t x, int bits)
{
    if (bits == 23) return ((double)(x >> 9) + 0.5) * (1.0 / 8388608.0);
    return ((double)x + 0.5) * (1.0 / 4294967296.0);
}

/* Standard normals r_4..r_26 of Eqs. (1)/(10) for one node and step; r[0..3]
 * are set to zero (the conserved modes receive no noise). */
void oracle_normals(uint64_t seed, uint32_t node, int64_t step, int bits, double r[Q])
{
    const double two_pi = 2.0 * 3.14159265358979323846;
    for (int k = 0; k < 4; ++k) r[k] = 0.0;
    for (uint32_t j = 0; j < 6; ++j) {
        uint32_t w[4];
        oracle_noise_words(seed, node, step, j, w);
        for (int p = 0; p < 2; ++p) {
            double u1 = uniform_of(w[2 * p], bits);
            double u2 = uniform_of(w[2 * p + 1], bits);
            double rad = sqrt(-2.0 * log(u1));
            double ang = two_pi * u2;
            int k = 4 + 4 * (int)j + 2 * p;
            r[k] = rad * cos(ang);
            if (k + 1 < Q) r[k + 1] = rad * sin(ang);
        }
    }
}

/* ----------------------------------------------------------------------- */
/* Parameters shared with the Python test driver (ctypes mirrors it).       */
/* ----------------------------------------------------------------------- */
typedef struct {
    int32_t nx, ny, nz;
    int32_t collision;   /* 0 = GMF-FLBM, Eq. (10); 1 = BGK-FLBM, Eq. (1) */
    double rho0, tau, kbt;
    uint64_t seed;
    int32_t noise_rho;   /* 0 = local rho in Eqs. (2),(9); 1 = rho0 */
    int32_t noise_bits;  /* 32 (double uniforms) or 23 (single-precision uniforms) */
} oracle_params;

/* ----------------------------------------------------------------------- */
/* Collision, written in the paper's own terms.                             */
/* ----------------------------------------------------------------------- */

/* Second-order equilibrium (Sec. II, Eq. (11)). */
void oracle_feq(double rho, const double u[3], double feq[Q])
{
    init_tables();
    for (int i = 0; i < Q; ++i) {
        const int *c = VEL[i];
        double cu = 0.0, quad = 0.0;
        for (int a = 0; a < 3; ++a) cu += c[a] * u[a];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                quad += ((double)(c[a] * c[b]) - CS2 * (a == b)) * u[a] * u[b];
        feq[i] = W[i] * rho * (1.0 + cu / CS2 + quad / (2.0 * CS2 * CS2));
    }
}

/* Density and momentum, Eqs. (3) and (4). */
static void hydro_moments(const double f[Q], double *rho, double ju[3])
{
    double r = 0.0, j0 = 0.0, j1 = 0.0, j2 = 0.0;
    for (int i = 0; i < Q; ++i) {
        r += f[i];
        j0 += f[i] * VEL[i][0];
        j1 += f[i] * VEL[i][1];
        j2 += f[i] * VEL[i][2];
    }
    *rho = r; ju[0] = j0; ju[1] = j1; ju[2] = j2;
}

/* Noise amplitude phi_k of Eq. (2) (k = 4..9 or BGK) or phi^g_k of Eq. (9). */
static double noise_amplitude(int k, double rho_n, double kbt, double omega, int unit_relaxation)
{
    if (unit_relaxation) return sqrt(rho_n * kbt * B[k] / CS2);
    return sqrt(rho_n * kbt * omega * (2.0 - omega) * B[k] / CS2);
}

/* One collision at a node: f -> f* (the right-hand side of Eq. (10), or of
 * Eq. (1) when p->collision == 1). */
void oracle_collide(const double f[Q], const oracle_params *p, uint32_t node, int64_t step, double fstar[Q])
{
    init_tables();
    const double omega = 1.0 / p->tau;
    double rho, ju[3], u[3], feq[Q], fneq[Q], r[Q];

    hydro_moments(f, &rho, ju);
    for (int a = 0; a < 3; ++a) u[a] = ju[a] / rho;
    oracle_feq(rho, u, feq);

    if (p->collision == 1) {
        /* BGK-FLBM: f^neq = f - f^eq, kept with memory (1 - omega). */
        for (int i = 0; i < Q; ++i) fneq[i] = f[i] - feq[i];
    } else {
        /* GMF-FLBM: f^neq rebuilt from its second-order Hermite coefficient,
         * Eq. (13), then projected back with Eq. (12). */
        double a2[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double s = 0.0;
                for (int i = 0; i < Q; ++i)
                    s += (f[i] - feq[i]) * ((double)(VEL[i][a] * VEL[i][b]) - CS2 * (a == b));
                a2[a][b] = s;
            }
        for (int i = 0; i < Q; ++i) {
            double s = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    s += ((double)(VEL[i][a] * VEL[i][b]) - CS2 * (a == b)) * a2[a][b];
            fneq[i] = W[i] * s / (2.0 * CS2 * CS2);
        }
    }

    double rho_n = p->noise_rho ? p->rho0 : rho;
    double amp[Q];
    for (int k = 0; k < Q; ++k) amp[k] = 0.0;
    if (p->kbt > 0.0) {
        oracle_normals(p->seed, node, step, p->noise_bits, r);
        for (int k = 4; k < Q; ++k) {
            int ghost = (k >= 10) && (p->collision == 0);
            amp[k] = noise_amplitude(k, rho_n, p->kbt, omega, ghost) * r[k];
        }
    }

    for (int i = 0; i < Q; ++i) {
        double hyd = 0.0, gho = 0.0;
        for (int k = 4; k <= 9; ++k) hyd += E[k][i] * amp[k] / B[k];
        for (int k = 10; k < Q; ++k) gho += E[k][i] * amp[k] / B[k];
        fstar[i] = feq[i] + (1.0 - omega) * fneq[i] + W[i] * hyd + W[i] * gho;
    }
}

/* The same collision carried out in moment space: m = E f; conserved moments
 * kept; k = 4..9 relaxed towards their equilibrium values with rate omega plus
 * noise; k = 10..26 replaced by noise only (GMF) or relaxed towards their
 * equilibrium projection (BGK); f* = W E^T B^-1 m*.  Used by the tests to show
 * that the literal form above and the moment-space reading agree. */
void oracle_collide_moment_space(const double f[Q], const oracle_params *p, uint32_t node, int64_t step,
                                 double fstar[Q])
{
    init_tables();
    const double omega = 1.0 / p->tau;
    double m[Q], meq[Q], feq[Q], rho, ju[3], u[3], r[Q];
    hydro_moments(f, &rho, ju);
    for (int a = 0; a < 3; ++a) u[a] = ju[a] / rho;
    oracle_feq(rho, u, feq);
    for (int k = 0; k < Q; ++k) {
        double s = 0.0, se = 0.0;
        for (int i = 0; i < Q; ++i) {
            s += E[k][i] * f[i];
            se += E[k][i] * feq[i];
        }
        m[k] = s;
        meq[k] = se;
    }
    double rho_n = p->noise_rho ? p->rho0 : rho;
    for (int k = 0; k < Q; ++k) r[k] = 0.0;
    if (p->kbt > 0.0) oracle_normals(p->seed, node, step, p->noise_bits, r);
    double mstar[Q];
    for (int k = 0; k < Q; ++k) {
        if (k < 4) {
            mstar[k] = m[k];
        } else if (k < 10 || p->collision == 1) {
            double amp = p->kbt > 0.0 ? noise_amplitude(k, rho_n, p->kbt, omega, 0) * r[k] : 0.0;
            mstar[k] = meq[k] + (1.0 - omega) * (m[k] - meq[k]) + amp;
        } else {
            /* GMF ghost mode: no deterministic content survives (the
             * second-order equilibrium is orthogonal to every ghost vector),
             * only the noise of Eq. (9) is left */
            mstar[k] = p->kbt > 0.0 ? noise_amplitude(k, rho_n, p->kbt, omega, 1) * r[k] : 0.0;
        }
    }
    for (int i = 0; i < Q; ++i) {
        double s = 0.0;
        for (int k = 0; k < Q; ++k) s += E[k][i] * mstar[k] / B[k];
        fstar[i] = W[i] * s;
    }
}

/* ----------------------------------------------------------------------- */
/* Lattice driver: collide at every node, then stream (Eq. (10) left side). */
/* ----------------------------------------------------------------------- */
static int64_t wrap(int64_t a, int64_t n)
{
    a %= n;
    return a < 0 ? a + n : a;
}

/* Advance f (canonical, f[i*N + n]) by nsteps starting at step index t0. */
int oracle_run(const oracle_params *p, double *f, int64_t t0, int64_t nsteps)
{
    init_tables();
    const int64_t nx = p->nx, ny = p->ny, nz = p->nz;
    const int64_t N = nx * ny * nz;
    if (N <= 0 || p->tau <= 0.5 || p->rho0 <= 0.0 || p->kbt < 0.0) return -1;
    double *next = (double *)malloc(sizeof(double) * Q * (size_t)N);
    if (!next) return -2;
    for (int64_t s = 0; s < nsteps; ++s) {
        const int64_t t = t0 + s;
#pragma omp parallel for schedule(static)
        for (int64_t z = 0; z < nz; ++z) {
            for (int64_t y = 0; y < ny; ++y) {
                for (int64_t x = 0; x < nx; ++x) {
                    const int64_t n = x + nx * (y + ny * z);
                    double fl[Q], fs[Q];
                    for (int i = 0; i < Q; ++i) fl[i] = f[i * N + n];
                    oracle_collide(fl, p, (uint32_t)n, t, fs);
                    for (int i = 0; i < Q; ++i) {
                        int64_t xd = wrap(x + VEL[i][0], nx);
                        int64_t yd = wrap(y + VEL[i][1], ny);
                        int64_t zd = wrap(z + VEL[i][2], nz);
                        next[i * N + xd + nx * (yd + ny * zd)] = fs[i];
                    }
                }
            }
        }
        memcpy(f, next, sizeof(double) * Q * (size_t)N);
    }
    free(next);
    return 0;
}

/* Rest equilibrium f_i = w_i rho0 (the initial state of every workload). */
void oracle_rest_state(const oracle_params *p, double *f)
{
    init_tables();
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    for (int i = 0; i < Q; ++i)
        for (int64_t n = 0; n < N; ++n) f[i * N + n] = W[i] * p->rho0;
}

/* Density and velocity fields (Eqs. (3), (4)); u laid out ux | uy | uz. */
void oracle_moments(const oracle_params *p, const double *f, double *rho, double *u)
{
    init_tables();
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    for (int64_t n = 0; n < N; ++n) {
        double fl[Q], r, ju[3];
        for (int i = 0; i < Q; ++i) fl[i] = f[i * N + n];
        hydro_moments(fl, &r, ju);
        rho[n] = r;
        for (int a = 0; a < 3; ++a) u[a * N + n] = ju[a] / r;
    }
}

/* Global mass and momentum sums. */
void oracle_totals(const oracle_params *p, const double *f, double out[4])
{
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    double m = 0.0, j0 = 0.0, j1 = 0.0, j2 = 0.0;
    for (int64_t n = 0; n < N; ++n)
        for (int i = 0; i < Q; ++i) {
            double v = f[i * N + n];
            m += v;
            j0 += v * VEL[i][0];
            j1 += v * VEL[i][1];
            j2 += v * VEL[i][2];
        }
    out[0] = m; out[1] = j0; out[2] = j1; out[3] = j2;
}

/* ----------------------------------------------------------------------- */
/* Observables of the Results section.                                       */
/*   Per-node observables (index o):                                         */
/*     0 drho = rho - rho0      1-3 j_a = rho u_a     4 sum_a j_a            */
/*     5 sum_a (Pi_aa - rho0 cs2)   6 sum_{a<b} Pi_ab     7-9 u_a            */
/*   Pi_ab = sum_i f_i c_ia c_ib is the momentum-flux tensor.                */
/*   sums[2*o] = sum_x o(x), sums[2*o+1] = sum_x o(x)^2.                     */
/*   Spectra (normalised DFT m(k) = N^-1/2 sum_x m(x) exp(-i k.x), k =      */
/*   2 pi n / L, averaged over every integer vector n of the shell):         */
/*     field 0 rho, 1 j (mean over the three components), 2 sum_a j_a,       */
/*     3 sum_a Pi_aa, 4 sum_{a<b} Pi_ab;  shells |n|^2 = 1,2,3,4,5,6,8,9.     */
/* ----------------------------------------------------------------------- */
#define NOBS 10
#define NSPEC 5
#define NSHELL 8
static const int SHELL_N2[NSHELL] = {1, 2, 3, 4, 5, 6, 8, 9};

static void node_observables(const oracle_params *p, const double fl[Q], double o[NOBS])
{
    double rho, ju[3], pi[3][3];
    hydro_moments(fl, &rho, ju);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int i = 0; i < Q; ++i) s += fl[i] * (double)(VEL[i][a] * VEL[i][b]);
            pi[a][b] = s;
        }
    o[0] = rho - p->rho0;
    o[1] = ju[0]; o[2] = ju[1]; o[3] = ju[2];
    o[4] = ju[0] + ju[1] + ju[2];
    o[5] = (pi[0][0] - p->rho0 * CS2) + (pi[1][1] - p->rho0 * CS2) + (pi[2][2] - p->rho0 * CS2);
    o[6] = pi[0][1] + pi[0][2] + pi[1][2];
    o[7] = ju[0] / rho; o[8] = ju[1] / rho; o[9] = ju[2] / rho;
}

void oracle_observables(const oracle_params *p, const double *f, double sums[2 * NOBS],
                        double spec[NSPEC * NSHELL])
{
    init_tables();
    const int64_t nx = p->nx, ny = p->ny, nz = p->nz, N = nx * ny * nz;
    double *field = (double *)malloc(sizeof(double) * NOBS * (size_t)N);
    for (int q = 0; q < 2 * NOBS; ++q) sums[q] = 0.0;
    for (int64_t n = 0; n < N; ++n) {
        double fl[Q], o[NOBS];
        for (int i = 0; i < Q; ++i) fl[i] = f[i * N + n];
        node_observables(p, fl, o);
        for (int q = 0; q < NOBS; ++q) {
            field[q * N + n] = o[q];
            sums[2 * q] += o[q];
            sums[2 * q + 1] += o[q] * o[q];
        }
    }
    /* brute-force DFT on every shell vector */
    const double two_pi = 2.0 * 3.14159265358979323846;
    const int src[NSPEC + 2] = {0, 1, 2, 3, 4, 5, 6}; /* rho, jx, jy, jz, jsum, pdiag, poff */
    double acc[NSPEC][NSHELL];
    int cnt[NSHELL];
    memset(acc, 0, sizeof(acc));
    memset(cnt, 0, sizeof(cnt));
    for (int a = -3; a <= 3; ++a)
        for (int b = -3; b <= 3; ++b)
            for (int c = -3; c <= 3; ++c) {
                int n2 = a * a + b * b + c * c, s = -1;
                for (int q = 0; q < NSHELL; ++q)
                    if (SHELL_N2[q] == n2) s = q;
                if (s < 0) continue;
                cnt[s] += 1;
                double re[7] = {0}, im[7] = {0};
                for (int64_t z = 0; z < nz; ++z)
                    for (int64_t y = 0; y < ny; ++y)
                        for (int64_t x = 0; x < nx; ++x) {
                            int64_t n = x + nx * (y + ny * z);
                            double ph = two_pi * ((double)(a * x) / nx + (double)(b * y) / ny + (double)(c * z) / nz);
                            double cr = cos(ph), ci = -sin(ph);
                            for (int q = 0; q < 7; ++q) {
                                re[q] += field[src[q] * N + n] * cr;
                                im[q] += field[src[q] * N + n] * ci;
                            }
                        }
                double pw[7];
                for (int q = 0; q < 7; ++q) pw[q] = (re[q] * re[q] + im[q] * im[q]) / (double)N;
                acc[0][s] += pw[0];
                acc[1][s] += (pw[1] + pw[2] + pw[3]) / 3.0;
                acc[2][s] += pw[4];
                acc[3][s] += pw[5];
                acc[4][s] += pw[6];
            }
    for (int m = 0; m < NSPEC; ++m)
        for (int s = 0; s < NSHELL; ++s) spec[m * NSHELL + s] = acc[m][s] / cnt[s];
    free(field);
}

/* ----------------------------------------------------------------------- */
/* Table access for the tests.                                               */
/* ----------------------------------------------------------------------- */
void oracle_tables(int32_t *vel, double *w, double *e, double *b, int32_t *nk, int32_t *muk)
{
    init_tables();
    for (int i = 0; i < Q; ++i) {
        for (int a = 0; a < 3; ++a) vel[3 * i + a] = VEL[i][a];
        w[i] = W[i];
    }
    for (int k = 0; k < Q; ++k) {
        b[k] = B[k];
        nk[k] = NK[k];
        muk[k] = MUK[k];
        for (int i = 0; i < Q; ++i) e[k * Q + i] = E[k][i];
    }
}

/* Threads of the OpenMP loop over z planes in oracle_run (timing only; the
 * result does not depend on it). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
