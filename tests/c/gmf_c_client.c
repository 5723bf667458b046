/*
 * A plain C client of the library's C ABI (include/gmf.h): no Python, no
 * torch.  The library owns the device workspace and the stream.
 *
 *   gmf_c_client validate            calls that touch no device: sizes,
 *                                    argument errors, error strings
 *   gmf_c_client run FILE STEPS      one 16^3 FP64 box (rho0 1, tau 1,
 *                                    k_B T 1e-4, seed 1) from rest, STEPS
 *                                    steps; checks mass and momentum
 *                                    conservation and the density moments,
 *                                    then writes f(x, STEPS) (27 N doubles,
 *                                    f[i N + n]) to FILE
 *
 * Exit status 0 when every check holds.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "gmf.h"

static int failures = 0;

static void check(int ok, const char* what)
{
    if (!ok) {
        fprintf(stderr, "FAIL: %s\n", what);
        ++failures;
    }
}

static gmf_options fp64_options(void)
{
    gmf_options opt;
    memset(&opt, 0, sizeof(opt));
    opt.precision = GMF_FP64;
    opt.collision = GMF_COLLISION_GMF;
    opt.graph_steps = -1;
    opt.storage = GMF_STORE_POPULATIONS;
    return opt;
}

static int validate(void)
{
    const gmf_replica rep = {16, 16, 16, 0, 1.0, 1.0, 1e-4, 1};
    const gmf_options opt = fp64_options();
    const size_t ws = gmf_workspace_bytes(&rep, 1, &opt);
    check(ws >= (size_t)2 * 27 * 8 * 16 * 16 * 16, "workspace holds two FP64 population buffers");
    check(gmf_workspace_bytes(&rep, 0, &opt) == 0, "no replicas: size 0");
    gmf_replica bad = rep;
    bad.tau = 0.5;
    check(gmf_workspace_bytes(&bad, 1, &opt) == 0, "tau <= 1/2: size 0");
    gmf_ctx* ctx = (gmf_ctx*)&bad;   /* must be overwritten with NULL */
    check(gmf_init(&bad, 1, &opt, NULL, 0, NULL, &ctx) == GMF_EINVAL, "init rejects tau <= 1/2");
    check(ctx == NULL, "rejected init leaves no context");
    check(gmf_init(&rep, 1, &opt, NULL, 0, NULL, NULL) == GMF_EINVAL, "init needs an output pointer");
    check(gmf_step(NULL, 1) == GMF_ESTATE, "step on NULL");
    check(gmf_stats(NULL, 0, NULL) == GMF_ESTATE, "stats on NULL");
    check(strcmp(gmf_strerror(GMF_EINVAL), "invalid argument") == 0, "error string");
    gmf_destroy(NULL);
    printf("validate: %d failure(s)\n", failures);
    return failures != 0;
}

static int run(const char* path, long steps)
{
    const gmf_replica rep = {16, 16, 16, 0, 1.0, 1.0, 1e-4, 1};
    const gmf_options opt = fp64_options();
    const size_t n = (size_t)16 * 16 * 16;
    gmf_ctx* ctx = NULL;
    int rc = gmf_init(&rep, 1, &opt, NULL, 0, NULL, &ctx);
    if (rc != GMF_OK) {
        fprintf(stderr, "gmf_init: %s\n", gmf_strerror(rc));
        return 1;
    }
    gmf_stats_t s0, s1;
    check(gmf_stats(ctx, 0, &s0) == GMF_OK, "stats at t = 0");
    check(gmf_step(ctx, steps) == GMF_OK, "step");
    check(gmf_stats(ctx, 0, &s1) == GMF_OK, "stats after the steps");
    int64_t t = -1;
    check(gmf_get_step(ctx, &t) == GMF_OK && t == steps, "step counter");
    check(fabs(s1.mass - s0.mass) < 1e-12 * s0.mass, "mass conserved");
    for (int a = 0; a < 3; ++a) check(fabs(s1.momentum[a] - s0.momentum[a]) < 1e-12 * s0.mass, "momentum conserved");
    double* rho = (double*)malloc(sizeof(double) * n);
    double* u = (double*)malloc(sizeof(double) * 3 * n);
    double* f = (double*)malloc(sizeof(double) * 27 * n);
    check(rho && u && f, "host buffers");
    if (rho && u && f) {
        check(gmf_moments(ctx, 0, rho, u) == GMF_OK, "moments");
        double mean = 0.0;
        for (size_t i = 0; i < n; ++i) mean += rho[i];
        mean /= (double)n;
        check(fabs(mean - 1.0) < 1e-12, "mean density rho0");
        check(gmf_get_populations(ctx, 0, f) == GMF_OK, "populations");
        FILE* fh = fopen(path, "wb");
        check(fh != NULL, "output file");
        if (fh) {
            check(fwrite(f, sizeof(double), 27 * n, fh) == 27 * n, "write");
            fclose(fh);
        }
    }
    check(gmf_moments(ctx, 1, rho, u) == GMF_EINVAL, "replica out of range");
    free(rho);
    free(u);
    free(f);
    gmf_destroy(ctx);
    printf("run: %ld steps, mass %.17g -> %.17g, %d failure(s)\n", steps, s0.mass, s1.mass, failures);
    return failures != 0;
}

int main(int argc, char** argv)
{
    if (argc == 2 && strcmp(argv[1], "validate") == 0) return validate();
    if (argc == 4 && strcmp(argv[1], "run") == 0) return run(argv[2], strtol(argv[3], NULL, 10));
    fprintf(stderr, "usage: %s validate | run FILE STEPS\n", argv[0]);
    return 2;
}
