"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

A small C driver includes the oracle's source and runs every entry point the
tests use (tables, rest state, the full update in both collisions with noise,
the moment-space collision, moments, totals, observables) on a ragged box
whose every neighbour wraps.  Any out-of-bounds access, leak or undefined
operation aborts the driver (no recovery), which fails the test.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include "gmf_oracle.c"
#include <stdio.h>

int main(void)
{
    int32_t vel[81];
    double w[Q], e[Q * Q], b[Q];
    int32_t nk[Q], mu[Q];
    oracle_tables(vel, w, e, b, nk, mu);
    for (int coll = 0; coll < 2; ++coll) {
        oracle_params p = {5, 3, 2, coll, 1.0, 0.7, 1e-4, 42u, 0, 32};
        const size_t n = (size_t)p.nx * p.ny * p.nz;
        double *f = (double *)malloc(sizeof(double) * Q * n);
        oracle_rest_state(&p, f);
        for (size_t i = 0; i < Q * n; ++i) f[i] *= 1.0 + 0.01 * (double)((i * 2654435761u) % 97) / 97.0;
        if (oracle_run(&p, f, 0, 7) != 0) return 2;
        double fs[Q], fm[Q];
        oracle_collide(f, &p, 3, 7, fs);
        oracle_collide_moment_space(f, &p, 3, 7, fm);
        double *rho = (double *)malloc(sizeof(double) * n), *u = (double *)malloc(sizeof(double) * 3 * n);
        oracle_moments(&p, f, rho, u);
        double tot[4], sums[2 * NOBS], spec[NSPEC * NSHELL];
        oracle_totals(&p, f, tot);
        oracle_observables(&p, f, sums, spec);
        printf("%.6f %.3e\n", tot[0], fs[0] - fm[0]);
        free(rho);
        free(u);
        free(f);
    }
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    src = tmp_path / "drv.c"
    src.write_text(DRIVER)
    exe = tmp_path / "drv"
    subprocess.run(["gcc", "-O1", "-g", "-ffp-contract=off", "-fopenmp", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", f"-I{os.path.join(ROOT, 'oracle')}",
                    str(src), "-o", str(exe), "-lm"], check=True)
    env = dict(os.environ, OMP_NUM_THREADS="1", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert run.returncode == 0, run.stderr[-3000:]
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr, run.stderr[-3000:]
    lines = run.stdout.split()
    assert len(lines) == 4
