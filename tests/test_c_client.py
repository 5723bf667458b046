"""The C ABI from a plain C program (tests/c/gmf_c_client.c): no Python
binding and no torch in that process; the library allocates its own
workspace and stream.  The CPU test makes only calls that touch no device;
the GPU test runs a 16^3 FP64 box and compares the populations it wrote with
the oracle's."""
import os
import subprocess

import numpy as np
import pytest

import c_client
import oracle
from gpu_common import say



def test_c_client_validates_without_a_device():
    exe = c_client.build()
    run = subprocess.run([exe, "validate"], capture_output=True, text=True, timeout=120)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "0 failure(s)" in run.stdout


@pytest.mark.gpu
def test_c_client_run_matches_oracle(tmp_path):
    exe = c_client.build()
    steps = 50
    out = tmp_path / "f.bin"
    say(f"C client: 16^3 FP64, {steps} steps")
    run = subprocess.run([exe, "run", str(out), str(steps)], capture_output=True, text=True, timeout=300)
    say("  " + run.stdout.strip())
    assert run.returncode == 0, run.stdout + run.stderr
    got = np.fromfile(out, dtype=np.float64)
    p = oracle.params(16, rho0=1.0, tau=1.0, kbt=1e-4, seed=1)
    ref = oracle.rest_state(p)
    oracle.run(p, ref, 0, steps)
    w = oracle.tables()[1]
    g_got = got.reshape(27, -1) - w[:, None]
    g_ref = ref.reshape(27, -1) - w[:, None]
    err = float(np.max(np.abs(g_got - g_ref)) / np.max(np.abs(g_ref)))
    say(f"  max|dg|/max|g| = {err:.2e}")
    assert err < 1e-11, err
