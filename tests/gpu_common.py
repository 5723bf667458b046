"""Shared helpers of the GPU tests (library through its C ABI, oracle on the CPU)."""
import sys

import numpy as np

import oracle
import paper_2601_03806_amd as gmf


def say(msg: str):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def oracle_params(spec, collision=gmf.COLLISION_GMF, precision=gmf.FP64, noise_rho=0):
    return oracle.params(spec.nx, spec.ny, spec.nz, rho0=spec.rho0, tau=spec.tau, kbt=spec.kbt, seed=spec.seed,
                         collision=collision, noise_rho=noise_rho,
                         noise_bits=32 if precision == gmf.FP64 else 23)


def shifted(f, w, rho0, n):
    """g = f - w rho0 for a canonical population array."""
    return f.reshape(27, n) - (w[:, None] * rho0)


def rel_err(a, b, w, rho0, n):
    """max |g_a - g_b| / max |g_b| with g = f - w rho0 (stricter than relative to f)."""
    ga, gb = shifted(a, w, rho0, n), shifted(b, w, rho0, n)
    return float(np.max(np.abs(ga - gb)) / max(np.max(np.abs(gb)), 1e-300))
