"""FP64 CPU oracle for GMF-FLBM (D3Q27), Python side.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the ``cpu_baseline`` leg of ``bench.py``; never by the library.

This module is a thin ctypes wrapper around ``gmf_oracle.c`` (the literal,
slow reading of the paper's Sec. II, Eqs. (1)-(13), Tables I-II).  It holds no
arithmetic of the method itself.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gmf_oracle.c")
_LIB = os.path.join(_HERE, "libgmf_oracle.so")

Q = 27
NOBS = 10
NSPEC = 5
NSHELL = 8
SHELL_N2 = (1, 2, 3, 4, 5, 6, 8, 9)

GMF = 0
BGK = 1


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP over z)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", _LIB + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("collision", ctypes.c_int32),
        ("rho0", ctypes.c_double), ("tau", ctypes.c_double), ("kbt", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("noise_rho", ctypes.c_int32), ("noise_bits", ctypes.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        i32p = ctypes.POINTER(ctypes.c_int32)
        P = ctypes.POINTER(Params)
        L.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.oracle_noise_words.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64, ctypes.c_uint32, u32p]
        L.oracle_normals.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64, ctypes.c_int, dp]
        L.oracle_feq.argtypes = [ctypes.c_double, dp, dp]
        L.oracle_collide.argtypes = [dp, P, ctypes.c_uint32, ctypes.c_int64, dp]
        L.oracle_collide_moment_space.argtypes = [dp, P, ctypes.c_uint32, ctypes.c_int64, dp]
        L.oracle_run.argtypes = [P, dp, ctypes.c_int64, ctypes.c_int64]
        L.oracle_run.restype = ctypes.c_int
        L.oracle_rest_state.argtypes = [P, dp]
        L.oracle_moments.argtypes = [P, dp, dp, dp]
        L.oracle_totals.argtypes = [P, dp, dp]
        L.oracle_observables.argtypes = [P, dp, dp, dp]
        L.oracle_tables.argtypes = [i32p, dp, dp, dp, i32p, i32p]
        L.oracle_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    if a.dtype != np.float64 or not a.flags.c_contiguous:
        raise ValueError("expected a C-contiguous float64 array")
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _u32p(a: np.ndarray):
    if a.dtype != np.uint32 or not a.flags.c_contiguous:
        raise ValueError("expected a C-contiguous uint32 array")
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def params(nx, ny=None, nz=None, *, rho0=1.0, tau=1.0, kbt=0.0, seed=1,
           collision=GMF, noise_rho=0, noise_bits=32) -> Params:
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    return Params(nx, ny, nz, collision, rho0, tau, kbt, seed, noise_rho, noise_bits)


def tables():
    """Velocity table c (27x3), weights w, basis e[k][i], norms b, n_k, mu_k."""
    vel = np.zeros(81, np.int32)
    w = np.zeros(Q)
    e = np.zeros(Q * Q)
    b = np.zeros(Q)
    nk = np.zeros(Q, np.int32)
    mu = np.zeros(Q, np.int32)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib().oracle_tables(vel.ctypes.data_as(i32p), _dp(w), _dp(e), _dp(b),
                        nk.ctypes.data_as(i32p), mu.ctypes.data_as(i32p))
    return vel.reshape(Q, 3), w, e.reshape(Q, Q), b, nk, mu


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().oracle_philox4x32_10(_u32p(c), _u32p(k), _u32p(out))
    return out


def noise_words(seed: int, node: int, step: int, block: int) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    lib().oracle_noise_words(seed, node, step, block, _u32p(out))
    return out


def normals(seed: int, node: int, step: int, bits: int = 32) -> np.ndarray:
    r = np.zeros(Q)
    lib().oracle_normals(seed, node, step, bits, _dp(r))
    return r


def feq(rho: float, u) -> np.ndarray:
    uu = np.ascontiguousarray(u, dtype=np.float64)
    if uu.size != 3:
        raise ValueError("feq: u needs three components")
    out = np.zeros(Q)
    lib().oracle_feq(rho, _dp(uu), _dp(out))
    return out


def collide(f, p: Params, node: int = 0, step: int = 0, moment_space: bool = False) -> np.ndarray:
    ff = np.ascontiguousarray(f, dtype=np.float64)
    if ff.size != Q:
        raise ValueError("collide: one node's 27 populations")
    out = np.zeros(Q)
    fn = lib().oracle_collide_moment_space if moment_space else lib().oracle_collide
    fn(_dp(ff), ctypes.byref(p), node, step, _dp(out))
    return out


def rest_state(p: Params) -> np.ndarray:
    f = np.zeros(Q * p.nx * p.ny * p.nz)
    lib().oracle_rest_state(ctypes.byref(p), _dp(f))
    return f


def _check_pops(p: Params, f: np.ndarray):
    if f.shape != (Q * p.nx * p.ny * p.nz,):
        raise ValueError(f"populations of shape {f.shape} for a {p.nx}x{p.ny}x{p.nz} box")


def run(p: Params, f: np.ndarray, t0: int, nsteps: int) -> np.ndarray:
    """Advance the canonical populations f (27*N, f[i*N+n]) in place."""
    _check_pops(p, f)
    rc = lib().oracle_run(ctypes.byref(p), _dp(f), t0, nsteps)
    if rc != 0:
        raise ValueError(f"oracle_run failed with {rc}")
    return f


def moments(p: Params, f: np.ndarray):
    _check_pops(p, f)
    N = p.nx * p.ny * p.nz
    rho = np.zeros(N)
    u = np.zeros(3 * N)
    lib().oracle_moments(ctypes.byref(p), _dp(f), _dp(rho), _dp(u))
    return rho, u.reshape(3, N)


def totals(p: Params, f: np.ndarray) -> np.ndarray:
    _check_pops(p, f)
    out = np.zeros(4)
    lib().oracle_totals(ctypes.byref(p), _dp(f), _dp(out))
    return out


def observables(p: Params, f: np.ndarray):
    """(sums[NOBS,2], spectra[NSPEC,NSHELL]) of one state; see gmf_oracle.c."""
    _check_pops(p, f)
    sums = np.zeros(2 * NOBS)
    spec = np.zeros(NSPEC * NSHELL)
    lib().oracle_observables(ctypes.byref(p), _dp(f), _dp(sums), _dp(spec))
    return sums.reshape(NOBS, 2), spec.reshape(NSPEC, NSHELL)


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loop (timing only; results do not depend on it)."""
    lib().oracle_set_threads(int(n))
