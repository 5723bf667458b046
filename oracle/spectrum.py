"""FP64 reference of the full-box shell spectra.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``; never by the library.

The Results section measures the structure factors S_m(|k|) = <|m(k)|^2> of
the density, momentum and stress fields from a normalised FFT of the whole box,
averaged over shells of equal |k|, and compares them with their equilibrium
values (the ER ratios).  This module computes one sample of those shell
averages from a canonical population state, in plain numpy:

  fields (as sampled by the library, pre-collision state f(x, t)):
      drho  = sum_i f_i - rho0                       (Eq. (3))
      j_a   = sum_i f_i c_ia                         (Eq. (4))
      jsum  = j_x + j_y + j_z
      pdiag = sum_a (Pi_aa - rho0 cs^2),  Pi_ab = sum_i f_i c_ia c_ib
      poff  = Pi_xy + Pi_xz + Pi_yz
  transform: m(k) = N^-1/2 sum_x m(x) exp(-i k.x), k_a = 2 pi n_a / L_a with
      integer n_a in [-L_a/2, L_a/2) (numpy.fft.fftn with norm="ortho");
  shells: shell s >= 1 holds the integer vectors with s - 1/2 <= |n| < s + 1/2
      (|n| rounded to the nearest integer); k = 0 is in no shell;
  spectra: rho -> |drho(k)|^2, j -> (|j_x(k)|^2 + |j_y(k)|^2 + |j_z(k)|^2) / 3,
      jsum -> |jsum(k)|^2, pdiag -> |pdiag(k)|^2, poff -> |poff(k)|^2,
      each averaged over the vectors of a shell.
"""
from __future__ import annotations

import numpy as np

from . import Q, tables

CS2 = 1.0 / 3.0
SPECTRA = ("rho", "j", "jsum", "pdiag", "poff")


def fields(p, f: np.ndarray) -> dict:
    """The six sampled fields of the canonical state f[i*N + n], each (nz, ny, nx)."""
    nx, ny, nz = p.nx, p.ny, p.nz
    N = nx * ny * nz
    c = tables()[0].astype(np.float64)                   # (27, 3), interface order
    F = np.asarray(f, dtype=np.float64).reshape(Q, N)
    rho = F.sum(axis=0)
    j = c.T @ F                                          # (3, N)
    pi = {(a, b): (c[:, a] * c[:, b]) @ F for a in range(3) for b in range(a, 3)}
    out = {
        "drho": rho - p.rho0,
        "jx": j[0], "jy": j[1], "jz": j[2],
        "pdiag": sum(pi[(a, a)] - p.rho0 * CS2 for a in range(3)),
        "poff": pi[(0, 1)] + pi[(0, 2)] + pi[(1, 2)],
    }
    return {k: v.reshape(nz, ny, nx) for k, v in out.items()}


def integer_frequencies(L: int) -> np.ndarray:
    """n = 0, 1, ..., then the negative ones: the order of the FFT output."""
    return np.rint(np.fft.fftfreq(L, d=1.0 / L)).astype(np.int64)


def shell_index(nx: int, ny: int, nz: int) -> np.ndarray:
    """Shell of every wave vector of the box, (nz, ny, nx); 0 only at k = 0."""
    n = [integer_frequencies(L) for L in (nz, ny, nx)]
    n2 = n[0][:, None, None] ** 2 + n[1][None, :, None] ** 2 + n[2][None, None, :] ** 2
    s = np.floor(np.sqrt(n2.astype(np.float64)) + 0.5).astype(np.int64)
    # exact criterion (2s - 1)^2 <= 4 |n|^2 < (2s + 1)^2 away from k = 0 (no ties: 4|n|^2 is even)
    nz0 = n2 > 0
    assert np.all((2 * s[nz0] - 1) ** 2 <= 4 * n2[nz0]) and np.all(4 * n2 < (2 * s + 1) ** 2)
    return s


def shell_counts(nx: int, ny: int, nz: int) -> np.ndarray:
    """Integer vectors per shell, shells 0..smax (shell 0 counts nothing)."""
    s = shell_index(nx, ny, nz).ravel()
    cnt = np.bincount(s, minlength=int(s.max()) + 1)
    cnt[0] = 0
    return cnt


def full_spectrum(p, f: np.ndarray):
    """Shell averages of the five spectra for one state: (5, nshell) and the counts."""
    fl = fields(p, f)
    hat = {k: np.fft.fftn(v, norm="ortho") for k, v in fl.items()}
    jsum = hat["jx"] + hat["jy"] + hat["jz"]
    power = [
        np.abs(hat["drho"]) ** 2,
        (np.abs(hat["jx"]) ** 2 + np.abs(hat["jy"]) ** 2 + np.abs(hat["jz"]) ** 2) / 3.0,
        np.abs(jsum) ** 2,
        np.abs(hat["pdiag"]) ** 2,
        np.abs(hat["poff"]) ** 2,
    ]
    s = shell_index(p.nx, p.ny, p.nz).ravel()
    keep = s > 0
    cnt = shell_counts(p.nx, p.ny, p.nz)
    out = np.zeros((len(SPECTRA), len(cnt)))
    for m, pw in enumerate(power):
        sums = np.bincount(s[keep], weights=pw.ravel()[keep], minlength=len(cnt))
        out[m] = np.where(cnt > 0, sums / np.maximum(cnt, 1), 0.0)
    return out, cnt
