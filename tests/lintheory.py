"""Exact and linearised theory used to pin the oracle and the GPU library.

Nothing here calls the oracle or the library.  Every object is built from the
mathematics, independently of the oracle's literal Table II formulas:

* the D3Q27 velocity set and weights come from the product of the D1Q3 set
  (w1(0) = 2/3, w1(+-1) = 1/6);
* the 27 Hermite vectors come from the tensor products h_a(cx) h_b(cy) h_c(cz)
  of the D1Q3 Hermite functions h0 = 1, h1 = c, h2 = c^2 - 1/3, in exact
  rationals;
* the GMF-FLBM collision, linearised about rest, is the 27x27 matrix
  C = W E^T B^-1 D E with D = diag(1,1,1,1, (1-omega) x 6, 0 x 17), and the
  noise covariance is Qn = W E^T B^-1 diag(phi^2) B^-1 E W (Eqs. (2), (9), (10));
* streaming is diagonal in Fourier space, f_i(k) <- exp(-i k.c_i) f*_i(k).
"""
from __future__ import annotations

from fractions import Fraction as Fr
from itertools import product

import numpy as np

CS2 = Fr(1, 3)
W1 = {-1: Fr(1, 6), 0: Fr(2, 3), 1: Fr(1, 6)}
NORM1 = (Fr(1), Fr(1, 3), Fr(2, 9))            # sum_c w1(c) h_a(c)^2

# (a, b, c) Hermite orders along x, y, z for each k, in Table II's print order
ABC = [
    (0, 0, 0),
    (1, 0, 0), (0, 1, 0), (0, 0, 1),
    (2, 0, 0), (0, 2, 0), (0, 0, 2),
    (1, 1, 0), (1, 0, 1), (0, 1, 1),
    (2, 1, 0), (2, 0, 1), (1, 2, 0), (1, 0, 2), (0, 2, 1), (0, 1, 2),
    (1, 1, 1),
    (2, 2, 0), (2, 0, 2), (0, 2, 2),
    (1, 1, 2), (1, 2, 1), (2, 1, 1),
    (2, 1, 2), (2, 2, 1), (1, 2, 2),
    (2, 2, 2),
]


def h1d(a: int, c: int) -> Fr:
    if a == 0:
        return Fr(1)
    if a == 1:
        return Fr(c)
    return Fr(c * c) - CS2


def weight(c) -> Fr:
    return W1[c[0]] * W1[c[1]] * W1[c[2]]


def basis_vector(k: int, c) -> Fr:
    a, b, g = ABC[k]
    return h1d(a, c[0]) * h1d(b, c[1]) * h1d(g, c[2])


def norm(k: int) -> Fr:
    a, b, g = ABC[k]
    return NORM1[a] * NORM1[b] * NORM1[g]


def all_velocities():
    return [c for c in product((-1, 0, 1), repeat=3)]


class Lattice:
    """Float matrices of the linearised GMF/BGK update for a given velocity order."""

    def __init__(self, vel):
        self.vel = np.asarray(vel, dtype=np.int64)
        q = len(self.vel)
        assert q == 27
        self.w = np.array([float(weight(tuple(c))) for c in self.vel])
        self.E = np.array([[float(basis_vector(k, tuple(c))) for c in self.vel] for k in range(27)])
        self.b = np.array([float(norm(k)) for k in range(27)])

    def collision(self, tau: float, bgk: bool = False) -> np.ndarray:
        om = 1.0 / tau
        d = np.zeros(27)
        d[:4] = 1.0
        d[4:10] = 1.0 - om
        d[10:] = (1.0 - om) if bgk else 0.0
        return (self.w[:, None] * self.E.T) @ np.diag(d / self.b) @ self.E

    def noise_cov(self, tau: float, kbt: float, rho0: float = 1.0, bgk: bool = False) -> np.ndarray:
        om = 1.0 / tau
        mu = rho0 * kbt / float(CS2)
        var = np.zeros(27)
        var[4:10] = mu * self.b[4:10] * om * (2.0 - om)
        var[10:] = mu * self.b[10:] * (om * (2.0 - om) if bgk else 1.0)
        M = (self.w[:, None] * self.E.T) @ np.diag(1.0 / self.b)
        return M @ np.diag(var) @ M.T

    def stream(self, kvec) -> np.ndarray:
        ph = np.exp(-1j * (self.vel @ np.asarray(kvec, dtype=float)))
        return np.diag(ph)

    def propagator(self, kvec, tau: float, bgk: bool = False) -> np.ndarray:
        return self.stream(kvec) @ self.collision(tau, bgk)

    # projection vectors of the hydrodynamic observables on delta f
    def obs_vectors(self):
        c = self.vel.astype(float)
        return {
            "rho": np.ones(27),
            "jx": c[:, 0], "jy": c[:, 1], "jz": c[:, 2],
            "jsum": c.sum(axis=1),
            "pdiag": (c ** 2).sum(axis=1),
            "poff": c[:, 0] * c[:, 1] + c[:, 0] * c[:, 2] + c[:, 1] * c[:, 2],
        }


def kvec_of(n, L):
    n = np.asarray(n, dtype=float)
    L = np.asarray(L, dtype=float)
    return 2.0 * np.pi * n / L


def covariance_history(lat: Lattice, kvecs, tau, kbt, steps, rho0=1.0, bgk=False,
                       record=None, start=None):
    """Sigma_t(k) = <f(k,t) f(k,t)^H> for the linearised stochastic update
    started at Sigma_0 (= 0 unless `start` is given).

    Returns a dict {t: array (nk, 27, 27)} for t in `record` (default: only the
    last step), with the orthonormal DFT convention (per-site normalisation).
    """
    kvecs = np.atleast_2d(np.asarray(kvecs, dtype=float))
    nk = len(kvecs)
    C = lat.collision(tau, bgk)
    Qn = lat.noise_cov(tau, kbt, rho0, bgk)
    ph = np.exp(-1j * (kvecs @ lat.vel.T.astype(float)))        # (nk, 27)
    A = ph[:, :, None] * C[None, :, :]                             # S(k) C
    Qk = ph[:, :, None] * Qn[None, :, :] * ph.conj()[:, None, :]   # S Qn S^H
    Sig = np.zeros((nk, 27, 27), complex) if start is None else np.array(start, complex)
    record = {steps} if record is None else set(record)
    out = {}
    AH = np.conj(np.transpose(A, (0, 2, 1)))
    for t in range(1, steps + 1):
        Sig = A @ Sig @ AH + Qk
        if t in record:
            out[t] = Sig.copy()
    return out


def shell_vectors(n2: int):
    r = int(np.ceil(np.sqrt(n2)))
    return [v for v in product(range(-r, r + 1), repeat=3) if v[0] ** 2 + v[1] ** 2 + v[2] ** 2 == n2]


def eig_closest(A: np.ndarray, target: complex):
    ev = np.linalg.eigvals(A)
    return ev[np.argmin(np.abs(ev - target))]
