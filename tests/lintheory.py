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


def hydro_window_covariance(lat: Lattice, kvecs, tau, kbt, t_samples, rho0=1.0):
    """Mean over the sample times t_samples of Sigma_h(k, t) = <h(k,t) h(k,t)^H>,
    h = E[:10] f the ten hydrodynamic moments of the pre-collision state, for
    the linearised GMF update started from rest (Sigma_h = 0 at t = 0).

    GMF keeps no ghost content, so the ten moments are a closed linear
    system: with T(k) = E[:10] S(k) W E^T B^-1 (10 x 27),
        h(t+1) = T D h(t) + T xi(t),
    D = diag(1, 1, 1, 1, (1-omega) x 6) on the ten moments, and xi the noise
    of the modes k = 4..26 (variances of Eqs. (2), (9)).  Returns (nk, 10, 10)."""
    kvecs = np.atleast_2d(np.asarray(kvecs, dtype=float))
    om = 1.0 / tau
    mu = rho0 * kbt / float(CS2)
    var = np.zeros(27)
    var[4:10] = mu * lat.b[4:10] * om * (2.0 - om)
    var[10:] = mu * lat.b[10:]
    back = (lat.w[:, None] * lat.E.T) / lat.b[None, :]               # W E^T B^-1 (27 x 27)
    ph = np.exp(-1j * (kvecs @ lat.vel.T.astype(float)))             # (nk, 27)
    T = lat.E[None, :10, :] * ph[:, None, :] @ back[None]             # (nk, 10, 27)
    d10 = np.array([1.0] * 4 + [1.0 - om] * 6)
    M = T[:, :, :10] * d10[None, None, :]
    Qh = (T * var[None, None, :]) @ np.conj(np.transpose(T, (0, 2, 1)))
    MH = np.conj(np.transpose(M, (0, 2, 1)))
    ts = sorted(set(int(t) for t in t_samples))
    want = set(ts)
    Sig = np.zeros((len(kvecs), 10, 10), complex)
    acc = np.zeros_like(Sig)
    for t in range(1, ts[-1] + 1):
        Sig = M @ Sig @ MH + Qh
        if t in want:
            acc += Sig
    return acc / len(ts)                  # a sample at t = 0 (rest) adds Sigma_h = 0


def signed_axis_map(rep, n):
    """A 3x3 signed permutation G with G rep = n (rep and n integer 3-vectors
    of equal sorted magnitudes)."""
    rep = tuple(int(v) for v in rep)
    n = tuple(int(v) for v in n)
    for perm in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
        G = np.zeros((3, 3), dtype=np.int64)
        ok = True
        for a in range(3):
            src = rep[perm[a]]
            if abs(src) != abs(n[a]):
                ok = False
                break
            G[a, perm[a]] = -1 if (src != 0 and src == -n[a]) else 1
        if ok:
            assert tuple(G @ np.array(rep)) == n
            return G
    raise ValueError(f"{n} is not a signed permutation of {rep}")


def shell_powers(lat: Lattice, L: int, shells, tau, kbt, t_samples, rho0=1.0):
    """Linear-theory shell spectra averaged over the sample times: for each
    shell (a list of integer wave vectors n of a cubic box of side L) the mean
    over its vectors of <|m(k)|^2>, orthonormal DFT, for the spectra
    rho, j (mean of the three components), sum_a j_a, sum_a Pi_aa and
    sum_{a<b} Pi_ab.  Returns an array (5, len(shells)).

    The lattice and the linearised update are invariant under the 48 signed
    axis permutations g, so Sigma(g k) is Sigma(k) with the velocities
    relabelled (c -> g c): an observable v at g k has the power of v(g c) at
    k.  The recursion runs once per orbit representative (|n_x| >= |n_y| >=
    |n_z| >= 0)."""
    vel = lat.vel
    index = {tuple(int(x) for x in c): i for i, c in enumerate(vel)}
    obs = lat.obs_vectors()
    names = ("rho", "jx", "jy", "jz", "jsum", "pdiag", "poff")
    reps = sorted({tuple(sorted((abs(int(a)) for a in n), reverse=True)) for sh in shells for n in sh})
    Sh = hydro_window_covariance(lat, [kvec_of(r, (L, L, L)) for r in reps], tau, kbt, t_samples, rho0)
    rep_index = {r: i for i, r in enumerate(reps)}
    out = np.zeros((5, len(shells)))
    for s, sh in enumerate(shells):
        acc = np.zeros(5)
        for n in sh:
            r = tuple(sorted((abs(int(a)) for a in n), reverse=True))
            G = signed_axis_map(r, n)
            perm = np.array([index[tuple(int(x) for x in G @ c)] for c in vel])   # i -> index of G c_i
            S = Sh[rep_index[r]]
            pw = {}
            for name in names:
                vg = obs[name][perm]                                  # v(G c_i)
                alpha = (lat.E[:10] @ (lat.w * vg)) / lat.b[:10]      # Hermite coefficients of v(G c)
                pw[name] = float(np.real(alpha @ S @ alpha))
            acc += [pw["rho"], (pw["jx"] + pw["jy"] + pw["jz"]) / 3, pw["jsum"], pw["pdiag"], pw["poff"]]
        out[:, s] = acc / len(sh)
    return out
