"""Lattice-level pins of the oracle: conservation, linear response against the
exact Fourier propagator, shear viscosity nu = cs2 (tau - 1/2) (Sec. II), and
the finite-time fluctuation statistics against the exact covariance recursion
of the linearised stochastic update.
"""
import math
from itertools import product

import numpy as np
import pytest

import oracle
import lintheory as lt

CS2 = 1.0 / 3.0


@pytest.fixture(scope="module")
def tabs():
    return oracle.tables()


def _fields(f, p):
    return f.reshape(27, p.nz, p.ny, p.nx)


@pytest.mark.parametrize("coll", [oracle.GMF, oracle.BGK])
def test_conservation_per_step(tabs, coll):
    vel, w, *_ = tabs
    L = 12
    p = oracle.params(L, tau=0.55, kbt=1e-4, seed=3, collision=coll)
    rng = np.random.default_rng(0)
    N = L ** 3
    f = (w[:, None] * (1 + 0.02 * rng.uniform(-1, 1, (27, N)))).ravel()
    c = vel.astype(float)

    def exact_totals(ff):
        # correctly rounded sums, so that only the collision's own rounding shows
        g = ff.reshape(27, N)
        return np.array([math.fsum(g.ravel())] + [math.fsum((g * c[:, a:a + 1]).ravel()) for a in range(3)])

    t0 = exact_totals(f)
    np.testing.assert_allclose(oracle.totals(p, f), t0, rtol=1e-12, atol=1e-12)
    eps = np.finfo(float).eps
    for s in range(20):
        oracle.run(p, f, s, 1)
        t = exact_totals(f)
        bound = 64 * N * eps * np.max(np.abs(f)) * (s + 1)
        assert np.all(np.abs(t - t0) <= bound), (s, t - t0, bound)


def test_linear_response_matches_fourier_propagator(tabs):
    """Small random perturbation of rest, no noise: every Fourier mode of the
    oracle's state after t steps equals A(k)^t applied to its initial value,
    A(k) = S(k) C (streaming times the linearised collision)."""
    vel, w, *_ = tabs
    L, T, eps = 8, 6, 1e-8
    lat = lt.Lattice(vel)
    for tau in (0.6, 1.7):
        p = oracle.params(L, tau=tau, kbt=0.0)
        rng = np.random.default_rng(int(tau * 10))
        N = L ** 3
        d0 = eps * rng.standard_normal((27, N))
        f = (w[:, None] + d0).ravel()
        oracle.run(p, f, 0, T)
        d1 = f.reshape(27, N) - w[:, None]
        F0 = np.fft.fftn(d0.reshape(27, L, L, L), axes=(1, 2, 3))
        F1 = np.fft.fftn(d1.reshape(27, L, L, L), axes=(1, 2, 3))
        err = 0.0
        for nz, ny, nx in product(range(L), repeat=3):
            k = lt.kvec_of((nx, ny, nz), (L, L, L))
            A = lat.propagator(k, tau)
            pred = np.linalg.matrix_power(A, T) @ F0[:, nz, ny, nx]
            err = max(err, np.max(np.abs(pred - F1[:, nz, ny, nx])))
        # the neglected nonlinearity is O(eps^2 N)
        assert err < 1e-13 * np.sqrt(N), err


@pytest.mark.parametrize("tau", [0.6, 1.0, 2.0])
def test_shear_wave_decay(tabs, tau):
    """Noise-free shear wave u_x = A sin(2 pi y / L): per-step decay factor equals
    the exact eigenvalue of the Fourier propagator (1e-8) and the viscosity
    nu = cs2 (tau - 1/2) of Sec. II to within the lattice's O(k^2) correction."""
    vel, w, *_ = tabs
    c = vel.astype(float)
    L, amp = 32, 1e-6
    p = oracle.params(1, L, 1, tau=tau, kbt=0.0)
    y = np.arange(L)
    ux = amp * np.sin(2 * np.pi * y / L)
    f = np.zeros((27, L))
    for j in range(L):
        f[:, j] = oracle.feq(1.0, [ux[j], 0.0, 0.0])
    f = f.ravel()

    def amplitude(ff):
        _, u = oracle.moments(p, ff)
        return 2.0 / L * np.sum(u[0] * np.sin(2 * np.pi * y / L))

    oracle.run(p, f, 0, 120)
    a0 = amplitude(f)
    oracle.run(p, f, 120, 1)
    a1 = amplitude(f)
    lam = a1 / a0
    k = 2 * np.pi / L
    lat = lt.Lattice(vel)
    nu = CS2 * (tau - 0.5)
    exact = lt.eig_closest(lat.propagator([0.0, k, 0.0], tau), np.exp(-nu * k * k))
    assert abs(exact.imag) < 1e-12
    assert abs(lam - exact.real) < 1e-8 * abs(lam)
    nu_eff = -np.log(lam) / (k * k)
    assert abs(nu_eff / nu - 1) < 0.02


def _theory_variances(lat, L, tau, kbt, steps_list):
    kv = [lt.kvec_of(n, (L, L, L)) for n in product(range(L), repeat=3)]
    ns = list(product(range(L), repeat=3))
    hist = lt.covariance_history(lat, kv, tau, kbt, max(steps_list), record=steps_list)
    vecs = lat.obs_vectors()
    out = {}
    N = L ** 3
    for t in steps_list:
        S = hist[t]
        res = {}
        for name, v in vecs.items():
            pw = np.real(np.einsum("i,kij,j->k", v, S, v))   # <|m(k)|^2> per k
            pw[0] = 0.0                                        # k = 0 drops out of a spatial variance
            res[name] = pw.sum() / N
            res[name + "_pw"] = pw
        out[t] = res
    return out, ns


@pytest.mark.slow
def test_finite_time_statistics(tabs):
    """Ensemble over seeds of the spatial variances and shell spectra of an
    8^3 box started at rest, against the exact covariance recursion
    Sigma_{t+1}(k) = A(k) Sigma_t(k) A(k)^H + S(k) Qn S(k)^H."""
    vel, w, *_ = tabs
    L, tau, kbt = 8, 0.6, 1e-5
    steps = [3, 30]
    lat = lt.Lattice(vel)
    theo, ns = _theory_variances(lat, L, tau, kbt, steps)
    nseeds = 40
    names = ["rho", "jx", "jy", "jz", "jsum", "pdiag", "poff"]
    obs_index = {"rho": 0, "jx": 1, "jy": 2, "jz": 3, "jsum": 4, "pdiag": 5, "poff": 6}
    samples = {t: {n: [] for n in names} for t in steps}
    spec_samples = {t: [] for t in steps}
    N = L ** 3
    for s in range(nseeds):
        p = oracle.params(L, tau=tau, kbt=kbt, seed=1000 + s)
        f = oracle.rest_state(p)
        t_prev = 0
        for t in steps:
            oracle.run(p, f, t_prev, t - t_prev)
            t_prev = t
            sums, spec = oracle.observables(p, f)
            for n in names:
                o = obs_index[n]
                samples[t][n].append(sums[o, 1] / N - (sums[o, 0] / N) ** 2)
            spec_samples[t].append(spec)
    for t in steps:
        for n in names:
            x = np.array(samples[t][n])
            se = x.std(ddof=1) / np.sqrt(len(x))
            assert abs(x.mean() - theo[t][n]) < 4.5 * se + 1e-3 * theo[t][n], (t, n, x.mean(), theo[t][n], se)
        # shell spectra: rho shell average on |n|^2 = 1 and 3
        sp = np.array(spec_samples[t])            # (nseeds, 5, 8)
        pw = theo[t]["rho_pw"]
        for shell_idx, n2 in ((0, 1), (2, 3)):
            sel = [i for i, nn in enumerate(ns) if sum(min(a, L - a) ** 2 for a in nn) == n2]
            th = pw[sel].mean()
            x = sp[:, 0, shell_idx]
            se = x.std(ddof=1) / np.sqrt(len(x))
            assert abs(x.mean() - th) < 4.5 * se, (t, n2, x.mean(), th, se)


def test_equilibrium_values_from_theory(tabs):
    """The stationary linear theory gives the equilibrium variances of the
    Results section: <drho^2> = rho0 kbt/cs2, <j_a^2> = rho0 kbt."""
    vel, *_ = tabs
    lat = lt.Lattice(vel)
    mu = 1e-4 / CS2
    S = mu * np.diag(lat.w)
    v = lat.obs_vectors()
    assert abs(v["rho"] @ S @ v["rho"] - 1e-4 / CS2) < 1e-18
    assert abs(v["jx"] @ S @ v["jx"] - 1e-4) < 1e-18
    assert abs(v["pdiag"] @ S @ v["pdiag"] - 5e-4) < 1e-17
    assert abs(v["poff"] @ S @ v["poff"] - 1e-4) < 1e-18


@pytest.mark.parametrize("box", [(6, 5, 4), (1, 7, 3)])
def test_observables_of_known_fields(tabs, box):
    """oracle_observables on f = f^eq(rho(x), u(x)) built from known fields
    (Eq. (11)): the equilibrium carries exactly rho, rho u and
    Pi = rho u u + rho cs2 I, so every per-node observable has a closed form.
    u_a must be j_a / rho (not j_a / rho0): the density field varies by +-40%."""
    vel, w, *_ = tabs
    nx, ny, nz = box
    N = nx * ny * nz
    rng = np.random.default_rng(N)
    rho0 = 1.1
    rho = rho0 * (1 + 0.4 * rng.uniform(-1, 1, N))
    u = 0.05 * rng.uniform(-1, 1, (3, N))
    f = np.empty((27, N))
    for n in range(N):
        f[:, n] = oracle.feq(rho[n], u[:, n])
    p = oracle.params(nx, ny, nz, rho0=rho0)
    sums, _ = oracle.observables(p, np.ascontiguousarray(f.reshape(-1)))
    j = rho * u
    expect = [rho - rho0, j[0], j[1], j[2], j.sum(axis=0),
              rho * (u * u).sum(axis=0) + 3 * CS2 * (rho - rho0),
              rho * (u[0] * u[1] + u[0] * u[2] + u[1] * u[2]),
              u[0], u[1], u[2]]
    for o, v in enumerate(expect):
        assert abs(sums[o, 0] - v.sum()) <= 1e-15 * N * max(np.abs(v).max(), 1e-3), (o, sums[o, 0], v.sum())
        assert abs(sums[o, 1] - (v * v).sum()) <= 1e-15 * N * max((v * v).max(), 1e-6), (o, sums[o, 1], (v * v).sum())
    # the j / rho0 reading would be off by far more than the tolerance
    assert abs((j[0] / rho0).sum() - u[0].sum()) > 1e-3
