"""Physics of the device path checked against linear theory rather than the
oracle's trajectory: the noise-free shear wave of Sec. II decays at the exact
eigenvalue of the lattice's Fourier propagator (tests/lintheory.py), whose
long-wave limit is the viscosity nu = cs2 (tau - 1/2), in both storages and
both precisions."""
import numpy as np
import pytest

import oracle
import lintheory as lt
import paper_2601_03806_amd as gmf
from gpu_common import say

pytestmark = pytest.mark.gpu

CS2 = 1.0 / 3.0


@pytest.mark.parametrize("storage", [gmf.STORE_POPULATIONS, gmf.STORE_MOMENTS])
@pytest.mark.parametrize("prec,tol", [(gmf.FP64, 1e-11), (gmf.FP32_SHIFTED, 3e-7)])
@pytest.mark.parametrize("tau", [0.6, 1.0, 2.0])
def test_shear_wave_decay_on_device(storage, prec, tol, tau):
    """u_x = A sin(2 pi y / L) on a 4 x 64 x 4 box (k_B T = 0) started from
    f^eq: after 100 steps (the faster modes at the same k have died out), the
    mean per-step decay factor over 200 more steps equals the propagator's
    eigenvalue closest to exp(-nu k^2), and the effective viscosity is nu
    within the lattice's O(k^2) correction."""
    vel, w, *_ = oracle.tables()
    L, amp = 64, 1e-4
    spec = gmf.ReplicaSpec(4, L, 4, 1.0, tau, 0.0, 1)
    n = spec.n
    y = (np.arange(n) // spec.nx) % L
    s = np.sin(2 * np.pi * y / L)
    f = np.stack([oracle.feq(1.0, [amp * s[j], 0.0, 0.0]) for j in range(n)], axis=1)
    say(f"shear wave tau={tau} prec={prec} storage={storage}")
    with gmf.Context([spec], precision=prec, storage=storage) as ctx:
        ctx.set_populations(f.ravel())
        ctx.step(100)
        a0 = 2.0 / n * np.sum(ctx.moments()[1][0] * s)
        ctx.step(200)
        a1 = 2.0 / n * np.sum(ctx.moments()[1][0] * s)
    lam = (a1 / a0) ** (1.0 / 200)
    k = 2 * np.pi / L
    nu = CS2 * (tau - 0.5)
    exact = lt.eig_closest(lt.Lattice(vel).propagator([0.0, k, 0.0], tau), np.exp(-nu * k * k))
    say(f"  per-step factor {lam:.12f}, propagator {exact.real:.12f}")
    assert abs(exact.imag) < 1e-12
    assert abs(lam - exact.real) < tol
    assert abs(-np.log(lam) / (k * k) / nu - 1) < 0.01


@pytest.fixture(scope="module")
def finite_time_theory():
    """Spatial variances of the observables of a 16^3 box started at rest
    (tau 0.6, k_B T 1e-5), at steps 3, 30 and 200, from the exact covariance
    recursion of the linearised update, Sigma_{t+1}(k) = A(k) Sigma_t(k) A(k)^H
    + S(k) Qn S(k)^H, summed over k != 0 (tests/lintheory.py)."""
    from itertools import product
    vel = oracle.tables()[0]
    lat = lt.Lattice(vel)
    L, steps = 16, (3, 30, 200)
    kv = [lt.kvec_of(n, (L, L, L)) for n in product(range(L), repeat=3)]
    hist = lt.covariance_history(lat, kv, 0.6, 1e-5, max(steps), record=steps)
    names = ("rho", "jx", "jy", "jz", "jsum", "pdiag", "poff")
    vecs = lat.obs_vectors()
    out = {}
    for t in steps:
        S = hist[t]
        v = []
        for name in names:
            pw = np.real(np.einsum("i,kij,j->k", vecs[name], S, vecs[name]))
            pw[0] = 0.0
            v.append(pw.sum() / L ** 3)
        out[t] = np.array(v)
    return out


@pytest.mark.slow
@pytest.mark.parametrize("storage", [gmf.STORE_POPULATIONS, gmf.STORE_MOMENTS])
def test_finite_time_variances_batched(finite_time_theory, storage):
    """64 replicas of a 16^3 box (seeds 1..64, tau 0.6, k_B T 1e-5) in one FP32
    batched context, started at rest: the ensemble mean of each replica's
    spatial variance of rho, j, sum j, sum Pi_aa and sum_{a<b} Pi_ab at steps
    3 (transient), 30 and 200 equals the exact linear theory within 4.5
    standard errors of the ensemble mean (plus 0.3% for the nonlinear and
    rounding terms the linear theory leaves out)."""
    specs = [gmf.ReplicaSpec(16, 16, 16, 1.0, 0.6, 1e-5, s + 1) for s in range(64)]
    say(f"finite-time variances, 64 x 16^3 batched, storage={storage}")
    with gmf.Context(specs, precision=gmf.FP32_SHIFTED, sample_every=1, graph_steps=0, storage=storage) as ctx:
        t_now = 0
        for t in (3, 30, 200):
            ctx.step(t - t_now)
            ctx.reset_stats()
            ctx.step(1)                    # samples f(., t)
            t_now = t + 1
            var = np.array([ctx.stats(r)["sum_var"][:7] for r in range(len(specs))])
            mean, se = var.mean(axis=0), var.std(axis=0, ddof=1) / np.sqrt(len(specs))
            th = finite_time_theory[t]
            say(f"  t={t}: measured/theory " + " ".join(f"{m / x:.4f}" for m, x in zip(mean, th)))
            assert np.all(np.abs(mean - th) < 4.5 * se + 3e-3 * th), (t, mean / th, se / th)
