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
