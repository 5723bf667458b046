"""Pins of the finite-time linear theory that the GPU statistics tests use as
their target (tests/lintheory.py): the ten-moment reduction of the GMF update
against the full 27x27 covariance recursion, the cubic-symmetry shortcut
against a direct evaluation at every wave vector, and the stationary limit
against the fluctuation-dissipation values."""
import numpy as np
import pytest

import oracle
import lintheory as lt

CS2 = 1.0 / 3.0


@pytest.fixture(scope="module")
def lat():
    return lt.Lattice(oracle.tables()[0])


def _direct_powers(lat, kvec, tau, kbt, ts):
    """<|v.f(k)|^2> averaged over ts from the full 27x27 recursion."""
    hist = lt.covariance_history(lat, [kvec], tau, kbt, max(ts), record=ts)
    S = sum(hist[t][0] for t in ts) / len(ts)
    v = lat.obs_vectors()
    return {name: float(np.real(vec @ S @ vec)) for name, vec in v.items()}


@pytest.mark.parametrize("tau", [0.51, 0.8, 2.0])
def test_ten_moment_reduction_equals_full_recursion(lat, tau):
    kbt = 1e-4
    ts = [3, 10, 37]
    L = 12
    v = lat.obs_vectors()
    for n in ((1, 0, 0), (2, 1, 0), (3, -2, 1)):
        k = lt.kvec_of(n, (L, L, L))
        direct = _direct_powers(lat, k, tau, kbt, ts)
        Sh = lt.hydro_window_covariance(lat, [k], tau, kbt, ts)[0]
        for name, vec in v.items():
            alpha = (lat.E[:10] @ (lat.w * vec)) / lat.b[:10]
            assert np.allclose(lat.E[:10].T @ alpha, vec, atol=1e-14)        # v lies in span{e_0..e_9}
            red = float(np.real(alpha @ Sh @ alpha))
            assert abs(red - direct[name]) <= 1e-12 * max(abs(direct[name]), 1e-20), (n, name, red, direct[name])


def test_symmetry_shortcut_equals_direct_evaluation(lat):
    """Shell averages from orbit representatives equal the direct average over
    every vector of the shell, also for sum_a j_a and sum_{a<b} Pi_ab, which
    are not invariant under sign flips."""
    tau, kbt, L = 0.6, 1e-4, 10
    ts = [4, 9]
    shells = [lt.shell_vectors(n2) for n2 in (1, 3, 5, 9)]
    got = lt.shell_powers(lat, L, shells, tau, kbt, ts)
    for s, sh in enumerate(shells):
        acc = np.zeros(5)
        for n in sh:
            d = _direct_powers(lat, lt.kvec_of(n, (L, L, L)), tau, kbt, ts)
            acc += [d["rho"], (d["jx"] + d["jy"] + d["jz"]) / 3, d["jsum"], d["pdiag"], d["poff"]]
        np.testing.assert_allclose(got[:, s], acc / len(sh), rtol=1e-11)


def test_stationary_limit_is_the_fdt_value(lat):
    """Long after the start the spectra reach the flat equilibrium values
    rho0 k_BT / cs2, rho0 k_BT, 3 rho0 k_BT, 5 rho0 k_BT, rho0 k_BT; shortly
    after it they are still far below (the finite-time target is not 1)."""
    kbt, L = 1e-4, 16
    shells = [lt.shell_vectors(n2) for n2 in (1, 2, 3)]
    flat = np.array([kbt / CS2, kbt, 3 * kbt, 5 * kbt, kbt])[:, None]
    late = lt.shell_powers(lat, L, shells, 1.0, kbt, [6000]) / flat
    np.testing.assert_allclose(late, 1.0, atol=1e-9)
    early = lt.shell_powers(lat, L, shells, 0.51, kbt, [200]) / flat
    assert early[0, 0] < 0.5
