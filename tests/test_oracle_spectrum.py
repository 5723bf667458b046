"""Pins of the oracle's full-box shell spectra (oracle/spectrum.py), from what
the mathematics fixes: exact shell membership and counts by enumeration, a
single Fourier mode landing in one shell with its closed-form power,
Parseval's identity over all shells, and agreement with the oracle's
independent brute-force DFT (gmf_oracle.c) on the shells both cover."""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import spectrum as sp
from paper_2601_03806_amd import workloads as wl


def _brute_counts(nx, ny, nz):
    """Enumerate every integer vector of the box and round |n| by an integer test."""
    def freqs(L):
        return [i if 2 * i < L else i - L for i in range(L)]
    cnt = {}
    for a, b, c in itertools.product(freqs(nx), freqs(ny), freqs(nz)):
        n2 = a * a + b * b + c * c
        if n2 == 0:
            continue
        s = 0
        while not ((2 * s - 1) ** 2 <= 4 * n2 < (2 * s + 1) ** 2):
            s += 1
        cnt[s] = cnt.get(s, 0) + 1
    return cnt


@pytest.mark.parametrize("box", [(8, 8, 8), (9, 8, 7), (12, 10, 6), (5, 1, 3), (16, 4, 2)])
def test_shell_counts_by_enumeration(box):
    cnt = sp.shell_counts(*box)
    brute = _brute_counts(*box)
    assert cnt.sum() == box[0] * box[1] * box[2] - 1
    assert {s: int(v) for s, v in enumerate(cnt) if v} == brute


def test_small_shells_of_a_cube():
    cnt = sp.shell_counts(8, 8, 8)
    # shell 1: |n|^2 in {1, 2}; shell 2: |n|^2 in {3, 4, 5, 6}
    assert cnt[1] == 6 + 12 and cnt[2] == 8 + 6 + 24 + 24


def _state_from_density(p, drho):
    """f_i = w_i (rho0 + drho(x)): a pure density perturbation at rest."""
    w = oracle.tables()[1]
    return np.ascontiguousarray((w[:, None] * (p.rho0 + drho.reshape(1, -1))).reshape(-1))


@pytest.mark.parametrize("n0", [(1, 0, 0), (2, 1, 0), (3, 2, 2), (0, -4, 1)])
def test_single_mode_lands_in_its_shell(n0):
    nx, ny, nz = 12, 10, 9
    p = oracle.params(nx, ny, nz, rho0=1.0)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    A = 1e-3
    phase = 2 * np.pi * (n0[0] * x / nx + n0[1] * y / ny + n0[2] * z / nz)
    drho = A * np.cos(phase)
    out, cnt = sp.full_spectrum(p, _state_from_density(p, drho))
    N = nx * ny * nz
    s0 = int(math.floor(math.sqrt(sum(v * v for v in n0)) + 0.5))
    expect = np.zeros(len(cnt))
    # cos splits into +n0 and -n0, each with |m(k)|^2 = N A^2 / 4
    expect[s0] = 2 * (N * A * A / 4) / cnt[s0]
    np.testing.assert_allclose(out[0], expect, rtol=1e-12, atol=1e-22)
    # at rest with f = w (rho0 + drho): pdiag = 3 cs^2 drho = drho, no momentum, no shear stress
    np.testing.assert_allclose(out[3], expect, rtol=1e-12, atol=1e-22)
    for m in (1, 2, 4):
        assert np.max(np.abs(out[m])) < 1e-28


def test_parseval_over_all_shells():
    """sum_s count_s S_m(s) = sum_x (m - mean m)^2 for every spectrum: no wave
    vector is dropped or counted twice."""
    nx, ny, nz = 10, 9, 8
    p = oracle.params(nx, ny, nz, rho0=1.0)
    w = oracle.tables()[1]
    f = wl.perturbed_populations(w, nx * ny * nz, amp=0.05, seed=3, velocity=0.05)
    out, cnt = sp.full_spectrum(p, f)
    fl = sp.fields(p, f)

    def var_sum(v):
        return float(np.sum((v - v.mean()) ** 2))
    jsum = fl["jx"] + fl["jy"] + fl["jz"]
    expect = [var_sum(fl["drho"]), (var_sum(fl["jx"]) + var_sum(fl["jy"]) + var_sum(fl["jz"])) / 3,
              var_sum(jsum), var_sum(fl["pdiag"]), var_sum(fl["poff"])]
    for m in range(5):
        assert math.isclose(float(np.sum(cnt * out[m])), expect[m], rel_tol=1e-12)


def test_agrees_with_brute_force_dft_on_common_shells():
    """The C oracle's direct DFT averages the shells |n|^2 = 1, 2, 3, 4, 5, 6;
    rounded shell 1 is |n|^2 in {1, 2} and rounded shell 2 is {3, 4, 5, 6}."""
    nx, ny, nz = 9, 8, 7
    p = oracle.params(nx, ny, nz, rho0=1.0, tau=0.7, kbt=1e-4, seed=5)
    w = oracle.tables()[1]
    f = wl.perturbed_populations(w, nx * ny * nz, amp=0.05, seed=11, velocity=0.05)
    oracle.run(p, f, 0, 3)
    out, cnt = sp.full_spectrum(p, f)
    _, brute = oracle.observables(p, f)          # (5, 8) at |n|^2 = 1, 2, 3, 4, 5, 6, 8, 9
    mult = {1: 6, 2: 12, 3: 8, 4: 6, 5: 24, 6: 24}
    idx = {n2: i for i, n2 in enumerate(oracle.SHELL_N2)}
    for shell, members in ((1, (1, 2)), (2, (3, 4, 5, 6))):
        total = sum(mult[n2] for n2 in members)
        assert cnt[shell] == total
        expect = sum(mult[n2] * brute[:, idx[n2]] for n2 in members) / total
        np.testing.assert_allclose(out[:, shell], expect, rtol=1e-11)


def test_brute_force_dft_matches_numpy_fft_on_every_exact_shell():
    """The C oracle's direct DFT against numpy's orthonormal FFT, restricted to
    exactly the integer vectors of each shell |n|^2 = 1, 2, 3, 4, 5, 6, 8, 9
    (8: the 12 vectors (+-2, +-2, 0) and permutations; 9: (+-3, 0, 0) and
    (+-2, +-2, +-1) and permutations, 30 in all).  Every box length is at
    least 7, so +-3 are distinct frequencies."""
    nx, ny, nz = 9, 8, 7
    N = nx * ny * nz
    p = oracle.params(nx, ny, nz, rho0=1.0, tau=0.7, kbt=1e-4, seed=5)
    w = oracle.tables()[1]
    f = wl.perturbed_populations(w, N, amp=0.05, seed=17, velocity=0.05)
    oracle.run(p, f, 0, 2)
    _, brute = oracle.observables(p, f)
    fl = sp.fields(p, f)
    jsum = fl["jx"] + fl["jy"] + fl["jz"]

    def power(v):
        # fields are x-fastest: reshape to (z, y, x) before the FFT
        return np.abs(np.fft.fftn(v.reshape(nz, ny, nx), norm="ortho")) ** 2
    pw = {"rho": power(fl["drho"]), "jx": power(fl["jx"]), "jy": power(fl["jy"]), "jz": power(fl["jz"]),
          "jsum": power(jsum), "pdiag": power(fl["pdiag"]), "poff": power(fl["poff"])}
    expected_counts = {1: 6, 2: 12, 3: 8, 4: 6, 5: 24, 6: 24, 8: 12, 9: 30}
    for s, n2 in enumerate(oracle.SHELL_N2):
        vecs = [v for v in itertools.product(range(-3, 4), repeat=3) if v[0] ** 2 + v[1] ** 2 + v[2] ** 2 == n2]
        assert len(vecs) == expected_counts[n2]
        idx = tuple(np.array([(c % nz, b % ny, a % nx) for a, b, c in vecs]).T)
        expect = [pw["rho"][idx].mean(), (pw["jx"][idx] + pw["jy"][idx] + pw["jz"][idx]).mean() / 3,
                  pw["jsum"][idx].mean(), pw["pdiag"][idx].mean(), pw["poff"][idx].mean()]
        np.testing.assert_allclose(brute[:, s], expect, rtol=1e-11, err_msg=f"|n|^2 = {n2}")
