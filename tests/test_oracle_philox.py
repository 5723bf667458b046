"""Pins of the oracle's noise generator.

Philox4x32-10 is checked against a third-party implementation, rocRAND's
engine (header-only source of the ROCm installation, compiled for the host
with g++: tests/c/rocrand_philox_ref.cpp), word for word, including the
counter layout (node, step low word, block, step high word) of the noise
words; also against a pure-Python implementation of the SC'11 description
(Salmon, Moraes, Dror, Shaw), the counter and key layout against its
definition, and the words for uniformity.  The Box-Muller normals
are checked for their distribution and against the transform written out from
the words.  (The device generator is checked word for word against the oracle
in the GPU tests.)
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle

MASK = 0xFFFFFFFF


def philox_ref(ctr, key, rounds=10):
    """Philox4x32 as described in the SC'11 paper, written with Python ints."""
    m0, m1 = 0xD2511F53, 0xCD9E8D57
    w0, w1 = 0x9E3779B9, 0xBB67AE85
    x = [int(v) for v in ctr]
    k = [int(v) for v in key]
    for r in range(rounds):
        if r:
            k = [(k[0] + w0) & MASK, (k[1] + w1) & MASK]
        p0 = m0 * x[0]
        p1 = m1 * x[2]
        x = [((p1 >> 32) ^ x[1] ^ k[0]) & MASK, p1 & MASK, ((p0 >> 32) ^ x[3] ^ k[1]) & MASK, p0 & MASK]
    return x


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCRAND = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    """Path of the rocRAND-engine reference program, built with g++."""
    if not os.path.exists(ROCRAND) or shutil.which("g++") is None:
        pytest.skip("rocRAND headers or g++ not available")
    exe = str(tmp_path_factory.mktemp("rocrand") / "philox_ref")
    subprocess.run(["g++", "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    os.path.join(ROOT, "tests", "c", "rocrand_philox_ref.cpp"), "-o", exe], check=True)
    return exe


def _rocrand_words(exe, cases):
    """cases: (seed, c0, c1, c2, c3) with c1 < 2^30 -> list of 4-word lists."""
    text = "".join(" ".join(str(int(v)) for v in c) + "\n" for c in cases)
    run = subprocess.run([exe], input=text, capture_output=True, text=True, timeout=60, check=True)
    return [[int(v) for v in line.split()] for line in run.stdout.strip().split("\n")]


def test_philox_matches_rocrand_engine(rocrand_ref):
    rng = np.random.default_rng(7)
    cases = [(0, 0, 0, 0, 0), (1, 0, 0, 0, 0), (2 ** 64 - 1, 2 ** 32 - 1, 2 ** 30 - 1, 2 ** 32 - 1, 2 ** 32 - 1)]
    for _ in range(200):
        cases.append((int(rng.integers(0, 2 ** 63)) * 2 + int(rng.integers(0, 2)), int(rng.integers(0, 2 ** 32)),
                      int(rng.integers(0, 2 ** 30)), int(rng.integers(0, 2 ** 32)), int(rng.integers(0, 2 ** 32))))
    ref = _rocrand_words(rocrand_ref, cases)
    for c, r in zip(cases, ref):
        key = np.array([c[0] & MASK, c[0] >> 32], np.uint32)
        assert list(map(int, oracle.philox(np.array(c[1:], np.uint32), key))) == r, c


def test_noise_words_layout_matches_rocrand_engine(rocrand_ref):
    """The noise words of (seed, node, step, block) are Philox4x32-10 at counter
    (node, step mod 2^32, block, step div 2^32): steps below and above 2^32."""
    picks = [(1, 0, 0, 0), (42, 4095, 199, 5), (2 ** 40 + 3, 2 ** 31 + 7, 2 ** 32 + 11, 3),
             (2 ** 64 - 1, 2 ** 32 - 1, 5 * 2 ** 32 + 2 ** 29, 1)]
    cases = [(s, n, t & MASK, b, t >> 32) for s, n, t, b in picks]
    ref = _rocrand_words(rocrand_ref, cases)
    for (s, n, t, b), r in zip(picks, ref):
        assert list(map(int, oracle.noise_words(s, n, t, b))) == r, (s, n, t, b)


def test_philox_matches_independent_implementation():
    rng = np.random.default_rng(0)
    for _ in range(300):
        ctr = rng.integers(0, 2 ** 32, size=4, dtype=np.uint64)
        key = rng.integers(0, 2 ** 32, size=2, dtype=np.uint64)
        got = oracle.philox(ctr.astype(np.uint32), key.astype(np.uint32))
        assert list(map(int, got)) == philox_ref(ctr, key)
    # edge words
    for ctr in ([0, 0, 0, 0], [MASK] * 4, [1, 0, 0, 0]):
        for key in ([0, 0], [MASK, MASK]):
            assert list(map(int, oracle.philox(ctr, key))) == philox_ref(ctr, key)


def test_noise_counter_layout():
    """Counter = (node, step_lo, block, step_hi), key = (seed_lo, seed_hi)."""
    seed = 0x0123456789ABCDEF
    step = (7 << 32) + 5
    for block in range(6):
        got = oracle.noise_words(seed, 1234, step, block)
        ref = philox_ref([1234, 5, block, 7], [seed & MASK, seed >> 32])
        assert list(map(int, got)) == ref


def test_philox_bits_uniform():
    words = np.array([oracle.noise_words(1, n, 0, 0) for n in range(4000)], dtype=np.uint64).ravel()
    bits = ((words[:, None] >> np.arange(32, dtype=np.uint64)) & 1).astype(float)
    frac = bits.mean(axis=0)
    se = 0.5 / np.sqrt(len(words))
    assert np.all(np.abs(frac - 0.5) < 5 * se)
    # avalanche: flipping one counter bit flips about half the output bits
    flips = []
    for n in range(500):
        a = np.array(oracle.noise_words(3, n, 11, 2), dtype=np.uint64)
        b = np.array(oracle.noise_words(3, n ^ 1, 11, 2), dtype=np.uint64)
        flips.append(sum(bin(int(v)).count("1") for v in (a ^ b)))
    assert abs(np.mean(flips) - 64) < 2.0


@pytest.mark.parametrize("bits", [32, 23])
def test_normals_distribution(bits):
    rs = np.array([oracle.normals(9, n, 17, bits)[4:] for n in range(6000)])  # (6000, 23)
    x = rs.ravel()
    assert abs(x.mean()) < 5 / np.sqrt(x.size)
    assert abs(x.var() - 1.0) < 5 * np.sqrt(2.0 / x.size)
    assert stats.kstest(x, "norm").pvalue > 1e-4
    # different moments are uncorrelated
    c = np.corrcoef(rs.T)
    off = c[~np.eye(23, dtype=bool)]
    assert np.max(np.abs(off)) < 5 / np.sqrt(rs.shape[0])


def test_normals_zero_for_conserved_and_keyed():
    r = oracle.normals(1, 5, 6)
    assert np.all(r[:4] == 0)
    assert not np.array_equal(r, oracle.normals(2, 5, 6))
    assert not np.array_equal(r, oracle.normals(1, 6, 6))
    assert not np.array_equal(r, oracle.normals(1, 5, 7))
    assert np.array_equal(r, oracle.normals(1, 5, 6))


def test_box_muller_pairs_from_words():
    """r_{4+4j}, r_{5+4j} come from words (x0, x1) of block j, r_{6+4j}, r_{7+4j}
    from (x2, x3): radius sqrt(-2 ln U1), angle 2 pi U2 with U = (x + 1/2) 2^-32."""
    seed, node, step = 77, 3, 4
    r = oracle.normals(seed, node, step)
    for j in range(6):
        w = oracle.noise_words(seed, node, step, j).astype(float)
        for p in range(2):
            u1 = (w[2 * p] + 0.5) / 2 ** 32
            u2 = (w[2 * p + 1] + 0.5) / 2 ** 32
            rad = np.sqrt(-2 * np.log(u1))
            k = 4 + 4 * j + 2 * p
            assert abs(r[k] - rad * np.cos(2 * np.pi * u2)) < 1e-14
            if k + 1 < 27:
                assert abs(r[k + 1] - rad * np.sin(2 * np.pi * u2)) < 1e-14
