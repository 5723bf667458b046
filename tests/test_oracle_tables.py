"""Pins of the oracle's Table I / Table II constants.

The oracle writes the Hermite vectors from the printed group formulas of
Table II; here they are rebuilt independently as tensor products of the D1Q3
Hermite functions (exact rationals) and checked against the printed b_k,
n_k, mu_k (tests/golden/table2_basis.txt) and the lattice isotropy conditions.
"""
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
import lintheory as lt

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_rows(name):
    rows = []
    with open(os.path.join(GOLD, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


@pytest.fixture(scope="module")
def tabs():
    return oracle.tables()


def test_velocity_set_groups(tabs):
    vel, w, e, b, nk, mu = tabs
    got = {tuple(v) for v in vel}
    assert got == set(lt.all_velocities())
    c2 = (vel ** 2).sum(axis=1)
    # Table I grouping: 0 rest, 1-6 faces, 7-18 edges, 19-26 corners
    assert c2[0] == 0 and (c2[1:7] == 1).all() and (c2[7:19] == 2).all() and (c2[19:] == 3).all()


def test_weights_match_table1(tabs):
    vel, w, *_ = tabs
    table = {int(r[0]): Fr(r[2]) for r in _read_rows("table1_weights.txt")}
    for i, v in enumerate(vel):
        assert w[i] == float(table[int((v ** 2).sum())])


def test_weights_isotropy(tabs):
    """Textbook isotropy of D3Q27 up to fourth order with c_s^2 = 1/3."""
    vel, w, *_ = tabs
    c = vel.astype(float)
    cs2 = 1.0 / 3.0
    assert abs(w.sum() - 1.0) < 1e-15
    np.testing.assert_allclose(np.einsum("i,ia->a", w, c), 0.0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, c, c), cs2 * np.eye(3), atol=1e-15)
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic->abc", w, c, c, c), 0.0, atol=1e-16)
    d = np.eye(3)
    iso4 = cs2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                       + np.einsum("ad,bc->abcd", d, d))
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c), iso4, atol=1e-15)


def test_weights_factorise(tabs):
    vel, w, *_ = tabs
    for i, v in enumerate(vel):
        assert w[i] == float(lt.weight(tuple(v)))


def test_basis_equals_tensor_products(tabs):
    vel, w, e, *_ = tabs
    for k in range(27):
        for i, v in enumerate(vel):
            assert abs(e[k, i] - float(lt.basis_vector(k, tuple(v)))) < 1e-15, (k, i)


def test_basis_orthogonality_exact(tabs):
    """sum_i w_i e_ki e_li = b_k delta_kl in exact rationals (tensor-product form)."""
    vel = [tuple(v) for v in tabs[0]]
    for k in range(27):
        for l in range(k, 27):
            s = sum(lt.weight(c) * lt.basis_vector(k, c) * lt.basis_vector(l, c) for c in vel)
            assert s == (lt.norm(k) if k == l else 0), (k, l)


def test_norms_match_table2(tabs):
    vel, w, e, b, nk, mu = tabs
    for r in _read_rows("table2_basis.txt"):
        k0, k1, n, m, bk = int(r[0]), int(r[1]), int(r[2]), int(r[3]), Fr(r[4])
        for k in range(k0, k1 + 1):
            assert nk[k] == n and mu[k] == m
            assert abs(b[k] - float(bk)) < 1e-16
            assert lt.norm(k) == bk
            # Sec. II relation b_k = n_k! cs^(2 n_k) / mu_k
            fact = 1
            for q in range(2, n + 1):
                fact *= q
            assert Fr(fact) * Fr(1, 3) ** n / m == bk


def test_hydrodynamic_ghost_split(tabs):
    """k = 0..9 are the Hermite tensors of order <= 2, k = 10..26 the ghosts."""
    for k in range(27):
        order = sum(lt.ABC[k])
        assert (order <= 2) == (k <= 9)
    assert (tabs[4][:10] <= 2).all() and (tabs[4][10:] >= 3).all()
