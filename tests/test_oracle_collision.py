"""Pins of the oracle's collision (Sec. II, Eqs. (10)-(13), and Eq. (1) for BGK).

Checks against closed forms and linear algebra, not against the oracle itself:
equilibrium moments, the filter as a projector, the omega = 1 special case,
the moment-space reading, and the fluctuation-dissipation fixed point.
"""
import numpy as np
import pytest

import oracle
import lintheory as lt

CS2 = 1.0 / 3.0


@pytest.fixture(scope="module")
def tabs():
    return oracle.tables()


def _random_state(rng, w, amp=0.05):
    """Populations near a moving equilibrium (all positive)."""
    return w * (1.0 + amp * rng.uniform(-1, 1, size=27)) * rng.uniform(0.9, 1.1)


@pytest.mark.parametrize("seed", range(5))
def test_feq_moments(tabs, seed):
    """Eq. (11): sum f^eq = rho, sum f^eq c = rho u, sum f^eq cc = rho uu + rho cs2 I."""
    vel, *_ = tabs
    c = vel.astype(float)
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 1.5)
    u = rng.uniform(-0.1, 0.1, 3)
    fe = oracle.feq(rho, u)
    assert abs(fe.sum() - rho) < 1e-15 * rho
    np.testing.assert_allclose(c.T @ fe, rho * u, atol=1e-15)
    pi = np.einsum("i,ia,ib->ab", fe, c, c)
    np.testing.assert_allclose(pi, rho * np.outer(u, u) + rho * CS2 * np.eye(3), atol=2e-15)


def _hermite_moments(e, f):
    return e @ f


@pytest.mark.parametrize("tau", [0.51, 0.8, 1.0, 2.0, 5.0])
def test_deterministic_moments(tabs, tau):
    """k_BT = 0: conserved moments kept, stress relaxed by (1-omega) about rho uu,
    ghost moments exactly removed (Sec. II filtering)."""
    vel, w, e, b, *_ = tabs
    c = vel.astype(float)
    rng = np.random.default_rng(int(tau * 100))
    om = 1.0 / tau
    for _ in range(10):
        f = _random_state(rng, w)
        p = oracle.params(1, tau=tau, kbt=0.0)
        fs = oracle.collide(f, p)
        m, ms = e @ f, e @ fs
        np.testing.assert_allclose(ms[:4], m[:4], atol=1e-15)
        rho = f.sum()
        u = (c.T @ f) / rho
        # Hermite second-order coefficients: diag k=4..6 and off-diag k=7..9
        uu = rho * np.array([u[0] * u[0], u[1] * u[1], u[2] * u[2], u[0] * u[1], u[0] * u[2], u[1] * u[2]])
        np.testing.assert_allclose(ms[4:10], uu + (1 - om) * (m[4:10] - uu), atol=1e-15)
        np.testing.assert_allclose(ms[10:], 0.0, atol=2e-16)


def test_omega_one_gives_equilibrium(tabs):
    """tau = 1, k_BT = 0: f* = f^eq(rho, u) (textbook BGK with omega = 1)."""
    vel, w, *_ = tabs
    c = vel.astype(float)
    rng = np.random.default_rng(7)
    for coll in (oracle.GMF, oracle.BGK):
        for _ in range(10):
            f = _random_state(rng, w)
            fs = oracle.collide(f, oracle.params(1, tau=1.0, kbt=0.0, collision=coll))
            rho = f.sum()
            np.testing.assert_allclose(fs, oracle.feq(rho, (c.T @ f) / rho), atol=5e-16, rtol=0)


def test_filter_is_projector(tabs):
    """omega = 0 (tau = inf), k_BT = 0 gives the filter P_h(f) = f^eq + f^neq_(2):
    P_h(P_h f) = P_h f and P_h f^eq = f^eq."""
    vel, w, *_ = tabs
    c = vel.astype(float)
    rng = np.random.default_rng(11)
    p = oracle.params(1, tau=float("inf"), kbt=0.0)
    for _ in range(20):
        f = _random_state(rng, w, amp=0.3)
        pf = oracle.collide(f, p)
        ppf = oracle.collide(pf, p)
        assert np.max(np.abs(ppf - pf)) < 1e-15
        rho = f.sum()
        fe = oracle.feq(rho, (c.T @ f) / rho)
        assert np.max(np.abs(oracle.collide(fe, p) - fe)) < 1e-15


def test_filter_matches_hydrodynamic_projector(tabs):
    """P_h is the w-orthogonal projector on span{e_0..e_9} (linear algebra)."""
    vel, w, *_ = tabs
    lat = lt.Lattice(vel)
    Eh = lat.E[:10]
    P = (w[:, None] * Eh.T) @ np.diag(1 / lat.b[:10]) @ Eh
    np.testing.assert_allclose(P @ P, P, atol=1e-15)
    rng = np.random.default_rng(3)
    p = oracle.params(1, tau=float("inf"), kbt=0.0)
    for _ in range(10):
        f = _random_state(rng, w, amp=0.3)
        # for f near rest the nonlinear terms cancel exactly in f^eq + f^neq_(2):
        # f^eq carries rho uu in its 2nd moment and f^neq_(2) carries a2 - rho uu
        np.testing.assert_allclose(oracle.collide(f, p), P @ f, atol=2e-16)


@pytest.mark.parametrize("tau", [0.51, 0.8, 2.0])
def test_gmf_collision_ignores_ghost_content(tabs, tau):
    """Eq. (10) keeps no deterministic ghost content: adding any combination of
    the ghost vectors w_i e_ki (k = 10..26) to f, which leaves rho, j and Pi
    unchanged, leaves f* unchanged (noise included), so the ten hydrodynamic
    moments of f are the whole state the GMF update depends on.  BGK (Eq. (1))
    relaxes the ghosts and does not have this property."""
    vel, w, e, b, *_ = tabs
    rng = np.random.default_rng(int(tau * 100))
    c = vel.astype(float)
    for node in range(6):
        f = _random_state(rng, w)
        ghost = (w[:, None] * e[10:].T) @ rng.normal(scale=1e-3, size=17)
        # the ghost directions carry no mass, momentum or stress
        np.testing.assert_allclose([ghost.sum(), *(c.T @ ghost)], 0.0, atol=1e-17)
        np.testing.assert_allclose(np.einsum("ia,ib,i->ab", c, c, ghost), 0.0, atol=1e-17)
        pg = oracle.params(1, tau=tau, kbt=1e-4, seed=7)
        a = oracle.collide(f, pg, node=node, step=5)
        g = oracle.collide(f + ghost, pg, node=node, step=5)
        assert np.max(np.abs(a - g)) < 1e-15
        pb = oracle.params(1, tau=tau, kbt=1e-4, seed=7, collision=oracle.BGK)
        assert np.max(np.abs(oracle.collide(f, pb, node=node, step=5) - oracle.collide(f + ghost, pb, node=node, step=5))) > 1e-6


@pytest.mark.parametrize("coll", [oracle.GMF, oracle.BGK])
@pytest.mark.parametrize("tau", [0.51, 0.7, 1.0, 3.0])
def test_moment_space_reading_agrees(tabs, coll, tau):
    vel, w, *_ = tabs
    rng = np.random.default_rng(int(tau * 10) + coll)
    p = oracle.params(1, tau=tau, kbt=1e-3, seed=99, collision=coll)
    for node in range(8):
        f = _random_state(rng, w)
        a = oracle.collide(f, p, node=node, step=3)
        b = oracle.collide(f, p, node=node, step=3, moment_space=True)
        assert np.max(np.abs(a - b)) < 1e-14 * np.max(np.abs(a))


def test_noise_enters_only_nonconserved_modes(tabs):
    vel, w, e, b, *_ = tabs
    rng = np.random.default_rng(5)
    f = _random_state(rng, w)
    p0 = oracle.params(1, tau=0.8, kbt=0.0)
    p1 = oracle.params(1, tau=0.8, kbt=1e-4, seed=17)
    d = e @ (oracle.collide(f, p1, 4, 9) - oracle.collide(f, p0, 4, 9))
    np.testing.assert_allclose(d[:4], 0.0, atol=2e-16)
    assert np.all(np.abs(d[4:]) > 0)


@pytest.mark.parametrize("coll", [oracle.GMF, oracle.BGK])
@pytest.mark.parametrize("tau", [0.55, 1.0, 2.0])
def test_fdt_fixed_point_one_step(tabs, coll, tau):
    """Fluctuation-dissipation fixed point: with delta f_i ~ N(0, mu w_i) i.i.d.
    (mu = rho0 k_BT / cs2) the post-collision state has the same covariance,
    mode by mode: <dm_k^2> = mu b_k for every k (linear theory; the noise
    amplitudes of Eqs. (2) and (9) are exactly what makes this hold)."""
    vel, w, e, b, *_ = tabs
    L = 24
    kbt = 1e-7
    mu = kbt / CS2
    N = L ** 3
    rng = np.random.default_rng(1234 + int(10 * tau) + coll)
    f = w[:, None] + np.sqrt(mu * w)[:, None] * rng.standard_normal((27, N))
    f = np.ascontiguousarray(f.reshape(-1))
    p = oracle.params(L, tau=tau, kbt=kbt, seed=5, collision=coll)
    oracle.run(p, f, 0, 1)
    g = f.reshape(27, N) - w[:, None]
    m = e @ g                     # (27, N) moments of the post-stream state
    var = (m ** 2).mean(axis=1) / (mu * b)
    se = np.sqrt(2.0 / N)
    assert np.all(np.abs(var - 1.0) < 5 * se), var
    # and the lattice-wide linear theory says the product Gaussian is stationary
    lat = lt.Lattice(vel)
    C = lat.collision(tau, bgk=(coll == oracle.BGK))
    Qn = lat.noise_cov(tau, kbt, bgk=(coll == oracle.BGK))
    S0 = mu * np.diag(w)
    np.testing.assert_allclose(C @ S0 @ C.T + Qn, S0, atol=1e-14 * mu)


@pytest.mark.parametrize("coll", [oracle.GMF, oracle.BGK])
@pytest.mark.parametrize("tau", [0.55, 1.0, 3.0])
def test_noise_rho_option_scales_amplitudes(tabs, coll, tau):
    """Eqs. (2) and (9) carry the density under a square root.  With noise_rho = 0
    the local rho of Eq. (3) enters, with noise_rho = 1 the reference rho0.  The
    noise part of f* (f* at k_BT > 0 minus f* at k_BT = 0, same node and step)
    is linear in the amplitudes, so mode by mode:
      noise(noise_rho = 1) = sqrt(rho0 / rho) * noise(noise_rho = 0),
    and under noise_rho = 1 it does not depend on the local density at all."""
    vel, w, e, b, *_ = tabs
    rng = np.random.default_rng(int(tau * 100) + 7 * coll)
    rho0 = 1.3
    for node, target in enumerate((0.55, 0.9, 1.2, 1.45, 1.8, 2.6)):
        f = _random_state(rng, w)
        f *= target / f.sum()               # local rho far from rho0
        rho = f.sum()
        det = oracle.collide(f, oracle.params(1, rho0=rho0, tau=tau, kbt=0.0, collision=coll), node, 11)

        def noise_part(nr, ff, fdet):
            p = oracle.params(1, rho0=rho0, tau=tau, kbt=2e-4, seed=23, collision=coll, noise_rho=nr)
            return e @ (oracle.collide(ff, p, node, 11) - fdet)      # moments k = 0..26
        m_loc = noise_part(0, f, det)
        m_ref = noise_part(1, f, det)
        # differences of O(rho) populations: rounding leaves ~1e-16 * rho in every moment
        tol = 4e-16 * rho
        np.testing.assert_allclose(m_loc[:4], 0.0, atol=tol)
        np.testing.assert_allclose(m_ref[:4], 0.0, atol=tol)
        np.testing.assert_allclose(m_ref[4:], np.sqrt(rho0 / rho) * m_loc[4:], rtol=1e-12, atol=tol)
        # a node with another local density: the rho0 noise is unchanged, the local one scales with sqrt(rho)
        s = 1.37
        det2 = oracle.collide(s * f, oracle.params(1, rho0=rho0, tau=tau, kbt=0.0, collision=coll), node, 11)
        np.testing.assert_allclose(noise_part(1, s * f, det2)[4:], m_ref[4:], rtol=1e-12, atol=s * tol)
        np.testing.assert_allclose(noise_part(0, s * f, det2)[4:], np.sqrt(s) * m_loc[4:], rtol=1e-12, atol=s * tol)
