"""Moment storage (the thread-safe formulation of Sec. II) on the GPU.

With storage=STORE_MOMENTS the library keeps the ten hydrodynamic moments of
f(x, t) per node instead of the 27 populations.  The GMF collision depends on
f only through those moments (pinned on the CPU in test_oracle_collision.py),
so the moment trajectory must equal the moments of the oracle's populations at
every step; the checks below compare the raw moments of g = f - w rho0
(rho - rho0, j, Pi - rho0 cs2 I) of the library's state (the second-order
Hermite populations it hands out carry exactly those moments) with the same
moments of the oracle's f.

Tolerances: FP64 1e-11 relative to the largest moment (rounding order only);
FP32 3e-5 per 100 steps (binary32 rounding of the stored moments and the
hardware transcendentals of the normals, as for FP32 populations).
"""

import numpy as np
import pytest

import oracle
from oracle import spectrum as sp
import paper_2601_03806_amd as gmf
from paper_2601_03806_amd import workloads as wl
from gpu_common import oracle_params, say

pytestmark = pytest.mark.gpu

MOM = gmf.STORE_MOMENTS


@pytest.fixture(scope="module")
def tabs():
    return oracle.tables()


def raw_moments(f, tabs, rho0, n):
    """(10, n) raw moments of g = f - w rho0: s0, jx, jy, jz, Pxx, Pyy, Pzz, Pxy, Pxz, Pyz."""
    c = np.asarray(tabs[0], dtype=float)
    g = f.reshape(27, n) - tabs[1][:, None] * rho0
    rows = [np.ones(27), c[:, 0], c[:, 1], c[:, 2], c[:, 0] ** 2, c[:, 1] ** 2, c[:, 2] ** 2,
            c[:, 0] * c[:, 1], c[:, 0] * c[:, 2], c[:, 1] * c[:, 2]]
    return np.stack([r @ g for r in rows])


def moment_err(got, ref, tabs, rho0, n):
    a, b = raw_moments(got, tabs, rho0, n), raw_moments(ref, tabs, rho0, n)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _run_pair(spec, steps, tabs, precision=gmf.FP64, f0=None, graph_steps=0, noise_rho=0):
    say(f"moment storage parity {spec} steps={steps} prec={precision} graph={graph_steps}")
    p = oracle_params(spec, precision=precision, noise_rho=noise_rho)
    f = oracle.rest_state(p) if f0 is None else f0.copy()
    with gmf.Context([spec], precision=precision, graph_steps=graph_steps, noise_rho=noise_rho,
                     storage=MOM) as ctx:
        assert ctx.config()["storage"] == "moments"
        if f0 is not None:
            ctx.set_populations(f0)
        ctx.step(steps)
        got = ctx.get_populations()
    oracle.run(p, f, 0, steps)
    return got, f


def test_moment_storage_fp64_200_steps(tabs):
    """16^3, tau 1, k_B T 1e-4, seed 1, 200 steps from rest."""
    spec = gmf.ReplicaSpec(16, 16, 16, 1.0, 1.0, 1e-4, 1)
    got, ref = _run_pair(spec, 200, tabs)
    assert moment_err(got, ref, tabs, 1.0, spec.n) < 1e-11


@pytest.mark.parametrize("tau", [0.51, 0.8, 2.0])
def test_moment_storage_ragged_random_state_fp64(tabs, tau):
    """Ragged box (partial tiles in x, y and z), a start with ghost content:
    the library keeps only its moments, which is all that the next collision uses."""
    spec = gmf.ReplicaSpec(13, 7, 5, 1.0, tau, 1e-4, 42)
    f0 = wl.perturbed_populations(tabs[1], spec.n, amp=0.05, seed=3, velocity=0.05)
    got, ref = _run_pair(spec, 40, tabs, f0=f0)
    assert moment_err(got, ref, tabs, 1.0, spec.n) < 1e-11


def test_moment_storage_fp32(tabs):
    spec = gmf.ReplicaSpec(16, 16, 16, 1.0, 1.0, 1e-4, 1)
    got, ref = _run_pair(spec, 200, tabs, precision=gmf.FP32_SHIFTED)
    assert moment_err(got, ref, tabs, 1.0, spec.n) < 6e-5
    spec = gmf.ReplicaSpec(13, 7, 5, 1.0, 0.7, 1e-4, 42)
    f0 = wl.perturbed_populations(tabs[1], spec.n, amp=0.01, seed=3, velocity=0.01)
    got, ref = _run_pair(spec, 100, tabs, precision=gmf.FP32_SHIFTED, f0=f0)
    assert moment_err(got, ref, tabs, 1.0, spec.n) < 3e-5


def test_moment_storage_noise_rho0_and_degenerate_boxes(tabs):
    """rho0 in the noise amplitudes; k_B T = 0; boxes of width 1 and 2 in every
    direction, where the haloed tile wraps onto itself."""
    spec = gmf.ReplicaSpec(8, 8, 8, 1.0, 0.6, 1e-4, 9)
    f0 = wl.perturbed_populations(tabs[1], spec.n, amp=0.05, seed=5, velocity=0.05)
    got, ref = _run_pair(spec, 20, tabs, f0=f0, noise_rho=1)
    assert moment_err(got, ref, tabs, 1.0, spec.n) < 1e-11
    for spec in (gmf.ReplicaSpec(1, 16, 1, 1.0, 0.9, 0.0, 1), gmf.ReplicaSpec(1, 1, 1, 1.0, 0.7, 1e-4, 2),
                 gmf.ReplicaSpec(3, 2, 1, 1.3, 1.5, 1e-5, 3), gmf.ReplicaSpec(2, 70, 2, 1.0, 0.8, 1e-4, 4)):
        f0 = wl.perturbed_populations(tabs[1], spec.n, rho0=spec.rho0, amp=0.05, seed=1, velocity=0.05)
        got, ref = _run_pair(spec, 10, tabs, f0=f0)
        assert moment_err(got, ref, tabs, spec.rho0, spec.n) < 1e-11, spec


def test_population_and_moment_storage_agree_fp32(tabs):
    """Same FP32 problem in both storages: the moments agree to binary32 rounding."""
    spec = gmf.ReplicaSpec(24, 20, 18, 1.0, 0.8, 1e-4, 6)
    out = {}
    for st in (gmf.STORE_POPULATIONS, MOM):
        with gmf.Context([spec], precision=gmf.FP32_SHIFTED, storage=st) as ctx:
            ctx.step(100)
            out[st] = ctx.get_populations()
    assert moment_err(out[MOM], out[gmf.STORE_POPULATIONS], tabs, 1.0, spec.n) < 3e-5


@pytest.mark.parametrize("prec", [gmf.FP64, gmf.FP32_SHIFTED])
def test_tilings_bitwise(monkeypatch, prec):
    """Every tile shape, tile depth and workgroup mapping gives the same bits:
    each node's arithmetic (its collision, and the order in which the three
    z slices of incoming populations are summed) does not depend on the tiling."""
    spec = gmf.ReplicaSpec(70, 37, 45, 1.0, 0.7, 1e-4, 13)
    ref = None
    tiles = ("64x8", "32x16", "32x8", "64x16")
    for tile in range(4):
        if prec == gmf.FP64 and tile == 3:
            continue                     # 64x16 needs more LDS than a CU has in FP64
        for tz in (16, 32, 128):
            for bmap in ("linear", "xcd", "xcd16"):
                monkeypatch.setenv("GMF_MTILE", f"{tile},{tz}")
                monkeypatch.setenv("GMF_BLOCK_MAP", bmap)
                with gmf.Context([spec], precision=prec, storage=MOM) as ctx:
                    cfg = ctx.config()
                    ctx.step(12)
                    got = ctx.get_populations()
                say(f"tiling {cfg['tile']} {cfg['block_map']}")
                assert cfg["tile"] == f"{tiles[tile]}x{tz}"   # the forced tiling is the one that ran
                if ref is None:
                    ref = got
                else:
                    assert np.array_equal(got, ref), (tile, tz, bmap)


def test_graph_batched_and_checkpoint_bitwise():
    specs = [gmf.ReplicaSpec(16, 12, 10, 1.0, 0.6, 1e-4, 7), gmf.ReplicaSpec(33, 9, 20, 1.0, 1.3, 1e-4, 8),
             gmf.ReplicaSpec(5, 70, 3, 1.0, 0.9, 1e-4, 9)]
    out = []
    for gs in (0, 8, 64):
        say(f"moment storage graph_steps={gs}")
        with gmf.Context(specs, precision=gmf.FP32_SHIFTED, graph_steps=gs, storage=MOM) as ctx:
            ctx.step(3)
            ctx.step(77)
            out.append([ctx.get_populations(r) for r in range(3)])
    for r in range(3):
        assert np.array_equal(out[0][r], out[1][r]) and np.array_equal(out[0][r], out[2][r])
        with gmf.Context([specs[r]], precision=gmf.FP32_SHIFTED, storage=MOM) as ctx:
            ctx.step(80)
            assert np.array_equal(ctx.get_populations(), out[0][r]), r
    # checkpoint: the handed-out populations carry the whole moment state
    with gmf.Context(specs[:1], precision=gmf.FP32_SHIFTED, storage=MOM) as ctx:
        ctx.step(50)
        snap = ctx.get_populations()
    with gmf.Context(specs[:1], precision=gmf.FP32_SHIFTED, storage=MOM) as ctx:
        ctx.step(50)
        ctx.set_populations(snap)
        assert np.array_equal(ctx.get_populations(), snap)
        ctx.step(30)
        assert np.array_equal(ctx.get_populations(), out[0][0])


def test_host_interface_moments_nodes_and_conservation(tabs):
    spec = gmf.ReplicaSpec(16, 16, 16, 1.0, 0.55, 1e-4, 2)
    f0 = wl.perturbed_populations(tabs[1], spec.n, amp=0.02, seed=2, velocity=0.02)
    p = oracle_params(spec)
    ref_tot = oracle.totals(p, f0)
    for prec, tol in ((gmf.FP64, 1e-12), (gmf.FP32_SHIFTED, 1e-5)):
        say(f"moment storage host interface prec={prec}")
        with gmf.Context([spec], precision=prec, storage=MOM) as ctx:
            ctx.set_populations(f0)
            back = ctx.get_populations()
            # the moments of f0 survive (FP32: rounded once to binary32)
            assert moment_err(back, f0, tabs, 1.0, spec.n) < (1e-14 if prec == gmf.FP64 else 1e-6)
            s0 = ctx.stats()
            assert abs(s0["mass"] - ref_tot[0]) < tol * ref_tot[0]
            for _ in range(5):
                ctx.step(20)
                s = ctx.stats()
                assert abs(s["mass"] - s0["mass"]) < tol * s0["mass"]
                assert np.all(np.abs(s["momentum"] - s0["momentum"]) < tol * s0["mass"])
            rho, u = ctx.moments()
            f = ctx.get_populations()
            nodes = wl.sample_nodes(spec.n, 50, seed=1)
            sub = ctx.get_nodes(nodes)
        assert np.array_equal(sub, f.reshape(27, spec.n)[:, nodes].T)
        orho, ou = oracle.moments(p, f)
        assert np.max(np.abs(rho - orho)) < 1e-13
        assert np.max(np.abs(u - ou)) < 1e-13


@pytest.mark.parametrize("box", [(12, 10, 8), (130, 5, 4)])
def test_moment_storage_sampler_matches_oracle(box):
    """Observables, variances and shell spectra sampled from the moment state
    equal the oracle's brute-force observables of the same populations."""
    spec = gmf.ReplicaSpec(*box, 1.0, 0.6, 1e-4, 5)
    p = oracle_params(spec)
    f = oracle.rest_state(p)
    say(f"moment storage sampler vs oracle {box}")
    with gmf.Context([spec], precision=gmf.FP64, sample_every=25, storage=MOM) as ctx:
        ctx.step(101)
        st = ctx.stats()
    N = spec.n
    exp_msq = np.zeros(10)
    exp_var = np.zeros(10)
    exp_spec = np.zeros((5, 8))
    t_prev = 0
    for t in (0, 25, 50, 75, 100):
        oracle.run(p, f, t_prev, t - t_prev)
        t_prev = t
        sums, spec_o = oracle.observables(p, f)
        m, m2 = sums[:, 0] / N, sums[:, 1] / N
        exp_msq += m2
        exp_var += m2 - m * m
        exp_spec += spec_o
    assert st["nsamples"] == 5
    np.testing.assert_allclose(st["sum_var"], exp_var, rtol=1e-10, atol=1e-20)
    np.testing.assert_allclose(st["sum_meansq"], exp_msq, rtol=1e-10, atol=1e-20)
    np.testing.assert_allclose(st["spectrum"], exp_spec, rtol=1e-9, atol=1e-20)


def test_moment_storage_full_spectrum_matches_oracle():
    spec = gmf.ReplicaSpec(20, 18, 12, 1.0, 0.8, 1e-4, 3)
    say("moment storage full spectrum")
    with gmf.Context([spec], precision=gmf.FP64, sample_every=20, spectrum=1, storage=MOM) as ctx:
        ctx.step(40)
        ctx.reset_stats()
        f40 = ctx.get_populations()
        ctx.step(1)
        got, cnt = ctx.spectrum()
    ref, rcnt = sp.full_spectrum(oracle_params(spec), f40)
    assert np.array_equal(cnt, rcnt)
    assert np.max(np.abs(got - ref) / np.max(np.abs(ref), axis=1, keepdims=True)) < 1e-12


def _neighbour(n, c, spec):
    x = n % spec.nx
    y = (n // spec.nx) % spec.ny
    z = n // (spec.nx * spec.ny)
    return ((x + c[0]) % spec.nx) + spec.nx * (((y + c[1]) % spec.ny) + spec.ny * ((z + c[2]) % spec.nz))


def _sampled_moment_check(ctx, spec, tabs, precision, count, seed):
    """One library step checked at sampled nodes x: the oracle collides the 27
    neighbours x - c_i (their populations from the library, with the node
    index and step of each) and streams population i into x; returns the
    largest deviation of the library's moments of x from those of that
    f(x, t + 1), relative to the largest such moment."""
    vel = tabs[0]
    t = ctx.t
    nodes = wl.sample_nodes(spec.n, count, seed=seed)
    src = np.array([[_neighbour(int(n), -np.asarray(vel[i]), spec) for i in range(27)] for n in nodes])
    before = ctx.get_nodes(src.ravel()).reshape(len(nodes), 27, 27)
    ctx.step(1)
    after = ctx.get_nodes(nodes)
    p = oracle_params(spec, precision=precision)
    worst, scale = 0.0, 0.0
    for j in range(len(nodes)):
        fx = np.array([oracle.collide(before[j, i], p, node=int(src[j, i]), step=t)[i] for i in range(27)])
        a = raw_moments(after[j], tabs, spec.rho0, 1)
        r = raw_moments(fx, tabs, spec.rho0, 1)
        worst = max(worst, float(np.max(np.abs(a - r))))
        scale = max(scale, float(np.max(np.abs(r))))
    return worst / scale


@pytest.mark.parametrize("precision,tol", [(gmf.FP32_SHIFTED, 3e-5), (gmf.FP64, 1e-12)])
def test_full_size_sampled_nodes_vs_oracle(tabs, precision, tol):
    """256^3, tau 0.8, k_BT 1e-4, seed 1, autotuned tiling and graph step loop
    (the benchmark's configuration): after 64 steps, one more step checked at
    100 sampled nodes against the oracle's collisions of their neighbours."""
    w = wl.bandwidth_headline("fp32" if precision == gmf.FP32_SHIFTED else "fp64")
    b = w.boxes[0]
    spec = gmf.ReplicaSpec(*b.n, rho0=b.rho0, tau=b.tau, kbt=b.kbt, seed=b.seed)
    say(f"moment storage full-size sampled parity {w.name}")
    with gmf.Context([spec], precision=precision, storage=MOM, tune=1) as ctx:
        say(f"  config {ctx.config()}")
        ctx.step(64)
        err = _sampled_moment_check(ctx, spec, tabs, precision, 100, seed=2)
    say(f"  max moment error {err:.2e}")
    assert err < tol


def test_largest_box_1024cube_with_sampling(tabs):
    """1024^3 (1.07e9 nodes; two 43 GB moment buffers and 26 GB of sampled
    fields), FP32, sampled every 2 steps: every offset past 2^32 bytes in the
    tile kernel and the host-interface kernels; sampled nodes match the
    oracle's collisions; mass and momentum are conserved; the sampled density
    variance is positive and finite after the first steps from rest."""
    spec = gmf.ReplicaSpec(1024, 1024, 1024, 1.0, 0.8, 1e-4, 3)
    say("1024^3 moment storage FP32 with sampling")
    with gmf.Context([spec], precision=gmf.FP32_SHIFTED, sample_every=2, storage=MOM) as ctx:
        s0 = ctx.stats()
        ctx.step(5)
        err = _sampled_moment_check(ctx, spec, tabs, gmf.FP32_SHIFTED, 60, seed=4)
        s1 = ctx.stats()
    say(f"  max moment error {err:.2e}")
    assert err < 3e-5, err
    assert abs(s1["mass"] - s0["mass"]) < 1e-6 * s0["mass"]
    assert np.all(np.abs(s1["momentum"]) < 1e-6 * s0["mass"])
    assert s1["nsamples"] == 3 and np.isfinite(s1["sum_var"]).all() and s1["sum_var"][0] > 0


def test_moment_storage_option_errors():
    spec = gmf.ReplicaSpec(8, 8, 8, 1.0, 1.0, 1e-4, 1)
    for kw in ({"collision": gmf.COLLISION_BGK}, {"streaming": gmf.STREAM_AA}):
        with pytest.raises(gmf.GmfError):
            gmf.Context([spec], storage=MOM, **kw)


@pytest.mark.slow
def test_moment_storage_tau_sweep_statistics():
    """64^3 at tau in {0.51, 0.6, 1, 2, 5}, k_B T = 1e-4, 2000 warm-up + 20000
    steps sampled every 10: the FP32 moment-storage variances and shell spectra
    are within 1% of FP64 population storage with the same seeds (paired noise),
    the bar that FP32 population storage meets."""
    w32 = wl.tau_sweep("fp32")
    specs = [gmf.ReplicaSpec(*b.n, rho0=b.rho0, tau=b.tau, kbt=b.kbt, seed=b.seed) for b in w32.boxes]
    out = {}
    for prec, st in ((gmf.FP32_SHIFTED, MOM), (gmf.FP64, gmf.STORE_POPULATIONS)):
        say(f"moment storage tau sweep prec={prec} storage={st}")
        with gmf.Context(specs, precision=prec, sample_every=w32.sample_every, storage=st) as ctx:
            ctx.step(w32.warmup)
            ctx.reset_stats()
            ctx.step(w32.steps)
            out[st] = [ctx.stats(r) for r in range(len(specs))]
    for r, s in enumerate(specs):
        a, b = out[MOM][r], out[gmf.STORE_POPULATIONS][r]
        assert a["nsamples"] == b["nsamples"] == w32.steps // w32.sample_every
        ratio = (a["sum_var"] / a["nsamples"]) / (b["sum_var"] / b["nsamples"])
        sratio = a["spectrum"] / b["spectrum"]
        say(f"  tau={s.tau}: variance ratios {np.round(ratio, 4)}; spectra {sratio.min():.4f}..{sratio.max():.4f}")
        assert np.all(np.abs(ratio - 1) < 0.01), (s.tau, ratio)
        assert np.all(np.abs(sratio - 1) < 0.01), (s.tau, sratio)
