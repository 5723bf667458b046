"""GPU parity of the fused stream+collide step against the FP64 oracle.

Tolerances:
  FP64: 1e-11 relative on g = f - w rho0 after 200 steps (the two sides differ
        only in rounding order and in last-ulp libm differences of the normals);
  FP32 shifted: 2e-5 relative on g per 100 steps (binary32 rounding of O(1e-2)
        shifted populations plus the hardware log2/sqrt/sin/cos of the normals).
"""
import numpy as np
import pytest

import oracle
import paper_2601_03806_amd as gmf
from paper_2601_03806_amd import workloads as wl
from gpu_common import oracle_params, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def w():
    return oracle.tables()[1]


def _run_pair(spec, steps, w, precision=gmf.FP64, collision=gmf.COLLISION_GMF, f0=None, graph_steps=0,
              noise_rho=0):
    say(f"parity {spec} steps={steps} prec={precision} coll={collision} graph={graph_steps}")
    p = oracle_params(spec, collision, precision, noise_rho)
    f = oracle.rest_state(p) if f0 is None else f0.copy()
    with gmf.Context([spec], precision=precision, collision=collision, graph_steps=graph_steps,
                     noise_rho=noise_rho) as ctx:
        if f0 is not None:
            ctx.set_populations(f0)
        ctx.step(steps)
        got = ctx.get_populations()
    oracle.run(p, f, 0, steps)
    return got, f


def test_noise_words_bit_identical():
    for seed, step, node0 in ((1, 0, 0), (0xDEADBEEFCAFEF00D, (3 << 32) + 17, 4000000000)):
        say(f"noise words seed={seed} step={step} node0={node0}")
        words, _ = gmf.noise_probe(seed, step, node0, 512)
        for j in range(0, 512, 7):
            for b in range(6):
                ref = oracle.noise_words(seed, node0 + j, step, b)
                assert np.array_equal(words[j, b], ref), (j, b)


def test_noise_normals_fp64_and_fp32():
    say("noise normals")
    _, r64 = gmf.noise_probe(5, 123, 77, 2000, gmf.FP64)
    _, r32 = gmf.noise_probe(5, 123, 77, 2000, gmf.FP32_SHIFTED)
    ref64 = np.array([oracle.normals(5, 77 + j, 123, 32)[4:] for j in range(2000)])
    ref23 = np.array([oracle.normals(5, 77 + j, 123, 23)[4:] for j in range(2000)])
    # FP64: the oracle's libm and the library's own log and sin/cos differ in the last bits only.
    # Error budget per Box-Muller pair of radius R: the oracle rounds 2 pi u2 before cos/sin
    # (|fl(2 pi) - 2 pi| + half an ulp of the angle <= 6.9e-16 rad), the radius (log within
    # 1 and 2 ulp, sqrt and -2 ln u rounded on each side) <= 3.9e-16 R, sin/cos (libm within
    # 1 ulp, the library's series within 2.5e-16) <= 3.6e-16, and the final product 2.2e-16 R:
    # |dr| <= 1.7e-15 R.  A per-value ulp bound cannot hold: near a zero of cos the angle's
    # rounding alone is many ulps of r.  The host build of the same functions measures
    # 8.6e-16 R at most over 8M pairs.
    # radius of the pair that feeds each r_k, from the oracle's words: r_{4+4j}, r_{5+4j} use
    # word 0 of block j, r_{6+4j}, r_{7+4j} word 2 (r_26 is the cosine half of block 5's second pair)
    words = np.array([[oracle.noise_words(5, 77 + n, 123, j) for j in range(6)] for n in range(2000)])
    radius = np.sqrt(-2.0 * np.log((words[:, :, [0, 0, 2, 2]].astype(np.float64) + 0.5) * 2.0 ** -32))
    radius = radius.reshape(2000, 24)[:, :23]
    assert np.all(np.abs(r64 - ref64) <= 1.7e-15 * radius), np.max(np.abs(r64 - ref64) / radius)
    # FP32: the same uniforms, hardware transcendentals
    assert np.max(np.abs(r32 - ref23)) < 5e-5 * np.max(np.abs(ref23))


def test_parity_small_fp64_200_steps(w):
    """16^3, tau = 1, k_B T = 1e-4, seed 1, 200 steps from rest (plain FP64)."""
    spec = gmf.ReplicaSpec(16, 16, 16, 1.0, 1.0, 1e-4, 1)
    got, ref = _run_pair(spec, 200, w)
    assert rel_err(got, ref, w, 1.0, spec.n) < 1e-11


@pytest.mark.parametrize("tau", [0.51, 0.8, 2.0])
@pytest.mark.parametrize("collision", [gmf.COLLISION_GMF, gmf.COLLISION_BGK])
def test_parity_ragged_random_state_fp64(w, tau, collision):
    """Ragged box (several workgroups, partial last one), random non-equilibrium start."""
    spec = gmf.ReplicaSpec(13, 7, 5, 1.0, tau, 1e-4, 42)
    f0 = wl.perturbed_populations(w, spec.n, amp=0.05, seed=3, velocity=0.05)
    got, ref = _run_pair(spec, 40, w, collision=collision, f0=f0)
    assert rel_err(got, ref, w, 1.0, spec.n) < 1e-11


@pytest.mark.parametrize("collision", [gmf.COLLISION_GMF, gmf.COLLISION_BGK])
def test_parity_ragged_random_state_fp32(w, collision):
    spec = gmf.ReplicaSpec(13, 7, 5, 1.0, 0.7, 1e-4, 42)
    f0 = wl.perturbed_populations(w, spec.n, amp=0.01, seed=3, velocity=0.01)
    got, ref = _run_pair(spec, 100, w, precision=gmf.FP32_SHIFTED, collision=collision, f0=f0)
    assert rel_err(got, ref, w, 1.0, spec.n) < 2e-5


def test_parity_small_fp32_200_steps(w):
    spec = gmf.ReplicaSpec(16, 16, 16, 1.0, 1.0, 1e-4, 1)
    got, ref = _run_pair(spec, 200, w, precision=gmf.FP32_SHIFTED)
    assert rel_err(got, ref, w, 1.0, spec.n) < 4e-5


def test_parity_noise_rho0_option(w):
    spec = gmf.ReplicaSpec(8, 8, 8, 1.0, 0.6, 1e-4, 9)
    f0 = wl.perturbed_populations(w, spec.n, amp=0.05, seed=5, velocity=0.05)
    got, ref = _run_pair(spec, 20, w, f0=f0, noise_rho=1)
    assert rel_err(got, ref, w, 1.0, spec.n) < 1e-11


def test_no_noise_and_degenerate_boxes(w):
    """k_B T = 0 (deterministic regularised BGK) and 1-wide boxes (every pull wraps)."""
    for spec in (gmf.ReplicaSpec(1, 16, 1, 1.0, 0.9, 0.0, 1), gmf.ReplicaSpec(1, 1, 1, 1.0, 0.7, 1e-4, 2),
                 gmf.ReplicaSpec(3, 2, 1, 1.3, 1.5, 1e-5, 3)):
        f0 = wl.perturbed_populations(w, spec.n, rho0=spec.rho0, amp=0.05, seed=1, velocity=0.05)
        got, ref = _run_pair(spec, 10, w, f0=f0)
        assert rel_err(got, ref, w, spec.rho0, spec.n) < 1e-11


def test_graph_equals_direct_bitwise():
    spec = gmf.ReplicaSpec(16, 12, 10, 1.0, 0.6, 1e-4, 7)
    out = []
    for gs in (0, 8, 64):
        say(f"graph_steps={gs}")
        with gmf.Context([spec], precision=gmf.FP32_SHIFTED, graph_steps=gs) as ctx:
            ctx.step(3)       # leave the first graph replay unaligned
            ctx.step(77)
            assert ctx.t == 80
            out.append(ctx.get_populations())
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])


def test_addressing_modes_bitwise(monkeypatch):
    """Plane-uniform and per-node addressing with storage groups of 27, 3 and 1
    give bit-identical trajectories (the layout changes, the arithmetic does
    not); so do the workgroup mappings, the occupancy caps and the autotuner's
    choice."""
    spec = gmf.ReplicaSpec(16, 32, 6, 1.0, 0.6, 1e-4, 21)      # plane of 512 nodes: every mode fits
    for prec in (gmf.FP64, gmf.FP32_SHIFTED):
        out = {}
        for mode in ("", "plane", "27", "3", "1"):
            monkeypatch.setenv("GMF_ADDRESSING", mode)
            say(f"addressing mode={mode or 'default'} prec={prec}")
            with gmf.Context([spec], precision=prec) as ctx:
                cfg = ctx.config()
                assert cfg["addressing"] == ("group27" if mode == "" else (mode if mode == "plane" else f"group{mode}"))
                ctx.step(12)
                out[mode] = ctx.get_populations()
        monkeypatch.delenv("GMF_ADDRESSING")
        # workgroups mapped to contiguous block ranges per XCD
        for bmap in ("xcd", "xcd16"):
            monkeypatch.setenv("GMF_BLOCK_MAP", bmap)
            for mode in ("plane", "27"):
                monkeypatch.setenv("GMF_ADDRESSING", mode)
                say(f"addressing mode={mode} block map {bmap} prec={prec}")
                with gmf.Context([spec], precision=prec) as ctx:
                    ctx.step(12)
                    out[bmap + mode] = ctx.get_populations()
        monkeypatch.delenv("GMF_ADDRESSING")
        monkeypatch.delenv("GMF_BLOCK_MAP")
        with gmf.Context([spec], precision=prec, tune=1) as ctx:
            ctx.step(12)
            out["tuned"] = ctx.get_populations()
        # occupancy caps of the step kernel (LDS reserved at launch)
        for cap in ("5", "4", "3"):
            monkeypatch.setenv("GMF_OCCUPANCY", cap)
            say(f"occupancy cap {cap} prec={prec}")
            with gmf.Context([spec], precision=prec) as ctx:
                assert ctx.config()["workgroups_per_cu"] == int(cap)
                ctx.step(12)
                out["occ" + cap] = ctx.get_populations()
        monkeypatch.delenv("GMF_OCCUPANCY")
        for mode in ("plane", "27", "3", "1", "xcdplane", "xcd27", "xcd16plane", "xcd1627", "tuned", "occ5", "occ4",
                     "occ3"):
            assert np.array_equal(out[""], out[mode]), mode


def test_batched_equals_single_bitwise():
    specs = [gmf.ReplicaSpec(16, 16, 16, 1.0, 0.51, 1e-4, 1), gmf.ReplicaSpec(12, 9, 7, 1.0, 2.0, 1e-4, 2),
             gmf.ReplicaSpec(32, 32, 32, 1.0, 0.8, 1e-4, 3)]
    for prec in (gmf.FP64, gmf.FP32_SHIFTED):
        say(f"batched vs single prec={prec}")
        with gmf.Context(specs, precision=prec) as ctx:
            ctx.step(30)
            batched = [ctx.get_populations(r) for r in range(len(specs))]
        for r, s in enumerate(specs):
            with gmf.Context([s], precision=prec) as ctx:
                ctx.step(30)
                assert np.array_equal(ctx.get_populations(), batched[r]), r


def test_checkpoint_resume_bitwise():
    spec = gmf.ReplicaSpec(16, 16, 16, 1.0, 0.7, 1e-4, 11)
    say("checkpoint/resume")
    with gmf.Context([spec], precision=gmf.FP64) as ctx:
        ctx.step(40)
        straight = ctx.get_populations()
    with gmf.Context([spec], precision=gmf.FP64) as ctx:
        ctx.step(25)
        snap = ctx.get_populations()
    with gmf.Context([spec], precision=gmf.FP64) as ctx:
        ctx.step(25)            # same step index, state overwritten by the snapshot
        ctx.set_populations(snap)
        ctx.step(15)
        assert np.array_equal(ctx.get_populations(), straight)


def test_get_set_roundtrip_and_nodes(w):
    spec = gmf.ReplicaSpec(9, 10, 11, 1.0, 0.9, 1e-4, 4)
    f0 = wl.perturbed_populations(w, spec.n, amp=0.05, seed=8)
    for prec in (gmf.FP64, gmf.FP32_SHIFTED):
        say(f"roundtrip prec={prec}")
        with gmf.Context([spec], precision=prec) as ctx:
            ctx.set_populations(f0)
            back = ctx.get_populations()
            if prec == gmf.FP64:
                assert np.array_equal(back, f0)
            else:
                assert np.max(np.abs(back - f0)) < 1e-8
            nodes = wl.sample_nodes(spec.n, 50, seed=1)
            sub = ctx.get_nodes(nodes)
            assert np.array_equal(sub, back.reshape(27, spec.n)[:, nodes].T)


def test_moments_and_conservation(w):
    spec = gmf.ReplicaSpec(16, 16, 16, 1.0, 0.55, 1e-4, 2)
    f0 = wl.perturbed_populations(w, spec.n, amp=0.02, seed=2, velocity=0.02)
    p = oracle_params(spec)
    ref_tot = oracle.totals(p, f0)
    for prec, tol, tol0 in ((gmf.FP64, 1e-12, 1e-13), (gmf.FP32_SHIFTED, 1e-5, 1e-6)):
        say(f"conservation prec={prec}")
        with gmf.Context([spec], precision=prec) as ctx:
            ctx.set_populations(f0)
            s0 = ctx.stats()
            for _ in range(5):
                ctx.step(20)
                s = ctx.stats()
                assert abs(s["mass"] - s0["mass"]) < tol * s0["mass"]
                assert np.all(np.abs(s["momentum"] - s0["momentum"]) < tol * s0["mass"])
            rho, u = ctx.moments()
            f = ctx.get_populations()
        # FP32 stores g = f - w rho0 rounded to binary32: the initial mass moves by ~1e-8
        assert abs(s0["mass"] - ref_tot[0]) < tol0 * ref_tot[0]
        orho, ou = oracle.moments(p, f)
        assert np.max(np.abs(rho - orho)) < 1e-13
        assert np.max(np.abs(u - ou)) < 1e-13


@pytest.mark.parametrize("box", [(12, 10, 8), (600, 3, 2), (130, 5, 4), (20, 130, 6)])
def test_sampled_statistics_match_oracle(w, box):
    """The fused sampler (observables, spatial variances, shell spectra) equals
    the oracle's brute-force observables of the same states; 600-wide rows take
    the first DFT stage through three passes of columns, 130-wide rows one
    plane per workgroup in one pass, and 130 rows in y are 33, 33, 33 and 31
    rows of the four wavefronts of a first-stage workgroup."""
    spec = gmf.ReplicaSpec(*box, 1.0, 0.6, 1e-4, 5)
    p = oracle_params(spec)
    f = oracle.rest_state(p)
    say(f"sampler vs oracle {box}")
    with gmf.Context([spec], precision=gmf.FP64, sample_every=25) as ctx:
        ctx.step(101)            # samples at t = 0, 25, 50, 75, 100
        st = ctx.stats()
    N = spec.n
    exp_mean = np.zeros(10)
    exp_msq = np.zeros(10)
    exp_var = np.zeros(10)
    exp_spec = np.zeros((5, 8))
    t_prev = 0
    for t in (0, 25, 50, 75, 100):
        oracle.run(p, f, t_prev, t - t_prev)
        t_prev = t
        sums, spec_o = oracle.observables(p, f)
        m, m2 = sums[:, 0] / N, sums[:, 1] / N
        exp_mean += m
        exp_msq += m2
        exp_var += m2 - m * m
        exp_spec += spec_o
    assert st["nsamples"] == 5
    np.testing.assert_allclose(st["sum_var"], exp_var, rtol=1e-10, atol=1e-20)
    np.testing.assert_allclose(st["sum_meansq"], exp_msq, rtol=1e-10, atol=1e-20)
    # spatial means of conserved quantities are roundoff-sized: absolute tolerance
    np.testing.assert_allclose(st["sum_mean"], exp_mean, rtol=1e-8, atol=1e-12)
    np.testing.assert_allclose(st["spectrum"], exp_spec, rtol=1e-9, atol=1e-20)


@pytest.mark.parametrize("storage", [gmf.STORE_POPULATIONS, gmf.STORE_MOMENTS])
@pytest.mark.parametrize("box", [(70, 130, 9), (12, 10, 8)])
def test_sampled_statistics_fp32_match_oracle_observables(w, box, storage):
    """The FP32 sampler (the first DFT stage with the observables in one
    kernel, then the z stage, the shell sums and the statistics) against the
    oracle's brute-force observables of the very states it sampled (read back
    as FP64 before each sampling step): they differ only by the FP32 moments
    the sampling step forms (about 1e-7 of each field), so variances, mean
    squares and the eight-shell spectra agree to 1e-5 relative.  70 x 130 rows
    take two column blocks of 64, one partly empty, and 130 rows split 33, 33,
    33, 31 over the four wavefronts; 12 x 10 x 8 puts five planes in one
    workgroup; moment storage forms the fields from the ten stored moments."""
    spec = gmf.ReplicaSpec(*box, 1.0, 0.6, 1e-4, 9)
    p = oracle_params(spec)
    N = spec.n
    exp_mean = np.zeros(10)
    exp_msq = np.zeros(10)
    exp_var = np.zeros(10)
    exp_spec = np.zeros((5, 8))
    say(f"FP32 sampler vs oracle observables {box} storage {storage}")
    with gmf.Context([spec], precision=gmf.FP32_SHIFTED, sample_every=25, storage=storage) as ctx:
        for t in (0, 25, 50, 75, 100):
            assert ctx.t == t
            sums, spec_o = oracle.observables(p, ctx.get_populations())
            m, m2 = sums[:, 0] / N, sums[:, 1] / N
            exp_mean += m
            exp_msq += m2
            exp_var += m2 - m * m
            exp_spec += spec_o
            ctx.step(25 if t < 100 else 1)
        st = ctx.stats()
    assert st["nsamples"] == 5
    np.testing.assert_allclose(st["sum_var"], exp_var, rtol=1e-5, atol=1e-20)
    np.testing.assert_allclose(st["sum_meansq"], exp_msq, rtol=1e-5, atol=1e-20)
    # spatial means of conserved quantities are roundoff-sized: absolute tolerance
    np.testing.assert_allclose(st["sum_mean"], exp_mean, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(st["spectrum"], exp_spec, rtol=1e-5, atol=1e-20)


def test_error_paths_on_device():
    import ctypes
    spec = gmf.ReplicaSpec(8, 8, 8, 1.0, 0.8, 1e-4, 1)
    lib = gmf.lib()
    with gmf.Context([spec]) as ctx:
        buf = np.zeros(4 * spec.n)
        dp = buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        assert lib.gmf_moments(ctx._h, 1, dp, dp) == gmf.GMF_EINVAL       # replica out of range
        assert lib.gmf_moments(ctx._h, -1, dp, dp) == gmf.GMF_EINVAL
        with pytest.raises(gmf.GmfError) as e:
            ctx.get_nodes([spec.n])                                         # node out of range
        assert e.value.code == gmf.GMF_EINVAL
        with pytest.raises(gmf.GmfError) as e:
            ctx.step(-1)
        assert e.value.code == gmf.GMF_EINVAL
        ctx.step(0)
        assert ctx.t == 0
        # the context still works after rejected calls
        ctx.step(3)
        assert ctx.t == 3 and np.isfinite(ctx.stats()["mass"])


def test_nan_injection_reports_unstable(w):
    spec = gmf.ReplicaSpec(8, 8, 8, 1.0, 0.8, 1e-4, 1)
    f0 = wl.perturbed_populations(w, spec.n, amp=0.01, seed=1)
    f0[5 * spec.n + 17] = np.nan
    with gmf.Context([spec], sample_every=1) as ctx:
        ctx.set_populations(f0)
        ctx.step(2)
        with pytest.raises(gmf.GmfError) as e:
            ctx.stats()
        assert e.value.code == gmf.GMF_EUNSTABLE


def test_tune_cache(tmp_path, monkeypatch):
    """GMF_TUNE_CACHE: an entry whose parameters do not fit is ignored and the
    tuner appends its choice; a second context with the same boxes takes the
    cached choice without timing again and reproduces the trajectory bit for
    bit, for population and moment storage."""
    cache = tmp_path / "tune.txt"
    # unfit entries (addressing mode 99, tile 7) and a line of an older format
    cache.write_text("v4p1c0s0_24x20x18 99 1 1 0 0\nm3p1_24x20x18 7 64 1 0 0\nv4p1c0s0_24x20x18 27 1 1\n")
    monkeypatch.setenv("GMF_TUNE_CACHE", str(cache))
    spec = gmf.ReplicaSpec(24, 20, 18, 1.0, 0.8, 1e-4, 6)
    for storage in (gmf.STORE_POPULATIONS, gmf.STORE_MOMENTS):
        say(f"tune cache storage={storage}")
        runs = []
        for _ in range(2):
            before = cache.read_text().splitlines()
            with gmf.Context([spec], precision=gmf.FP32_SHIFTED, tune=1, storage=storage) as ctx:
                cfg = ctx.config()
                ctx.step(10)
                runs.append((cfg, ctx.get_populations(), len(cache.read_text().splitlines()) - len(before)))
        assert runs[0][2] == 1 and runs[1][2] == 0, (runs[0][2], runs[1][2])   # timed once, then cached
        assert runs[0][0] == runs[1][0]
        assert np.array_equal(runs[0][1], runs[1][1])


@pytest.mark.parametrize("precision", [gmf.FP64, gmf.FP32_SHIFTED])
def test_conservation_guard(w, precision):
    """gmf_stats measures mass and momentum drift from the replica's reference
    (taken at init and at every set_populations, as stored) and reports
    GMF_EUNSTABLE past the bound on a finite state.  The drift is forced
    through set_populations: a second state with more mass replaces the first,
    and the first state's reference is restored, as a resume of the first run
    would do."""
    spec = gmf.ReplicaSpec(12, 10, 9, 1.0, 0.7, 1e-4, 3)
    say(f"conservation guard prec={precision}")
    bound = 1e-10 if precision == gmf.FP64 else 1e-4
    with gmf.Context([spec], precision=precision) as ctx:
        st = ctx.stats()
        assert st["drift"] == 0.0 and st["drift_bound"] == bound
        assert abs(st["mass_ref"] - spec.n) < 1e-9 * spec.n
        ctx.step(30)
        st = ctx.stats()
        assert st["drift"] < (1e-13 if precision == gmf.FP64 else 1e-6), st["drift"]
        f0 = wl.perturbed_populations(w, spec.n, amp=0.05, seed=2, velocity=0.05)
        ctx.set_populations(f0)
        st0 = ctx.stats()
        assert st0["drift"] == 0.0 and st0["mass_ref"] == st0["mass"]
        assert np.array_equal(st0["momentum_ref"], st0["momentum"])
        ref0 = np.array([st0["mass_ref"], *st0["momentum_ref"]])
        ctx.step(20)
        assert ctx.stats()["drift"] < (1e-13 if precision == gmf.FP64 else 1e-6)
        # a state with 1% more mass: its own reference, so no drift ...
        ctx.set_populations(1.01 * f0)
        assert ctx.stats()["drift"] == 0.0
        # ... until the first run's reference comes back
        ctx.set_reference(ref0)
        with pytest.raises(gmf.GmfError) as e:
            ctx.stats()
        assert e.value.code == gmf.GMF_EUNSTABLE
        st = ctx.stats(allow_unstable=True)
        assert st["nonfinite"] == 0 and np.isfinite(st["mass"])
        assert abs(st["drift"] - 0.01) < 1e-3 and st["drift"] > bound
        # re-baseline on the current state: stable again
        ctx.set_reference()
        assert ctx.stats()["drift"] == 0.0
        # invalid references and replicas
        for bad in ([0.0, 0, 0, 0], [np.nan, 0, 0, 0], [1.0, np.inf, 0, 0]):
            with pytest.raises(gmf.GmfError) as e:
                ctx.set_reference(bad)
            assert e.value.code == gmf.GMF_EINVAL
        with pytest.raises(gmf.GmfError) as e:
            ctx.set_reference(None, r=1)
        assert e.value.code == gmf.GMF_EINVAL


@pytest.mark.parametrize("every,gs", [(3, 8), (0, 7), (100001, 64), (1, 4)])
def test_prepare_captures_every_graph(every, gs):
    """gmf_prepare captures every graph a run launches, so the run itself
    captures none; graphs never exceed graph_steps steps, whatever the sampling
    cadence (a very long odd cadence included); the trajectory and the
    accumulators equal direct launches bit for bit."""
    spec = gmf.ReplicaSpec(10, 8, 6, 1.0, 0.6, 1e-4, 8)
    say(f"prepare sample_every={every} graph_steps={gs}")
    out = []
    for g in (0, gs):
        with gmf.Context([spec], precision=gmf.FP32_SHIFTED, sample_every=every, graph_steps=g) as ctx:
            ctx.step(5)
            ctx.prepare(131)
            before = ctx.launch_counts()
            ctx.step(131)
            after = ctx.launch_counts()
            assert after["graphs_captured"] == before["graphs_captured"] <= 6
            assert after["graph_steps"] + after["direct_steps"] == 136
            if g:
                assert after["graph_launches"] > 0
                assert after["graph_steps"] - before["graph_steps"] <= g * (after["graph_launches"] - before["graph_launches"])
            else:
                assert after["graph_launches"] == 0 and after["graphs_captured"] == 0
            st = ctx.stats()
            out.append((ctx.get_populations(), st["sum_var"], st["spectrum"], st["nsamples"]))
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)
