"""Full-box shell spectra on the device against the oracle's FFT reference
(oracle/spectrum.py): per sample, the oracle transforms the canonical state
that the library holds at the sampled step; the library's accumulated shell
averages must equal the oracle's sums over the same samples.  Also: the
integer shell sums make the spectra reproducible bit for bit (graph against
direct launches, batched against single replicas), and the equilibrium
spectra of a 64^3 box are flat at their fluctuation-dissipation values."""
import numpy as np
import pytest

import oracle
from oracle import spectrum as sp
import paper_2601_03806_amd as gmf
from paper_2601_03806_amd import workloads as wl
from gpu_common import oracle_params, say

pytestmark = pytest.mark.gpu

CS2 = 1.0 / 3.0


@pytest.fixture(scope="module")
def w():
    return oracle.tables()[1]


def _sampled_run(specs, prec, every, nsamples, f0s=None, graph_steps=0):
    """Sample at t = 0, every, 2 every, ...; return the library's spectra and
    the canonical states at the sampled steps."""
    states = [[] for _ in specs]
    with gmf.Context(specs, precision=prec, sample_every=every, spectrum=1, graph_steps=graph_steps) as ctx:
        if f0s is not None:
            for r, f0 in enumerate(f0s):
                ctx.set_populations(f0, r)
        for _ in range(nsamples):
            for r in range(len(specs)):
                states[r].append(ctx.get_populations(r))
            ctx.step(every)
        st = [ctx.stats(r) for r in range(len(specs))]
        out = [ctx.spectrum(r) for r in range(len(specs))]
    for s in st:
        assert s["nsamples"] == nsamples
    return out, states


def _oracle_sums(spec, prec, states):
    p = oracle_params(spec, precision=prec)
    tot = None
    for f in states:
        s, cnt = sp.full_spectrum(p, f)
        tot = s if tot is None else tot + s
    return tot, cnt


@pytest.mark.parametrize("prec,rtol", [(gmf.FP64, 1e-12), (gmf.FP32_SHIFTED, 1e-6)])
def test_full_spectrum_matches_oracle(w, prec, rtol):
    specs = [gmf.ReplicaSpec(12, 10, 8, 1.0, 0.7, 1e-4, 3), gmf.ReplicaSpec(16, 4, 2, 1.0, 1.3, 1e-4, 4),
             gmf.ReplicaSpec(5, 6, 3, 1.0, 0.55, 1e-4, 5), gmf.ReplicaSpec(1, 8, 4, 1.0, 2.0, 1e-4, 6)]
    f0s = [wl.perturbed_populations(w, s.n, amp=0.03, seed=10 + r, velocity=0.03) for r, s in enumerate(specs)]
    say(f"full spectrum vs oracle prec={prec}")
    out, states = _sampled_run(specs, prec, 5, 5, f0s)
    for r, s in enumerate(specs):
        got, cnt = out[r]
        ref, rcnt = _oracle_sums(s, prec, states[r])
        assert np.array_equal(cnt, rcnt), r
        scale = np.max(np.abs(ref), axis=1, keepdims=True)
        err = np.max(np.abs(got - ref) / scale)
        say(f"  replica {r} {s.nx}x{s.ny}x{s.nz}: max rel err {err:.2e}")
        assert err < rtol, (r, err)


def test_full_spectrum_bitwise_graph_and_batched():
    specs = [gmf.ReplicaSpec(12, 10, 8, 1.0, 0.7, 1e-4, 3), gmf.ReplicaSpec(20, 9, 6, 1.0, 0.9, 1e-4, 8)]
    res = {}
    for gs in (0, 10):
        say(f"full spectrum graph={gs}")
        with gmf.Context(specs, precision=gmf.FP32_SHIFTED, sample_every=5, spectrum=1, graph_steps=gs) as ctx:
            ctx.step(40)
            res[gs] = [ctx.spectrum(r)[0] for r in range(2)]
    for r in range(2):
        assert np.array_equal(res[0][r], res[10][r]), r
    for r, s in enumerate(specs):
        with gmf.Context([s], precision=gmf.FP32_SHIFTED, sample_every=5, spectrum=1) as ctx:
            ctx.step(40)
            assert np.array_equal(ctx.spectrum()[0], res[0][r]), r
    # reset clears them
    with gmf.Context(specs, precision=gmf.FP32_SHIFTED, sample_every=5, spectrum=1) as ctx:
        ctx.step(10)
        ctx.reset_stats()
        assert not np.any(ctx.spectrum(1)[0])


def test_spectrum_option_errors():
    with gmf.Context([gmf.ReplicaSpec(8, 8, 8, 1.0, 1.0, 1e-4, 1)], sample_every=5) as ctx:
        with pytest.raises(gmf.GmfError):
            ctx.spectrum()


@pytest.mark.slow
def test_equilibrium_spectra_are_flat():
    """64^3, tau 1, k_B T 1e-4: after 2000 warm-up steps, 1000 samples (every
    10 steps) of the shell spectra equal the equilibrium values rho0 k_BT / cs2
    (density), rho0 k_BT (j), 3 rho0 k_BT (jsum), 5 rho0 k_BT (pdiag) and
    rho0 k_BT (poff) at every shell s = 4 .. 32 within 3%, and on average
    within 1%."""
    kbt = 1e-4
    spec = gmf.ReplicaSpec(64, 64, 64, 1.0, 1.0, kbt, 1)
    flat = np.array([kbt / CS2, kbt, 3 * kbt, 5 * kbt, kbt])[:, None]
    for prec in (gmf.FP32_SHIFTED, gmf.FP64):
        say(f"equilibrium spectra prec={prec}")
        with gmf.Context([spec], precision=prec, sample_every=10, spectrum=1) as ctx:
            ctx.step(2000)
            ctx.reset_stats()
            ctx.step(10000)
            nsamp = ctx.stats()["nsamples"]
            sums, cnt = ctx.spectrum()
        er = sums[:, 4:33] / nsamp / flat
        say("  ER mean per spectrum " + " ".join(f"{v:.4f}" for v in er.mean(axis=1)) +
            f"; worst shell {np.max(np.abs(er - 1)):.4f}")
        assert nsamp == 1000
        assert np.all(np.abs(er - 1) < 0.03)
        assert np.all(np.abs(er.mean(axis=1) - 1) < 0.01)


@pytest.mark.parametrize("box,prec,rtol", [((96, 64, 80), gmf.FP32_SHIFTED, 1e-6), ((60, 72, 50), gmf.FP64, 1e-12),
                                           ((1024, 6, 5), gmf.FP64, 1e-12), ((2, 3, 1024), gmf.FP64, 1e-12),
                                           ((128, 512, 64), gmf.FP32_SHIFTED, 1e-6),
                                           ((512, 64, 128), gmf.FP64, 1e-12),
                                           ((64, 1024, 96), gmf.FP32_SHIFTED, 1e-6),
                                           ((256, 256, 256), gmf.FP32_SHIFTED, 1e-6)])
def test_full_spectrum_large_boxes(box, prec, rtol):
    """Mixed-radix lines (96 = 16 2 3, 80 = 16 5, 60, 72, 50), the longest
    lines (1024 along x, y and z), every power-of-two length 64 .. 1024 of the
    kernels with fixed stages along each axis, and the 256^3 headline box, one
    sample of the equilibrating fluid 40 steps from rest, against the oracle's
    FFT of the same state."""
    spec = gmf.ReplicaSpec(*box, 1.0, 0.8, 1e-4, 1)
    say(f"full spectrum {box} prec={prec}")
    with gmf.Context([spec], precision=prec, sample_every=20, spectrum=1) as ctx:
        ctx.step(40)                      # samples t = 0 and 20
        ctx.reset_stats()
        f40 = ctx.get_populations()
        ctx.step(1)                       # samples t = 40
        got, cnt = ctx.spectrum()
    ref, rcnt = sp.full_spectrum(oracle_params(spec, precision=prec), f40)
    assert np.array_equal(cnt, rcnt)
    err = np.max(np.abs(got - ref) / np.max(np.abs(ref), axis=1, keepdims=True))
    say(f"  max rel err {err:.2e}")
    assert err < rtol


def test_full_spectrum_bitwise_across_pass_orders_and_batching():
    """The integer shell sums do not depend on the order of the passes (pass
    by pass over all fields, or group by group), and a replica's spectra do
    not depend on the other replicas of its context, also when the replicas'
    lines go through different kernel classes (64^3: fixed stages; 12 x 10 x 8:
    stages chosen at run time)."""
    import os
    specs = [gmf.ReplicaSpec(64, 64, 64, 1.0, 0.8, 1e-4, 21), gmf.ReplicaSpec(12, 10, 8, 1.0, 0.7, 1e-4, 22)]
    old = os.environ.get("GMF_FFT_ORDER")
    res = {}
    try:
        for order in ("0", "1"):
            os.environ["GMF_FFT_ORDER"] = order
            say(f"full spectrum pass order {order}")
            with gmf.Context(specs, precision=gmf.FP32_SHIFTED, sample_every=5, spectrum=1) as ctx:
                ctx.step(20)
                res[order] = [ctx.spectrum(r)[0] for r in range(2)]
    finally:
        if old is None:
            os.environ.pop("GMF_FFT_ORDER", None)
        else:
            os.environ["GMF_FFT_ORDER"] = old
    for r in range(2):
        assert np.any(res["0"][r]), r
        assert np.array_equal(res["0"][r], res["1"][r]), r
    for r, s in enumerate(specs):
        say(f"full spectrum single replica {r}")
        with gmf.Context([s], precision=gmf.FP32_SHIFTED, sample_every=5, spectrum=1) as ctx:
            ctx.step(20)
            assert np.array_equal(ctx.spectrum()[0], res["1"][r]), r


@pytest.mark.parametrize("graph_steps,storage", [(0, gmf.STORE_POPULATIONS), (20, gmf.STORE_POPULATIONS),
                                                 (20, gmf.STORE_MOMENTS)])
def test_sampling_overlap_is_bitwise(graph_steps, storage):
    """With a second stream (the default for moment storage, GMF_SAMPLE_OVERLAP=1
    forces it) the sampling kernels are forked after each sampling step and
    joined before the next one writes the fields: the statistics and full-box
    spectra equal those of the same run with everything on one stream
    (GMF_SAMPLE_OVERLAP=0) bit for bit, through graphs and direct launches,
    for samples 1, 3 and 10 steps apart (with 10 the runs end six steps after
    their last sample, so gmf_step's own join is exercised)."""
    import os
    specs = [gmf.ReplicaSpec(64, 48, 40, 1.0, 0.8, 1e-4, 31), gmf.ReplicaSpec(20, 18, 16, 1.0, 0.6, 1e-4, 32)]
    old = os.environ.get("GMF_SAMPLE_OVERLAP")
    res = {}
    try:
        for ov in ("1", "0"):
            os.environ["GMF_SAMPLE_OVERLAP"] = ov
            for every in (1, 3, 10):
                say(f"sampling overlap {ov} every {every} graph_steps {graph_steps} storage {storage}")
                with gmf.Context(specs, precision=gmf.FP32_SHIFTED, sample_every=every, spectrum=1,
                                 graph_steps=graph_steps, storage=storage) as ctx:
                    ctx.step(13)
                    ctx.step(24)
                    st = [ctx.stats(r) for r in range(2)]
                    sp = [ctx.spectrum(r)[0] for r in range(2)]
                    f = ctx.get_populations(0)
                res[(ov, every)] = (st, sp, f)
    finally:
        if old is None:
            os.environ.pop("GMF_SAMPLE_OVERLAP", None)
        else:
            os.environ["GMF_SAMPLE_OVERLAP"] = old
    for every in (1, 3, 10):
        (sa, pa, fa), (sb, pb, fb) = res[("1", every)], res[("0", every)]
        assert np.array_equal(fa, fb)
        for r in range(2):
            assert sa[r]["nsamples"] == sb[r]["nsamples"] > 0
            for k in ("sum_mean", "sum_meansq", "sum_var", "spectrum"):
                assert np.array_equal(sa[r][k], sb[r][k]), (every, r, k)
            assert np.any(pa[r]) and np.array_equal(pa[r], pb[r]), (every, r)
