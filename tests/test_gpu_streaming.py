"""In-place AA streaming (one population buffer) against the two-buffer A/B
pull.  Both run the same arithmetic on different addresses, so the
trajectories must be bit-identical after every step, odd or even; the host
interface must read and write the canonical state f(x, t) in both storage
states of the AA buffer; and the AA path must meet the oracle bar on its own."""
import numpy as np
import pytest

import oracle
import paper_2601_03806_amd as gmf
from paper_2601_03806_amd import workloads as wl
from gpu_common import oracle_params, rel_err, say

pytestmark = pytest.mark.gpu

RAGGED = gmf.ReplicaSpec(13, 7, 5, 1.0, 0.57, 1e-4, 9)
PLANE = gmf.ReplicaSpec(16, 32, 6, 1.0, 0.6, 1e-4, 21)      # plane of 512 nodes: every addressing mode fits


@pytest.fixture(scope="module")
def w():
    return oracle.tables()[1]


def _snapshots(spec, streaming, prec, coll=gmf.COLLISION_GMF, graph_steps=0, chunks=(3, 4, 1, 9), f0=None,
               tune=0):
    """Canonical states after each chunk of steps (odd and even step counts)."""
    out = []
    with gmf.Context([spec], precision=prec, collision=coll, graph_steps=graph_steps, streaming=streaming,
                     tune=tune) as ctx:
        assert ctx.config()["streaming"] == ("AA" if streaming == gmf.STREAM_AA else "A/B") or tune
        if f0 is not None:
            ctx.set_populations(f0)
        for c in chunks:
            ctx.step(c)
            out.append(ctx.get_populations())
    return out


@pytest.mark.parametrize("prec", [gmf.FP64, gmf.FP32_SHIFTED])
@pytest.mark.parametrize("coll", [gmf.COLLISION_GMF, gmf.COLLISION_BGK])
def test_aa_equals_ab_bitwise(w, prec, coll):
    for spec in (RAGGED, PLANE):
        f0 = wl.perturbed_populations(w, spec.n, amp=0.03, seed=3, velocity=0.03)
        for gs in (0, 8):
            say(f"AA vs A/B {spec.nx}x{spec.ny}x{spec.nz} prec={prec} coll={coll} graph={gs}")
            ab = _snapshots(spec, gmf.STREAM_AB, prec, coll, gs, f0=f0)
            aa = _snapshots(spec, gmf.STREAM_AA, prec, coll, gs, f0=f0)
            for k, (x, y) in enumerate(zip(ab, aa)):
                assert np.array_equal(x, y), (k, float(np.max(np.abs(x - y))))


def test_aa_parity_with_oracle_fp64(w):
    """16^3, tau 1, k_BT 1e-4, seed 1: the AA path against the oracle after an
    odd (199) and an even (200) number of steps."""
    spec = gmf.ReplicaSpec(16, 16, 16, 1.0, 1.0, 1e-4, 1)
    p = oracle_params(spec)
    ref = oracle.rest_state(p)
    say("AA parity with the oracle, 16^3 FP64")
    with gmf.Context([spec], precision=gmf.FP64, streaming=gmf.STREAM_AA) as ctx:
        ctx.step(199)
        got199 = ctx.get_populations()
        ctx.step(1)
        got200 = ctx.get_populations()
    oracle.run(p, ref, 0, 199)
    assert rel_err(got199, ref, w, 1.0, spec.n) < 1e-11
    oracle.run(p, ref, 199, 1)
    assert rel_err(got200, ref, w, 1.0, spec.n) < 1e-11


def test_aa_addressing_modes_bitwise(monkeypatch):
    for prec in (gmf.FP64, gmf.FP32_SHIFTED):
        ref = _snapshots(PLANE, gmf.STREAM_AB, prec, chunks=(5, 6))
        for mode in ("plane", "27", "3", "1"):
            monkeypatch.setenv("GMF_ADDRESSING", mode)
            say(f"AA addressing mode={mode} prec={prec}")
            got = _snapshots(PLANE, gmf.STREAM_AA, prec, chunks=(5, 6))
            for k in range(2):
                assert np.array_equal(ref[k], got[k]), (mode, k)
        monkeypatch.delenv("GMF_ADDRESSING")


def test_aa_host_interface_at_odd_step(w):
    """At an odd step the AA buffer holds every population at its node under the
    opposite velocity: get/set, node lists, moments and conservation sums must
    still see the canonical state."""
    spec = RAGGED
    f1 = wl.perturbed_populations(w, spec.n, amp=0.04, seed=12, velocity=0.02)
    nodes = wl.sample_nodes(spec.n, 40, seed=3)
    res = {}
    for s in (gmf.STREAM_AB, gmf.STREAM_AA):
        say(f"host interface at odd step streaming={s}")
        with gmf.Context([spec], precision=gmf.FP64, streaming=s) as ctx:
            ctx.step(7)
            ctx.set_populations(f1)                         # overwrite at t = 7
            back = ctx.get_populations()
            assert np.array_equal(back, f1)
            sub = ctx.get_nodes(nodes)
            assert np.array_equal(sub, f1.reshape(27, spec.n)[:, nodes].T)
            rho, u = ctx.moments()
            st = ctx.stats()
            ctx.step(5)                                     # t = 12
            res[s] = (rho, u, st["mass"], st["momentum"], ctx.get_populations())
    a, b = res[gmf.STREAM_AB], res[gmf.STREAM_AA]
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert a[2] == b[2] and np.array_equal(a[3], b[3])
    assert np.array_equal(a[4], b[4])


def test_aa_sampling_equals_ab():
    """Sampling at odd and even steps (every 3) reads the fields of the step
    kernel: identical accumulators under both patterns, graph and direct."""
    spec = gmf.ReplicaSpec(12, 10, 8, 1.0, 0.6, 1e-4, 5)
    st = {}
    for s in (gmf.STREAM_AB, gmf.STREAM_AA):
        for gs in (0, 12):
            say(f"sampling streaming={s} graph={gs}")
            with gmf.Context([spec], precision=gmf.FP32_SHIFTED, sample_every=3, graph_steps=gs, streaming=s) as ctx:
                ctx.step(31)
                st[(s, gs)] = ctx.stats()
    ref = st[(gmf.STREAM_AB, 0)]
    assert ref["nsamples"] == 11
    for key, v in st.items():
        for name in ("sum_mean", "sum_meansq", "sum_var", "spectrum"):
            assert np.array_equal(ref[name], v[name]), (key, name)


def test_tuned_pattern_and_single_buffer_workspace():
    """tune = 1 may pick either pattern (same trajectory); an AA-only context
    needs one population buffer less."""
    spec = PLANE
    ref = _snapshots(spec, gmf.STREAM_AB, gmf.FP32_SHIFTED, chunks=(5, 6))
    for s in (gmf.STREAM_AUTO, gmf.STREAM_AA):
        say(f"tuned streaming option={s}")
        got = _snapshots(spec, s, gmf.FP32_SHIFTED, chunks=(5, 6), tune=1)
        for k in range(2):
            assert np.array_equal(ref[k], got[k]), (s, k)
    ab = gmf.workspace_bytes([spec], precision=gmf.FP32_SHIFTED, streaming=gmf.STREAM_AB)
    aa = gmf.workspace_bytes([spec], precision=gmf.FP32_SHIFTED, streaming=gmf.STREAM_AA)
    assert ab - aa >= 27 * 4 * spec.n
