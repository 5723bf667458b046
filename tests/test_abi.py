"""The C ABI library loads and exports what include/gmf.h declares; argument
validation that needs no device (CPU only: no compute call is made)."""
import ctypes
import os
import re


import paper_2601_03806_amd as gmf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "gmf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gmf_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("gmf_init", "gmf_step", "gmf_moments", "gmf_stats"):
        assert required in names
    assert set(names) == set(gmf.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = gmf.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_struct_layouts():
    assert ctypes.sizeof(gmf.Replica) == 48
    assert ctypes.sizeof(gmf.Options) == 36
    # 3 int64 + 4 doubles + 3*10 doubles + 40 doubles + 16 int32 + the conservation guard's 6 doubles
    assert ctypes.sizeof(gmf.Stats) == 8 * 3 + 8 * 4 + 8 * 30 + 8 * 40 + 4 * 16 + 8 * 6


def _ws(specs, **kw):
    return gmf.workspace_bytes([gmf.ReplicaSpec(*s) for s in specs], **kw)


def test_workspace_bytes_and_validation():
    ok = _ws([(16, 16, 16, 1.0, 1.0, 1e-4, 1)])
    # two FP64 population buffers dominate
    assert ok >= 2 * 27 * 8 * 16 ** 3
    f32 = _ws([(16, 16, 16, 1.0, 1.0, 1e-4, 1)], precision=gmf.FP32_SHIFTED)
    assert 2 * 27 * 4 * 16 ** 3 <= f32 < ok
    # invalid replicas -> 0
    assert _ws([(16, 16, 16, 1.0, 0.5, 1e-4, 1)]) == 0          # tau <= 1/2
    assert _ws([(16, 16, 16, 1.0, float("nan"), 1e-4, 1)]) == 0
    assert _ws([(0, 16, 16, 1.0, 1.0, 1e-4, 1)]) == 0           # empty box
    assert _ws([(16, 16, 16, 0.0, 1.0, 1e-4, 1)]) == 0          # rho0 <= 0
    assert _ws([(16, 16, 16, 1.0, 1.0, -1e-4, 1)]) == 0         # k_B T < 0
    assert _ws([(1001, 1001, 1001, 1.0, 1.0, 1e-4, 1)]) == 0    # no addressing mode fits (FP64)
    assert _ws([(16, 16, 16, 1.0, 1.0, 1e-4, 1)], precision=7) == 0
    assert _ws([(16, 16, 16, 1.0, 1.0, 1e-4, 1)], sample_every=-1) == 0
    assert _ws([(2048, 4096, 1, 1.0, 1.0, 1e-4, 1)], sample_every=10) > 0    # wide planes can be sampled
    assert _ws([(16, 16, 16, 1.0, 1.0, 1e-4, 1)], streaming=3) == 0           # unknown streaming pattern
    # the in-place AA pattern needs one population buffer instead of two
    aa = _ws([(16, 16, 16, 1.0, 1.0, 1e-4, 1)], streaming=gmf.STREAM_AA)
    assert ok - aa >= 27 * 8 * 16 ** 3
    assert _ws([(16, 16, 16, 1.0, 1.0, 1e-4, 1)], streaming=gmf.STREAM_AB) == ok
    # full-box spectra: need sampling and box lengths with prime factors 2, 3, 5 (at most 1024)
    base = _ws([(12, 10, 8, 1.0, 1.0, 1e-4, 1)], sample_every=5)
    with_spec = _ws([(12, 10, 8, 1.0, 1.0, 1e-4, 1)], sample_every=5, spectrum=1)
    assert with_spec >= base + 3 * 16 * 960
    assert _ws([(12, 10, 8, 1.0, 1.0, 1e-4, 1)], spectrum=1) == 0                  # no sampling
    assert _ws([(14, 10, 8, 1.0, 1.0, 1e-4, 1)], sample_every=5, spectrum=1) == 0  # factor 7
    assert _ws([(2048, 8, 8, 1.0, 1.0, 1e-4, 1)], sample_every=5, spectrum=1) == 0  # longer than 1024
    assert _ws([(12, 10, 8, 1.0, 1.0, 1e-4, 1)], sample_every=5, spectrum=2) == 0
    # the longest lines along every axis, both precisions (a z line of 1024 FP64 points fills a tile)
    for box in ((2, 3, 1024), (1024, 6, 5), (3, 1024, 2), (1024, 1024, 2), (1024, 2, 1024)):
        for prec in (gmf.FP64, gmf.FP32_SHIFTED):
            assert _ws([box + (1.0, 1.0, 1e-4, 1)], precision=prec, sample_every=5, spectrum=1) > 0, (box, prec)
    # moment storage: two buffers of ten moments instead of 27 populations; GMF
    # collision and the two-buffer scheme only
    mom = _ws([(16, 16, 16, 1.0, 1.0, 1e-4, 1)], storage=gmf.STORE_MOMENTS)
    assert 2 * 10 * 8 * 16 ** 3 <= mom <= ok - 2 * 17 * 8 * 16 ** 3
    assert _ws([(16, 16, 16, 1.0, 1.0, 1e-4, 1)], storage=gmf.STORE_MOMENTS, streaming=gmf.STREAM_AB) == mom
    assert _ws([(16, 16, 16, 1.0, 1.0, 1e-4, 1)], storage=gmf.STORE_MOMENTS, collision=gmf.COLLISION_BGK) == 0
    assert _ws([(16, 16, 16, 1.0, 1.0, 1e-4, 1)], storage=gmf.STORE_MOMENTS, streaming=gmf.STREAM_AA) == 0
    assert _ws([(16, 16, 16, 1.0, 1.0, 1e-4, 1)], storage=2) == 0
    assert _ws([(512, 512, 512, 1.0, 0.55, 1e-5, 1)], storage=gmf.STORE_MOMENTS, sample_every=10,
               spectrum=1) > 2 * 10 * 8 * 512 ** 3
    # fewer than 2^32 nodes in one context (its 32-bit workgroup counts)
    assert _ws([(1024, 1024, 1024, 1.0, 1.0, 1e-4, 1)] * 4, precision=gmf.FP32_SHIFTED) == 0
    assert _ws([(1024, 1024, 1024, 1.0, 1.0, 1e-4, 1)] * 3, precision=gmf.FP32_SHIFTED) > 0
    # sampling: the first DFT stage's partial sums (6 * 28 per plane and block of 64 columns) at 32-bit offsets
    assert _ws([(512, 1, 65600, 1.0, 1.0, 1e-4, 1)], precision=gmf.FP32_SHIFTED, sample_every=10) > 0
    assert _ws([(1, 1, 1 << 24, 1.0, 1.0, 1e-4, 1)], sample_every=10) > 0
    assert _ws([(1, 1, 1 << 24, 1.0, 1.0, 1e-4, 1)] * 2, sample_every=10) == 0
    assert _ws([(1, 1, 1 << 25, 1.0, 1.0, 1e-4, 1)]) > 0
    assert _ws([(1, 1, 1 << 25, 1.0, 1.0, 1e-4, 1)], sample_every=10) == 0
    # the 512^3 stress workload fits both precisions
    assert _ws([(512, 512, 512, 1.0, 0.55, 1e-5, 1)]) > 2 * 27 * 8 * 512 ** 3
    assert _ws([(512, 512, 512, 1.0, 0.55, 1e-5, 1)], precision=gmf.FP32_SHIFTED) > 0


def test_init_rejects_before_touching_the_device():
    lib = gmf.lib()
    reps = gmf.make_replicas([gmf.ReplicaSpec(8, 8, 8, 1.0, 0.4, 1e-4, 1)])
    opt = gmf.make_options()
    h = ctypes.c_void_p()
    assert lib.gmf_init(reps, 1, ctypes.byref(opt), None, 0, None, ctypes.byref(h)) == gmf.GMF_EINVAL
    assert lib.gmf_init(reps, 0, ctypes.byref(opt), None, 0, None, ctypes.byref(h)) == gmf.GMF_EINVAL
    good = gmf.make_replicas([gmf.ReplicaSpec(8, 8, 8, 1.0, 0.8, 1e-4, 1)])
    need = lib.gmf_workspace_bytes(good, 1, ctypes.byref(opt))
    # a caller workspace that is too small
    assert lib.gmf_init(good, 1, ctypes.byref(opt), ctypes.c_void_p(256), need - 1, None,
                        ctypes.byref(h)) == gmf.GMF_EINVAL
    # NULL context
    assert lib.gmf_step(None, 1) == gmf.GMF_ESTATE
    assert lib.gmf_stats(None, 0, None) == gmf.GMF_ESTATE
    assert lib.gmf_get_occupancy(None, None) == gmf.GMF_ESTATE
    assert lib.gmf_prepare(None, 1) == gmf.GMF_ESTATE
    assert lib.gmf_get_launch_counts(None, None, None, None, None) == gmf.GMF_ESTATE
    assert lib.gmf_set_reference(None, 0, None) == gmf.GMF_ESTATE
    assert lib.gmf_noise_probe(1, 0, 0, -1, 0, None, None) == gmf.GMF_EINVAL
    # the allocation-free probe rejects sizes beyond its fixed scratch before any device call
    assert gmf.PROBE_MAX_NODES == 16384
    assert lib.gmf_noise_probe_noalloc(1, 0, 0, gmf.PROBE_MAX_NODES + 1, 0, None, None, None) == gmf.GMF_EINVAL
    assert lib.gmf_noise_probe_noalloc(1, 0, 0, -1, 0, None, None, None) == gmf.GMF_EINVAL
    assert lib.gmf_noise_probe_noalloc(1, 0, 0, 8, 7, None, None, None) == gmf.GMF_EINVAL
    assert lib.gmf_noise_probe_noalloc(1, 0, 0xFFFFFFFF, 2, 0, None, None, None) == gmf.GMF_EINVAL
    assert lib.gmf_noise_probe_noalloc(1, 0, 0, 0, 0, None, None, None) == gmf.GMF_OK
    # the bandwidth probes check pointers, alignment and size before any device call
    assert lib.gmf_copy_probe(None, ctypes.c_void_p(256), 16, None) == gmf.GMF_EINVAL
    assert lib.gmf_copy_probe(ctypes.c_void_p(256), ctypes.c_void_p(512), 24, None) == gmf.GMF_EINVAL
    assert lib.gmf_read_probe(None, 16, ctypes.c_void_p(256), None) == gmf.GMF_EINVAL
    assert lib.gmf_read_probe(ctypes.c_void_p(256), 16, None, None) == gmf.GMF_EINVAL
    assert lib.gmf_read_probe(ctypes.c_void_p(264), 16, ctypes.c_void_p(256), None) == gmf.GMF_EINVAL
    assert lib.gmf_read_probe(ctypes.c_void_p(256), 0, ctypes.c_void_p(256), None) == gmf.GMF_EINVAL
    assert lib.gmf_read_probe(ctypes.c_void_p(256), 40, ctypes.c_void_p(256), None) == gmf.GMF_EINVAL
    assert lib.gmf_read_probe(ctypes.c_void_p(256), 16, ctypes.c_void_p(258), None) == gmf.GMF_EINVAL
    assert gmf.strerror(gmf.GMF_EUNSTABLE).startswith("non-finite")
