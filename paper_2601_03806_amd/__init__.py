"""Python binding of the gfx950 GMF-FLBM library (libgmf.so, C ABI in include/gmf.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch supplies the device workspace and the stream.  There is no
fallback: if the shared library is missing, importing the binding raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgmf.so")

GMF_OK = 0
GMF_EINVAL = -1
GMF_ENOMEM = -2
GMF_EDEVICE = -3
GMF_ESTATE = -4
GMF_EUNSTABLE = -5

FP64 = 0
FP32_SHIFTED = 1
COLLISION_GMF = 0
COLLISION_BGK = 1
STREAM_AUTO = 0
STREAM_AB = 1
STREAM_AA = 2
STORE_POPULATIONS = 0
STORE_MOMENTS = 1

NOBS = 10
NSPEC = 5
NSHELL = 8
OBS_NAMES = ("drho", "jx", "jy", "jz", "jsum", "pdiag", "poff", "ux", "uy", "uz")
SPEC_NAMES = ("rho", "j", "jsum", "pdiag", "poff")
Q = 27

EXPORTED = (
    "gmf_workspace_bytes", "gmf_init", "gmf_step", "gmf_moments", "gmf_stats", "gmf_reset_stats",
    "gmf_get_populations", "gmf_set_populations", "gmf_get_nodes", "gmf_get_step", "gmf_noise_probe",
    "gmf_get_config", "gmf_copy_probe", "gmf_read_probe", "gmf_destroy", "gmf_strerror", "gmf_spectrum",
    "gmf_get_tiling", "gmf_get_occupancy", "gmf_prepare", "gmf_get_launch_counts", "gmf_set_reference",
    "gmf_noise_probe_noalloc",
)
PROBE_MAX_NODES = 16384


class Replica(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("rho0", ctypes.c_double), ("tau", ctypes.c_double),
                ("kbt", ctypes.c_double), ("seed", ctypes.c_uint64)]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("collision", ctypes.c_int32), ("noise_rho", ctypes.c_int32),
                ("sample_every", ctypes.c_int32), ("graph_steps", ctypes.c_int32), ("tune", ctypes.c_int32),
                ("streaming", ctypes.c_int32), ("spectrum", ctypes.c_int32), ("storage", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("nsamples", ctypes.c_int64), ("nonfinite", ctypes.c_int64),
                ("mass", ctypes.c_double), ("momentum", ctypes.c_double * 3),
                ("sum_mean", ctypes.c_double * NOBS), ("sum_meansq", ctypes.c_double * NOBS),
                ("sum_var", ctypes.c_double * NOBS), ("spectrum", (ctypes.c_double * NSHELL) * NSPEC),
                ("shell_n2", ctypes.c_int32 * NSHELL), ("shell_count", ctypes.c_int32 * NSHELL),
                ("mass_ref", ctypes.c_double), ("momentum_ref", ctypes.c_double * 3),
                ("drift", ctypes.c_double), ("drift_bound", ctypes.c_double)]


class GmfError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


_lib = None


def lib() -> ctypes.CDLL:
    """Load libgmf.so (build it first with paper_2601_03806_amd.build.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                              "(python -c 'import __graft_entry__ as g; g.build()')")
        # PyTorch ships its own HIP runtime under the same soname; loading torch
        # first makes the library bind to that one runtime, so that device
        # pointers and streams handed over by torch are valid in the library.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        dp = ctypes.POINTER(ctypes.c_double)
        L.gmf_workspace_bytes.argtypes = [ctypes.POINTER(Replica), ctypes.c_int32, ctypes.POINTER(Options)]
        L.gmf_workspace_bytes.restype = ctypes.c_size_t
        L.gmf_init.argtypes = [ctypes.POINTER(Replica), ctypes.c_int32, ctypes.POINTER(Options), vp,
                               ctypes.c_size_t, vp, ctypes.POINTER(vp)]
        L.gmf_step.argtypes = [vp, ctypes.c_int64]
        L.gmf_prepare.argtypes = [vp, ctypes.c_int64]
        L.gmf_get_launch_counts.argtypes = [vp] + [ctypes.POINTER(ctypes.c_int64)] * 3 + [ctypes.POINTER(ctypes.c_int32)]
        L.gmf_set_reference.argtypes = [vp, ctypes.c_int32, dp]
        L.gmf_moments.argtypes = [vp, ctypes.c_int32, dp, dp]
        L.gmf_stats.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(Stats)]
        L.gmf_reset_stats.argtypes = [vp]
        L.gmf_get_populations.argtypes = [vp, ctypes.c_int32, dp]
        L.gmf_set_populations.argtypes = [vp, ctypes.c_int32, dp]
        L.gmf_get_nodes.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32, dp]
        L.gmf_get_step.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
        L.gmf_noise_probe.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.POINTER(ctypes.c_uint32), dp]
        L.gmf_noise_probe_noalloc.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32, ctypes.c_int32,
                                              ctypes.c_int32, ctypes.POINTER(ctypes.c_uint32), dp, vp]
        L.gmf_get_config.argtypes = [vp] + [ctypes.POINTER(ctypes.c_int32)] * 6
        L.gmf_get_tiling.argtypes = [vp] + [ctypes.POINTER(ctypes.c_int32)] * 4
        L.gmf_get_occupancy.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
        L.gmf_spectrum.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, dp, ctypes.POINTER(ctypes.c_int64),
                                   ctypes.POINTER(ctypes.c_int32)]
        L.gmf_copy_probe.argtypes = [vp, vp, ctypes.c_size_t, vp]
        L.gmf_copy_probe.restype = ctypes.c_int
        L.gmf_read_probe.argtypes = [vp, ctypes.c_size_t, vp, vp]
        L.gmf_read_probe.restype = ctypes.c_int
        L.gmf_destroy.argtypes = [vp]
        L.gmf_destroy.restype = None
        L.gmf_strerror.argtypes = [ctypes.c_int]
        L.gmf_strerror.restype = ctypes.c_char_p
        for name in ("gmf_init", "gmf_step", "gmf_moments", "gmf_stats", "gmf_reset_stats",
                     "gmf_get_populations", "gmf_set_populations", "gmf_get_nodes", "gmf_get_step",
                     "gmf_noise_probe", "gmf_get_config", "gmf_spectrum", "gmf_get_tiling", "gmf_get_occupancy",
                     "gmf_prepare", "gmf_get_launch_counts", "gmf_set_reference", "gmf_noise_probe_noalloc"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().gmf_strerror(code).decode()


def _check(rc: int, where: str):
    if rc != GMF_OK:
        raise GmfError(rc, where)


def _dp(a: np.ndarray):
    if a.dtype != np.float64 or not a.flags.c_contiguous:
        raise ValueError("expected a C-contiguous float64 array")
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class ReplicaSpec:
    nx: int
    ny: int
    nz: int
    rho0: float = 1.0
    tau: float = 1.0
    kbt: float = 0.0
    seed: int = 1

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz


def make_replicas(specs):
    arr = (Replica * len(specs))()
    for i, s in enumerate(specs):
        arr[i] = Replica(s.nx, s.ny, s.nz, 0, s.rho0, s.tau, s.kbt, s.seed)
    return arr


def make_options(precision=FP64, collision=COLLISION_GMF, noise_rho=0, sample_every=0, graph_steps=-1, tune=0,
                 streaming=STREAM_AUTO, spectrum=0, storage=STORE_POPULATIONS):
    o = Options()
    o.precision, o.collision, o.noise_rho = precision, collision, noise_rho
    o.sample_every, o.graph_steps, o.tune = sample_every, graph_steps, tune
    o.streaming, o.spectrum, o.storage = streaming, spectrum, storage
    return o


def workspace_bytes(specs, **opts) -> int:
    reps = make_replicas(specs)
    o = make_options(**opts)
    return int(lib().gmf_workspace_bytes(reps, len(specs), ctypes.byref(o)))


def noise_probe(seed: int, step: int, node0: int, count: int, precision: int = FP64):
    words = np.zeros(24 * count, np.uint32)
    normals = np.zeros(23 * count)
    rc = lib().gmf_noise_probe(seed, step, node0, count, precision,
                               words.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), _dp(normals))
    _check(rc, "gmf_noise_probe")
    return words.reshape(count, 6, 4), normals.reshape(count, 23)


def noise_probe_noalloc(seed: int, step: int, node0: int, count: int, precision: int = FP64, stream=None):
    """noise_probe through the allocation-free entry point (at most PROBE_MAX_NODES
    nodes; on a torch stream or the legacy stream)."""
    words = np.zeros(24 * count, np.uint32)
    normals = np.zeros(23 * count)
    sp = None if stream is None else int(stream.cuda_stream)
    rc = lib().gmf_noise_probe_noalloc(seed, step, node0, count, precision,
                                       words.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), _dp(normals), sp)
    _check(rc, "gmf_noise_probe_noalloc")
    return words.reshape(count, 6, 4), normals.reshape(count, 23)


def copy_probe(src_ptr: int, dst_ptr: int, nbytes: int, stream=None):
    """Enqueue the library's streaming copy (bandwidth reference) on a torch stream."""
    sp = None if stream is None else int(stream.cuda_stream)
    _check(lib().gmf_copy_probe(src_ptr, dst_ptr, nbytes, sp), "gmf_copy_probe")


def read_probe(src_ptr: int, nbytes: int, flag_ptr: int, stream=None):
    """Enqueue the library's plain read of a device buffer (read-bandwidth reference) on a torch stream;
    flag_ptr is a device uint32 set to 1 if a value read is not finite."""
    sp = None if stream is None else int(stream.cuda_stream)
    _check(lib().gmf_read_probe(src_ptr, nbytes, flag_ptr, sp), "gmf_read_probe")


class Context:
    """A set of replicas advanced together by the library (one C context).

    Device memory comes from a torch uint8 tensor (``workspace='torch'``) or
    from the library itself (``workspace=None``); the stream is a torch stream
    (``stream`` = torch.cuda.Stream) or the library's own (``stream=None``).
    """

    def __init__(self, specs, *, precision=FP64, collision=COLLISION_GMF, noise_rho=0, sample_every=0,
                 graph_steps=-1, tune=0, streaming=STREAM_AUTO, spectrum=0, storage=STORE_POPULATIONS,
                 workspace="torch", stream=None):
        self.specs = list(specs)
        self._reps = make_replicas(self.specs)
        self._opt = make_options(precision, collision, noise_rho, sample_every, graph_steps, tune, streaming,
                                 spectrum, storage)
        self.precision = precision
        self._ws = None
        ws_ptr, ws_bytes = None, 0
        if workspace == "torch":
            import torch
            ws_bytes = int(lib().gmf_workspace_bytes(self._reps, len(self.specs), ctypes.byref(self._opt)))
            if ws_bytes == 0:
                raise GmfError(GMF_EINVAL, "gmf_workspace_bytes")
            self._ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
            ws_ptr = self._ws.data_ptr()
        self.stream = stream
        sp = None if stream is None else int(stream.cuda_stream)
        h = ctypes.c_void_p()
        rc = lib().gmf_init(self._reps, len(self.specs), ctypes.byref(self._opt), ws_ptr, ws_bytes, sp,
                            ctypes.byref(h))
        _check(rc, "gmf_init")
        self._h = h

    # lifecycle -------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().gmf_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # stepping --------------------------------------------------------------
    def step(self, n: int = 1):
        _check(lib().gmf_step(self._h, int(n)), "gmf_step")

    def prepare(self, n: int):
        """Capture every graph that step(n) would launch, without running anything."""
        _check(lib().gmf_prepare(self._h, int(n)), "gmf_prepare")

    def launch_counts(self) -> dict:
        g, gs, d = (ctypes.c_int64() for _ in range(3))
        c = ctypes.c_int32()
        _check(lib().gmf_get_launch_counts(self._h, ctypes.byref(g), ctypes.byref(gs), ctypes.byref(d),
                                           ctypes.byref(c)), "gmf_get_launch_counts")
        return {"graph_launches": g.value, "graph_steps": gs.value, "direct_steps": d.value,
                "graphs_captured": c.value}

    def set_reference(self, ref=None, r: int = 0):
        """Conservation reference of replica r: None takes the current state's mass
        and momentum, else (mass, mx, my, mz)."""
        if ref is None:
            _check(lib().gmf_set_reference(self._h, r, None), "gmf_set_reference")
        else:
            a = np.ascontiguousarray(ref, dtype=np.float64)
            if a.size != 4:
                raise ValueError("set_reference: (mass, mx, my, mz)")
            _check(lib().gmf_set_reference(self._h, r, _dp(a)), "gmf_set_reference")

    @property
    def t(self) -> int:
        v = ctypes.c_int64()
        _check(lib().gmf_get_step(self._h, ctypes.byref(v)), "gmf_get_step")
        return v.value

    def config(self):
        a, b, c, d, e, x = (ctypes.c_int32() for _ in range(6))
        _check(lib().gmf_get_config(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d),
                                    ctypes.byref(e), ctypes.byref(x)), "gmf_get_config")
        st, tx, ty, tz = (ctypes.c_int32() for _ in range(4))
        _check(lib().gmf_get_tiling(self._h, ctypes.byref(st), ctypes.byref(tx), ctypes.byref(ty), ctypes.byref(tz)),
               "gmf_get_tiling")
        occ = ctypes.c_int32()
        _check(lib().gmf_get_occupancy(self._h, ctypes.byref(occ)), "gmf_get_occupancy")
        cfg = {"nodes_per_thread": a.value, "block": b.value, "graph_steps": c.value,
               "addressing": "plane" if d.value == 0 else ("none" if d.value < 0 else f"group{d.value}"),
               "streaming": "AA" if e.value == STREAM_AA else "A/B",
               "block_map": f"xcd/{x.value}" if x.value else "linear",
               "storage": "moments" if st.value == STORE_MOMENTS else "populations",
               "workgroups_per_cu": occ.value}
        if st.value == STORE_MOMENTS:
            cfg["tile"] = f"{tx.value}x{ty.value}x{tz.value}"
        return cfg

    # data ------------------------------------------------------------------
    def moments(self, r: int = 0):
        n = self.specs[r].n
        rho = np.zeros(n)
        u = np.zeros(3 * n)
        _check(lib().gmf_moments(self._h, r, _dp(rho), _dp(u)), "gmf_moments")
        return rho, u.reshape(3, n)

    def stats(self, r: int = 0, allow_unstable: bool = False) -> dict:
        s = Stats()
        rc = lib().gmf_stats(self._h, r, ctypes.byref(s))
        if rc == GMF_EUNSTABLE and allow_unstable:
            pass
        else:
            _check(rc, "gmf_stats")
        return {
            "step": s.step, "nsamples": s.nsamples, "nonfinite": s.nonfinite, "rc": rc,
            "mass": s.mass, "momentum": np.array(s.momentum[:]),
            "sum_mean": np.array(s.sum_mean[:]), "sum_meansq": np.array(s.sum_meansq[:]),
            "sum_var": np.array(s.sum_var[:]),
            "spectrum": np.array([list(row) for row in s.spectrum]),
            "shell_n2": np.array(s.shell_n2[:]), "shell_count": np.array(s.shell_count[:]),
            "mass_ref": s.mass_ref, "momentum_ref": np.array(s.momentum_ref[:]),
            "drift": s.drift, "drift_bound": s.drift_bound,
        }

    def reset_stats(self):
        _check(lib().gmf_reset_stats(self._h), "gmf_reset_stats")

    def spectrum(self, r: int = 0):
        """Full-box shell spectra (needs spectrum=1): sums over the samples of the
        shell averages, (5, nshell) in GMF_SPEC_* order, and the shell counts."""
        ns = ctypes.c_int32()
        _check(lib().gmf_spectrum(self._h, r, 0, None, None, ctypes.byref(ns)), "gmf_spectrum")
        sums = np.zeros(NSPEC * ns.value)
        counts = np.zeros(ns.value, np.int64)
        rc = lib().gmf_spectrum(self._h, r, ns.value, _dp(sums), counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                ctypes.byref(ns))
        _check(rc, "gmf_spectrum")
        return sums.reshape(NSPEC, ns.value), counts

    def get_populations(self, r: int = 0) -> np.ndarray:
        f = np.zeros(Q * self.specs[r].n)
        _check(lib().gmf_get_populations(self._h, r, _dp(f)), "gmf_get_populations")
        return f

    def set_populations(self, f: np.ndarray, r: int = 0):
        ff = np.ascontiguousarray(f, dtype=np.float64)
        if ff.size != Q * self.specs[r].n:
            raise ValueError(f"set_populations: {ff.size} values for a replica of {self.specs[r].n} nodes x {Q}")
        _check(lib().gmf_set_populations(self._h, r, _dp(ff)), "gmf_set_populations")

    def get_nodes(self, nodes, r: int = 0) -> np.ndarray:
        nd = np.ascontiguousarray(nodes, dtype=np.int64).ravel()
        out = np.zeros((len(nd), Q))
        rc = lib().gmf_get_nodes(self._h, r, nd.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(nd), _dp(out))
        _check(rc, "gmf_get_nodes")
        return out
