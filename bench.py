#!/usr/bin/env python3
"""Benchmark of the fused GMF-FLBM D3Q27 stream+collide step on one MI355X.

Default workload: 256^3 periodic box, rho0 = 1, tau = 0.8, k_B T = 1e-4, seed 1,
FP32 shifted populations in SoA layout, HIP-graph step loop: the bandwidth
headline (two 1.8 GB population buffers, far larger than the 256 MB last-level
cache).  The same JSON line also reports the plain FP64 single-replica form on
the same box, the batched ensemble (32 x 32^3 + 16 x 48^3 + 16 x 64^3 replicas
in one launch per step), and the FP64 CPU oracle timed on the host cores.

A step is one pass of the whole fused step (pull, moments, relaxation, ghost
filter, Philox noise, back-projection, write) over every node.  Inputs are
resident in device memory before timing starts.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
BYTES_PER_NODE = {"fp32": 216, "fp64": 432}   # 27 loads + 27 stores per node update
MOM_BYTES_PER_NODE = {"fp32": 80, "fp64": 160}  # moment storage: 10 loads + 10 stores per node update
METRIC = "GLUPS & % HBM roofline, FP32-batched vs FP64-plain, at matched variance accuracy"


# sources of each step kernel: a committed counter profile counts for the
# kernel only while these files are unchanged
KERNEL_SOURCES = {
    "step": ("gmf_kernels.hip", "gmf_collide.hpp", "gmf_device.hpp", "gmf_math.hpp", "gmf_internal.hpp"),
    "mstep": ("gmf_mstep.hip", "gmf_collide.hpp", "gmf_device.hpp", "gmf_math.hpp", "gmf_internal.hpp"),
}
VALU_PEAK = 256 * 4 * 2.4e9 / 4 / 1e9   # wave64 VALU instructions per ns: 256 CUs x 4 SIMDs, one per 4 cycles


def kernel_source_hash(kernel: str = "step") -> str:
    """Hash of the kernel's sources without comments and blank lines, so that
    an edit of the documentation does not retire a counter profile."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2601_03806_amd", "csrc", f)) as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        for line in text.splitlines():
            code = line.split("//", 1)[0].strip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def variant_key(cfg: dict) -> str:
    """Step-kernel variant as named in profiles/traffic.json."""
    if cfg.get("storage") == "moments":
        return f"moments/{cfg['tile']}/{cfg['block_map']}"
    occ = cfg.get("workgroups_per_cu", 0)
    return (f"{cfg['addressing']}/{cfg['streaming']}/npt{cfg['nodes_per_thread']}/{cfg['block_map']}" +
            (f"/occ{occ}" if occ else ""))


def profiled(kernel_key: str, nodes: int, cfg: dict, field: str = "bytes_per_launch"):
    """A per-launch figure (HBM bytes, VALU instructions) of the step-kernel
    variant that ran, from the committed rocprofv3 counter summary, if it was
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = data.get(kernel_key)
    kernel = "mstep" if kernel_key.startswith("mstep") else "step"
    if not ent or ent.get("source_hash") != kernel_source_hash(kernel) or ent.get("nodes") != nodes:
        return None
    var = ent.get("variants", {}).get(variant_key(cfg))
    return None if var is None else var.get(field)


def graph_len(steps: int, cap: int = 64) -> int:
    """Steps per captured graph for a timed loop of `steps` steps: the longest
    length up to `cap` that divides it, so that the loop is whole graph replays."""
    return next(g for g in range(max(1, min(cap, steps)), 0, -1) if steps % g == 0)


def time_context(ctx, stream, steps, warmup, torch, loops=None, key=None):
    """Seconds for `steps` steps after `warmup` untimed ones.  Every graph the
    timed steps launch is captured beforehand (gmf_prepare), so the timed
    region holds graph replays and kernels only; what ran is recorded in
    loops[key] from the library's launch counters."""
    ctx.step(warmup)
    ctx.prepare(steps)
    torch.cuda.synchronize()
    before = ctx.launch_counts()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ctx.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    after = ctx.launch_counts()
    if loops is not None:
        loops[key] = {"steps_per_graph": ctx.config()["graph_steps"],
                      "graph_replays": after["graph_launches"] - before["graph_launches"],
                      "graph_steps": after["graph_steps"] - before["graph_steps"],
                      "direct_steps": after["direct_steps"] - before["direct_steps"],
                      "captured_in_timed_region": after["graphs_captured"] - before["graphs_captured"]}
    return e0.elapsed_time(e1) / 1e3   # seconds


# launch variants of the step kernels, forced one after the other for the
# rocprofv3 counter runs (--profile-variants): GMF_ADDRESSING, GMF_BLOCK_MAP,
# GMF_OCCUPANCY and GMF_MTILE select them (tune 0)
PROFILE_MAPS = ("linear", "xcd", "xcd16")


def profile_variants(args, torch, gmf, wl):
    """Run every launch variant of one step kernel for 2 + args.steps steps in
    a fixed order, on the workload that the bench line quotes it for; return
    the variants as they ran (bench-line key, configuration, kernel launches),
    so that the step-kernel dispatches of a counter run map onto them in order."""
    stream = torch.cuda.Stream()
    kind = args.profile_variants
    if kind == "ensemble":
        we = wl.ensemble()
        specs = [gmf.ReplicaSpec(*bx.n, rho0=bx.rho0, tau=bx.tau, kbt=bx.kbt, seed=bx.seed) for bx in we.boxes]
        combos = [({"GMF_ADDRESSING": a, "GMF_BLOCK_MAP": m, "GMF_OCCUPANCY": str(k)}, st)
                  for a in ("1", "3", "27", "plane") for st in (gmf.STREAM_AB, gmf.STREAM_AA)
                  for m in PROFILE_MAPS for k in (0, 5)]
        prec, storage = gmf.FP32_SHIFTED, gmf.STORE_POPULATIONS
    else:
        b = wl.bandwidth_headline("fp64" if kind == "fp64" else "fp32").boxes[0]
        specs = [gmf.ReplicaSpec(*b.n, rho0=b.rho0, tau=b.tau, kbt=b.kbt, seed=b.seed)]
        if kind == "moments":
            combos = [({"GMF_MTILE": f"{t},{z}", "GMF_BLOCK_MAP": m}, gmf.STREAM_AB)
                      for t in range(4) for z in (32, 64, 128) for m in PROFILE_MAPS]
            prec, storage = gmf.FP32_SHIFTED, gmf.STORE_MOMENTS
        else:
            combos = [({"GMF_ADDRESSING": a, "GMF_BLOCK_MAP": m, "GMF_OCCUPANCY": str(k)}, gmf.STREAM_AB)
                      for a in ("27", "plane") for m in PROFILE_MAPS for k in (0, 5, 4, 3)]
            prec = gmf.FP64 if kind == "fp64" else gmf.FP32_SHIFTED
            storage = gmf.STORE_POPULATIONS
    ran, seen = [], set()
    for env, st in combos:
        old = {k: os.environ.get(k) for k in env}
        os.environ.update(env)
        try:
            with gmf.Context(specs, precision=prec, stream=stream, tune=0, storage=storage, streaming=st,
                             graph_steps=graph_len(args.steps)) as ctx:
                cfg = ctx.config()
                key = variant_key(cfg)
                if key in seen:      # an override that does not fit falls back to a variant already run
                    continue
                seen.add(key)
                time_context(ctx, stream, args.steps, 2, torch)
                ran.append({"key": key, "config": cfg, "launches": 2 + args.steps})
                print(f"[bench] variant {key}", file=sys.stderr, flush=True)
        finally:
            for k, v in old.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v
    torch.cuda.synchronize()
    return {"profile_variants": kind, "nodes": sum(sp.n for sp in specs), "steps": args.steps, "variants": ran}


def profile_sampler(args, torch, gmf, wl):
    """The headline box sampled every 10 steps with the full-box spectra, the
    default launch variant (tune 0): the sampler and spectrum kernels for the
    counter runs, in the precision of --precision and the storage of --storage."""
    stream = torch.cuda.Stream()
    b = wl.bandwidth_headline(args.precision).boxes[0]
    spec = gmf.ReplicaSpec(*b.n, rho0=b.rho0, tau=b.tau, kbt=b.kbt, seed=b.seed)
    steps = max(10, args.steps // 10 * 10)
    prec = gmf.FP64 if args.precision == "fp64" else gmf.FP32_SHIFTED
    storage = gmf.STORE_MOMENTS if args.storage == "moments" else gmf.STORE_POPULATIONS
    with gmf.Context([spec], precision=prec, stream=stream, tune=0, sample_every=10, spectrum=1, storage=storage,
                     graph_steps=graph_len(steps)) as ctx:
        sec = time_context(ctx, stream, steps, 10, torch)
        cfg = ctx.config()
    return {"profile_sampler": True, "precision": args.precision, "storage": args.storage, "nodes": spec.n, "steps": steps, "seconds": sec, "config": cfg}


def run_gpu(args, torch, gmf, wl):
    stream = torch.cuda.Stream()
    out = {}
    loops = out.setdefault("step_loops", {})
    streaming = {"auto": gmf.STREAM_AUTO, "ab": gmf.STREAM_AB, "aa": gmf.STREAM_AA}[args.streaming]
    if args.workload == "ensemble":
        # profiling runs of the batched form alone: the 64-replica ensemble
        we = wl.ensemble()
        specs = [gmf.ReplicaSpec(*bx.n, rho0=bx.rho0, tau=bx.tau, kbt=bx.kbt, seed=bx.seed) for bx in we.boxes]
        with gmf.Context(specs, precision=gmf.FP32_SHIFTED, stream=stream, tune=args.tune, streaming=streaming,
                         graph_steps=graph_len(args.steps)) as ctx:
            print(f"[bench] {we.name}: warmup {args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
            sec = time_context(ctx, stream, args.steps, args.warmup, torch, loops, "headline")
            mass = sum(ctx.stats(r)["mass"] for r in range(len(specs)))
            mass0 = sum(sp.n * sp.rho0 for sp in specs)
            out["headline"] = {"seconds": sec, "nodes": we.nodes, "steps": args.steps, "config": ctx.config(),
                               "mass_drift_rel": abs(mass - mass0) / mass0}
        torch.cuda.synchronize()
        return out
    # bandwidth headline: FP32 shifted (FP64 plain in profiling runs of that kernel)
    w = wl.bandwidth_headline(args.precision)
    b = w.boxes[0]
    spec = gmf.ReplicaSpec(*b.n, rho0=b.rho0, tau=b.tau, kbt=b.kbt, seed=b.seed)
    storage = gmf.STORE_MOMENTS if args.storage == "moments" else gmf.STORE_POPULATIONS
    head_prec = gmf.FP64 if args.precision == "fp64" else gmf.FP32_SHIFTED
    with gmf.Context([spec], precision=head_prec, stream=stream, tune=args.tune, storage=storage,
                     streaming=streaming, graph_steps=graph_len(args.steps)) as ctx:
        print(f"[bench] {w.name} ({args.storage}): warmup {args.warmup}, steps {args.steps}", file=sys.stderr,
              flush=True)
        sec = time_context(ctx, stream, args.steps, args.warmup, torch, loops, "headline")
        st = ctx.stats()
        out["headline"] = {"seconds": sec, "nodes": spec.n, "steps": args.steps, "config": ctx.config(),
                       "mass_drift_rel": abs(st["mass"] - spec.n * b.rho0) / (spec.n * b.rho0)}
    torch.cuda.synchronize()
    if not args.skip_extra:
        # plain FP64, same box
        w64 = wl.bandwidth_headline("fp64")
        s64 = max(10, args.steps // 5)
        with gmf.Context([spec], precision=gmf.FP64, stream=stream, tune=args.tune, graph_steps=graph_len(s64)) as ctx:
            print(f"[bench] fp64 {w64.name}: steps {s64}", file=sys.stderr, flush=True)
            sec = time_context(ctx, stream, s64, max(2, args.warmup // 5), torch, loops, "fp64")
            out["fp64"] = {"seconds": sec, "nodes": spec.n, "steps": s64, "config": ctx.config()}
        torch.cuda.synchronize()
        # batched ensemble
        we = wl.ensemble()
        specs = [gmf.ReplicaSpec(*bx.n, rho0=bx.rho0, tau=bx.tau, kbt=bx.kbt, seed=bx.seed) for bx in we.boxes]
        se = max(20, args.steps)
        with gmf.Context(specs, precision=gmf.FP32_SHIFTED, stream=stream, tune=args.tune,
                         graph_steps=graph_len(se)) as ctx:
            print(f"[bench] batched {we.name}: steps {se}", file=sys.stderr, flush=True)
            sec = time_context(ctx, stream, se, args.warmup, torch, loops, "batched")
            out["batched"] = {"seconds": sec, "nodes": we.nodes, "steps": se, "config": ctx.config(),
                              "workload": we.name}
        torch.cuda.synchronize()
        with gmf.Context(specs, precision=gmf.FP32_SHIFTED, stream=stream, tune=args.tune,
                         storage=gmf.STORE_MOMENTS, graph_steps=graph_len(se)) as ctx:
            print(f"[bench] batched {we.name}, moment storage: steps {se}", file=sys.stderr, flush=True)
            sec = time_context(ctx, stream, se, args.warmup, torch, loops, "batched_mom")
            out["batched_mom"] = {"seconds": sec, "nodes": we.nodes, "steps": se, "config": ctx.config(),
                                  "workload": we.name}
        torch.cuda.synchronize()
        # the headline box with the in-place AA pattern (one population buffer: half the memory)
        sa = max(20, args.steps // 4)
        with gmf.Context([spec], precision=gmf.FP32_SHIFTED, stream=stream, tune=args.tune,
                         streaming=gmf.STREAM_AA, graph_steps=graph_len(sa)) as ctx:
            print(f"[bench] fp32 AA streaming: steps {sa}", file=sys.stderr, flush=True)
            sec = time_context(ctx, stream, sa, args.warmup, torch, loops, "aa")
            out["aa"] = {"seconds": sec, "nodes": spec.n, "steps": sa, "config": ctx.config()}
        torch.cuda.synchronize()
        # the headline box with the fused sampler on (every 10 steps: variances and shell spectra);
        # at least 100 timed steps (10 samples), so that a sample's cost is averaged over several
        ss = max(100, args.steps // 4) // 10 * 10
        with gmf.Context([spec], precision=gmf.FP32_SHIFTED, stream=stream, tune=args.tune,
                         sample_every=10, graph_steps=graph_len(ss)) as ctx:
            print(f"[bench] fp32 sampled every 10: steps {ss}", file=sys.stderr, flush=True)
            sec = time_context(ctx, stream, ss, 10, torch, loops, "sampled")
            out["sampled"] = {"seconds": sec, "nodes": spec.n, "steps": ss}
        torch.cuda.synchronize()
        # the headline box with the full-box shell spectra as well (FFT of six fields per sample)
        with gmf.Context([spec], precision=gmf.FP32_SHIFTED, stream=stream, tune=args.tune,
                         sample_every=10, spectrum=1, graph_steps=graph_len(ss)) as ctx:
            print(f"[bench] fp32 sampled every 10 with full spectra: steps {ss}", file=sys.stderr, flush=True)
            sec = time_context(ctx, stream, ss, 10, torch, loops, "spectrum")
            out["spectrum"] = {"seconds": sec, "nodes": spec.n, "steps": ss}
        torch.cuda.synchronize()
        # the headline box in moment storage (ten moments per node), both precisions
        for prec, key, st in ((gmf.FP32_SHIFTED, "mom_fp32", max(20, args.steps // 4)),
                              (gmf.FP64, "mom_fp64", max(10, args.steps // 10))):
            with gmf.Context([spec], precision=prec, stream=stream, tune=args.tune,
                             storage=gmf.STORE_MOMENTS, graph_steps=graph_len(st)) as ctx:
                print(f"[bench] {key} moment storage: steps {st}", file=sys.stderr, flush=True)
                sec = time_context(ctx, stream, st, 4, torch, loops, key)
                out[key] = {"seconds": sec, "nodes": spec.n, "steps": st, "config": ctx.config()}
            torch.cuda.synchronize()
        print("[bench] variance accuracy: 64^3 tau sweep, FP32 batched vs FP64", file=sys.stderr, flush=True)
        out["variance_accuracy"] = variance_accuracy(torch, gmf, wl, stream)
        # 512^3 precision-stress box, both precisions
        wp = wl.precision_stress("fp32")
        bp = wp.boxes[0]
        sp = gmf.ReplicaSpec(*bp.n, rho0=bp.rho0, tau=bp.tau, kbt=bp.kbt, seed=bp.seed)
        for prec, key, st in ((gmf.FP32_SHIFTED, "fp32_512", 40), (gmf.FP64, "fp64_512", 20)):
            with gmf.Context([sp], precision=prec, stream=stream, tune=args.tune, graph_steps=graph_len(st)) as ctx:
                print(f"[bench] {key}: steps {st}", file=sys.stderr, flush=True)
                sec = time_context(ctx, stream, st, 4, torch, loops, key)
                out[key] = {"seconds": sec, "nodes": sp.n, "steps": st, "config": ctx.config()}
            torch.cuda.synchronize()
    return out


def variance_accuracy(torch, gmf, wl, stream):
    """The accuracy half of the metric, outside the timed region: the 64^3 tau
    sweep (tau 0.51, 0.6, 1, 2, 5, k_B T 1e-4, one batched context per
    precision, same seeds so the noise is paired), 2000 warm-up + 20000 steps
    sampled every 10. Reports FP32-shifted over FP64-plain variance ratios of
    the ten sampled observables and both precisions' ratios to the
    equilibrium values (rho0 k_BT / cs2 for drho, rho0 k_BT for j and u,
    3 rho0 k_BT for sum j, 5 rho0 k_BT for sum Pi_aa, rho0 k_BT for
    sum_{a<b} Pi_ab; times 1 - 1/N for a spatial variance)."""
    import numpy as np
    w = wl.tau_sweep("fp32")
    specs = [gmf.ReplicaSpec(*b.n, rho0=b.rho0, tau=b.tau, kbt=b.kbt, seed=b.seed) for b in w.boxes]
    kbt, n = w.boxes[0].kbt, specs[0].n
    theory = np.array([3 * kbt, kbt, kbt, kbt, 3 * kbt, 5 * kbt, kbt, kbt, kbt, kbt]) * (1 - 1.0 / n)
    var, rate = {}, {}
    t0 = time.perf_counter()
    for prec in (gmf.FP32_SHIFTED, gmf.FP64):
        with gmf.Context(specs, precision=prec, sample_every=w.sample_every, stream=stream, tune=1) as ctx:
            ctx.step(w.warmup)
            ctx.reset_stats()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ctx.step(w.steps)
            e1.record(stream)
            st = [ctx.stats(r) for r in range(len(specs))]
            torch.cuda.synchronize()
            rate[prec] = sum(sp.n for sp in specs) * w.steps / (e0.elapsed_time(e1) / 1e3) / 1e9
        var[prec] = np.array([s["sum_var"] / s["nsamples"] for s in st])
    torch.cuda.synchronize()
    ratio = var[gmf.FP32_SHIFTED] / var[gmf.FP64]
    er32, er64 = var[gmf.FP32_SHIFTED] / theory, var[gmf.FP64] / theory
    return {"workload": w.name, "taus": [b.tau for b in w.boxes], "samples": w.steps // w.sample_every,
            "fp32_over_fp64_variance": {"min": round(float(ratio.min()), 8), "max": round(float(ratio.max()), 8),
                                        "max_abs_dev": float(f"{float(np.max(np.abs(ratio - 1))):.3e}")},
            "er_fp64": {"min": round(float(er64.min()), 4), "max": round(float(er64.max()), 4)},
            "er_fp32": {"min": round(float(er32.min()), 4), "max": round(float(er32.max()), 4)},
            "er_fp64_tau_ge_0.6": {"min": round(float(er64[1:].min()), 4), "max": round(float(er64[1:].max()), 4)},
            # rate of the sampled step loop (five 64^3 boxes in one batched context, sampled
            # every 10 steps); the buffers (28 / 57 MB) stay in the last-level cache
            "glups_sampled_every10": {"fp32": round(rate[gmf.FP32_SHIFTED], 3), "fp64": round(rate[gmf.FP64], 3)},
            "seconds": round(time.perf_counter() - t0, 1)}


def copy_probe(torch, gmf, gbytes=1.812, reps=20):
    """The library's streaming copy of one 256^3 FP32 population buffer: the
    practical bandwidth ceiling, and the reference that scales the rocprofv3
    FETCH_SIZE / WRITE_SIZE counters to bytes."""
    n = (int(gbytes * 1e9) // 16) * 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    for _ in range(3):
        gmf.copy_probe(a.data_ptr(), b.data_ptr(), 4 * n, s)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        gmf.copy_probe(a.data_ptr(), b.data_ptr(), 4 * n, s)
    e1.record(s)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    return {"bytes_read_plus_written": 2 * 4 * n, "seconds": sec, "gbs": 2 * 4 * n / sec / 1e9}


def read_probe(torch, gmf, gbytes=1.812, reps=5):
    """Read rates of the library's plain read of one 256^3 FP32 population
    buffer: right after the library's copy has written it (the situation of
    every spectrum pass, which reads what the pass before it wrote), once more
    straight after that, and of the copy's source buffer, which was only read
    before.  The first is the ceiling of kernels that read freshly written
    data; each figure is the mean over `reps` rounds, HIP events around one
    launch."""
    n = (int(gbytes * 1e9) // 16) * 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    names = ("after_write", "again", "read_only_buffer")
    ms = {k: 0.0 for k in names}
    for r in range(reps + 1):
        gmf.copy_probe(a.data_ptr(), b.data_ptr(), 4 * n, s)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        for i, buf in enumerate((b, b, a)):
            ev[2 * i].record(s)
            gmf.read_probe(buf.data_ptr(), 4 * n, flag.data_ptr(), s)
            ev[2 * i + 1].record(s)
        torch.cuda.synchronize()
        if r:   # the first round warms up
            for i, k in enumerate(names):
                ms[k] += ev[2 * i].elapsed_time(ev[2 * i + 1]) / reps
    assert int(flag.item()) == 0
    return {"bytes": 4 * n, **{f"{k}_gbs": round(4 * n / (ms[k] * 1e-3) / 1e9, 1) for k in names}}


def cpu_baseline(target_seconds=12.0):
    """The FP64 oracle as written, on the host, on a bounded sample of the
    headline workload itself (the 256^3 box, tau 0.8, k_B T 1e-4, seed 1, from
    rest): OpenMP over z planes on every thread it gets, as many whole steps as
    fit in about target_seconds (the reported value); then one thread on a 64^3
    box with the same parameters."""
    import oracle

    def rate(L, seconds):
        p = oracle.params(L, rho0=1.0, tau=0.8, kbt=1e-4, seed=1)
        f = oracle.rest_state(p)
        t0 = time.perf_counter()
        oracle.run(p, f, 0, 1)                       # sizes the run
        dt = time.perf_counter() - t0
        steps = max(1, int(seconds / max(dt, 1e-6)))
        t0 = time.perf_counter()
        oracle.run(p, f, 1, steps)
        dt = time.perf_counter() - t0
        return L ** 3 * steps / dt / 1e9, steps, dt

    threads = oracle.num_threads()
    glups, steps, dt = rate(256, target_seconds)
    oracle.set_threads(1)
    glups1, steps1, dt1 = rate(64, target_seconds / 3)
    oracle.set_threads(threads)
    cpu = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next(l.split(":", 1)[1].strip() for l in fh if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"value": glups, "unit": "GLUPS", "cores": threads, "kind": "oracle",
            "sample": f"256^3 FP64 GMF-FLBM (the headline box: tau=0.8, kbt=1e-4, seed 1, from rest), {steps} step{'s' * (steps != 1)} "
                      f"({dt:.1f} s) on {threads} threads; single thread on 64^3 with the same parameters "
                      f"{glups1:.3g} GLUPS ({steps1} step{'s' * (steps1 != 1)}, {dt1:.1f} s)",
            "value_single_thread": glups1, "cpu": cpu, "host_cpus": os.cpu_count()}


def make_line(args, res) -> dict:
    """The bench's JSON line (without the oracle timing) from the timed
    results of run_gpu: the headline figures, its roofline and the extra
    workloads that ran."""
    rh = res["headline"]
    glups = rh["nodes"] * rh["steps"] / rh["seconds"] / 1e9
    ms = rh["seconds"] / rh["steps"] * 1e3
    # roofline of the step kernel: algorithmic bytes per launch over its average
    # launch duration, i.e. the events around the timed region over its launches
    # (the timed region is whole replays of graphs captured beforehand, which
    # launch the step kernel back to back; "step_loop" records what ran)
    kernel_s = rh["seconds"] / rh["steps"]
    bpn = (MOM_BYTES_PER_NODE if args.storage == "moments" else BYTES_PER_NODE)[args.precision]
    achieved = bpn * rh["nodes"] / kernel_s / 1e9
    line = {
        "metric": METRIC,
        "value": round(glups, 4),
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic (equilibrium fluid at rest, rho0=1, Philox noise)",
        "config": ({"workload": "d3q27_ensemble_64rep_fp32", "replicas": 64,
                    "boxes": "32 x 32^3 + 16 x 48^3 + 16 x 64^3", "rho0": 1.0, "kbt": 1e-4, "seeds": "1..64"}
                   if args.workload == "ensemble" else
                   {"workload": f"d3q27_256cube_{args.precision}_tau0.8", "lattice": [256, 256, 256], "rho0": 1.0,
                    "tau": 0.8, "kbt": 1e-4, "seed": 1}) | {
                   "precision": "fp64_plain" if args.precision == "fp64" else "fp32_shifted",
                   "layout": ("ten moments per node, A/B" if args.storage == "moments" else
                              "row-interleaved populations, " + ("in-place AA" if rh["config"]["streaming"] == "AA"
                                                                 else "A/B pull")),
                   "kernel_config": rh["config"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": profiled(("mstep" if args.storage == "moments" else "step") + f"_{args.precision}_" +
                                         ("ensemble" if args.workload == "ensemble" else "256"),
                                         rh["nodes"], rh["config"])},
        "hbm_frac": round(achieved / HBM_PEAK_GBS, 4),
        "mass_drift_rel": rh["mass_drift_rel"],
        "step_loop": res.get("step_loops", {}).get("headline"),
    }
    if "fp64" in res:
        r = res["fp64"]
        g = r["nodes"] * r["steps"] / r["seconds"] / 1e9
        gbs = BYTES_PER_NODE["fp64"] * g
        line["fp64_plain"] = {"workload": "d3q27_256cube_fp64_tau0.8", "glups": round(g, 4),
                              "ms_per_step": round(r["seconds"] / r["steps"] * 1e3, 5),
                              "gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                              "traffic": profiled("step_fp64_256", r["nodes"], r["config"]),
                              "steps": r["steps"], "kernel_config": r["config"]}
    if "batched" in res:
        r = res["batched"]
        g = r["nodes"] * r["steps"] / r["seconds"] / 1e9
        gbs = BYTES_PER_NODE["fp32"] * g
        line["fp32_batched"] = {"workload": r["workload"], "replicas": 64, "glups": round(g, 4),
                                "ms_per_step": round(r["seconds"] / r["steps"] * 1e3, 5),
                                "gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                                "traffic": profiled("step_fp32_ensemble", r["nodes"], r["config"]),
                                "steps": r["steps"], "kernel_config": r["config"]}
    if "batched_mom" in res:
        r = res["batched_mom"]
        g = r["nodes"] * r["steps"] / r["seconds"] / 1e9
        line["fp32_batched_moment_storage"] = {"workload": r["workload"] + ", moment storage", "replicas": 64,
                                               "glups": round(g, 4),
                                               "ms_per_step": round(r["seconds"] / r["steps"] * 1e3, 5),
                                               "steps": r["steps"], "kernel_config": r["config"]}
    if "aa" in res:
        r = res["aa"]
        g = r["nodes"] * r["steps"] / r["seconds"] / 1e9
        gbs = BYTES_PER_NODE["fp32"] * g
        line["fp32_aa_one_buffer"] = {"workload": "d3q27_256cube_fp32_tau0.8, in-place AA streaming",
                                      "glups": round(g, 4), "gbs": round(gbs, 1),
                                      "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "steps": r["steps"],
                                      "kernel_config": r["config"]}
    if "sampled" in res:
        r = res["sampled"]
        g = r["nodes"] * r["steps"] / r["seconds"] / 1e9
        line["fp32_sampled_every10"] = {"workload": "d3q27_256cube_fp32_tau0.8 with sampling", "glups": round(g, 4),
                                        "ms_per_step": round(r["seconds"] / r["steps"] * 1e3, 5),
                                        "overhead_vs_unsampled": round(glups / g - 1, 4)}
    if "spectrum" in res:
        r = res["spectrum"]
        g = r["nodes"] * r["steps"] / r["seconds"] / 1e9
        line["fp32_full_spectrum_every10"] = {
            "workload": "d3q27_256cube_fp32_tau0.8 with sampling and full-box shell spectra", "glups": round(g, 4),
            "ms_per_step": round(r["seconds"] / r["steps"] * 1e3, 5), "overhead_vs_unsampled": round(glups / g - 1, 4)}
    for key, bpn, name in (("fp32_512", "fp32", "d3q27_512cube_fp32_tau0.55"), ("fp64_512", "fp64", "d3q27_512cube_fp64_tau0.55")):
        if key in res:
            r = res[key]
            g = r["nodes"] * r["steps"] / r["seconds"] / 1e9
            gbs = BYTES_PER_NODE[bpn] * g
            line[key] = {"workload": name, "glups": round(g, 4), "gbs": round(gbs, 1),
                         "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "steps": r["steps"], "kernel_config": r["config"]}
    for key, bpn in (("mom_fp32", "fp32"), ("mom_fp64", "fp64")):
        if key in res:
            r = res[key]
            g = r["nodes"] * r["steps"] / r["seconds"] / 1e9
            gbs = MOM_BYTES_PER_NODE[bpn] * g
            line[f"{bpn}_moment_storage"] = {
                "workload": f"d3q27_256cube_{bpn}_tau0.8, moment storage (ten moments per node)",
                "glups": round(g, 4), "ms_per_step": round(r["seconds"] / r["steps"] * 1e3, 5),
                "gbs_algorithmic": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                "steps": r["steps"], "kernel_config": r["config"]}
            if bpn == "fp32":
                # the kernel is bound by its vector ALU work: VALU instructions per
                # launch (committed counter profile) over the live launch time
                valu = profiled("mstep_fp32_256", r["nodes"], r["config"], "valu_insts_per_launch")
                ns = r["seconds"] / r["steps"] * 1e9
                line[f"{bpn}_moment_storage"]["roofline"] = {
                    "bound": "alu", "unit": "wave64 VALU instructions per ns", "peak": VALU_PEAK,
                    "achieved": None if valu is None else round(valu / ns, 1),
                    "frac": None if valu is None else round(valu / ns / VALU_PEAK, 4),
                    "traffic": profiled("mstep_fp32_256", r["nodes"], r["config"])}
    if "variance_accuracy" in res:
        line["variance_accuracy"] = res["variance_accuracy"]
    # what each extra timed loop ran (graph replays, direct launches)
    extra_loops = {k: v for k, v in res.get("step_loops", {}).items() if k != "headline"}
    if extra_loops:
        line["extra_step_loops"] = extra_loops
    return line


def parse_args(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--tune", type=int, default=1, help="1: autotune the kernel variant at init (default)")
    ap.add_argument("--skip-extra", action="store_true", help="only the FP32 headline (profiling runs)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    ap.add_argument("--storage", choices=("populations", "moments"), default="populations",
                    help="storage of the FP32 256^3 headline run (moments: profiling of the moment-storage kernel)")
    ap.add_argument("--precision", choices=("fp32", "fp64"), default="fp32",
                    help="precision of the 256^3 headline run (fp64: profiling of the FP64 kernel, with --skip-extra)")
    ap.add_argument("--streaming", choices=("auto", "ab", "aa"), default="auto",
                    help="streaming pattern of the headline run (auto: A/B, or the tuner's choice with --tune 1)")
    ap.add_argument("--workload", choices=("box", "ensemble"), default="box",
                    help="headline run: the 256^3 box, or the 64-replica FP32 ensemble (profiling, with --skip-extra)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only time a plain device copy of one population buffer (bandwidth reference)")
    ap.add_argument("--read-probe", action="store_true",
                    help="only time a plain device read of one population buffer, right after a write and again")
    ap.add_argument("--profile-variants", choices=("fp32", "fp64", "ensemble", "moments"),
                    help="profiling: run every launch variant of one step kernel in a fixed order (tune 0)")
    ap.add_argument("--profile-sampler", action="store_true",
                    help="profiling: the 256^3 box sampled every 10 steps with full-box spectra (tune 0; --precision)")
    args = ap.parse_args(argv)
    if args.precision == "fp64" and not (args.skip_extra or args.profile_sampler):
        ap.error("--precision fp64 profiles the FP64 kernel alone: add --skip-extra")
    if args.workload == "ensemble" and (not args.skip_extra or args.precision != "fp32" or args.storage != "populations"):
        ap.error("--workload ensemble profiles the FP32 population kernel of the ensemble alone: add --skip-extra")
    return args


def main():
    args = parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (replicas and z slabs would "
              "shard over GPUs as independent contexts). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2601_03806_amd as gmf
    from paper_2601_03806_amd import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(int(os.environ.get("LOCAL_RANK", 0)))
    gmf.lib()   # fail loudly if the HIP library is missing
    if args.copy_probe:
        print(json.dumps({"copy_probe": copy_probe(torch, gmf)}), flush=True)
        return
    if args.read_probe:
        print(json.dumps({"read_probe": read_probe(torch, gmf), "copy_probe": copy_probe(torch, gmf)}), flush=True)
        return
    if args.profile_variants:
        print(json.dumps(profile_variants(args, torch, gmf, wl)), flush=True)
        return
    if args.profile_sampler:
        print(json.dumps(profile_sampler(args, torch, gmf, wl)), flush=True)
        return

    res = run_gpu(args, torch, gmf, wl)
    line = make_line(args, res)
    if not args.no_cpu and int(os.environ.get("RANK", 0)) == 0:
        print("[bench] oracle timing on the host", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
