"""bench.py's JSON line keeps its contract (CPU only: the line is assembled
from synthetic timing results, no GPU is touched)."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
N256 = 256 ** 3


def _cfg(**kw):
    c = {"nodes_per_thread": 1, "block": 256, "graph_steps": 64, "addressing": "group27", "streaming": "A/B",
         "block_map": "xcd/16", "storage": "populations"}
    c.update(kw)
    return c


def _results():
    mom = _cfg(block=640, addressing="none", block_map="xcd/64", storage="moments", tile="32x16x128")
    return {
        "headline": {"seconds": 1.2, "nodes": N256, "steps": 2000, "config": _cfg(), "mass_drift_rel": 1e-10},
        "fp64": {"seconds": 0.5, "nodes": N256, "steps": 400, "config": _cfg(addressing="plane", block_map="xcd/8192")},
        "batched": {"seconds": 0.53, "nodes": 7012352, "steps": 2000, "config": _cfg(streaming="AA"),
                    "workload": "d3q27_ensemble_64rep_fp32"},
        "batched_mom": {"seconds": 0.5, "nodes": 7012352, "steps": 2000, "config": mom,
                        "workload": "d3q27_ensemble_64rep_fp32"},
        "aa": {"seconds": 0.32, "nodes": N256, "steps": 500, "config": _cfg(streaming="AA")},
        "sampled": {"seconds": 0.32, "nodes": N256, "steps": 500},
        "spectrum": {"seconds": 0.4, "nodes": N256, "steps": 500},
        "mom_fp32": {"seconds": 0.24, "nodes": N256, "steps": 500, "config": mom},
        "mom_fp64": {"seconds": 0.29, "nodes": N256, "steps": 200, "config": mom},
        "fp32_512": {"seconds": 0.2, "nodes": 512 ** 3, "steps": 40, "config": _cfg(addressing="plane")},
        "fp64_512": {"seconds": 0.2, "nodes": 512 ** 3, "steps": 20, "config": _cfg(addressing="plane")},
        "variance_accuracy": {"workload": "d3q27_64cube_5tau_fp32"},
    }


def test_line_keeps_the_contract():
    args = bench.parse_args([])
    line = bench.make_line(args, _results())
    json.dumps(line)   # serialisable
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert key in line, key
    assert line["metric"] == bench.METRIC and line["unit"] == "GLUPS" and line["n_gpus"] == 1
    assert (line["steps"], line["warmup"]) == (2000, 50)
    assert line["higher_is_better"] is True and line["scaling"] == "weak" and line["vs_baseline"] is None
    assert line["dtype"] == "f32" and line["config"]["workload"] == "d3q27_256cube_fp32_tau0.8"
    assert "model" not in line["config"]
    # value: node updates per second of the timed loop; ms per step
    assert abs(line["value"] - N256 * 2000 / 1.2 / 1e9) < 1e-3
    assert abs(line["ms_per_step"] - 0.6) < 1e-9
    rf = line["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert abs(rf["achieved"] - 216 * N256 / 0.6e-3 / 1e9) < 0.1
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-4
    assert "traffic" in rf
    for extra in ("fp64_plain", "fp32_batched", "fp32_batched_moment_storage", "fp32_aa_one_buffer",
                  "fp32_sampled_every10", "fp32_full_spectrum_every10", "fp32_512", "fp64_512",
                  "fp32_moment_storage", "fp64_moment_storage", "variance_accuracy"):
        assert extra in line, extra
    assert abs(line["fp64_plain"]["hbm_frac"] - 432 * N256 * 400 / 0.5 / 1e9 / 8000) < 1e-4
    assert line["fp32_moment_storage"]["roofline"]["bound"] == "alu"


def test_fp64_and_moment_profiling_lines():
    res = _results()
    line = bench.make_line(bench.parse_args(["--precision", "fp64", "--skip-extra"]), {"headline": res["headline"]})
    assert line["dtype"] == "f64" and line["config"]["workload"] == "d3q27_256cube_fp64_tau0.8"
    assert abs(line["roofline"]["achieved"] - 432 * N256 / 0.6e-3 / 1e9) < 0.1
    ens = dict(res["batched"], mass_drift_rel=0.0)
    line = bench.make_line(bench.parse_args(["--workload", "ensemble", "--skip-extra"]), {"headline": ens})
    assert line["config"]["workload"] == "d3q27_ensemble_64rep_fp32" and line["config"]["replicas"] == 64
    assert abs(line["roofline"]["achieved"] - 216 * 7012352 / (0.53 / 2000) / 1e9) < 0.1
    head = dict(res["mom_fp32"], mass_drift_rel=0.0)
    line = bench.make_line(bench.parse_args(["--storage", "moments", "--skip-extra"]), {"headline": head})
    assert abs(line["roofline"]["achieved"] - 80 * N256 / (0.24 / 500) / 1e9) < 0.1


def test_multi_gpu_request_exits_with_a_message():
    run = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert run.returncode == 2 and "one GPU" in run.stderr
    run = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--precision", "fp64"],
                         capture_output=True, text=True, timeout=120)
    assert run.returncode == 2 and "--skip-extra" in run.stderr
    run = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "ensemble"],
                         capture_output=True, text=True, timeout=120)
    assert run.returncode == 2 and "--skip-extra" in run.stderr


def test_timed_loops_are_whole_graph_replays():
    """Every timed loop's graph length divides its step count, so the loop is
    whole replays of graphs captured before timing (the driver's --steps 20
    and the default 2000 included), and the line records what ran."""
    for steps in (1, 7, 10, 20, 40, 200, 500, 2000, 4096):
        g = bench.graph_len(steps)
        assert 1 <= g <= 64 and steps % g == 0
    assert bench.graph_len(20) == 20 and bench.graph_len(2000) == 50
    res = _results()
    res["step_loops"] = {"headline": {"steps_per_graph": 50, "graph_replays": 40, "graph_steps": 2000,
                                      "direct_steps": 0, "captured_in_timed_region": 0},
                         "fp64": {"steps_per_graph": 50, "graph_replays": 8, "graph_steps": 400,
                                  "direct_steps": 0, "captured_in_timed_region": 0}}
    line = bench.make_line(bench.parse_args([]), res)
    assert line["step_loop"]["graph_steps"] == 2000 and line["step_loop"]["direct_steps"] == 0
    assert line["extra_step_loops"]["fp64"]["graph_replays"] == 8
