"""Host logic of the captured step loop (gmf_graphplan.hpp), compiled for the
CPU: over many sampling cadences, graph lengths, start steps and splits of a
run into gmf_step calls, every graph a run launches is one that the prepare
walk captured beforehand, no graph is longer than graph_steps, at most six
distinct graphs exist, sampling steps sit alone in their graphs, and the units
cover the run exactly.  Also a sampling cadence far beyond any graph length
(the graph length no longer grows with it)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2601_03806_amd", "csrc")

DRIVER = r"""
#include "gmf_graphplan.hpp"
#include <cstdio>
#include <random>
#include <set>
using namespace gmf;
static int fail(const char* what, long s, long G, long t0, long n) {
    printf("FAIL %s s=%ld G=%ld t0=%ld n=%ld\n", what, s, G, t0, n);
    return 1;
}
int main() {
    std::mt19937_64 rng(2601);
    long cases = 0;
    for (int it = 0; it < 20000; ++it) {
        const long s = (it % 5 == 0) ? 0 : (long)(rng() % 40) + (it % 7 == 0 ? 1000 : 0);
        const long G = (long)(rng() % 70);
        const long t0 = (long)(rng() % 500);
        GraphPlan p{s, G};
        std::set<long> prepared;
        // a run split into up to four gmf_step calls, prepared before each
        long t = t0;
        const int calls = 1 + (int)(rng() % 4);
        std::set<long> used;
        for (int c = 0; c < calls; ++c) {
            const long n = (long)(rng() % 300);
            walk_graph_units(p, t, n, [&](long tt, long len, bool smp) {
                prepared.insert(graph_key(tt, len, smp));
                return 0;
            });
            long left = n;
            while (left > 0) {
                bool smp = false;
                const long len = plan_unit(p, t, left, &smp);
                if (len == 0) { t += 1; left -= 1; continue; }
                if (len > G || len > left) return fail("length", s, G, t, n);
                if (smp && (len != 1 || s == 0 || t % s != 0)) return fail("sampling unit", s, G, t, n);
                for (long j = smp ? 1 : 0; j < len; ++j)
                    if (s > 0 && (t + j) % s == 0) return fail("sample inside a run", s, G, t, n);
                const long key = graph_key(t, len, smp);
                if (!prepared.count(key)) return fail("not prepared", s, G, t, n);
                used.insert(key);
                t += len;
                left -= len;
            }
            if (left != 0) return fail("coverage", s, G, t, n);
        }
        if (used.size() > 6) return fail("too many graphs", s, G, t0, 0);
        ++cases;
    }
    // a cadence far beyond any graph length: graphs stay at G steps and the
    // prepare walk stays short (3 s + 2 G + 2 steps at most, skipping runs)
    {
        GraphPlan p{(long)2147483647, 64};
        long visits = 0;
        walk_graph_units(p, 5, (long)1 << 40, [&](long, long len, bool) { ++visits; return len > 64 ? 1 : 0; });
        if (visits > 20) return fail("long walk", p.sample_every, 64, 5, visits);
        bool smp;
        if (plan_unit(p, 0, 1000, &smp) != 1 || !smp) return fail("first sample", p.sample_every, 64, 0, 1000);
        if (plan_unit(p, 1, (long)1 << 40, &smp) != 64 || smp) return fail("run", p.sample_every, 64, 1, 0);
    }
    printf("ok %ld\n", cases);
    return 0;
}
"""


def test_graph_plan(tmp_path):
    src = tmp_path / "plan.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "plan"
    subprocess.run(["g++", "-O2", "-std=c++17", f"-I{CSRC}", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout
