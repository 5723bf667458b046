// gmf_graphplan.hpp -- which steps of a run go into captured HIP graphs.
//
// Host-only logic of the step loop (no HIP types), kept apart so that the CPU
// tests compile it with the host compiler.  A graph holds either one sampling
// step (step kernel, observables, statistics and spectra) or a run of `len`
// non-sampling steps; its kernels read the step index from a device counter
// that the graph advances by its length.  What a graph enqueues depends only
// on the parity of its first step (A/B buffers, AA pull/local halves) and on
// those two kinds, so it is keyed by (parity, len, sampling).  Lengths are the
// context's graph_steps G or, between two samples closer than that, the
// remainder (sample_every - 1) mod G of the run from one sample to the next:
// at most six graphs per context, none longer than G steps, whatever the
// sampling cadence.
#pragma once

#include <stdint.h>

#include <algorithm>

namespace gmf {

struct GraphPlan {
    int64_t sample_every;   // > 0: step t samples when t % sample_every == 0
    int64_t graph_steps;    // G; 0: every step is launched directly
};

inline int64_t graph_key(int64_t t, int64_t len, bool sample)
{
    return (len << 2) | ((int64_t)sample << 1) | (t & 1);
}

// The launch unit that starts at step t >= 0 with n steps left: a graph of the
// returned length (*sample: a sampling step), or 0 for one direct step.
inline int64_t plan_unit(const GraphPlan& p, int64_t t, int64_t n, bool* sample)
{
    *sample = false;
    const int64_t G = p.graph_steps, s = p.sample_every;
    if (G <= 0 || n <= 0) return 0;
    if (s > 0 && t % s == 0) {
        *sample = true;
        return 1;
    }
    const int64_t d = s > 0 ? s - t % s : INT64_MAX;   // non-sampling steps before the next sample
    const int64_t m = std::min(n, d);
    if (m >= G) return G;
    if (s > 0 && m == d && m == (s - 1) % G) return m;
    return 0;
}

// Visit every unit (t, len, sample) whose graph a run of n steps from step t0
// would launch, possibly with repeats, without running anything; visit returns
// nonzero to stop (that value is returned).  The units repeat with the step's
// parity and its place in the sampling cadence, so the walk covers the steps
// up to the first sample (at most sample_every; a run entered part-way plans
// its units differently), then one period of both (lcm(2, sample_every) <=
// 2 sample_every steps), plus two graph lengths; inside a long run between
// samples it keeps two full-length units and skips an even number of the
// rest, which leaves every later unit's parity unchanged.
template <class Visit>
int walk_graph_units(const GraphPlan& p, int64_t t0, int64_t n, Visit&& visit)
{
    const int64_t G = p.graph_steps, s = p.sample_every;
    if (G <= 0) return 0;
    int64_t t = t0;
    int64_t left = std::min<int64_t>(n, 3 * std::max<int64_t>(s, 0) + 2 * G + 2);
    while (left > 0) {
        bool sample = false;
        const int64_t len = plan_unit(p, t, left, &sample);
        if (len == 0) {
            t += 1;
            left -= 1;
            continue;
        }
        if (const int rc = visit(t, len, sample)) return rc;
        t += len;
        left -= len;
        if (len == G && !sample) {
            const int64_t d = s > 0 ? (t % s == 0 ? 0 : s - t % s) : left;
            const int64_t skip = std::max<int64_t>(0, (std::min(left, d) / G - 1) / 2 * 2) * G;
            t += skip;
            left -= skip;
        }
    }
    return 0;
}

}  // namespace gmf
