// hipGraph capture of step loops.  A loop of nsteps steps is captured once
// per (scheme, dt, nsteps, output pointers) and replayed, so a
// long run costs one graph launch instead of 2-3 kernel launches per step.
// The grid keeps the last few distinct loops (kGraphCacheEntries), so
// callers that alternate step counts or outputs do not re-capture.
// Only kernels are captured (no memset or memcpy nodes).  One graph holds
// at most kGraphMaxSteps steps: a longer call without per-step outputs
// replays a graph of that many steps and launches the remainder directly;
// a longer call with per-step outputs (every step writes its own entry, so
// no graph can be replayed) is launched directly.
#include <hip/hip_runtime.h>

#include "asd_internal.h"

using namespace asd;

static int run_graph(asd_grid g, int kind, double dt, int nsteps, const StepOut& out) {
    // callers only come here with a capturable (non-default) stream
    if (!g->graph_valid) {
        for (GraphEntry& e : g->graphs) {
            if (e.exec) (void)hipGraphExecDestroy(e.exec);
            e = GraphEntry{};
        }
        g->graph_valid = true;
    }
    GraphEntry* hit = nullptr;
    GraphEntry* victim = nullptr;  // an empty entry if there is one, else the least recently used
    for (GraphEntry& e : g->graphs) {
        if (e.exec && e.kind == kind && e.dt == dt && e.nsteps == nsteps && e.energy == out.energy &&
            e.series == out.series)
            hit = &e;
        const uint64_t age = e.exec ? e.last_use : 0;
        if (!victim || age < (victim->exec ? victim->last_use : 0)) victim = &e;
    }
    if (!hit) {
        if (victim->exec) (void)hipGraphExecDestroy(victim->exec);
        *victim = GraphEntry{};
        hipError_t e = hipStreamBeginCapture(g->st, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return asd_fail(ASD_EHIP, "begin capture: %s", hipGetErrorString(e));
        const int rc = kind == 1 ? enqueue_si_loop(g, dt, nsteps, out) : enqueue_explicit_loop(g, dt, nsteps, out);
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(g->st, &graph);
        if (rc != ASD_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e2 != hipSuccess) return asd_fail(ASD_EHIP, "end capture: %s", hipGetErrorString(e2));
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return asd_fail(ASD_EHIP, "graph instantiate: %s", hipGetErrorString(e));
        victim->exec = exec;
        victim->kind = kind;
        victim->dt = dt;
        victim->nsteps = nsteps;
        victim->energy = out.energy;
        victim->series = out.series;
        hit = victim;
    }
    hit->last_use = ++g->graph_clock;
    hipError_t e = hipGraphLaunch(hit->exec, g->st);
    if (e != hipSuccess) return asd_fail(ASD_EHIP, "graph launch: %s", hipGetErrorString(e));
    return ASD_OK;
}

static constexpr int kGraphMaxSteps = 2048;

static int run_graph_chunked(asd_grid g, int kind, double dt, int nsteps, const StepOut& out) {
    auto direct = [&](int n) {
        return kind == 1 ? enqueue_si_loop(g, dt, n, out) : enqueue_explicit_loop(g, dt, n, out);
    };
    if (nsteps <= kGraphMaxSteps) return run_graph(g, kind, dt, nsteps, out);
    if (out.any()) return direct(nsteps);
    int rc = ASD_OK, done = 0;
    for (; rc == ASD_OK && nsteps - done >= kGraphMaxSteps; done += kGraphMaxSteps)
        rc = run_graph(g, kind, dt, kGraphMaxSteps, out);
    if (rc == ASD_OK && done < nsteps) rc = direct(nsteps - done);
    return rc;
}

int run_si_graph(asd_grid g, double dt, int nsteps, const StepOut& out) {
    return run_graph_chunked(g, 1, dt, nsteps, out);
}
int run_explicit_graph(asd_grid g, double dt, int nsteps, const StepOut& out) {
    return run_graph_chunked(g, 2, dt, nsteps, out);
}
