// Launch-shape control, the autotuner and single-kernel measurement helpers.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "../../include/asd_extra.h"
#include "asd_internal.h"

using namespace asd;

extern "C" int asd_get_sweep_config(asd_grid g, int32_t axis, int32_t* wpl, int32_t* lpw, int32_t* P,
                                    int32_t* mmax) {
    if (!g) return asd_fail(ASD_EINVAL, "grid is NULL");
    if (axis < 0 || axis >= g->d.ndim) return asd_fail(ASD_EINVAL, "bad axis %d", axis);
    if (!wpl || !lpw || !P || !mmax) return asd_fail(ASD_EINVAL, "NULL output");
    const SweepCfg& c = g->cfg[axis];
    *wpl = c.wpl;
    *lpw = c.lpw;
    *P = c.P;
    *mmax = c.mmax;
    return ASD_OK;
}

static bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

extern "C" int asd_set_sweep_kernel(asd_grid g, int32_t axis, int32_t wpl, int32_t lpw, int32_t io,
                                    int32_t variant) {
    if (!g) return asd_fail(ASD_EINVAL, "grid is NULL");
    if (axis < 0 || axis >= g->d.ndim) return asd_fail(ASD_EINVAL, "bad axis %d", axis);
    if (!is_pow2(wpl) || !is_pow2(lpw)) return asd_fail(ASD_EINVAL, "wpl and lpw must be powers of two");
    if (io != 1 && io != 2) return asd_fail(ASD_EINVAL, "io must be 1 or 2");
    if (variant != SWEEP_FACE_SLOTS && variant != SWEEP_CELL_SLOTS)
        return asd_fail(ASD_EINVAL, "variant must be 0 (face slots) or 1 (cell slots)");
    if (variant == SWEEP_CELL_SLOTS && io != 1) return asd_fail(ASD_EINVAL, "the cell-slot variant takes io = 1");
    SweepCfg c;
    const bool chi = (g->d.flags & ASD_FLAG_PER_CELL_CHI) != 0;
    if (!choose_sweep_cfg((int)g->es, g->d.ndim, (int)g->d.n[axis], chi, wpl, lpw, &c, io, variant) ||
        c.wpl != wpl || c.lpw != lpw || c.io != io || c.variant != variant)
        return asd_fail(ASD_EUNSUPPORTED, "launch shape wpl=%d lpw=%d io=%d variant=%d does not fit", wpl, lpw, io,
                        variant);
    g->cfg[axis] = c;
    g->graph_valid = false;
    return ASD_OK;
}

extern "C" int asd_set_sweep_shape(asd_grid g, int32_t axis, int32_t wpl, int32_t lpw, int32_t io) {
    return asd_set_sweep_kernel(g, axis, wpl, lpw, io, SWEEP_FACE_SLOTS);
}

extern "C" int asd_set_sweep_config(asd_grid g, int32_t axis, int32_t wpl, int32_t lpw) {
    return asd_set_sweep_shape(g, axis, wpl, lpw, 1);
}

extern "C" int asd_get_sweep_io(asd_grid g, int32_t axis, int32_t* io) {
    if (!g) return asd_fail(ASD_EINVAL, "grid is NULL");
    if (axis < 0 || axis >= g->d.ndim) return asd_fail(ASD_EINVAL, "bad axis %d", axis);
    if (!io) return asd_fail(ASD_EINVAL, "NULL output");
    *io = g->cfg[axis].io;
    return ASD_OK;
}

extern "C" int asd_get_sweep_variant(asd_grid g, int32_t axis, int32_t* variant) {
    if (!g) return asd_fail(ASD_EINVAL, "grid is NULL");
    if (axis < 0 || axis >= g->d.ndim) return asd_fail(ASD_EINVAL, "bad axis %d", axis);
    if (!variant) return asd_fail(ASD_EINVAL, "NULL output");
    *variant = g->cfg[axis].variant;
    return ASD_OK;
}

extern "C" int asd_set_graphs(asd_grid g, int32_t mode) {
    if (!g) return asd_fail(ASD_EINVAL, "grid is NULL");
    if (mode != ASD_GRAPHS_OFF && mode != ASD_GRAPHS_AUTO && mode != ASD_GRAPHS_ALWAYS)
        return asd_fail(ASD_EINVAL, "graph mode must be ASD_GRAPHS_OFF, _AUTO or _ALWAYS");
    g->graph_mode = mode;
    g->graph_valid = false;
    return ASD_OK;
}

// Buffers of sweep `axis` run in isolation: input = the state that sweep
// reads during a step (T for the first sweep, else a scratch state), output
// = a scratch state that no later timed launch reads.  T is never written.
static void bench_buffers(asd_grid g, int axis, const void** in, void** out) {
    if (axis == 0) {
        *in = g->T;
        *out = g->tmp[0];
    } else if (axis == 1) {
        *in = g->tmp[0];
        *out = g->tmp[1];
    } else {
        *in = g->tmp[1];
        *out = g->tmp[0];
    }
}

// Fill the scratch inputs of sweeps 1.. with one real sweep chain from T.
static int bench_prepare_inputs(asd_grid g, double dt) {
    for (int axis = 0; axis + 1 < g->d.ndim; ++axis) {
        const void* in = axis == 0 ? g->T : g->tmp[axis - 1];
        int rc = enqueue_sweep(g, axis, dt, in, g->tmp[axis], 0, no_reduce(), nullptr, nullptr);
        if (rc) return rc;
    }
    return ASD_OK;
}

extern "C" int asd_bench_sweep(asd_grid g, int32_t axis, double dt, int32_t reps) {
    if (!g) return asd_fail(ASD_EINVAL, "grid is NULL");
    if (axis < 0 || axis >= g->d.ndim) return asd_fail(ASD_EINVAL, "bad axis %d", axis);
    if (!(std::isfinite(dt) && dt > 0.0)) return asd_fail(ASD_EINVAL, "dt must be finite and > 0");
    if (reps < 0) return asd_fail(ASD_EINVAL, "reps must be >= 0");
    int rc = check_fields(g, true);
    if (rc) return rc;
    rc = prepare(g, dt);
    if (rc) return rc;
    if (reps == 0) return bench_prepare_inputs(g, dt);
    const void* in;
    void* out;
    bench_buffers(g, axis, &in, &out);
    for (int r = 0; r < reps; ++r) {
        rc = enqueue_sweep(g, axis, dt, in, out, 0, no_reduce(), nullptr, nullptr);
        if (rc) return rc;
    }
    return ASD_OK;
}

extern "C" int asd_bench_copy(const void* src, void* dst, size_t nbytes, void* stream) {
    if (!src || !dst) return asd_fail(ASD_EINVAL, "NULL pointer");
    if (nbytes % 4) return asd_fail(ASD_EINVAL, "nbytes must be a multiple of 4");
    hipError_t e = launch_copy<float>((const float*)src, (float*)dst, (int64_t)(nbytes / 4), (hipStream_t)stream);
    if (e != hipSuccess) return asd_fail(ASD_EHIP, "copy launch: %s", hipGetErrorString(e));
    return ASD_OK;
}

extern "C" int asd_bench_copy_wide(const void* src, void* dst, size_t nbytes, void* stream) {
    if (!src || !dst) return asd_fail(ASD_EINVAL, "NULL pointer");
    if (nbytes % 4) return asd_fail(ASD_EINVAL, "nbytes must be a multiple of 4");
    if (((uintptr_t)src | (uintptr_t)dst) & 15) return asd_fail(ASD_EINVAL, "src and dst must be 16-byte aligned");
    hipError_t e = launch_copy_wide(src, dst, nbytes, (hipStream_t)stream);
    if (e != hipSuccess) return asd_fail(ASD_EHIP, "copy launch: %s", hipGetErrorString(e));
    return ASD_OK;
}

// ------------------------------------------------------------- autotuner

// Time reps whole steps (every sweep in order, each reading what the
// previous one wrote, as in the step loop) with the launch shapes cfg[],
// on the two scratch buffers: the first sweep reads T, T is never written.
static int time_chain(asd_grid g, double dt, int reps, const SweepCfg* cfg, float* ms) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return asd_fail(ASD_EHIP, "event create");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return asd_fail(ASD_EHIP, "event create");
    }
    const void* in = g->T;
    int cur = 0;  // scratch buffer written next
    auto chain = [&](int steps) {
        int rc = ASD_OK;
        for (int s = 0; s < steps && !rc; ++s)
            for (int d = 0; d < g->d.ndim && !rc; ++d) {
                void* out = g->tmp[cur];
                rc = enqueue_sweep(g, d, dt, in, out, 0, no_reduce(), &cfg[d], nullptr);
                in = out;
                cur ^= 1;
            }
        return rc;
    };
    int rc = chain(1);  // warm-up
    if (!rc && hipEventRecord(e0, g->st) != hipSuccess) rc = asd_fail(ASD_EHIP, "event record");
    if (!rc) rc = chain(reps);
    if (!rc && hipEventRecord(e1, g->st) != hipSuccess) rc = asd_fail(ASD_EHIP, "event record");
    if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = asd_fail(ASD_EHIP, "event sync");
    if (!rc && hipEventElapsedTime(ms, e0, e1) != hipSuccess) rc = asd_fail(ASD_EHIP, "elapsed");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

// Autotuner: for each sweep axis in turn, every admissible (tile body,
// waves per line, lines per workgroup, io) shape is timed inside whole steps
// (the other axes at their current shapes), and the fastest is kept; two
// passes.  A shape's time
// is the best of three timings: shapes a few per cent apart are otherwise
// ranked by the noise of a single sub-millisecond timing.
extern "C" int asd_tune(asd_grid g, double dt, int32_t reps) {
    if (!g) return asd_fail(ASD_EINVAL, "grid is NULL");
    if (!(std::isfinite(dt) && dt > 0.0)) return asd_fail(ASD_EINVAL, "dt must be finite and > 0");
    if (reps < 1) return asd_fail(ASD_EINVAL, "reps must be >= 1");
    int rc = check_fields(g, true);
    if (rc) return rc;
    rc = prepare(g, dt);
    if (rc) return rc;
    const bool chi = (g->d.flags & ASD_FLAG_PER_CELL_CHI) != 0;
    SweepCfg cur[3] = {g->cfg[0], g->cfg[1], g->cfg[2]};
    for (int pass = 0; pass < 2; ++pass) {
        for (int axis = 0; axis < g->d.ndim; ++axis) {
            SweepCfg best = cur[axis];
            float best_ms = 1e30f;
            for (int variant = SWEEP_FACE_SLOTS; variant <= SWEEP_CELL_SLOTS; ++variant)
            for (int io = 1; io <= (variant == SWEEP_CELL_SLOTS ? 1 : 2); ++io)
            for (int wpl = 1; wpl <= 16; wpl *= 2) {
                for (int lpw = 1; wpl * lpw * io <= 16; lpw *= 2) {
                    SweepCfg c;
                    if (!choose_sweep_cfg((int)g->es, g->d.ndim, (int)g->d.n[axis], chi, wpl, lpw, &c, io, variant))
                        continue;
                    if (c.wpl != wpl || c.lpw != lpw || c.io != io || c.variant != variant) continue;
                    SweepCfg trial[3] = {cur[0], cur[1], cur[2]};
                    trial[axis] = c;
                    float ms = 1e30f;
                    for (int t = 0; t < 3; ++t) {
                        float one = 0.f;
                        rc = time_chain(g, dt, reps, trial, &one);
                        if (rc) return rc;
                        ms = std::min(ms, one);
                    }
                    if (ms < best_ms) {
                        best_ms = ms;
                        best = c;
                    }
                }
            }
            cur[axis] = best;
        }
    }
    for (int a = 0; a < 3; ++a) g->cfg[a] = cur[a];
    g->graph_valid = false;
    return ASD_OK;
}
