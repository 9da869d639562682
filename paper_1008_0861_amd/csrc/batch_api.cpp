// Batched independent 2-D problems (asd_batch_*): each problem is a full
// grid (its own slice of the workspace, face coefficients and T* buffer);
// the batch adds the launch tables of the persistent and grouped kernels,
// the largest-first assignment of problems to workgroups, and an autotuner
// that picks the schedule (persistent / grouped) and workgroup size by
// timing them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/asd_extra.h"
#include "asd_internal.h"

using namespace asd;

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

static const int kBatchRingSlots = 4;
struct asd_batch_s {
    asd_desc d0{};
    int nprob = 0;
    hipStream_t st = nullptr;
    std::vector<asd_grid> sub;
    std::vector<double> dt;
    std::vector<char*> sub_ws;
    // launch shape shared by every problem in the batch kernels
    int mmax = 8, nthreads = 512, mode = 0;
    int variant = SWEEP_FACE_SLOTS;  // tile body of every problem's sweeps
    size_t lds = 0;
    std::vector<SweepCfg> cfg;  // [2 * p + d]
    // device tables (workspace) and their host images
    char* d_probs = nullptr;
    int* d_off = nullptr;
    int* d_list = nullptr;
    int* d_gs[2] = {nullptr, nullptr};
    int nwg = 0, ngroups[2] = {0, 0};
    std::vector<char> h_probs;
    std::vector<int> h_off, h_list, h_gs[2];
    bool dirty = true;
    // per-problem outputs (workspace): status bits, last (E, min, max), and
    // the ring of grouped-mode y-sweep partials
    unsigned* d_flags = nullptr;
    double* d_stats = nullptr;
    double* d_ring = nullptr;
    int ring_slots = kBatchRingSlots;
    int64_t ring_tiles = 0;  // tiles per ring slot (at most one per y-sweep line)
    // captured step loops: (mode, nsteps, energy) of the current tables
    bool use_graphs = true;
    uint64_t version = 1;   // bumped whenever the tables or the launch shape change
    struct Entry { hipGraphExec_t exec = nullptr; int mode = 0, nsteps = 0; double* energy = nullptr;
                   uint64_t version = 0, last_use = 0; };
    Entry graphs[4];
    uint64_t clock = 0;
};

static const int kMaxWorkgroups = 1024;

static size_t probs_bytes(const asd_desc* d0, int nprob) {
    const size_t one = d0->dtype == ASD_F64 ? sizeof(BatchProblem<double>) : sizeof(BatchProblem<float>);
    return align256(one * (size_t)nprob);
}
static size_t table_bytes(int nprob) {
    return align256(sizeof(int) * (size_t)(kMaxWorkgroups + 1)) + align256(sizeof(int) * (size_t)nprob) +
           2 * align256(sizeof(int) * (size_t)(nprob + 1));
}
// y-sweep lines of all problems (an upper bound of their y-sweep tiles)
static int64_t ring_tiles_for(const asd_desc* descs, int nprob) {
    int64_t t = 0;
    for (int p = 0; p < nprob; ++p) t += descs[p].n[0];
    return t;
}
static size_t outputs_bytes(const asd_desc* descs, int nprob) {
    return align256(sizeof(unsigned) * (size_t)nprob) + align256(3 * sizeof(double) * (size_t)nprob) +
           align256((size_t)kBatchRingSlots * ring_tiles_for(descs, nprob) * 3 * sizeof(double));
}

static int check_descs(const asd_desc* descs, int32_t nprob) {
    if (!descs) return asd_fail(ASD_EINVAL, "descs is NULL");
    if (nprob < 1) return asd_fail(ASD_EINVAL, "nprob must be >= 1");
    for (int p = 0; p < nprob; ++p) {
        int rc = validate_desc(&descs[p]);
        if (rc) return rc;
        if (descs[p].ndim != 2) return asd_fail(ASD_EUNSUPPORTED, "batched problems must be 2-D");
        if (descs[p].bc != descs[0].bc || descs[p].dtype != descs[0].dtype || descs[p].limiter != descs[0].limiter)
            return asd_fail(ASD_EINVAL, "problem %d: bc, dtype and limiter must match problem 0", p);
        if ((descs[p].flags & ASD_FLAG_PER_CELL_CHI) || descs[p].chi_exp != 0.0)
            return asd_fail(ASD_EUNSUPPORTED, "batched problems take a constant chi_par");
        if (descs[p].flags & (ASD_FLAG_FOUR_STEP | ASD_FLAG_REVERSE_ORDER))
            return asd_fail(ASD_EUNSUPPORTED, "batched problems take the 2-step scheme in the order x, y");
    }
    return ASD_OK;
}

extern "C" int asd_batch_workspace_bytes(const asd_desc* descs, int32_t nprob, size_t* bytes) {
    int rc = check_descs(descs, nprob);
    if (rc) return rc;
    if (!bytes) return asd_fail(ASD_EINVAL, "bytes is NULL");
    size_t tot = probs_bytes(descs, nprob) + table_bytes(nprob) + outputs_bytes(descs, nprob);
    for (int p = 0; p < nprob; ++p) {
        size_t b = 0;
        rc = asd_workspace_bytes(&descs[p], &b);
        if (rc) return rc;
        tot += align256(b);
    }
    *bytes = tot;
    return ASD_OK;
}

// Launch shape of problem line length n for a fixed workgroup size.
// A problem's line shape under the batch's workgroup size and per-lane
// capacity mmax: the fewest waves per line that fit, and the tile's own
// capacity, mmax or (when its lines fit) mmax / 2 (the batch kernels run
// either; a line shorter than the batch's longest then does not pad every
// lane to the longest one's capacity).
static bool batch_line_cfg(int es, int n, int nthreads, int mmax, int variant, SweepCfg* out) {
    // capacity 16 on the face body: lines of 257-512 cells take half a wave
    // each (32 lanes of 9-16 cells, two lines per wave); shorter lines do
    // better on the one-line tiles of capacity 4 or 8
    if (variant == SWEEP_FACE_SLOTS && mmax == 16 && n > 256 && (n + 31) / 32 <= 16 && nthreads >= 64) {
        const int lpw = nthreads / 32;
        if (sweep_lds(es, 2, n, lpw, 1, nthreads, 16, variant, 1) <= kLdsLimit) {
            out->wpl = 1;
            out->lpw = lpw;
            out->P = 32;
            out->mmax = 16;
            out->io = 1;
            out->variant = variant;
            out->half = 1;
            return true;
        }
    }
    for (int wpl = 1; 64 * wpl <= nthreads; wpl *= 2) {
        const int P = std::min(64 * wpl, pow2_floor(n));
        const int m = (n + P - 1) / P;
        if (m > mmax) continue;
        const int lpw = nthreads / (64 * wpl);
        // the tile's own capacity: mmax, mmax / 2, or (capacity 16) 4
        int own = mmax >= 4 && 2 * m <= mmax ? mmax / 2 : mmax;
        if (mmax == 16 && m <= 4) own = 4;
        if (sweep_lds(es, 2, n, lpw, wpl, nthreads, own, variant) > kLdsLimit) continue;
        out->wpl = wpl;
        out->lpw = lpw;
        out->P = P;
        out->mmax = own;
        out->variant = variant;
        out->half = 0;
        return true;
    }
    return false;
}

// Choose the per-lane capacity (the smallest from mmax_from up that fits
// every problem) for a workgroup size and tile body; fills b->cfg and
// b->lds.  A larger capacity gives long lines fewer waves each.
static int batch_shape(asd_batch b, int nthreads, int variant, int mmax_from = 4) {
    const int es = b->d0.dtype == ASD_F64 ? 8 : 4;
    for (int mmax : {4, 8, 16}) {
        if (mmax < mmax_from) continue;
        if (nthreads > sweep_threads_cap(es, mmax, variant)) continue;
        std::vector<SweepCfg> cfg(2 * b->nprob);
        size_t lds = 0;
        bool ok = true;
        for (int p = 0; p < b->nprob && ok; ++p) {
            for (int d = 0; d < 2 && ok; ++d) {
                const int n = (int)b->sub[p]->d.n[d];
                ok = batch_line_cfg(es, n, nthreads, mmax, variant, &cfg[2 * p + d]);
                if (ok)
                    lds = std::max(lds, sweep_lds(es, 2, n, cfg[2 * p + d].lpw, cfg[2 * p + d].wpl, nthreads,
                                                  cfg[2 * p + d].mmax, variant, cfg[2 * p + d].half));
            }
        }
        if (!ok) continue;
        b->mmax = mmax;
        b->nthreads = nthreads;
        b->variant = variant;
        b->cfg = cfg;
        b->lds = lds;
        b->dirty = true;
        ++b->version;
        return ASD_OK;
    }
    return asd_fail(ASD_EUNSUPPORTED, "no batch launch shape with %d threads and tile body %d fits every problem",
                    nthreads, variant);
}

extern "C" int asd_batch_init(const asd_desc* descs, int32_t nprob, void* dev_ws, size_t ws_bytes, void* stream,
                              asd_batch* out) {
    size_t need = 0;
    int rc = asd_batch_workspace_bytes(descs, nprob, &need);
    if (rc) return rc;
    if (!out) return asd_fail(ASD_EINVAL, "out is NULL");
    if (!dev_ws || ((uintptr_t)dev_ws & 255)) return asd_fail(ASD_EWORKSPACE, "workspace NULL or not 256-byte aligned");
    if (ws_bytes < need) return asd_fail(ASD_EWORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    asd_batch b = new (std::nothrow) asd_batch_s();
    if (!b) return asd_fail(ASD_EINVAL, "out of host memory");
    b->d0 = descs[0];
    b->nprob = nprob;
    b->st = (hipStream_t)stream;
    char* cur = (char*)dev_ws;
    b->d_probs = cur;
    cur += probs_bytes(descs, nprob);
    b->d_off = (int*)cur;
    cur += align256(sizeof(int) * (size_t)(kMaxWorkgroups + 1));
    b->d_list = (int*)cur;
    cur += align256(sizeof(int) * (size_t)nprob);
    for (int d = 0; d < 2; ++d) {
        b->d_gs[d] = (int*)cur;
        cur += align256(sizeof(int) * (size_t)(nprob + 1));
    }
    b->d_flags = (unsigned*)cur;
    cur += align256(sizeof(unsigned) * (size_t)nprob);
    b->d_stats = (double*)cur;
    cur += align256(3 * sizeof(double) * (size_t)nprob);
    b->ring_tiles = ring_tiles_for(descs, nprob);
    b->d_ring = (double*)cur;
    cur += align256((size_t)b->ring_slots * b->ring_tiles * 3 * sizeof(double));
    b->sub.assign(nprob, nullptr);
    b->dt.assign(nprob, 0.0);
    for (int p = 0; p < nprob; ++p) {
        size_t wb = 0;
        asd_workspace_bytes(&descs[p], &wb);
        rc = asd_init_grid(&descs[p], cur, wb, stream, &b->sub[p]);
        if (rc) {
            asd_batch_destroy(b);
            return rc;
        }
        b->sub[p]->graph_mode = ASD_GRAPHS_OFF;
        // the sequential schedule's folds report into the batch's per-problem status
        b->sub[p]->flags = b->d_flags + p;
        b->sub[p]->stats = b->d_stats + 3 * p;
        cur += align256(wb);
    }
    rc = batch_shape(b, 512, SWEEP_FACE_SLOTS);
    if (rc) rc = batch_shape(b, 256, SWEEP_FACE_SLOTS);
    if (rc) {
        asd_batch_destroy(b);
        return rc;
    }
    *out = b;
    return ASD_OK;
}

static void drop_graphs(asd_batch b) {
    for (auto& e : b->graphs) {
        if (e.exec) (void)hipGraphExecDestroy(e.exec);
        e = asd_batch_s::Entry{};
    }
}

extern "C" int asd_batch_destroy(asd_batch b) {
    if (!b) return asd_fail(ASD_EINVAL, "batch is NULL");
    drop_graphs(b);
    for (asd_grid g : b->sub)
        if (g) asd_destroy(g);
    delete b;
    return ASD_OK;
}

extern "C" int asd_batch_set_problem(asd_batch b, int32_t p, void* dev_T, void* dev_bx, void* dev_by, double dt) {
    if (!b) return asd_fail(ASD_EINVAL, "batch is NULL");
    if (p < 0 || p >= b->nprob) return asd_fail(ASD_EINVAL, "problem index %d out of range", p);
    if (!(std::isfinite(dt) && dt > 0.0)) return asd_fail(ASD_EINVAL, "dt must be finite and > 0");
    asd_grid g = b->sub[p];
    int rc = asd_set_field(g, ASD_FIELD_T, dev_T, g->N, g->d.dtype);
    if (!rc) rc = asd_set_field(g, ASD_FIELD_BX, dev_bx, g->N, g->d.dtype);
    if (!rc) rc = asd_set_field(g, ASD_FIELD_BY, dev_by, g->N, g->d.dtype);
    if (rc) return rc;
    b->dt[p] = dt;
    b->dirty = true;
    ++b->version;
    return ASD_OK;
}

extern "C" int asd_batch_set_block(asd_batch b, int32_t nthreads) {
    if (!b) return asd_fail(ASD_EINVAL, "batch is NULL");
    if (nthreads != 256 && nthreads != 512 && nthreads != 1024)
        return asd_fail(ASD_EINVAL, "nthreads must be 256, 512 or 1024");
    return batch_shape(b, nthreads, b->variant);
}

extern "C" int asd_batch_set_variant(asd_batch b, int32_t variant) {
    if (!b) return asd_fail(ASD_EINVAL, "batch is NULL");
    if (variant != SWEEP_FACE_SLOTS && variant != SWEEP_CELL_SLOTS)
        return asd_fail(ASD_EINVAL, "variant must be 0 (face slots) or 1 (cell slots)");
    return batch_shape(b, b->nthreads, variant);
}

extern "C" int asd_batch_set_capacity(asd_batch b, int32_t mmax) {
    if (!b) return asd_fail(ASD_EINVAL, "batch is NULL");
    if (mmax != 4 && mmax != 8 && mmax != 16) return asd_fail(ASD_EINVAL, "capacity must be 4, 8 or 16");
    return batch_shape(b, b->nthreads, b->variant, mmax);
}

extern "C" int asd_batch_get_variant(asd_batch b, int32_t* variant) {
    if (!b) return asd_fail(ASD_EINVAL, "batch is NULL");
    if (!variant) return asd_fail(ASD_EINVAL, "NULL output");
    *variant = b->variant;
    return ASD_OK;
}

// Build (if needed) and upload the launch tables.
template <typename T>
static int batch_tables(asd_batch b) {
    if (!b->dirty) return ASD_OK;
    const int np = b->nprob;
    b->h_probs.assign(sizeof(BatchProblem<T>) * np, 0);
    BatchProblem<T>* probs = (BatchProblem<T>*)b->h_probs.data();
    std::vector<double> load(np);
    for (int p = 0; p < np; ++p) {
        asd_grid g = b->sub[p];
        for (int d = 0; d < 2; ++d) {
            const void* in = d == 0 ? g->T : g->tmp[0];
            void* out = d == 0 ? g->tmp[0] : g->T;
            int rc = fill_sweep_params<T>(g, d, in, out, 0, b->cfg[2 * p + d], &probs[p].sweep[d]);
            if (rc) return rc;
            const int nt1 = probs[p].sweep[d].nt1, lpw = b->cfg[2 * p + d].lpw;
            probs[p].ngroups[d] = (nt1 + lpw - 1) / lpw;
            probs[p].mmax[d] = b->cfg[2 * p + d].mmax;
            probs[p].half[d] = b->cfg[2 * p + d].half;
        }
        probs[p].dirichlet = g->d.bc == ASD_BC_DIRICHLET;
        probs[p].dV = g->d.h[0] * g->d.h[1];
        load[p] = (double)g->N;
    }
    // largest first, each to the least-loaded workgroup
    b->nwg = std::min(np, kMaxWorkgroups);
    std::vector<int> order(np);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return load[a] > load[c]; });
    std::vector<double> wl(b->nwg, 0.0);
    std::vector<std::vector<int>> owned(b->nwg);
    for (int p : order) {
        const int w = (int)(std::min_element(wl.begin(), wl.end()) - wl.begin());
        owned[w].push_back(p);
        wl[w] += load[p];
    }
    b->h_off.assign(b->nwg + 1, 0);
    b->h_list.clear();
    for (int w = 0; w < b->nwg; ++w) {
        b->h_off[w] = (int)b->h_list.size();
        b->h_list.insert(b->h_list.end(), owned[w].begin(), owned[w].end());
    }
    b->h_off[b->nwg] = (int)b->h_list.size();
    for (int d = 0; d < 2; ++d) {
        b->h_gs[d].assign(np + 1, 0);
        for (int p = 0; p < np; ++p) b->h_gs[d][p + 1] = b->h_gs[d][p] + probs[p].ngroups[d];
        b->ngroups[d] = b->h_gs[d][np];
    }
    for (int p = 0; p < np; ++p) probs[p].tile0 = b->h_gs[1][p];
    if (b->ngroups[1] > b->ring_tiles) return asd_fail(ASD_EUNSUPPORTED, "more y-sweep tiles than ring entries");
    // synchronous uploads: the tables change only with the problem set
    hipError_t e = hipMemcpy(b->d_probs, b->h_probs.data(), b->h_probs.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->d_off, b->h_off.data(), sizeof(int) * b->h_off.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->d_list, b->h_list.data(), sizeof(int) * b->h_list.size(), hipMemcpyHostToDevice);
    for (int d = 0; d < 2 && e == hipSuccess; ++d)
        e = hipMemcpy(b->d_gs[d], b->h_gs[d].data(), sizeof(int) * (np + 1), hipMemcpyHostToDevice);
    if (e != hipSuccess) return asd_fail(ASD_EHIP, "batch tables: %s", hipGetErrorString(e));
    b->dirty = false;
    ++b->version;
    return ASD_OK;
}

// The kernels of one batch call (eager, or under stream capture).
template <typename T>
static int enqueue_batch(asd_batch b, int nsteps, int mode, double* energy) {
    const BatchProblem<T>* probs = (const BatchProblem<T>*)b->d_probs;
    const bool dir = b->d0.bc == ASD_BC_DIRICHLET;
    BatchOut out{};
    if (energy) {
        out.energy = energy;
        out.stride = nsteps + 1;
        out.flags = b->d_flags;
        out.stats = b->d_stats;
        out.partials = b->d_ring;
        out.slot_stride = (int)(b->ring_tiles * 3);
    }
    hipError_t e = hipSuccess;
    if (energy) e = launch_batch_reduce0<T>(probs, b->nprob, out, b->st);
    if (mode == 0) {
        if (e == hipSuccess)
            e = launch_batch_persistent<T>(probs, b->d_off, b->d_list, b->nwg, nsteps, b->mmax, b->nthreads, b->lds,
                                           b->d0.limiter, dir, b->variant, out, b->st);
    } else {
        int used = 0;
        for (int s = 0; s < nsteps && e == hipSuccess; ++s) {
            for (int d = 0; d < 2 && e == hipSuccess; ++d) {
                double* part = energy && d == 1 ? b->d_ring + (size_t)used * out.slot_stride : nullptr;
                e = launch_batch_grouped<T>(probs, b->d_gs[d], b->nprob, b->ngroups[d], d, b->mmax, b->nthreads,
                                            b->lds, b->d0.limiter, dir, b->variant, part, b->st);
            }
            if (e == hipSuccess && energy && (++used == b->ring_slots || s == nsteps - 1)) {
                BatchOut f = out;
                f.first = s + 2 - used;
                f.count = used;
                f.last = s == nsteps - 1;
                e = launch_batch_fold<T>(probs, b->nprob, f, b->st);
                used = 0;
            }
        }
    }
    if (e != hipSuccess) return asd_fail(ASD_EHIP, "batch launch: %s", hipGetErrorString(e));
    return ASD_OK;
}

// Replay (capturing on first use) the graph of a call: one graph launch per
// call, the four most recently used (mode, nsteps, energy) kept.
template <typename T>
static int run_batch_graph(asd_batch b, int nsteps, int mode, double* energy) {
    asd_batch_s::Entry* hit = nullptr;
    asd_batch_s::Entry* victim = nullptr;
    for (auto& en : b->graphs) {
        if (en.exec && en.version != b->version) {
            (void)hipGraphExecDestroy(en.exec);
            en = asd_batch_s::Entry{};
        }
        if (en.exec && en.mode == mode && en.nsteps == nsteps && en.energy == energy) hit = &en;
        const uint64_t age = en.exec ? en.last_use : 0;
        if (!victim || age < (victim->exec ? victim->last_use : 0)) victim = &en;
    }
    if (!hit) {
        if (victim->exec) (void)hipGraphExecDestroy(victim->exec);
        *victim = asd_batch_s::Entry{};
        hipError_t e = hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return asd_fail(ASD_EHIP, "begin capture: %s", hipGetErrorString(e));
        const int rc = enqueue_batch<T>(b, nsteps, mode, energy);
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(b->st, &graph);
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
        victim->mode = mode;
        victim->nsteps = nsteps;
        victim->energy = energy;
        victim->version = b->version;
        hit = victim;
    }
    hit->last_use = ++b->clock;
    hipError_t e = hipGraphLaunch(hit->exec, b->st);
    if (e != hipSuccess) return asd_fail(ASD_EHIP, "graph launch: %s", hipGetErrorString(e));
    return ASD_OK;
}

static constexpr int kBatchGraphMaxSteps = 2048;

template <typename T>
static int batch_step_t(asd_batch b, int nsteps, int mode, double* energy) {
    for (int p = 0; p < b->nprob; ++p) {
        asd_grid g = b->sub[p];
        if (!(b->dt[p] > 0.0)) return asd_fail(ASD_ENOTSET, "problem %d has not been set", p);
        int rc = check_fields(g, true);
        if (rc) return rc;
        const bool was_valid = g->coef_valid && g->coef_dt == b->dt[p];
        rc = prepare(g, b->dt[p]);
        if (rc) return rc;
        if (!was_valid) b->dirty = true;
    }
    if (mode == 1) {
        for (int p = 0; p < b->nprob; ++p) {
            StepOut o;
            o.energy = energy ? energy + (size_t)p * (nsteps + 1) : nullptr;
            int rc = enqueue_si_loop(b->sub[p], b->dt[p], nsteps, o);
            if (rc) return rc;
        }
        return ASD_OK;
    }
    int rc = batch_tables<T>(b);
    if (rc) return rc;
    // a captured call holds (2 + 1/ring) nsteps launches: calls longer than
    // the cap launch directly, as the single grids do
    if (b->use_graphs && b->st && nsteps >= 2 && nsteps <= kBatchGraphMaxSteps)
        return run_batch_graph<T>(b, nsteps, mode, energy);
    return enqueue_batch<T>(b, nsteps, mode, energy);
}

extern "C" int asd_batch_step_energy(asd_batch b, int32_t nsteps, int32_t mode, double* dev_energy) {
    if (!b) return asd_fail(ASD_EINVAL, "batch is NULL");
    if (nsteps < 0) return asd_fail(ASD_EINVAL, "nsteps must be >= 0");
    if (mode < -1 || mode > 2) return asd_fail(ASD_EINVAL, "mode must be -1 (tuned), 0, 1 or 2");
    if (mode == -1) mode = b->mode;
    if (nsteps == 0 && !dev_energy) return ASD_OK;
    return b->d0.dtype == ASD_F64 ? batch_step_t<double>(b, nsteps, mode, dev_energy)
                                  : batch_step_t<float>(b, nsteps, mode, dev_energy);
}

extern "C" int asd_batch_step(asd_batch b, int32_t nsteps, int32_t mode) {
    return asd_batch_step_energy(b, nsteps, mode, nullptr);
}

extern "C" int asd_batch_set_graphs(asd_batch b, int32_t on) {
    if (!b) return asd_fail(ASD_EINVAL, "batch is NULL");
    b->use_graphs = on != 0;
    return ASD_OK;
}

extern "C" int asd_batch_status(asd_batch b, uint32_t* flags, double* stats) {
    if (!b) return asd_fail(ASD_EINVAL, "batch is NULL");
    if (!flags) return asd_fail(ASD_EINVAL, "flags is NULL");
    hipError_t e = hipStreamSynchronize(b->st);
    if (e == hipSuccess) e = hipMemcpy(flags, b->d_flags, sizeof(unsigned) * (size_t)b->nprob, hipMemcpyDeviceToHost);
    if (e == hipSuccess && stats)
        e = hipMemcpy(stats, b->d_stats, 3 * sizeof(double) * (size_t)b->nprob, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return asd_fail(ASD_EHIP, "batch status: %s", hipGetErrorString(e));
    // sticky until read: clear them now they are reported
    e = launch_fill_u32(b->d_flags, 0u, b->nprob, b->st);
    if (e != hipSuccess) return asd_fail(ASD_EHIP, "flags reset: %s", hipGetErrorString(e));
    return ASD_OK;
}

// Time the persistent and grouped schedules at every admissible workgroup
// size, per-lane capacity and tile body on `probe_steps` steps each and keep
// the fastest as mode -1.  The problems' T are advanced by the probes; callers reset them
// afterwards.
extern "C" int asd_batch_tune(asd_batch b, int32_t probe_steps, int32_t* best_mode, int32_t* best_threads) {
    if (!b) return asd_fail(ASD_EINVAL, "batch is NULL");
    if (probe_steps < 1) return asd_fail(ASD_EINVAL, "probe_steps must be >= 1");
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return asd_fail(ASD_EHIP, "event create");
    float best = 1e30f;
    int bm = 0, bt = b->nthreads, bv = b->variant, bx = b->mmax;
    int rc = ASD_OK;
    for (int variant : {(int)SWEEP_FACE_SLOTS, (int)SWEEP_CELL_SLOTS})
    for (int mx : {4, 8, 16})
    for (int nt : {256, 512, 1024}) {
        if (rc) break;
        if (batch_shape(b, nt, variant, mx) != ASD_OK || b->mmax != mx) continue;
        for (int mode : {0, 2}) {
            rc = asd_batch_step(b, probe_steps, mode);  // warm-up (tables, coefficients, graph capture)
            if (rc) break;
            if (hipEventRecord(e0, b->st) != hipSuccess) { rc = asd_fail(ASD_EHIP, "event record"); break; }
            rc = asd_batch_step(b, probe_steps, mode);
            if (rc) break;
            float ms = 0.f;
            if (hipEventRecord(e1, b->st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = asd_fail(ASD_EHIP, "event timing");
                break;
            }
            if (ms < best) {
                best = ms;
                bm = mode;
                bt = nt;
                bv = variant;
                bx = mx;
            }
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    rc = batch_shape(b, bt, bv, bx);
    if (rc) return rc;
    b->mode = bm;
    if (best_mode) *best_mode = bm;
    if (best_threads) *best_threads = bt;
    return ASD_OK;
}
