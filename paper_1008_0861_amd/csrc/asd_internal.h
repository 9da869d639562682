// Host-side internals of libasd (grid handle, sweep configurations).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/asd.h"
#include "../../include/asd_extra.h"
#include "asd_device.h"
#include "asd_launch.h"

// Launch shape of one sweep: waves per line (wpl, the solve's), lines per
// workgroup, segments per line (power of two), the compiled per-lane
// capacity MMAX, io (1 or 2): staging and stores run on io times the
// solve's waves, and the tile body (face slots, or cell slots with io = 1).
struct SweepCfg {
    int wpl = 1, lpw = 1, P = 2, mmax = 1, io = 1;
    int variant = asd::SWEEP_FACE_SLOTS;
    int half = 0;  // two lines per wave (32 lanes per line; face body, batches only)
    int nthreads() const { return (half ? 32 : 64 * wpl * io) * lpw; }
};

// gfx950: 160 KiB of LDS per workgroup; keep 2 KiB for static shared data.
static constexpr size_t kLdsLimit = 160 * 1024 - 2048;

inline int pow2_floor(int v) {
    int p = 1;
    while (p * 2 <= v) p *= 2;
    return p;
}

inline int ilog2(int v) {
    int l = 0;
    while ((1 << (l + 1)) <= v) ++l;
    return l;
}

// LDS layout and bytes of a sweep launch (slot rows of the lpw lines and the
// interface-exchange buffers) for either tile body.
inline asd::TileLayout sweep_layout(int es, int ndim, int n, int lpw, int wpl, int nthreads, int mmax, int variant,
                                    int half = 0) {
    const int P = half ? 32 : std::min(64 * wpl, pow2_floor(n));
    return variant == asd::SWEEP_CELL_SLOTS ? asd::tile_layout_cell(es, ndim, n, lpw, nthreads, wpl, ilog2(P), mmax)
                                            : asd::tile_layout(es, ndim, n, lpw, nthreads, wpl, ilog2(P), mmax);
}
inline size_t sweep_lds(int es, int ndim, int n, int lpw, int wpl, int nthreads, int mmax,
                        int variant = asd::SWEEP_FACE_SLOTS, int half = 0) {
    return (size_t)sweep_layout(es, ndim, n, lpw, wpl, nthreads, mmax, variant, half).total;
}

inline int sweep_threads_cap(int es, int mmax, int variant = asd::SWEEP_FACE_SLOTS) {
    return variant == asd::SWEEP_CELL_SLOTS ? asd::sweep_cell_max_threads(es, mmax) : asd::sweep_max_threads(es, mmax);
}

// Fill *out for a line of n cells.  want_wpl / want_lpw: 0 = heuristic.
// Returns false if no configuration fits.
inline bool choose_sweep_cfg_wpl(int es, int ndim, int n, bool chi, int wpl, int want_lpw, SweepCfg* out, int io = 1,
                                 int variant = asd::SWEEP_FACE_SLOTS);

inline bool choose_sweep_cfg(int es, int ndim, int n, bool chi, int want_wpl, int want_lpw, SweepCfg* out,
                             int io = 1, int variant = asd::SWEEP_FACE_SLOTS) {
    if (want_wpl > 0) return choose_sweep_cfg_wpl(es, ndim, n, chi, want_wpl, want_lpw, out, io, variant);
    // heuristic: the fewest waves per line that keep <= pref cells per lane;
    // otherwise the feasible shape with the fewest cells per lane
    const int pref = es == 8 ? 8 : 16;
    SweepCfg best;
    bool found = false;
    for (int wpl = 1; wpl <= 16; wpl *= 2) {
        SweepCfg c;
        if (!choose_sweep_cfg_wpl(es, ndim, n, chi, wpl, want_lpw, &c, 1, variant)) continue;
        if (c.mmax <= pref) {
            *out = c;
            return true;
        }
        if (!found || c.mmax < best.mmax) {
            best = c;
            found = true;
        }
    }
    if (found) *out = best;
    return found;
}

inline bool choose_sweep_cfg_wpl(int es, int ndim, int n, bool chi, int wpl, int want_lpw, SweepCfg* out, int io,
                                 int variant) {
    if (wpl < 1 || wpl > 16 || (wpl & (wpl - 1))) return false;
    if (io != 1 && io != 2) return false;
    if (variant != asd::SWEEP_FACE_SLOTS && variant != asd::SWEEP_CELL_SLOTS) return false;
    if (variant == asd::SWEEP_CELL_SLOTS && io != 1) return false;
    const int P = std::min(64 * wpl, pow2_floor(n));
    const int m = (n + P - 1) / P;
    int mmax = 1;
    while (mmax < m) mmax *= 2;
    if (mmax > 16) return false;
    const int cap = sweep_threads_cap(es, mmax, variant);
    const int tpl = 64 * wpl * io;  // threads per line
    if (tpl > cap) return false;
    int lpw = want_lpw;
    if (lpw <= 0) lpw = std::max(1, 256 / (64 * wpl));
    while (lpw > 1 && (tpl * lpw > cap || sweep_lds(es, ndim, n, lpw, wpl, tpl * lpw, mmax, variant) > kLdsLimit))
        lpw /= 2;
    if (tpl * lpw > cap) return false;
    if (sweep_lds(es, ndim, n, lpw, wpl, tpl * lpw, mmax, variant) > kLdsLimit) return false;
    out->wpl = wpl;
    out->lpw = lpw;
    out->P = P;
    out->mmax = mmax;
    out->io = io;
    out->variant = variant;
    return true;
}

// One captured step loop, keyed on what the capture baked in.
struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    int kind = 0;  // 1 = semi-implicit, 2 = explicit
    double dt = 0.0;
    int nsteps = 0;
    double* energy = nullptr;
    double* series = nullptr;
    uint64_t last_use = 0;
};
static constexpr int kGraphCacheEntries = 4;
// ASD_GRAPHS_AUTO captures calls of at least this many steps; shorter calls
// launch directly (a graph launch starts its first kernel several
// microseconds later than a direct launch, more than the host-side launch
// cost of a short call)
static constexpr int kGraphMinSteps = 64;
static constexpr int kAuxEvents = 5;

struct asd_grid_s {
    asd_desc d{};
    hipStream_t st = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    int64_t N = 0;
    size_t es = 4;
    void* T = nullptr;
    void* b[3] = {nullptr, nullptr, nullptr};
    void* chi = nullptr;
    void* src = nullptr;       // source Q (optional), natural layout
    bool ws_inited = false;
    bool coef_valid = false;   // face coefficients computed for coef_dt
    double coef_dt = 0.0;
    void* tmp[2] = {nullptr, nullptr};
    char* coef[3][3] = {};     // [sweep][alpha, beta_t1, beta_t2], sweep's input layout
    double* ring = nullptr;    // reduction partials: ring_slots + 1 slots of max_blocks (sum, min, max)
    int ring_slots = 2;
    int64_t max_blocks = 0;
    unsigned* flags = nullptr;
    double* stats = nullptr;
    SweepCfg cfg[3];
    // graph cache of step loops: a few captured loops, least recently used
    // replaced first; graph_valid = false marks every entry stale (fields,
    // coefficients or launch shapes changed)
    int graph_mode = ASD_GRAPHS_AUTO;  // ASD_GRAPHS_OFF / _AUTO / _ALWAYS
    bool graph_valid = false;
    GraphEntry graphs[kGraphCacheEntries];
    uint64_t graph_clock = 0;
    // the adjoint's second stream (recomputation beside the reverse pass)
    // and its events; created by the first adjoint call that needs them
    hipStream_t aux = nullptr;
    hipEvent_t aux_ev[kAuxEvents] = {};
};

// whether a step call of nsteps steps replays a captured graph (only on a
// non-default stream)
inline bool graphs_for(asd_grid_s* g, int nsteps) {
    if (!g->st || nsteps < 2) return false;
    return g->graph_mode == ASD_GRAPHS_ALWAYS || (g->graph_mode == ASD_GRAPHS_AUTO && nsteps >= kGraphMinSteps);
}

// capi.cpp
int asd_fail(int code, const char* fmt, ...);
int validate_desc(const asd_desc* d);
size_t grid_workspace_bytes(const asd_desc* desc);  // desc validated
// Fill a grid handle over a workspace (desc validated; no device work).
int init_grid_in_place(asd_grid_s* g, const asd_desc* desc, void* dev_ws, size_t ws_bytes, void* stream);
int check_dt(asd_grid g, double dt, bool explicit_scheme);
// Sweep mode bits (the rhs_mode argument of fill_sweep_params / enqueue_sweep).
enum : int {
    SWEEP_SOLVE_ONLY = 1,   // right-hand side = U (no transverse term)
    SWEEP_KEEP_LAYOUT = 2,  // output in the input layout
    SWEEP_SOURCE = 4,       // dt Q joins the right-hand side (input in the natural layout)
    SWEEP_REDUCE_INPUT = 8, // the reduction (red) sums the input state instead of the output
};

template <typename T>
int fill_sweep_params(asd_grid g, int d, const void* in, void* out, int rhs_mode, const SweepCfg& c,
                      asd::SweepParams<T>* P);
int check_fields(asd_grid g, bool need_T);
int prepare(asd_grid g, double dt);  // dt > 0: face coefficients for dt
int64_t layout_stride(const asd_grid g, int L, int a);
asd::ReduceParams no_reduce();
// Per-step outputs of a step loop (each nullable): energies, FP64[nsteps+1];
// series of (energy, min T, max T), FP64[3 (nsteps+1)].
struct StepOut {
    double* energy = nullptr;
    double* series = nullptr;
    bool any() const { return energy || series; }
    const double* e0() const { return energy ? energy : series; }  // energy of the initial state
};
// Fold of count consecutive reductions into entries first .. first+count-1 of out.
asd::FoldParams make_fold(asd_grid g, const double* partials, int nblocks, int count, const StepOut& out, int first);
inline double* ring_slot(asd_grid g, int i) { return g->ring + (size_t)i * g->max_blocks * 3; }
// out2 (nullable): the output also written in the input layout (sweeps
// whose output layout is transposed).
int enqueue_sweep(asd_grid g, int d, double dt, const void* in, void* out, int rhs_mode,
                  const asd::ReduceParams& red, const SweepCfg* cfg,
                  int* nblocks_out, void* out2 = nullptr);
int enqueue_si_loop(asd_grid g, double dt, int nsteps, const StepOut& out);
int enqueue_explicit_loop(asd_grid g, double dt, int nsteps, const StepOut& out);
int enqueue_permute_2d(asd_grid g, const void* in, void* out, bool a_to_b);
int enqueue_explicit(asd_grid g, double dt, const void* src, void* dst, const asd::ReduceParams& red,
                     int* nblocks_out);
int enqueue_copy(asd_grid g, const void* src, void* dst);
int enqueue_reduce(asd_grid g, const void* x, const StepOut& out, asd::FoldParams* fold);
int enqueue_fold(asd_grid g, const asd::FoldParams& f);
// graph.cpp
int run_si_graph(asd_grid g, double dt, int nsteps, const StepOut& out);
int run_explicit_graph(asd_grid g, double dt, int nsteps, const StepOut& out);
