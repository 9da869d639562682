// Host-side internals of libasd (grid handle, sweep configurations).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/asd.h"
#include "asd_device.h"
#include "asd_launch.h"

// Launch shape of one sweep: waves per line, lines per workgroup, segments
// per line (power of two), and the compiled per-lane capacity MMAX.
struct SweepCfg {
    int wpl = 1, lpw = 1, P = 2, mmax = 1;
    int nthreads() const { return 64 * wpl * lpw; }
};

// gfx950: 160 KiB of LDS per workgroup; keep 2 KiB for static shared data.
static constexpr size_t kLdsLimit = 160 * 1024 - 2048;

inline int pow2_floor(int v) {
    int p = 1;
    while (p * 2 <= v) p *= 2;
    return p;
}

inline size_t sweep_lds(int es, int ndim, int n, int lpw, int nthreads, bool chi) {
    const int LS = es == 8 ? asd::lds_line_stride<double>(n) : asd::lds_line_stride<float>(n);
    const int narr = (ndim == 2 ? 4 : 6) + (chi ? 1 : 0);
    return (size_t)es * ((size_t)narr * lpw * LS + 4 * (size_t)nthreads);
}

inline int sweep_threads_cap(int es, int mmax) {
    const int bytes = es * mmax;
    return bytes >= 64 ? 256 : (bytes >= 32 ? 512 : 1024);
}

// Fill *out for a line of n cells.  want_wpl / want_lpw: 0 = heuristic.
// Returns false if no configuration fits.
inline bool choose_sweep_cfg(int es, int ndim, int n, bool chi, int want_wpl, int want_lpw, SweepCfg* out) {
    const int pref = es == 8 ? 8 : 16;
    int wpl = want_wpl;
    if (wpl <= 0) {
        wpl = 1;
        while (wpl < 16) {
            const int P = std::min(64 * wpl, pow2_floor(n));
            if ((n + P - 1) / P <= pref) break;
            wpl *= 2;
        }
    }
    if (wpl < 1 || wpl > 16 || (wpl & (wpl - 1))) return false;
    const int P = std::min(64 * wpl, pow2_floor(n));
    const int m = (n + P - 1) / P;
    int mmax = 1;
    while (mmax < m) mmax *= 2;
    if (mmax > 16) return false;
    const int cap = sweep_threads_cap(es, mmax);
    if (64 * wpl > cap) return false;
    int lpw = want_lpw;
    if (lpw <= 0) lpw = std::max(1, 256 / (64 * wpl));
    while (lpw > 1 && (64 * wpl * lpw > cap || sweep_lds(es, ndim, n, lpw, 64 * wpl * lpw, chi) > kLdsLimit))
        lpw /= 2;
    if (64 * wpl * lpw > cap) return false;
    if (sweep_lds(es, ndim, n, lpw, 64 * wpl * lpw, chi) > kLdsLimit) return false;
    out->wpl = wpl;
    out->lpw = lpw;
    out->P = P;
    out->mmax = mmax;
    return true;
}

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
    bool layouts_dirty = true;
    bool ws_inited = false;
    void* tmp[2] = {nullptr, nullptr};
    char* bl[3][3] = {};
    char* chil[3] = {};
    double* partials = nullptr;
    int64_t max_blocks = 0;
    unsigned* ticket = nullptr;
    unsigned* flags = nullptr;
    double* stats = nullptr;
    double* e0 = nullptr;
    SweepCfg cfg[3];
    // graph cache of the step loop
    bool use_graphs = true;
    bool graph_valid = false;
    hipGraphExec_t graph_exec = nullptr;
    int graph_kind = 0;  // 1 = semi-implicit, 2 = explicit
    double graph_dt = 0.0;
    int graph_nsteps = 0;
    double* graph_energy = nullptr;
};

// capi.cpp
int asd_fail(int code, const char* fmt, ...);
int check_fields(asd_grid g, bool need_T);
int prepare(asd_grid g);
int64_t layout_stride(const asd_grid g, int L, int a);
asd::ReduceParams no_reduce();
asd::ReduceParams make_reduce(asd_grid g, double* energy_out, const double* e0);
int enqueue_sweep(asd_grid g, int d, double dt, const void* in, void* out, int rhs_mode,
                  const asd::ReduceParams& red, const SweepCfg* cfg);
int enqueue_si_step(asd_grid g, double dt, const void* src, void* dst, const asd::ReduceParams& red);
int enqueue_explicit(asd_grid g, double dt, const void* src, void* dst, const asd::ReduceParams& red);
int enqueue_copy(asd_grid g, const void* src, void* dst);
int enqueue_reduce(asd_grid g, const void* x, double* energy_out, const double* e0);
// graph.cpp
int run_si_graph(asd_grid g, double dt, int nsteps, double* energy);
int run_explicit_graph(asd_grid g, double dt, int nsteps, double* energy);
