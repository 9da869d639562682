// asd_adjoint_step: reverse-mode derivative of nsteps 2-D semi-implicit
// steps with respect to the initial state and a per-cell chi.
//
// Forward states are checkpointed every ckpt_every steps; the reverse pass
// walks the segments backwards, recomputing each segment's states (T^n and
// T*, which the x sweep stores in both layouts) from its checkpoint, then
// runs per step, last step first:
//     mu_y = A_y^-1 lambda                       (line solves, y)
//     lambda* = mu_y + J_Sy(T*)^T mu_y; chi grads from the y faces
//     mu_x = A_x^-1 lambda*                      (line solves, x)
//     lambda  = mu_x + J_Sx(T^n)^T mu_x; chi grads from the x faces
// The line solves reuse the forward sweep kernel in solve-only mode (A_d is
// symmetric).  All buffers live in the caller's adjoint workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "asd_internal.h"

using namespace asd;

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct AdjPlan {
    int nck;         // checkpoints (states at steps 0, k, 2k, ...)
    int k;
    int nbuf;        // segment state sets: 2 when there are several segments
    size_t field;    // bytes per state
    size_t total;
};

static AdjPlan adj_plan(asd_grid g, int nsteps, int k) {
    AdjPlan p{};
    p.k = k;
    p.nck = nsteps > 0 ? (nsteps + k - 1) / k : 1;
    p.nbuf = p.nck > 1 ? 2 : 1;
    p.field = align256((size_t)g->N * g->es);
    // checkpoints + per state set (k recomputed states + k T*) + transposed
    // scratch + lambda (both layouts) + mu
    p.total = p.field * ((size_t)p.nck + (size_t)(2 * k * p.nbuf) + 4);
    return p;
}

// The second stream and the events of the overlapped reverse pass, created
// on a grid's first adjoint call with several segments (default priority,
// no implicit ordering with other streams: only the events order it).
static int adj_streams(asd_grid g) {
    if (g->aux) return ASD_OK;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
        return asd_fail(ASD_EHIP, "adjoint: stream create failed");
    for (int i = 0; i < kAuxEvents; ++i) {
        if (hipEventCreateWithFlags(&g->aux_ev[i], hipEventDisableTiming) != hipSuccess) {
            for (int j = 0; j < i; ++j) (void)hipEventDestroy(g->aux_ev[j]);
            (void)hipStreamDestroy(s);
            return asd_fail(ASD_EHIP, "adjoint: event create failed");
        }
    }
    g->aux = s;
    return ASD_OK;
}

// enqueue_* launch on g->st: this points it at another stream for a scope
struct OnStream {
    asd_grid g;
    hipStream_t saved;
    OnStream(asd_grid g_, hipStream_t s) : g(g_), saved(g_->st) { g->st = s; }
    ~OnStream() { g->st = saved; }
};

// `waiter` waits for what `signaller` has enqueued so far
static int stream_wait(hipStream_t signaller, hipStream_t waiter, hipEvent_t ev) {
    if (hipEventRecord(ev, signaller) != hipSuccess || hipStreamWaitEvent(waiter, ev, 0) != hipSuccess)
        return asd_fail(ASD_EHIP, "adjoint: stream ordering failed");
    return ASD_OK;
}

static int adj_check(asd_grid g, int nsteps, int k) {
    if (!g) return asd_fail(ASD_EINVAL, "grid is NULL");
    if (g->d.ndim != 2) return asd_fail(ASD_EUNSUPPORTED, "the adjoint is built for 2-D grids");
    if (nsteps < 0) return asd_fail(ASD_EINVAL, "nsteps must be >= 0");
    if (k < 1) return asd_fail(ASD_EINVAL, "ckpt_every must be >= 1");
    return ASD_OK;
}

extern "C" int asd_adjoint_workspace_bytes(asd_grid g, int32_t nsteps, int32_t ckpt_every, size_t* bytes) {
    int rc = adj_check(g, nsteps, ckpt_every);
    if (rc) return rc;
    if (!bytes) return asd_fail(ASD_EINVAL, "bytes is NULL");
    *bytes = adj_plan(g, nsteps, ckpt_every).total;
    return ASD_OK;
}


template <typename T>
static int stencil(asd_grid g, int d, double dt, const void* mu, const void* U, const void* X, void* lam_out,
                   bool lam_b, void* gchi) {
    AdjParams<T> P{};
    P.mu = (const T*)mu;
    P.U = (const T*)U;
    P.X = (const T*)X;
    P.b[0] = (const T*)g->b[0];
    P.b[1] = (const T*)g->b[1];
    P.chi = (g->d.flags & ASD_FLAG_PER_CELL_CHI) ? (const T*)g->chi : nullptr;
    P.lam_out = (T*)lam_out;
    P.gchi = (T*)gchi;
    P.nx = (int)g->d.n[0];
    P.ny = (int)g->d.n[1];
    P.d = d;
    P.dt = dt;
    P.hn = g->d.h[d];
    P.ht = g->d.h[1 - d];
    P.chi_par = g->d.chi_par;
    P.chi_perp = g->d.chi_perp;
    P.ka = dt / (P.hn * P.hn);
    P.kb = dt / (P.hn * P.ht);
    P.periodic = g->d.bc == ASD_BC_PERIODIC;
    P.limiter = g->d.limiter;
    P.lam_b = lam_b ? 1 : 0;
    hipError_t e = launch_adjoint_stencil<T>(P, g->st);
    if (e != hipSuccess) return asd_fail(ASD_EHIP, "adjoint stencil: %s", hipGetErrorString(e));
    return ASD_OK;
}

// The forward steps of asd_adjoint_forward: the grid's T advanced in place
// (x sweep T -> tmp0, y sweep tmp0 -> T, as in the stepping loop), with the
// states at steps 0, k, 2k, ... written to the workspace's checkpoint
// fields (the y sweep of a checkpoint step writes there directly and the
// next step reads it there).  The last step always ends in T.
static int forward_ckpt(asd_grid g, double dt, int nsteps, int k, char* ws) {
    const AdjPlan pl = adj_plan(g, nsteps, k);
    auto ck = [&](int c) { return (void*)(ws + (size_t)c * pl.field); };
    int rc = enqueue_copy(g, g->T, ck(0));
    const void* in = g->T;
    for (int s = 0; s < nsteps && rc == ASD_OK; ++s) {
        rc = enqueue_sweep(g, 0, dt, in, g->tmp[0], 0, no_reduce(), nullptr, nullptr);
        if (rc) break;
        const int c = (s + 1) / k;
        void* out = ((s + 1) % k == 0 && c < pl.nck) ? ck(c) : g->T;
        rc = enqueue_sweep(g, 1, dt, g->tmp[0], out, 0, no_reduce(), nullptr, nullptr);
        in = out;
    }
    return rc;
}

// stored: the checkpoints are already in ws (asd_adjoint_forward); T0 unused.
//
// With several segments the recomputation of segment c-1 (on the grid's
// second stream) overlaps the reverse pass over segment c (on the grid's
// stream): the two work on different state sets (c & 1), and each waits
// only for what it reads.  Event i of the grid:
//   0: fork (the reverse pass's inputs are ready) and the final join,
//   1 + s: state set s has been recomputed,  3 + s: set s has been consumed.
template <typename T>
static int adjoint_t(asd_grid g, double dt, int nsteps, int k, const void* T0, const void* lamN, void* gT0,
                     void* gchi, char* ws, bool stored) {
    const AdjPlan pl = adj_plan(g, nsteps, k);
    char* cur = ws;
    auto take = [&]() {
        char* p = cur;
        cur += pl.field;
        return (void*)p;
    };
    std::vector<void*> ck(pl.nck);
    for (int c = 0; c < pl.nck; ++c) ck[c] = take();
    std::vector<void*> S[2], TS[2];  // per set: recomputed states T^{ck k + i} (i >= 1), T* of each step
    for (int s = 0; s < pl.nbuf; ++s) {
        S[s].assign(k + 1, nullptr);
        for (int i = 1; i <= k; ++i) S[s][i] = take();
    }
    for (int s = 0; s < pl.nbuf; ++s) {
        TS[s].assign(k, nullptr);
        for (int i = 0; i < k; ++i) TS[s][i] = take();
    }
    void* tB = take();
    void* lam = take();   // lambda* (after a y sweep's reverse), layout A
    void* lamB = take();  // lambda^n (after an x sweep's reverse), layout B: the y solve's input
    void* mu = take();
    int rc = ASD_OK;
    // forward pass: checkpoints at steps 0, k, 2k, ...
    if (!stored) rc = enqueue_copy(g, T0, ck[0]);
    if (rc) return rc;
    for (int c = 1; c < pl.nck && !stored; ++c) {
        const void* in = ck[c - 1];
        for (int i = 0; i < k; ++i) {
            void* out = (i == k - 1) ? ck[c] : S[0][1];
            rc = enqueue_sweep(g, 0, dt, in, tB, 0, no_reduce(), nullptr, nullptr);
            if (rc) return rc;
            rc = enqueue_sweep(g, 1, dt, tB, out, 0, no_reduce(), nullptr, nullptr);
            if (rc) return rc;
            in = out;
        }
    }
    // reverse pass
    rc = enqueue_permute_2d(g, lamN, lamB, true);
    if (rc) return rc;
    if (gchi) {
        // a fill kernel, not a memset: callers may capture this into a graph
        hipError_t e = g->es == 8 ? launch_fill_f64((double*)gchi, 0.0, g->N, g->st)
                                  : launch_fill_u32((unsigned*)gchi, 0u, g->N, g->st);
        if (e != hipSuccess) return asd_fail(ASD_EHIP, "clear grad_chi: %s", hipGetErrorString(e));
    }
    auto seg_len = [&](int c) { return std::min(k, nsteps - c * k); };
    // segment c's states T^{ck k + i}, i = 0 .. len, in set s: the last is
    // the next checkpoint, except in the last segment
    auto state = [&](int c, int s, int i) -> void* {
        if (i == 0) return ck[c];
        if (i == seg_len(c) && c + 1 < pl.nck) return ck[c + 1];
        return S[s][i];
    };
    auto recompute = [&](int c, int s) {
        const int len = seg_len(c);
        const bool last_stored = c + 1 < pl.nck;
        for (int i = 0; i < len; ++i) {
            // T* in the y sweep's layout (tB) and, second store, in the
            // natural layout the stencils read (TS)
            int r = enqueue_sweep(g, 0, dt, state(c, s, i), tB, 0, no_reduce(), nullptr, nullptr, TS[s][i]);
            if (r) return r;
            if (i + 1 == len && last_stored) break;  // that y sweep's output is stored
            r = enqueue_sweep(g, 1, dt, tB, state(c, s, i + 1), 0, no_reduce(), nullptr, nullptr);
            if (r) return r;
        }
        return ASD_OK;
    };
    auto reverse = [&](int c, int s) {
        for (int i = seg_len(c) - 1; i >= 0; --i) {
            // y sweep: T* -> T^{n+1}; lambda arrives in the y solve's layout
            int r = enqueue_sweep(g, 1, dt, lamB, mu, 1, no_reduce(), nullptr, nullptr);
            if (r) return r;
            r = stencil<T>(g, 1, dt, mu, TS[s][i], state(c, s, i + 1), lam, false, gchi);
            if (r) return r;
            // x sweep: T^n -> T*; the solve writes mu in the natural layout
            // directly (line-contiguous store, no transpose), the stencil
            // writes lambda^n in the layout of the next y solve
            r = enqueue_sweep(g, 0, dt, lam, mu, SWEEP_SOLVE_ONLY | SWEEP_KEEP_LAYOUT, no_reduce(), nullptr, nullptr);
            if (r) return r;
            r = stencil<T>(g, 0, dt, mu, state(c, s, i), TS[s][i], lamB, true, gchi);
            if (r) return r;
        }
        return ASD_OK;
    };
    const int last = pl.nck - 1;
    if (pl.nbuf == 1) {
        rc = recompute(0, 0);
        if (rc == ASD_OK) rc = reverse(0, 0);
    } else {
        rc = adj_streams(g);
        if (rc) return rc;
        hipStream_t mst = g->st, aux = g->aux;
        rc = stream_wait(mst, aux, g->aux_ev[0]);
        auto recompute_aux = [&](int c) {
            OnStream on(g, aux);
            int r = recompute(c, c & 1);
            if (r == ASD_OK && hipEventRecord(g->aux_ev[1 + (c & 1)], aux) != hipSuccess)
                r = asd_fail(ASD_EHIP, "adjoint: event record failed");
            return r;
        };
        if (rc == ASD_OK) rc = recompute_aux(last);
        for (int c = last; c >= 0 && rc == ASD_OK; --c) {
            if (c >= 1) {
                // set (c - 1) & 1 was last read by the reverse pass over c + 1
                if (c + 1 <= last && hipStreamWaitEvent(aux, g->aux_ev[3 + ((c + 1) & 1)], 0) != hipSuccess)
                    rc = asd_fail(ASD_EHIP, "adjoint: stream wait failed");
                if (rc == ASD_OK) rc = recompute_aux(c - 1);
            }
            if (rc == ASD_OK && hipStreamWaitEvent(mst, g->aux_ev[1 + (c & 1)], 0) != hipSuccess)
                rc = asd_fail(ASD_EHIP, "adjoint: stream wait failed");
            if (rc == ASD_OK) rc = reverse(c, c & 1);
            if (rc == ASD_OK && hipEventRecord(g->aux_ev[3 + (c & 1)], mst) != hipSuccess)
                rc = asd_fail(ASD_EHIP, "adjoint: event record failed");
        }
        // join: nothing of this call stays pending on the second stream,
        // also when an enqueue above failed
        const int rj = stream_wait(aux, mst, g->aux_ev[0]);
        if (rc == ASD_OK) rc = rj;
    }
    if (rc) return rc;
    return enqueue_permute_2d(g, lamB, gT0, false);
}

// Checks shared by the three adjoint entry points; on success the grid's
// coefficients are prepared for dt.
static int adj_validate(asd_grid g, double dt, int nsteps, int k, bool grad_chi, const void* ws, size_t ws_bytes) {
    int rc = adj_check(g, nsteps, k);
    if (rc) return rc;
    if (!(std::isfinite(dt) && dt > 0.0)) return asd_fail(ASD_EINVAL, "dt must be finite and > 0");
    if (grad_chi && !(g->d.flags & ASD_FLAG_PER_CELL_CHI))
        return asd_fail(ASD_EINVAL, "grad_chi needs ASD_FLAG_PER_CELL_CHI");
    if (g->d.flags & (ASD_FLAG_FOUR_STEP | ASD_FLAG_REVERSE_ORDER))
        return asd_fail(ASD_EUNSUPPORTED, "the adjoint is of the 2-step scheme in the order x, y");
    if (g->d.chi_exp != 0.0) return asd_fail(ASD_EUNSUPPORTED, "the adjoint takes a chi that does not depend on T");
    if (g->d.bc == ASD_BC_DIRICHLET || g->src)
        return asd_fail(ASD_EUNSUPPORTED, "the adjoint is for periodic or insulating grids without a source");
    if (!ws) return asd_fail(ASD_EWORKSPACE, "adjoint workspace is NULL");
    if ((uintptr_t)ws & 255) return asd_fail(ASD_EWORKSPACE, "adjoint workspace must be 256-byte aligned");
    const AdjPlan pl = adj_plan(g, nsteps, k);
    if (ws_bytes < pl.total)
        return asd_fail(ASD_EWORKSPACE, "adjoint workspace too small: %zu < %zu bytes", ws_bytes, pl.total);
    rc = check_fields(g, false);
    if (rc) return rc;
    return prepare(g, dt);
}

extern "C" int asd_adjoint_step(asd_grid g, double dt, int32_t nsteps, int32_t ckpt_every, const void* dev_T0,
                                const void* dev_lambda_final, void* dev_grad_T0, void* dev_grad_chi, void* dev_adj_ws,
                                size_t adj_ws_bytes) {
    if (g && (!dev_T0 || !dev_lambda_final || !dev_grad_T0)) return asd_fail(ASD_EINVAL, "NULL state pointer");
    int rc = adj_validate(g, dt, nsteps, ckpt_every, dev_grad_chi != nullptr, dev_adj_ws, adj_ws_bytes);
    if (rc) return rc;
    return g->es == 8 ? adjoint_t<double>(g, dt, nsteps, ckpt_every, dev_T0, dev_lambda_final, dev_grad_T0,
                                          dev_grad_chi, (char*)dev_adj_ws, false)
                      : adjoint_t<float>(g, dt, nsteps, ckpt_every, dev_T0, dev_lambda_final, dev_grad_T0,
                                         dev_grad_chi, (char*)dev_adj_ws, false);
}

extern "C" int asd_adjoint_forward(asd_grid g, double dt, int32_t nsteps, int32_t ckpt_every, void* dev_adj_ws,
                                   size_t adj_ws_bytes) {
    int rc = adj_validate(g, dt, nsteps, ckpt_every, false, dev_adj_ws, adj_ws_bytes);
    if (rc) return rc;
    return forward_ckpt(g, dt, nsteps, ckpt_every, (char*)dev_adj_ws);
}

extern "C" int asd_adjoint_step_stored(asd_grid g, double dt, int32_t nsteps, int32_t ckpt_every,
                                       const void* dev_lambda_final, void* dev_grad_T0, void* dev_grad_chi,
                                       void* dev_adj_ws, size_t adj_ws_bytes) {
    if (g && (!dev_lambda_final || !dev_grad_T0)) return asd_fail(ASD_EINVAL, "NULL state pointer");
    int rc = adj_validate(g, dt, nsteps, ckpt_every, dev_grad_chi != nullptr, dev_adj_ws, adj_ws_bytes);
    if (rc) return rc;
    return g->es == 8 ? adjoint_t<double>(g, dt, nsteps, ckpt_every, nullptr, dev_lambda_final, dev_grad_T0,
                                          dev_grad_chi, (char*)dev_adj_ws, true)
                      : adjoint_t<float>(g, dt, nsteps, ckpt_every, nullptr, dev_lambda_final, dev_grad_T0,
                                         dev_grad_chi, (char*)dev_adj_ws, true);
}
