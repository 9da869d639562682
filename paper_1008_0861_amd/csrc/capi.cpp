// C ABI of libasd: argument validation, workspace carve-up, data layouts
// and the step drivers that enqueue the gfx950 kernels.
//
// Layouts.  The user's arrays are x-fastest ("A").  Each sweep reads its
// input with the sweep axis contiguous and writes its output transposed so
// that the next sweep's axis is contiguous again:
//   2-D:  x-sweep  A=[y][x] -> B=[x][y];  y-sweep B -> A
//   3-D:  x-sweep  A=[z][y][x] -> B=[z][x][y];  y-sweep B -> C=[y][x][z];
//         z-sweep  C -> A
// The face coefficients of each sweep (alpha, beta_t) depend only on dt, b
// and chi: they are computed once per dt in that sweep's input layout, in
// the caller's workspace, and the sweeps read them instead of b.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "../../include/asd.h"
#include "../../include/asd_extra.h"
#include "asd_launch.h"
#include "asd_internal.h"

using namespace asd;

static thread_local std::string g_err;

int asd_fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

static int hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return ASD_OK;
    return asd_fail(ASD_EHIP, "%s: %s", what, hipGetErrorString(e));
}

extern "C" const char* asd_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------------ description

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int validate_desc(const asd_desc* d) {
    if (!d) return asd_fail(ASD_EINVAL, "desc is NULL");
    if (d->ndim != 2 && d->ndim != 3) return asd_fail(ASD_EINVAL, "ndim must be 2 or 3 (got %d)", d->ndim);
    if (d->bc != ASD_BC_PERIODIC && d->bc != ASD_BC_INSULATING && d->bc != ASD_BC_DIRICHLET)
        return asd_fail(ASD_EINVAL, "bad boundary condition %d", d->bc);
    if (d->dtype != ASD_F32 && d->dtype != ASD_F64) return asd_fail(ASD_EINVAL, "bad dtype %d", d->dtype);
    if (d->limiter < ASD_LIM_VANLEER || d->limiter > ASD_LIM_LINEAR)
        return asd_fail(ASD_EINVAL, "bad limiter %d", d->limiter);
    if (d->reserved != 0) return asd_fail(ASD_EINVAL, "reserved must be 0");
    if (d->flags & ~(ASD_FLAG_PER_CELL_CHI | ASD_FLAG_ALLOW_UNSTABLE | ASD_FLAG_FOUR_STEP | ASD_FLAG_REVERSE_ORDER))
        return asd_fail(ASD_EINVAL, "unknown flags 0x%x", d->flags);
    const int64_t nmin = d->bc == ASD_BC_PERIODIC ? 3 : 2;
    for (int q = 0; q < d->ndim; ++q) {
        if (d->n[q] < nmin)
            return asd_fail(ASD_ESHAPE, "n[%d] = %lld, need >= %lld for this boundary", q,
                            (long long)d->n[q], (long long)nmin);
        if (d->n[q] > (1 << 20)) return asd_fail(ASD_EUNSUPPORTED, "n[%d] too large", q);
        if (!finite_pos(d->h[q])) return asd_fail(ASD_EINVAL, "h[%d] must be finite and > 0", q);
    }
    if (d->ndim == 2 && d->n[2] != 1) return asd_fail(ASD_ESHAPE, "n[2] must be 1 in 2-D");
    if (d->ndim == 3 && (d->flags & ASD_FLAG_REVERSE_ORDER))
        return asd_fail(ASD_EUNSUPPORTED, "the reverse sweep order is for 2-D grids");
    if (!finite_pos(d->chi_par)) return asd_fail(ASD_EINVAL, "chi_par must be finite and > 0");
    if (!std::isfinite(d->chi_perp) || d->chi_perp < 0.0 || d->chi_perp > d->chi_par)
        return asd_fail(ASD_EINVAL, "chi_perp must be in [0, chi_par]");
    if (d->chi_exp != 0.0) {
        if (!std::isfinite(d->chi_exp) || d->chi_exp < 0.0 || d->chi_exp > 8.0)
            return asd_fail(ASD_EINVAL, "chi_exp must be in (0, 8]");
        if (!finite_pos(d->chi_tref)) return asd_fail(ASD_EINVAL, "chi_tref must be finite and > 0");
        if (d->flags & ASD_FLAG_PER_CELL_CHI)
            return asd_fail(ASD_EINVAL, "chi_exp and ASD_FLAG_PER_CELL_CHI exclude each other");
    }
    const int64_t N = d->n[0] * d->n[1] * (d->ndim == 3 ? d->n[2] : 1);
    if (N > (int64_t)INT32_MAX) return asd_fail(ASD_EUNSUPPORTED, "grid too large (more than 2^31-1 cells)");
    for (int q = 0; q < d->ndim; ++q) {
        SweepCfg c;
        if (!choose_sweep_cfg(d->dtype == ASD_F64 ? 8 : 4, d->ndim, (int)d->n[q],
                              (d->flags & ASD_FLAG_PER_CELL_CHI) != 0, 0, 0, &c))
            return asd_fail(ASD_EUNSUPPORTED, "lines of %lld cells along axis %d do not fit in LDS",
                            (long long)d->n[q], q);
    }
    return ASD_OK;
}

static int64_t cells(const asd_desc* d) { return d->n[0] * d->n[1] * (d->ndim == 3 ? d->n[2] : 1); }

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Workspace plan: offsets of each region.
struct WsPlan {
    size_t tmp[2], coef[3][3], partials, small, total;
    int64_t max_blocks;
    int ring_slots;
};

// Reduction partials: a ring of slots, one per step whose energy is still
// to be folded (folded together every ring_slots steps), plus one slot for
// standalone reductions.  The ring holds up to 32 slots within 4 MiB.
static int ring_slots_for(int64_t max_blocks) {
    const size_t slot = (size_t)max_blocks * 3 * sizeof(double);
    const size_t k = ((size_t)4 << 20) / slot;
    return (int)std::max<size_t>(2, std::min<size_t>(32, k));
}

static int64_t max_reduce_blocks(const asd_desc* d) {
    // sweeps at their smallest (one line per block), explicit tiles, reductions
    int64_t N = cells(d), mb = 1024;
    for (int q = 0; q < d->ndim; ++q) mb = std::max<int64_t>(mb, N / d->n[q]);
    int n[3] = {(int)d->n[0], (int)d->n[1], d->ndim == 3 ? (int)d->n[2] : 1};
    mb = std::max<int64_t>(mb, explicit_num_blocks(d->ndim, n));
    return mb;
}

static WsPlan plan_ws(const asd_desc* d) {
    WsPlan p{};
    const size_t es = d->dtype == ASD_F64 ? 8 : 4;
    const size_t fb = align256((size_t)cells(d) * es);
    size_t off = 0;
    const int ntmp = 2;  // sweep intermediates / explicit ping-pong / benchmark outputs
    for (int i = 0; i < 2; ++i) p.tmp[i] = (size_t)-1;
    for (int i = 0; i < ntmp; ++i) { p.tmp[i] = off; off += fb; }
    // face coefficients: per sweep direction alpha and one beta per transverse axis
    for (int dd = 0; dd < 3; ++dd)
        for (int q = 0; q < 3; ++q) p.coef[dd][q] = (size_t)-1;
    for (int dd = 0; dd < d->ndim; ++dd)
        for (int q = 0; q < d->ndim; ++q) { p.coef[dd][q] = off; off += fb; }
    p.max_blocks = max_reduce_blocks(d);
    p.ring_slots = ring_slots_for(p.max_blocks);
    p.partials = off;
    off += align256((size_t)(p.ring_slots + 1) * p.max_blocks * 3 * sizeof(double));
    p.small = off;
    off += 256;
    p.total = off;
    return p;
}

extern "C" int asd_workspace_bytes(const asd_desc* desc, size_t* bytes) {
    int rc = validate_desc(desc);
    if (rc) return rc;
    if (!bytes) return asd_fail(ASD_EINVAL, "bytes is NULL");
    *bytes = plan_ws(desc).total;
    return ASD_OK;
}

// ------------------------------------------------------------------ grid

size_t grid_workspace_bytes(const asd_desc* desc) { return plan_ws(desc).total; }

int init_grid_in_place(asd_grid_s* g, const asd_desc* desc, void* dev_ws, size_t ws_bytes, void* stream) {
    WsPlan p = plan_ws(desc);
    if (!dev_ws) return asd_fail(ASD_EWORKSPACE, "workspace is NULL");
    if ((uintptr_t)dev_ws & 255) return asd_fail(ASD_EWORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < p.total)
        return asd_fail(ASD_EWORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, p.total);
    g->d = *desc;
    g->st = (hipStream_t)stream;
    g->ws = (char*)dev_ws;
    g->ws_bytes = ws_bytes;
    g->N = cells(desc);
    g->es = desc->dtype == ASD_F64 ? 8 : 4;
    for (int i = 0; i < 2; ++i) g->tmp[i] = p.tmp[i] == (size_t)-1 ? nullptr : g->ws + p.tmp[i];
    for (int dd = 0; dd < 3; ++dd)
        for (int q = 0; q < 3; ++q) g->coef[dd][q] = p.coef[dd][q] == (size_t)-1 ? nullptr : g->ws + p.coef[dd][q];
    g->ring = (double*)(g->ws + p.partials);
    g->ring_slots = p.ring_slots;
    g->max_blocks = p.max_blocks;
    char* sm = g->ws + p.small;
    g->flags = (unsigned*)sm;
    g->stats = (double*)(sm + 8);   // 3 doubles
    for (int q = 0; q < desc->ndim; ++q) {
        if (!choose_sweep_cfg((int)g->es, desc->ndim, (int)desc->n[q],
                              (desc->flags & ASD_FLAG_PER_CELL_CHI) != 0, 0, 0, &g->cfg[q]))
            return asd_fail(ASD_EUNSUPPORTED, "no sweep configuration for axis %d", q);
    }
    return ASD_OK;
}

extern "C" int asd_init_grid(const asd_desc* desc, void* dev_ws, size_t ws_bytes, void* stream,
                             asd_grid* out) {
    int rc = validate_desc(desc);
    if (rc) return rc;
    if (!out) return asd_fail(ASD_EINVAL, "out is NULL");
    asd_grid_s* g = new (std::nothrow) asd_grid_s();
    if (!g) return asd_fail(ASD_EINVAL, "out of host memory");
    rc = init_grid_in_place(g, desc, dev_ws, ws_bytes, stream);
    if (rc) {
        delete g;
        return rc;
    }
    *out = g;
    return ASD_OK;
}

extern "C" int asd_destroy(asd_grid g) {
    if (!g) return asd_fail(ASD_EINVAL, "grid is NULL");
    for (GraphEntry& e : g->graphs)
        if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (g->aux) {
        (void)hipStreamSynchronize(g->aux);
        for (hipEvent_t& e : g->aux_ev) (void)hipEventDestroy(e);
        (void)hipStreamDestroy(g->aux);
    }
    delete g;
    return ASD_OK;
}

extern "C" int asd_set_field(asd_grid g, int32_t field, void* dev_ptr, int64_t nelem, int32_t dtype) {
    if (!g) return asd_fail(ASD_EINVAL, "grid is NULL");
    if (!dev_ptr) return asd_fail(ASD_EINVAL, "field pointer is NULL");
    if (dtype != g->d.dtype) return asd_fail(ASD_EDTYPE, "dtype %d does not match the grid (%d)", dtype, g->d.dtype);
    if (nelem != g->N)
        return asd_fail(ASD_ESHAPE, "nelem %lld does not match the grid (%lld cells)", (long long)nelem,
                        (long long)g->N);
    switch (field) {
        case ASD_FIELD_T: g->T = dev_ptr; break;
        case ASD_FIELD_BX: g->b[0] = dev_ptr; g->coef_valid = false; break;
        case ASD_FIELD_BY: g->b[1] = dev_ptr; g->coef_valid = false; break;
        case ASD_FIELD_BZ:
            if (g->d.ndim != 3) return asd_fail(ASD_EINVAL, "BZ set on a 2-D grid");
            g->b[2] = dev_ptr;
            g->coef_valid = false;
            break;
        case ASD_FIELD_CHI:
            if (!(g->d.flags & ASD_FLAG_PER_CELL_CHI))
                return asd_fail(ASD_EINVAL, "CHI set without ASD_FLAG_PER_CELL_CHI");
            g->chi = dev_ptr;
            g->coef_valid = false;
            break;
        case ASD_FIELD_Q: g->src = dev_ptr; break;
        default: return asd_fail(ASD_EINVAL, "unknown field %d", field);
    }
    g->graph_valid = false;
    return ASD_OK;
}

int check_fields(asd_grid g, bool need_T) {
    if (need_T && !g->T) return asd_fail(ASD_ENOTSET, "field T is not set");
    for (int q = 0; q < g->d.ndim; ++q)
        if (!g->b[q]) return asd_fail(ASD_ENOTSET, "field b%c is not set", "xyz"[q]);
    if ((g->d.flags & ASD_FLAG_PER_CELL_CHI) && !g->chi) return asd_fail(ASD_ENOTSET, "field CHI is not set");
    return ASD_OK;
}

// ------------------------------------------------------------- layouts

// stride of axis a (0=x,1=y,2=z) in layout L
int64_t layout_stride(const asd_grid g, int L, int a) {
    const int64_t nx = g->d.n[0], ny = g->d.n[1], nz = g->d.ndim == 3 ? g->d.n[2] : 1;
    if (L == 0) { const int64_t s[3] = {1, nx, nx * ny}; return s[a]; }
    if (L == 1) { const int64_t s[3] = {ny, 1, nx * ny}; return s[a]; }  // [z][x][y]
    const int64_t s[3] = {nz, nx * nz, 1};                               // [y][x][z]
    return s[a];
}

// the three sweeps: axis, input layout, output layout, t1 (fastest of out), t2
struct SweepGeom { int d, Lin, Lout, t1, t2; };
static SweepGeom sweep_geom(int ndim, int d) {
    if (ndim == 2) {
        if (d == 0) return {0, 0, 1, 1, 2};
        return {1, 1, 0, 0, 2};
    }
    if (d == 0) return {0, 0, 1, 1, 2};
    if (d == 1) return {1, 1, 2, 2, 0};
    return {2, 2, 0, 0, 1};
}

static std::once_flag g_attr_once;
static hipError_t g_attr_err = hipSuccess;

// Face coefficients of sweep d for step dt into g->coef[d], in the sweep's
// input layout.  U: chi(T) from this state (same layout), or nullptr for a
// constant or per-cell chi.
template <typename T>
static int enqueue_coef_t(asd_grid g, int d, double dt, const void* U) {
    const int nd = g->d.ndim;
    const SweepGeom G = sweep_geom(nd, d);
    CoefParams<T> C{};
    for (int q = 0; q < 3; ++q) C.b[q] = q < nd ? (const T*)g->b[q] : nullptr;
    C.chi = (g->d.flags & ASD_FLAG_PER_CELL_CHI) ? (const T*)g->chi : nullptr;
    C.U = (const T*)U;
    C.chi_exp = g->d.chi_exp;
    C.chi_tref = g->d.chi_tref;
    C.alpha = (T*)g->coef[d][0];
    C.beta1 = (T*)g->coef[d][1];
    C.beta2 = nd == 3 ? (T*)g->coef[d][2] : nullptr;
    C.n[0] = (int)g->d.n[0];
    C.n[1] = (int)g->d.n[1];
    C.n[2] = nd == 3 ? (int)g->d.n[2] : 1;
    C.d = G.d;
    C.t1 = G.t1;
    C.t2 = G.t2;
    for (int a = 0; a < 3; ++a) C.so[a] = (int)layout_stride(g, G.Lin, a);
    const double hd = g->d.h[G.d];
    const double h1 = g->d.h[G.t1];
    const double h2 = nd == 3 ? g->d.h[G.t2] : 1.0;
    // the 4-step scheme solves its normal operator at dt/2 (Eq. 4step)
    const double dt_n = (g->d.flags & ASD_FLAG_FOUR_STEP) ? 0.5 * dt : dt;
    C.cnn = dt_n / (hd * hd);
    C.ct1 = dt / (hd * h1);
    C.ct2 = dt / (hd * h2);
    C.chi_par = g->d.chi_par;
    C.chi_perp = g->d.chi_perp;
    C.periodic = g->d.bc == ASD_BC_PERIODIC;
    C.dirichlet = g->d.bc == ASD_BC_DIRICHLET;
    C.ndim = nd;
    return hip_check(launch_coef<T>(C, g->st), "coefficient launch");
}

static int enqueue_coef(asd_grid g, int d, double dt, const void* U) {
    return g->es == 8 ? enqueue_coef_t<double>(g, d, dt, U) : enqueue_coef_t<float>(g, d, dt, U);
}

template <typename T>
static int do_prepare(asd_grid g, double dt) {
    std::call_once(g_attr_once, [] {
        g_attr_err = sweep_set_lds_limits((int)kLdsLimit);
        if (g_attr_err == hipSuccess) g_attr_err = batch_set_lds_limits((int)kLdsLimit);
    });
    if (g_attr_err != hipSuccess) return hip_check(g_attr_err, "kernel attributes");
    if (!g->ws_inited) {
        int rc = hip_check(launch_fill_u32(g->flags, 0u, 1, g->st), "fill");
        if (rc) return rc;
        g->ws_inited = true;
    }
    if (dt > 0.0 && !(g->coef_valid && g->coef_dt == dt)) {
        for (int d = 0; d < g->d.ndim; ++d) {
            int rc = enqueue_coef_t<T>(g, d, dt, nullptr);
            if (rc) return rc;
        }
        g->coef_valid = true;
        g->coef_dt = dt;
        g->graph_valid = false;
    }
    return ASD_OK;
}

int prepare(asd_grid g, double dt) { return g->es == 8 ? do_prepare<double>(g, dt) : do_prepare<float>(g, dt); }

// --------------------------------------------------------------- sweeps

ReduceParams no_reduce() {
    ReduceParams r{};
    return r;
}

FoldParams make_fold(asd_grid g, const double* partials, int nblocks, int count, const StepOut& out, int first) {
    FoldParams f{};
    f.partials = partials;
    f.nblocks = nblocks;
    f.count = count;
    f.slot_stride = (int)(g->max_blocks * 3);
    f.energy_out = out.energy ? out.energy + first : nullptr;
    f.series_out = out.series ? out.series + 3 * first : nullptr;
    f.stats_out = g->stats;
    f.flags = g->flags;
    // the energy is conserved only without T = 0 walls and sources; a fold
    // that starts at entry 0 checks against its own reduction 0
    const bool conserved = g->d.bc != ASD_BC_DIRICHLET && !g->src;
    f.e0 = first > 0 && conserved ? out.e0() : nullptr;
    f.e0_slot0 = first == 0 && conserved;
    double dv = 1.0;
    for (int q = 0; q < g->d.ndim; ++q) dv *= g->d.h[q];
    f.dV = dv;
    return f;
}

// Parameters of sweep d of grid g from `in` to `out` with launch shape c.
template <typename T>
int fill_sweep_params(asd_grid g, int d, const void* in, void* out, int rhs_mode, const SweepCfg& c,
                      SweepParams<T>* Pout) {
    const SweepGeom G = sweep_geom(g->d.ndim, d);
    SweepParams<T> P{};
    P.U = (const T*)in;
    P.out = (T*)out;
    P.alpha = (const T*)g->coef[d][0];
    P.beta1 = (const T*)g->coef[d][1];
    P.beta2 = g->d.ndim == 3 ? (const T*)g->coef[d][2] : nullptr;
    const int64_t nz = g->d.ndim == 3 ? g->d.n[2] : 1;
    const int64_t nax[3] = {g->d.n[0], g->d.n[1], nz};
    P.n = (int)nax[G.d];
    P.nt1 = (int)nax[G.t1];
    P.nt2 = (int)nax[G.t2];
    P.si_n = (int)layout_stride(g, G.Lin, G.d);
    P.si_t1 = (int)layout_stride(g, G.Lin, G.t1);
    P.si_t2 = (int)layout_stride(g, G.Lin, G.t2);
    // SWEEP_KEEP_LAYOUT: the output keeps the input layout (line-contiguous
    // stores) instead of the sweep's transposed output layout
    const int Lout = (rhs_mode & SWEEP_KEEP_LAYOUT) ? G.Lin : G.Lout;
    P.so_n = (int)layout_stride(g, Lout, G.d);
    P.so_t1 = (int)layout_stride(g, Lout, G.t1);
    P.so_t2 = (int)layout_stride(g, Lout, G.t2);
    P.periodic = g->d.bc == ASD_BC_PERIODIC;
    P.dirichlet = g->d.bc == ASD_BC_DIRICHLET;
    P.limiter = g->d.limiter;
    P.wpl = c.wpl;
    P.lpw = c.lpw;
    P.P = c.P;
    P.nseg_log2 = ilog2(c.P);
    P.spl_log2 = c.half ? 5 : ilog2(64 * c.wpl);
    P.io_log2 = ilog2(c.io);
    P.lpw_log2 = ilog2(c.lpw);
    P.rhs_mode = rhs_mode & SWEEP_SOLVE_ONLY;
    P.lds = sweep_layout((int)sizeof(T), g->d.ndim, P.n, c.lpw, c.wpl, c.nthreads(), c.mmax, c.variant, c.half);
    if (P.si_n != 1) return asd_fail(ASD_EUNSUPPORTED, "sweep input must be contiguous along the line");
    *Pout = P;
    return ASD_OK;
}
template int fill_sweep_params<float>(asd_grid, int, const void*, void*, int, const SweepCfg&, SweepParams<float>*);
template int fill_sweep_params<double>(asd_grid, int, const void*, void*, int, const SweepCfg&, SweepParams<double>*);

template <typename T>
static int enqueue_sweep_t(asd_grid g, int d, double dt, const void* in, void* out, int rhs_mode,
                           const ReduceParams& red, const SweepCfg* override_cfg, int* nblocks_out, void* out2) {
    // the coefficients were computed for dt by prepare() (or enqueue_coef)
    const SweepCfg& c = override_cfg ? *override_cfg : g->cfg[d];
    SweepParams<T> P;
    int rc = fill_sweep_params<T>(g, d, in, out, rhs_mode, c, &P);
    if (rc) return rc;
    if (out2) {
        if (P.so_t1 != 1) return asd_fail(ASD_EUNSUPPORTED, "a second output needs a transposed-output sweep");
        P.out2 = (T*)out2;
    }
    if ((rhs_mode & SWEEP_SOURCE) && g->src) {
        if (sweep_geom(g->d.ndim, d).Lin != 0)
            return asd_fail(ASD_EUNSUPPORTED, "the source enters a sweep that reads the natural layout");
        P.Q = (const T*)g->src;
        P.dtq = (T)dt;
    }
    P.red = red;
    P.red_in = (rhs_mode & SWEEP_REDUCE_INPUT) != 0;
    const int nb1 = (P.nt1 + c.lpw - 1) / c.lpw;
    const int64_t nblocks = (int64_t)nb1 * P.nt2;
    if (nblocks_out) *nblocks_out = (int)nblocks;
    if (red.partials && nblocks > g->max_blocks)
        return asd_fail(ASD_EUNSUPPORTED, "too many blocks for the reduction scratch");
    const size_t lds = sweep_lds((int)sizeof(T), g->d.ndim, P.n, c.lpw, c.wpl, c.nthreads(), c.mmax, c.variant, c.half);
    return hip_check(launch_sweep<T>(P, g->d.ndim, c.mmax, dim3((unsigned)nblocks), dim3(c.nthreads()), lds, g->st,
                                     c.variant),
                     "sweep launch");
}

int enqueue_sweep(asd_grid g, int d, double dt, const void* in, void* out, int rhs_mode, const ReduceParams& red,
                  const SweepCfg* cfg, int* nblocks_out, void* out2) {
    return g->es == 8 ? enqueue_sweep_t<double>(g, d, dt, in, out, rhs_mode, red, cfg, nblocks_out, out2)
                      : enqueue_sweep_t<float>(g, d, dt, in, out, rhs_mode, red, cfg, nblocks_out, out2);
}

// 2-D layout change A = [y][x] -> B = [x][y] (a_to_b) or back.
int enqueue_permute_2d(asd_grid g, const void* in, void* out, bool a_to_b) {
    const int nx = (int)g->d.n[0], ny = (int)g->d.n[1];
    const int n[3] = {a_to_b ? nx : ny, a_to_b ? ny : nx, 1};
    // a B array is a dense (nx, ny) array with y fastest
    const int64_t ds[3] = {a_to_b ? ny : nx, 1, (int64_t)nx * ny};
    hipError_t e = g->es == 8 ? launch_permute<double>((const double*)in, (double*)out, n, ds, g->st)
                              : launch_permute<float>((const float*)in, (float*)out, n, ds, g->st);
    return hip_check(e, "permute launch");
}

// Reduce a state into the standalone slot; returns the fold that finishes it.
int enqueue_reduce(asd_grid g, const void* x, const StepOut& out, FoldParams* fold) {
    const int nb = reduce_num_blocks(g->N);
    ReduceParams r{};
    r.partials = ring_slot(g, g->ring_slots);
    hipError_t e = g->es == 8 ? launch_reduce<double>((const double*)x, g->N, r, nb, g->st)
                              : launch_reduce<float>((const float*)x, g->N, r, nb, g->st);
    *fold = make_fold(g, r.partials, nb, 1, out, 0);
    return hip_check(e, "reduce launch");
}

int enqueue_fold(asd_grid g, const FoldParams& f) {
    if (!f.partials) return ASD_OK;
    return hip_check(launch_fold(f, g->st), "fold launch");
}

int check_dt(asd_grid g, double dt, bool explicit_scheme) {
    if (!finite_pos(dt)) return asd_fail(ASD_EINVAL, "dt must be finite and > 0");
    // the source enters the first sweep, which must read the natural layout
    if (!explicit_scheme && g->src && (g->d.flags & ASD_FLAG_REVERSE_ORDER))
        return asd_fail(ASD_EUNSUPPORTED, "a source term needs the sweep order x, y");
    // chi(T): the diffusivity follows the state, the caller bounds dt
    if ((g->d.flags & ASD_FLAG_ALLOW_UNSTABLE) || g->d.chi_exp != 0.0) return ASD_OK;
    const double chi = g->d.chi_par;
    double hmin2 = g->d.h[0] * g->d.h[0], sum_inv = 0.0;
    for (int q = 0; q < g->d.ndim; ++q) {
        hmin2 = std::min(hmin2, g->d.h[q] * g->d.h[q]);
        sum_inv += 1.0 / (g->d.h[q] * g->d.h[q]);
    }
    if (explicit_scheme) {
        if (g->d.ndim == 2 && chi * dt * sum_inv > 1.0)
            return asd_fail(ASD_EUNSTABLE, "explicit dt above the 2-D limit (chi dt sum 1/h^2 = %g > 1)", chi * dt * sum_inv);
        if (g->d.ndim == 3 && chi * dt / hmin2 > 0.444)
            return asd_fail(ASD_EUNSTABLE, "explicit dt above the 3-D limit (chi dt/h^2 = %g > 0.444)", chi * dt / hmin2);
    } else if (g->d.ndim == 3 && !(g->d.flags & ASD_FLAG_FOUR_STEP) && chi * dt / hmin2 > 8.25) {
        return asd_fail(ASD_EUNSTABLE, "3-D semi-implicit dt above the limit (chi dt/h^2 = %g > 8.25)", chi * dt / hmin2);
    }
    return ASD_OK;
}

// The whole multi-step call as a kernel sequence (used eagerly and under
// graph capture).  Outputs: the initial state is reduced and folded first;
// every step's last kernel writes per-block partials into the next ring
// slot, and one fold launch turns a full ring (or the last steps) into the
// outputs of each of those steps, off the sweeps' critical path.
// Workgroups of one launch of sweep d in the grid's current launch shape.
static int64_t sweep_num_blocks(asd_grid g, int d) {
    const SweepGeom G = sweep_geom(g->d.ndim, d);
    const int64_t nz = g->d.ndim == 3 ? g->d.n[2] : 1;
    const int64_t nax[3] = {g->d.n[0], g->d.n[1], nz};
    const int lpw = g->cfg[d].lpw;
    return (nax[G.t1] + lpw - 1) / lpw * nax[G.t2];
}

int enqueue_si_loop(asd_grid g, double dt, int nsteps, const StepOut& outs) {
    const int nd = g->d.ndim;
    const bool four = (g->d.flags & ASD_FLAG_FOUR_STEP) != 0;
    const bool reverse = (g->d.flags & ASD_FLAG_REVERSE_ORDER) != 0;  // 2-D only
    int rc = ASD_OK;
    // The initial state's energy: reduced by the first sweep, which reads
    // every cell of it once (2-step scheme in the order x, y, no source), and
    // folded before the first steps' fold; else by a standalone reduction.
    const bool fuse_e0 = outs.any() && nsteps > 0 && !four && !reverse && !g->src;
    // when the first sweep and the step's last sweep launch as many blocks,
    // the initial state's partials take ring slot 0 and are folded with the
    // first steps' (one fold launch fewer per call)
    const bool e0_in_ring = fuse_e0 && sweep_num_blocks(g, 0) == sweep_num_blocks(g, g->d.ndim - 1);
    FoldParams f0{};
    bool f0_pending = false;
    if (outs.any() && !fuse_e0) {
        rc = enqueue_reduce(g, g->T, outs, &f0);
        if (rc == ASD_OK) rc = enqueue_fold(g, f0);
    }
    // Reverse order (y, x): the state lives in layout B between steps, in
    // tmp1: T -> tmp1 before the first step, tmp1 -> T after the last.
    if (reverse && nsteps > 0 && rc == ASD_OK) rc = enqueue_permute_2d(g, g->T, g->tmp[1], true);
    // chi(T) (section 3.3): each sweep's coefficients from that sweep's input
    const bool chi_of_T = g->d.chi_exp != 0.0;
    auto sweep = [&](int d, const void* src, void* dst, int mode, const ReduceParams& red, int* nb) {
        int r = chi_of_T ? enqueue_coef(g, d, dt, src) : ASD_OK;
        if (r == ASD_OK) r = enqueue_sweep(g, d, dt, src, dst, mode, red, nullptr, nb);
        return r;
    };
    int used = e0_in_ring ? 1 : 0;  // ring slots holding unfolded entries
    for (int s = 0; s < nsteps && rc == ASD_OK; ++s) {
        const void* in = reverse ? g->tmp[1] : g->T;
        for (int i = 0; i < nd && rc == ASD_OK; ++i) {
            const int d = reverse ? nd - 1 - i : i;
            const bool produce = outs.any() && i == nd - 1;
            const int src = i == 0 ? SWEEP_SOURCE : 0;  // dt Q joins the first sweep
            ReduceParams red = no_reduce();
            if (produce) red.partials = ring_slot(g, used);
            const bool red_in = fuse_e0 && s == 0 && i == 0;
            if (red_in) red.partials = e0_in_ring ? ring_slot(g, 0) : ring_slot(g, g->ring_slots);
            int nb = 0;
            void* out;
            if (reverse) {
                // y: B (tmp1) -> A (tmp0); x: A (tmp0) -> B (tmp1).  The 4-step
                // intermediate (input layout) goes to T, free meanwhile.
                out = d == 1 ? g->tmp[0] : g->tmp[1];
                if (!four) {
                    rc = sweep(d, in, out, src, red, &nb);
                } else {
                    rc = sweep(d, in, g->T, SWEEP_KEEP_LAYOUT | src, no_reduce(), nullptr);
                    if (rc == ASD_OK) rc = sweep(d, g->T, out, SWEEP_SOLVE_ONLY, red, &nb);
                }
            } else if (!four) {
                out = (d == nd - 1) ? g->T : g->tmp[d];
                rc = sweep(d, in, out, src | (red_in ? SWEEP_REDUCE_INPUT : 0), red, &nb);
                if (red_in && !e0_in_ring) {
                    f0 = make_fold(g, red.partials, nb, 1, outs, 0);
                    f0_pending = true;
                }
            } else {
                // 4-step: transverse term at dt with the first half-step
                // solve, written in the input layout, then the second
                // half-step solve into the next sweep's layout.  States:
                // T -> tmp0 (-> T in 3-D) -> T.
                out = d == 0 ? g->tmp[0] : g->T;
                rc = sweep(d, in, g->tmp[1], SWEEP_KEEP_LAYOUT | src, no_reduce(), nullptr);
                if (rc == ASD_OK) rc = sweep(d, g->tmp[1], out, SWEEP_SOLVE_ONLY, red, &nb);
            }
            if (rc == ASD_OK && produce && (++used == g->ring_slots || s == nsteps - 1)) {
                // entry 0 first: the later folds check the drift against it
                if (f0_pending) {
                    rc = enqueue_fold(g, f0);
                    f0_pending = false;
                }
                if (rc == ASD_OK) rc = enqueue_fold(g, make_fold(g, ring_slot(g, 0), nb, used, outs, s + 2 - used));
                used = 0;
            }
            in = out;
        }
    }
    if (reverse && nsteps > 0 && rc == ASD_OK) rc = enqueue_permute_2d(g, g->tmp[1], g->T, false);
    return rc;
}

extern "C" int asd_step_semi_implicit(asd_grid g, double dt, int32_t nsteps, double* dev_energy) {
    if (!g) return asd_fail(ASD_EINVAL, "grid is NULL");
    if (nsteps < 0) return asd_fail(ASD_EINVAL, "nsteps must be >= 0");
    int rc = check_dt(g, dt, false);
    if (rc) return rc;
    rc = check_fields(g, true);
    if (rc) return rc;
    rc = prepare(g, dt);
    if (rc) return rc;
    // the legacy default stream cannot be captured: launch eagerly there
    StepOut o;
    o.energy = dev_energy;
    if (graphs_for(g, nsteps)) return run_si_graph(g, dt, nsteps, o);
    return enqueue_si_loop(g, dt, nsteps, o);
}

template <typename T>
static int enqueue_explicit_t(asd_grid g, double dt, const void* src, void* dst, const ReduceParams& red,
                              int* nblocks_out) {
    ExplicitParams<T> P{};
    P.U = (const T*)src;
    P.out = (T*)dst;
    for (int q = 0; q < 3; ++q) P.b[q] = q < g->d.ndim ? (const T*)g->b[q] : nullptr;
    P.chi = (g->d.flags & ASD_FLAG_PER_CELL_CHI) ? (const T*)g->chi : nullptr;
    P.n[0] = (int)g->d.n[0];
    P.n[1] = (int)g->d.n[1];
    P.n[2] = g->d.ndim == 3 ? (int)g->d.n[2] : 1;
    for (int d = 0; d < 3; ++d) {
        const double hd = d < g->d.ndim ? g->d.h[d] : 1.0;
        P.cn[d] = (T)(dt / (hd * hd));
        for (int t = 0; t < 3; ++t) {
            const double ht = t < g->d.ndim ? g->d.h[t] : 1.0;
            P.ct[d][t] = (T)(dt / (hd * ht));
        }
    }
    P.chi_par = (T)g->d.chi_par;
    P.chi_perp = (T)g->d.chi_perp;
    P.chi_exp = g->d.chi_exp;
    P.chi_tref = g->d.chi_tref;
    P.periodic = g->d.bc == ASD_BC_PERIODIC;
    P.dirichlet = g->d.bc == ASD_BC_DIRICHLET;
    P.Q = (const T*)g->src;
    P.dtq = (T)dt;
    P.limiter = g->d.limiter;
    P.red = red;
    return hip_check(launch_explicit<T>(P, g->d.ndim, g->st, nblocks_out), "explicit launch");
}

int enqueue_explicit(asd_grid g, double dt, const void* src, void* dst, const ReduceParams& red,
                     int* nblocks_out) {
    return g->es == 8 ? enqueue_explicit_t<double>(g, dt, src, dst, red, nblocks_out)
                      : enqueue_explicit_t<float>(g, dt, src, dst, red, nblocks_out);
}

int enqueue_copy(asd_grid g, const void* src, void* dst) {
    hipError_t e = g->es == 8 ? launch_copy<double>((const double*)src, (double*)dst, g->N, g->st)
                              : launch_copy<float>((const float*)src, (float*)dst, g->N, g->st);
    return hip_check(e, "copy launch");
}

// Explicit steps ping-pong between T and tmp[0]; an odd count ends with a
// copy.  Energy partials go through the ring as in the semi-implicit loop.
int enqueue_explicit_loop(asd_grid g, double dt, int nsteps, const StepOut& outs) {
    int rc = ASD_OK;
    if (outs.any()) {
        FoldParams f0;
        rc = enqueue_reduce(g, g->T, outs, &f0);
        if (rc == ASD_OK) rc = enqueue_fold(g, f0);
    }
    void* a = g->T;
    void* b = g->tmp[0];
    int used = 0;
    for (int s = 0; s < nsteps && rc == ASD_OK; ++s) {
        ReduceParams red = no_reduce();
        if (outs.any()) red.partials = ring_slot(g, used);
        int nb = 0;
        rc = enqueue_explicit(g, dt, a, b, red, &nb);
        if (rc == ASD_OK && outs.any() && (++used == g->ring_slots || s == nsteps - 1)) {
            rc = enqueue_fold(g, make_fold(g, ring_slot(g, 0), nb, used, outs, s + 2 - used));
            used = 0;
        }
        std::swap(a, b);
    }
    if (rc == ASD_OK && a != g->T) rc = enqueue_copy(g, a, g->T);
    return rc;
}

extern "C" int asd_step_explicit_limited(asd_grid g, double dt, int32_t nsteps, double* dev_energy) {
    if (!g) return asd_fail(ASD_EINVAL, "grid is NULL");
    if (nsteps < 0) return asd_fail(ASD_EINVAL, "nsteps must be >= 0");
    int rc = check_dt(g, dt, true);
    if (rc) return rc;
    rc = check_fields(g, true);
    if (rc) return rc;
    rc = prepare(g, 0.0);
    if (rc) return rc;
    StepOut o;
    o.energy = dev_energy;
    if (graphs_for(g, nsteps)) return run_explicit_graph(g, dt, nsteps, o);
    return enqueue_explicit_loop(g, dt, nsteps, o);
}

extern "C" int asd_step_series(asd_grid g, int32_t scheme, double dt, int32_t nsteps, double* dev_series) {
    if (!g) return asd_fail(ASD_EINVAL, "grid is NULL");
    if (scheme != ASD_SCHEME_SEMI_IMPLICIT && scheme != ASD_SCHEME_EXPLICIT)
        return asd_fail(ASD_EINVAL, "bad scheme %d", scheme);
    if (nsteps < 0) return asd_fail(ASD_EINVAL, "nsteps must be >= 0");
    if (!dev_series) return asd_fail(ASD_EINVAL, "series is NULL");
    const bool ex = scheme == ASD_SCHEME_EXPLICIT;
    int rc = check_dt(g, dt, ex);
    if (rc) return rc;
    rc = check_fields(g, true);
    if (rc) return rc;
    rc = prepare(g, ex ? 0.0 : dt);
    if (rc) return rc;
    StepOut o;
    o.series = dev_series;
    if (graphs_for(g, nsteps))
        return ex ? run_explicit_graph(g, dt, nsteps, o) : run_si_graph(g, dt, nsteps, o);
    return ex ? enqueue_explicit_loop(g, dt, nsteps, o) : enqueue_si_loop(g, dt, nsteps, o);
}

extern "C" int asd_status(asd_grid g, uint32_t* flags, double* stats) {
    if (!g) return asd_fail(ASD_EINVAL, "grid is NULL");
    if (!flags) return asd_fail(ASD_EINVAL, "flags is NULL");
    int rc = check_fields(g, true);
    if (rc) return rc;
    rc = prepare(g, 0.0);
    if (rc) return rc;
    FoldParams f;
    rc = enqueue_reduce(g, g->T, StepOut{}, &f);
    if (rc) return rc;
    rc = enqueue_fold(g, f);
    if (rc) return rc;
    rc = hip_check(hipStreamSynchronize(g->st), "stream synchronize");
    if (rc) return rc;
    unsigned fl = 0;
    double st[3];
    rc = hip_check(hipMemcpy(&fl, g->flags, sizeof fl, hipMemcpyDeviceToHost), "flags copy");
    if (rc) return rc;
    rc = hip_check(hipMemcpy(st, g->stats, sizeof st, hipMemcpyDeviceToHost), "stats copy");
    if (rc) return rc;
    *flags = fl;
    if (stats) memcpy(stats, st, sizeof st);
    // flags are sticky between status calls: clear them now they are reported
    return hip_check(launch_fill_u32(g->flags, 0u, 1, g->st), "flags reset");
}
