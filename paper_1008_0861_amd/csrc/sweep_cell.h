// The cell-slot variant of the line-tile body of one directional sweep of
// the split semi-implicit scheme (section 2, Eqs. xup / yup; 3-D
// generalisation of section 2.1).  Same operation as sweep_tile.h:
//
//     out = (1 + dt D_nn)^-1 ( U + F_{p+1/2} - F_{p-1/2} )      along each line
//
// (computed as U + A^-1 (Phi_{p+1/2} - Phi_{p-1/2}), Phi_f = F_f + alpha_f (U_{p+1} - U_p),
// the same solution in increment form) with, at the face between line
// cells p and p+1,
//     alpha_f = dt D_nn,f / h_n^2                  (precomputed, coef.hip)
//     F_f     = sum_t beta_t,f L(s_t(p+1), s_t(p))  beta_t,f = dt D_nt,f/(h_n h_t)
//     s_t(c)  = L(U[c+e_t] - U[c], U[c] - U[c-e_t])  (limited cell slope)
// Wall faces (insulating walls) have alpha = beta = 0 in the coefficient
// arrays, so every line is handled as a cyclic system.  T = 0 walls use odd
// ghosts (U[-1] = -U[0]): the transverse neighbours of a wall line are
// negated copies, and a wall face of cell c adds 2 alpha_w to its diagonal
// and -2 alpha_w U_c to its right-hand side (no coupling across the wrap);
// the two alpha_w of a line arrive in its wrap-face coefficient entry.  A
// source adds dt Q to U in the right-hand side (not in the slopes).
//
// How it differs from sweep_tile.h: the staging phase only packs each
// cell's slope, coefficients and state into a 16-byte LDS slot
// (tile_layout_cell), with no dependence between neighbouring lanes, and
// the solve phase evaluates the faces of its segment from the slots.  The
// staging chain is shorter and the LDS tile twice as large: this variant is
// the faster one on lines short enough that one tile per CU leaves the
// sweep latency-bound (1024-cell lines in FP32), the face-slot variant on
// long lines.  The autotuner picks per sweep.
//
// gfx950 mapping.  A workgroup owns `lpw` neighbouring lines; each line is
// owned by `wpl` waves (a wave never spans two lines, so every per-line
// quantity is wave-uniform and lives in scalar registers).  Phase 1 streams
// the lines (and the neighbouring lines needed for the transverse slopes)
// from HBM with coalesced loads, all issued before use, and packs each
// cell's slope, coefficients and state into one LDS slot (tile_layout_cell).
// Phase 2 splits each line into P contiguous segments, one per lane, dealt
// to the line's waves in turn; a lane reads its segment's slots (one vector
// LDS read per cell), builds the rows and eliminates the segment interior
// in registers, leaving one interface unknown per segment (its last cell).
// The P interface unknowns form a cyclic tridiagonal system (the Schur
// complement), solved by parallel cyclic reduction in log2(P) steps: every
// step whose stride is at least wpl pairs two lanes of one wave (a
// shuffle); only the log2(wpl) shorter strides go through LDS.  Each
// equation is kept normalised (unit diagonal), so a reduction step costs
// one reciprocal.  Phase 3 writes the tile back, transposed when the output
// layout has the transverse axis fastest (the next sweep then reads
// contiguous lines again).  The systems are symmetric, strictly diagonally
// dominant M-matrices: no pivoting anywhere.
//
// LIMC: the limiter as a compile-time constant (straight-line code), or -1
// to read it from the parameters.  EXT: compile in T = 0 walls, the source
// term and the second output copy (read from the parameters); without it
// that code is absent and the host never passes any of them.
#pragma once

#include "asd_device.h"
#include "asd_launch.h"

namespace asd {
namespace cell {

// Per-thread view of one tile: lines l1_0 .. l1_0+lpw-1 (transverse
// coordinate t2 = l2) of the sweep described by P, staged in the LDS buffer
// starting at buf.  Threads [q*spl, (q+1)*spl) own line q of the tile
// (spl = 64*wpl lanes: a power of two, so line membership is a shift,
// uniform over a wave).
template <typename T>
struct TileCtx {
    int l1_0, l2, q, k, l1;
    int line_ok;
    unsigned char* buf;
    unsigned char* row1;
    unsigned char* row2;
    const T *gU, *gU1m, *gU1p, *gU2m, *gU2p, *gA, *gB1, *gB2, *gQ;
    int neg1m, neg1p, neg2m, neg2p;  // T = 0 walls: that transverse neighbour is the odd ghost
    int ok1, ok2;        // LDS offsets of the thread's first cell (k) in its line's rows
    int ostep1, ostep2;  // LDS bytes between cells spl apart
};

template <typename T, int NDIM, bool EXT>
__device__ __forceinline__ TileCtx<T> cell_ctx(const SweepParams<T>& P, int l1_0, int l2, unsigned char* buf) {
    constexpr int ES = (int)sizeof(T);
    const TileLayout& Lo = P.lds;
    const int spl = 64 * P.wpl;
    const int pad = Lo.pad;
    const bool periodic = P.periodic != 0;
    const bool solve_only = P.rhs_mode != 0;
    TileCtx<T> c;
    c.l1_0 = l1_0;
    c.l2 = l2;
    c.q = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> P.spl_log2);
    c.k = threadIdx.x & (spl - 1);
    c.l1 = l1_0 + c.q;
    c.line_ok = c.l1 < P.nt1;
    c.buf = buf;
    c.row1 = buf + c.q * Lo.row1;
    c.row2 = buf + Lo.rows2_at + c.q * Lo.row2;
    // element offsets of this line and of its transverse neighbours (the
    // boundary rule applies once per line, not per cell)
    const int l1 = c.l1;
    const unsigned base = c.line_ok ? (unsigned)(l1 * P.si_t1 + l2 * P.si_t2) : 0u;
    unsigned base1m = base, base1p = base, base2m = base, base2p = base;
    if (c.line_ok && !solve_only) {
        base1m = base + (int)(nb_coord(l1 - 1, P.nt1, periodic) - l1) * P.si_t1;
        base1p = base + (int)(nb_coord(l1 + 1, P.nt1, periodic) - l1) * P.si_t1;
        if (NDIM == 3) {
            base2m = base + (int)(nb_coord(l2 - 1, P.nt2, periodic) - l2) * P.si_t2;
            base2p = base + (int)(nb_coord(l2 + 1, P.nt2, periodic) - l2) * P.si_t2;
        }
    }
    const bool dir = EXT && P.dirichlet != 0;
    c.neg1m = dir && l1 == 0;
    c.neg1p = dir && l1 == P.nt1 - 1;
    c.neg2m = dir && NDIM == 3 && l2 == 0;
    c.neg2p = dir && NDIM == 3 && l2 == P.nt2 - 1;
    c.gU = P.U + base;
    c.gU1m = P.U + base1m;
    c.gU1p = P.U + base1p;
    c.gU2m = P.U + base2m;
    c.gU2p = P.U + base2p;
    c.gA = P.alpha + base;
    c.gB1 = P.beta1 + base;
    c.gB2 = NDIM == 3 ? P.beta2 + base : nullptr;
    c.gQ = EXT && P.Q ? P.Q + base : nullptr;
    // spl is a multiple of the pad period, so cells spl apart are a fixed
    // number of bytes apart in LDS
    c.ok1 = cell_off1(c.k, ES, pad);
    c.ok2 = cell_off2(c.k, ES, pad);
    c.ostep1 = spl * 4 * ES + ((spl >> pad) << 4);
    c.ostep2 = (spl + (spl >> pad)) * 2 * ES;
    return c;
}

// Global data of CH of the thread's cells (k + (it0 + j) spl, j < CH).
template <typename T, int NDIM, int CH>
struct CellLoads {
    T u[CH], u1m[CH], u1p[CH], u2m[CH], u2p[CH], va[CH], vb1[CH], vb2[CH], q[CH];
};

// ---------------- phase 1a: coalesced loads of a chunk of cells.  Lane k of
// the line takes cells k, k+spl, ... (at most MMAX of them: the host
// guarantees n <= MMAX*spl).  All loads are issued before any is used; cells
// past the line end are clamped to the line's last cell.
template <typename T, int NDIM, int CH, bool EXT>
__device__ __forceinline__ void load_cells(const SweepParams<T>& P, const TileCtx<T>& c, int it0,
                                           CellLoads<T, NDIM, CH>& r) {
    constexpr int ES = (int)sizeof(T);
    const bool solve_only = P.rhs_mode != 0;
#pragma unroll
    for (int j = 0; j < CH; ++j) {
        const unsigned p = (unsigned)(c.k + ((it0 + j) << P.spl_log2));
        const unsigned bo = min(p, (unsigned)(P.n - 1)) * (unsigned)ES;
        r.u[j] = ldg_off(c.gU, bo);
        r.va[j] = ldg_off(c.gA, bo);
        // T = 0 walls need beta1 of the last cell (the left wall) in every sweep
        if (EXT && solve_only && P.dirichlet) r.vb1[j] = ldg_off(c.gB1, bo);
        if (EXT && P.Q) r.q[j] = ldg_off(c.gQ, bo);
        if (!solve_only) {
            r.u1m[j] = ldg_off(c.gU1m, bo);
            r.u1p[j] = ldg_off(c.gU1p, bo);
            r.vb1[j] = ldg_off(c.gB1, bo);
            if (NDIM == 3) {
                r.u2m[j] = ldg_off(c.gU2m, bo);
                r.u2p[j] = ldg_off(c.gU2p, bo);
                r.vb2[j] = ldg_off(c.gB2, bo);
            }
        }
    }
}

// ---------------- phase 1b: limited transverse slopes, packed into the
// cells' LDS slots (and the copy of cell 0 after the last cell).
template <typename T, int NDIM, int CH, int LIMC, bool EXT>
__device__ __forceinline__ void stage_cells(const SweepParams<T>& P, const TileCtx<T>& c, int it0,
                                            const CellLoads<T, NDIM, CH>& r) {
    constexpr int ES = (int)sizeof(T);
    const bool solve_only = P.rhs_mode != 0;
    const int lim = LIMC >= 0 ? LIMC : P.limiter;
    const int n = P.n;
    if (!c.line_ok) return;
#pragma unroll
    for (int j = 0; j < CH; ++j) {
        const int p = c.k + ((it0 + j) << P.spl_log2);
        if (p >= n) continue;
        // solve-only sweeps store zero slopes and transverse coefficients:
        // their transverse flux is then exactly zero
        T s1 = T(0), b1 = T(0), s2 = T(0), b2 = T(0);
        const T u = r.u[j];
        if (!solve_only) {
            s1 = EXT ? cell_slope<T>(lim, c.neg1m ? -u : r.u1m[j], u, c.neg1p ? -u : r.u1p[j])
                     : cell_slope<T>(lim, r.u1m[j], u, r.u1p[j]);
            b1 = r.vb1[j];
            if (NDIM == 3) {
                s2 = EXT ? cell_slope<T>(lim, c.neg2m ? -u : r.u2m[j], u, c.neg2p ? -u : r.u2p[j])
                         : cell_slope<T>(lim, r.u2m[j], u, r.u2p[j]);
                b2 = r.vb2[j];
            }
        }
        // the right-hand side's U (the slopes above use the state itself)
        const T us = EXT && P.Q ? u + P.dtq * r.q[j] : u;
        T a = r.va[j];
        if (EXT && P.dirichlet && p == n - 1) {
            // wrap face: no coupling and no transverse flux; its two wall
            // coefficients and this cell's U go to the spare slot after the
            // copy of cell 0
            lds_put4<T>(c.row1 + cell_off1(n + 1, ES, P.lds.pad), r.vb1[j], a, us, T(0));
            a = T(0);
            b1 = T(0);
        }
        lds_put4<T>(c.row1 + c.ok1 + (it0 + j) * c.ostep1, s1, a, b1, us);
        if (NDIM == 3) lds_put2<T>(c.row2 + c.ok2 + (it0 + j) * c.ostep2, s2, b2);
        if (p == 0) {  // the copy of cell 0 after the last cell
            lds_put4<T>(c.row1 + cell_off1(n, ES, P.lds.pad), s1, a, b1, us);
            if (NDIM == 3) lds_put2<T>(c.row2 + cell_off2(n, ES, P.lds.pad), s2, b2);
        }
    }
}

// Phases 2-3 of a staged tile: every thread of the block must call it; it
// ends with a barrier so that the tile's LDS buffer may be refilled.
// smem: the block's LDS base (exchange buffers).  Returns the thread's FP64
// sum and min / max of the values it wrote.  FULL: every segment holds
// exactly MMAX cells (an aligned tile layout), so the segment length is a
// compile-time constant and the per-cell bounds tests vanish.
template <typename T, int NDIM, int MMAX, int LIMC, bool EXT, bool FULL>
__device__ __forceinline__ void cell_solve_store(const SweepParams<T>& P, const TileCtx<T>& ctx, unsigned char* smem,
                                            double& lsum, T& lmin, T& lmax) {
    constexpr int ES = (int)sizeof(T);
    constexpr int SLOT = 4 * ES;  // bytes of a cell slot / exchange slot
    constexpr int UPOS = 3 * ES;  // byte offset of U inside a cell slot
    const int n = P.n;
    const int lpw = P.lpw;
    const int spl = 64 * P.wpl;
    const int tid = threadIdx.x;
    const int nthreads = blockDim.x;
    const int lim = LIMC >= 0 ? LIMC : P.limiter;
    const TileLayout& Lo = P.lds;
    const int pad = Lo.pad;
    const int spl_log2 = P.spl_log2;
    const int q = ctx.q, k = ctx.k, l1 = ctx.l1, l1_0 = ctx.l1_0, l2 = ctx.l2;
    const bool line_ok = ctx.line_ok;
    unsigned char* row1 = ctx.row1;
    unsigned char* row2 = ctx.row2;
    const int ok1 = ctx.ok1, ostep1 = ctx.ostep1;

    // ---------------- phase 2: per-lane segment elimination
    // Segments are interleaved over the line's waves: lane l of wave w owns
    // segment kseg = l * wpl + w.
    const int wpl_log2 = spl_log2 - 6;
    const int nseg = 1 << P.nseg_log2;
    const int kseg = ((k & 63) << wpl_log2) | (k >> 6);
    const bool active = line_ok && kseg < nseg;
    const int s0 = active ? (kseg * n) >> P.nseg_log2 : 0;
    const int m = FULL ? MMAX : (active ? (((kseg + 1) * n) >> P.nseg_log2) - s0 : 1);
    const int os0 = cell_off1(s0, ES, pad);  // the segment's first slot

    // The segment's slots: index 0 is the left neighbour cell s0-1 (mod n),
    // index c+1 is cell s0+c, c = 0..MMAX (slots past the segment's right
    // neighbour hold values that are ignored).  The segment's own slots are
    // consecutive; the neighbours are found separately where a pad or the
    // wrap may lie between (the copy of cell 0 covers the wrap on the
    // right).  All reads are issued before any arithmetic.
    T cs1[MMAX + 2], ca[MMAX + 2], cb1[MMAX + 2], cu[MMAX + 2], cs2[MMAX + 2], cb2[MMAX + 2];
    {
        int jl = s0 - 1;
        if (jl < 0) jl += n;
        const int jr = s0 + MMAX;  // right neighbour of an aligned segment (m == MMAX)
        const int os2 = cell_off2(s0, ES, pad);
        const int ol1 = cell_off1(jl, ES, pad), ol2 = cell_off2(jl, ES, pad);
        const int or1 = Lo.aligned ? cell_off1(jr, ES, pad) : os0 + MMAX * SLOT;
        const int or2 = Lo.aligned ? cell_off2(jr, ES, pad) : os2 + MMAX * 2 * ES;
        lds_get4<T>(row1 + ol1, cs1[0], ca[0], cb1[0], cu[0]);
        if (NDIM == 3) lds_get2<T>(row2 + ol2, cs2[0], cb2[0]);
#pragma unroll
        for (int c = 0; c < MMAX; ++c) {
            lds_get4<T>(row1 + os0 + c * SLOT, cs1[c + 1], ca[c + 1], cb1[c + 1], cu[c + 1]);
            if (NDIM == 3) lds_get2<T>(row2 + os2 + c * 2 * ES, cs2[c + 1], cb2[c + 1]);
        }
        lds_get4<T>(row1 + or1, cs1[MMAX + 1], ca[MMAX + 1], cb1[MMAX + 1], cu[MMAX + 1]);
        if (NDIM == 3) lds_get2<T>(row2 + or2, cs2[MMAX + 1], cb2[MMAX + 1]);
    }

    T av[MMAX], bv[MMAX], cv[MMAX], rv[MMAX];
    T gv[MMAX], hv[MMAX], wv[MMAX];
    T ae = T(0), be = T(1), ce = T(0), re = T(0);  // row of the segment's last cell
    {
        // Face f = 0..MMAX lies between slots f and f+1.  The line system
        // A x = U + F_{+} - F_{-} is solved in increment form,
        // x = U + delta with A delta = Phi_{+} - Phi_{-} and the face flux
        // Phi_f = F_f + alpha_f (U_right - U_left): algebraically the same
        // solution, but the solve's rounding now scales with |delta| rather
        // than |x|, and the right-hand side telescopes exactly.
        T phi_prev = T(0), alpha_prev = T(0);
#pragma unroll
        for (int f = 0; f <= MMAX; ++f) {
            T phi = ca[f] * (cu[f + 1] - cu[f]) + cb1[f] * limit2<T>(lim, cs1[f + 1], cs1[f]);
            if (NDIM == 3) phi += cb2[f] * limit2<T>(lim, cs2[f + 1], cs2[f]);
            if (f > 0) {
                const int i = f - 1;  // cell s0 + i, faces (f-1, f)
                av[i] = -alpha_prev;
                cv[i] = -ca[f];
                bv[i] = T(1) + alpha_prev + ca[f];
                rv[i] = phi - phi_prev;
                const bool last = f == m;
                ae = last ? av[i] : ae;
                be = last ? bv[i] : be;
                ce = last ? cv[i] : ce;
                re = last ? rv[i] : re;
            }
            alpha_prev = ca[f];
            phi_prev = phi;
        }
    }
    // T = 0 walls: the wall faces of the line's first and last cells (the
    // rows above saw zero coupling and flux across the wrap face)
    if (EXT && P.dirichlet && active && (s0 == 0 || s0 + m == n)) {
        T aL, aR, uR, unused;
        lds_get4<T>(row1 + cell_off1(n + 1, ES, pad), aL, aR, uR, unused);
        if (s0 == 0) {
            const T e = T(2) * aL;
            bv[0] += e;
            rv[0] -= e * cu[1];
            if (m == 1) {
                be += e;
                re -= e * cu[1];
            }
        }
        if (s0 + m == n) {
            const T e = T(2) * aR;
            be += e;
            re -= e * uR;
        }
    }
    // interior elimination: x_i = g_i - h_i x_{i+1} + w_i X_left, i = 0..m-2
    T gp = T(0), hp = T(0), wp = T(1);
#pragma unroll
    for (int i = 0; i < MMAX - 1; ++i) {
        if (i < m - 1) {
            const T inv = fast_rcp<T>(bv[i] - av[i] * hp);
            gv[i] = (rv[i] - av[i] * gp) * inv;
            hv[i] = cv[i] * inv;
            wv[i] = -av[i] * wp * inv;
            gp = gv[i];
            hp = hv[i];
            wp = wv[i];
        }
    }
    // first cell as a function of both interface unknowns: x_0 = Y + Uc XL + V XR
    T Y = T(0), Uc = T(0), V = T(1);
    if (m >= 2) {
        Y = gp;
        Uc = wp;
        V = -hp;
#pragma unroll
        for (int i = MMAX - 3; i >= 0; --i) {
            if (i <= m - 3) {
                Y = gv[i] - hv[i] * Y;
                Uc = wv[i] - hv[i] * Uc;
                V = -hv[i] * V;
            }
        }
    }

    // Reduced row of this segment's interface unknown X_k (its last cell),
    // kept normalised:  Ra X_{k-1} + X_k + Rc X_{k+1} = Rd.  It needs the
    // right neighbour's first-cell expression (Y, Uc, V).
    T Ra, Rc, Rd, XR, XL;
    if (P.wpl == 1) {
        // one wave per line: lane == segment; shuffles only, no barrier
        const int kr = (k + 1) & (nseg - 1);
        const T Yp = __shfl(Y, kr, 64), Up = __shfl(Uc, kr, 64), Vp = __shfl(V, kr, 64);
        if (active) {
            const T ib = fast_rcp<T>(be - ae * hp + ce * Up);
            Ra = ae * wp * ib;
            Rc = ce * Vp * ib;
            Rd = (re - ae * gp - ce * Yp) * ib;
        } else {
            Ra = T(0); Rc = T(0); Rd = T(0);
        }
        for (int s = 1; s < nseg; s <<= 1) {
            const int km = (k - s) & (nseg - 1), kp = (k + s) & (nseg - 1);
            const T am = __shfl(Ra, km, 64), cm = __shfl(Rc, km, 64), dm = __shfl(Rd, km, 64);
            const T ap = __shfl(Ra, kp, 64), cp = __shfl(Rc, kp, 64), dp = __shfl(Rd, kp, 64);
            if (k < nseg) {
                const T ib = fast_rcp<T>(T(1) - Ra * cm - Rc * ap);
                const T na = -Ra * am, nc = -Rc * cp, nd = Rd - Ra * dm - Rc * dp;
                Ra = na * ib;
                Rc = nc * ib;
                Rd = nd * ib;
            }
        }
        XR = Rd * fast_rcp<T>(T(1) + Ra + Rc);
        XL = __shfl(XR, (k - 1) & (nseg - 1), 64);
    } else {
        // several waves per line.  Exchanges between waves go through two
        // LDS buffers used alternately: a buffer is rewritten only after the
        // barrier that follows the last reads of it, so each exchange costs
        // one barrier.  Segment j's entry sits at the index of the thread
        // that owns it, (j mod wpl)*64 + j/wpl: a wave's stores are
        // contiguous.
        const int lb = q * spl;
        const int wmask = P.wpl - 1;
        auto slot = [&](int b, int j) -> unsigned char* {
            const int t = ((j & wmask) << 6) + (j >> wpl_log2);
            if (b == 0) return smem + Lo.pcr0_at + (lb + t) * SLOT;
            return Lo.pcr1_at < 0 ? row1 + cell_off1(t, ES, pad) : smem + Lo.pcr1_at + (lb + t) * SLOT;
        };
        int cur = 0;
        // Segments of at least 4 cells (MMAX >= 8, or a full tile with
        // MMAX >= 4): one exchange gives every segment its reduced row and
        // the stride-1 reduction step.  Segment k publishes the four numbers
        // that define its row given the first-cell expression (Y', U', V') of
        // segment k+1,
        //   ib = 1 / (A1 + A2 U'),  Ra = A3 ib,  Rc = A2 V' ib,  Rd = (A4 - A2 Y') ib,
        // and its own first-cell expression, in its second and third slots
        // (read by no other lane, and dead once the lane has read its
        // segment; the back substitution rewrites their U words only after
        // further barriers); a lane then forms rows k-1, k and k+1 itself.
        // Shorter segments exchange the first-cell expressions through
        // buffer 0 (its own area: other waves may still be reading the slot
        // rows) and take the stride-1 step in the loop below.
        constexpr bool MERGED = MMAX >= 8 || (FULL && MMAX >= 4);
        int s_first = 1;
        if constexpr (MERGED) {
            const T A1 = be - ae * hp, A2 = ce, A3 = ae * wp, A4 = re - ae * gp;
            if (active) {
                lds_put4<T>(row1 + cell_off1(s0 + 1, ES, pad), A1, A2, A3, A4);
                lds_put3<T>(row1 + cell_off1(s0 + 2, ES, pad), Y, Uc, V);
            }
            __syncthreads();
            if (active) {
                auto row = [](T a1, T a2, T a3, T a4, T yp, T up, T vp, T& ra, T& rc, T& rd) {
                    const T ib = fast_rcp<T>(a1 + a2 * up);
                    ra = a3 * ib;
                    rc = a2 * vp * ib;
                    rd = (a4 - a2 * yp) * ib;
                };
                auto seg_start = [&](int j) { return FULL ? j * MMAX : (j * n) >> P.nseg_log2; };
                const int sm = seg_start((kseg - 1) & (nseg - 1));
                const int sp1 = seg_start((kseg + 1) & (nseg - 1));
                const int sp2 = seg_start((kseg + 2) & (nseg - 1));
                T m1, m2, m3, m4, q1, q2, q3, q4, y1, u1, v1, y2, u2, v2, unused;
                lds_get4<T>(row1 + cell_off1(sm + 1, ES, pad), m1, m2, m3, m4);
                lds_get4<T>(row1 + cell_off1(sp1 + 1, ES, pad), q1, q2, q3, q4);
                lds_get4<T>(row1 + cell_off1(sp1 + 2, ES, pad), y1, u1, v1, unused);
                lds_get4<T>(row1 + cell_off1(sp2 + 2, ES, pad), y2, u2, v2, unused);
                T am, cm, dm, a0, c0, d0, ap, cp, dp;
                row(m1, m2, m3, m4, Y, Uc, V, am, cm, dm);   // row k-1 (its right neighbour is k)
                row(A1, A2, A3, A4, y1, u1, v1, a0, c0, d0);  // row k
                row(q1, q2, q3, q4, y2, u2, v2, ap, cp, dp);  // row k+1
                const T ib = fast_rcp<T>(T(1) - a0 * cm - c0 * ap);
                Ra = -a0 * am * ib;
                Rc = -c0 * cp * ib;
                Rd = (d0 - a0 * dm - c0 * dp) * ib;
            } else {
                Ra = T(0); Rc = T(0); Rd = T(0);
            }
            s_first = 2;
            // the next exchange takes buffer 0: buffer 1 may lie in the slot
            // rows, whose private slots other lanes may not have read yet
            // (no barrier separates those reads from the next exchange's
            // writes); buffer 1 is used only after that exchange's barrier
            cur = 1;
        } else {
            lds_put3<T>(slot(0, kseg), Y, Uc, V);
            __syncthreads();
            T Yp, Up, Vp, unused;
            lds_get4<T>(slot(0, (kseg + 1) & (nseg - 1)), Yp, Up, Vp, unused);
            if (active) {
                const T ib = fast_rcp<T>(be - ae * hp + ce * Up);
                Ra = ae * wp * ib;
                Rc = ce * Vp * ib;
                Rd = (re - ae * gp - ce * Yp) * ib;
            } else {
                Ra = T(0); Rc = T(0); Rd = T(0);
            }
        }
        // (further) strides below wpl: partners in other waves
        for (int s = s_first; s < nseg && s < P.wpl; s <<= 1) {
            cur ^= 1;
            lds_put3<T>(slot(cur, kseg), Ra, Rc, Rd);
            __syncthreads();
            if (active) {
                T am, cm, dm, ap, cp, dp, unused;
                lds_get4<T>(slot(cur, (kseg - s) & (nseg - 1)), am, cm, dm, unused);
                lds_get4<T>(slot(cur, (kseg + s) & (nseg - 1)), ap, cp, dp, unused);
                const T ib = fast_rcp<T>(T(1) - Ra * cm - Rc * ap);
                const T na = -Ra * am, nc = -Rc * cp, nd = Rd - Ra * dm - Rc * dp;
                Ra = na * ib;
                Rc = nc * ib;
                Rd = nd * ib;
            }
        }
        // strides wpl and up: partners are lanes of this wave, s / wpl apart
        // (the line's nseg / wpl segments of this wave sit in its first lanes)
        const int lane = k & 63;
        for (int s = P.wpl; s < nseg; s <<= 1) {
            const int nl = nseg >> wpl_log2, sl = s >> wpl_log2;
            const int lm = (lane - sl) & (nl - 1), lp = (lane + sl) & (nl - 1);
            const T am = __shfl(Ra, lm, 64), cm = __shfl(Rc, lm, 64), dm = __shfl(Rd, lm, 64);
            const T ap = __shfl(Ra, lp, 64), cp = __shfl(Rc, lp, 64), dp = __shfl(Rd, lp, 64);
            if (active) {
                const T ib = fast_rcp<T>(T(1) - Ra * cm - Rc * ap);
                const T na = -Ra * am, nc = -Rc * cp, nd = Rd - Ra * dm - Rc * dp;
                Ra = na * ib;
                Rc = nc * ib;
                Rd = nd * ib;
            }
        }
        XR = Rd * fast_rcp<T>(T(1) + Ra + Rc);
        cur ^= 1;
        *reinterpret_cast<T*>(slot(cur, kseg)) = XR;
        __syncthreads();
        XL = *reinterpret_cast<const T*>(slot(cur, (kseg - 1) & (nseg - 1)));
    }

    // ---------------- back substitution: x = U + delta, written over U in
    // the lane's own slots (the U positions are never part of an exchange)
    // (the FP64 sum, min and max of the written values, or of the input
    // state's: U of the slots, the source being excluded by the host)
    const bool red_in = P.red_in != 0;
    lsum = 0.0;
    lmin = T(__builtin_huge_val());
    lmax = T(-__builtin_huge_val());
    if (active) {
        T dn = XR;
#pragma unroll
        for (int i = MMAX - 1; i >= 0; --i) {
            if (i < m) {
                T d = XR;
                if (i < MMAX - 1 && i != m - 1) d = gv[i] - hv[i] * dn + wv[i] * XL;
                dn = d;
                const T x = cu[i + 1] + d;
                *reinterpret_cast<T*>(row1 + os0 + i * SLOT + UPOS) = x;
                const T rv = red_in ? cu[i + 1] : x;
                lsum += (double)rv;
                lmin = rv < lmin ? rv : lmin;
                lmax = rv > lmax ? rv : lmax;
            }
        }
    }
    __syncthreads();

    // ---------------- phase 3: store the tile
    if (P.so_t1 == 1) {
        // transposed output (t1 fastest): consecutive threads take the lpw
        // lines of one position p, so each store covers lpw adjacent elements
        const int lpw_log2 = P.lpw_log2;
        const int ncell = lpw * n;
        const int qq = tid & (lpw - 1);
        const int p0 = tid >> lpw_log2;
        const int pstep = nthreads >> lpw_log2;
        T* ob = P.out + (l1_0 + l2 * P.so_t2);
        const bool qq_ok = l1_0 + qq < P.nt1;
        // second copy in the input layout (EXT instantiations only): lpw runs
        // of consecutive cells per store
        T* ob2 = EXT && P.out2 && qq_ok ? P.out2 + (unsigned)((l1_0 + qq) * P.si_t1 + l2 * P.si_t2) : nullptr;
        // pstep == spl: consecutive positions of a thread are ostep1 apart in LDS
        const unsigned char* rq = ctx.buf + qq * Lo.row1 + UPOS + cell_off1(p0, ES, pad);
        const unsigned o0 = (unsigned)(p0 * P.so_n + qq);
        const unsigned ostep = (unsigned)(pstep * P.so_n);
#pragma unroll
        for (int it = 0; it < MMAX; ++it) {
            if (tid + it * nthreads >= ncell) break;
            if (qq_ok) {
                const T x = *reinterpret_cast<const T*>(rq + it * ostep1);
                // 2-D: a 32-bit byte offset from the uniform base (a 2-D field
                // stays below 4 GiB); 3-D: a 32-bit element index
                if (NDIM == 2)
                    stg_off(ob, (o0 + it * ostep) * (unsigned)ES, x);
                else
                    ob[o0 + it * ostep] = x;
                if (ob2) ob2[p0 + it * pstep] = x;
            }
        }
    } else if (line_ok) {
        // line-contiguous output
        T* ob = P.out + (l1 * P.so_t1 + l2 * P.so_t2);
#pragma unroll
        for (int it = 0; it < MMAX; ++it) {
            const int p = k + (it << spl_log2);
            if (p >= n) break;
            ob[(unsigned)(p * P.so_n)] = *reinterpret_cast<const T*>(row1 + ok1 + it * ostep1 + UPOS);
        }
    }

    __syncthreads();  // the LDS may be refilled by the next tile
}

// One whole tile (phases 1-3) in LDS buffer 0, loading in chunks of up to 8
// cells per thread.
template <typename T, int NDIM, int MMAX, int LIMC, bool EXT = false>
__device__ __forceinline__ void sweep_tile(const SweepParams<T>& P, int l1_0, int l2, unsigned char* smem,
                                           double& lsum, T& lmin, T& lmax) {
    const TileCtx<T> c = cell_ctx<T, NDIM, EXT>(P, l1_0, l2, smem);
    constexpr int CH = MMAX < 8 ? MMAX : 8;
#pragma unroll
    for (int it0 = 0; it0 < MMAX; it0 += CH) {
        if ((it0 << P.spl_log2) >= P.n) break;
        CellLoads<T, NDIM, CH> r;
        load_cells<T, NDIM, CH, EXT>(P, c, it0, r);
        stage_cells<T, NDIM, CH, LIMC, EXT>(P, c, it0, r);
    }
    __syncthreads();
    if (P.lds.aligned)
        cell_solve_store<T, NDIM, MMAX, LIMC, EXT, true>(P, c, smem, lsum, lmin, lmax);
    else
        cell_solve_store<T, NDIM, MMAX, LIMC, EXT, false>(P, c, smem, lsum, lmin, lmax);
}

}  // namespace cell
}  // namespace asd
