// The line-tile body of one directional sweep of the split semi-implicit scheme (section 2,
// Eqs. xup / yup; 3-D generalisation of section 2.1):
//
//     out = (1 + dt D_nn)^-1 ( U + F_{p+1/2} - F_{p-1/2} )      along each line
//
// computed in increment form, out = U + delta with
//     A delta = Phi_{p+1/2} - Phi_{p-1/2},   Phi_f = F_f + alpha_f (U_{p+1} - U_p)
// (the same solution; the solve's rounding then scales with |delta|, not
// |out|), where at the face f between line cells p and p+1
//     alpha_f = dt D_nn,f / h_n^2                  (precomputed, coef.hip)
//     F_f     = sum_t beta_t,f L(s_t(p+1), s_t(p))  beta_t,f = dt D_nt,f/(h_n h_t)
//     s_t(c)  = L(U[c+e_t] - U[c], U[c] - U[c-e_t])  (limited cell slope)
// and A has -alpha_{p-1/2}, 1 + alpha_{p-1/2} + alpha_{p+1/2}, -alpha_{p+1/2}
// on row p.  Wall faces (insulating walls) have alpha = beta = 0 in the
// coefficient arrays, so every line is handled as a cyclic system.  T = 0
// walls use odd ghosts (U[-1] = -U[0]): the transverse neighbours of a wall
// line are negated copies, the wrap face carries nothing, and a wall face
// of cell c adds 2 alpha_w to its diagonal and -2 alpha_w U_c to its
// right-hand side (the two alpha_w of a line arrive in its wrap-face
// coefficient entry).  A source adds dt Q to the right-hand side.
//
// gfx950 mapping.  A workgroup owns `lpw` neighbouring lines; each line is
// owned by `wpl` waves (a wave never spans two lines, so every per-line
// quantity is wave-uniform).
//   Phase 1 streams the lines (and the neighbouring lines the transverse
//   slopes need) from HBM with coalesced loads, all issued before use.  Each
//   wave takes a contiguous range of 64-cell chunks, lane k cell k of each:
//   a lane evaluates the face after its cell, taking the next cell's state
//   and slope from lane k+1 by a DPP rotation of the wave (lane 63 from lane
//   0 of the next chunk).  Every face is evaluated once, with no exchange
//   between waves, and the pair (alpha_f, Phi_f) goes to the face's LDS slot.
//   Phase 2 splits each line into P contiguous segments, one per lane, dealt
//   to the line's waves in turn; a lane reads its segment's face slots,
//   builds its rows and eliminates the segment interior in registers,
//   leaving one interface unknown per segment (its last cell).  The P
//   interface unknowns form a cyclic tridiagonal system (the Schur
//   complement), solved by parallel cyclic reduction in log2(P) steps:
//   every step whose stride is at least wpl pairs two lanes of one wave (a
//   shuffle); only the log2(wpl) shorter strides go through LDS.  Each
//   equation is kept normalised (unit diagonal), so a reduction step costs
//   one reciprocal.  The back substitution writes each cell's increment into
//   its face slot.
//   Phase 3 adds the increments to U (read again from cache, issued before
//   the solve so that the solve hides the latency) and writes the
//   tile, transposed when the output layout has the transverse axis fastest
//   (the next sweep then reads contiguous lines again).  The FP64 sum and
//   the min / max of the written values are reduced here when asked for.
// The systems are symmetric, strictly diagonally dominant M-matrices: no
// pivoting anywhere.
//
// LIMC: the limiter as a compile-time constant (straight-line code), or -1
// to read it from the parameters.  EXT: compile in T = 0 walls, the source
// term and the second output copy (read from the parameters); without it
// that code is absent and the host never passes any of them.
#pragma once

#include "asd_device.h"
#include "asd_launch.h"

namespace asd {

// Two-element slot accesses (one 8- or 16-byte LDS access).
template <typename T>
__device__ __forceinline__ void lds_put_pair(unsigned char* p, T a, T b);
template <>
__device__ __forceinline__ void lds_put_pair<float>(unsigned char* p, float a, float b) {
    *reinterpret_cast<float2*>(p) = make_float2(a, b);
}
template <>
__device__ __forceinline__ void lds_put_pair<double>(unsigned char* p, double a, double b) {
    *reinterpret_cast<double2*>(p) = make_double2(a, b);
}
template <typename T>
__device__ __forceinline__ void lds_get_pair(const unsigned char* p, T& a, T& b);
template <>
__device__ __forceinline__ void lds_get_pair<float>(const unsigned char* p, float& a, float& b) {
    const float2 v = *reinterpret_cast<const float2*>(p);
    a = v.x;
    b = v.y;
}
template <>
__device__ __forceinline__ void lds_get_pair<double>(const unsigned char* p, double& a, double& b) {
    const double2 v = *reinterpret_cast<const double2*>(p);
    a = v.x;
    b = v.y;
}

// Per-thread view of one tile: lines l1_0 .. l1_0+lpw-1 (transverse
// coordinate t2 = l2) of the sweep described by P, staged in the LDS buffer
// starting at buf.  Threads [q*sio, (q+1)*sio) own line q of the tile for
// staging and stores (sio = 64*wpl*io lanes: a power of two, so line
// membership is a shift, uniform over a wave); the first spl = 64*wpl of
// them also solve it.
template <typename T>
struct TileCtx {
    int l1_0, l2, q, k, w, lane, l1;
    int line_ok;
    unsigned base;  // element offset of the line in the input layout
    unsigned char* buf;
    unsigned char* row1;
    const T *gU, *gU1m, *gU1p, *gU2m, *gU2p, *gA, *gB1, *gB2;
    int neg1m, neg1p, neg2m, neg2p;  // T = 0 walls: that transverse neighbour is the odd ghost
};

// HALF: two lines per wave (lanes 0-31 and 32-63), a line's solve spread
// over 32 lanes (short lines in batches); the line index is then per lane.
template <typename T, int NDIM, bool EXT, bool HALF = false>
__device__ __forceinline__ TileCtx<T> tile_ctx(const SweepParams<T>& P, int l1_0, int l2, unsigned char* buf) {
    const int sio_log2 = P.spl_log2 + P.io_log2;
    const bool periodic = P.periodic != 0;
    const bool solve_only = P.rhs_mode != 0;
    TileCtx<T> c;
    c.l1_0 = l1_0;
    c.l2 = l2;
    if constexpr (HALF) {
        c.q = (int)threadIdx.x >> 5;
        c.k = threadIdx.x & 31;
        c.w = 0;
        c.lane = c.k;
    } else {
        c.q = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> sio_log2);
        c.k = threadIdx.x & ((1 << sio_log2) - 1);
        c.w = __builtin_amdgcn_readfirstlane(c.k >> 6);
        c.lane = c.k & 63;
    }
    c.l1 = l1_0 + c.q;
    c.line_ok = c.l1 < P.nt1;
    c.buf = buf;
    c.row1 = buf + c.q * P.lds.row1;
    // element offsets of this line and of its transverse neighbours (the
    // boundary rule applies once per line, not per cell)
    const int l1 = c.l1;
    const unsigned base = c.line_ok ? (unsigned)(l1 * P.si_t1 + l2 * P.si_t2) : 0u;
    c.base = base;
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
    return c;
}

// Phase 1, staging.  Wave w of a line owns the chunks c0 .. c0+jn-1 of 64
// cells (chunk c: cells 64c .. 64c+63; c0 = w * cpw, cpw = ceil(nch / wpl),
// nch = ceil(n / 64)), and lane k takes cell 64c+k of each.  The right
// neighbour of a lane's cell is in lane k+1 (a rotation of the wave by one
// lane), except for lane 63, whose neighbour is lane 0 of the next chunk:
// the next chunk of the wave, or for the wave's last chunk one extra chunk
// loaded only for that (the first chunk of the next wave's range, or chunk 0
// past the line's end: the periodic wrap).
template <typename T>
struct ChunkData {
    T u, u1m, u1p, u2m, u2p, a, b1, b2;
};

// Loads of chunk `chunk` (face data too when `face`), all issued before use.
// Cell n is cell 0 on a periodic line (the wrap neighbour); cells past the
// line's end are otherwise clamped to its last cell (their values are not
// used).
template <typename T, int NDIM, bool HALF = false>
__device__ __forceinline__ void load_chunk(const SweepParams<T>& P, const TileCtx<T>& c, int chunk, bool face,
                                           ChunkData<T>& r) {
    constexpr int ES = (int)sizeof(T);
    constexpr int CL = HALF ? 5 : 6;  // log2 of the cells per chunk (lanes per line)
    const bool solve_only = P.rhs_mode != 0;
    const int n = P.n;
    int p = (chunk << CL) + c.lane;
    if ((chunk << CL) + (1 << CL) - 1 >= n) p = p < n ? p : (p == n && P.periodic ? 0 : n - 1);  // wave-uniform test
    const unsigned bo = (unsigned)p * (unsigned)ES;
    r.u = ldg_off(c.gU, bo);
    if (!solve_only) {
        r.u1m = ldg_off(c.gU1m, bo);
        r.u1p = ldg_off(c.gU1p, bo);
        if (NDIM == 3) {
            r.u2m = ldg_off(c.gU2m, bo);
            r.u2p = ldg_off(c.gU2p, bo);
        }
    }
    if (face) {
        r.a = ldg_off(c.gA, bo);
        if (!solve_only) {
            r.b1 = ldg_off(c.gB1, bo);
            if (NDIM == 3) r.b2 = ldg_off(c.gB2, bo);
        }
    }
}

// Lane i takes v of lane i+1 mod 64 (a DPP rotation of the whole wave).
template <typename T>
__device__ __forceinline__ T rotate_down(T v) {
    return dpp_mov<0x134, 0xf>(v, v);
}
// The same within each half of the wave (lane i takes lane i+1 mod 32 of
// its half): two lines per wave.
template <typename T>
__device__ __forceinline__ T rotate_down_half(T v, int lane32) {
    return __shfl(v, (lane32 + 1) & 31, 32);
}

// Stages the tile's faces: for every cell p of the line,
//   Phi_f = alpha_f (U_{p+1} - U_p) + sum_t beta_t,f L(s_t(p+1), s_t(p))
// and (alpha_f, Phi_f) into the face's slot.  Loads go in batches of up to
// nine chunks; the last chunk of a batch waits for the next batch's first
// (its lane 63 needs it).
template <typename T, int NDIM, int MMAX, int LIMC, bool EXT, bool HALF = false>
__device__ __forceinline__ void stage_tile(const SweepParams<T>& P, const TileCtx<T>& c) {
    constexpr int ES = (int)sizeof(T);
    constexpr int CL = HALF ? 5 : 6;  // log2 of the cells per chunk
    auto rot = [&](T v) { return HALF ? rotate_down_half<T>(v, c.lane) : rotate_down<T>(v); };
    constexpr int CH = MMAX < 8 ? MMAX + 1 : 9;
    const bool solve_only = P.rhs_mode != 0;
    const int lim = LIMC >= 0 ? LIMC : P.limiter;
    const int n = P.n;
    const int wio_log2 = HALF ? 0 : P.spl_log2 + P.io_log2 - 6;  // staging waves per line: wpl * io
    const int nch = (n + (1 << CL) - 1) >> CL;
    const int cpw = (nch + (1 << wio_log2) - 1) >> wio_log2;
    const int c0 = c.w * cpw;
    const int jn = min(cpw, nch - c0);  // this wave's chunks (wave-uniform, may be <= 0)
    if (jn <= 0 || !c.line_ok) return;
    const int cnext = c0 + jn < nch ? c0 + jn : 0;
    // the chunk whose faces wait for its successor: own data and its rotation
    T pu = T(0), ps1 = T(0), ps2 = T(0), pa = T(0), pb1 = T(0), pb2 = T(0);
    T ru = T(0), rs1 = T(0), rs2 = T(0);
    // (guards rather than early exits keep the unrolled batch arrays in registers)
#pragma unroll
    for (int j0 = 0; j0 <= MMAX; j0 += CH) {
        if (j0 > jn) continue;
        ChunkData<T> r[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int jj = j0 + j;  // chunk jj of the wave; jj == jn: the extra chunk
            if (jj <= jn) load_chunk<T, NDIM, HALF>(P, c, jj < jn ? c0 + jj : cnext, jj < jn, r[j]);
        }
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int jj = j0 + j;
            if (jj > jn) continue;
            const T u = r[j].u;
            T s1 = T(0), s2 = T(0);
            if (!solve_only) {
                s1 = EXT ? cell_slope<T>(lim, c.neg1m ? -u : r[j].u1m, u, c.neg1p ? -u : r[j].u1p)
                         : cell_slope<T>(lim, r[j].u1m, u, r[j].u1p);
                if (NDIM == 3)
                    s2 = EXT ? cell_slope<T>(lim, c.neg2m ? -u : r[j].u2m, u, c.neg2p ? -u : r[j].u2p)
                             : cell_slope<T>(lim, r[j].u2m, u, r[j].u2p);
            }
            const T nru = rot(u);
            T nrs1 = T(0), nrs2 = T(0);
            if (!solve_only) {
                nrs1 = rot(s1);
                if (NDIM == 3) nrs2 = rot(s2);
            }
            if (jj > 0) {
                // faces of chunk jj-1: the right neighbours from its own
                // rotation, lane 63's from this chunk's lane 0
                const bool last_lane = c.lane == (1 << CL) - 1;
                const T un = last_lane ? nru : ru;
                const int p = ((c0 + jj - 1) << CL) + c.lane;
                if (p < n) {
                    T a = pa;
                    T phi = a * (un - pu);
                    if (!solve_only) {
                        phi += pb1 * limit2<T>(lim, last_lane ? nrs1 : rs1, ps1);
                        if (NDIM == 3) phi += pb2 * limit2<T>(lim, last_lane ? nrs2 : rs2, ps2);
                    }
                    if (EXT && P.dirichlet && p == n - 1) {
                        // the wrap face couples nothing; its coefficient entry holds the
                        // line's two wall coefficients, read by the solve
                        a = T(0);
                        phi = T(0);
                    }
                    lds_put_pair<T>(c.row1 + slot_off(p, ES, P.lds.pad), a, phi);
                }
            }
            pu = u;
            ps1 = s1;
            ps2 = s2;
            pa = r[j].a;
            pb1 = r[j].b1;
            pb2 = r[j].b2;
            ru = nru;
            rs1 = nrs1;
            rs2 = nrs2;
        }
    }
}

// Phases 2-3 of a staged tile: every thread of the block must call it.
// smem: the block's LDS base (exchange buffers).  Returns the thread's FP64
// sum and min / max of the values it wrote when the launch reduces (else
// 0, +inf, -inf).  FULL: every segment holds exactly MMAX cells (an aligned
// tile layout), so the segment length is a compile-time constant and the
// per-cell bounds tests vanish.  REUSE: the block stages another tile in
// the same LDS afterwards (a closing barrier).
template <typename T, int NDIM, int MMAX, int LIMC, bool EXT, bool FULL, bool REUSE, bool HALF = false>
__device__ __forceinline__ void solve_store(const SweepParams<T>& P, const TileCtx<T>& ctx, unsigned char* smem,
                                            const T (&uu)[MMAX], double& lsum, T& lmin, T& lmax) {
    constexpr int ES = (int)sizeof(T);
    constexpr int SLOT = 2 * ES;   // bytes of a face slot
    constexpr int XSLOT = 4 * ES;  // bytes of an exchange entry
    const int n = P.n;
    const int lpw = P.lpw;
    const int spl = 64 * P.wpl;
    const int tid = threadIdx.x;
    const int nthreads = blockDim.x;
    const TileLayout& Lo = P.lds;
    const int pad = Lo.pad;
    const int spl_log2 = P.spl_log2;
    const int q = ctx.q, k = ctx.k, l1 = ctx.l1, l1_0 = ctx.l1_0, l2 = ctx.l2;
    const bool line_ok = ctx.line_ok;
    unsigned char* row1 = ctx.row1;

    // ---------------- phase 2: per-lane segment elimination
    // Segments are interleaved over the line's waves: lane l of wave w owns
    // segment kseg = l * wpl + w.
    const int wpl_log2 = HALF ? 0 : spl_log2 - 6;
    constexpr int SW = HALF ? 32 : 64;  // lanes that exchange by shuffles: one line's
    const int sio_log2 = spl_log2 + P.io_log2;
    const int nseg = 1 << P.nseg_log2;
    const bool part = k < spl;  // this thread takes part in the solve
    const int kseg = HALF ? k : ((k & 63) << wpl_log2) | (k >> 6);
    const bool active = part && line_ok && kseg < nseg;
    const int s0 = active ? (FULL ? kseg * MMAX : (kseg * n) >> P.nseg_log2) : 0;
    const int m = FULL ? MMAX : (active ? (((kseg + 1) * n) >> P.nseg_log2) - s0 : 1);
    const int os0 = slot_off(s0, ES, pad);  // the segment's first slot

    // The faces of the segment: index 0 is the face before cell s0 (the last
    // face of the previous segment, or the wrap face), index i+1 the face
    // after cell s0+i, i = 0..MMAX-1 (faces past the segment's end are read
    // from the row's spare slots and ignored).  The segment's own slots are
    // consecutive.  All reads are issued before any arithmetic.
    T fa[MMAX + 1], fp[MMAX + 1];
    {
        int jl = s0 - 1;
        if (jl < 0) jl += n;
        lds_get_pair<T>(row1 + slot_off(jl, ES, pad), fa[0], fp[0]);
        if constexpr (FULL && (MMAX % 2) == 0) {
#pragma unroll
            for (int c = 0; c < MMAX; c += 2)
                lds_get4<T>(row1 + os0 + c * SLOT, fa[c + 1], fp[c + 1], fa[c + 2], fp[c + 2]);
        } else {
#pragma unroll
            for (int c = 0; c < MMAX; ++c) lds_get_pair<T>(row1 + os0 + c * SLOT, fa[c + 1], fp[c + 1]);
        }
    }

    T av[MMAX], bv[MMAX], cv[MMAX], rv[MMAX];
#pragma unroll
    for (int i = 0; i < MMAX; ++i) {
        av[i] = -fa[i];
        cv[i] = -fa[i + 1];
        bv[i] = T(1) + fa[i] + fa[i + 1];
        rv[i] = fp[i + 1] - fp[i];
    }
    if (EXT && active) {
        const T* lineU = P.U + ctx.base;
        if (P.Q) {
            // the source joins the right-hand side (input in the natural layout)
            const T* lineQ = P.Q + ctx.base;
#pragma unroll
            for (int i = 0; i < MMAX; ++i)
                if (i < m) rv[i] += P.dtq * lineQ[s0 + i];
        }
        if (P.dirichlet) {
            // T = 0 walls: the wall faces of the line's first and last cells
            // (alpha of the right wall and beta1 of the left wall sit in the
            // wrap-face entry of the coefficient arrays)
            if (s0 == 0) {
                const T e = T(2) * P.beta1[ctx.base + n - 1];
                bv[0] += e;
                rv[0] -= e * lineU[0];
            }
            if (s0 + m == n) {
                const T e = T(2) * P.alpha[ctx.base + n - 1];
                const T ul = lineU[n - 1];
#pragma unroll
                for (int i = 0; i < MMAX; ++i) {
                    if (i == m - 1) {
                        bv[i] += e;
                        rv[i] -= e * ul;
                    }
                }
            }
        }
    }
    T ae = av[MMAX - 1], be = bv[MMAX - 1], ce = cv[MMAX - 1], re = rv[MMAX - 1];  // row of the last cell
    if (!FULL) {
#pragma unroll
        for (int i = 0; i < MMAX; ++i) {
            const bool last = i == m - 1;
            ae = last ? av[i] : ae;
            be = last ? bv[i] : be;
            ce = last ? cv[i] : ce;
            re = last ? rv[i] : re;
        }
    }
    // interior elimination: x_i = g_i - h_i x_{i+1} + w_i X_left, i = 0..m-2
    T gv[MMAX], hv[MMAX], wv[MMAX];
    T gp = T(0), hp = T(0), wp = T(1);
#pragma unroll
    for (int i = 0; i < MMAX - 1; ++i) {
        if (FULL || i < m - 1) {
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
    if (FULL ? MMAX >= 2 : m >= 2) {
        Y = gp;
        Uc = wp;
        V = -hp;
#pragma unroll
        for (int i = MMAX - 3; i >= 0; --i) {
            if (FULL || i <= m - 3) {
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
        const T Yp = __shfl(Y, kr, SW), Up = __shfl(Uc, kr, SW), Vp = __shfl(V, kr, SW);
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
            const T am = __shfl(Ra, km, SW), cm = __shfl(Rc, km, SW), dm = __shfl(Rd, km, SW);
            const T ap = __shfl(Ra, kp, SW), cp = __shfl(Rc, kp, SW), dp = __shfl(Rd, kp, SW);
            if (k < nseg) {
                const T ib = fast_rcp<T>(T(1) - Ra * cm - Rc * ap);
                const T na = -Ra * am, nc = -Rc * cp, nd = Rd - Ra * dm - Rc * dp;
                Ra = na * ib;
                Rc = nc * ib;
                Rd = nd * ib;
            }
        }
        XR = Rd * fast_rcp<T>(T(1) + Ra + Rc);
        XL = __shfl(XR, (k - 1) & (nseg - 1), SW);
    } else {
        // several waves per line.  Exchanges between waves go through two
        // LDS buffers used alternately: a buffer is rewritten only after the
        // barrier that follows the last reads of it, so each exchange costs
        // one barrier.  Segment j's entry sits at the index of the thread
        // that owns it, (j mod wpl)*64 + j/wpl: a wave's stores are
        // contiguous.
        // Segments of MMAX >= 8 cells on an aligned tile keep both buffers
        // in their own face slots 4..7, which only the owner reads before
        // the first exchange (the last face slot, which the next segment
        // also reads, is rewritten only after that exchange's barrier).
        constexpr bool INSLOT = FULL && MMAX >= 8;
        const int lb = q << sio_log2;
        const int wmask = P.wpl - 1;
        unsigned char* const xbuf0 = smem + Lo.pcr0_at + lb * XSLOT;
        unsigned char* const xbuf1 = smem + Lo.pcr1_at + lb * XSLOT;
        auto xslot = [&](int b, int j) -> unsigned char* {
            if constexpr (INSLOT) return row1 + slot_off(j * MMAX, ES, pad) + (4 + 2 * b) * SLOT;
            const int t = ((j & wmask) << 6) + (j >> wpl_log2);
            return (b == 0 ? xbuf0 : xbuf1) + t * XSLOT;
        };
        int cur = 0;
        // Segments of MMAX >= 8 cells on an aligned tile: one exchange gives
        // every segment its reduced row and the stride-1 reduction step.
        // Segment k publishes the four numbers that define its row given the
        // first-cell expression (Y', U', V') of segment k+1,
        //   ib = 1 / (A1 + A2 U'),  Ra = A3 ib,  Rc = A2 V' ib,  Rd = (A4 - A2 Y') ib,
        // and its own first-cell expression, in its first four face slots
        // (read by no other lane: only the segment's last face slot is also
        // read by the next segment, and the back substitution rewrites them
        // only after further barriers); a lane then forms rows k-1, k and
        // k+1 itself.  Otherwise the first-cell expressions go through
        // buffer 0 and the stride-1 step runs in the loop below.
        constexpr bool MERGED = FULL && MMAX >= 8;
        int s_first = 1;
        if constexpr (MERGED) {
            const T A1 = be - ae * hp, A2 = ce, A3 = ae * wp, A4 = re - ae * gp;
            if (active) {
                lds_put4<T>(row1 + os0, A1, A2, A3, A4);
                lds_put4<T>(row1 + os0 + 2 * SLOT, Y, Uc, V, T(0));
            }
            __syncthreads();
            if (active) {
                auto row = [](T a1, T a2, T a3, T a4, T yp, T up, T vp, T& ra, T& rc, T& rd) {
                    const T ib = fast_rcp<T>(a1 + a2 * up);
                    ra = a3 * ib;
                    rc = a2 * vp * ib;
                    rd = (a4 - a2 * yp) * ib;
                };
                const int om = slot_off(((kseg - 1) & (nseg - 1)) * MMAX, ES, pad);
                const int op1 = slot_off(((kseg + 1) & (nseg - 1)) * MMAX, ES, pad);
                const int op2 = slot_off(((kseg + 2) & (nseg - 1)) * MMAX, ES, pad);
                T m1, m2, m3, m4, q1, q2, q3, q4, y1, u1, v1, y2, u2, v2, unused;
                lds_get4<T>(row1 + om, m1, m2, m3, m4);
                lds_get4<T>(row1 + op1, q1, q2, q3, q4);
                lds_get4<T>(row1 + op1 + 2 * SLOT, y1, u1, v1, unused);
                lds_get4<T>(row1 + op2 + 2 * SLOT, y2, u2, v2, unused);
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
            cur = 1;  // the next exchange takes buffer 0
        } else {
            if (part) lds_put4<T>(xslot(0, kseg), Y, Uc, V, T(0));
            __syncthreads();
            T Yp, Up, Vp, unused;
            lds_get4<T>(xslot(0, (kseg + 1) & (nseg - 1)), Yp, Up, Vp, unused);
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
            if (part) lds_put4<T>(xslot(cur, kseg), Ra, Rc, Rd, T(0));
            __syncthreads();
            if (active) {
                T am, cm, dm, ap, cp, dp, unused;
                lds_get4<T>(xslot(cur, (kseg - s) & (nseg - 1)), am, cm, dm, unused);
                lds_get4<T>(xslot(cur, (kseg + s) & (nseg - 1)), ap, cp, dp, unused);
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
        if (part) *reinterpret_cast<T*>(xslot(cur, kseg)) = XR;
        __syncthreads();
        XL = *reinterpret_cast<const T*>(xslot(cur, (kseg - 1) & (nseg - 1)));
    }

    // ---------------- back substitution: each cell's increment goes into the
    // second element of its face slot (no exchange reads those after this)
    if (active) {
        T dn = XR;
#pragma unroll
        for (int i = MMAX - 1; i >= 0; --i) {
            if (FULL || i < m) {
                T d = XR;
                if (i < MMAX - 1 && (FULL || i != m - 1)) d = gv[i] - hv[i] * dn + wv[i] * XL;
                dn = d;
                *reinterpret_cast<T*>(row1 + os0 + i * SLOT + ES) = d;
            }
        }
    }
    __syncthreads();

    // ---------------- phase 3: out = U + delta, stored
    const bool reduce = P.red.partials != nullptr;
    const bool red_in = P.red_in != 0;  // the input's cells instead (each stored cell once)
    lsum = 0.0;
    lmin = T(__builtin_huge_val());
    lmax = T(-__builtin_huge_val());
    if (P.so_t1 == 1) {
        // transposed output (t1 fastest): consecutive threads take the lpw
        // lines of one position p, so each store covers lpw adjacent elements
        const int lpw_log2 = P.lpw_log2;
        const int qq = tid & (lpw - 1);
        const int p0 = tid >> lpw_log2;
        const int pstep = nthreads >> lpw_log2;
        const int lq = l1_0 + qq;
        const bool qq_ok = lq < P.nt1;
        T* ob = P.out + (l1_0 + l2 * P.so_t2);
        // second copy in the input layout (EXT instantiations only): lpw runs
        // of consecutive cells per store
        T* ob2 = EXT && P.out2 && qq_ok ? P.out2 + (unsigned)(lq * P.si_t1 + l2 * P.si_t2) : nullptr;
        const unsigned char* rq = ctx.buf + qq * Lo.row1;
#pragma unroll
        for (int it = 0; it < MMAX; ++it) {
            const int p = p0 + it * pstep;
            if (p >= n) break;
            if (qq_ok) {
                T unused, d;
                lds_get_pair<T>(rq + slot_off(p, ES, pad), unused, d);
                const T x = uu[it] + d;
                // 2-D: a 32-bit byte offset from the uniform base (a 2-D field
                // stays below 4 GiB); 3-D: a 32-bit element index
                if (NDIM == 2)
                    stg_off(ob, (unsigned)(p * P.so_n + qq) * (unsigned)ES, x);
                else
                    ob[(unsigned)(p * P.so_n + qq)] = x;
                if (ob2) ob2[p] = x;
                if (reduce) {
                    const T rv = red_in ? uu[it] : x;
                    lsum += (double)rv;
                    lmin = rv < lmin ? rv : lmin;
                    lmax = rv > lmax ? rv : lmax;
                }
            }
        }
    } else if (line_ok) {
        // line-contiguous output
        T* ob = P.out + (l1 * P.so_t1 + l2 * P.so_t2);
#pragma unroll
        for (int it = 0; it < MMAX; ++it) {
            const int p = k + (it << sio_log2);
            if (p >= n) break;
            T unused, d;
            lds_get_pair<T>(row1 + slot_off(p, ES, pad), unused, d);
            const T x = uu[it] + d;
            ob[(unsigned)(p * P.so_n)] = x;
            if (reduce) {
                const T rv = red_in ? uu[it] : x;
                lsum += (double)rv;
                lmin = rv < lmin ? rv : lmin;
                lmax = rv > lmax ? rv : lmax;
            }
        }
    }
    if (REUSE) __syncthreads();  // the LDS may be refilled by the next tile
}

// U at the cells the thread stores in phase 3, in the store's mapping:
// transposed output (t1 fastest): thread tid takes line tid mod lpw at
// positions tid / lpw + it * (nthreads / lpw); line-contiguous output: the
// thread's line at positions k + it * sio.  Cells past the line end get 0.
template <typename T, int MMAX>
__device__ __forceinline__ void load_store_u(const SweepParams<T>& P, const TileCtx<T>& c, T (&uu)[MMAX]) {
    const int n = P.n;
    if (P.so_t1 == 1) {
        const int tid = threadIdx.x;
        const int qq = tid & (P.lpw - 1);
        const int p0 = tid >> P.lpw_log2;
        const int pstep = (int)blockDim.x >> P.lpw_log2;
        const int lq = c.l1_0 + qq;
        const bool qq_ok = lq < P.nt1;
        // the tile's first line as a uniform base, the lane's line and cell
        // as a 32-bit byte offset (the tile's lines span a few MB at most)
        const T* tileU = P.U + (unsigned)(c.l1_0 * P.si_t1 + c.l2 * P.si_t2);
        const unsigned ob0 = qq_ok ? (unsigned)(qq * P.si_t1) * (unsigned)sizeof(T) : 0u;
#pragma unroll
        for (int it = 0; it < MMAX; ++it) {
            const int p = p0 + it * pstep;
            uu[it] = (qq_ok && p < n) ? ldg_off(tileU, ob0 + (unsigned)p * (unsigned)sizeof(T)) : T(0);
        }
    } else {
        const T* lineU = P.U + c.base;
#pragma unroll
        for (int it = 0; it < MMAX; ++it) {
            const int p = c.k + (it << (P.spl_log2 + P.io_log2));
            uu[it] = (c.line_ok && p < n) ? ldg_off(lineU, (unsigned)p * (unsigned)sizeof(T)) : T(0);
        }
    }
}

// One whole tile (phases 1-3) in the LDS buffer at smem.  REUSE: the caller
// stages further tiles in the same LDS afterwards.
template <typename T, int NDIM, int MMAX, int LIMC, bool EXT = false, bool REUSE = false, bool HALF = false>
__device__ __forceinline__ void sweep_tile(const SweepParams<T>& P, int l1_0, int l2, unsigned char* smem,
                                           double& lsum, T& lmin, T& lmax) {
    const TileCtx<T> c = tile_ctx<T, NDIM, EXT, HALF>(P, l1_0, l2, smem);
    stage_tile<T, NDIM, MMAX, LIMC, EXT, HALF>(P, c);
    // U of the cells this thread stores in phase 3 (same lines, still in
    // cache): loaded now, so that the solve hides their latency
    T uu[MMAX];
    load_store_u<T, MMAX>(P, c, uu);
    __syncthreads();
    if (P.lds.aligned)
        solve_store<T, NDIM, MMAX, LIMC, EXT, true, REUSE, HALF>(P, c, smem, uu, lsum, lmin, lmax);
    else
        solve_store<T, NDIM, MMAX, LIMC, EXT, false, REUSE, HALF>(P, c, smem, uu, lsum, lmin, lmax);
}

}  // namespace asd
