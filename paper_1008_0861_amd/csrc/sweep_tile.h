// The line-tile body of one directional sweep of the split semi-implicit scheme (section 2,
// Eqs. xup / yup; 3-D generalisation of section 2.1):
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
// arrays, so every line is handled as a cyclic system.
//
// gfx950 mapping.  A workgroup owns `lpw` neighbouring lines; each line is
// owned by `wpl` waves.  Phase 1 streams the lines (and the neighbouring
// lines needed for the transverse slopes) from HBM into LDS with coalesced
// loads, all issued before use.  Phase 2 splits each line into P contiguous
// segments, one per lane; a lane eliminates its segment interior in
// registers, leaving one interface unknown per segment (its last cell).
// The P interface unknowns form a cyclic tridiagonal system (the Schur
// complement), solved by parallel cyclic reduction in log2(P) steps: across
// lanes with shuffles when a wave owns the line, through LDS otherwise.
// Each equation is kept normalised (unit diagonal), so a reduction step
// costs one reciprocal.  Phase 3 writes the tile back, transposed when the
// output layout has the transverse axis fastest (the next sweep then reads
// contiguous lines again).  The systems are symmetric, strictly diagonally
// dominant M-matrices: no pivoting anywhere.
#pragma once

#include "asd_device.h"
#include "asd_launch.h"

namespace asd {

// One tile: lines l1_0 .. l1_0+lpw-1 (transverse coordinate t2 = l2) of the
// sweep described by P.  Every thread of the block must call it; it ends
// with a barrier so that consecutive tiles may reuse the LDS.  Returns the
// thread's FP64 sum and min / max of the values it wrote.
template <typename T, int NDIM, int MMAX>
__device__ __forceinline__ void sweep_tile(const SweepParams<T>& P, int l1_0, int l2, unsigned char* smem_raw,
                                           double& lsum, T& lmin, T& lmax) {
    T* smem = reinterpret_cast<T*>(smem_raw);
    const int n = P.n;
    const int LS = lds_line_stride<T>(n);
    const int lpw = P.lpw;
    const int seg_per_line = 64 * P.wpl;  // lanes per line
    const int tid = threadIdx.x;
    const int nthreads = blockDim.x;
    const bool solve_only = P.rhs_mode != 0;

    // LDS regions, each lpw * LS elements
    T* sU = smem;
    T* sA = sU + lpw * LS;
    T* sS1 = sA + lpw * LS;
    T* sB1 = sS1 + lpw * LS;
    T* sS2 = sB1 + lpw * LS;                    // 3-D only
    T* sB2 = sS2 + (NDIM == 3 ? lpw * LS : 0);  // 3-D only
    T* pcr = sB2 + (NDIM == 3 ? lpw * LS : 0);  // 3 * nthreads elements
    T* pA = pcr;
    T* pC = pA + nthreads;
    T* pD = pC + nthreads;

    const bool periodic = P.periodic != 0;
    const int lim = P.limiter;

    // Threads [q*spl, (q+1)*spl) own line q of the tile (spl = 64*wpl lanes;
    // powers of two, so line membership is a shift).
    const int spl_log2 = P.spl_log2;
    const int q = tid >> spl_log2;
    const int k = tid & (seg_per_line - 1);
    const int l1 = l1_0 + q;
    const bool line_ok = l1 < P.nt1;
    // element offsets of this line and of its transverse neighbours (the
    // boundary rule applies once per line, not per cell)
    const unsigned base = line_ok ? (unsigned)(l1 * P.si_t1 + l2 * P.si_t2) : 0u;
    unsigned base1m = base, base1p = base, base2m = base, base2p = base;
    if (line_ok && !solve_only) {
        base1m = base + (int)(nb_coord(l1 - 1, P.nt1, periodic) - l1) * P.si_t1;
        base1p = base + (int)(nb_coord(l1 + 1, P.nt1, periodic) - l1) * P.si_t1;
        if (NDIM == 3) {
            base2m = base + (int)(nb_coord(l2 - 1, P.nt2, periodic) - l2) * P.si_t2;
            base2p = base + (int)(nb_coord(l2 + 1, P.nt2, periodic) - l2) * P.si_t2;
        }
    }

    // ---------------- phase 1: coalesced loads -> LDS (U, alpha, slopes, beta)
    // Lane k of the line loads cells k, k+spl, ... (at most MMAX of them: the
    // host guarantees n <= MMAX*spl).  All loads of a chunk of up to 8 cells
    // are issued before any is used; cells past the line end are clamped to
    // the line's first cell.
    constexpr int CH = MMAX < 8 ? MMAX : 8;
    const T* rowU = sU + q * LS;
#pragma unroll
    for (int it0 = 0; it0 < MMAX; it0 += CH) {
        if (it0 << spl_log2 >= n) break;
        T u[CH], u1m[CH], u1p[CH], u2m[CH], u2p[CH], va[CH], vb1[CH], vb2[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int p = k + ((it0 + j) << spl_log2);
            const unsigned pc = p < n ? (unsigned)p : 0u;
            u[j] = P.U[base + pc];
            va[j] = P.alpha[base + pc];
            if (!solve_only) {
                u1m[j] = P.U[base1m + pc];
                u1p[j] = P.U[base1p + pc];
                vb1[j] = P.beta1[base + pc];
                if (NDIM == 3) {
                    u2m[j] = P.U[base2m + pc];
                    u2p[j] = P.U[base2p + pc];
                    vb2[j] = P.beta2[base + pc];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int p = k + ((it0 + j) << spl_log2);
            if (!line_ok || p >= n) continue;
            const int li = q * LS + lds_pad<T>(p);
            sU[li] = u[j];
            sA[li] = va[j];
            if (!solve_only) {
                sS1[li] = cell_slope<T>(lim, u1m[j], u[j], u1p[j]);
                sB1[li] = vb1[j];
                if (NDIM == 3) {
                    sS2[li] = cell_slope<T>(lim, u2m[j], u[j], u2p[j]);
                    sB2[li] = vb2[j];
                }
            }
        }
    }
    __syncthreads();

    // ---------------- phase 2: per-lane segment elimination
    const int nseg = 1 << P.nseg_log2;
    const bool active = line_ok && k < nseg;
    const int s0 = active ? (k * n) >> P.nseg_log2 : 0;
    const int m = active ? (((k + 1) * n) >> P.nseg_log2) - s0 : 1;

    T av[MMAX], bv[MMAX], cv[MMAX], rv[MMAX];
    T gv[MMAX], hv[MMAX], wv[MMAX];
    T ae = T(0), be = T(1), ce = T(0), re = T(0);  // row of the segment's last cell
    {
        // faces f = 0..m: the face between cells j0 = s0-1+f and j0+1 (mod n).
        // The line system A x = U + F_{+} - F_{-} is solved in increment
        // form, x = U + delta with A delta = Phi_{+} - Phi_{-} and the face
        // flux Phi_f = F_f + alpha_f (U_{j0+1} - U_{j0}): algebraically the
        // same solution, but the solve's rounding now scales with |delta|
        // rather than |x|, and the right-hand side telescopes exactly.
        T phi_prev = T(0), alpha_prev = T(0);
        const T* rowA = sA + q * LS;
        const T* rowS1 = sS1 + q * LS;
        const T* rowS2 = sS2 + q * LS;
        const T* rowB1 = sB1 + q * LS;
        const T* rowB2 = sB2 + q * LS;
#pragma unroll
        for (int f = 0; f <= MMAX; ++f) {
            if (f <= m && active) {
                int j0 = s0 - 1 + f;
                if (j0 < 0) j0 += n;
                int j1 = j0 + 1;
                if (j1 == n) j1 = 0;
                const int i0 = lds_pad<T>(j0), i1 = lds_pad<T>(j1);
                const T alpha = rowA[i0];
                T phi = alpha * (rowU[i1] - rowU[i0]);
                if (!solve_only) {
                    phi += rowB1[i0] * limit2<T>(lim, rowS1[i1], rowS1[i0]);
                    if (NDIM == 3) phi += rowB2[i0] * limit2<T>(lim, rowS2[i1], rowS2[i0]);
                }
                if (f > 0) {
                    const int i = f - 1;  // cell s0 + i, faces (f-1, f)
                    av[i] = -alpha_prev;
                    cv[i] = -alpha;
                    bv[i] = T(1) + alpha_prev + alpha;
                    rv[i] = phi - phi_prev;
                    if (f == m) { ae = av[i]; be = bv[i]; ce = cv[i]; re = rv[i]; }
                }
                alpha_prev = alpha;
                phi_prev = phi;
            }
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
    const int kr = (k + 1) & (nseg - 1);
    if (P.wpl == 1) {
        // one wave per line: lane == segment; shuffles, no barrier
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
        // several waves per line: the same reduction through LDS
        const int lb = q * seg_per_line;  // this line's slots
        pA[tid] = Y;
        pC[tid] = Uc;
        pD[tid] = V;
        __syncthreads();
        {
            const T Yp = pA[lb + kr], Up = pC[lb + kr], Vp = pD[lb + kr];
            if (active) {
                const T ib = fast_rcp<T>(be - ae * hp + ce * Up);
                Ra = ae * wp * ib;
                Rc = ce * Vp * ib;
                Rd = (re - ae * gp - ce * Yp) * ib;
            } else {
                Ra = T(0); Rc = T(0); Rd = T(0);
            }
        }
        __syncthreads();
        pA[tid] = Ra; pC[tid] = Rc; pD[tid] = Rd;
        __syncthreads();
        for (int s = 1; s < nseg; s <<= 1) {
            T na = Ra, nc = Rc, nd = Rd;
            if (k < nseg) {
                const int km = lb + ((k - s) & (nseg - 1));
                const int kp = lb + ((k + s) & (nseg - 1));
                const T am = pA[km], cm = pC[km], dm = pD[km];
                const T ap = pA[kp], cp = pC[kp], dp = pD[kp];
                const T ib = fast_rcp<T>(T(1) - Ra * cm - Rc * ap);
                na = -Ra * am * ib;
                nc = -Rc * cp * ib;
                nd = (Rd - Ra * dm - Rc * dp) * ib;
            }
            __syncthreads();
            Ra = na; Rc = nc; Rd = nd;
            pA[tid] = Ra; pC[tid] = Rc; pD[tid] = Rd;
            __syncthreads();
        }
        XR = Rd * fast_rcp<T>(T(1) + Ra + Rc);
        pA[tid] = XR;
        __syncthreads();
        XL = pA[lb + ((k - 1) & (nseg - 1))];
    }

    // ---------------- back substitution: x = U + delta, into LDS (reuse sU;
    // each lane reads and overwrites only its own cells)
    lsum = 0.0;
    lmin = T(__builtin_huge_val());
    lmax = T(-__builtin_huge_val());
    if (active) {
        T* rowX = sU + q * LS;
        T dn = XR;
        {
            const int ix = lds_pad<T>(s0 + m - 1);
            const T x = rowX[ix] + XR;
            rowX[ix] = x;
            lsum = (double)x;
            lmin = lmax = x;
        }
#pragma unroll
        for (int i = MMAX - 2; i >= 0; --i) {
            if (i <= m - 2) {
                const T d = gv[i] - hv[i] * dn + wv[i] * XL;
                dn = d;
                const int ix = lds_pad<T>(s0 + i);
                const T x = rowX[ix] + d;
                rowX[ix] = x;
                lsum += (double)x;
                lmin = x < lmin ? x : lmin;
                lmax = x > lmax ? x : lmax;
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
#pragma unroll
        for (int it = 0; it < MMAX; ++it) {
            const int idx = tid + it * nthreads;
            if (idx >= ncell) break;
            const int qq = idx & (lpw - 1), p = idx >> lpw_log2;
            if (l1_0 + qq >= P.nt1) continue;
            P.out[(unsigned)(p * P.so_n + (l1_0 + qq) + l2 * P.so_t2)] = sU[qq * LS + lds_pad<T>(p)];
        }
    } else {
        // line-contiguous output
        const unsigned obase = line_ok ? (unsigned)(l1 * P.so_t1 + l2 * P.so_t2) : 0u;
#pragma unroll
        for (int it = 0; it < MMAX; ++it) {
            const int p = k + (it << spl_log2);
            if (p >= n) break;
            if (line_ok) P.out[obase + (unsigned)(p * P.so_n)] = rowU[lds_pad<T>(p)];
        }
    }

    __syncthreads();  // the LDS may be refilled by the next tile
}

}  // namespace asd
