// One directional sweep of the split semi-implicit scheme (section 2,
// Eqs. xup / yup; 3-D generalisation of section 2.1):
//
//     out = (1 + dt D_nn)^-1 ( U + F_{p+1/2} - F_{p-1/2} )      along each line
//
// with, at the face between line cells p and p+1,
//     b_f     = (b_p + b_{p+1}) / 2                       (arithmetic mean)
//     chi_f   = chi_par, or the harmonic mean of the two cells
//     alpha_f = dt (chi_perp + (chi_f - chi_perp) bn_f^2) / h_n^2
//     F_f     = dt (chi_f - chi_perp) bn_f sum_t bt_f L(s_t(p+1), s_t(p)) / (h_n h_t)
//     s_t(c)  = L(U[c+e_t] - U[c], U[c] - U[c-e_t])       (limited cell slope)
// and wall faces (insulating walls) carrying no flux.
//
// gfx950 mapping.  A workgroup owns `lpw` neighbouring lines; each line is
// owned by `wpl` waves.  Phase 1 streams the lines (and the neighbouring
// lines needed for the transverse slopes) from HBM with coalesced loads into
// LDS.  Phase 2 splits each line into P contiguous segments, one per lane;
// a lane eliminates its segment interior in registers, leaving one interface
// unknown per segment (the segment's last cell).  The P interface unknowns
// form a cyclic tridiagonal system (the Schur complement), solved by
// parallel cyclic reduction in LDS in log2(P) steps; lanes then
// back-substitute their interiors.  Phase 3 writes the line tile back,
// optionally transposed (so the next sweep again reads contiguous lines).
// All systems are symmetric, strictly diagonally dominant M-matrices, so no
// pivoting is needed anywhere.
#include "asd_device.h"
#include "asd_launch.h"

namespace asd {

template <typename T, int NDIM, int MMAX>
__global__ void __launch_bounds__((SweepBounds<T, MMAX>::max_threads)) sweep_kernel(SweepParams<T> P) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* smem = reinterpret_cast<T*>(smem_raw);
    const int n = P.n;
    const int LS = lds_line_stride<T>(n);
    const int lpw = P.lpw;
    const int seg_per_line = 64 * P.wpl;  // lanes per line
    const int tid = threadIdx.x;
    const int nthreads = blockDim.x;

    // LDS regions, each lpw * LS elements
    T* sU = smem;
    T* sS1 = sU + lpw * LS;
    T* sS2 = sS1 + lpw * LS;            // 3-D only
    T* sBn = sS2 + (NDIM == 3 ? lpw * LS : 0);
    T* sB1 = sBn + lpw * LS;
    T* sB2 = sB1 + lpw * LS;            // 3-D only
    T* sChi = sB2 + (NDIM == 3 ? lpw * LS : 0);  // only if per-cell chi
    T* pcr = sChi + (P.chi ? lpw * LS : 0);       // 4 * nthreads elements
    T* pA = pcr;
    T* pB = pA + nthreads;
    T* pC = pB + nthreads;
    T* pD = pC + nthreads;

    // XCD-aware block order: consecutive logical blocks on the same XCD so
    // that the halo lines and the partial lines of a transposed store are
    // shared through that XCD's L2.
    int blk = blockIdx.x;
    const int nblk = gridDim.x;
    if ((nblk & 7) == 0) blk = (blk & 7) * (nblk >> 3) + (blk >> 3);
    const int nb1 = (P.nt1 + lpw - 1) / lpw;
    const int l2 = blk / nb1;
    const int l1_0 = (blk - l2 * nb1) * lpw;
    const bool periodic = P.periodic != 0;
    const int lim = P.limiter;
    const bool solve_only = P.rhs_mode != 0;

    // ---------------- phase 1: coalesced load of U, slopes, b, chi -> LDS
    const bool line_fast_in = (P.si_n == 1);
    const int ncell = lpw * n;
    for (int idx = tid; idx < ncell; idx += nthreads) {
        int q, p;
        if (line_fast_in) { q = idx / n; p = idx - q * n; }
        else { p = idx / lpw; q = idx - p * lpw; }
        const int l1 = l1_0 + q;
        if (l1 >= P.nt1) continue;
        const int64_t c = (int64_t)p * P.si_n + (int64_t)l1 * P.si_t1 + (int64_t)l2 * P.si_t2;
        const T u = P.U[c];
        const int li = q * LS + lds_pad<T>(p);
        sU[li] = u;
        if (!solve_only) {
            const int64_t cm = c + (nb_coord(l1 - 1, P.nt1, periodic) - l1) * P.si_t1;
            const int64_t cp = c + (nb_coord(l1 + 1, P.nt1, periodic) - l1) * P.si_t1;
            sS1[li] = cell_slope<T>(lim, P.U[cm], u, P.U[cp]);
            if (NDIM == 3) {
                const int64_t dm = c + (nb_coord(l2 - 1, P.nt2, periodic) - l2) * P.si_t2;
                const int64_t dp = c + (nb_coord(l2 + 1, P.nt2, periodic) - l2) * P.si_t2;
                sS2[li] = cell_slope<T>(lim, P.U[dm], u, P.U[dp]);
                sB2[li] = P.bt2[c];
            }
            sB1[li] = P.bt1[c];
        }
        sBn[li] = P.bn[c];
        if (P.chi) sChi[li] = P.chi[c];
    }
    __syncthreads();

    // ---------------- phase 2: per-lane segment elimination
    const int q = tid / seg_per_line;
    const int k = tid - q * seg_per_line;
    const int nseg = P.P;
    const bool line_ok = (l1_0 + q) < P.nt1;
    const bool active = line_ok && k < nseg;
    const int s0 = active ? (int)(((int64_t)k * n) / nseg) : 0;
    const int m = active ? (int)(((int64_t)(k + 1) * n) / nseg) - s0 : 1;
    const T chi_perp = P.chi_perp;

    T av[MMAX], bv[MMAX], cv[MMAX], rv[MMAX];
    T gv[MMAX], hv[MMAX], wv[MMAX];
    T ae = T(0), be = T(1), ce = T(0), re = T(0);  // row of the segment's last cell
    {
        // faces f = 0..m: face between cells j = s0-1+f and j+1
        T alpha_prev = T(0), flux_prev = T(0);
        const T* rowU = sU + q * LS;
        const T* rowS1 = sS1 + q * LS;
        const T* rowS2 = sS2 + q * LS;
        const T* rowBn = sBn + q * LS;
        const T* rowB1 = sB1 + q * LS;
        const T* rowB2 = sB2 + q * LS;
        const T* rowChi = sChi + q * LS;
#pragma unroll
        for (int f = 0; f <= MMAX; ++f) {
            if (f <= m && active) {
                int j0 = s0 - 1 + f, j1 = s0 + f;
                T alpha = T(0), flux = T(0);
                bool wall = false;
                if (j0 < 0) { if (periodic) j0 += n; else wall = true; }
                if (j1 >= n) { if (periodic) j1 -= n; else wall = true; }
                if (!wall) {
                    const int i0 = lds_pad<T>(j0), i1 = lds_pad<T>(j1);
                    const T bnf = T(0.5) * (rowBn[i0] + rowBn[i1]);
                    T chif = P.chi_par;
                    if (P.chi) chif = harmonic<T>(rowChi[i0], rowChi[i1]);
                    const T dpar = chif - chi_perp;
                    alpha = P.cnn * (chi_perp + dpar * bnf * bnf);
                    if (!solve_only) {
                        const T b1f = T(0.5) * (rowB1[i0] + rowB1[i1]);
                        T tr = P.cnt1 * b1f * limit2<T>(lim, rowS1[i1], rowS1[i0]);
                        if (NDIM == 3) {
                            const T b2f = T(0.5) * (rowB2[i0] + rowB2[i1]);
                            tr += P.cnt2 * b2f * limit2<T>(lim, rowS2[i1], rowS2[i0]);
                        }
                        flux = dpar * bnf * tr;
                    }
                }
                if (f > 0) {
                    const int i = f - 1;  // cell s0 + i, faces (f-1, f)
                    av[i] = -alpha_prev;
                    cv[i] = -alpha;
                    bv[i] = T(1) + alpha_prev + alpha;
                    rv[i] = rowU[lds_pad<T>(s0 + i)] + flux - flux_prev;
                    if (f == m) { ae = av[i]; be = bv[i]; ce = cv[i]; re = rv[i]; }
                }
                alpha_prev = alpha;
                flux_prev = flux;
            }
        }
    }
    // interior elimination: x_i = g_i - h_i x_{i+1} + w_i X_left, i = 0..m-2
    T gp = T(0), hp = T(0), wp = T(1);
#pragma unroll
    for (int i = 0; i < MMAX - 1; ++i) {
        if (i < m - 1) {
            const T inv = T(1) / (bv[i] - av[i] * hp);
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
    // exchange (Y, Uc, V) with the segment to the right
    pA[tid] = Y;
    pB[tid] = Uc;
    pC[tid] = V;
    __syncthreads();
    T Ra = T(0), Rb = T(0), Rc = T(0), Rd = T(1);
    {
        const int base = q * seg_per_line;
        const int kr = (k + 1 == nseg) ? 0 : k + 1;
        const T Yp = pA[base + kr], Up = pB[base + kr], Vp = pC[base + kr];
        if (active) {
            Ra = ae * wp;
            Rb = be - ae * hp + ce * Up;
            Rc = ce * Vp;
            Rd = re - ae * gp - ce * Yp;
        } else {
            Ra = T(0); Rb = T(1); Rc = T(0); Rd = T(0);
        }
    }
    __syncthreads();
    // ---------------- cyclic reduction over the nseg interface unknowns
    {
        const int base = q * seg_per_line;
        pA[tid] = Ra; pB[tid] = Rb; pC[tid] = Rc; pD[tid] = Rd;
        __syncthreads();
        for (int s = 1; s < nseg; s <<= 1) {
            T na = Ra, nb = Rb, nc = Rc, nd = Rd;
            if (k < nseg) {
                const int km = base + ((k - s) & (nseg - 1));
                const int kp = base + ((k + s) & (nseg - 1));
                const T am = pA[km], bm = pB[km], cm = pC[km], dm = pD[km];
                const T ap = pA[kp], bp = pB[kp], cp = pC[kp], dp = pD[kp];
                const T k1 = Ra / bm, k2 = Rc / bp;
                na = -k1 * am;
                nc = -k2 * cp;
                nb = Rb - k1 * cm - k2 * ap;
                nd = Rd - k1 * dm - k2 * dp;
            }
            __syncthreads();
            Ra = na; Rb = nb; Rc = nc; Rd = nd;
            pA[tid] = Ra; pB[tid] = Rb; pC[tid] = Rc; pD[tid] = Rd;
            __syncthreads();
        }
    }
    const T XR = Rd / (Ra + Rb + Rc);
    pA[tid] = XR;
    __syncthreads();
    const T XL = pA[q * seg_per_line + ((k - 1) & (nseg - 1))];

    // ---------------- back substitution, result into LDS (reuse sU)
    double lsum = 0.0, lmin = __builtin_huge_val(), lmax = -__builtin_huge_val();
    if (active) {
        T* rowX = sU + q * LS;
        T xn = XR;
        rowX[lds_pad<T>(s0 + m - 1)] = XR;
        lsum = (double)XR;
        lmin = lmax = (double)XR;
#pragma unroll
        for (int i = MMAX - 2; i >= 0; --i) {
            if (i <= m - 2) {
                const T x = gv[i] - hv[i] * xn + wv[i] * XL;
                rowX[lds_pad<T>(s0 + i)] = x;
                xn = x;
                lsum += (double)x;
                lmin = fmin(lmin, (double)x);
                lmax = fmax(lmax, (double)x);
            }
        }
    }
    __syncthreads();

    // ---------------- phase 3: store the tile (transposed when out is t1-fastest)
    const bool line_fast_out = (P.so_t1 != 1);
    for (int idx = tid; idx < ncell; idx += nthreads) {
        int qq, p;
        if (line_fast_out) { qq = idx / n; p = idx - qq * n; }
        else { p = idx / lpw; qq = idx - p * lpw; }
        const int l1 = l1_0 + qq;
        if (l1 >= P.nt1) continue;
        const int64_t c = (int64_t)p * P.so_n + (int64_t)l1 * P.so_t1 + (int64_t)l2 * P.so_t2;
        P.out[c] = sU[qq * LS + lds_pad<T>(p)];
    }

    // ---------------- fused FP64 energy / min / max (deterministic)
    if (P.red.partials) block_reduce_and_finish(P.red, lsum, lmin, lmax);
}

template <typename T, int NDIM>
static hipError_t launch_sweep_dim(const SweepParams<T>& P, int mmax, dim3 grid, dim3 block, size_t lds,
                                   hipStream_t st) {
#define ASD_SWEEP_CASE(MM)                                           \
    case MM:                                                         \
        hipLaunchKernelGGL((sweep_kernel<T, NDIM, MM>), grid, block, lds, st, P); \
        return hipGetLastError();
    switch (mmax) {
        ASD_SWEEP_CASE(1)
        ASD_SWEEP_CASE(2)
        ASD_SWEEP_CASE(4)
        ASD_SWEEP_CASE(8)
        ASD_SWEEP_CASE(16)
        default: return hipErrorInvalidValue;
    }
#undef ASD_SWEEP_CASE
}

// Raise the dynamic-LDS limit of every sweep instantiation to the gfx950
// maximum.  Called once per process, before any launch or stream capture.
template <typename T, int NDIM>
static hipError_t set_attrs_dim(int bytes) {
    const void* fns[] = {(const void*)sweep_kernel<T, NDIM, 1>, (const void*)sweep_kernel<T, NDIM, 2>,
                         (const void*)sweep_kernel<T, NDIM, 4>, (const void*)sweep_kernel<T, NDIM, 8>,
                         (const void*)sweep_kernel<T, NDIM, 16>};
    for (const void* f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t sweep_set_lds_limits(int bytes) {
    hipError_t e = set_attrs_dim<float, 2>(bytes);
    if (e == hipSuccess) e = set_attrs_dim<float, 3>(bytes);
    if (e == hipSuccess) e = set_attrs_dim<double, 2>(bytes);
    if (e == hipSuccess) e = set_attrs_dim<double, 3>(bytes);
    return e;
}

template <typename T>
hipError_t launch_sweep(const SweepParams<T>& P, int ndim, int mmax, dim3 grid, dim3 block,
                        size_t lds, hipStream_t st) {
    if (ndim == 2) return launch_sweep_dim<T, 2>(P, mmax, grid, block, lds, st);
    return launch_sweep_dim<T, 3>(P, mmax, grid, block, lds, st);
}

template hipError_t launch_sweep<float>(const SweepParams<float>&, int, int, dim3, dim3, size_t,
                                        hipStream_t);
template hipError_t launch_sweep<double>(const SweepParams<double>&, int, int, dim3, dim3, size_t,
                                         hipStream_t);

}  // namespace asd
