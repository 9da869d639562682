// Reverse mode of one directional sweep (2-D).
//
// Forward sweep along axis d (section 2, Eq. xup / yup):
//     x = A_d^-1 (U + S_d(U)),   A_d = I + sum_f alpha_f (e_c - e_c')(e_c - e_c')^T,
//     S_d(U)_c = F_{c+1/2} - F_{c-1/2},  F_f = beta_f G_f(U),
//     G_f = L(sigma_c', sigma_c),  sigma_c = L(U[c+e_t] - U[c], U[c] - U[c-e_t]),
// with c' = c + e_d.  Given mu = A_d^-1 lambda (A_d is symmetric, so the
// same line solver gives it), the input adjoint is
//     lambda_U = mu + J_S(U)^T mu,
// and the face parameters receive
//     dL/dalpha_f = -(mu_c - mu_c') (x_c - x_c'),   dL/dbeta_f = (mu_c - mu_c') G_f,
// chained to the face diffusivity (alpha, beta are linear in chi_f) and
// through the harmonic mean to the two cells' chi.
//
// One fused gather kernel per sweep axis, no atomics: per face, the weights
// w_f dG/dsigma (w_f = beta_f (mu_c - mu_c')) and dL/dchi_f; per cell, the
// contributions of its own slope and of the slopes of its two transverse
// neighbours, and its two faces' chi terms.
// Arithmetic is in the storage precision; arrays are x-fastest ("layout
// A"), except that lambda may be written y-fastest ("layout B", the y
// sweep's input layout).
// Limiter derivatives: zero where a*b <= 0 (kinks included); minmod takes
// its first argument on |a| == |b|; MC takes 2a, then 2b, then (a+b)/2.
#include "asd_device.h"
#include "asd_launch.h"

namespace asd {

// value and partial derivatives of the two-argument limiter (van Leer's
// quotients through a refined reciprocal, as in the forward sweeps), without
// branches: every candidate is formed and the result selected.  LIMC >= 0
// fixes the limiter at compile time; -1 reads lim.
template <int LIMC, typename C>
__device__ __forceinline__ C dlim2(int lim_rt, C a, C b, C* d1, C* d2) {
    const int lim = LIMC >= 0 ? LIMC : lim_rt;
    if (lim == LIM_LINEAR) {
        *d1 = C(0.5);
        *d2 = C(0.5);
        return C(0.5) * (a + b);
    }
    const bool pos = a * b > C(0.0);
    C v, g1, g2;
    if (lim == LIM_VANLEER) {
        // a + b != 0 wherever the result is used (a, b of one sign)
        const C r = fast_rcp<C>(a + b), r2 = r * r;
        g1 = C(2.0) * b * b * r2;
        g2 = C(2.0) * a * a * r2;
        v = C(2.0) * a * b * r;
    } else if (lim == LIM_MINMOD) {
        const bool first = fabs(a) <= fabs(b);
        v = first ? a : b;
        g1 = first ? C(1.0) : C(0.0);
        g2 = first ? C(0.0) : C(1.0);
    } else {  // MC
        const bool first = fabs(C(2.0) * a) <= fabs(C(2.0) * b);
        const C m = first ? C(2.0) * a : C(2.0) * b;
        const C mean = C(0.5) * (a + b);
        const bool use_m = fabs(m) <= fabs(mean);
        v = use_m ? m : mean;
        g1 = use_m ? (first ? C(2.0) : C(0.0)) : C(0.5);
        g2 = use_m ? (first ? C(0.0) : C(2.0)) : C(0.5);
    }
    *d1 = pos ? g1 : C(0.0);
    *d2 = pos ? g2 : C(0.0);
    return pos ? v : C(0.0);
}

// ------------------------------------------------ fused streaming kernels
// One wave per band of 64 columns (lane = column, halo lanes at the band's
// edges) and a strip of AdjStream::RS rows: the strip's inputs are loaded
// at once (one memory latency per wave), then walked row by row: each row's
// face quantities are formed once and kept in registers while the rows
// above and below need them; neighbours across columns come by DPP lane
// rotations.
struct AdjStream {
    static constexpr int RS = 4;     // rows per wave
    static constexpr int WAVES = 4;  // waves per block
};

// lane i takes v of lane i+1 / i-1 (rotations of the whole wave: the lanes
// that wrap are halo lanes, whose results are discarded)
template <typename C>
__device__ __forceinline__ C lane_from_right(C v) { return dpp_mov<0x134, 0xf>(v, v); }
template <typename C>
__device__ __forceinline__ C lane_from_left(C v) { return dpp_mov<0x13C, 0xf>(v, v); }

// Coordinate c of a cell up to two cells outside [0, n): periodic wrap or
// insulating clamp.  Halo lanes farther out hold values no updated cell
// uses; they are clamped to a valid index.
__device__ __forceinline__ int adj_nb(int c, int n, bool periodic) {
    if (c < 0) return periodic && c + n >= 0 ? c + n : 0;
    if (c >= n) return periodic && c - n < n ? c - n : n - 1;
    return c;
}

// Face quantities between cells 0 and 1 along the face normal: weights to
// the slopes of cell 1 (W1) and cell 0 (W2), and dL/dchi_f (GF).
template <typename T, int LIMC>
__device__ __forceinline__ void adj_face(const AdjParams<T>& P, T s0, T s1, T bn0, T bn1, T bt0, T bt1, T c0, T c1,
                                         T mu0, T mu1, T x0, T x1, T& W1, T& W2, T& GF) {
    T LG1, LG2;
    const T Gf = dlim2<LIMC, T>(P.limiter, s1, s0, &LG1, &LG2);
    const T bn = T(0.5) * (bn0 + bn1);
    const T bt = T(0.5) * (bt0 + bt1);
    T chif = (T)P.chi_par;
    if (P.chi) chif = (c0 + c1) != T(0) ? T(2) * c0 * c1 * fast_rcp<T>(c0 + c1) : T(0);
    const T dpar = chif - (T)P.chi_perp;
    const T kbt = (T)P.kb * bn * bt;
    const T dm = mu0 - mu1;
    const T w = kbt * dpar * dm;
    W1 = w * LG1;
    W2 = w * LG2;
    const T dLdalpha = -dm * (x0 - x1);
    const T dLdbeta = dm * Gf;
    GF = dLdalpha * (T)P.ka * bn * bn + dLdbeta * kbt;
}

// d/dchi of the harmonic face mean, times the face's dL/dchi_f
template <typename C>
__device__ __forceinline__ C adj_chi_term(C gf, C cj, C co) {
    const C s = cj + co;
    const C r = fast_rcp<C>(s);
    const C v = gf * C(2) * co * co * (r * r);
    return s == C(0) ? C(0) : v;
}

// The raw loads of one cell row.
template <typename T>
struct AdjRaw {
    T mu, X, bn, bt, ch;
};
// Element c of a (uniform) base array through a 32-bit byte offset: the
// load takes the scalar base and one lane offset register, without 64-bit
// address arithmetic per load (arrays stay below 4 GiB).
template <typename T>
__device__ __forceinline__ T ld32(const T* base, unsigned c) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + c * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ AdjRaw<T> adj_load(const AdjParams<T>& P, unsigned c, int dn) {
    AdjRaw<T> r;
    r.mu = ld32(P.mu, c);
    r.X = ld32(P.X, c);
    r.bn = ld32(P.b[dn], c);
    r.bt = ld32(P.b[1 - dn], c);
    r.ch = P.chi ? ld32(P.chi, c) : T(0);
    return r;
}

template <typename T>
__device__ __forceinline__ void adj_store(const AdjParams<T>& P, int x, int y, T acc, T g) {
    const unsigned j = (unsigned)(x + y * P.nx);
    P.lam_out[P.lam_b ? (unsigned)(x * P.ny + y) : j] = acc;
    if (P.gchi) P.gchi[j] += g;
}

// Faces along x (d = 0), slopes along y: a wave updates the 62 columns
// between its halo lanes.  Row y's face quantities need the slope of cell
// (x, y) along y (U of rows y-1 .. y+1); its update needs those of rows
// y-1 .. y+1.
template <typename T, int LIMC>
__global__ void __launch_bounds__(256) adj_stream_x_kernel(AdjParams<T> P) {
    constexpr int RS = AdjStream::RS;
    const int nx = P.nx, ny = P.ny;
    const int lane = threadIdx.x & 63;
    const int blk = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    // wave-uniform (readfirstlane): the row arithmetic stays scalar
    const int wave = blk * AdjStream::WAVES + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int ncb = (nx + 61) / 62, nrs = (ny + RS - 1) / RS;
    if (wave >= ncb * nrs) return;  // wave-uniform; no block barrier follows
    const int cb = wave % ncb, ys = (wave / ncb) * RS;
    const int x = cb * 62 - 1 + lane;
    const bool periodic = P.periodic != 0;
    const int xc = adj_nb(x, nx, periodic);
    const bool right_face = periodic || x + 1 <= nx - 1;  // face (x, x+1) lies inside
    const bool left_face = periodic || x - 1 >= 0;        // face (x-1, x) lies inside
    const bool out_lane = lane >= 1 && lane <= 62 && x < nx;
    const int lim = P.limiter;

    // one row's face quantities (all lanes take part: lane rotations)
    struct Row {
        T psi, l1, l2, mu, ch, chr, chl, gfr, gfl;
    };
    auto face_row = [&](T um, T uc, T up, const AdjRaw<T>& r) {
        Row o;
        const T sg = dlim2<LIMC, T>(lim, up - uc, uc - um, &o.l1, &o.l2);
        o.mu = r.mu;
        o.ch = P.chi ? r.ch : (T)P.chi_par;
        const T X = r.X, bn = r.bn, bt = r.bt;
        o.chr = lane_from_right(o.ch);
        T W1, W2, GF;
        adj_face<T, LIMC>(P, sg, lane_from_right(sg), bn, lane_from_right(bn), bt, lane_from_right(bt), o.ch, o.chr, o.mu,
                    lane_from_right(o.mu), X, lane_from_right(X), W1, W2, GF);
        if (!right_face) { W1 = T(0); W2 = T(0); GF = T(0); }
        const T W1l = lane_from_left(W1);
        o.psi = W2 + (left_face ? W1l : T(0));
        o.gfr = GF;
        o.gfl = lane_from_left(GF);
        o.chl = lane_from_left(o.ch);
        return o;
    };
    auto row_at = [&](int y) { return (unsigned)(xc + adj_nb(y, ny, periodic) * nx); };

    // the strip's inputs, all loads in flight at once: U of rows ys-2 ..
    // ys+RS+1, the other fields of rows ys-1 .. ys+RS
    T ub[RS + 4];
    AdjRaw<T> rb[RS + 2];
#pragma unroll
    for (int i = 0; i < RS + 4; ++i) ub[i] = ld32(P.U, row_at(ys - 2 + i));
#pragma unroll
    for (int i = 0; i < RS + 2; ++i) rb[i] = adj_load<T>(P, row_at(ys - 1 + i), 0);
    Row prev = face_row(ub[0], ub[1], ub[2], rb[0]);
    Row cur = face_row(ub[1], ub[2], ub[3], rb[1]);
#pragma unroll
    for (int r = 0; r < RS; ++r) {
        // rows past ny (last strip) are computed from clamped or wrapped
        // loads and not stored
        const int y = ys + r;
        const Row next = face_row(ub[r + 2], ub[r + 3], ub[r + 4], rb[r + 2]);
        // mirrored neighbours at insulating walls: the clamped loads give U_c
        const bool us = !periodic && y + 1 > ny - 1, ds = !periodic && y - 1 < 0;
        if (out_lane && y < ny) {
            T acc = cur.mu + cur.psi * ((us ? T(0) : -cur.l1) + (ds ? T(0) : cur.l2));
            if (periodic || y - 1 >= 0) acc += prev.psi * prev.l1;
            if (periodic || y + 1 <= ny - 1) acc -= next.psi * next.l2;
            T g = T(0);
            if (P.gchi) {
                if (right_face) g += adj_chi_term(cur.gfr, cur.ch, cur.chr);
                if (left_face) g += adj_chi_term(cur.gfl, cur.ch, cur.chl);
            }
            adj_store<T>(P, x, y, acc, g);
        }
        prev = cur;
        cur = next;
    }
}

// Faces along y (d = 1), slopes along x: a wave updates the 60 columns
// between two halo lanes on each side (an updated cell needs the slopes of
// its left and right neighbours, which need their own neighbours).  Row y's
// update needs the faces (y-1, y) and (y, y+1).
template <typename T, int LIMC>
__global__ void __launch_bounds__(256) adj_stream_y_kernel(AdjParams<T> P) {
    constexpr int RS = AdjStream::RS;
    const int nx = P.nx, ny = P.ny;
    const int lane = threadIdx.x & 63;
    const int blk = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    // wave-uniform (readfirstlane): the row arithmetic stays scalar
    const int wave = blk * AdjStream::WAVES + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int ncb = (nx + 59) / 60, nrs = (ny + RS - 1) / RS;
    if (wave >= ncb * nrs) return;  // wave-uniform; no block barrier follows
    const int cb = wave % ncb, ys = (wave / ncb) * RS;
    const int x = cb * 60 - 2 + lane;
    const bool periodic = P.periodic != 0;
    const int xc = adj_nb(x, nx, periodic);
    // mirrored neighbours at insulating walls: the clamped loads give U_c
    const bool us = !periodic && x + 1 > nx - 1, ds = !periodic && x - 1 < 0;
    const bool out_lane = lane >= 2 && lane <= 61 && x < nx;
    const int lim = P.limiter;

    struct Row {
        T sg, l1, l2, mu, X, bn, bt, ch;
    };
    auto make_row = [&](T u_raw, const AdjRaw<T>& r) {
        Row o;
        const T u = u_raw;
        const T ur = lane_from_right(u), ul = lane_from_left(u);
        o.sg = dlim2<LIMC, T>(lim, ur - u, u - ul, &o.l1, &o.l2);
        o.mu = r.mu;
        o.X = r.X;
        o.bn = r.bn;
        o.bt = r.bt;
        o.ch = P.chi ? r.ch : (T)P.chi_par;
        return o;
    };
    // face between rows y and y+1 (a, b): W1 to b's slope, W2 to a's
    auto face = [&](int y, const Row& a, const Row& b, T& W1, T& W2, T& GF) {
        adj_face<T, LIMC>(P, a.sg, b.sg, a.bn, b.bn, a.bt, b.bt, a.ch, b.ch, a.mu, b.mu, a.X, b.X, W1, W2, GF);
        if (!(periodic || (y >= 0 && y + 1 <= ny - 1))) { W1 = T(0); W2 = T(0); GF = T(0); }
    };
    auto row_at = [&](int y) { return (unsigned)(xc + adj_nb(y, ny, periodic) * nx); };

    // the strip's inputs, rows ys-1 .. ys+RS, all loads in flight at once
    T ub[RS + 2];
    AdjRaw<T> rb[RS + 2];
#pragma unroll
    for (int i = 0; i < RS + 2; ++i) {
        ub[i] = ld32(P.U, row_at(ys - 1 + i));
        rb[i] = adj_load<T>(P, row_at(ys - 1 + i), 1);
    }
    Row A = make_row(ub[0], rb[0]);
    Row B = make_row(ub[1], rb[1]);
    T W1p, W2p, GFp;  // face (ys-1, ys)
    face(ys - 1, A, B, W1p, W2p, GFp);
#pragma unroll
    for (int r = 0; r < RS; ++r) {
        const int y = ys + r;  // rows past ny (last strip): computed, not stored
        const Row C = make_row(ub[r + 2], rb[r + 2]);
        T W1, W2, GF;
        face(y, B, C, W1, W2, GF);
        const T psi = W2 + ((periodic || y - 1 >= 0) ? W1p : T(0));
        const T from_l = lane_from_left(psi * B.l1);   // psi(x-1) d sigma(x-1)/dp
        const T from_r = lane_from_right(psi * B.l2);  // psi(x+1) d sigma(x+1)/dq
        if (out_lane && y < ny) {
            T acc = B.mu + psi * ((us ? T(0) : -B.l1) + (ds ? T(0) : B.l2));
            if (periodic || x - 1 >= 0) acc += from_l;
            if (periodic || x + 1 <= nx - 1) acc -= from_r;
            T g = T(0);
            if (P.gchi) {
                if (periodic || y + 1 <= ny - 1) g += adj_chi_term(GF, B.ch, C.ch);
                if (periodic || y - 1 >= 0) g += adj_chi_term(GFp, B.ch, A.ch);
            }
            adj_store<T>(P, x, y, acc, g);
        }
        W1p = W1;
        GFp = GF;
        A = B;
        B = C;
    }
    (void)W2p;
}

template <typename T>
hipError_t launch_adjoint_stencil(const AdjParams<T>& P, hipStream_t st) {
    const int cols = P.d == 0 ? 62 : 60;
    const long waves = (long)((P.nx + cols - 1) / cols) * ((P.ny + AdjStream::RS - 1) / AdjStream::RS);
    long nb = (waves + AdjStream::WAVES - 1) / AdjStream::WAVES;
    nb = (nb + 7) & ~7L;  // a multiple of 8 for the XCD-aware block order
    const dim3 grid((unsigned)nb), block(64 * AdjStream::WAVES);
    const bool vl = P.limiter == LIM_VANLEER;
    if (P.d == 0) {
        if (vl) hipLaunchKernelGGL((adj_stream_x_kernel<T, LIM_VANLEER>), grid, block, 0, st, P);
        else hipLaunchKernelGGL((adj_stream_x_kernel<T, -1>), grid, block, 0, st, P);
    } else {
        if (vl) hipLaunchKernelGGL((adj_stream_y_kernel<T, LIM_VANLEER>), grid, block, 0, st, P);
        else hipLaunchKernelGGL((adj_stream_y_kernel<T, -1>), grid, block, 0, st, P);
    }
    return hipGetLastError();
}

template hipError_t launch_adjoint_stencil<float>(const AdjParams<float>&, hipStream_t);
template hipError_t launch_adjoint_stencil<double>(const AdjParams<double>&, hipStream_t);

}  // namespace asd
