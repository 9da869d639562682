// Explicit limited step (the time-step-limited baseline of sections 1 and
// 3): forward Euler of the same conservative operator, every face from T^n:
//
//   T^{n+1}_c = T^n_c + sum_d [ alpha_{c+1/2}(T_{c+e} - T_c) - alpha_{c-1/2}(T_c - T_{c-e})
//                               + F_{c+1/2} - F_{c-1/2} ]
//
// with alpha_f and F_f defined exactly as in the semi-implicit sweep (plus
// dt Q with a source).  T = 0 walls stage odd ghosts (-U, with the cell's b
// and chi) in the halo, so a wall face takes the normal flux
// alpha_w (-U_c - U_c) and a transverse flux that vanishes (the limited
// difference of a cell and its odd ghost is zero).
//
// gfx950 mapping: each wave owns a small block of cells, one column per
// lane (2-D: a band of rows; 3-D: rows x planes), loads it with a one-cell
// halo, and evaluates every face once (lane shifts across columns,
// registers across rows and planes).  No LDS staging.
#include "asd_device.h"
#include "asd_launch.h"

namespace asd {

// Neighbour coordinate with the boundary rule, in 32 bits (periodic wraps,
// walls clamp; the odd ghost's sign is applied by the caller).
__device__ __forceinline__ int nb_coord32(int c, int n, bool periodic) {
    if (c < 0) return periodic ? n - 1 : 0;
    if (c >= n) return periodic ? 0 : n - 1;
    return c;
}

// 2-D: one wave streams down a band of ExStream::TY rows of 64 columns
// (lane = column).  Lanes 0 and 63 hold the halo columns, so a wave updates
// the 62 columns between them; the row above and the row below the band
// are halo rows.  All loads of the band are issued first, in row order, so
// the first rows are updated while the later ones are still arriving.
// Every face is evaluated once: a cell's left x face is its left lane's
// right x face (a lane shift), its lower y face the upper y face of the
// previous row (kept in a register).  No LDS and no barrier (except the
// block's final reduction).
struct ExStream {
    static constexpr int COLS = 62;  // updated columns per wave
    static constexpr int TY = 4;     // rows per wave
    static constexpr int WAVES = 4;  // waves per block
};

// from_right: the value of lane+1 (the column to the right); from_left: that
// of lane-1.  The edge lanes receive values they never use.
template <typename T>
__device__ __forceinline__ T from_right(T v) { return __shfl_down(v, 1, 64); }
template <typename T>
__device__ __forceinline__ T from_left(T v) { return __shfl_up(v, 1, 64); }

template <typename T, int LIMC>
__global__ void __launch_bounds__(256) explicit_stream2d_kernel(ExplicitParams<T> P) {
    constexpr int TY = ExStream::TY, NR = TY + 2;  // rows y0-1 .. y0+TY
    const int nx = P.n[0], ny = P.n[1];
    const int lane = threadIdx.x & 63;
    // XCD-aware block order (the grid is a multiple of 8 blocks): bands that
    // share halo rows run on one XCD and share its L2
    const int blk = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    const int wave = blk * ExStream::WAVES + (threadIdx.x >> 6);
    const int ncb = (nx + ExStream::COLS - 1) / ExStream::COLS;
    const int nrb = (ny + TY - 1) / TY;
    double lsum = 0.0, lmin = __builtin_huge_val(), lmax = -__builtin_huge_val();
    if (wave < ncb * nrb) {  // wave-uniform
        const int cb = wave % ncb, rb = wave / ncb;
        const int x = cb * ExStream::COLS - 1 + lane;  // this lane's column (halo lanes may lie outside)
        const int y0 = rb * TY;
        const bool periodic = P.periodic != 0;
        const bool dir = P.dirichlet != 0;
        const int lim = LIMC >= 0 ? LIMC : P.limiter;
        const bool pchi = P.chi != nullptr || P.chi_exp != 0.0;
        const int xc = nb_coord32(x, nx, periodic);
        const bool xout = xc != x;
        // the band's rows: state (odd ghosts negated), b and chi
        T u[NR], bx[NR], by[NR], ch[NR], q[TY];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int y = y0 - 1 + r;
            const int yc = nb_coord32(y, ny, periodic);
            const unsigned c = (unsigned)xc + (unsigned)yc * (unsigned)nx;
            const T v = P.U[c];
            // odd ghost: one sign flip per axis on which the cell lies outside
            u[r] = dir && (xout != (yc != y)) ? -v : v;
            bx[r] = P.b[0][c];
            by[r] = P.b[1][c];
            ch[r] = P.chi ? P.chi[c] : P.chi_par;
            // chi(T): the cell's value from T^n, in FP64 (section 3.3)
            if (P.chi_exp != 0.0) ch[r] = (T)((double)P.chi_par * pow((double)v / P.chi_tref, P.chi_exp));
            if (r >= 1 && r <= TY && P.Q) q[r - 1] = P.Q[c];
        }
        const T cn0 = P.cn[0], cn1 = P.cn[1], ct01 = P.ct[0][1], ct10 = P.ct[1][0];
        const T chi_par = P.chi_par, chi_perp = P.chi_perp;
        auto face = [&](T u0, T u1, T bn0, T bn1, T bt0, T bt1, T c0, T c1, T s0, T s1, T cn, T ct) {
            // face between cells 0 and 1 along the normal axis: bn = normal
            // component of b, bt = transverse component, s = transverse slopes
            const T bnf = T(0.5) * (bn0 + bn1);
            const T chif = pchi ? harmonic<T>(c0, c1) : chi_par;
            const T dpar = chif - chi_perp;
            const T alpha = cn * (chi_perp + dpar * bnf * bnf);
            const T btf = T(0.5) * (bt0 + bt1);
            const T flux = dpar * bnf * (ct * btf * limit2<T>(lim, s1, s0));
            return alpha * (u1 - u0) + flux;
        };
        // slopes along x of a row (lane shifts), along y of a row (registers)
        auto slope_x = [&](T uc) { return cell_slope<T>(lim, from_left(uc), uc, from_right(uc)); };
        const bool xwall = !periodic && !dir && (x < 0 || x + 1 > nx - 1);  // this lane's right x face
        const bool out_col = lane >= 1 && lane <= ExStream::COLS && x < nx;
        // upper y face of row y0-1 (the lower face of the first row)
        T sx_prev = slope_x(u[0]);
        T sx_cur = slope_x(u[1]);
        T fy_low;
        {
            const bool ywall = !periodic && !dir && (y0 - 1 < 0 || y0 > ny - 1);
            fy_low = ywall ? T(0) : face(u[0], u[1], by[0], by[1], bx[0], bx[1], ch[0], ch[1], sx_prev, sx_cur, cn1, ct10);
        }
#pragma unroll
        for (int r = 1; r <= TY; ++r) {
            const int y = y0 - 1 + r;
            // x faces of row r: this lane's right face, and its left face from the left lane
            const T sy = cell_slope<T>(lim, u[r - 1], u[r], u[r + 1]);
            T fxr = face(u[r], from_right(u[r]), bx[r], from_right(bx[r]), by[r], from_right(by[r]), ch[r],
                         from_right(ch[r]), sy, from_right(sy), cn0, ct01);
            fxr = xwall ? T(0) : fxr;
            const T fxl = from_left(fxr);
            // upper y face of row r
            const T sx_next = slope_x(u[r + 1]);
            const bool ywall = !periodic && !dir && (y < 0 || y + 1 > ny - 1);
            T fyh = face(u[r], u[r + 1], by[r], by[r + 1], bx[r], bx[r + 1], ch[r], ch[r + 1], sx_cur, sx_next,
                         cn1, ct10);
            fyh = ywall ? T(0) : fyh;
            T acc = T(0);
            acc += -fxl;
            acc += fxr;
            acc += -fy_low;
            acc += fyh;
            if (out_col && y < ny) {
                const T uc = u[r];
                const T un = P.Q ? (uc + P.dtq * q[r - 1]) + acc : uc + acc;
                P.out[(unsigned)x + (unsigned)y * (unsigned)nx] = un;
                lsum += (double)un;
                lmin = fmin(lmin, (double)un);
                lmax = fmax(lmax, (double)un);
            }
            fy_low = fyh;
            sx_cur = sx_next;
        }
    }
    if (P.red.partials) block_partials(P.red.partials, lsum, lmin, lmax);
}

// 3-D: the same scheme as the 2-D streaming kernel, one wave per block of
// 62 columns x ExStream3<T>::TY rows x ExStream3<T>::TZ planes (lane =
// column).  A wave loads its block plus a one-cell halo on every side (all
// loads first, in plane order), evaluates every face once (x faces by a lane
// shift, y faces between rows and z faces between planes in registers) and
// updates its cells.  No LDS and no barrier apart from the final reduction.
template <typename T>
struct ExStream3 {
    static constexpr int COLS = 62;
    static constexpr int TY = 2;  // rows per wave
    static constexpr int TZ = 2;  // planes per wave
    static constexpr int WAVES = 4;
};

template <typename T, int LIMC>
__global__ void __launch_bounds__(256) explicit_stream3d_kernel(ExplicitParams<T> P) {
    using S = ExStream3<T>;
    constexpr int TY = S::TY, TZ = S::TZ, NR = TY + 2, NP = TZ + 2;
    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    const int lane = threadIdx.x & 63;
    const int blk = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);  // XCD-aware order
    const int wave = blk * S::WAVES + (threadIdx.x >> 6);
    const int ncb = (nx + S::COLS - 1) / S::COLS, nrb = (ny + TY - 1) / TY, nzb = (nz + TZ - 1) / TZ;
    double lsum = 0.0, lmin = __builtin_huge_val(), lmax = -__builtin_huge_val();
    if (wave < ncb * nrb * nzb) {  // wave-uniform
        const int cb = wave % ncb, rb = (wave / ncb) % nrb, zb = wave / (ncb * nrb);
        const int x = cb * S::COLS - 1 + lane;
        const int y0 = rb * TY, z0 = zb * TZ;
        const bool periodic = P.periodic != 0;
        const bool dir = P.dirichlet != 0;
        const int lim = LIMC >= 0 ? LIMC : P.limiter;
        const bool pchi = P.chi != nullptr || P.chi_exp != 0.0;
        const int xc = nb_coord32(x, nx, periodic);
        const bool xout = xc != x;
        const unsigned sy = (unsigned)nx, sz = (unsigned)nx * (unsigned)ny;
        // the block and its halo: plane q is z0-1+q, row r is y0-1+r
        T u[NP][NR], bx[NP][NR], by[NP][NR], bz[NP][NR], ch[NP][NR], q[TZ][TY];
#pragma unroll
        for (int pq = 0; pq < NP; ++pq) {
            const int z = z0 - 1 + pq;
            const int zc = nb_coord32(z, nz, periodic);
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const int y = y0 - 1 + r;
                const int yc = nb_coord32(y, ny, periodic);
                const unsigned c = (unsigned)xc + (unsigned)yc * sy + (unsigned)zc * sz;
                const T v = P.U[c];
                // odd ghost: one sign flip per axis on which the cell lies outside
                const int nout = (int)xout + (int)(yc != y) + (int)(zc != z);
                u[pq][r] = dir && (nout & 1) ? -v : v;
                bx[pq][r] = P.b[0][c];
                by[pq][r] = P.b[1][c];
                bz[pq][r] = P.b[2][c];
                ch[pq][r] = P.chi ? P.chi[c] : P.chi_par;
                // chi(T): the cell's value from T^n, in FP64 (section 3.3)
                if (P.chi_exp != 0.0) ch[pq][r] = (T)((double)P.chi_par * pow((double)v / P.chi_tref, P.chi_exp));
                if (P.Q && pq >= 1 && pq <= TZ && r >= 1 && r <= TY) q[pq - 1][r - 1] = P.Q[c];
            }
        }
        const T chi_par = P.chi_par, chi_perp = P.chi_perp;
        // face between cells 0 and 1 along the normal axis n; a and b are the
        // two transverse axes in increasing order (components ta, tb of b,
        // limited slopes sa, sb)
        auto face = [&](T u0, T u1, T bn0, T bn1, T ta0, T ta1, T tb0, T tb1, T c0, T c1, T sa0, T sa1, T sb0,
                        T sb1, T cn, T cta, T ctb) {
            const T bnf = T(0.5) * (bn0 + bn1);
            const T chif = pchi ? harmonic<T>(c0, c1) : chi_par;
            const T dpar = chif - chi_perp;
            const T alpha = cn * (chi_perp + dpar * bnf * bnf);
            T tr = T(0);
            tr += cta * (T(0.5) * (ta0 + ta1)) * limit2<T>(lim, sa1, sa0);
            tr += ctb * (T(0.5) * (tb0 + tb1)) * limit2<T>(lim, sb1, sb0);
            const T flux = dpar * bnf * tr;
            return alpha * (u1 - u0) + flux;
        };
        // limited slopes: along x for every loaded cell (lane shifts), along
        // y for the inner rows, along z for the inner planes
        T sxs[NP][NR], sys[NP][NR], szs[NP][NR];
#pragma unroll
        for (int pq = 0; pq < NP; ++pq) {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                sxs[pq][r] = cell_slope<T>(lim, from_left(u[pq][r]), u[pq][r], from_right(u[pq][r]));
                sys[pq][r] = (r >= 1 && r <= TY) ? cell_slope<T>(lim, u[pq][r - 1], u[pq][r], u[pq][r + 1]) : T(0);
                szs[pq][r] = (pq >= 1 && pq <= TZ) ? cell_slope<T>(lim, u[pq - 1][r], u[pq][r], u[pq + 1][r]) : T(0);
            }
        }
        const bool xwall = !periodic && !dir && (x < 0 || x + 1 > nx - 1);
        const bool out_col = lane >= 1 && lane <= S::COLS && x < nx;
        // lower z faces of the first plane
        T fz_lo[TY];
        {
            const bool zwall = !periodic && !dir && (z0 - 1 < 0 || z0 > nz - 1);
#pragma unroll
            for (int r = 1; r <= TY; ++r) {
                const T f = face(u[0][r], u[1][r], bz[0][r], bz[1][r], bx[0][r], bx[1][r], by[0][r], by[1][r], ch[0][r],
                                 ch[1][r], sxs[0][r], sxs[1][r], sys[0][r], sys[1][r], P.cn[2], P.ct[2][0], P.ct[2][1]);
                fz_lo[r - 1] = zwall ? T(0) : f;
            }
        }
#pragma unroll
        for (int pq = 1; pq <= TZ; ++pq) {
            const int z = z0 - 1 + pq;
            // y faces of this plane, rows r and r+1, r = 0 .. TY
            T fy[TY + 1];
#pragma unroll
            for (int r = 0; r <= TY; ++r) {
                const int y = y0 - 1 + r;
                const bool ywall = !periodic && !dir && (y < 0 || y + 1 > ny - 1);
                const T f = face(u[pq][r], u[pq][r + 1], by[pq][r], by[pq][r + 1], bx[pq][r], bx[pq][r + 1], bz[pq][r],
                                 bz[pq][r + 1], ch[pq][r], ch[pq][r + 1], sxs[pq][r], sxs[pq][r + 1], szs[pq][r],
                                 szs[pq][r + 1], P.cn[1], P.ct[1][0], P.ct[1][2]);
                fy[r] = ywall ? T(0) : f;
            }
            const bool zwall = !periodic && !dir && (z < 0 || z + 1 > nz - 1);
#pragma unroll
            for (int r = 1; r <= TY; ++r) {
                const int y = y0 - 1 + r;
                T fxr = face(u[pq][r], from_right(u[pq][r]), bx[pq][r], from_right(bx[pq][r]), by[pq][r],
                             from_right(by[pq][r]), bz[pq][r], from_right(bz[pq][r]), ch[pq][r], from_right(ch[pq][r]),
                             sys[pq][r], from_right(sys[pq][r]), szs[pq][r], from_right(szs[pq][r]), P.cn[0],
                             P.ct[0][1], P.ct[0][2]);
                fxr = xwall ? T(0) : fxr;
                const T fxl = from_left(fxr);
                T fzh = face(u[pq][r], u[pq + 1][r], bz[pq][r], bz[pq + 1][r], bx[pq][r], bx[pq + 1][r], by[pq][r],
                             by[pq + 1][r], ch[pq][r], ch[pq + 1][r], sxs[pq][r], sxs[pq + 1][r], sys[pq][r],
                             sys[pq + 1][r], P.cn[2], P.ct[2][0], P.ct[2][1]);
                fzh = zwall ? T(0) : fzh;
                T acc = T(0);
                acc += -fxl;
                acc += fxr;
                acc += -fy[r - 1];
                acc += fy[r];
                acc += -fz_lo[r - 1];
                acc += fzh;
                if (out_col && y < ny && z < nz) {
                    const T uc = u[pq][r];
                    const T un = P.Q ? (uc + P.dtq * q[pq - 1][r - 1]) + acc : uc + acc;
                    P.out[(unsigned)x + (unsigned)y * sy + (unsigned)z * sz] = un;
                    lsum += (double)un;
                    lmin = fmin(lmin, (double)un);
                    lmax = fmax(lmax, (double)un);
                }
                fz_lo[r - 1] = fzh;
            }
        }
    }
    if (P.red.partials) block_partials(P.red.partials, lsum, lmin, lmax);
}

// Blocks of an explicit launch: a multiple of 8 for the XCD-aware order.
template <typename T>
static int explicit_blocks_t(int ndim, const int n[3]) {
    int waves, per_block;
    if (ndim == 2) {
        waves = ((n[0] + ExStream::COLS - 1) / ExStream::COLS) * ((n[1] + ExStream::TY - 1) / ExStream::TY);
        per_block = ExStream::WAVES;
    } else {
        using S = ExStream3<T>;
        waves = ((n[0] + S::COLS - 1) / S::COLS) * ((n[1] + S::TY - 1) / S::TY) * ((n[2] + S::TZ - 1) / S::TZ);
        per_block = S::WAVES;
    }
    const int blocks = (waves + per_block - 1) / per_block;
    return (blocks + 7) & ~7;
}

// The larger of the two precisions' block counts (sizes the reduction scratch).
int explicit_num_blocks(int ndim, const int n[3]) {
    const int a = explicit_blocks_t<float>(ndim, n), b = explicit_blocks_t<double>(ndim, n);
    return a > b ? a : b;
}

template <typename T>
hipError_t launch_explicit(const ExplicitParams<T>& P, int ndim, hipStream_t st, int* nblocks_out) {
    const int nb = explicit_blocks_t<T>(ndim, P.n);
    if (nblocks_out) *nblocks_out = nb;
    const bool vl = P.limiter == LIM_VANLEER;
    if (ndim == 2) {
        constexpr int NT = 64 * ExStream::WAVES;
        if (vl) hipLaunchKernelGGL((explicit_stream2d_kernel<T, LIM_VANLEER>), dim3(nb), dim3(NT), 0, st, P);
        else hipLaunchKernelGGL((explicit_stream2d_kernel<T, -1>), dim3(nb), dim3(NT), 0, st, P);
    } else {
        constexpr int NT = 64 * ExStream3<T>::WAVES;
        if (vl) hipLaunchKernelGGL((explicit_stream3d_kernel<T, LIM_VANLEER>), dim3(nb), dim3(NT), 0, st, P);
        else hipLaunchKernelGGL((explicit_stream3d_kernel<T, -1>), dim3(nb), dim3(NT), 0, st, P);
    }
    return hipGetLastError();
}

template hipError_t launch_explicit<float>(const ExplicitParams<float>&, int, hipStream_t, int*);
template hipError_t launch_explicit<double>(const ExplicitParams<double>&, int, hipStream_t, int*);

}  // namespace asd
