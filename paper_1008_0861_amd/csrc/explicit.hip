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
// gfx950 mapping.  2-D: each wave streams down a short band of rows, one
// column per lane, with every face evaluated once (explicit_stream2d_kernel).
// 3-D (explicit3d_kernel): one workgroup per tile of TX x TY x TZ cells; the tile plus a
// one-cell halo of U, b (and chi) is staged through LDS with coalesced loads,
// the limited cell slopes along every axis are computed once per staged cell,
// and each thread then updates its cells.
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

// 3-D tile of TX x TY x TZ cells with a one-cell halo, NT threads; each
// thread updates NC / NT cells.  32 x 4 x 2 keeps the FP64 tile within 64 KB
// of LDS.
struct ExTile {
    static constexpr int TX = 32, TY = 4, TZ = 2;
    static constexpr int BX = TX + 2, BY = TY + 2, BZ = TZ + 2;
    static constexpr int NB = BX * BY * BZ;
    static constexpr int NC = TX * TY * TZ;
    static constexpr int NT = 256;
};

// 3-D grids.  LIMC: the limiter as a compile-time constant (van Leer, the
// default), or -1 to read it from the parameters.
template <typename T, int LIMC>
__global__ void __launch_bounds__(256) explicit3d_kernel(ExplicitParams<T> P) {
    constexpr int NDIM = 3;
    using TL = ExTile;
    __shared__ T sU[TL::NB];
    __shared__ T sB[NDIM][TL::NB];
    __shared__ T sS[NDIM][TL::NB];  // limited slope along each axis
    __shared__ T sChi[TL::NB];

    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    const int gx = (nx + TL::TX - 1) / TL::TX, gy = (ny + TL::TY - 1) / TL::TY;
    int blk = blockIdx.x;
    const int x0 = (blk % gx) * TL::TX;
    blk /= gx;
    const int y0 = (blk % gy) * TL::TY;
    const int z0 = (blk / gy) * TL::TZ;
    const bool periodic = P.periodic != 0;
    const bool dir = P.dirichlet != 0;
    const int lim = LIMC >= 0 ? LIMC : P.limiter;
    // cell indices fit 32 bits (grids hold fewer than 2^31 cells)
    const unsigned sy = (unsigned)nx, sz = (unsigned)nx * (unsigned)ny;

    // stage the box [x0-1, x0+TX] x [y0-1, y0+TY] (x [z0-1, z0+TZ]); all of a
    // thread's loads are issued before any is stored to LDS
    constexpr int IT = (TL::NB + TL::NT - 1) / TL::NT;
    {
        T vu[IT], vb[NDIM][IT], vc[IT];
        bool vneg[IT];
#pragma unroll
        for (int j = 0; j < IT; ++j) {
            const int i = threadIdx.x + j * TL::NT;
            const int ii = i < TL::NB ? i : 0;
            const int bx = ii % TL::BX, by = (ii / TL::BX) % TL::BY, bz = ii / (TL::BX * TL::BY);
            // cells beyond the far edge of a partial tile map to valid cells (never used)
            const int gx0 = x0 - 1 + bx, gy0 = y0 - 1 + by, gz0 = z0 - 1 + bz;
            const int x = nb_coord32(gx0, nx, periodic);
            const int y = nb_coord32(gy0, ny, periodic);
            const int z = NDIM == 3 ? nb_coord32(gz0, nz, periodic) : 0;
            const unsigned c = (unsigned)x + (unsigned)y * sy + (unsigned)z * sz;
            // odd ghost: one sign flip per axis on which the cell lies outside
            const int nout = (x != gx0) + (y != gy0) + (NDIM == 3 && z != gz0);
            vneg[j] = dir && (nout & 1);
            vu[j] = P.U[c];
#pragma unroll
            for (int d = 0; d < NDIM; ++d) vb[d][j] = P.b[d][c];
            if (P.chi) vc[j] = P.chi[c];
        }
#pragma unroll
        for (int j = 0; j < IT; ++j) {
            const int i = threadIdx.x + j * TL::NT;
            if (i >= TL::NB) continue;
            sU[i] = vneg[j] ? -vu[j] : vu[j];
#pragma unroll
            for (int d = 0; d < NDIM; ++d) sB[d][i] = vb[d][j];
            if (P.chi) sChi[i] = vc[j];
            // chi(T): the cell's value from T^n, in FP64 (section 3.3)
            if (P.chi_exp != 0.0) sChi[i] = (T)((double)P.chi_par * pow((double)vu[j] / P.chi_tref, P.chi_exp));
        }
    }
    __syncthreads();
    const int bstr[3] = {1, TL::BX, TL::BX * TL::BY};
    const int bdim[3] = {TL::BX, TL::BY, TL::BZ};
    for (int i = threadIdx.x; i < TL::NB; i += blockDim.x) {
        const int bc[3] = {i % TL::BX, (i / TL::BX) % TL::BY, i / (TL::BX * TL::BY)};
#pragma unroll
        for (int d = 0; d < NDIM; ++d) {
            T s = T(0);
            if (bc[d] > 0 && bc[d] < bdim[d] - 1)
                s = cell_slope<T>(lim, sU[i - bstr[d]], sU[i], sU[i + bstr[d]]);
            sS[d][i] = s;
        }
    }
    __syncthreads();

    double lsum = 0.0, lmin = __builtin_huge_val(), lmax = -__builtin_huge_val();
#pragma unroll
    for (int cc = threadIdx.x; cc < TL::NC; cc += TL::NT) {
    const int tx = cc % TL::TX, ty = (cc / TL::TX) % TL::TY, tz = cc / (TL::TX * TL::TY);
    const int x = x0 + tx, y = y0 + ty, z = z0 + tz;
    const bool inside = x < nx && y < ny && (NDIM == 2 || z < nz);
    if (inside) {
        const int bi = (tx + 1) + (ty + 1) * TL::BX + (NDIM == 3 ? (tz + 1) * TL::BX * TL::BY : 0);
        const int gc[3] = {x, y, z};
        const T uc = sU[bi];
        T acc = T(0);
#pragma unroll
        for (int d = 0; d < NDIM; ++d) {
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                // face between cells c0 = (side ? c : c - e_d) and c1 = c0 + e_d
                const int i0 = side ? bi : bi - bstr[d];
                const int i1 = i0 + bstr[d];
                const int g0 = side ? gc[d] : gc[d] - 1;
                const bool wall = !periodic && !dir && (g0 < 0 || g0 + 1 > P.n[d] - 1);
                if (wall) continue;
                const T bnf = T(0.5) * (sB[d][i0] + sB[d][i1]);
                T chif = P.chi_par;
                if (P.chi || P.chi_exp != 0.0) chif = harmonic<T>(sChi[i0], sChi[i1]);
                const T dpar = chif - P.chi_perp;
                const T alpha = P.cn[d] * (P.chi_perp + dpar * bnf * bnf);
                T tr = T(0);
#pragma unroll
                for (int t = 0; t < NDIM; ++t) {
                    if (t == d) continue;
                    const T btf = T(0.5) * (sB[t][i0] + sB[t][i1]);
                    tr += P.ct[d][t] * btf * limit2<T>(lim, sS[t][i1], sS[t][i0]);
                }
                const T flux = dpar * bnf * tr;
                const T diff = sU[i1] - sU[i0];
                // the face adds +(alpha diff + F) to c0 and -(..) to c1
                acc += side ? (alpha * diff + flux) : -(alpha * diff + flux);
            }
        }
        const unsigned co = (unsigned)x + (unsigned)y * sy + (unsigned)z * sz;
        const T un = P.Q ? (uc + P.dtq * P.Q[co]) + acc : uc + acc;
        P.out[co] = un;
        lsum += (double)un;
        lmin = fmin(lmin, (double)un);
        lmax = fmax(lmax, (double)un);
    }
    }
    if (P.red.partials) block_partials(P.red.partials, lsum, lmin, lmax);
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

// Blocks of an explicit launch (also sizes the reduction scratch).
int explicit_num_blocks(int ndim, const int n[3]) {
    if (ndim == 2) {
        const int waves = ((n[0] + ExStream::COLS - 1) / ExStream::COLS) * ((n[1] + ExStream::TY - 1) / ExStream::TY);
        const int blocks = (waves + ExStream::WAVES - 1) / ExStream::WAVES;
        return (blocks + 7) & ~7;  // a multiple of 8 for the XCD-aware order
    }
    using TL = ExTile;
    return ((n[0] + TL::TX - 1) / TL::TX) * ((n[1] + TL::TY - 1) / TL::TY) *
           ((n[2] + TL::TZ - 1) / TL::TZ);
}

template <typename T>
hipError_t launch_explicit(const ExplicitParams<T>& P, int ndim, hipStream_t st, int* nblocks_out) {
    const int nb = explicit_num_blocks(ndim, P.n);
    if (nblocks_out) *nblocks_out = nb;
    const bool vl = P.limiter == LIM_VANLEER;
    if (ndim == 2) {
        constexpr int NT = 64 * ExStream::WAVES;
        if (vl) hipLaunchKernelGGL((explicit_stream2d_kernel<T, LIM_VANLEER>), dim3(nb), dim3(NT), 0, st, P);
        else hipLaunchKernelGGL((explicit_stream2d_kernel<T, -1>), dim3(nb), dim3(NT), 0, st, P);
    } else {
        if (vl) hipLaunchKernelGGL((explicit3d_kernel<T, LIM_VANLEER>), dim3(nb), dim3(ExTile::NT), 0, st, P);
        else hipLaunchKernelGGL((explicit3d_kernel<T, -1>), dim3(nb), dim3(ExTile::NT), 0, st, P);
    }
    return hipGetLastError();
}

template hipError_t launch_explicit<float>(const ExplicitParams<float>&, int, hipStream_t, int*);
template hipError_t launch_explicit<double>(const ExplicitParams<double>&, int, hipStream_t, int*);

}  // namespace asd
