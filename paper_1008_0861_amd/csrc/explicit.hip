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
// gfx950 mapping: one workgroup per tile of TX x TY x TZ cells.  The tile
// plus a one-cell halo of U, b (and chi) is staged through LDS with
// coalesced loads; the limited cell slopes along every axis are computed
// once per staged cell; each thread then updates one cell.
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

// Tile of TX x TY (x TZ) cells with a one-cell halo, NT threads; each thread
// updates NC / NT cells.  2-D: 64 x 16 in FP32 (halo overhead 1.16, 4 cells
// per thread), 64 x 8 in FP64 (32 KB of LDS, several tiles per CU); 3-D:
// 32 x 4 x 2, which keeps the FP64 tile within 64 KB of LDS.
template <typename T, int NDIM>
struct ExTile {
    static constexpr int TX = NDIM == 2 ? 64 : 32;
    static constexpr int TY = NDIM == 2 ? (sizeof(T) == 4 ? 16 : 8) : 4;
    static constexpr int TZ = NDIM == 2 ? 1 : 2;
    static constexpr int BX = TX + 2, BY = TY + 2, BZ = NDIM == 2 ? 1 : TZ + 2;
    static constexpr int NB = BX * BY * BZ;
    static constexpr int NC = TX * TY * TZ;
    static constexpr int NT = 256;
};

// LIMC: the limiter as a compile-time constant (van Leer, the default), or -1
// to read it from the parameters.
template <typename T, int NDIM, int LIMC>
__global__ void __launch_bounds__(256) explicit_kernel(ExplicitParams<T> P) {
    using TL = ExTile<T, NDIM>;
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

template <typename T>
int explicit_num_blocks_t(int ndim, const int n[3]) {
    if (ndim == 2) {
        using TL = ExTile<T, 2>;
        return ((n[0] + TL::TX - 1) / TL::TX) * ((n[1] + TL::TY - 1) / TL::TY);
    }
    using TL = ExTile<T, 3>;
    return ((n[0] + TL::TX - 1) / TL::TX) * ((n[1] + TL::TY - 1) / TL::TY) *
           ((n[2] + TL::TZ - 1) / TL::TZ);
}

// Blocks of an explicit launch, the larger of the two precisions' tilings
// (sizes the reduction scratch).
int explicit_num_blocks(int ndim, const int n[3]) {
    const int a = explicit_num_blocks_t<float>(ndim, n), b = explicit_num_blocks_t<double>(ndim, n);
    return a > b ? a : b;
}

template <typename T>
hipError_t launch_explicit(const ExplicitParams<T>& P, int ndim, hipStream_t st, int* nblocks_out) {
    const int nb = explicit_num_blocks_t<T>(ndim, P.n);
    if (nblocks_out) *nblocks_out = nb;
    const bool vl = P.limiter == LIM_VANLEER;
    if (ndim == 2) {
        if (vl) hipLaunchKernelGGL((explicit_kernel<T, 2, LIM_VANLEER>), dim3(nb), dim3(ExTile<T, 2>::NT), 0, st, P);
        else hipLaunchKernelGGL((explicit_kernel<T, 2, -1>), dim3(nb), dim3(ExTile<T, 2>::NT), 0, st, P);
    } else {
        if (vl) hipLaunchKernelGGL((explicit_kernel<T, 3, LIM_VANLEER>), dim3(nb), dim3(ExTile<T, 3>::NT), 0, st, P);
        else hipLaunchKernelGGL((explicit_kernel<T, 3, -1>), dim3(nb), dim3(ExTile<T, 3>::NT), 0, st, P);
    }
    return hipGetLastError();
}

template hipError_t launch_explicit<float>(const ExplicitParams<float>&, int, hipStream_t, int*);
template hipError_t launch_explicit<double>(const ExplicitParams<double>&, int, hipStream_t, int*);

}  // namespace asd
