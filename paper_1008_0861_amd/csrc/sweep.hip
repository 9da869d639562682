// One directional sweep of the split semi-implicit scheme (section 2,
// Eqs. xup / yup): kernel wrappers and launchers.  Two variants of the tile
// body compute the same sweep: face slots (sweep_tile.h: faces evaluated
// while the tile is staged, 8-byte LDS slots) and cell slots
// (sweep_cell.h: 16-byte cell slots, faces evaluated in the solve); the
// description of the method and of its gfx950 mapping is in those files.
#include "sweep_cell.h"
#include "sweep_tile.h"

namespace asd {

// The parameters every wave needs before its first global load arrive as
// leading scalar arguments, which the build preloads into scalar registers
// at wave launch (gfx950 kernel-argument preloading, at most 14 dwords): the
// wave then issues its loads without first waiting on a scalar load of the
// argument block.  The remaining fields are read from P as usual; the
// leading arguments override the copies of those fields in P.
//   packed: bits 0-3 log2(64 wpl), 4-7 log2(lpw), 8 periodic, 9 solve only,
//           10-14 LDS pad, 15 aligned tile layout, 16 log2(io).
template <typename T, int NDIM, int MMAX, int LIMC, bool EXT>
__global__ void __launch_bounds__((SweepBounds<T, MMAX>::max_threads))
    sweep_kernel(const T* U, const T* alpha, const T* beta1, int n, int nt1, int si_t1, int si_t2, int nb1,
                 int nblk, int packed, int row1, SweepParams<T> Pk) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    SweepParams<T> P = Pk;
    P.U = U;
    P.alpha = alpha;
    P.beta1 = beta1;
    P.n = n;
    P.nt1 = nt1;
    P.si_t1 = si_t1;
    P.si_t2 = si_t2;
    P.spl_log2 = packed & 15;
    P.wpl = 1 << (P.spl_log2 - 6);
    P.lpw_log2 = (packed >> 4) & 15;
    P.lpw = 1 << P.lpw_log2;
    P.periodic = (packed >> 8) & 1;
    P.rhs_mode = (packed >> 9) & 1;
    P.lds.pad = (packed >> 10) & 31;
    P.lds.aligned = (packed >> 15) & 1;
    P.io_log2 = (packed >> 16) & 1;
    P.lds.row1 = row1;
    // XCD-aware block order: consecutive logical blocks on the same XCD so
    // that halo lines and the partial lines of a transposed store are shared
    // through that XCD's L2.
    int blk = blockIdx.x;
    if ((nblk & 7) == 0) blk = (blk & 7) * (nblk >> 3) + (blk >> 3);
    const int l2 = blk / nb1;
    const int l1_0 = (blk - l2 * nb1) * P.lpw;
    double lsum;
    T lmin, lmax;
    sweep_tile<T, NDIM, MMAX, LIMC, EXT>(P, l1_0, l2, smem_raw, lsum, lmin, lmax);
    // FP64 energy / min / max partials (folded by a later launch)
    if (P.red.partials) block_partials<T>(P.red.partials, lsum, lmin, lmax);
}

// The cell-slot variant: the same leading arguments (io is always 1).
template <typename T, int NDIM, int MMAX, int LIMC, bool EXT>
__global__ void __launch_bounds__((SweepCellBounds<T, MMAX>::max_threads))
    sweep_cell_kernel(const T* U, const T* alpha, const T* beta1, int n, int nt1, int si_t1, int si_t2, int nb1,
                      int nblk, int packed, int row1, SweepParams<T> Pk) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    SweepParams<T> P = Pk;
    P.U = U;
    P.alpha = alpha;
    P.beta1 = beta1;
    P.n = n;
    P.nt1 = nt1;
    P.si_t1 = si_t1;
    P.si_t2 = si_t2;
    P.spl_log2 = packed & 15;
    P.wpl = 1 << (P.spl_log2 - 6);
    P.lpw_log2 = (packed >> 4) & 15;
    P.lpw = 1 << P.lpw_log2;
    P.periodic = (packed >> 8) & 1;
    P.rhs_mode = (packed >> 9) & 1;
    P.lds.pad = (packed >> 10) & 31;
    P.lds.aligned = (packed >> 15) & 1;
    P.io_log2 = 0;
    P.lds.row1 = row1;
    int blk = blockIdx.x;
    if ((nblk & 7) == 0) blk = (blk & 7) * (nblk >> 3) + (blk >> 3);
    const int l2 = blk / nb1;
    const int l1_0 = (blk - l2 * nb1) * P.lpw;
    double lsum;
    T lmin, lmax;
    cell::sweep_tile<T, NDIM, MMAX, LIMC, EXT>(P, l1_0, l2, smem_raw, lsum, lmin, lmax);
    if (P.red.partials) block_partials<T>(P.red.partials, lsum, lmin, lmax);
}

// Van Leer (the default limiter) gets its own straight-line instantiation;
// the other limiters share one that reads the limiter at run time, and T = 0
// walls or a source take a third that also reads those.
template <typename T, int NDIM>
static hipError_t launch_sweep_dim(const SweepParams<T>& P, int mmax, dim3 grid, dim3 block, size_t lds,
                                   hipStream_t st, int variant) {
    // T = 0 walls, a source or a second output take the EXT instantiation
    const bool ext = P.dirichlet || P.Q || P.out2;
    const bool cellv = variant == SWEEP_CELL_SLOTS;
    if (P.lpw != (1 << P.lpw_log2) || 64 * P.wpl != (1 << P.spl_log2) || P.spl_log2 > 15 || P.lpw_log2 > 15 ||
        P.lds.pad < 0 || P.lds.pad > 31 || P.io_log2 < 0 || P.io_log2 > 1 || (cellv && P.io_log2 != 0) ||
        (variant != SWEEP_FACE_SLOTS && !cellv) || (int)block.x != (P.lpw << (P.spl_log2 + P.io_log2)) ||
        (int)block.x > (cellv ? sweep_cell_max_threads((int)sizeof(T), mmax) : sweep_max_threads((int)sizeof(T), mmax)))
        return hipErrorInvalidValue;
    // the kernel's leading (preloaded) arguments; P.rhs_mode holds 0 or SWEEP_SOLVE_ONLY
    const int nb1 = (P.nt1 + P.lpw - 1) / P.lpw;
    const int packed = P.spl_log2 | (P.lpw_log2 << 4) | ((P.periodic != 0) << 8) | ((P.rhs_mode != 0) << 9) |
                       (P.lds.pad << 10) | ((P.lds.aligned != 0) << 15) | ((P.io_log2 & 1) << 16);
#define ASD_SWEEP_ARGS P.U, P.alpha, P.beta1, P.n, P.nt1, P.si_t1, P.si_t2, nb1, (int)grid.x, packed, P.lds.row1, P
#define ASD_SWEEP_LAUNCH(KERNEL, MM)                                                                          \
    do {                                                                                                      \
        if (ext)                                                                                              \
            hipLaunchKernelGGL((KERNEL<T, NDIM, MM, -1, true>), grid, block, lds, st, ASD_SWEEP_ARGS);        \
        else if (P.limiter == LIM_VANLEER)                                                                    \
            hipLaunchKernelGGL((KERNEL<T, NDIM, MM, LIM_VANLEER, false>), grid, block, lds, st, ASD_SWEEP_ARGS); \
        else                                                                                                  \
            hipLaunchKernelGGL((KERNEL<T, NDIM, MM, -1, false>), grid, block, lds, st, ASD_SWEEP_ARGS);       \
    } while (0)
#define ASD_SWEEP_CASE(MM)                                      \
    case MM:                                                    \
        if (cellv) ASD_SWEEP_LAUNCH(sweep_cell_kernel, MM);     \
        else ASD_SWEEP_LAUNCH(sweep_kernel, MM);                \
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
#undef ASD_SWEEP_LAUNCH
#undef ASD_SWEEP_ARGS
}

// Raise the dynamic-LDS limit of every sweep instantiation to the gfx950
// maximum.  Called once per process, before any launch or stream capture.
template <typename T, int NDIM, int LIMC, bool EXT>
static hipError_t set_attrs_lim(int bytes) {
    const void* fns[] = {(const void*)sweep_kernel<T, NDIM, 1, LIMC, EXT>, (const void*)sweep_kernel<T, NDIM, 2, LIMC, EXT>,
                         (const void*)sweep_kernel<T, NDIM, 4, LIMC, EXT>, (const void*)sweep_kernel<T, NDIM, 8, LIMC, EXT>,
                         (const void*)sweep_kernel<T, NDIM, 16, LIMC, EXT>,
                         (const void*)sweep_cell_kernel<T, NDIM, 1, LIMC, EXT>,
                         (const void*)sweep_cell_kernel<T, NDIM, 2, LIMC, EXT>,
                         (const void*)sweep_cell_kernel<T, NDIM, 4, LIMC, EXT>,
                         (const void*)sweep_cell_kernel<T, NDIM, 8, LIMC, EXT>,
                         (const void*)sweep_cell_kernel<T, NDIM, 16, LIMC, EXT>};
    for (const void* f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
template <typename T, int NDIM>
static hipError_t set_attrs_dim(int bytes) {
    hipError_t e = set_attrs_lim<T, NDIM, LIM_VANLEER, false>(bytes);
    if (e == hipSuccess) e = set_attrs_lim<T, NDIM, -1, false>(bytes);
    if (e == hipSuccess) e = set_attrs_lim<T, NDIM, -1, true>(bytes);
    return e;
}

hipError_t sweep_set_lds_limits(int bytes) {
    hipError_t e = set_attrs_dim<float, 2>(bytes);
    if (e == hipSuccess) e = set_attrs_dim<float, 3>(bytes);
    if (e == hipSuccess) e = set_attrs_dim<double, 2>(bytes);
    if (e == hipSuccess) e = set_attrs_dim<double, 3>(bytes);
    return e;
}

template <typename T>
hipError_t launch_sweep(const SweepParams<T>& P, int ndim, int mmax, dim3 grid, dim3 block, size_t lds,
                        hipStream_t st, int variant) {
    if (ndim == 2) return launch_sweep_dim<T, 2>(P, mmax, grid, block, lds, st, variant);
    return launch_sweep_dim<T, 3>(P, mmax, grid, block, lds, st, variant);
}

template hipError_t launch_sweep<float>(const SweepParams<float>&, int, int, dim3, dim3, size_t, hipStream_t, int);
template hipError_t launch_sweep<double>(const SweepParams<double>&, int, int, dim3, dim3, size_t,
                                         hipStream_t, int);

}  // namespace asd
