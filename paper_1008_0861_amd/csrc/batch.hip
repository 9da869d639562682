// Batched semi-implicit steps over many independent 2-D problems of uneven
// sizes (each problem: section 2, Eqs. xup / yup, with its own grid, b,
// chi_par and dt).  Both kernels run the line tiles of sweep_tile.h.
//
// batch_persistent_kernel: one launch for all problems and all steps.
//   Workgroup w owns the problems list[off[w] .. off[w+1]) (assigned by the
//   host, largest first, to the least-loaded workgroup) and advances each of
//   them through every step; the x sweep of a problem writes its T* with
//   ordinary stores, a block barrier makes them visible to the whole
//   workgroup, and the y sweep reads them.  No workgroup ever waits for
//   another, so the launch needs no co-residency.
// batch_grouped_kernel: one launch per sweep for all problems; block b
//   finds its problem by binary search in a prefix table of line groups.
// EXT: T = 0 walls (the batch's problems share one boundary condition); the
// tiles then read the wall flag and the limiter from each problem's
// parameters.
#include "sweep_tile.h"

namespace asd {

template <typename T, int MMAX, int LIMC, bool EXT>
__global__ void __launch_bounds__((SweepBounds<T, MMAX>::max_threads))
    batch_persistent_kernel(const BatchProblem<T>* probs, const int* off, const int* list, int nsteps) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int i0 = off[blockIdx.x], i1 = off[blockIdx.x + 1];
    double lsum;
    T lmin, lmax;
    for (int i = i0; i < i1; ++i) {
        const BatchProblem<T>* bp = probs + list[i];
        for (int s = 0; s < nsteps; ++s) {
#pragma unroll 1
            for (int d = 0; d < 2; ++d) {
                const SweepParams<T> P = bp->sweep[d];
                const int ng = bp->ngroups[d];
                for (int g = 0; g < ng; ++g)
                    sweep_tile<T, 2, MMAX, LIMC, EXT, true>(P, g * P.lpw, 0, smem_raw, lsum, lmin, lmax);
                // sweep_tile ends with a block barrier: this sweep's stores are
                // visible to every thread of the workgroup before the next sweep
            }
        }
    }
}

template <typename T, int MMAX, int LIMC, bool EXT>
__global__ void __launch_bounds__((SweepBounds<T, MMAX>::max_threads))
    batch_grouped_kernel(const BatchProblem<T>* probs, const int* group_start, int nprob, int d) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int b = blockIdx.x;
    int lo = 0, hi = nprob;  // group_start[lo] <= b < group_start[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (group_start[mid] <= b) lo = mid;
        else hi = mid;
    }
    const SweepParams<T> P = probs[lo].sweep[d];
    double lsum;
    T lmin, lmax;
    sweep_tile<T, 2, MMAX, LIMC, EXT>(P, (b - group_start[lo]) * P.lpw, 0, smem_raw, lsum, lmin, lmax);
}

template <typename T, int MMAX, int LIMC, bool EXT>
static hipError_t set_batch_attrs_lim(int bytes) {
    hipError_t e = hipFuncSetAttribute((const void*)batch_persistent_kernel<T, MMAX, LIMC, EXT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)batch_grouped_kernel<T, MMAX, LIMC, EXT>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    return e;
}
template <typename T, int MMAX>
static hipError_t set_batch_attrs(int bytes) {
    hipError_t e = set_batch_attrs_lim<T, MMAX, LIM_VANLEER, false>(bytes);
    if (e == hipSuccess) e = set_batch_attrs_lim<T, MMAX, -1, false>(bytes);
    if (e == hipSuccess) e = set_batch_attrs_lim<T, MMAX, -1, true>(bytes);
    return e;
}

hipError_t batch_set_lds_limits(int bytes) {
    hipError_t e = set_batch_attrs<float, 4>(bytes);
    if (e == hipSuccess) e = set_batch_attrs<float, 8>(bytes);
    if (e == hipSuccess) e = set_batch_attrs<float, 16>(bytes);
    if (e == hipSuccess) e = set_batch_attrs<double, 4>(bytes);
    if (e == hipSuccess) e = set_batch_attrs<double, 8>(bytes);
    if (e == hipSuccess) e = set_batch_attrs<double, 16>(bytes);
    return e;
}

// The problems of a batch share one limiter and boundary condition
// (checked by the host); van Leer without walls has its own straight-line
// instantiation, T = 0 walls take the EXT one.
#define ASD_BATCH_LAUNCH(KERNEL, MM, ...)                                                   \
    do {                                                                                    \
        if (dirichlet)                                                                      \
            hipLaunchKernelGGL((KERNEL<T, MM, -1, true>), __VA_ARGS__);                     \
        else if (limiter == LIM_VANLEER)                                                    \
            hipLaunchKernelGGL((KERNEL<T, MM, LIM_VANLEER, false>), __VA_ARGS__);           \
        else                                                                                \
            hipLaunchKernelGGL((KERNEL<T, MM, -1, false>), __VA_ARGS__);                    \
    } while (0)

template <typename T>
hipError_t launch_batch_persistent(const BatchProblem<T>* probs, const int* off, const int* list, int nwg, int nsteps,
                                   int mmax, int nthreads, size_t lds, int limiter, int dirichlet, hipStream_t st) {
    switch (mmax) {
        case 4: ASD_BATCH_LAUNCH(batch_persistent_kernel, 4, dim3(nwg), dim3(nthreads), lds, st, probs, off, list, nsteps); break;
        case 8: ASD_BATCH_LAUNCH(batch_persistent_kernel, 8, dim3(nwg), dim3(nthreads), lds, st, probs, off, list, nsteps); break;
        case 16: ASD_BATCH_LAUNCH(batch_persistent_kernel, 16, dim3(nwg), dim3(nthreads), lds, st, probs, off, list, nsteps); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_grouped(const BatchProblem<T>* probs, const int* group_start, int nprob, int ngroups, int d,
                                int mmax, int nthreads, size_t lds, int limiter, int dirichlet, hipStream_t st) {
    switch (mmax) {
        case 4: ASD_BATCH_LAUNCH(batch_grouped_kernel, 4, dim3(ngroups), dim3(nthreads), lds, st, probs, group_start, nprob, d); break;
        case 8: ASD_BATCH_LAUNCH(batch_grouped_kernel, 8, dim3(ngroups), dim3(nthreads), lds, st, probs, group_start, nprob, d); break;
        case 16: ASD_BATCH_LAUNCH(batch_grouped_kernel, 16, dim3(ngroups), dim3(nthreads), lds, st, probs, group_start, nprob, d); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
#undef ASD_BATCH_LAUNCH

template hipError_t launch_batch_persistent<float>(const BatchProblem<float>*, const int*, const int*, int, int, int,
                                                   int, size_t, int, int, hipStream_t);
template hipError_t launch_batch_persistent<double>(const BatchProblem<double>*, const int*, const int*, int, int,
                                                    int, int, size_t, int, int, hipStream_t);
template hipError_t launch_batch_grouped<float>(const BatchProblem<float>*, const int*, int, int, int, int, int,
                                                size_t, int, int, hipStream_t);
template hipError_t launch_batch_grouped<double>(const BatchProblem<double>*, const int*, int, int, int, int, int,
                                                 size_t, int, int, hipStream_t);

}  // namespace asd
