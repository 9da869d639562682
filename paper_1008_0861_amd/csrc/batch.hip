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
//   another, so the launch needs no co-residency.  As a workgroup holds all
//   of a problem's tiles, it also reduces the problem's FP64 energy, min and
//   max after every step itself (fixed order, no atomics on the sums).
// batch_grouped_kernel: one launch per sweep for all problems; block b
//   finds its problem by binary search in a prefix table of line groups.
//   With outputs, every y-sweep block writes its (sum, min, max) partial into
//   a ring slot, and batch_fold_kernel folds each problem's partials later.
// EXT: T = 0 walls (the batch's problems share one boundary condition); the
// tiles then read the wall flag and the limiter from each problem's
// parameters.
#include "sweep_cell.h"
#include "sweep_tile.h"

namespace asd {

// Status bits of an FP64 (energy, min, max) after a step; e0 the energy of
// the call's initial state (drift is not flagged with T = 0 walls).
__device__ __forceinline__ unsigned status_bits(double E, double mn, double mx, double e0, bool drift) {
    unsigned fl = 0;
    // isfinite, not x - x != 0: contracted, E - E is the rounding error of
    // the product that formed E
    if (!__builtin_isfinite(E) || !__builtin_isfinite(mn) || !__builtin_isfinite(mx)) fl |= 1u;
    if (mn < 0.0) fl |= 2u;
    if (drift && fabs(E - e0) > 1e-6 * fabs(e0)) fl |= 4u;
    return fl;
}

// Block-wide (sum, min, max) of every thread's values, in a fixed order;
// thread 0 receives the result.  Every thread must call it.
template <typename M>
__device__ __forceinline__ void block_reduce3(double s, M mn, M mx, double& S, double& MN, double& MX) {
    __shared__ double r_s[16], r_mn[16], r_mx[16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    s = wave_sum_lane63(s);
    mn = wave_min_lane63<M>(mn);
    mx = wave_max_lane63<M>(mx);
    if (lane == 63) {
        r_s[wid] = s;
        r_mn[wid] = (double)mn;
        r_mx[wid] = (double)mx;
    }
    __syncthreads();
    S = 0.0;
    MN = r_mn[0];
    MX = r_mx[0];
    if (threadIdx.x == 0) {
        for (int w = 0; w < nw; ++w) {
            S += r_s[w];
            MN = fmin(MN, r_mn[w]);
            MX = fmax(MX, r_mx[w]);
        }
    }
    __syncthreads();  // r_* may be refilled by the next call
}

// One line tile of a batch problem on either tile body (CELL: the
// cell-slot body of sweep_cell.h).  Both end with a block barrier.
template <typename T, int MMAX, int LIMC, bool EXT, bool CELL, bool REUSE, bool HALF = false>
__device__ __forceinline__ void batch_tile(const SweepParams<T>& P, int l1_0, unsigned char* smem, double& lsum,
                                           T& lmin, T& lmax) {
    if constexpr (CELL)
        cell::sweep_tile<T, 2, MMAX, LIMC, EXT>(P, l1_0, 0, smem, lsum, lmin, lmax);
    else
        sweep_tile<T, 2, MMAX, LIMC, EXT, REUSE, HALF>(P, l1_0, 0, smem, lsum, lmin, lmax);
}
// The tile at the problem's own capacity mm (MMAX, MMAX / 2, or 4 in the
// capacity-16 kernels) and line packing (half: two lines per wave,
// capacity-16 face-body kernels only); uniform over the block, which
// belongs to one problem.
template <typename T, int MMAX, int LIMC, bool EXT, bool CELL, bool REUSE>
__device__ __forceinline__ void batch_tile_cap(int mm, int half, const SweepParams<T>& P, int l1_0,
                                               unsigned char* smem, double& lsum, T& lmin, T& lmax) {
    if constexpr (MMAX == 16 && !CELL) {
        if (half) {
            batch_tile<T, MMAX, LIMC, EXT, CELL, REUSE, true>(P, l1_0, smem, lsum, lmin, lmax);
            return;
        }
    }
    if constexpr (MMAX == 16) {
        if (mm <= 4) {
            batch_tile<T, 4, LIMC, EXT, CELL, REUSE>(P, l1_0, smem, lsum, lmin, lmax);
            return;
        }
    }
    if constexpr (MMAX >= 4) {
        if (mm < MMAX) {
            batch_tile<T, MMAX / 2, LIMC, EXT, CELL, REUSE>(P, l1_0, smem, lsum, lmin, lmax);
            return;
        }
    }
    batch_tile<T, MMAX, LIMC, EXT, CELL, REUSE>(P, l1_0, smem, lsum, lmin, lmax);
}
template <typename T, int MMAX, bool CELL>
struct BatchBounds {
    static constexpr int max_threads = CELL ? SweepCellBounds<T, MMAX>::max_threads : SweepBounds<T, MMAX>::max_threads;
};

template <typename T, int MMAX, int LIMC, bool EXT, bool CELL>
__global__ void __launch_bounds__((BatchBounds<T, MMAX, CELL>::max_threads))
    batch_persistent_kernel(const BatchProblem<T>* probs, const int* off, const int* list, int nsteps, BatchOut out) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int i0 = off[blockIdx.x], i1 = off[blockIdx.x + 1];
    double lsum;
    T lmin, lmax;
    for (int i = i0; i < i1; ++i) {
        const int pi = list[i];
        const BatchProblem<T>* bp = probs + pi;
        for (int s = 0; s < nsteps; ++s) {
#pragma unroll 1
            for (int d = 0; d < 2; ++d) {
                SweepParams<T> P = bp->sweep[d];
                const bool reduce = out.energy && d == 1;
                // any non-null pointer switches the tiles' reductions on; the
                // tiles never write through it
                P.red.partials = reduce ? out.energy : nullptr;
                double acc = 0.0;
                T amin = T(__builtin_huge_val()), amax = T(-__builtin_huge_val());
                const int ng = bp->ngroups[d];
                for (int g = 0; g < ng; ++g) {
                    batch_tile_cap<T, MMAX, LIMC, EXT, CELL, true>(bp->mmax[d], bp->half[d], P, g * P.lpw, smem_raw,
                                                                  lsum, lmin, lmax);
                    acc += lsum;
                    amin = lmin < amin ? lmin : amin;
                    amax = lmax > amax ? lmax : amax;
                }
                // sweep_tile ends with a block barrier: this sweep's stores are
                // visible to every thread of the workgroup before the next sweep
                if (reduce) {
                    double S, MN, MX;
                    block_reduce3<T>(acc, amin, amax, S, MN, MX);
                    if (threadIdx.x == 0) {
                        const double E = S * bp->dV;
                        double* e = out.energy + (size_t)pi * out.stride;
                        e[s + 1] = E;
                        const unsigned fl = status_bits(E, MN, MX, e[0], !bp->dirichlet);
                        if (fl) atomicOr(out.flags + pi, fl);
                        if (s == nsteps - 1) {
                            out.stats[3 * pi] = E;
                            out.stats[3 * pi + 1] = MN;
                            out.stats[3 * pi + 2] = MX;
                        }
                    }
                }
            }
        }
    }
}

template <typename T, int MMAX, int LIMC, bool EXT, bool CELL>
__global__ void __launch_bounds__((BatchBounds<T, MMAX, CELL>::max_threads))
    batch_grouped_kernel(const BatchProblem<T>* probs, const int* group_start, int nprob, int d, double* partials) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int b = blockIdx.x;
    int lo = 0, hi = nprob;  // group_start[lo] <= b < group_start[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (group_start[mid] <= b) lo = mid;
        else hi = mid;
    }
    SweepParams<T> P = probs[lo].sweep[d];
    P.red.partials = partials;
    double lsum;
    T lmin, lmax;
    batch_tile_cap<T, MMAX, LIMC, EXT, CELL, false>(probs[lo].mmax[d], probs[lo].half[d], P,
                                                    (b - group_start[lo]) * P.lpw, smem_raw, lsum, lmin, lmax);
    // block b's partial sits at index b: problem p's y-sweep tiles are
    // tile0[p] .. tile0[p] + ngroups[1] - 1
    if (partials) block_partials<T>(partials, lsum, lmin, lmax);
}

// Block p: FP64 energy of problem p's current state (its x-sweep input).
template <typename T>
__global__ void __launch_bounds__(1024) batch_reduce0_kernel(const BatchProblem<T>* probs, BatchOut out) {
    const BatchProblem<T>& bp = probs[blockIdx.x];
    const SweepParams<T>& P = bp.sweep[0];
    const int N = P.n * P.nt1;
    // four loads in flight per thread (four partial sums, combined in a
    // fixed order)
    constexpr int U4 = 4;
    double s4[U4] = {0.0, 0.0, 0.0, 0.0};
    T mn = T(__builtin_huge_val()), mx = T(-__builtin_huge_val());
    const int stride = (int)blockDim.x * U4;
    for (int i0 = threadIdx.x; i0 < N; i0 += stride) {
        T v[U4];
#pragma unroll
        for (int u = 0; u < U4; ++u) {
            const int i = i0 + u * (int)blockDim.x;
            v[u] = i < N ? P.U[i] : T(0);
        }
#pragma unroll
        for (int u = 0; u < U4; ++u) {
            if (i0 + u * (int)blockDim.x < N) {
                s4[u] += (double)v[u];
                mn = v[u] < mn ? v[u] : mn;
                mx = v[u] > mx ? v[u] : mx;
            }
        }
    }
    const double s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    double S, MN, MX;
    block_reduce3<T>(s, mn, mx, S, MN, MX);
    if (threadIdx.x == 0) out.energy[(size_t)blockIdx.x * out.stride] = S * bp.dV;
}

// Block (p, c): fold ring slot c of the y-sweep partials of problem p into
// its energy entry out.first + c.
template <typename T>
__global__ void __launch_bounds__(256) batch_fold_kernel(const BatchProblem<T>* probs, BatchOut out) {
    const int p = blockIdx.x, c = blockIdx.y;
    const BatchProblem<T>& bp = probs[p];
    const double* part = out.partials + (size_t)c * out.slot_stride + 3 * (size_t)bp.tile0;
    const int nb = bp.ngroups[1];
    double s = 0.0, mn = __builtin_huge_val(), mx = -__builtin_huge_val();
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        s += part[3 * i];
        mn = fmin(mn, part[3 * i + 1]);
        mx = fmax(mx, part[3 * i + 2]);
    }
    double S, MN, MX;
    block_reduce3<double>(s, mn, mx, S, MN, MX);
    if (threadIdx.x == 0) {
        const double E = S * bp.dV;
        double* e = out.energy + (size_t)p * out.stride;
        e[out.first + c] = E;
        const unsigned fl = status_bits(E, MN, MX, e[0], !bp.dirichlet);
        if (fl) atomicOr(out.flags + p, fl);
        if (out.last && c == out.count - 1) {
            out.stats[3 * p] = E;
            out.stats[3 * p + 1] = MN;
            out.stats[3 * p + 2] = MX;
        }
    }
}

template <typename T, int MMAX, int LIMC, bool EXT>
static hipError_t set_batch_attrs_lim(int bytes) {
    const void* fns[] = {(const void*)batch_persistent_kernel<T, MMAX, LIMC, EXT, false>,
                         (const void*)batch_grouped_kernel<T, MMAX, LIMC, EXT, false>,
                         (const void*)batch_persistent_kernel<T, MMAX, LIMC, EXT, true>,
                         (const void*)batch_grouped_kernel<T, MMAX, LIMC, EXT, true>};
    for (const void* f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
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
#define ASD_BATCH_LAUNCH_BODY(KERNEL, MM, CELL, ...)                                        \
    do {                                                                                    \
        if (dirichlet)                                                                      \
            hipLaunchKernelGGL((KERNEL<T, MM, -1, true, CELL>), __VA_ARGS__);               \
        else if (limiter == LIM_VANLEER)                                                    \
            hipLaunchKernelGGL((KERNEL<T, MM, LIM_VANLEER, false, CELL>), __VA_ARGS__);     \
        else                                                                                \
            hipLaunchKernelGGL((KERNEL<T, MM, -1, false, CELL>), __VA_ARGS__);              \
    } while (0)
#define ASD_BATCH_LAUNCH(KERNEL, MM, ...)                                                   \
    do {                                                                                    \
        if (variant == SWEEP_CELL_SLOTS) ASD_BATCH_LAUNCH_BODY(KERNEL, MM, true, __VA_ARGS__);  \
        else ASD_BATCH_LAUNCH_BODY(KERNEL, MM, false, __VA_ARGS__);                         \
    } while (0)

template <typename T>
hipError_t launch_batch_persistent(const BatchProblem<T>* probs, const int* off, const int* list, int nwg, int nsteps,
                                   int mmax, int nthreads, size_t lds, int limiter, int dirichlet, int variant,
                                   const BatchOut& out, hipStream_t st) {
    if ((variant != SWEEP_FACE_SLOTS && variant != SWEEP_CELL_SLOTS) ||
        nthreads > (variant == SWEEP_CELL_SLOTS ? sweep_cell_max_threads((int)sizeof(T), mmax)
                                                : sweep_max_threads((int)sizeof(T), mmax)))
        return hipErrorInvalidValue;
    switch (mmax) {
        case 4: ASD_BATCH_LAUNCH(batch_persistent_kernel, 4, dim3(nwg), dim3(nthreads), lds, st, probs, off, list, nsteps, out); break;
        case 8: ASD_BATCH_LAUNCH(batch_persistent_kernel, 8, dim3(nwg), dim3(nthreads), lds, st, probs, off, list, nsteps, out); break;
        case 16: ASD_BATCH_LAUNCH(batch_persistent_kernel, 16, dim3(nwg), dim3(nthreads), lds, st, probs, off, list, nsteps, out); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_grouped(const BatchProblem<T>* probs, const int* group_start, int nprob, int ngroups, int d,
                                int mmax, int nthreads, size_t lds, int limiter, int dirichlet, int variant,
                                double* partials, hipStream_t st) {
    if ((variant != SWEEP_FACE_SLOTS && variant != SWEEP_CELL_SLOTS) ||
        nthreads > (variant == SWEEP_CELL_SLOTS ? sweep_cell_max_threads((int)sizeof(T), mmax)
                                                : sweep_max_threads((int)sizeof(T), mmax)))
        return hipErrorInvalidValue;
    switch (mmax) {
        case 4: ASD_BATCH_LAUNCH(batch_grouped_kernel, 4, dim3(ngroups), dim3(nthreads), lds, st, probs, group_start, nprob, d, partials); break;
        case 8: ASD_BATCH_LAUNCH(batch_grouped_kernel, 8, dim3(ngroups), dim3(nthreads), lds, st, probs, group_start, nprob, d, partials); break;
        case 16: ASD_BATCH_LAUNCH(batch_grouped_kernel, 16, dim3(ngroups), dim3(nthreads), lds, st, probs, group_start, nprob, d, partials); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
#undef ASD_BATCH_LAUNCH
#undef ASD_BATCH_LAUNCH_BODY

template <typename T>
hipError_t launch_batch_reduce0(const BatchProblem<T>* probs, int nprob, const BatchOut& out, hipStream_t st) {
    hipLaunchKernelGGL(batch_reduce0_kernel<T>, dim3(nprob), dim3(1024), 0, st, probs, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_fold(const BatchProblem<T>* probs, int nprob, const BatchOut& out, hipStream_t st) {
    hipLaunchKernelGGL(batch_fold_kernel<T>, dim3(nprob, out.count), dim3(256), 0, st, probs, out);
    return hipGetLastError();
}

#define ASD_BATCH_INST(T)                                                                                        \
    template hipError_t launch_batch_persistent<T>(const BatchProblem<T>*, const int*, const int*, int, int, int, \
                                                   int, size_t, int, int, int, const BatchOut&, hipStream_t);     \
    template hipError_t launch_batch_grouped<T>(const BatchProblem<T>*, const int*, int, int, int, int, int,     \
                                                size_t, int, int, int, double*, hipStream_t);                   \
    template hipError_t launch_batch_reduce0<T>(const BatchProblem<T>*, int, const BatchOut&, hipStream_t);      \
    template hipError_t launch_batch_fold<T>(const BatchProblem<T>*, int, const BatchOut&, hipStream_t);
ASD_BATCH_INST(float)
ASD_BATCH_INST(double)
#undef ASD_BATCH_INST

}  // namespace asd
