// Small kernels of libasd: layout permutation (re-laying b and chi out so
// that every sweep reads contiguous lines), a standalone FP64 reduction of
// a state, fills and copies.
#include "asd_device.h"
#include "asd_launch.h"

namespace asd {

// Tiled permutation: the block reads a 32 x 32 tile of the (y, x) plane of
// source slice z coalesced along x and writes it coalesced along the
// destination's fastest axis when that is y.  The general 3-D permutations
// used here move x or y into the fastest position; z-fastest outputs are
// written with the plane loop below.
template <typename T>
__global__ void __launch_bounds__(256) permute_kernel(const T* __restrict__ in, T* __restrict__ out,
                                                     int nx, int ny, int nz, int64_t dsx, int64_t dsy,
                                                     int64_t dsz) {
    __shared__ T tile[32][33];
    const int tilesx = (nx + 31) / 32, tilesy = (ny + 31) / 32;
    int b = blockIdx.x;
    const int tx0 = (b % tilesx) * 32;
    b /= tilesx;
    const int ty0 = (b % tilesy) * 32;
    const int z = b / tilesy;
    const int lx = threadIdx.x & 31, ly = threadIdx.x >> 5;  // 32 x 8
    for (int r = ly; r < 32; r += 8) {
        const int x = tx0 + lx, y = ty0 + r;
        if (x < nx && y < ny) tile[r][lx] = in[(int64_t)x + (int64_t)y * nx + (int64_t)z * nx * ny];
    }
    __syncthreads();
    if (dsy == 1) {
        // destination has y fastest: write rows of the tile transposed
        for (int r = ly; r < 32; r += 8) {
            const int y = ty0 + lx, x = tx0 + r;
            if (x < nx && y < ny) out[(int64_t)x * dsx + y + (int64_t)z * dsz] = tile[lx][r];
        }
    } else {
        for (int r = ly; r < 32; r += 8) {
            const int x = tx0 + lx, y = ty0 + r;
            if (x < nx && y < ny) out[(int64_t)x * dsx + (int64_t)y * dsy + (int64_t)z * dsz] = tile[r][lx];
        }
    }
}

template <typename T>
hipError_t launch_permute(const T* in, T* out, const int n[3], const int64_t ds[3], hipStream_t st) {
    const int tilesx = (n[0] + 31) / 32, tilesy = (n[1] + 31) / 32;
    const int64_t nb = (int64_t)tilesx * tilesy * n[2];
    hipLaunchKernelGGL(permute_kernel<T>, dim3((unsigned)nb), dim3(256), 0, st, in, out, n[0], n[1],
                       n[2], ds[0], ds[1], ds[2]);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(256) reduce_kernel(const T* __restrict__ x, int64_t N, ReduceParams R) {
    // partials only; a later launch folds them
    double s = 0.0, mn = __builtin_huge_val(), mx = -__builtin_huge_val();
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double v = (double)x[i];
        s += v;
        mn = fmin(mn, v);
        mx = fmax(mx, v);
    }
    block_partials(R.partials, s, mn, mx);
}

__global__ void __launch_bounds__(256) fold_kernel(FoldParams f) { fold_partials(f); }

hipError_t launch_fold(const FoldParams& f, hipStream_t st) {
    if (f.count < 1) return hipSuccess;
    hipLaunchKernelGGL(fold_kernel, dim3(f.count), dim3(256), 0, st, f);
    return hipGetLastError();
}

int reduce_num_blocks(int64_t N) {
    int64_t nb = (N + 256 * 8 - 1) / (256 * 8);
    if (nb < 1) nb = 1;
    if (nb > 1024) nb = 1024;
    return (int)nb;
}

template <typename T>
hipError_t launch_reduce(const T* x, int64_t N, const ReduceParams& R, int nblocks, hipStream_t st) {
    hipLaunchKernelGGL(reduce_kernel<T>, dim3(nblocks), dim3(256), 0, st, x, N, R);
    return hipGetLastError();
}

__global__ void fill_u32_kernel(unsigned* p, unsigned v, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void fill_f64_kernel(double* p, double v, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
hipError_t launch_fill_u32(unsigned* p, unsigned v, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}
hipError_t launch_fill_f64(double* p, double v, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_f64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

// Plain streaming copy (also the calibration kernel for HBM byte counters).
template <typename T>
__global__ void __launch_bounds__(256) copy_kernel(const T* __restrict__ in, T* __restrict__ out, int64_t N) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = in[i];
}
template <typename T>
hipError_t launch_copy(const T* in, T* out, int64_t N, hipStream_t st) {
    int64_t nb = (N + 255) / 256;
    if (nb > 8192) nb = 8192;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(copy_kernel<T>, dim3((unsigned)nb), dim3(256), 0, st, in, out, N);
    return hipGetLastError();
}

// Streaming copy for the practical bandwidth ceiling: 16-byte accesses,
// each thread keeps kWideUnroll loads in flight before its stores, and the
// block's accesses of one round are contiguous (coalesced).  nvec 16-byte
// vectors; the caller copies any remainder.
static constexpr int kWideUnroll = 4;
__global__ void __launch_bounds__(256) copy_wide_kernel(const float4* __restrict__ in, float4* __restrict__ out,
                                                        int64_t nvec) {
    const int64_t base = (int64_t)blockIdx.x * (256 * kWideUnroll) + threadIdx.x;
    float4 v[kWideUnroll];
#pragma unroll
    for (int j = 0; j < kWideUnroll; ++j) {
        const int64_t i = base + j * 256;
        if (i < nvec) v[j] = in[i];
    }
#pragma unroll
    for (int j = 0; j < kWideUnroll; ++j) {
        const int64_t i = base + j * 256;
        if (i < nvec) out[i] = v[j];
    }
}
hipError_t launch_copy_wide(const void* in, void* out, size_t nbytes, hipStream_t st) {
    const int64_t nvec = (int64_t)(nbytes / 16);
    if (nvec > 0) {
        const int64_t nb = (nvec + 256 * kWideUnroll - 1) / (256 * kWideUnroll);
        if (nb > INT32_MAX) return hipErrorInvalidValue;
        hipLaunchKernelGGL(copy_wide_kernel, dim3((unsigned)nb), dim3(256), 0, st, (const float4*)in, (float4*)out,
                           nvec);
    }
    const int64_t tail = (int64_t)(nbytes - 16 * (size_t)nvec) / 4;  // nbytes is a multiple of 4
    if (tail > 0)
        hipLaunchKernelGGL(copy_kernel<float>, dim3(1), dim3(256), 0, st, (const float*)in + 4 * nvec,
                           (float*)out + 4 * nvec, tail);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(256) axpy_kernel(T* __restrict__ y, const T* __restrict__ x, T a, int64_t N) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] += a * x[i];
}
template <typename T>
hipError_t launch_axpy(T* y, const T* x, T a, int64_t N, hipStream_t st) {
    int64_t nb = (N + 255) / 256;
    if (nb > 8192) nb = 8192;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(axpy_kernel<T>, dim3((unsigned)nb), dim3(256), 0, st, y, x, a, N);
    return hipGetLastError();
}

#define ASD_INST(T)                                                                          \
    template hipError_t launch_permute<T>(const T*, T*, const int*, const int64_t*, hipStream_t); \
    template hipError_t launch_reduce<T>(const T*, int64_t, const ReduceParams&, int, hipStream_t); \
    template hipError_t launch_copy<T>(const T*, T*, int64_t, hipStream_t);                  \
    template hipError_t launch_axpy<T>(T*, const T*, T, int64_t, hipStream_t);
ASD_INST(float)
ASD_INST(double)
#undef ASD_INST

}  // namespace asd
