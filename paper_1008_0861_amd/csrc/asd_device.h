// Device-side helpers shared by the gfx950 kernels of libasd.
//
// Scheme: Sharma & Hammett, "A Fast Semi-implicit Method for Anisotropic
// Diffusion", section 2.  Face heat flux = normal part (implicit, one
// tridiagonal solve per grid line) + transverse part (explicit, built from a
// limited face difference of the temperature).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace asd {

enum Limiter : int { LIM_VANLEER = 0, LIM_MINMOD = 1, LIM_MC = 2, LIM_LINEAR = 3 };

// Reciprocals from the hardware approximation.  approx_rcp: FP32
// v_rcp_f32 as is (1 ulp, used inside the limiter, whose rounding cannot
// affect conservation).  fast_rcp: refined by Newton steps
// x <- x + x (1 - d x) (one in FP32, two in FP64), used by the line solves,
// where a biased reciprocal would bias the column sums of the inverse and
// make the total energy drift.
template <typename T>
__device__ __forceinline__ T approx_rcp(T d);
template <>
__device__ __forceinline__ float approx_rcp<float>(float d) {
    return __builtin_amdgcn_rcpf(d);
}
template <typename T>
__device__ __forceinline__ T fast_rcp(T d);
template <>
__device__ __forceinline__ float fast_rcp<float>(float d) {
    const float x = __builtin_amdgcn_rcpf(d);
    return fmaf(x, fmaf(-d, x, 1.0f), x);
}
template <>
__device__ __forceinline__ double fast_rcp<double>(double d) {
    double x = __builtin_amdgcn_rcp(d);
    double e = fma(-d, x, 1.0);
    x = fma(x, e, x);
    e = fma(-d, x, 1.0);
    return fma(x, e, x);
}
template <>
__device__ __forceinline__ double approx_rcp<double>(double d) {
    return fast_rcp<double>(d);
}

// Two-argument limiters of section 2: van Leer (Eq. vanLeer), minmod, and
// monotonised central (minmod of 2a, 2b, (a+b)/2); LINEAR is the plain mean
// used in the linear stability analysis (section 2.1).
template <typename T>
__device__ __forceinline__ T limit2(int lim, T a, T b) {
    const T ab = a * b;
    if (lim == LIM_LINEAR) return T(0.5) * (a + b);
    if (!(ab > T(0))) return T(0);
    if (lim == LIM_VANLEER) return T(2) * ab * approx_rcp<T>(a + b);
    const T aa = fabs(a), bb = fabs(b);
    T m;
    if (lim == LIM_MINMOD) {
        m = fmin(aa, bb);
    } else {  // LIM_MC
        m = fmin(fmin(T(2) * aa, T(2) * bb), T(0.5) * fabs(a + b));
    }
    return a > T(0) ? m : -m;
}

// Per-cell limited slope along a transverse axis: L(U+ - U, U - U-).
// The face difference of section 2 is then L(slope(c+e_d), slope(c)).
template <typename T>
__device__ __forceinline__ T cell_slope(int lim, T um, T u, T up) {
    return limit2<T>(lim, up - u, u - um);
}

// Harmonic mean of two diffusivities (face value of a per-cell chi).
template <typename T>
__device__ __forceinline__ T harmonic(T a, T b) {
    const T s = a + b;
    return s != T(0) ? T(2) * a * b / s : T(0);
}

// Neighbour coordinate along an axis of length n: periodic wrap or
// insulating mirror (the ghost cell repeats the wall cell).
__device__ __forceinline__ int64_t nb_coord(int64_t c, int64_t n, bool periodic) {
    if (c < 0) return periodic ? n - 1 : 0;
    if (c >= n) return periodic ? 0 : n - 1;
    return c;
}

// Shared-memory index with one pad element per 32 (FP32) / 16 (FP64)
// elements, so that lanes walking contiguous segments of a line hit
// distinct LDS banks.
template <typename T>
__device__ __forceinline__ int lds_pad(int p) {
    return sizeof(T) == 4 ? p + (p >> 5) : p + (p >> 4);
}
template <typename T>
__host__ __device__ inline int lds_line_stride(int n) {
    int s = (sizeof(T) == 4) ? n + (n >> 5) + 1 : n + (n >> 4) + 1;
    return s | 1;  // odd stride: consecutive lines start in different banks
}

// Wave / block reductions used by the fused FP64 energy epilogue.
__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

}  // namespace asd
