// Kernel parameter blocks and launchers of libasd (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace asd {

// Fused FP64 reduction of a state: per-block partials (sum, min, max), then
// the last block to finish (atomic ticket) folds them in a fixed order, so
// the result does not depend on block scheduling.
struct ReduceParams {
    double* partials;    // 3 doubles per block; nullptr disables the reduction
    unsigned* ticket;    // zero before the launch; reset to zero by the last block
    double* energy_out;  // nullable: receives sum * dV
    double* stats_out;   // nullable: {sum * dV, min, max}
    unsigned* flags;     // nullable: ORed with status bits
    const double* e0;    // nullable: reference energy for the drift flag
    double dV;
};

template <typename T>
struct SweepParams {
    const T* U;     // input state
    T* out;         // output state (never aliases U)
    const T* bn;    // b along the sweep axis, in U's layout
    const T* bt1;   // b along transverse axis 1
    const T* bt2;   // b along transverse axis 2 (3-D)
    const T* chi;   // per-cell chi in U's layout, or nullptr
    int n;          // line length
    int nt1, nt2;   // lines along transverse axes 1, 2 (nt2 = 1 in 2-D)
    int64_t si_n, si_t1, si_t2;  // input strides, elements
    int64_t so_n, so_t1, so_t2;  // output strides, elements
    T cnn;          // dt / h_n^2
    T cnt1, cnt2;   // dt / (h_n h_t1), dt / (h_n h_t2)
    T chi_par, chi_perp;
    int periodic;
    int limiter;
    int wpl;        // waves per line
    int lpw;        // lines per workgroup
    int P;          // segments per line: power of two, <= 64*wpl, <= n
    int rhs_mode;   // 0: full sweep; 1: solve only (right-hand side = U)
    ReduceParams red;
};

// Largest workgroup a sweep instantiation is compiled for (register budget
// of the per-lane segment arrays: seven arrays of MMAX values).
template <typename T, int MMAX>
struct SweepBounds {
    static constexpr int bytes = (int)sizeof(T) * MMAX;
    static constexpr int max_threads = bytes >= 64 ? 256 : (bytes >= 32 ? 512 : 1024);
};
template <typename T>
hipError_t launch_sweep(const SweepParams<T>& P, int ndim, int mmax, dim3 grid, dim3 block,
                        size_t lds, hipStream_t st);
hipError_t sweep_set_lds_limits(int bytes);

// ---------------------------------------------------------------- explicit
template <typename T>
struct ExplicitParams {
    const T* U;
    T* out;
    const T* b[3];
    const T* chi;
    int n[3];
    T cn[3];         // dt / h_d^2
    T ct[3][3];      // dt / (h_d h_t)
    T chi_par, chi_perp;
    int periodic;
    int limiter;
    ReduceParams red;
};
template <typename T>
hipError_t launch_explicit(const ExplicitParams<T>& P, int ndim, hipStream_t st, int* nblocks_out);
int explicit_num_blocks(int ndim, const int n[3]);

// --------------------------------------------------------------- utilities
// out[perm] = in: copy a dense (nz, ny, nx) array into another axis order.
// dst_stride[d] is the destination stride of source axis d (x=0, y=1, z=2).
template <typename T>
hipError_t launch_permute(const T* in, T* out, const int n[3], const int64_t dst_stride[3],
                          hipStream_t st);
// Standalone FP64 reduction of a dense array of N elements.
template <typename T>
hipError_t launch_reduce(const T* x, int64_t N, const ReduceParams& red, int nblocks, hipStream_t st);
int reduce_num_blocks(int64_t N);
hipError_t launch_fill_u32(unsigned* p, unsigned v, int64_t count, hipStream_t st);
hipError_t launch_fill_f64(double* p, double v, int64_t count, hipStream_t st);
template <typename T>
hipError_t launch_copy(const T* in, T* out, int64_t N, hipStream_t st);
template <typename T>
hipError_t launch_axpy(T* y, const T* x, T a, int64_t N, hipStream_t st);

// ------------------------------------------------- block reduction epilogue
__device__ __forceinline__ void block_reduce_and_finish(const ReduceParams& R, double s, double mn,
                                                        double mx) {
    __shared__ double red_s[16], red_mn[16], red_mx[16];
    __shared__ int last;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    for (int off = 32; off > 0; off >>= 1) {
        s += __shfl_xor(s, off, 64);
        mn = fmin(mn, __shfl_xor(mn, off, 64));
        mx = fmax(mx, __shfl_xor(mx, off, 64));
    }
    if (lane == 0) { red_s[wid] = s; red_mn[wid] = mn; red_mx[wid] = mx; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ts = 0.0, tmn = red_mn[0], tmx = red_mx[0];
        for (int w = 0; w < nw; ++w) {
            ts += red_s[w];
            tmn = fmin(tmn, red_mn[w]);
            tmx = fmax(tmx, red_mx[w]);
        }
        double* pp = R.partials + 3 * (size_t)blockIdx.x;
        pp[0] = ts;
        pp[1] = tmn;
        pp[2] = tmx;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned t = atomicAdd(R.ticket, 1u);
        last = (t == gridDim.x - 1) ? 1 : 0;
    }
    __syncthreads();
    if (!last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    // fixed-order fold: thread i takes partials i, i+nthreads, ...
    double ts = 0.0, tmn = __builtin_huge_val(), tmx = -__builtin_huge_val();
    for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x) {
        const volatile double* pp = R.partials + 3 * (size_t)b;
        ts += pp[0];
        tmn = fmin(tmn, pp[1]);
        tmx = fmax(tmx, pp[2]);
    }
    for (int off = 32; off > 0; off >>= 1) {
        ts += __shfl_xor(ts, off, 64);
        tmn = fmin(tmn, __shfl_xor(tmn, off, 64));
        tmx = fmax(tmx, __shfl_xor(tmx, off, 64));
    }
    __syncthreads();
    if (lane == 0) { red_s[wid] = ts; red_mn[wid] = tmn; red_mx[wid] = tmx; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double S = 0.0, MN = red_mn[0], MX = red_mx[0];
        for (int w = 0; w < nw; ++w) {
            S += red_s[w];
            MN = fmin(MN, red_mn[w]);
            MX = fmax(MX, red_mx[w]);
        }
        const double E = S * R.dV;
        if (R.energy_out) *R.energy_out = E;
        if (R.stats_out) { R.stats_out[0] = E; R.stats_out[1] = MN; R.stats_out[2] = MX; }
        if (R.flags) {
            unsigned f = 0;
            if (!(E == E) || E - E != 0.0 || !(MN == MN) || !(MX == MX) || MX - MX != 0.0) f |= 1u;
            if (MN < 0.0) f |= 2u;
            if (R.e0) {
                const double e0 = *R.e0;
                if (fabs(E - e0) > 1e-6 * fabs(e0)) f |= 4u;
            }
            if (f) atomicOr(R.flags, f);
        }
        *R.ticket = 0u;
    }
}

}  // namespace asd
