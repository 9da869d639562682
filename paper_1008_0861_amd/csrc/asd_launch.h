// Kernel parameter blocks and launchers of libasd (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "asd_device.h"

namespace asd {

// Fused FP64 reduction of a state, without any cross-block fence: the
// producing launch writes one (sum, min, max) partial per block; a later
// fold_kernel launch on the same stream folds them in a fixed order, so the
// result is deterministic and the kernel boundary makes the partials
// visible.  One fold launch can finish several reductions (consecutive
// steps' partials, slot_stride doubles apart): block b folds reduction b.
struct ReduceParams {
    double* partials;    // 3 doubles per block; nullptr disables the reduction
};
struct FoldParams {
    const double* partials;  // nullptr: nothing to fold
    int nblocks;         // producing blocks per reduction
    int count;           // reductions folded by this launch
    int slot_stride;     // doubles between the partials of consecutive reductions
    double* energy_out;  // nullable: receives sum * dV, one value per reduction
    double* series_out;  // nullable: receives {sum * dV, min, max} per reduction
    double* stats_out;   // nullable: {sum * dV, min, max} of the last reduction
    unsigned* flags;     // nullable: ORed with status bits
    const double* e0;    // nullable: reference energy for the drift flag
    int e0_slot0;        // the drift reference is reduction 0 of this launch (each block folds it too)
    double dV;
};

template <typename T>
struct SweepParams {
    const T* U;       // input state
    T* out;           // output state (never aliases U)
    const T* alpha;   // normal coefficient of the face after each cell, in U's layout
    const T* beta1;   // transverse coefficient (axis t1) of that face
    const T* beta2;   // transverse coefficient (axis t2), 3-D only
    int n;            // line length (input is contiguous along the line)
    int nt1, nt2;     // lines along transverse axes 1, 2 (nt2 = 1 in 2-D)
    int si_n, si_t1, si_t2;  // input strides, elements
    int so_n, so_t1, so_t2;  // output strides, elements
    // nseg_log2 completes the 16-byte block of the output strides: every
    // sweep instantiation uses all four, so the kernel's one scalar load of
    // them has no dead register that the compiler could reuse (and wait for)
    // before the wave's first global load
    int nseg_log2;    // log2(P)
    int periodic;
    int dirichlet;    // T = 0 walls: odd ghosts; the wrap-face entries of alpha / beta1
                      // hold the right / left wall coefficients of the line
    const T* Q;       // source added to the right-hand side (nullptr: none), U's layout
    T dtq;            // its factor (dt)
    int limiter;
    int wpl;          // waves per line
    int lpw;          // lines per workgroup
    int P;            // segments per line: power of two, <= 64*wpl, <= n
    int spl_log2;     // log2(64*wpl)
    int io_log2;      // log2(io): staging and stores use 64*wpl*io threads per line (io = 1 or 2)
    int lpw_log2;     // log2(lpw)
    int rhs_mode;     // 0: full sweep; 1: solve only (right-hand side = U)
    int red_in;       // the block partials reduce the input state (each cell once) instead of the output
    TileLayout lds;   // LDS layout of a tile (tile_layout / tile_layout_cell)
    ReduceParams red;
    // nullable: the output written a second time in U's layout (transposed-
    // output sweeps, EXT instantiations).  Last, so that the fields before it
    // keep the offsets the kernels' first scalar loads are laid out for.
    T* out2;
};

// Face coefficients of the sweep along axis d, written in that sweep's
// input layout (out strides): for every cell c, the face between c and
// c + e_d (wrapping when periodic; zero for an insulating wall face).  With
// T = 0 walls the entry of the last cell of each line holds the two wall
// coefficients: alpha = that of the right wall (from the last cell's b and
// chi), beta1 = that of the left wall (from the first cell's), beta2 = 0.
template <typename T>
struct CoefParams {
    const T* b[3];       // cell-centred b, x-fastest
    const T* chi;        // per-cell chi or nullptr
    const T* U;          // chi from this state (sweep-input layout), or nullptr
    double chi_exp, chi_tref;  // chi = chi_par (U / chi_tref)^chi_exp when U is set
    T* alpha;
    T* beta1;
    T* beta2;            // 3-D only
    int n[3];
    int d, t1, t2;       // sweep axis and the two transverse axes
    int so[3];           // output stride of axes x, y, z
    double cnn, ct1, ct2;  // dt/h_d^2, dt/(h_d h_t1), dt/(h_d h_t2)
    double chi_par, chi_perp;
    int periodic, dirichlet, ndim;
};
template <typename T>
hipError_t launch_coef(const CoefParams<T>& C, hipStream_t st);

// Largest workgroup of a sweep instantiation (register budget of the
// per-lane segment arrays, about eleven arrays of MMAX values): FP32 keeps
// segments of up to 16 cells within 128 registers, i.e. four waves per
// SIMD; FP64 needs twice the registers per value.
__host__ __device__ constexpr int sweep_max_threads(int es, int mmax) {
    return es == 4 ? 1024 : (es * mmax >= 128 ? 256 : (es * mmax >= 64 ? 512 : 1024));
}

template <typename T, int MMAX>
struct SweepBounds {
    static constexpr int bytes = (int)sizeof(T) * MMAX;
    static constexpr int max_threads = sweep_max_threads((int)sizeof(T), MMAX);
};
// The two tile bodies of a sweep (same result; see sweep.hip).
enum SweepVariant : int { SWEEP_FACE_SLOTS = 0, SWEEP_CELL_SLOTS = 1 };
// The cell-slot variant keeps seven arrays of MMAX values per lane.
__host__ __device__ constexpr int sweep_cell_max_threads(int es, int mmax) {
    return es * mmax >= 128 ? 256 : (es * mmax >= 32 ? 512 : 1024);
}
template <typename T, int MMAX>
struct SweepCellBounds {
    static constexpr int max_threads = sweep_cell_max_threads((int)sizeof(T), MMAX);
};
template <typename T>
hipError_t launch_sweep(const SweepParams<T>& P, int ndim, int mmax, dim3 grid, dim3 block,
                        size_t lds, hipStream_t st, int variant);
hipError_t sweep_set_lds_limits(int bytes);

// ---------------------------------------------------------------- explicit
template <typename T>
struct ExplicitParams {
    const T* U;
    T* out;
    const T* b[3];
    const T* chi;
    double chi_exp, chi_tref;  // != 0: per-cell chi = chi_par (U / chi_tref)^chi_exp
    int n[3];
    T cn[3];         // dt / h_d^2
    T ct[3][3];      // dt / (h_d h_t)
    T chi_par, chi_perp;
    int periodic;
    int dirichlet;   // T = 0 walls: odd ghosts, wall faces carry normal flux
    const T* Q;      // source (nullptr: none): out += dtq Q
    T dtq;
    int limiter;
    ReduceParams red;
};
template <typename T>
hipError_t launch_explicit(const ExplicitParams<T>& P, int ndim, hipStream_t st, int* nblocks_out);
int explicit_num_blocks(int ndim, const int n[3]);

// ------------------------------------------------------------------- batch
// One problem of a batch: its x sweep (T -> T*, transposed) and y sweep
// (T* -> T), the number of line groups (tiles) of each, the per-lane
// capacity of each sweep's tiles (the batch's MMAX, or half of it when the
// problem's lines fit: a shorter line then runs the smaller tile instead of
// padding every lane to the batch's capacity), where its y-sweep tiles start
// in the batch-wide tile numbering, and its cell volume.
template <typename T>
struct BatchProblem {
    SweepParams<T> sweep[2];
    int ngroups[2];
    int mmax[2];
    int half[2];  // two lines per wave (capacity-16 face-body tiles of 257-512-cell lines)
    int tile0;        // first y-sweep tile of this problem among all problems' y-sweep tiles
    int dirichlet;    // T = 0 walls (the energy is not conserved: no drift flag)
    double dV;
};
// Per-problem FP64 outputs of a batch call (all nullable together: energy
// == nullptr switches them off).
struct BatchOut {
    double* energy;       // [nprob][stride]: sum T dV of the initial state and after every step
    int stride;           // nsteps + 1 of the call
    int first;            // entry written by the next reduction (grouped-mode folds)
    unsigned* flags;      // [nprob]: ORed status bits (NONFINITE 1, NEG_T 2, ENERGY_DRIFT 4)
    double* stats;        // [3 nprob]: E, min T, max T after the call's last step
    double* partials;     // grouped schedule: per-tile (sum, min, max) of the y sweeps, a ring of slots
    int slot_stride;      // doubles between the ring's slots
    int count;            // grouped-mode fold: slots to fold
    int last;             // grouped-mode fold: the fold that reaches the call's last step
};
template <typename T>
hipError_t launch_batch_persistent(const BatchProblem<T>* probs, const int* off, const int* list, int nwg, int nsteps,
                                   int mmax, int nthreads, size_t lds, int limiter, int dirichlet, int variant,
                                   const BatchOut& out, hipStream_t st);
template <typename T>
hipError_t launch_batch_grouped(const BatchProblem<T>* probs, const int* group_start, int nprob, int ngroups, int d,
                                int mmax, int nthreads, size_t lds, int limiter, int dirichlet, int variant,
                                double* partials, hipStream_t st);
// Energy of every problem's current state into out.energy[p * stride + 0].
template <typename T>
hipError_t launch_batch_reduce0(const BatchProblem<T>* probs, int nprob, const BatchOut& out, hipStream_t st);
// Fold out.count ring slots of grouped-mode y-sweep partials into the
// entries out.first .. out.first + count - 1 of every problem.
template <typename T>
hipError_t launch_batch_fold(const BatchProblem<T>* probs, int nprob, const BatchOut& out, hipStream_t st);
hipError_t batch_set_lds_limits(int bytes);

// ----------------------------------------------------------------- adjoint
// Reverse mode of one 2-D sweep along d (adjoint.hip); arrays x-fastest.
template <typename T>
struct AdjParams {
    const T* mu;      // A_d^-1 lambda
    const T* U;       // the sweep's input state
    const T* X;       // the sweep's output state
    const T* b[2];
    const T* chi;     // per-cell chi or nullptr (then chi_par)
    T* lam_out;       // mu + J_S^T mu
    T* gchi;          // nullable: += dL/dchi per cell
    int nx, ny, d;
    double dt, hn, ht, chi_par, chi_perp;
    double ka, kb;    // dt / hn^2 and dt / (hn ht): alpha_f = ka chi_f b_n^2, beta_f = kb (chi_f - chi_perp) b_n b_t
    int periodic, limiter;
    int lam_b;        // 1: lam_out is written y-fastest ("layout B"), else x-fastest
};
template <typename T>
hipError_t launch_adjoint_stencil(const AdjParams<T>& P, hipStream_t st);

// --------------------------------------------------------------- utilities
// out[perm] = in: copy a dense (nz, ny, nx) array into another axis order.
// dst_stride[d] is the destination stride of source axis d (x=0, y=1, z=2).
template <typename T>
hipError_t launch_permute(const T* in, T* out, const int n[3], const int64_t dst_stride[3],
                          hipStream_t st);
// Standalone FP64 reduction of a dense array of N elements (partials only).
template <typename T>
hipError_t launch_reduce(const T* x, int64_t N, const ReduceParams& red, int nblocks, hipStream_t st);
// One block folding the partials of an earlier launch.
hipError_t launch_fold(const FoldParams& f, hipStream_t st);
int reduce_num_blocks(int64_t N);
hipError_t launch_fill_u32(unsigned* p, unsigned v, int64_t count, hipStream_t st);
hipError_t launch_fill_f64(double* p, double v, int64_t count, hipStream_t st);
template <typename T>
hipError_t launch_copy(const T* in, T* out, int64_t N, hipStream_t st);
template <typename T>
hipError_t launch_axpy(T* y, const T* x, T a, int64_t N, hipStream_t st);
// Streaming copy of nbytes (a multiple of 4) with 16-byte accesses where
// both pointers are 16-byte aligned.
hipError_t launch_copy_wide(const void* in, void* out, size_t nbytes, hipStream_t st);

// ------------------------------------------------- block reduction epilogue
// Block-wide (sum, min, max); every thread must call it.  Writes the
// block's partial.
template <typename M>
__device__ __forceinline__ void block_partials(double* partials, double s, M mn, M mx) {
    __shared__ double red_s[16], red_mn[16], red_mx[16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    s = wave_sum_lane63(s);
    mn = wave_min_lane63<M>(mn);
    mx = wave_max_lane63<M>(mx);
    if (lane == 63) { red_s[wid] = s; red_mn[wid] = (double)mn; red_mx[wid] = (double)mx; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ts = 0.0, tmn = red_mn[0], tmx = red_mx[0];
        for (int w = 0; w < nw; ++w) {
            ts += red_s[w];
            tmn = fmin(tmn, red_mn[w]);
            tmx = fmax(tmx, red_mx[w]);
        }
        double* pp = partials + 3 * (size_t)blockIdx.x;
        pp[0] = ts;
        pp[1] = tmn;
        pp[2] = tmx;
    }
}

// Block-wide fold of nblocks partials (sum, min, max) in a fixed order
// (thread i takes i, i+nthreads, ..., then a fixed tree); thread 0 gets
// the result.  Every thread must call it.
__device__ __forceinline__ void fold_slot(const double* part, int nblocks, double& S, double& MN, double& MX) {
    __shared__ double fs[16], fmn[16], fmx[16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    double ts = 0.0, tmn = __builtin_huge_val(), tmx = -__builtin_huge_val();
    for (int i = threadIdx.x; i < nblocks; i += blockDim.x) {
        const double* pp = part + 3 * (size_t)i;
        ts += pp[0];
        tmn = fmin(tmn, pp[1]);
        tmx = fmax(tmx, pp[2]);
    }
    ts = wave_sum_lane63(ts);
    tmn = wave_min_lane63<double>(tmn);
    tmx = wave_max_lane63<double>(tmx);
    if (lane == 63) { fs[wid] = ts; fmn[wid] = tmn; fmx[wid] = tmx; }
    __syncthreads();
    S = 0.0;
    MN = fmn[0];
    MX = fmx[0];
    if (threadIdx.x == 0) {
        for (int w = 0; w < nw; ++w) {
            S += fs[w];
            MN = fmin(MN, fmn[w]);
            MX = fmax(MX, fmx[w]);
        }
    }
    __syncthreads();  // fs may be refilled by the next call
}

// Fold reduction b = blockIdx.x of f.
__device__ __forceinline__ void fold_partials(const FoldParams& f) {
    const int b = blockIdx.x;
    double S, MN, MX;
    fold_slot(f.partials + (size_t)b * f.slot_stride, f.nblocks, S, MN, MX);
    // drift reference folded by this block too, in the same order as block 0
    double S0 = 0.0, MN0, MX0;
    if (f.e0_slot0 && b > 0) fold_slot(f.partials, f.nblocks, S0, MN0, MX0);
    if (threadIdx.x == 0) {
        const double E = S * f.dV;
        if (f.energy_out) f.energy_out[b] = E;
        if (f.series_out) { f.series_out[3 * b] = E; f.series_out[3 * b + 1] = MN; f.series_out[3 * b + 2] = MX; }
        if (f.stats_out && b == f.count - 1) { f.stats_out[0] = E; f.stats_out[1] = MN; f.stats_out[2] = MX; }
        if (f.flags) {
            unsigned fl = 0;
            // isfinite, not x - x != 0: with contraction E - E becomes
            // fma(S, dV, -E), the product's rounding error
            if (!__builtin_isfinite(E) || !__builtin_isfinite(MN) || !__builtin_isfinite(MX)) fl |= 1u;
            if (MN < 0.0) fl |= 2u;
            if (f.e0 || (f.e0_slot0 && b > 0)) {
                const double e0 = f.e0 ? *f.e0 : S0 * f.dV;
                if (fabs(E - e0) > 1e-6 * fabs(e0)) fl |= 4u;
            }
            if (fl) atomicOr(f.flags, fl);
        }
    }
}

}  // namespace asd
