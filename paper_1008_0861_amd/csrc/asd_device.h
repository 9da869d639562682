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

// LDS layout of one sweep tile (byte offsets; computed by the host, stored
// in the sweep parameters).  Each line of the tile owns a row of face
// slots of two elements [A, PHI]: the normal coefficient alpha and the
// face flux Phi of the face after the cell (computed once, while the tile
// is staged).  The back substitution writes the solved increment over PHI
// for the store phase.  A few spare slots follow the n slots of a line, so
// that a lane may read a whole MMAX-cell window past the line's end (the
// values there are ignored).  When every segment of the line has the same
// power-of-two length, a 16-byte pad follows every 2^pad slots, 2^pad being
// the distance between the segments of neighbouring lanes, so that those
// lanes hit distinct banks; no segment then contains a pad, and a segment's
// slots are always consecutive.  When several waves share a line, the
// interface reduction exchanges through two buffers with one 4-element
// entry per thread; on aligned tiles with segments of at least 8 cells the
// buffers live in the segments' own face slots instead (no extra bytes).
__host__ __device__ inline int slot_off(int p, int es, int pad) { return p * 2 * es + ((p >> pad) << 4); }

static constexpr int kRowSpare = 17;  // spare slots after the n face slots of a line

struct TileLayout {
    int aligned;   // every segment has the kernel's maximal length (pads in use)
    int pad;       // log2 of the slots per pad (30: no pad)
    int row1;      // bytes per line, slot rows
    int pcr0_at;   // offset of exchange buffer 0 (several waves per line)
    int pcr1_at;   // offset of exchange buffer 1 (cell-slot layout: -1 = inside the slot rows)
    int total;     // bytes
    int row2;      // cell-slot layout, 3-D: bytes per line of the pair rows
    int rows2_at;  // cell-slot layout, 3-D: offset of the pair rows
};

__host__ __device__ inline TileLayout tile_layout(int es, int ndim, int n, int lpw, int nthreads, int wpl,
                                                  int nseg_log2, int mmax) {
    (void)ndim;
    TileLayout L;
    L.row2 = 0;
    L.rows2_at = 0;
    const int m = n >> nseg_log2;
    L.aligned = (m << nseg_log2) == n && m == mmax;  // mmax is a power of two
    L.pad = 30;
    if (L.aligned && m * wpl >= 2) {
        int l = 0;
        while ((2 << l) <= m * wpl) ++l;
        L.pad = l;  // 2^pad = m * wpl: segments of neighbouring lanes
    }
    int r1 = (slot_off(n + kRowSpare, es, L.pad) + 15) & ~15;
    if (((r1 >> 4) & 1) == 0) r1 += 16;  // odd number of 16-byte units: rows start in different banks
    L.row1 = r1;
    int at = lpw * r1;
    L.pcr0_at = at;
    L.pcr1_at = at;
    // several waves per line exchange through two buffers, except on aligned
    // tiles of at least 8 cells per segment, which keep them in face slots
    if (wpl > 1 && !(L.aligned && m >= 8)) {
        L.pcr1_at = at + nthreads * 4 * es;
        at += 2 * nthreads * 4 * es;
    }
    L.total = at;
    return L;
}

// The cell-slot layout of the second sweep variant (sweep_cell.h): each
// line owns a row of cell slots of four elements [S1, A, B1, U] (the
// limited transverse slope, the normal and transverse coefficients of the
// face after the cell, and the state, replaced by the solution once the
// line is solved); in 3-D a second row holds the pairs [S2, B2].  Slot n
// repeats cell 0 and a few spare slots follow.  Pads as in tile_layout.
// With several waves per line the interface reduction has two exchange
// buffers of one slot per thread; the second lives in the dead [S1, A, B1]
// part of the line's first slots when the line has at least as many cells
// as lanes (pcr1_at = -1).
__host__ __device__ inline int cell_off1(int p, int es, int pad) { return p * 4 * es + ((p >> pad) << 4); }
__host__ __device__ inline int cell_off2(int p, int es, int pad) { return (p + (p >> pad)) * 2 * es; }

__host__ __device__ inline TileLayout tile_layout_cell(int es, int ndim, int n, int lpw, int nthreads, int wpl,
                                                       int nseg_log2, int mmax) {
    TileLayout L;
    const int m = n >> nseg_log2;
    L.aligned = (m << nseg_log2) == n && m == mmax;
    L.pad = 30;
    if (L.aligned && m * wpl >= 2) {
        int l = 0;
        while ((2 << l) <= m * wpl) ++l;
        L.pad = l;
    }
    int r1 = cell_off1(n + 1 + kRowSpare, es, L.pad);
    if (((r1 >> 4) & 1) == 0) r1 += 16;
    L.row1 = r1;
    int r2 = 0;
    if (ndim == 3) {
        r2 = (cell_off2(n + 1 + kRowSpare, es, L.pad) + 15) & ~15;
        if (((r2 >> 4) & 1) == 0) r2 += 16;
    }
    L.row2 = r2;
    L.rows2_at = lpw * r1;
    int at = L.rows2_at + lpw * r2;
    L.pcr0_at = at;
    L.pcr1_at = -1;
    if (wpl > 1) {
        at += nthreads * 4 * es;
        if (64 * wpl > n) {
            L.pcr1_at = at;
            at += nthreads * 4 * es;
        }
    }
    L.total = at;
    return L;
}

// 16-byte-aligned LDS accesses of slots (4 elements), triples and pairs.
template <typename T>
__device__ __forceinline__ void lds_put4(unsigned char* p, T a, T b, T c, T d);
template <>
__device__ __forceinline__ void lds_put4<float>(unsigned char* p, float a, float b, float c, float d) {
    *reinterpret_cast<float4*>(p) = make_float4(a, b, c, d);
}
template <>
__device__ __forceinline__ void lds_put4<double>(unsigned char* p, double a, double b, double c, double d) {
    reinterpret_cast<double2*>(p)[0] = make_double2(a, b);
    reinterpret_cast<double2*>(p)[1] = make_double2(c, d);
}
template <typename T>
__device__ __forceinline__ void lds_get4(const unsigned char* p, T& a, T& b, T& c, T& d);
template <>
__device__ __forceinline__ void lds_get4<float>(const unsigned char* p, float& a, float& b, float& c, float& d) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    a = v.x; b = v.y; c = v.z; d = v.w;
}
template <>
__device__ __forceinline__ void lds_get4<double>(const unsigned char* p, double& a, double& b, double& c,
                                                 double& d) {
    const double2 v0 = reinterpret_cast<const double2*>(p)[0];
    const double2 v1 = reinterpret_cast<const double2*>(p)[1];
    a = v0.x; b = v0.y; c = v1.x; d = v1.y;
}
// Global load at a 32-bit byte offset from a wave-uniform base (a scalar
// base plus a vector offset, no 64-bit address arithmetic per load).
template <typename T>
__device__ __forceinline__ T ldg_off(const T* base, unsigned byte_off) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const unsigned char*>(base) + byte_off);
}
template <typename T>
__device__ __forceinline__ void stg_off(T* base, unsigned byte_off, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<unsigned char*>(base) + byte_off) = v;
}

// first three elements of a slot only (the fourth is left untouched)
template <typename T>
__device__ __forceinline__ void lds_put3(unsigned char* p, T a, T b, T c) {
    T* q = reinterpret_cast<T*>(p);
    q[0] = a;
    q[1] = b;
    q[2] = c;
}
template <typename T>
__device__ __forceinline__ void lds_put2(unsigned char* p, T a, T b) {
    T* q = reinterpret_cast<T*>(p);
    q[0] = a;
    q[1] = b;
}
template <typename T>
__device__ __forceinline__ void lds_get2(const unsigned char* p, T& a, T& b) {
    const T* q = reinterpret_cast<const T*>(p);
    a = q[0];
    b = q[1];
}

// Wave reductions with DPP lane moves, in a fixed order: pairs, quads,
// half rows and rows of 16 lanes; then rows 1 and 3 take rows 0 and 2, and
// rows 2-3 take row 1.  Lane 63 ends with the result over all 64 lanes.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_f32(float old, float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL, ROWS, 0xf, false));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double old, double v) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), CTRL, ROWS, 0xf, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL, int ROWS, typename T>
__device__ __forceinline__ T dpp_mov(T old, T v) {
    if constexpr (sizeof(T) == 8) return dpp_f64<CTRL, ROWS>(old, v);
    else return dpp_f32<CTRL, ROWS>(old, v);
}
enum : int { DPP_QP_1032 = 0xB1, DPP_QP_2301 = 0x4E, DPP_ROW_MIRROR = 0x140, DPP_ROW_HALF_MIRROR = 0x141,
             DPP_ROW_BCAST15 = 0x142, DPP_ROW_BCAST31 = 0x143 };

__device__ __forceinline__ double wave_sum_lane63(double v) {
    v += dpp_mov<DPP_QP_1032, 0xf>(0.0, v);
    v += dpp_mov<DPP_QP_2301, 0xf>(0.0, v);
    v += dpp_mov<DPP_ROW_HALF_MIRROR, 0xf>(0.0, v);
    v += dpp_mov<DPP_ROW_MIRROR, 0xf>(0.0, v);
    v += dpp_mov<DPP_ROW_BCAST15, 0xa>(0.0, v);
    v += dpp_mov<DPP_ROW_BCAST31, 0xc>(0.0, v);
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_min_lane63(T v) {
    v = fmin(v, dpp_mov<DPP_QP_1032, 0xf>(v, v));
    v = fmin(v, dpp_mov<DPP_QP_2301, 0xf>(v, v));
    v = fmin(v, dpp_mov<DPP_ROW_HALF_MIRROR, 0xf>(v, v));
    v = fmin(v, dpp_mov<DPP_ROW_MIRROR, 0xf>(v, v));
    v = fmin(v, dpp_mov<DPP_ROW_BCAST15, 0xa>(v, v));
    v = fmin(v, dpp_mov<DPP_ROW_BCAST31, 0xc>(v, v));
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_max_lane63(T v) {
    v = fmax(v, dpp_mov<DPP_QP_1032, 0xf>(v, v));
    v = fmax(v, dpp_mov<DPP_QP_2301, 0xf>(v, v));
    v = fmax(v, dpp_mov<DPP_ROW_HALF_MIRROR, 0xf>(v, v));
    v = fmax(v, dpp_mov<DPP_ROW_MIRROR, 0xf>(v, v));
    v = fmax(v, dpp_mov<DPP_ROW_BCAST15, 0xa>(v, v));
    v = fmax(v, dpp_mov<DPP_ROW_BCAST31, 0xc>(v, v));
    return v;
}

}  // namespace asd
