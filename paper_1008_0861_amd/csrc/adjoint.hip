// Reverse mode of one directional sweep (2-D).
//
// Forward sweep along axis d (section 2, Eq. xup / yup):
//     x = A_d^-1 (U + S_d(U)),   A_d = I + sum_f alpha_f (e_c - e_c')(e_c - e_c')^T,
//     S_d(U)_c = F_{c+1/2} - F_{c-1/2},  F_f = beta_f G_f(U),
//     G_f = L(sigma_c', sigma_c),  sigma_c = L(U[c+e_t] - U[c], U[c] - U[c-e_t]),
// with c' = c + e_d.  Given mu = A_d^-1 lambda (A_d is symmetric, so the
// same line solver gives it), the input adjoint is
//     lambda_U = mu + J_S(U)^T mu,
// and the face parameters receive
//     dL/dalpha_f = -(mu_c - mu_c') (x_c - x_c'),   dL/dbeta_f = (mu_c - mu_c') G_f,
// chained to the face diffusivity (alpha, beta are linear in chi_f) and
// through the harmonic mean to the two cells' chi.
//
// One fused gather kernel per sweep axis, no atomics: per face, the weights
// w_f dG/dsigma (w_f = beta_f (mu_c - mu_c')) and dL/dchi_f; per cell, the
// contributions of its own slope and of the slopes of its two transverse
// neighbours, and its two faces' chi terms.
// Arithmetic is FP64 inside; arrays are x-fastest ("layout A").
// Limiter derivatives: zero where a*b <= 0 (kinks included); minmod takes
// its first argument on |a| == |b|; MC takes 2a, then 2b, then (a+b)/2.
#include "asd_device.h"
#include "asd_launch.h"

namespace asd {

// value and partial derivatives of the two-argument limiter (van Leer's
// quotients through a refined reciprocal, as in the forward sweeps)
__device__ __forceinline__ double dlim2(int lim, double a, double b, double* d1, double* d2) {
    if (lim == LIM_LINEAR) {
        *d1 = 0.5;
        *d2 = 0.5;
        return 0.5 * (a + b);
    }
    *d1 = 0.0;
    *d2 = 0.0;
    if (!(a * b > 0.0)) return 0.0;
    if (lim == LIM_VANLEER) {
        const double r = fast_rcp<double>(a + b), r2 = r * r;
        *d1 = 2.0 * b * b * r2;
        *d2 = 2.0 * a * a * r2;
        return 2.0 * a * b * r;
    }
    if (lim == LIM_MINMOD) {
        if (fabs(a) <= fabs(b)) { *d1 = 1.0; return a; }
        *d2 = 1.0;
        return b;
    }
    // MC
    double m, m1, m2;
    if (fabs(2.0 * a) <= fabs(2.0 * b)) { m = 2.0 * a; m1 = 2.0; m2 = 0.0; }
    else { m = 2.0 * b; m1 = 0.0; m2 = 2.0; }
    const double mean = 0.5 * (a + b);
    if (fabs(m) <= fabs(mean)) { *d1 = m1; *d2 = m2; return m; }
    *d1 = 0.5;
    *d2 = 0.5;
    return mean;
}

// ------------------------------------------------ fused streaming kernels
// One wave per band of AdjStream::TY rows and 64 columns (lane = column):
// the face quantities stay in registers, neighbours across columns come by
// lane shifts and across rows from registers.
struct AdjStream {
    static constexpr int TY = 2;     // rows per wave
    static constexpr int WAVES = 4;  // waves per block
};

__device__ __forceinline__ double lane_from_right(double v) { return __shfl_down(v, 1, 64); }
__device__ __forceinline__ double lane_from_left(double v) { return __shfl_up(v, 1, 64); }

// Coordinate c of a cell up to two cells outside [0, n): periodic wrap or
// insulating clamp.  Halo lanes farther out hold values no updated cell
// uses; they are clamped to a valid index.
__device__ __forceinline__ int adj_nb(int c, int n, bool periodic) {
    if (c < 0) return periodic && c + n >= 0 ? c + n : 0;
    if (c >= n) return periodic && c - n < n ? c - n : n - 1;
    return c;
}

// Face quantities between cells 0 and 1 along the face normal: weights to
// the slopes of cell 1 (W1) and cell 0 (W2), and dL/dchi_f (GF).
template <typename T>
__device__ __forceinline__ void adj_face(const AdjParams<T>& P, double s0, double s1, double bn0, double bn1, double bt0,
                                         double bt1, double c0, double c1, double mu0, double mu1, double x0, double x1,
                                         double& W1, double& W2, double& GF) {
    double LG1, LG2;
    const double Gf = dlim2(P.limiter, s1, s0, &LG1, &LG2);
    const double bn = 0.5 * (bn0 + bn1);
    const double bt = 0.5 * (bt0 + bt1);
    double chif = P.chi_par;
    if (P.chi) chif = (c0 + c1) != 0.0 ? 2.0 * c0 * c1 * fast_rcp<double>(c0 + c1) : 0.0;
    const double dpar = chif - P.chi_perp;
    const double beta = P.dt * dpar * bn * bt / (P.hn * P.ht);
    const double dm = mu0 - mu1;
    const double w = beta * dm;
    W1 = w * LG1;
    W2 = w * LG2;
    const double dLdalpha = -dm * (x0 - x1);
    const double dLdbeta = dm * Gf;
    GF = dLdalpha * P.dt * bn * bn / (P.hn * P.hn) + dLdbeta * P.dt * bn * bt / (P.hn * P.ht);
}

// d/dchi of the harmonic face mean, times the face's dL/dchi_f
__device__ __forceinline__ double adj_chi_term(double gf, double cj, double co) {
    const double s = cj + co;
    if (s == 0.0) return 0.0;
    const double r = fast_rcp<double>(s);
    return gf * 2.0 * co * co * (r * r);
}

// Faces along x (d = 0), slopes along y: a wave updates the 62 columns
// between its halo lanes; rows y0-2 .. y0+TY+1 of U (slopes of the rows
// y0-1 .. y0+TY whose faces the band needs).
template <typename T>
__global__ void __launch_bounds__(256) adj_stream_x_kernel(AdjParams<T> P) {
    constexpr int TY = AdjStream::TY, NF = TY + 2, NU = TY + 4;
    const int nx = P.nx, ny = P.ny;
    const int lane = threadIdx.x & 63;
    const int blk = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    const int wave = blk * AdjStream::WAVES + (threadIdx.x >> 6);
    const int ncb = (nx + 61) / 62, nrb = (ny + TY - 1) / TY;
    if (wave >= ncb * nrb) return;  // wave-uniform; no block barrier follows
    const int cb = wave % ncb, rb = wave / ncb;
    const int x = cb * 62 - 1 + lane;
    const int y0 = rb * TY;
    const bool periodic = P.periodic != 0;
    const int xc = adj_nb(x, nx, periodic);
    double u[NU];
#pragma unroll
    for (int r = 0; r < NU; ++r) u[r] = (double)P.U[xc + adj_nb(y0 - 2 + r, ny, periodic) * nx];
    double mu[NF], X[NF], bn[NF], bt[NF], ch[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const int c = xc + adj_nb(y0 - 1 + f, ny, periodic) * nx;
        mu[f] = (double)P.mu[c];
        X[f] = (double)P.X[c];
        bn[f] = (double)P.b[0][c];
        bt[f] = (double)P.b[1][c];
        ch[f] = P.chi ? (double)P.chi[c] : P.chi_par;
    }
    const bool right_face = periodic || x + 1 <= nx - 1;  // face (x, x+1) lies inside
    const bool left_face = periodic || x - 1 >= 0;        // face (x-1, x) lies inside
    double psi[NF], l1[NF], l2[NF], gfr[NF], gfl[NF], chr[NF], chl[NF];
    bool us[NF], ds[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const int y = y0 - 1 + f;
        const double uc = u[f + 1];
        us[f] = !periodic && y + 1 > ny - 1;  // mirrored neighbours: the clamped loads give U_c
        ds[f] = !periodic && y - 1 < 0;
        const double sg = dlim2(P.limiter, u[f + 2] - uc, uc - u[f], &l1[f], &l2[f]);
        double W1, W2, GF;
        adj_face<T>(P, sg, lane_from_right(sg), bn[f], lane_from_right(bn[f]), bt[f], lane_from_right(bt[f]), ch[f],
                    lane_from_right(ch[f]), mu[f], lane_from_right(mu[f]), X[f], lane_from_right(X[f]), W1, W2, GF);
        if (!right_face) { W1 = 0.0; W2 = 0.0; GF = 0.0; }
        const double W1l = lane_from_left(W1), GFl = lane_from_left(GF);
        psi[f] = W2 + (left_face ? W1l : 0.0);
        gfr[f] = GF;
        gfl[f] = GFl;
        chr[f] = lane_from_right(ch[f]);
        chl[f] = lane_from_left(ch[f]);
    }
    // every lane shift is done: the halo lanes may leave
    if (lane < 1 || lane > 62 || x >= nx) return;
#pragma unroll
    for (int f = 1; f <= TY; ++f) {
        const int y = y0 - 1 + f;
        if (y >= ny) break;
        const int j = x + y * nx;
        double acc = mu[f] + psi[f] * ((us[f] ? 0.0 : -l1[f]) + (ds[f] ? 0.0 : l2[f]));
        if (periodic || y - 1 >= 0) acc += psi[f - 1] * l1[f - 1];
        if (periodic || y + 1 <= ny - 1) acc -= psi[f + 1] * l2[f + 1];
        P.lam_out[j] = (T)acc;
        if (P.gchi) {
            double g = 0.0;
            if (right_face) g += adj_chi_term(gfr[f], ch[f], chr[f]);
            if (left_face) g += adj_chi_term(gfl[f], ch[f], chl[f]);
            P.gchi[j] = (T)((double)P.gchi[j] + g);
        }
    }
}

// Faces along y (d = 1), slopes along x: a wave updates the 60 columns
// between two halo lanes on each side (an updated cell needs the slopes of
// its left and right neighbours, which need their own neighbours); rows
// y0-1 .. y0+TY.
template <typename T>
__global__ void __launch_bounds__(256) adj_stream_y_kernel(AdjParams<T> P) {
    constexpr int TY = AdjStream::TY, NF = TY + 2;
    const int nx = P.nx, ny = P.ny;
    const int lane = threadIdx.x & 63;
    const int blk = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    const int wave = blk * AdjStream::WAVES + (threadIdx.x >> 6);
    const int ncb = (nx + 59) / 60, nrb = (ny + TY - 1) / TY;
    if (wave >= ncb * nrb) return;  // wave-uniform; no block barrier follows
    const int cb = wave % ncb, rb = wave / ncb;
    const int x = cb * 60 - 2 + lane;
    const int y0 = rb * TY;
    const bool periodic = P.periodic != 0;
    const int xc = adj_nb(x, nx, periodic);
    double u[NF], mu[NF], X[NF], bn[NF], bt[NF], ch[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const int c = xc + adj_nb(y0 - 1 + f, ny, periodic) * nx;
        u[f] = (double)P.U[c];
        mu[f] = (double)P.mu[c];
        X[f] = (double)P.X[c];
        bn[f] = (double)P.b[1][c];
        bt[f] = (double)P.b[0][c];
        ch[f] = P.chi ? (double)P.chi[c] : P.chi_par;
    }
    // slopes along x of every row (mirrored neighbours: the clamped loads give U_c)
    const bool us = !periodic && x + 1 > nx - 1, ds = !periodic && x - 1 < 0;
    double sg[NF], l1[NF], l2[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f)
        sg[f] = dlim2(P.limiter, lane_from_right(u[f]) - u[f], u[f] - lane_from_left(u[f]), &l1[f], &l2[f]);
    // faces (f, f+1), f = 0 .. TY
    double W1[NF - 1], W2[NF - 1], GF[NF - 1];
#pragma unroll
    for (int f = 0; f < NF - 1; ++f) {
        const int y = y0 - 1 + f;
        adj_face<T>(P, sg[f], sg[f + 1], bn[f], bn[f + 1], bt[f], bt[f + 1], ch[f], ch[f + 1], mu[f], mu[f + 1], X[f],
                    X[f + 1], W1[f], W2[f], GF[f]);
        if (!(periodic || (y >= 0 && y + 1 <= ny - 1))) { W1[f] = 0.0; W2[f] = 0.0; GF[f] = 0.0; }
    }
    // psi of rows 1 .. TY, and the neighbours' contributions through their slopes
    double psi[NF], from_l[NF], from_r[NF];
#pragma unroll
    for (int f = 1; f <= TY; ++f) {
        const int y = y0 - 1 + f;
        psi[f] = W2[f] + ((periodic || y - 1 >= 0) ? W1[f - 1] : 0.0);
        from_l[f] = lane_from_left(psi[f] * l1[f]);   // psi(x-1) d sigma(x-1)/dp
        from_r[f] = lane_from_right(psi[f] * l2[f]);  // psi(x+1) d sigma(x+1)/dq
    }
    // every lane shift is done: the halo lanes may leave
    if (lane < 2 || lane > 61 || x >= nx) return;
#pragma unroll
    for (int f = 1; f <= TY; ++f) {
        const int y = y0 - 1 + f;
        if (y >= ny) break;
        const int j = x + y * nx;
        double acc = mu[f] + psi[f] * ((us ? 0.0 : -l1[f]) + (ds ? 0.0 : l2[f]));
        if (periodic || x - 1 >= 0) acc += from_l[f];
        if (periodic || x + 1 <= nx - 1) acc -= from_r[f];
        P.lam_out[j] = (T)acc;
        if (P.gchi) {
            double g = 0.0;
            if (periodic || y + 1 <= ny - 1) g += adj_chi_term(GF[f], ch[f], ch[f + 1]);
            if (periodic || y - 1 >= 0) g += adj_chi_term(GF[f - 1], ch[f], ch[f - 1]);
            P.gchi[j] = (T)((double)P.gchi[j] + g);
        }
    }
}
template <typename T>
hipError_t launch_adjoint_stencil(const AdjParams<T>& P, hipStream_t st) {
    const int cols = P.d == 0 ? 62 : 60;
    const long waves = (long)((P.nx + cols - 1) / cols) * ((P.ny + AdjStream::TY - 1) / AdjStream::TY);
    long nb = (waves + AdjStream::WAVES - 1) / AdjStream::WAVES;
    nb = (nb + 7) & ~7L;  // a multiple of 8 for the XCD-aware block order
    if (P.d == 0)
        hipLaunchKernelGGL(adj_stream_x_kernel<T>, dim3((unsigned)nb), dim3(64 * AdjStream::WAVES), 0, st, P);
    else
        hipLaunchKernelGGL(adj_stream_y_kernel<T>, dim3((unsigned)nb), dim3(64 * AdjStream::WAVES), 0, st, P);
    return hipGetLastError();
}

template hipError_t launch_adjoint_stencil<float>(const AdjParams<float>&, hipStream_t);
template hipError_t launch_adjoint_stencil<double>(const AdjParams<double>&, hipStream_t);

}  // namespace asd
