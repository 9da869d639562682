// Face coefficients of one sweep direction (section 2): at the face between
// cell c and c + e_d,
//     b_f     = (b_c + b_{c+e_d}) / 2      (arithmetic mean, not renormalised)
//     chi_f   = chi_par, or the harmonic mean of the two cells' chi (a per-cell
//               field, or chi_par (U / T_ref)^p of a state U, section 3.3)
//     alpha_f = dt (chi_perp + (chi_f - chi_perp) b_d,f^2) / h_d^2
//     beta_t  = dt (chi_f - chi_perp) b_d,f b_t,f / (h_d h_t)
// A wall face (c on the last plane) gets zeros, except with T = 0 walls:
// there the entry holds the wall coefficients of the line (the right wall's
// alpha in alpha, the left wall's in beta1), each from its own cell's b and
// chi, since the wall face has no second cell.
// Computed in FP64 and rounded once to the grid's type.  With a constant or
// per-cell chi they depend on dt, b and chi only and a step loop computes
// them once; with chi(T) they are recomputed from each sweep's input.
#include "asd_device.h"
#include "asd_launch.h"

namespace asd {

// chi of one cell: the per-cell field, chi_par (U / T_ref)^p of the state, or chi_par
template <typename T>
__device__ __forceinline__ double coef_cell_chi(const CoefParams<T>& C, int i, const int xyz[3]) {
    if (C.U) {
        // the state is in the output (sweep-input) layout
        const int o = xyz[0] * C.so[0] + xyz[1] * C.so[1] + xyz[2] * C.so[2];
        return C.chi_par * pow((double)C.U[o] / C.chi_tref, C.chi_exp);
    }
    if (C.chi) return (double)C.chi[i];
    return C.chi_par;
}

template <typename T>
__global__ void __launch_bounds__(256) coef_kernel(CoefParams<T> C) {
    const int nx = C.n[0], ny = C.n[1], nz = C.n[2];
    const int N = nx * ny * nz;
    // 64-bit loop index: the stride would overflow int near N = 2^31 (each i < N fits an int)
    for (int64_t i64 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i64 < N; i64 += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)i64;
        const int xyz[3] = {i % nx, (i / nx) % ny, i / (nx * ny)};
        int nbr[3] = {xyz[0], xyz[1], xyz[2]};
        nbr[C.d] += 1;
        const bool wall = nbr[C.d] == C.n[C.d] && !C.periodic;
        if (nbr[C.d] == C.n[C.d]) nbr[C.d] = 0;
        const int j = nbr[0] + nbr[1] * nx + nbr[2] * nx * ny;
        double a = 0.0, b1 = 0.0, b2 = 0.0;
        if (!wall) {
            double bf[3] = {0.0, 0.0, 0.0};
            for (int q = 0; q < C.ndim; ++q) bf[q] = 0.5 * ((double)C.b[q][i] + (double)C.b[q][j]);
            double chif = C.chi_par;
            if (C.U || C.chi) {
                const double x0 = coef_cell_chi(C, i, xyz), x1 = coef_cell_chi(C, j, nbr);
                chif = (x0 + x1) != 0.0 ? 2.0 * x0 * x1 / (x0 + x1) : 0.0;
            }
            const double dpar = chif - C.chi_perp;
            a = C.cnn * (C.chi_perp + dpar * bf[C.d] * bf[C.d]);
            b1 = C.ct1 * dpar * bf[C.d] * bf[C.t1];
            if (C.ndim == 3) b2 = C.ct2 * dpar * bf[C.d] * bf[C.t2];
        } else if (C.dirichlet) {
            // right wall from cell i (last of its line), left wall from cell j (first)
            const double bi = (double)C.b[C.d][i], bj = (double)C.b[C.d][j];
            a = C.cnn * (C.chi_perp + (coef_cell_chi(C, i, xyz) - C.chi_perp) * bi * bi);
            b1 = C.cnn * (C.chi_perp + (coef_cell_chi(C, j, nbr) - C.chi_perp) * bj * bj);
        }
        const int o = xyz[0] * C.so[0] + xyz[1] * C.so[1] + xyz[2] * C.so[2];
        C.alpha[o] = (T)a;
        C.beta1[o] = (T)b1;
        if (C.ndim == 3) C.beta2[o] = (T)b2;
    }
}

template <typename T>
hipError_t launch_coef(const CoefParams<T>& C, hipStream_t st) {
    const long N = (long)C.n[0] * C.n[1] * C.n[2];
    long nb = (N + 255) / 256;
    if (nb > 16384) nb = 16384;
    hipLaunchKernelGGL(coef_kernel<T>, dim3((unsigned)nb), dim3(256), 0, st, C);
    return hipGetLastError();
}

template hipError_t launch_coef<float>(const CoefParams<float>&, hipStream_t);
template hipError_t launch_coef<double>(const CoefParams<double>&, hipStream_t);

}  // namespace asd
