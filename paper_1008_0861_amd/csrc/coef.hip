// Face coefficients of one sweep direction (section 2): at the face between
// cell c and c + e_d,
//     b_f     = (b_c + b_{c+e_d}) / 2      (arithmetic mean, not renormalised)
//     chi_f   = chi_par, or the harmonic mean of the two cells' chi (a per-cell
//               field, or chi_par (U / T_ref)^p of a state U, section 4)
//     alpha_f = dt (chi_perp + (chi_f - chi_perp) b_d,f^2) / h_d^2
//     beta_t  = dt (chi_f - chi_perp) b_d,f b_t,f / (h_d h_t)
// A wall face (insulating boundary, c on the last plane) gets zeros.
// Computed in FP64 and rounded once to the grid's type.  With a constant or
// per-cell chi they depend on dt, b and chi only and a step loop computes
// them once; with chi(T) they are recomputed from each sweep's input.
#include "asd_device.h"
#include "asd_launch.h"

namespace asd {

template <typename T>
__global__ void __launch_bounds__(256) coef_kernel(CoefParams<T> C) {
    const int nx = C.n[0], ny = C.n[1], nz = C.n[2];
    const int N = nx * ny * nz;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        const int xyz[3] = {i % nx, (i / nx) % ny, i / (nx * ny)};
        int nbr[3] = {xyz[0], xyz[1], xyz[2]};
        nbr[C.d] += 1;
        bool wall = false;
        if (nbr[C.d] == C.n[C.d]) {
            if (C.periodic) nbr[C.d] = 0;
            else wall = true;
        }
        double a = 0.0, b1 = 0.0, b2 = 0.0;
        if (!wall) {
            const int j = nbr[0] + nbr[1] * nx + nbr[2] * nx * ny;
            double bf[3] = {0.0, 0.0, 0.0};
            for (int q = 0; q < C.ndim; ++q) bf[q] = 0.5 * ((double)C.b[q][i] + (double)C.b[q][j]);
            double chif = C.chi_par;
            if (C.U) {
                // the state is in the output (sweep-input) layout
                const int o0 = xyz[0] * C.so[0] + xyz[1] * C.so[1] + xyz[2] * C.so[2];
                const int o1 = nbr[0] * C.so[0] + nbr[1] * C.so[1] + nbr[2] * C.so[2];
                const double x0 = C.chi_par * pow((double)C.U[o0] / C.chi_tref, C.chi_exp);
                const double x1 = C.chi_par * pow((double)C.U[o1] / C.chi_tref, C.chi_exp);
                chif = (x0 + x1) != 0.0 ? 2.0 * x0 * x1 / (x0 + x1) : 0.0;
            } else if (C.chi) {
                const double x0 = (double)C.chi[i], x1 = (double)C.chi[j];
                chif = (x0 + x1) != 0.0 ? 2.0 * x0 * x1 / (x0 + x1) : 0.0;
            }
            const double dpar = chif - C.chi_perp;
            a = C.cnn * (C.chi_perp + dpar * bf[C.d] * bf[C.d]);
            b1 = C.ct1 * dpar * bf[C.d] * bf[C.t1];
            if (C.ndim == 3) b2 = C.ct2 * dpar * bf[C.d] * bf[C.t2];
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
