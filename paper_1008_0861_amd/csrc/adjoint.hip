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
// Two gather kernels, no atomics, one thread per cell: face_kernel
// evaluates per face the weights w_f dG/dsigma (w_f = beta_f (mu_c - mu_c'))
// and dL/dchi_f; cell_kernel sums, per cell, the contributions of its own
// slope and of the slopes of its two transverse neighbours, and its two
// faces' chi terms.
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

// A cell and its neighbours.  Each thread owns one cell: block b covers 256
// consecutive cells of row b / ncx (no per-cell integer division).
struct AdjCell {
    int x, y, c;
    bool ok;
};
__device__ __forceinline__ AdjCell adj_cell_of_thread(int nx, int ny) {
    const int ncx = (nx + 255) >> 8;
    const int by = (int)blockIdx.x / ncx;  // wave-uniform
    AdjCell r;
    r.x = ((int)blockIdx.x - by * ncx) * 256 + (int)threadIdx.x;
    r.y = by;
    r.ok = r.x < nx && r.y < ny;
    r.c = r.x + r.y * nx;
    return r;
}

struct AdjGeom {
    int nx, ny, d, t;
    bool periodic;
};

// Cell (x, y) moved by s = +-1 along axis ax: its coordinates in (mx, my)
// and its index, or -1 if it leaves an insulating domain.
__device__ __forceinline__ int moved(const AdjGeom& G, int x, int y, int ax, int s, int* mx, int* my) {
    int c[2] = {x, y};
    const int n = ax == 0 ? G.nx : G.ny;
    int v = c[ax] + s;
    if (v < 0 || v >= n) {
        if (!G.periodic) return -1;
        v += v < 0 ? n : -n;
    }
    c[ax] = v;
    *mx = c[0];
    *my = c[1];
    return c[0] + c[1] * G.nx;
}
__device__ __forceinline__ int moved(const AdjGeom& G, int x, int y, int ax, int s) {
    int mx, my;
    return moved(G, x, y, ax, s, &mx, &my);
}

template <typename T>
__global__ void __launch_bounds__(256) adj_face_kernel(AdjParams<T> P) {
    const AdjGeom G{P.nx, P.ny, P.d, 1 - P.d, P.periodic != 0};
    const AdjCell C = adj_cell_of_thread(P.nx, P.ny);
    if (!C.ok) return;
    const int x = C.x, y = C.y, c = C.c;
    int xp, yp;
    const int cp = moved(G, x, y, G.d, +1, &xp, &yp);
    if (cp < 0) {  // wall face
        P.W1[c] = T(0);
        P.W2[c] = T(0);
        P.GF[c] = T(0);
        return;
    }
    // slopes of the two cells along t (mirror ghosts at insulating walls)
    auto slope = [&](int cx, int cy, int cc) {
        int up = moved(G, cx, cy, G.t, +1), dn = moved(G, cx, cy, G.t, -1);
        if (up < 0) up = cc;
        if (dn < 0) dn = cc;
        const double u = (double)P.U[cc];
        double d1, d2;
        return dlim2(P.limiter, (double)P.U[up] - u, u - (double)P.U[dn], &d1, &d2);
    };
    const double s0 = slope(x, y, c), s1 = slope(xp, yp, cp);
    double LG1, LG2;
    const double Gf = dlim2(P.limiter, s1, s0, &LG1, &LG2);
    const double bn = 0.5 * ((double)P.b[G.d][c] + (double)P.b[G.d][cp]);
    const double bt = 0.5 * ((double)P.b[G.t][c] + (double)P.b[G.t][cp]);
    double chif = P.chi_par;
    if (P.chi) {
        const double a = (double)P.chi[c], b = (double)P.chi[cp];
        chif = (a + b) != 0.0 ? 2.0 * a * b * fast_rcp<double>(a + b) : 0.0;
    }
    const double dpar = chif - P.chi_perp;
    const double beta = P.dt * dpar * bn * bt / (P.hn * P.ht);
    const double dm = (double)P.mu[c] - (double)P.mu[cp];
    const double w = beta * dm;
    P.W1[c] = (T)(w * LG1);  // to the slope of the right cell cp
    P.W2[c] = (T)(w * LG2);  // to the slope of the left cell c
    const double dLdalpha = -dm * ((double)P.X[c] - (double)P.X[cp]);
    const double dLdbeta = dm * Gf;
    P.GF[c] = (T)(dLdalpha * P.dt * bn * bn / (P.hn * P.hn) + dLdbeta * P.dt * bn * bt / (P.hn * P.ht));
}

template <typename T>
__global__ void __launch_bounds__(256) adj_cell_kernel(AdjParams<T> P) {
    const AdjGeom G{P.nx, P.ny, P.d, 1 - P.d, P.periodic != 0};
    const AdjCell C = adj_cell_of_thread(P.nx, P.ny);
    if (!C.ok) return;
    const int x = C.x, y = C.y, j = C.c;
    // psi(c) = sum over the two faces of c of w dG/dsigma_c
    auto psi = [&](int cx, int cy, int cc) {
        double v = (double)P.W2[cc];
        const int cm = moved(G, cx, cy, G.d, -1);
        if (cm >= 0) v += (double)P.W1[cm];
        return v;
    };
    // slope partials of cell c: sigma_c = L(p, q), p = U[up] - U[c], q = U[c] - U[dn]
    auto slope_d = [&](int cx, int cy, int cc, double* l1, double* l2, bool* up_self, bool* dn_self) {
        int up = moved(G, cx, cy, G.t, +1), dn = moved(G, cx, cy, G.t, -1);
        *up_self = up < 0;
        *dn_self = dn < 0;
        if (up < 0) up = cc;
        if (dn < 0) dn = cc;
        const double u = (double)P.U[cc];
        dlim2(P.limiter, (double)P.U[up] - u, u - (double)P.U[dn], l1, l2);
    };
    double l1, l2;
    bool us, ds;
    slope_d(x, y, j, &l1, &l2, &us, &ds);
    // d sigma_j / d U_j: -l1 through p (unless p is identically zero at a
    // mirrored wall), +l2 through q (likewise)
    double acc = (double)P.mu[j] + psi(x, y, j) * ((us ? 0.0 : -l1) + (ds ? 0.0 : l2));
    int xm, ym;
    const int jm = moved(G, x, y, G.t, -1, &xm, &ym);  // its slope's p involves U_j
    if (jm >= 0) {
        double m1, m2;
        bool mus, mds;
        slope_d(xm, ym, jm, &m1, &m2, &mus, &mds);
        acc += psi(xm, ym, jm) * m1;
    }
    int xq, yq;
    const int jp = moved(G, x, y, G.t, +1, &xq, &yq);  // its slope's q involves U_j
    if (jp >= 0) {
        double p1, p2;
        bool pus, pds;
        slope_d(xq, yq, jp, &p1, &p2, &pus, &pds);
        acc -= psi(xq, yq, jp) * p2;
    }
    P.lam_out[j] = (T)acc;
    if (P.gchi) {
        // chi_f = 2 a b / (a + b): d/da = 2 b^2 / (a + b)^2
        double g = 0.0;
        const double cj = (double)P.chi[j];
        const int jr = moved(G, x, y, G.d, +1);
        if (jr >= 0) {
            const double cr = (double)P.chi[jr], s = cj + cr;
            if (s != 0.0) {
                const double r = fast_rcp<double>(s);
                g += (double)P.GF[j] * 2.0 * cr * cr * (r * r);
            }
        }
        const int jl = moved(G, x, y, G.d, -1);
        if (jl >= 0) {
            const double cl = (double)P.chi[jl], s = cj + cl;
            if (s != 0.0) {
                const double r = fast_rcp<double>(s);
                g += (double)P.GF[jl] * 2.0 * cl * cl * (r * r);
            }
        }
        P.gchi[j] = (T)((double)P.gchi[j] + g);
    }
}

template <typename T>
hipError_t launch_adjoint_stencil(const AdjParams<T>& P, hipStream_t st) {
    const long nb = (long)((P.nx + 255) >> 8) * P.ny;  // one thread per cell
    hipLaunchKernelGGL(adj_face_kernel<T>, dim3((unsigned)nb), dim3(256), 0, st, P);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(adj_cell_kernel<T>, dim3((unsigned)nb), dim3(256), 0, st, P);
    return hipGetLastError();
}

template hipError_t launch_adjoint_stencil<float>(const AdjParams<float>&, hipStream_t);
template hipError_t launch_adjoint_stencil<double>(const AdjParams<double>&, hipStream_t);

}  // namespace asd
