/*
 * Serial FP64 reference ("oracle") for the directionally split semi-implicit
 * anisotropic diffusion scheme of Sharma & Hammett, "A Fast Semi-implicit
 * Method for Anisotropic Diffusion" (arXiv:1008.0861).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this file.  It shares no code, header,
 * table or helper with the GPU library; it is plain C99, serial, FP64, built
 * with -ffp-contract=off, and loops in the natural order so that every line
 * can be checked against the paper by eye.  A second build of the same
 * source with OpenMP (liborc_omp.so) shares the independent lines of each
 * sweep out over the host's cores for the all-core timing baseline; each
 * line's arithmetic is unchanged, so both builds agree bit for bit.
 *
 * Layout of every cell array: index (k*ny + j)*nx + i, i (x) fastest.
 *
 * What is computed (paper section 2):
 *   dT/dt = -div q,  q = -D grad T,  D = chi_perp I + (chi_face - chi_perp) b b^T
 *   (the Braginskii split; with chi_perp = 0 this is q = -chi b (b.grad T),
 *   Eq. aniso_cond / heat_flux).
 *   One step (Eq. op_2step, generalised to 3-D as in section 2.1):
 *     T* = (1 + dt D_xx)^-1 (1 - dt D_xy [- dt D_xz]) T^n        (Eq. xup)
 *     T^{n+1} = (1 + dt D_yy)^-1 (1 - dt D_yx [- dt D_yz]) T*   (Eq. yup)
 *     [3-D: then the z sweep with transverse terms from T**]
 *   The 4-step variant (section 2.1, Eq. 4step) keeps the explicit
 *   transverse term of each direction at dt and applies its implicit normal
 *   operator twice at dt/2:
 *     T* = (1 + dt D_xx/2)^-2 (1 - dt D_xy) T^n,  then y (and z) alike.
 *   The "normal" term of each sweep is implicit (one tridiagonal system per
 *   grid line); the "transverse" term is explicit and uses the limited face
 *   difference of section 2 (van Leer by default, Eq. vanLeer; minmod and MC
 *   are the alternatives the paper mentions; "linear" is the arithmetic mean
 *   used in the linear stability analysis, section 2.1).
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - face b: arithmetic mean of the two cells sharing the face, not
 *     renormalised (section 2, "simple averaging");
 *   - variable chi: harmonic mean of the two cells (section 2, citing the
 *     earlier explicit paper);
 *   - insulating walls: zero total flux through wall faces, mirror ghosts for
 *     transverse differences (section 3.1, reflective boundary);
 *   - periodic lines: cyclic tridiagonal, solved by Thomas + Sherman-Morrison;
 *   - 4-argument limiter L(a,b,c,d) = L(L(a,b),L(c,d)) for every limiter,
 *     (a,b) taken from the cell on the + side of the face;
 *   - the explicit limited step is forward Euler of the same unsplit
 *     operator, every face evaluated from T^n;
 *   - temperature-dependent chi_par (chi ~ T^(5/2), section 3.3): per-cell
 *     values from the state the sweep reads (T^n, T*, ...), harmonic mean
 *     at each face, as for a per-cell chi field;
 *   - fixed-temperature walls (T = 0 on the boundary, the smooth test of
 *     section 3.2): odd ghosts U[-1] = -U[0], U[n] = -U[n-1] (zero on the
 *     wall face), the wall face's b and chi those of its cell, no
 *     transverse flux through a wall face (the limited difference of a cell
 *     and its odd ghost vanishes), normal flux alpha_w (U_ghost - U_cell)
 *     taken implicitly: 2 alpha_w on the diagonal of the wall cell's row;
 *   - source Q (same section): dt Q added to the right-hand side of the
 *     first sweep of each step (forward Euler in the explicit scheme).
 */
#include <math.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <string.h>

#define ORC_BC_PERIODIC 0
#define ORC_BC_INSULATING 1
#define ORC_BC_DIRICHLET 2

#define ORC_LIM_VANLEER 0
#define ORC_LIM_MINMOD 1
#define ORC_LIM_MC 2
#define ORC_LIM_LINEAR 3

typedef struct {
    int ndim;         /* 2 or 3 */
    long n[3];        /* cells along x, y, z (n[2] == 1 when ndim == 2) */
    double h[3];      /* cell widths */
    int bc;           /* ORC_BC_* (same on every axis) */
    int limiter;      /* ORC_LIM_* */
    double chi_par;   /* parallel diffusivity when chi == NULL */
    double chi_perp;  /* isotropic part of the tensor */
    const double *b[3]; /* cell-centred components of the unit vector b */
    const double *chi;  /* optional per-cell chi_par (NULL: constant) */
    double chi_exp;     /* != 0: chi_par(T) = chi_par (T / chi_tref)^chi_exp, from the */
    double chi_tref;    /*       state the sweep (or explicit step) reads (section 3.3)   */
    const double *src;  /* optional per-cell source Q (NULL: none) */
} orc_grid;

/* ------------------------------------------------------------------ */
/* Limiters (section 2, Eq. vanLeer, and the minmod / MC alternatives) */
/* ------------------------------------------------------------------ */

static double sgn(double a) { return a > 0.0 ? 1.0 : (a < 0.0 ? -1.0 : 0.0); }

static double min2(double a, double b) { return a < b ? a : b; }

/* Two-argument limiter. */
double orc_lim2(int lim, double a, double b)
{
    switch (lim) {
    case ORC_LIM_VANLEER:
        /* van Leer: harmonic-type mean when the two differences agree in sign */
        if (a * b > 0.0) return 2.0 * a * b / (a + b);
        return 0.0;
    case ORC_LIM_MINMOD:
        if (a * b > 0.0) return sgn(a) * min2(fabs(a), fabs(b));
        return 0.0;
    case ORC_LIM_MC:
        /* monotonised central: minmod(2a, 2b, (a+b)/2) */
        if (a * b > 0.0)
            return sgn(a) * min2(min2(2.0 * fabs(a), 2.0 * fabs(b)), 0.5 * fabs(a + b));
        return 0.0;
    case ORC_LIM_LINEAR:
        return 0.5 * (a + b);
    default:
        return NAN;
    }
}

/* Four-argument form: L(a,b,c,d) = L(L(a,b), L(c,d)) (section 2). */
double orc_lim4(int lim, double a, double b, double c, double d)
{
    return orc_lim2(lim, orc_lim2(lim, a, b), orc_lim2(lim, c, d));
}

/* ------------------------------------------------------------------ */
/* Tridiagonal solvers                                                 */
/* ------------------------------------------------------------------ */

/*
 * Thomas algorithm for  lo[i] x[i-1] + di[i] x[i] + up[i] x[i+1] = r[i],
 * i = 0..n-1 (lo[0] and up[n-1] ignored).  No pivoting: the systems built
 * here are symmetric, strictly diagonally dominant M-matrices.
 * Returns 0, or -1 on a zero pivot / bad size.
 */
int orc_thomas(long n, const double *lo, const double *di, const double *up,
               const double *r, double *x)
{
    if (n < 1) return -1;
    double *cp = (double *)malloc(sizeof(double) * (size_t)n);
    double *dp = (double *)malloc(sizeof(double) * (size_t)n);
    if (!cp || !dp) { free(cp); free(dp); return -1; }
    double piv = di[0];
    if (piv == 0.0) { free(cp); free(dp); return -1; }
    cp[0] = (n > 1 ? up[0] : 0.0) / piv;
    dp[0] = r[0] / piv;
    for (long i = 1; i < n; ++i) {
        piv = di[i] - lo[i] * cp[i - 1];
        if (piv == 0.0) { free(cp); free(dp); return -1; }
        cp[i] = (i < n - 1 ? up[i] : 0.0) / piv;
        dp[i] = (r[i] - lo[i] * dp[i - 1]) / piv;
    }
    x[n - 1] = dp[n - 1];
    for (long i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
    free(cp);
    free(dp);
    return 0;
}

/*
 * Cyclic tridiagonal system: as above, plus the corner couplings lo[0]
 * (row 0 to x[n-1]) and up[n-1] (row n-1 to x[0]).  Solved with the
 * Sherman-Morrison construction of Numerical Recipes (cited by the paper):
 * A = B + u v^T with B tridiagonal, u = (g, 0, .., 0, up[n-1]),
 * v = (1, 0, .., 0, lo[0]/g), g = -di[0].  Needs n >= 3.
 */
int orc_cyclic(long n, const double *lo, const double *di, const double *up,
               const double *r, double *x)
{
    if (n < 3) return -1;
    const double alpha = up[n - 1]; /* bottom-left corner */
    const double beta = lo[0];      /* top-right corner */
    const double gamma = -di[0];
    double *bb = (double *)malloc(sizeof(double) * (size_t)n);
    double *u = (double *)malloc(sizeof(double) * (size_t)n);
    double *z = (double *)malloc(sizeof(double) * (size_t)n);
    if (!bb || !u || !z) { free(bb); free(u); free(z); return -1; }
    memcpy(bb, di, sizeof(double) * (size_t)n);
    bb[0] = di[0] - gamma;
    bb[n - 1] = di[n - 1] - alpha * beta / gamma;
    int rc = orc_thomas(n, lo, bb, up, r, x);
    if (rc == 0) {
        for (long i = 0; i < n; ++i) u[i] = 0.0;
        u[0] = gamma;
        u[n - 1] = alpha;
        rc = orc_thomas(n, lo, bb, up, u, z);
    }
    if (rc == 0) {
        const double fact = (x[0] + beta * x[n - 1] / gamma) /
                            (1.0 + z[0] + beta * z[n - 1] / gamma);
        for (long i = 0; i < n; ++i) x[i] -= fact * z[i];
    }
    free(bb);
    free(u);
    free(z);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Grid helpers                                                        */
/* ------------------------------------------------------------------ */

static long cell_index(const orc_grid *g, const long p[3])
{
    return (p[2] * g->n[1] + p[1]) * g->n[0] + p[0];
}

/*
 * Value of U at cell p displaced by s (= +1 or -1) along axis t, with the
 * boundary rule: periodic wraps, insulating mirrors (U[-1] = U[0],
 * U[n] = U[n-1], which gives zero normal gradient at the wall), Dirichlet
 * mirrors with the opposite sign (U[-1] = -U[0], U[n] = -U[n-1]: the
 * linear interpolant vanishes on the wall face).
 */
static double ghost_value(const orc_grid *g, const double *U, const long p[3], int t, int s)
{
    long q[3] = {p[0], p[1], p[2]};
    long m = q[t] + s;
    double sign = 1.0;
    if (m < 0 || m >= g->n[t]) {
        if (g->bc == ORC_BC_PERIODIC) {
            m = m < 0 ? g->n[t] - 1 : 0;
        } else {
            m = q[t];
            if (g->bc == ORC_BC_DIRICHLET) sign = -1.0;
        }
    }
    q[t] = m;
    return sign * U[cell_index(g, q)];
}

/* Cell diffusivity from the state U: chi_par (T / chi_tref)^chi_exp. */
static double cell_chi_of_T(const orc_grid *g, const double *U, long c)
{
    return g->chi_par * pow(U[c] / g->chi_tref, g->chi_exp);
}

/* Diffusivity of one cell: chi_par, the per-cell field, or chi_par(T). */
static double cell_chi(const orc_grid *g, const double *U, long c)
{
    if (g->chi_exp != 0.0) return cell_chi_of_T(g, U, c);
    if (g->chi) return g->chi[c];
    return g->chi_par;
}

/* Face diffusivity: chi_par, or the harmonic mean of the two cells' values
 * (a per-cell field, or chi_par(T) of the state U). */
static double face_chi(const orc_grid *g, const double *U, long c0, long c1)
{
    double a, b;
    if (g->chi_exp != 0.0) {
        a = cell_chi_of_T(g, U, c0);
        b = cell_chi_of_T(g, U, c1);
    } else if (g->chi) {
        a = g->chi[c0];
        b = g->chi[c1];
    } else {
        return g->chi_par;
    }
    if (a + b == 0.0) return 0.0;
    return 2.0 * a * b / (a + b);
}

/*
 * Coefficients of the face between cells p0 and p1 = p0 + e_d:
 *   alpha      = dt_n * D_dd / h_d^2              (normal, implicit part)
 *   beta[t]    = dt_t * D_dt / (h_d h_t), t != d  (transverse, explicit part)
 * with b at the face the arithmetic mean of the two cells (dt_n = dt_t = dt
 * in the 2-step scheme).
 */
static void face_coefficients(const orc_grid *g, const double *U, int d, const long p0[3], const long p1[3],
                              double dt_n, double dt_t, double *alpha, double beta[3])
{
    const long c0 = cell_index(g, p0), c1 = cell_index(g, p1);
    double bf[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < g->ndim; ++q) bf[q] = 0.5 * (g->b[q][c0] + g->b[q][c1]);
    const double chif = face_chi(g, U, c0, c1);
    const double dnn = g->chi_perp + (chif - g->chi_perp) * bf[d] * bf[d];
    *alpha = dt_n * dnn / (g->h[d] * g->h[d]);
    for (int t = 0; t < 3; ++t) beta[t] = 0.0;
    for (int t = 0; t < g->ndim; ++t) {
        if (t == d) continue;
        const double dnt = (chif - g->chi_perp) * bf[d] * bf[t];
        beta[t] = dt_t * dnt / (g->h[d] * g->h[t]);
    }
}

/*
 * Limited transverse difference at the face between p0 and p1 = p0 + e_d,
 * transverse axis t, from state U (section 2):
 *   a = U[p1+e_t] - U[p1],  b = U[p1] - U[p1-e_t],
 *   c = U[p0+e_t] - U[p0],  d = U[p0] - U[p0-e_t],   L(a,b,c,d).
 */
static double transverse_difference(const orc_grid *g, const double *U, const long p0[3],
                                    const long p1[3], int t)
{
    const double u1 = U[cell_index(g, p1)], u0 = U[cell_index(g, p0)];
    const double a = ghost_value(g, U, p1, t, +1) - u1;
    const double b = u1 - ghost_value(g, U, p1, t, -1);
    const double c = ghost_value(g, U, p0, t, +1) - u0;
    const double dd = u0 - ghost_value(g, U, p0, t, -1);
    return orc_lim4(g->limiter, a, b, c, dd);
}

/*
 * Normal coefficient alpha and transverse flux F of face "k + 1/2" of a line
 * along axis d (between line cell k and cell k+1, wrapping for periodic).
 * Wall faces (k = -1 or k = n-1 when not periodic) have F = 0; an
 * insulating wall has alpha = 0, a Dirichlet wall the alpha of a face whose
 * b and chi are those of its one cell.  Returns 1 for a wall face.
 */
static int line_face(const orc_grid *g, const double *U, int d, const long base[3], long k,
                     double dt_n, double dt_t, double *alpha, double *flux)
{
    const long n = g->n[d];
    *alpha = 0.0;
    *flux = 0.0;
    long k0 = k, k1 = k + 1;
    if (g->bc == ORC_BC_PERIODIC) {
        k0 = (k0 + n) % n;
        k1 = (k1 + n) % n;
    } else if (k0 < 0 || k1 > n - 1) {
        if (g->bc == ORC_BC_DIRICHLET) {
            long p[3] = {base[0], base[1], base[2]};
            p[d] = k0 < 0 ? k1 : k0; /* the wall's cell */
            const long c = cell_index(g, p);
            const double bd = g->b[d][c];
            const double dnn = g->chi_perp + (cell_chi(g, U, c) - g->chi_perp) * bd * bd;
            *alpha = dt_n * dnn / (g->h[d] * g->h[d]);
        }
        return 1;
    }
    long p0[3] = {base[0], base[1], base[2]}, p1[3] = {base[0], base[1], base[2]};
    p0[d] = k0;
    p1[d] = k1;
    double beta[3];
    face_coefficients(g, U, d, p0, p1, dt_n, dt_t, alpha, beta);
    double f = 0.0;
    for (int t = 0; t < g->ndim; ++t) {
        if (t == d) continue;
        f += beta[t] * transverse_difference(g, U, p0, p1, t);
    }
    *flux = f;
    return 0;
}

/* ------------------------------------------------------------------ */
/* One directional sweep (Eq. xup / yup)                               */
/* ------------------------------------------------------------------ */

/*
 * out = (1 + dt_n D_dd)^-1 (U + transverse fluxes of U at dt_t + dt_q Q)
 * along axis d.  Every coefficient is computed from the complete input U
 * before out is written (out must not alias U).  dt_t = 0 is a pure
 * implicit solve; dt_q = 0 (or no source) adds nothing.
 */
/* One line of a sweep: base gives the line's coordinates on the two other axes. */
static int sweep_line(const orc_grid *g, int d, double dt_n, double dt_t, double dt_q, const double *U,
                      double *out, const long base[3])
{
    const long n = g->n[d];
    double *alpha = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    double *flux = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    int *wall = (int *)malloc(sizeof(int) * (size_t)(n + 1));
    double *lo = (double *)malloc(sizeof(double) * (size_t)n);
    double *di = (double *)malloc(sizeof(double) * (size_t)n);
    double *up = (double *)malloc(sizeof(double) * (size_t)n);
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *x = (double *)malloc(sizeof(double) * (size_t)n);
    int rc = 0;
    if (!alpha || !flux || !wall || !lo || !di || !up || !r || !x) rc = -1;
    if (rc == 0) {
        /* faces k + 1/2 for k = -1 .. n-1; entry k+1 holds face k+1/2 */
        for (long k = -1; k < n; ++k)
            wall[k + 1] = line_face(g, U, d, base, k, dt_n, dt_t, &alpha[k + 1], &flux[k + 1]);
        for (long i = 0; i < n; ++i) {
            const double am = alpha[i];     /* face i - 1/2 */
            const double ap = alpha[i + 1]; /* face i + 1/2 */
            long p[3] = {base[0], base[1], base[2]};
            p[d] = i;
            lo[i] = -am;
            up[i] = -ap;
            di[i] = 1.0 + am + ap;
            /* a Dirichlet wall face couples the cell to its odd ghost
               (x_ghost = -x_cell): 2 alpha on the diagonal, no
               off-diagonal entry (insulating walls have alpha = 0) */
            if (wall[i]) { lo[i] = 0.0; di[i] += am; }
            if (wall[i + 1]) { up[i] = 0.0; di[i] += ap; }
            const long c = cell_index(g, p);
            r[i] = U[c] + flux[i + 1] - flux[i];
            if (g->src && dt_q != 0.0) r[i] += dt_q * g->src[c];
        }
        if (g->bc == ORC_BC_PERIODIC)
            rc = orc_cyclic(n, lo, di, up, r, x);
        else
            rc = orc_thomas(n, lo, di, up, r, x);
        for (long i = 0; rc == 0 && i < n; ++i) {
            long p[3] = {base[0], base[1], base[2]};
            p[d] = i;
            out[cell_index(g, p)] = x[i];
        }
    }
    free(alpha);
    free(flux);
    free(wall);
    free(lo);
    free(di);
    free(up);
    free(r);
    free(x);
    return rc;
}

/*
 * out = (1 + dt_n D_dd)^-1 (U + transverse fluxes of U at dt_t + dt_q Q)
 * along axis d.  Every coefficient is computed from the complete input U
 * before out is written (out must not alias U).  dt_t = 0 is a pure
 * implicit solve; dt_q = 0 (or no source) adds nothing.  The lines are
 * independent: a build with OpenMP (liborc_omp.so, the all-core timing
 * baseline) shares them out over threads; each line's arithmetic is the
 * same either way.
 */
int orc_sweep3(const orc_grid *g, int d, double dt_n, double dt_t, double dt_q, const double *U, double *out)
{
    const long n = g->n[d];
    if (g->bc == ORC_BC_PERIODIC && n < 3) return -1;
    if (n < 2) return -1;
    /* the two axes other than d enumerate the lines */
    const int ax1 = (d + 1) % 3, ax2 = (d + 2) % 3;
    const long n1 = g->n[ax1], nlines = g->n[ax1] * g->n[ax2];
    int rc = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) reduction(| : rc)
#endif
    for (long l = 0; l < nlines; ++l) {
        long base[3];
        base[d] = 0;
        base[ax1] = l % n1;
        base[ax2] = l / n1;
        rc |= sweep_line(g, d, dt_n, dt_t, dt_q, U, out, base);
    }
    return rc ? -1 : 0;
}

/* Threads the oracle's sweeps use (1 without OpenMP). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int orc_sweep2(const orc_grid *g, int d, double dt_n, double dt_t, const double *U, double *out)
{
    return orc_sweep3(g, d, dt_n, dt_t, 0.0, U, out);
}

/* One sweep of the 2-step scheme (Eq. xup / yup): normal and transverse at dt. */
int orc_sweep(const orc_grid *g, int d, double dt, const double *U, double *out)
{
    return orc_sweep2(g, d, dt, dt, U, out);
}

static long cell_count(const orc_grid *g) { return g->n[0] * g->n[1] * g->n[2]; }

/* E = sum_c T_c dV, accumulated in index order. */
double orc_energy(const orc_grid *g, const double *T)
{
    double dv = 1.0;
    for (int q = 0; q < g->ndim; ++q) dv *= g->h[q];
    double s = 0.0;
    const long N = cell_count(g);
    for (long c = 0; c < N; ++c) s += T[c];
    return s * dv;
}

static int grid_ok(const orc_grid *g)
{
    if (!g || (g->ndim != 2 && g->ndim != 3)) return 0;
    if (g->ndim == 2 && g->n[2] != 1) return 0;
    for (int q = 0; q < g->ndim; ++q) {
        if (g->n[q] < 2 || !(g->h[q] > 0.0) || !g->b[q]) return 0;
        if (g->bc == ORC_BC_PERIODIC && g->n[q] < 3) return 0;
    }
    if (g->bc < ORC_BC_PERIODIC || g->bc > ORC_BC_DIRICHLET) return 0;
    if (g->chi_exp != 0.0 && (!(g->chi_tref > 0.0) || g->chi)) return 0;
    return 1;
}

/*
 * nsteps semi-implicit steps, in place on T.  Each sweep takes its
 * transverse differences from its own input (T^n, then T*, then T**).
 * flags: ORC_SI_FOUR_STEP for the 4-step scheme (Eq. 4step: per direction
 * the transverse term at dt with a normal solve at dt/2, then a second
 * normal solve at dt/2); ORC_SI_REVERSE for the reverse sweep order
 * (y then x, or z, y, x), which section 2 allows in place of x then y.
 * energy (nullable) receives nsteps+1 values.
 */
#define ORC_SI_FOUR_STEP 1
#define ORC_SI_REVERSE 2
int orc_step_si_ex(const orc_grid *g, double dt, int nsteps, double *T, double *energy, int flags)
{
    if (!grid_ok(g) || nsteps < 0 || !T) return -1;
    const long N = cell_count(g);
    double *tmp = (double *)malloc(sizeof(double) * (size_t)N);
    if (!tmp) return -1;
    int rc = 0;
    if (energy) energy[0] = orc_energy(g, T);
    for (int s = 0; rc == 0 && s < nsteps; ++s) {
        for (int i = 0; rc == 0 && i < g->ndim; ++i) {
            const int d = (flags & ORC_SI_REVERSE) ? g->ndim - 1 - i : i;
            const double dt_q = i == 0 ? dt : 0.0; /* the source enters the first sweep */
            if (flags & ORC_SI_FOUR_STEP) {
                rc = orc_sweep3(g, d, 0.5 * dt, dt, dt_q, T, tmp);
                if (rc == 0) rc = orc_sweep2(g, d, 0.5 * dt, 0.0, tmp, T);
            } else {
                rc = orc_sweep3(g, d, dt, dt, dt_q, T, tmp);
                if (rc == 0) memcpy(T, tmp, sizeof(double) * (size_t)N);
            }
        }
        if (energy) energy[s + 1] = orc_energy(g, T);
    }
    free(tmp);
    return rc;
}

/* The 2-step scheme in the order x, y (, z) (Eqs. xup / yup, op_2step). */
int orc_step_si(const orc_grid *g, double dt, int nsteps, double *T, double *energy)
{
    return orc_step_si_ex(g, dt, nsteps, T, energy, 0);
}

/* The 4-step scheme (Eq. 4step) in the order x, y (, z). */
int orc_step_si4(const orc_grid *g, double dt, int nsteps, double *T, double *energy)
{
    return orc_step_si_ex(g, dt, nsteps, T, energy, ORC_SI_FOUR_STEP);
}

/*
 * Explicit limited step (the CFL-bound baseline):
 *   T^{n+1}_c = T^n_c + sum_d [ alpha_{c+1/2}(T_{c+e} - T_c) - alpha_{c-1/2}(T_c - T_{c-e})
 *                               + F_{c+1/2} - F_{c-1/2} ],
 * every alpha and F from T^n.
 */
int orc_step_explicit(const orc_grid *g, double dt, int nsteps, double *T, double *energy)
{
    if (!grid_ok(g) || nsteps < 0 || !T) return -1;
    const long N = cell_count(g);
    double *nxt = (double *)malloc(sizeof(double) * (size_t)N);
    if (!nxt) return -1;
    if (energy) energy[0] = orc_energy(g, T);
    for (int s = 0; s < nsteps; ++s) {
        for (long c = 0; c < N; ++c) nxt[c] = T[c] + (g->src ? dt * g->src[c] : 0.0);
        for (int d = 0; d < g->ndim; ++d) {
            const long n = g->n[d];
            int ax1 = (d + 1) % 3, ax2 = (d + 2) % 3;
            for (long l2 = 0; l2 < g->n[ax2]; ++l2) {
                for (long l1 = 0; l1 < g->n[ax1]; ++l1) {
                    long base[3];
                    base[d] = 0;
                    base[ax1] = l1;
                    base[ax2] = l2;
                    for (long i = 0; i < n; ++i) {
                        double am, fm, ap, fp;
                        line_face(g, T, d, base, i - 1, dt, dt, &am, &fm);
                        line_face(g, T, d, base, i, dt, dt, &ap, &fp);
                        long p[3] = {base[0], base[1], base[2]};
                        p[d] = i;
                        const double tc = T[cell_index(g, p)];
                        /* at a wall: insulating alpha = 0; Dirichlet uses the odd ghost */
                        const double tp = ghost_value(g, T, p, d, +1);
                        const double tm = ghost_value(g, T, p, d, -1);
                        nxt[cell_index(g, p)] += ap * (tp - tc) - am * (tc - tm) + fp - fm;
                    }
                }
            }
        }
        memcpy(T, nxt, sizeof(double) * (size_t)N);
        if (energy) energy[s + 1] = orc_energy(g, T);
    }
    free(nxt);
    return 0;
}

/* dt from the Courant factor: dt = ncfl * min_d h_d^2 / (4 chi_max)  (Eq. ncfl). */
double orc_dt_from_ncfl(const orc_grid *g, double ncfl)
{
    double hmin2 = g->h[0] * g->h[0];
    for (int q = 1; q < g->ndim; ++q)
        if (g->h[q] * g->h[q] < hmin2) hmin2 = g->h[q] * g->h[q];
    double cmax = g->chi_par;
    if (g->chi) {
        cmax = 0.0;
        const long N = cell_count(g);
        for (long c = 0; c < N; ++c)
            if (g->chi[c] > cmax) cmax = g->chi[c];
    }
    return ncfl * hmin2 / (4.0 * cmax);
}

/* Size of the struct, so the loader can check its own mirror of it. */
long orc_grid_sizeof(void) { return (long)sizeof(orc_grid); }
