/*
 * asd.h — C ABI of libasd, an MI355X (gfx950) implementation of the
 * conservative, directionally split, semi-implicit scheme for anisotropic
 * diffusion of Sharma & Hammett, "A Fast Semi-implicit Method for
 * Anisotropic Diffusion" (arXiv:1008.0861), with the explicit limited
 * scheme beside it as the time-step-limited baseline.
 *
 * Equation solved (section 2, Eqs. aniso_cond and heat_flux, plus an
 * optional isotropic part and an optional source, section 3.2):
 *     dT/dt = div( D grad T ) + Q,   D = chi_perp I + (chi - chi_perp) b b^T,
 * b a given cell-centred unit vector, chi = chi_par (constant), a per-cell
 * field or chi_par (T / T_ref)^p, averaged harmonically at faces.
 *
 * Conventions shared by every entry point
 *   - Return value: ASD_OK (0) or a negative ASD_E* code.  Nothing throws or
 *     exits.  asd_last_error() returns a message for the calling thread.
 *   - Arguments are validated before any HIP call; an invalid call leaves
 *     the grid unchanged and enqueues nothing.
 *   - Memory: the library never allocates device memory.  Device arrays are
 *     borrowed from the caller (they must stay alive while work that uses
 *     them is in flight); scratch space is the caller's workspace.  The
 *     library owns only the small host-side handle.
 *   - Work is enqueued on the stream given to asd_init_grid and the calls
 *     return after enqueue (asd_status synchronises that stream).
 *   - Cell arrays are dense, x fastest: index (k*ny + j)*nx + i (2-D: nz = 1).
 *     Element type is the grid's dtype (float or double) for T, b and chi.
 *   - A grid handle must not be used from two threads at once.
 */
#ifndef ASD_H
#define ASD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define ASD_OK 0
#define ASD_EINVAL (-1)      /* bad scalar argument: dt <= 0 or not finite, h <= 0, enum out of range, null pointer */
#define ASD_ESHAPE (-2)      /* element count does not match the grid, n too small */
#define ASD_EDTYPE (-3)      /* dtype does not match the grid */
#define ASD_ENOTSET (-4)     /* a field needed by the call has not been set */
#define ASD_EWORKSPACE (-5)  /* workspace missing, misaligned or too small */
#define ASD_EUNSTABLE (-6)   /* dt beyond the scheme's stability limit (see below) */
#define ASD_EHIP (-7)        /* the HIP runtime reported an error */
#define ASD_EUNSUPPORTED (-8) /* valid but not supported by this library (e.g. line too long for LDS) */

/* boundary conditions (same on every axis) */
#define ASD_BC_PERIODIC 0    /* periodic box (section 3.3); lines are cyclic tridiagonal systems */
#define ASD_BC_INSULATING 1  /* reflective walls, dT/dn = 0 (section 3.1); zero flux through wall faces */
#define ASD_BC_DIRICHLET 2   /* T = 0 on the walls (section 3.2): odd ghost cells (T_ghost = -T_cell),
                                the wall face's b and chi those of its cell, its normal flux
                                implicit in the sweeps, no transverse flux through it.  Not for
                                the adjoint */

/* element types */
#define ASD_F32 0
#define ASD_F64 1

/* limiters for the transverse face difference (section 2) */
#define ASD_LIM_VANLEER 0    /* Eq. vanLeer, the paper's default */
#define ASD_LIM_MINMOD 1
#define ASD_LIM_MC 2         /* monotonised central */
#define ASD_LIM_LINEAR 3     /* plain average (the linear stability analysis, section 2.1) */

/* fields for asd_set_field */
#define ASD_FIELD_T 0        /* temperature, advanced in place by the step calls */
#define ASD_FIELD_BX 1
#define ASD_FIELD_BY 2
#define ASD_FIELD_BZ 3
#define ASD_FIELD_CHI 4      /* per-cell chi_par; needs ASD_FLAG_PER_CELL_CHI */
#define ASD_FIELD_Q 5        /* optional source Q per cell (section 3.2): dt Q joins the right-hand
                                side of the first sweep of each step (the x sweep; EUNSUPPORTED
                                with ASD_FLAG_REVERSE_ORDER), forward Euler in the explicit
                                scheme.  Read in place at every step.  Not for the adjoint */

/* asd_desc.flags */
#define ASD_FLAG_PER_CELL_CHI 1u   /* chi is a per-cell field, harmonic mean at faces */
#define ASD_FLAG_ALLOW_UNSTABLE 2u /* skip the EUNSTABLE check */
#define ASD_FLAG_FOUR_STEP 4u      /* asd_step_semi_implicit takes the 4-step scheme (section 2.1, Eq. 4step) */
#define ASD_FLAG_REVERSE_ORDER 8u  /* 2-D: sweep y then x every step (section 2 allows either order) */

/* asd_status flags */
#define ASD_STATUS_NONFINITE 1u    /* NaN/Inf in energy or T */
#define ASD_STATUS_NEG_T 2u        /* min T < 0 */
#define ASD_STATUS_ENERGY_DRIFT 4u /* |E - E0| > 1e-6 |E0| (FP64 sums of the state); never
                                      raised with T = 0 walls or a source */

typedef struct asd_grid_s *asd_grid;

/* Problem description.  Uniform Cartesian grid, cell-centred (section 2). */
typedef struct {
    int32_t ndim;     /* 2 or 3 */
    int32_t bc;       /* ASD_BC_* */
    int32_t dtype;    /* ASD_F32 or ASD_F64: type of T, b and chi */
    int32_t limiter;  /* ASD_LIM_* */
    int64_t n[3];     /* cells along x, y, z; n[2] must be 1 when ndim == 2.
                         n >= 2 (insulating) or n >= 3 (periodic) on every axis.  Every
                         grid line is solved in one workgroup's LDS: n <= 16109 on every
                         axis in FP32 (and n = 16384) and n <= 4096 in FP64, else
                         ASD_EUNSUPPORTED; fewer than 2^31 cells in all */
    double h[3];      /* cell widths (> 0); h[2] ignored in 2-D */
    double chi_par;   /* parallel diffusivity (> 0) when chi is not per cell */
    double chi_perp;  /* isotropic part (>= 0, <= chi) */
    uint32_t flags;   /* ASD_FLAG_* */
    uint32_t reserved; /* must be 0 */
    double chi_exp;   /* 0: chi_par constant (or per cell).  != 0: temperature-dependent
                         chi_par(T) = chi_par (T / chi_tref)^chi_exp (chi ~ T^(5/2) in the
                         paper's application, section 3.3), per cell from the state each sweep
                         (or explicit step) reads, harmonic mean at faces; 0 < chi_exp <= 8,
                         T > 0, no per-cell chi, no EUNSTABLE checks (the caller picks dt),
                         not for the adjoint or batched problems */
    double chi_tref;  /* reference temperature of chi_exp (> 0) */
} asd_desc;

/* Message describing the last error on the calling thread ("" if none). */
const char *asd_last_error(void);

/* Bytes of device workspace asd_init_grid needs for this description:
 * temporary states of the sweeps, re-laid-out copies of b (and chi), and
 * reduction scratch.  Pure host computation. */
int asd_workspace_bytes(const asd_desc *desc, size_t *bytes);

/* Create a grid handle.  dev_ws: device workspace of at least
 * asd_workspace_bytes bytes, 256-byte aligned, owned by the caller and used
 * exclusively by this grid until asd_destroy.  stream: the hipStream_t all
 * work is enqueued on (NULL = default stream).  No device work is enqueued. */
int asd_init_grid(const asd_desc *desc, void *dev_ws, size_t ws_bytes, void *stream, asd_grid *out);

/* Borrow a device array for a field (ASD_FIELD_*).  nelem must equal the
 * cell count, dtype the grid's dtype.  b and chi are read (and re-laid-out
 * into the workspace) at the next step call after they are set; set them
 * again after changing their contents.  T is read and overwritten in place
 * by every step call. */
int asd_set_field(asd_grid g, int32_t field, void *dev_ptr, int64_t nelem, int32_t dtype);

/* nsteps steps of the split semi-implicit scheme (section 2, Eqs. xup and
 * yup; operator form Eq. op_2step; in 3-D a third sweep along z, each sweep
 * taking its transverse differences from its own input state, section 2.1):
 *     T* = (1 + dt D_xx)^-1 (1 - dt D_xy [- dt D_xz]) T^n, then y (then z).
 * The normal term of each sweep is one tridiagonal solve per grid line.
 * dev_energy: NULL or a device FP64 array of nsteps+1 entries that receives
 * sum T dV of the initial state and after every step (FP64 accumulation).
 * EUNSTABLE: 3-D with chi dt / min h^2 > 8.25 (section 2.1) unless
 * ASD_FLAG_ALLOW_UNSTABLE.  nsteps may be 0.
 * With ASD_FLAG_FOUR_STEP the step is the 4-step scheme (section 2.1,
 * Eq. 4step): per direction the transverse term at dt and the normal
 * operator applied twice at dt/2,
 *     T* = (1 + dt D_xx/2)^-2 (1 - dt D_xy [- dt D_xz]) T^n, then y (then z),
 * two tridiagonal solves per line and direction; unconditionally stable in
 * 3-D as well (no EUNSTABLE). */
int asd_step_semi_implicit(asd_grid g, double dt, int32_t nsteps, double *dev_energy);

/* nsteps steps of the explicit limited scheme (forward Euler of the same
 * operator, all faces from T^n; the CFL-bound baseline of sections 1 and 3).
 * EUNSTABLE: chi dt sum_d 1/h_d^2 > 1 in 2-D (section 1: dt < dx^2/(2 chi))
 * or chi dt / min h^2 > 0.444 in 3-D (section 2.1), unless ALLOW_UNSTABLE.
 * dev_energy as above. */
int asd_step_explicit_limited(asd_grid g, double dt, int32_t nsteps, double *dev_energy);

/* Reverse-mode derivative of nsteps semi-implicit steps (2-D).  Given the
 * initial state dev_T0 and lambda_N = dL/dT_N (dev_lambda_final), computes
 * dL/dT_0 into dev_grad_T0 and, when dev_grad_chi is not NULL, dL/dchi per
 * cell (needs ASD_FLAG_PER_CELL_CHI).  The forward states are recomputed
 * from checkpoints taken every ckpt_every steps.  dev_adj_ws: device scratch
 * of asd_adjoint_workspace_bytes bytes (the checkpoints, two segments' states
 * and four work fields).  The grid's T field is not touched.  With more than
 * one segment the recomputation of the next segment runs on a second stream
 * of the grid's own (created on the first such call, default priority, freed
 * by asd_destroy) beside the reverse pass; the work is ordered by events and
 * joined back into the grid's stream before the call returns.  That first
 * call creates the stream and its events, so it must not run while the
 * grid's stream is being captured into a graph; later calls may.
 * The derivative of a limiter at a kink (ab = 0) is taken as zero. */
int asd_adjoint_workspace_bytes(asd_grid g, int32_t nsteps, int32_t ckpt_every, size_t *bytes);
int asd_adjoint_step(asd_grid g, double dt, int32_t nsteps, int32_t ckpt_every, const void *dev_T0,
                     const void *dev_lambda_final, void *dev_grad_T0, void *dev_grad_chi,
                     void *dev_adj_ws, size_t adj_ws_bytes);

/* The same derivative split into its forward and reverse halves, for
 * callers that run the forward steps anyway (a differentiable step map):
 * asd_adjoint_forward advances the grid's T in place by nsteps semi-implicit
 * steps (the states of asd_step_semi_implicit, without energy output) and
 * stores the states at steps 0, k, 2k, ... (k = ckpt_every) in the first
 * ceil(nsteps/k) fields of dev_adj_ws (asd_adjoint_workspace_bytes bytes).
 * asd_adjoint_step_stored then computes what asd_adjoint_step computes from
 * those stored states instead of from dev_T0, without the checkpoint pass;
 * it must be given the same grid, dt, nsteps and ckpt_every, and the grid's
 * b and chi fields must not change in between.  It leaves the checkpoints in
 * place, so several reverse passes (several lambda_N) can follow one forward.
 * Errors as for asd_adjoint_step. */
int asd_adjoint_forward(asd_grid g, double dt, int32_t nsteps, int32_t ckpt_every, void *dev_adj_ws,
                        size_t adj_ws_bytes);
int asd_adjoint_step_stored(asd_grid g, double dt, int32_t nsteps, int32_t ckpt_every,
                            const void *dev_lambda_final, void *dev_grad_T0, void *dev_grad_chi,
                            void *dev_adj_ws, size_t adj_ws_bytes);

/* Synchronise the grid's stream and report status flags (ASD_STATUS_*)
 * from an FP64 reduction of the current T; stats (nullable, 3 doubles)
 * receives {sum T dV, min T, max T}. */
int asd_status(asd_grid g, uint32_t *flags, double *stats);

/* Release the handle (does not free borrowed or workspace memory). */
int asd_destroy(asd_grid g);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation): nsteps
 * steps of asd_step_semi_implicit on the grid `desc` in one call, with no
 * handle, no workspace argument and no allocation.  The scratch (T*, face
 * coefficients, reduction slots, status word) is a static device array of
 * asd_noalloc_scratch_bytes() bytes (64 MiB) that each GPU holds until the
 * process ends; the call uses the array of the current device.  Grids whose
 * asd_workspace_bytes exceeds it are refused with ASD_EUNSUPPORTED (2-D
 * grids up to about 2.6 million cells in FP32, 1.3 million in FP64).
 * dev_T is advanced in place; dev_bx, dev_by (dev_bz in 3-D, dev_chi with
 * ASD_FLAG_PER_CELL_CHI) are read; dev_energy as for asd_step_semi_implicit.
 * No source term; the steps are launched directly on `stream` (no graph).
 * Every call on a GPU shares that GPU's array and rewrites all of it that it
 * uses: calls that overlap on one GPU (two streams, two threads) race. */
size_t asd_noalloc_scratch_bytes(void);
int asd_step_semi_implicit_noalloc(const asd_desc *desc, void *dev_T, const void *dev_bx, const void *dev_by,
                                   const void *dev_bz, const void *dev_chi, double dt, int32_t nsteps,
                                   double *dev_energy, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ASD_H */
