/*
 * asd_extra.h — batched problems, launch tuning and measurement helpers of
 * libasd.  Same conventions as asd.h (status codes, borrowed memory,
 * caller-provided workspace, stream-ordered enqueue).
 */
#ifndef ASD_EXTRA_H
#define ASD_EXTRA_H

#include "asd.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ batch
 * Many independent 2-D problems of uneven sizes advanced together: the
 * semi-implicit step of asd.h (section 2, Eqs. xup / yup) applied to each
 * problem with its own grid, b field, chi_par and dt.  Problems share bc
 * (periodic, insulating or T = 0 walls; no source term), dtype and limiter
 * (taken from descs[0]); each desc gives n, h, chi_par, chi_perp of its
 * problem.  FP32 or FP64; ndim must be 2. */
typedef struct asd_batch_s *asd_batch;

/* Workspace bytes for nprob problems (descs: host array of nprob). */
int asd_batch_workspace_bytes(const asd_desc *descs, int32_t nprob, size_t *bytes);

/* Create a batch; dev_ws as for asd_init_grid.  No device work is enqueued. */
int asd_batch_init(const asd_desc *descs, int32_t nprob, void *dev_ws, size_t ws_bytes, void *stream,
                   asd_batch *out);

/* Borrow the device arrays of problem p (T advanced in place; bx, by read at
 * the next step call) and set its time step dt (> 0, finite). */
int asd_batch_set_problem(asd_batch b, int32_t p, void *dev_T, void *dev_bx, void *dev_by, double dt);

/* nsteps steps of every problem.  Problems must be 2-D with a constant
 * chi_par; every problem gets its own dt.
 *   mode 0: one persistent launch for all problems and all steps
 *           (work-groups own whole problems, assigned largest first);
 *   mode 1: one launch per problem per sweep (the sequential reference);
 *   mode 2: one launch per sweep for all problems (grouped line tiles);
 *   mode -1: the schedule chosen by asd_batch_tune (0 before tuning).
 * Modes 0 and 2 with nsteps >= 2 on a non-default stream are captured into
 * one graph and replayed: the whole call is one graph launch. */
int asd_batch_step(asd_batch b, int32_t nsteps, int32_t mode);

/* asd_batch_step with per-problem FP64 outputs: dev_energy (device, FP64,
 * nprob * (nsteps + 1) entries, problem-major) receives sum T dV of every
 * problem's initial state and after every step, and the per-problem status
 * (see asd_batch_status) is updated: NONFINITE, NEG_T and ENERGY_DRIFT
 * (|E - E0| > 1e-6 |E0| against the call's initial energy; not with T = 0
 * walls).  Mode 0 reduces inside the persistent launch (each workgroup holds
 * all of a problem's tiles); mode 2 has every y-sweep tile write a partial
 * and folds them per problem; mode 1 uses each problem's own step loop.
 * dev_energy NULL: as asd_batch_step.  Modes 0 and 2 on a non-default
 * stream run as one captured graph per call (up to 2048 steps; see
 * asd_batch_set_graphs). */
int asd_batch_step_energy(asd_batch b, int32_t nsteps, int32_t mode, double *dev_energy);

/* Synchronise the batch's stream and copy the per-problem status bits
 * (ASD_STATUS_*, host array of nprob) and, when stats is not NULL, the last
 * energy-producing call's final {sum T dV, min T, max T} per problem (host
 * array of 3 nprob).  The bits are sticky until read and cleared here. */
int asd_batch_status(asd_batch b, uint32_t *flags, double *stats);

/* Enable (1, the default) or disable (0) graph capture of batch calls. */
int asd_batch_set_graphs(asd_batch b, int32_t on);

/* Work-group size of the batch kernels: 256, 512 or 1024 threads
 * (EUNSUPPORTED if some problem's lines do not fit). */
int asd_batch_set_block(asd_batch b, int32_t nthreads);

/* Tile body of the batch kernels (ASD_SWEEP_FACE_SLOTS, the default, or
 * ASD_SWEEP_CELL_SLOTS; see asd_set_sweep_kernel) at the current work-group
 * size: EINVAL for another value, EUNSUPPORTED if some problem's lines do
 * not fit that body. */
int asd_batch_set_variant(asd_batch b, int32_t variant);
int asd_batch_get_variant(asd_batch b, int32_t *variant);

/* Per-lane capacity of the batch kernels: the smallest of 4, 8, 16 cells at
 * or above mmax that fits every problem at the current work-group size and
 * tile body (each problem then runs that capacity, half of it, or with
 * capacity 16 also 4).  With capacity 16 on the face-slot body, problems
 * whose lines have 257 to 512 cells run two lines per wave (32 lanes per
 * line).  EINVAL for mmax other
 * than 4, 8 or 16, EUNSUPPORTED if nothing fits. */
int asd_batch_set_capacity(asd_batch b, int32_t mmax);

/* Autotuner: time modes 0 and 2 at every admissible work-group size,
 * per-lane capacity (4, 8 or 16 cells) and tile body on probe_steps steps
 * (this advances the problems' T), keep the
 * fastest for mode -1 and report it (nullable outputs; the body through
 * asd_batch_get_variant).  Synchronises the stream. */
int asd_batch_tune(asd_batch b, int32_t probe_steps, int32_t *best_mode, int32_t *best_threads);

int asd_batch_destroy(asd_batch b);

/* ------------------------------------------------------------ diagnostics
 * nsteps steps of the semi-implicit scheme (ASD_SCHEME_SEMI_IMPLICIT, as
 * asd_step_semi_implicit, with the grid's ASD_FLAG_FOUR_STEP and
 * ASD_FLAG_REVERSE_ORDER) or of the explicit limited scheme
 * (ASD_SCHEME_EXPLICIT, as asd_step_explicit_limited), recording for the
 * initial state and after every step the FP64 energy sum T dV and the
 * minimum and maximum of T (the monotonicity diagnostics of section 3.1).
 * dev_series: device FP64 array of 3 (nsteps+1) entries, (E, Tmin, Tmax)
 * per state.  Errors as for the two step calls. */
#define ASD_SCHEME_SEMI_IMPLICIT 0
#define ASD_SCHEME_EXPLICIT 1
int asd_step_series(asd_grid g, int32_t scheme, double dt, int32_t nsteps, double *dev_series);

/* ----------------------------------------------------------------- tuning
 * Launch shape of the sweep along `axis`: waves per line (wpl), lines per
 * work-group (lpw), segments per line (P) and per-lane capacity (mmax). */
int asd_get_sweep_config(asd_grid g, int32_t axis, int32_t *wpl, int32_t *lpw, int32_t *P, int32_t *mmax);

/* Request a launch shape (wpl, lpw powers of two); EUNSUPPORTED if it does
 * not fit the register or LDS budget.  Same as asd_set_sweep_shape with
 * io = 1. */
int asd_set_sweep_config(asd_grid g, int32_t axis, int32_t wpl, int32_t lpw);

/* Launch shape with io (1 or 2): the loads, face evaluation and stores of a
 * line run on io * wpl waves, the line solve on wpl of them (a workgroup has
 * 64 * wpl * io * lpw threads).  Face-slot tile body.  EUNSUPPORTED if it
 * does not fit. */
int asd_set_sweep_shape(asd_grid g, int32_t axis, int32_t wpl, int32_t lpw, int32_t io);

/* Launch shape and tile body of the sweep along `axis`.  Both bodies compute
 * the same sweep of section 2 (Eqs. xup / yup) and differ in their LDS use:
 *   ASD_SWEEP_FACE_SLOTS (0): faces evaluated while a tile is staged,
 *       8 bytes of LDS per cell in FP32 (longer lines fit; io 1 or 2);
 *   ASD_SWEEP_CELL_SLOTS (1): cells staged as 16-byte slots, faces evaluated
 *       in the solve (a shorter staging chain; io must be 1).
 * EINVAL for a bad argument, EUNSUPPORTED if the shape does not fit the
 * register or LDS budget of that body.  The autotuner (asd_tune) tries both. */
#define ASD_SWEEP_FACE_SLOTS 0
#define ASD_SWEEP_CELL_SLOTS 1
int asd_set_sweep_kernel(asd_grid g, int32_t axis, int32_t wpl, int32_t lpw, int32_t io, int32_t variant);

/* The io factor of the sweep along `axis` (see asd_set_sweep_shape). */
int asd_get_sweep_io(asd_grid g, int32_t axis, int32_t *io);

/* The tile body (ASD_SWEEP_FACE_SLOTS / ASD_SWEEP_CELL_SLOTS) of the sweep
 * along `axis`. */
int asd_get_sweep_variant(asd_grid g, int32_t axis, int32_t *variant);

/* Time every admissible (tile body, wpl, lpw, io) of each sweep on the grid's stream with
 * HIP events (reps whole steps each, best of three timings, T -> workspace,
 * T unchanged) and keep the fastest; two passes over the axes.  Needs T and
 * b set.  Synchronises the stream. */
int asd_tune(asd_grid g, double dt, int32_t reps);

/* hipGraph capture of multi-step calls (only with a non-default stream):
 * ASD_GRAPHS_OFF launches every call directly; ASD_GRAPHS_AUTO (the
 * default) captures calls of 64 steps or more and launches shorter calls
 * directly (a graph launch starts its first kernel later than a direct
 * launch, which costs a short call more than the host-side launches do);
 * ASD_GRAPHS_ALWAYS captures every call of 2 steps or more.  A captured call
 * is replayed from a small per-grid cache.  A graph holds at most 2048
 * steps: longer calls replay it and launch the remainder directly, or, when
 * they produce per-step outputs, launch every step directly.  EINVAL for
 * another mode. */
#define ASD_GRAPHS_OFF 0
#define ASD_GRAPHS_AUTO 1
#define ASD_GRAPHS_ALWAYS 2
int asd_set_graphs(asd_grid g, int32_t mode);

/* ------------------------------------------------------------ measurement
 * Time one sweep kernel in isolation.  reps == 0: enqueue one sweep chain
 * from T into the workspace so that every sweep's input holds a valid
 * state.  reps > 0: enqueue reps launches of the sweep along `axis`, from
 * its input state to a workspace buffer.  T is never written. */
int asd_bench_sweep(asd_grid g, int32_t axis, double dt, int32_t reps);

/* Plain streaming copy of nbytes (multiple of 4) from src to dst on stream:
 * the calibration kernel for HBM byte counters. */
int asd_bench_copy(const void *src, void *dst, size_t nbytes, void *stream);

/* Streaming copy of nbytes (multiple of 4; src and dst 16-byte aligned) with
 * 16-byte accesses and several loads in flight per lane: the practical HBM
 * bandwidth ceiling the kernels are measured against. */
int asd_bench_copy_wide(const void *src, void *dst, size_t nbytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ASD_EXTRA_H */
