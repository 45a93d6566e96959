/*
 * apdvm -- asymptotic-preserving IMEX Runge-Kutta stepper for the six-velocity
 * (D2Q6) lattice-Boltzmann-type discrete velocity model in the low-Mach diffusive
 * scaling (Dimarco, Klar, Koefler, Pareschi, arXiv 2512.19847), on MI355X (gfx950).
 *
 * The library evolves the six scaled moments (u1, u2, theta, v1, v2, q) of the
 * populations (Section 2.1: the populations and these moments are in one-to-one
 * correspondence) on a doubly periodic, cell-centred nx x ny grid.  One call of
 * apdvm_step advances every simulation of a context by one time step of a globally
 * stiffly accurate IMEX Runge-Kutta method: for each implicit stage, the local
 * implicit relaxation of v (Algorithm 1, step 1), the periodic Helmholtz equation
 * for theta (step 2, solved exactly by a 2D FFT), the velocity update (step 3) and
 * the local implicit relaxation of q (step 4), with the space discretisation of
 * Section 3.2 in its high-order form (WENO5 Lax-Friedrichs fluxes and fourth-order
 * central differences).
 *
 * Conventions for every entry point:
 *  - Host arrays are float64, row-major [ny][nx] (x fastest), owned by the caller and
 *    copied in or out; device arrays follow the same layout and are caller-owned.
 *  - Every call returns an apdvm_status.  A call that fails validation changes
 *    nothing.  No entry point throws or aborts.
 *  - Work is enqueued on the stream given at creation.  apdvm_step enqueues (and
 *    synchronises only when a finite check falls inside the call, see
 *    apdvm_set_finite_check); the host get_* calls synchronise that stream before
 *    returning.  Within a step the library may run part of each stage on a second
 *    stream of its own, forked from and joined back to the creation stream inside the
 *    step (see apdvm_set_overlap), so ordering against the creation stream is as if
 *    every launch were on it.
 *  - A context is not thread-safe: calls on one context must not overlap.
 */
#ifndef APDVM_H
#define APDVM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  APDVM_OK = 0,
  APDVM_ERR_ARG = 1,       /* a size, pointer or parameter is out of range        */
  APDVM_ERR_VELSET = 2,    /* the velocity set is not the paper's six velocities   */
  APDVM_ERR_TABLEAU = 3,   /* tableau not GSA / not ARS-type / malformed           */
  APDVM_ERR_NOMEM = 4,     /* device allocation failed or workspace too small      */
  APDVM_ERR_HIP = 5,       /* a HIP runtime call failed                            */
  APDVM_ERR_NONFINITE = 6, /* input or state holds NaN or Inf                      */
  APDVM_ERR_STATE = 7      /* call out of order (e.g. step before set_fields)      */
} apdvm_status;

typedef enum {
  APDVM_FP64 = 0,       /* every plane and every operation in float64             */
  APDVM_FP32_SPLIT = 1  /* u, v, q and stage terms stored and transported in
                           float32; history sums feeding the implicit relaxations
                           and the Helmholtz right-hand side accumulated in float64;
                           theta and the whole Helmholtz solve in float64          */
} apdvm_precision;

/*
 * One simulation.  Grid: periodic box [0, lx) x [0, ly), cell centres
 * ((i + 1/2) lx/nx, (j + 1/2) ly/ny) (Section 3.2).  nx, ny must be even, >= 8, and
 * of the form 2^a 3^b; each at most 8192.
 *
 * Velocity set: q must be 6.  cx, cy may be NULL (the paper's set
 * c_i = (cos(pi(i-1)/3), sin(pi(i-1)/3)), Section 2.1) or point to 6 values each,
 * which must equal that set to 1e-12, else APDVM_ERR_VELSET.
 *
 * eps >= 0 is the Knudsen number (eps = 0 runs the exact limit scheme); mach > 0.
 * tau < 0 derives tau = 4 eps / mach (eps = Ma/Re and the limit Reynolds number is
 * 4/tau, Section 2); tau >= 0 is used as given (the paper's tests use 0 and 0.05).
 *
 * Tableau: s stages (2 <= s <= 8), a_ex and a_im s x s row-major, b_ex and b_im of
 * length s (Section 3.1).  Must be globally stiffly accurate, a_ex strictly lower
 * triangular and a_im lower triangular, and either of ARS type (a_im[0][0] = 0,
 * a_im[i][0] = 0, nonzero diagonal after the first stage) or of type A (every diagonal
 * entry nonzero, s <= 7; run internally as s + 1 stages whose first is the state at
 * time n with zero coefficients); else APDVM_ERR_TABLEAU.
 *
 * dt > 0 is used as given.  dt <= 0 derives the largest dt with
 *   ct dt max(umax, 1, tau eps / (tau eps^2 + ct dt)) <= cfl h  and
 *   ct dt (tau/4) ct dt / (tau eps^2 + ct dt) <= c_visc h^2,
 * h = min(lx/nx, ly/ny), ct the largest explicit stage abscissa, umax the largest
 * |u| of the fields given to apdvm_set_fields (the derivation happens there), and 1
 * the Lax-Friedrichs dissipation speed (alpha = 1, Section 3.2), whose jump term acts
 * explicitly.
 *
 * Space discretisation (Section 3.2): weno_order 5 (or 0) reconstructs every
 * Lax-Friedrichs flux with fifth-order WENO (Jiang-Shu), 3 with the third-order WENO of
 * the convergence tables of Section 4.1; central_order 4 (or 0) uses fourth-order
 * central differences for D0.u, D0 theta, D0^2:B(v) and D_Delta (and the matching
 * Fourier symbol in the Helmholtz solve), 2 the second-order ones printed in Section
 * 3.2.  Both must be the same for every instance of a context; else APDVM_ERR_ARG.
 */
typedef struct {
  int32_t nx, ny;
  double lx, ly;
  int32_t q;
  const double *cx, *cy;
  double eps, mach, tau;
  int32_t s;
  const double *a_ex, *b_ex, *a_im, *b_im;
  double dt, cfl, c_visc;
  int32_t precision; /* apdvm_precision; must be the same for every instance */
  int32_t weno_order, central_order; /* 5 / 4 (0 = default) or 3 / 2 */
} apdvm_config;

typedef struct apdvm_ctx apdvm_ctx;

/* Bytes of device workspace that apdvm_create needs for these configurations
 * (n >= 1 instances sharing one tableau and precision).  Host-only; no GPU call. */
apdvm_status apdvm_workspace_bytes(int32_t n, const apdvm_config *cfgs, size_t *bytes);

/* Create a context holding n >= 1 independent simulations, all advanced together by
 * apdvm_step.  All instances must share s, the tableau and the precision.
 * dev_ws: device workspace of ws_bytes >= apdvm_workspace_bytes, owned by the caller
 * and outliving the context; NULL makes the library allocate (and free) its own.
 * hip_stream: a hipStream_t cast to void*, or NULL for the default stream.
 * On success *out receives the context. */
apdvm_status apdvm_create(int32_t n, const apdvm_config *cfgs, void *dev_ws,
                          size_t ws_bytes, void *hip_stream, apdvm_ctx **out);

/* Initial fields of instance k from host arrays.  v1 and v2 may both be NULL (then
 * v = F(u) = (1/2 (u2^2 - u1^2), u1 u2), local equilibrium); q may be NULL (then 0).
 * Rejects NaN/Inf (APDVM_ERR_NONFINITE, nothing changed).  The fields also become the
 * snapshot of the finite check (apdvm_set_finite_check).  The step counter is not
 * changed (a checkpoint restore is set_fields for every instance, then apdvm_set_step).
 * Synchronises the stream. */
apdvm_status apdvm_set_fields(apdvm_ctx *ctx, int32_t k, const double *u1,
                              const double *u2, const double *theta, const double *v1,
                              const double *v2, const double *q);

/* Same from six device arrays of nx*ny float64 each (u1, u2, theta, v1, v2, q; no
 * NULLs), read on the context's stream: the caller makes their contents complete in
 * that stream's order (produced on it, or an event it waits on).  The values are checked
 * on the device first (APDVM_ERR_NONFINITE if any is NaN or Inf, nothing changed), in
 * the same pass that gives the mean of theta and max |u| for the dt rule; in the
 * FP32-split form the rounding to float runs on the device.  Synchronises the stream
 * before returning, so the arrays may be reused afterwards. */
apdvm_status apdvm_set_fields_device(apdvm_ctx *ctx, int32_t k, const double *const dev[6]);

/* Initial fields of instance k from populations F[6][ny][nx] (host, float64), mapped
 * to scaled moments by R = 1 + 2 eps^2 theta, U = eps u, V = eps^2 v, Q = eps^3 q with
 * (R, U, V, Q) the moments of F for the basis 1, c, 1/2 - c_x^2, c_x c_y,
 * c_x (c_y^2 - 1/4).  Needs eps > 0. */
apdvm_status apdvm_set_populations(apdvm_ctx *ctx, int32_t k, const double *F);

/* Enqueue nsteps >= 0 time steps of every instance on the context's stream.  Per
 * implicit stage: step 1 (fused into the previous stage's terms), then the right-hand
 * side and the Helmholtz solve of step 2 beside the parts of steps 3 and 4 that do not
 * involve theta(i) (q(i), and u(i) short of its dt a_ii D0 theta(i) term), then the
 * completion of u(i) with the stage's reusable terms.
 * After every K-th step (K from apdvm_set_finite_check) the state of every instance is
 * checked on the device; a state that passes becomes the snapshot.  If any check of the
 * call fails, the call synchronises, makes the snapshot (the last state that passed, of
 * every instance) the current state again, sets the step counter back to its step and
 * returns APDVM_ERR_NONFINITE.  A call containing a check synchronises the stream at its
 * end, so such calls cannot be captured into a caller's graph (set K = 0 for that). */
apdvm_status apdvm_step(apdvm_ctx *ctx, int64_t nsteps);

/* Finite check of apdvm_step every `every` steps (counted by the step counter; 0 turns it
 * off).  Default 64, or the value of the environment variable APDVM_FINITE_EVERY at
 * apdvm_create.  Cost per check: one read of the six state planes and, when it passes,
 * one copy of them into the snapshot.  Host-only. */
apdvm_status apdvm_set_finite_check(apdvm_ctx *ctx, int32_t every);

/* Copy the six fields of instance k to host arrays (any pointer may be NULL to skip
 * that field).  Synchronises the stream. */
apdvm_status apdvm_get_fields(apdvm_ctx *ctx, int32_t k, double *u1, double *u2,
                              double *theta, double *v1, double *v2, double *q);

/* Same into six device arrays of nx*ny float64 each (NULL entries skipped), enqueued on
 * the context's stream and not synchronised: a consumer on another stream waits for it
 * (an event recorded on the context's stream after this call). */
apdvm_status apdvm_get_fields_device(apdvm_ctx *ctx, int32_t k, double *const dev[6]);

/* Physical moments of instance k (host): rho = 1 + 2 eps^2 theta, u, and the pressure
 * p = theta - |u|^2 / 2 (Section 2.1).  Synchronises the stream. */
apdvm_status apdvm_get_moments(apdvm_ctx *ctx, int32_t k, double *rho, double *u1,
                               double *u2, double *p);

/* Populations F[6][ny][nx] of instance k (host), the inverse of the map of
 * apdvm_set_populations.  Needs eps > 0.  Synchronises the stream. */
apdvm_status apdvm_get_populations(apdvm_ctx *ctx, int32_t k, double *F);

/* Time step, tau and the number of steps taken, for instance k. */
apdvm_status apdvm_get_info(apdvm_ctx *ctx, int32_t k, double *dt, double *tau,
                            int64_t *step);

/* Set the step counter (checkpoint restore: set_fields + set_step). */
apdvm_status apdvm_set_step(apdvm_ctx *ctx, int64_t step);

/* Diagnostics of instance k, computed on the device and synchronised:
 * out[0] sum theta h_x h_y, out[1] sum u1 h_x h_y, out[2] sum u2 h_x h_y,
 * out[3] max |D0.u| (central divergence of the context's central_order, the divergence
 * diagnostic of Section 4), out[4] min vorticity, out[5] max vorticity (the same central
 * D_x u2 - D_y u1), out[6] kinetic energy 1/2 sum |u|^2 h_x h_y, out[7] 1 if every
 * value of the six fields is finite else 0. */
apdvm_status apdvm_diagnostics(apdvm_ctx *ctx, int32_t k, double out[8]);

/* For callers that cannot allocate (code under HIP graph capture, tight serving loops):
 * apdvm_diagnostics of instance k with the eight values written to the device array
 * dev_out[8] (caller-owned) in the same order, enqueued on the context's stream and not
 * synchronised; no allocation, memset or host copy.  The per-workgroup partials live in
 * a static device array of the library (64 KiB, 1024 records, one per GPU, held until
 * the process ends): the workgroups loop over the tiles of larger instances, so every
 * instance size fits, and APDVM_ERR_ARG would report a record count beyond 1024.  Every
 * call on a GPU uses that GPU's array and overwrites the records it reads, so calls that
 * overlap on one GPU (other contexts or streams) race; calls in stream order do not.
 * The values equal those of apdvm_diagnostics bit for bit. */
apdvm_status apdvm_diagnostics_device(apdvm_ctx *ctx, int32_t k, double *dev_out);

/* Number of kernel launches one apdvm_step(ctx, 1) enqueues (for profiling). */
apdvm_status apdvm_launches_per_step(apdvm_ctx *ctx, int32_t *count);

/* Launch mode.  on = 0 (default): every kernel of a step is launched on its own.
 * on = 1: each step replays a HIP graph of the step's launches (with the fork and join
 * of the second stream as graph dependencies), captured on first use; needs a created
 * (non-NULL) stream at apdvm_create, else APDVM_ERR_ARG. */
apdvm_status apdvm_set_graph(apdvm_ctx *ctx, int32_t on);

/* Stream structure of a step.  on = 1 (default): per stage, the Helmholtz right-hand
 * side and solve (classes 0-3) run on the context's second stream while the theta-free
 * part of steps 3 and 4 (class 4) and the q part of the stage terms (class 6) run on the
 * creation stream; the stage-terms launch (class 5) waits for both.  on = 0: every launch
 * on the creation stream, in the same order; results identical to on = 1 bit for bit.
 * on = 2: every launch on the creation stream, with the update launch (class 4) after
 * the solve completing u, Hu and L theta of the stage from its theta itself (the
 * theta part of Algorithm 1, step 3), so the stage-terms launch reads the finished u and
 * the intermediate u* and hu make no round trip through memory; in the FP32-split form
 * the stage-terms launch also forms te2 D_W q (so class 6 is not launched); results
 * equal those of on = 0 and 1 to rounding (in the FP32-split form the float increment is
 * rounded once, after the theta part, instead of before it).  apdvm_autotune picks the
 * fastest.  Synchronises both streams when the setting changes. */
apdvm_status apdvm_set_overlap(apdvm_ctx *ctx, int32_t on);

/* Current stream structure (1: solve beside steps 3 and 4, 0: one stream, 2: one stream
 * with the theta completion in the update launch).  Host-only. */
apdvm_status apdvm_get_overlap(apdvm_ctx *ctx, int32_t *on);

/* Kernel classes of a step, used by the profiling and tuning calls below:
 * 0 step-2 right-hand side, 1 Helmholtz rows forward FFT (half spectra stored
 * column-major), 2 Helmholtz columns (FFT along y of whole contiguous columns, symbol
 * divide, inverse FFT), 3 Helmholtz rows inverse FFT, 4 steps 3 and 4 short of theta (q,
 * and u without its theta gradient), 5 completion of u with theta and the stage terms
 * reused by later stages, together with step 1 (the relaxation of v) of the next stage,
 * 6 the q part te2 D_W q of the stage terms (WENO of q +- v, before theta is known). */
#define APDVM_NUM_KERNEL_CLASSES 7

/* From now on time every launch of kernel class cls with a pair of HIP events that
 * hipExtLaunchKernelGGL sets at the start and end of the kernel's own execution (cls = -1
 * stops).  A step with timed launches runs launch by launch with every launch on the
 * creation stream, so that each timed launch runs by itself; other steps replay the graph
 * when graphs are on and use the second stream when overlap is on.  Synchronises the
 * stream and clears earlier timings. */
apdvm_status apdvm_timing_enable(apdvm_ctx *ctx, int32_t cls);

/* Bracket the timed class only in every stride-th step (stride >= 1, default 1; every
 * launch of the class within such a step), counted from apdvm_timing_enable: the events
 * cost a little time themselves, so a throughput run can sample the class instead of
 * timing each launch.  Host-only. */
apdvm_status apdvm_timing_stride(apdvm_ctx *ctx, int32_t stride);

/* Synchronise, then return the number of timed launches since apdvm_timing_enable and
 * the sum of their durations in milliseconds. */
apdvm_status apdvm_timing_read(apdvm_ctx *ctx, int64_t *launches, double *total_ms);

/* Algorithmic bytes that one step moves through the kernels of class cls (-1: every
 * class): each plane a launch must read or write counted once, summed over the
 * instances; and the number of such launches per step.  Host-only. */
apdvm_status apdvm_traffic(apdvm_ctx *ctx, int32_t cls, double *bytes_per_step,
                           int32_t *launches_per_step);

/* Launch-shape choices as apdvm_autotune reports them and apdvm_set_tuning takes them
 * (APDVM_TUNING_LEN entries): entries 0..6 per kernel class, with the tile height (8 or
 * 16 rows of 64 cells) for the stencil classes 0, 4, 5 and 6 (the FFT entries read 1);
 * entries 7, 8, 9 and 10 the workgroup threads (256 or 512) of classes 0, 4, 5 and 6.
 * Shapes: 64 x 8 or 64 x 16 tiles on 256 or 512 threads. */
#define APDVM_TUNING_LEN 11

/* Autotune the launch shapes and the stream structure: for the stencil kernel classes (0,
 * 4, 5, 6) each shape is timed with HIP events over steps_per_trial steps of the live
 * simulation, once with the kernels of structures 0 and 1 and once with those of
 * structure 2 (apdvm_set_overlap), and the fastest of each set is kept.  Then whole steps
 * of the three structures, each with its shapes, are timed in the context's launch mode,
 * twice each and interleaved, each run at least 2 steps_per_trial steps and about 10 ms,
 * and the fastest kept.  The state, the step counter and the launch mode are restored
 * afterwards (this call allocates a temporary device copy of the state).  If the
 * environment variable APDVM_TUNE_CACHE names a file, a previous choice for the same
 * context shape is read from it and no trial runs; new choices are appended to it.
 * choice (NULL, or APDVM_TUNING_LEN entries) receives the shape choice.  Needs fields on
 * every instance. */
apdvm_status apdvm_autotune(apdvm_ctx *ctx, int32_t steps_per_trial, int32_t *choice);

/* Set the launch shapes directly (APDVM_TUNING_LEN entries, the format apdvm_autotune
 * reports): a (tile height, threads) pair among the shapes above for classes 0, 4, 5 and
 * 6; the other entries are ignored.  APDVM_ERR_ARG for any other pair.  Host-only. */
apdvm_status apdvm_set_tuning(apdvm_ctx *ctx, const int32_t *choice);

/* Release the context (and the workspace if the library allocated it).  NULL ok. */
void apdvm_destroy(apdvm_ctx *ctx);

/* Batched form (hundreds of independent simulations of uneven sizes and eps / Ma
 * advanced together).  A context already holds any number of instances, each
 * with its own grid, eps, tau, dt and FFT plan, and every launch of a step covers all of
 * them through its work tables; these names are the same calls under the batch
 * vocabulary (apdvm_batch is the context type). */
typedef struct apdvm_ctx apdvm_batch;
apdvm_status apdvm_batch_create(int32_t n, const apdvm_config *cfgs, void *dev_ws,
                                size_t ws_bytes, void *hip_stream, apdvm_batch **out);
apdvm_status apdvm_batch_set_fields(apdvm_batch *b, int32_t k, const double *u1,
                                    const double *u2, const double *theta, const double *v1,
                                    const double *v2, const double *q);
apdvm_status apdvm_batch_step(apdvm_batch *b, int64_t nsteps);
apdvm_status apdvm_batch_get_fields(apdvm_batch *b, int32_t k, double *u1, double *u2,
                                    double *theta, double *v1, double *v2, double *q);
void apdvm_batch_destroy(apdvm_batch *b);

/* Static text for a status code. */
const char *apdvm_status_string(apdvm_status s);

#ifdef __cplusplus
}
#endif

#endif /* APDVM_H */
