/*
 * lddmm.h -- C ABI of liblddmm, landmark geodesic shooting on MI355X (gfx950).
 *
 * The library computes, on one GPU, the objects of landmark matching by
 * geodesic shooting (paper Sec. 2.1):
 *
 *   kernel       g_ij = exp(-|q_i - q_j|^2 / (2 sigma^2))
 *   Hamiltonian  H(q,p) = 1/2 sum_ij g_ij p_i . p_j                   (eq. 1)
 *   flow         dq/dt = dH/dp, dp/dt = -dH/dq, explicit Euler with
 *                dt = 1/T over t in [0,1], q and p updated together   (eq. 2; Alg. 1)
 *   loss         L(p0) = H(q0,p0) + lambda sum_i |q_i(1) - x_i|^2     (eq. 3)
 *   gradient     dL/dp0 by the exact adjoint of the discrete Euler map,
 *                run backwards in time                                (Alg. 1)
 *   solver       L-BFGS over p0                                       (Sec. 2.1; Alg. 1)
 *   velocity     v(x,t) = sum_l g(|q_l(t) - x|) p_l(t) at any points x, and
 *                the flow of points carried by the landmark motion    (eq. 4)
 *
 * Options per call (lddmm_params): the precision of the pair sums, trajectory
 * checkpointing, the energy term taken at t = 1 instead of t = 0 (the loss as
 * Alg. 1 evaluates it), a planar specialisation (Sec. 2.5) and classical
 * Runge-Kutta steps in place of the Euler steps (an extension).
 *
 * Conventions shared by every call:
 *   - Point sets (q0, p0, target, q1, p1, grad) are DEVICE pointers to [n][3]
 *     row-major FP64 arrays owned by the caller.  They must not overlap one
 *     another.  Results are always FP64, whatever the pair-sum precision.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Every call enqueues its work on that stream and returns without
 *     waiting; outputs are valid once the stream has reached that point.
 *   - Device scalars (loss, H0) are written by the GPU, in stream order.
 *   - Functions never throw and never abort.  Invalid arguments are reported
 *     synchronously (LDDMM_EINVAL) before any work is enqueued; a detail
 *     string is then available from lddmm_last_error().  A HIP runtime
 *     failure is LDDMM_EDEVICE.  Non-finite intermediates are flagged on the
 *     device and reported by lddmm_ctx_check().
 *   - A context serialises its calls: one context must not be used from two
 *     threads at once, nor on two streams whose work overlaps, because every
 *     call reuses the context's workspace.
 *   - Evaluations (lddmm_shoot_forward/_grad/_grad_all, lddmm_flow) enqueue
 *     kernels and device-to-device copies only, so a stream capture records
 *     them into a hipGraph whose replays repeat them.  The workspace must
 *     already be large enough when capture starts (one uncaptured call of the
 *     same shape), and a graph stays valid only until a call on a larger
 *     problem makes the context grow (reallocate) its workspace.
 */
#ifndef LDDMM_H
#define LDDMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LDDMM_OK = 0,
  LDDMM_ENOTCONV = 1,      /* solver stopped without meeting its tolerance; result written */
  LDDMM_EINVAL = -1,       /* invalid argument */
  LDDMM_ENOMEM = -2,       /* device allocation failed */
  LDDMM_EDEVICE = -3,      /* HIP runtime error */
  LDDMM_ENONFINITE = -4,   /* NaN or Inf met on the device */
  LDDMM_EBUSY = -5         /* result not ready yet */
} lddmm_status;

/* Precision of the O(N^2) pair sums.  State, Euler updates, H, the loss and
 * the optimiser are FP64 in every mode. */
typedef enum {
  LDDMM_FP32 = 0,          /* FP32 pair terms, one running FP32 sum per wave */
  LDDMM_FP32_COMP = 1,     /* FP32 pair terms, FP32 sums of 72 pairs folded into FP64 */
  LDDMM_FP64 = 2           /* FP64 throughout */
} lddmm_precision;

/* Energy term of the loss.  INITIAL: H(q0, p0), as in eq. 3.  FINAL:
 * H(q(1), p(1)), the energy as Alg. 1 evaluates it after its forward loop;
 * the two agree as dt -> 0 (H is conserved by the continuous flow).  With
 * FINAL the gradients are the adjoint at t = 0 alone (no direct dependence
 * of the energy on q0, p0), at the cost of one more forward pair-sum launch
 * per evaluation.  The server supports INITIAL only. */
typedef enum { LDDMM_ENERGY_INITIAL = 0, LDDMM_ENERGY_FINAL = 1 } lddmm_energy;

/* Time stepping of eq. 2 over [0, 1] in T steps of dt = 1/T.  EULER: explicit
 * Euler steps with q and p updated together (Alg. 1, forward loop).  RK4: the
 * classical fourth-order Runge-Kutta step of the same field f = (Hp, -Hq),
 *   k1 = f(y), k2 = f(y + dt/2 k1), k3 = f(y + dt/2 k2), k4 = f(y + dt k3),
 *   y' = y + dt/6 (k1 + 2 k2 + 2 k3 + k4),
 * an extension beyond the paper's steps: four pair-sum launches per step
 * forward and four backward, errors O(dt^4) instead of O(dt).  The gradients
 * are the exact adjoint of the stage equations, and the flow of points takes
 * the same stages.  The trajectory keeps the four stage states of every step
 * (4 T + 1 records; 4 s + 1 with checkpoints every s steps).  A server
 * takes the integrator of its configuration for every job. */
typedef enum { LDDMM_EULER = 0, LDDMM_RK4 = 1 } lddmm_integrator;

typedef struct {
  int32_t n;               /* landmarks, 1..2^26 */
  int32_t T;               /* time steps, 1..2^20 (dt = 1/T) */
  double sigma;            /* Gaussian kernel width (standard deviation), > 0 */
  double lambda;           /* mismatch weight, >= 0 */
  int32_t precision;       /* lddmm_precision */
  int32_t ckpt_every;      /* 0: keep the whole trajectory; s > 0: keep every
                              s-th FP64 state and recompute each segment of s
                              steps before its backward pass (same results) */
  int32_t energy;          /* lddmm_energy: the loss's energy term */
  int32_t dim;             /* 3 (or 0): landmarks in 3D.  2: planar problem, the
                              z components of every input are 0; the pair sums
                              leave the z terms out (about 30 % fewer
                              instructions per pair) and every z output is 0.
                              Inputs with a non-zero z give undefined results.
                              A server takes planar and 3D jobs side by side. */
  int32_t integrator;      /* lddmm_integrator (0: Euler steps) */
} lddmm_params;

typedef struct lddmm_ctx lddmm_ctx;

/* A context binds one GPU and owns a device workspace (trajectory, adjoint
 * state, partial sums), grown on demand and reused across calls, plus the
 * solver's workspace (lddmm_solve).
 *   device           : HIP device ordinal
 *   hbm_budget_bytes : cap on the two workspaces together, in bytes; a call
 *                      whose workspace would exceed it fails with ENOMEM
 *                      before enqueuing anything, and the context stays
 *                      usable.  0: no cap (limited by the device's memory).
 *   out              : receives the context
 * Errors: EINVAL (null out, bad device), EDEVICE. */
lddmm_status lddmm_ctx_create(int device, size_t hbm_budget_bytes, lddmm_ctx** out);

/* Waits for the context's pending work, frees the workspace and the context.
 * NULL is accepted. */
lddmm_status lddmm_ctx_destroy(lddmm_ctx* ctx);

/* Device workspace, in bytes, that a call with *params needs.  Pure host
 * computation.  Errors: EINVAL. */
lddmm_status lddmm_workspace_size(const lddmm_params* params, size_t* bytes);

/* Forward shooting (Alg. 1, forward loop; eq. 2): integrates (q, p) from
 * (q0, p0) over T steps of params->integrator (Euler by default).
 *   q0, p0 : in,  [n][3] device FP64
 *   q1, p1 : out, [n][3] device FP64, q(1) and p(1); either may be NULL
 *   H0     : out, device FP64 scalar H(q0,p0) (eq. 1); may be NULL
 * Errors: EINVAL, ENOMEM, EDEVICE. */
lddmm_status lddmm_shoot_forward(lddmm_ctx* ctx, const lddmm_params* params, const double* q0,
                                 const double* p0, double* q1, double* p1, double* H0,
                                 void* stream);

/* Loss and gradient (Alg. 1 ComputeGradient; eq. 3): one forward pass, the
 * loss, and one adjoint pass.
 *   q0, p0, target : in,  [n][3] device FP64 (template, momentum, target x)
 *   out3           : out, 3 device FP64 scalars {L, H(q0,p0), sum_i |q_i(1)-x_i|^2}
 *   grad           : out, [n][3] device FP64, dL/dp0
 *   q1             : out, [n][3] device FP64 q(1); may be NULL
 * Errors: EINVAL, ENOMEM, EDEVICE. */
lddmm_status lddmm_shoot_grad(lddmm_ctx* ctx, const lddmm_params* params, const double* q0,
                              const double* p0, const double* target, double* out3,
                              double* grad, double* q1, void* stream);

/* lddmm_shoot_grad for callers that cannot allocate device memory (code
 * under hipGraph stream capture, tight serving loops, hosts that forbid
 * hipMalloc): the same arguments, kernels and results (bitwise), but the
 * workspace is a fixed device array of 64 MiB that the library holds on every
 * GPU it runs on until the process ends, instead of the context's growable
 * workspace.  The call allocates nothing (no hipMalloc, hipFree or event
 * creation) and is not timed by lddmm_ctx_set_timing.
 *   limit : the workspace lddmm_workspace_size reports for *params must be
 *           at most 64 MiB (e.g. n = 4096 with T = 40 in FP32-compensated
 *           mode takes 8.3 MiB; n = 16384, T = 100 takes 63 MiB with the
 *           whole trajectory and 26 MiB with ckpt_every = 10); larger
 *           problems fail with ENOMEM before anything is enqueued.  The
 *           context's hbm_budget_bytes does not apply (nothing is allocated).
 *   sharing: every call on one GPU, from any context, uses that GPU's one
 *           array; nothing in it needs to start at zero, and each call
 *           writes every part it reads.  Calls whose work overlaps on one GPU
 *           (two streams, two threads, two contexts) race and give undefined
 *           results: serialise them.
 * Errors: EINVAL (as lddmm_shoot_grad; ctx must not be NULL), ENOMEM (limit),
 * EDEVICE. */
lddmm_status lddmm_shoot_grad_noalloc(lddmm_ctx* ctx, const lddmm_params* params,
                                      const double* q0, const double* p0, const double* target,
                                      double* out3, double* grad, double* q1, void* stream);

/* Options of lddmm_solve (L-BFGS over p0 with a strong-Wolfe line search;
 * Nocedal & Wright, Numerical Optimization, Algs. 3.5, 3.6 and 7.4). */
typedef struct {
  int32_t max_iter;        /* accepted steps (the paper's I), >= 0 */
  int32_t m;               /* curvature pairs kept, 1..16 */
  int32_t max_fev;         /* evaluations per line search, >= 1 */
  double gtol;             /* converged when |g| <= gtol max(1, |p0|) */
  double ftol_rel;         /* converged when the relative decrease of L is below
                              this (0 disables the test) */
  double c1, c2;           /* Wolfe constants, 0 < c1 < c2 < 1 */
  int32_t init;            /* start: 0 p0 = 0; 1 p0 = (target - q0)/T (Alg. 1);
                              2 the caller's p0 */
} lddmm_solve_opts;

typedef struct {
  double loss;             /* L at the returned p0 */
  double H0;               /* H(q0, p0) */
  double mismatch;         /* sum_i |q_i(1) - x_i|^2 */
  double grad_norm;        /* |dL/dp0| at the returned p0 */
  double avg_dist;         /* mean_i |q_i(1) - x_i| (Sec. 3.1 AverageDist) */
  double max_dist;         /* max_i |q_i(1) - x_i|  (Sec. 3.1 MaxDist) */
  int32_t iters;           /* accepted L-BFGS steps */
  int32_t fevals;          /* loss+gradient evaluations, line-search trials included */
  int32_t status;          /* lddmm_status of the solve */
} lddmm_solve_result;

/* Default options: max_iter 100, m 5, max_fev 20, gtol 1e-8 for FP64 pair
 * sums and 1e-6 for FP32, ftol_rel 0, c1 1e-4, c2 0.9, init 0.
 * Errors: EINVAL. */
lddmm_status lddmm_solve_opts_default(int32_t precision, lddmm_solve_opts* opts);

/* Registration by geodesic shooting (Alg. 1): minimises the loss of eq. 3
 * over p0 with L-BFGS that runs on the GPU (every loss+gradient evaluation,
 * line-search decision and two-loop recursion is device work; the host only
 * launches evaluations and polls a completion flag).  Blocks until done.
 *   q0, target : in,  [n][3] device FP64
 *   p0_inout   : in (opts->init == 2) / out, [n][3] device FP64, the solution
 *   result     : out, host struct, may be NULL
 *   trace      : out, host array of 2 (opts->max_iter + 1) doubles, may be
 *                NULL: (L, |g|) at the start and after each accepted step
 * Returns LDDMM_OK (converged), LDDMM_ENOTCONV (iteration cap or failed
 * line search; p0 is the last accepted iterate), LDDMM_ENONFINITE, or an
 * error (EINVAL, ENOMEM, EDEVICE). */
lddmm_status lddmm_solve(lddmm_ctx* ctx, const lddmm_params* params, const lddmm_solve_opts* opts,
                         const double* q0, const double* target, double* p0_inout,
                         lddmm_solve_result* result, double* trace, void* stream);

/* ---- Serving: continuous batching of registrations ----------------------
 * A server owns one GPU stream, a preallocated HBM arena and a worker
 * thread.  Submitted registrations (host inputs, copied at submit) are
 * admitted first come first served whenever a slot is free and the job's
 * device footprint (lddmm_server_job_footprint) fits the arena; every running
 * job keeps its trajectory, adjoint and L-BFGS state on the device.  Each
 * round advances all running jobs by one loss+gradient evaluation and one
 * optimiser step through batched pair-sum launches replayed from a captured
 * hipGraph; jobs join at the next round after admission and leave when their
 * optimiser finishes.  A job's result does not depend on the other jobs in
 * the batch (same decomposition, same summation order).  All jobs of a
 * server share T, the precision and the integrator; each job may be planar
 * (lddmm_params.dim = 2) or 3D, and takes the energy term at t = 0. */
typedef struct lddmm_server lddmm_server;

typedef struct {
  int32_t device;
  int32_t max_slots;          /* jobs on the GPU at once, 1..1024 */
  int32_t max_n;              /* largest n accepted, 1..2^20 */
  int32_t T;                  /* time steps of every job, 1..2^20 */
  int32_t precision;          /* lddmm_precision of every job */
  size_t hbm_budget_bytes;    /* arena for job state, allocated at create */
  int32_t integrator;         /* lddmm_integrator of every job (0: Euler steps) */
} lddmm_server_config;

typedef struct {
  double submit_s, admit_s, done_s;   /* seconds on the server's steady clock */
} lddmm_job_times;

typedef struct {
  int64_t queued, running, completed;
  int64_t rounds;             /* batched rounds launched */
  int64_t job_evaluations;    /* loss+gradient evaluations summed over jobs */
  size_t hbm_used_bytes, hbm_budget_bytes;
} lddmm_server_stats;

/* Errors: EINVAL, ENOMEM (arena), EDEVICE. */
lddmm_status lddmm_server_create(const lddmm_server_config* cfg, lddmm_server** out);

/* Device bytes one job of n landmarks and m curvature pairs occupies. */
lddmm_status lddmm_server_job_footprint(const lddmm_server_config* cfg, int32_t n, int32_t m,
                                        size_t* bytes);

/* Queues a registration.  q0, target (and p0 when opts->init == 2) are HOST
 * [n][3] FP64 arrays, copied before the call returns.  params->T and
 * ->precision must equal the server's; ckpt_every is ignored.
 * Errors: EINVAL, ENOMEM (footprint larger than the whole arena), EDEVICE. */
lddmm_status lddmm_server_submit(lddmm_server* srv, const lddmm_params* params,
                                 const lddmm_solve_opts* opts, const double* q0,
                                 const double* target, const double* p0, int64_t* job_id);

/* Result of a job: LDDMM_EBUSY while it is queued or running; once done, the
 * solve status (OK, ENOTCONV, ENONFINITE) with p0_out ([n][3] host, may be
 * NULL), result and times filled, after which the id is released.
 * EINVAL for an unknown id, EDEVICE if the server failed. */
lddmm_status lddmm_server_poll(lddmm_server* srv, int64_t job_id, double* p0_out,
                               lddmm_solve_result* result, lddmm_job_times* times);

/* Blocks until the job can be polled (timeout_s < 0: no limit); EBUSY on
 * timeout, EINVAL for an unknown id. */
lddmm_status lddmm_server_wait(lddmm_server* srv, int64_t job_id, double timeout_s);

lddmm_status lddmm_server_stats_get(lddmm_server* srv, lddmm_server_stats* out);

/* Detail of the server's last error. */
const char* lddmm_server_last_error(lddmm_server* srv);

/* Stops the worker after its current round, drops queued and unfinished
 * jobs and frees everything.  NULL is accepted. */
lddmm_status lddmm_server_destroy(lddmm_server* srv);

/* Loss and all its gradients: as lddmm_shoot_grad, plus (each optional)
 *   grad_q0 : out, [n][3] device FP64, dL/dq0 = a(0) + Hq(q0,p0): the adjoint
 *             of q at t = 0 plus the energy term's own dependence on q0
 *   grad_x  : out, [n][3] device FP64, dL/dx = -2 lambda (q(1) - x)
 * (eq. 3 differentiated through the discrete flow; with them the template
 * and the target can be optimised too).  Errors: EINVAL, ENOMEM, EDEVICE. */
lddmm_status lddmm_shoot_grad_all(lddmm_ctx* ctx, const lddmm_params* params, const double* q0,
                                  const double* p0, const double* target, double* out3,
                                  double* grad_p0, double* grad_q0, double* grad_x, double* q1,
                                  void* stream);

/* Velocity field of the landmark motion at arbitrary points (eq. 4, with the
 * Hamiltonian's Gaussian): v(x_i) = sum_l exp(-|q_l - x_i|^2 / (2 sigma^2)) p_l.
 *   params : n, sigma and precision are used (T and ckpt_every are ignored;
 *            lambda must still be valid)
 *   q, p   : in, [n][3] device FP64, one landmark state (q(t), p(t))
 *   m      : number of points, 0..2^30 (0: nothing is launched)
 *   x      : in, [m][3] device FP64 points
 *   v      : out, [m][3] device FP64 velocities
 * The pair sums run in the precision mode, as in the forward step; a
 * point's result does not depend on m.  Errors: EINVAL, ENOMEM, EDEVICE. */
lddmm_status lddmm_velocity(lddmm_ctx* ctx, const lddmm_params* params, const double* q,
                            const double* p, int32_t m, const double* x, double* v,
                            void* stream);

/* The deformation applied to arbitrary points: shoots the landmarks from
 * (q0, p0) as lddmm_shoot_forward does and carries m points along, each
 * Euler step moving a point by dt v(x, t) (eq. 4) with the landmark state of
 * the same step t, so that a point placed on a landmark follows it.
 *   q0, p0 : in, [n][3] device FP64
 *   m      : number of points, 0..2^30
 *   x0     : in, [m][3] device FP64 points at t = 0
 *   x1     : out, [m][3] device FP64 points at t = 1 (may be the same buffer
 *            as x0)
 *   q1, p1 : out, optional, [n][3] device FP64 landmark state at t = 1
 * With ckpt_every = s in (0, T) only s + 1 trajectory slots are kept and the
 * points advance segment by segment (workspace + 24 m bytes); results are
 * bitwise the same as with the whole trajectory.  A point's result does not
 * depend on m or on the other points.  Errors: EINVAL, ENOMEM, EDEVICE. */
lddmm_status lddmm_flow(lddmm_ctx* ctx, const lddmm_params* params, const double* q0,
                        const double* p0, int32_t m, const double* x0, double* x1, double* q1,
                        double* p1, void* stream);

/* Waits for the context's work on `stream` and reports whether any call
 * since the last check produced a non-finite loss (then ENONFINITE, and the
 * flag is cleared).  Errors: EINVAL, EDEVICE. */
lddmm_status lddmm_ctx_check(lddmm_ctx* ctx, void* stream);

/* Per-kernel timing, for benchmarks.  While enabled, every launch of the
 * forward and of the adjoint pair-sum kernel and of the point-flow kernel
 * carries two HIP events of the call's stream (the stream the kernel runs
 * on), tied by hipExtLaunchKernel to the start and the end of the kernel's
 * execution; durations accumulate until read.  The results are the same as
 * with timing off.  Off by default.  Errors: EINVAL. */
typedef struct {
  double fwd_ms;           /* summed duration of forward pair-kernel launches */
  double adj_ms;           /* summed duration of adjoint pair-kernel launches */
  int64_t fwd_launches;
  int64_t adj_launches;
  double flow_ms;          /* summed duration of point-flow / velocity kernel launches */
  int64_t flow_launches;
} lddmm_timing;

lddmm_status lddmm_ctx_set_timing(lddmm_ctx* ctx, int enable);

/* Waits for the recorded launches to finish and returns their totals since
 * the last reset; reset != 0 starts a new accumulation.  Errors: EINVAL,
 * EDEVICE. */
lddmm_status lddmm_ctx_timing(lddmm_ctx* ctx, lddmm_timing* out, int reset);

/* Static description of a status code; never NULL. */
const char* lddmm_status_string(lddmm_status status);

/* Detail of the last error reported by a call on ctx (empty string if none;
 * calls on one context are serialised by the caller, so this is the error
 * of the latest such call that failed).  With ctx == NULL: the detail of the
 * last error this thread got from a call made without a usable context.
 * The string stays valid until the next failing call on the same context
 * (or, for ctx == NULL, in the same thread). */
const char* lddmm_last_error(lddmm_ctx* ctx);

/* Library version, "major.minor.patch". */
const char* lddmm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LDDMM_H */
