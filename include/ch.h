/*
 * ch.h -- C ABI of the MI355X (gfx950) Parareal library for the Cahn-Hilliard
 * equation  u_t + eps^2 Lap^2 u = Lap f(u),  f(u) = u^3 - u,  u = Lap u = 0 on
 * the boundary of (0,1)^d  (paper: Section 1, equation (1.1)).
 *
 * The library advances many independent instances ("problems") of the
 * equation, each split into N time slices of length dT = T/N (Section 2).
 * All device memory is owned by the caller: the library never allocates
 * device memory; it asks for a workspace size and works inside the buffer it
 * is given.  Every call is asynchronous on the given HIP stream.  The only HIP
 * objects the library creates are side streams (default priority) and
 * events, with which the one-workgroup-per-instance coarse sweeps of several
 * grid-size classes run side by side; they are forked from and joined back
 * to the given stream, so the caller sees stream order, also under stream
 * capture.  Launches whose workgroups wait for each other (group launches)
 * never run beside other launches of the same call.
 *
 * Data layout (all float64, row-major, interior points only, y slowest):
 *   one state           : n^d values, index iy*n + ix;
 *   "slice layout"      : for instance i, N_i states (the inputs of its N_i
 *                         slices), instances packed in creation order;
 *                         ch_layout() reports the offsets;
 *   "iterate layout"    : for instance i, N_i + 1 states U_0..U_N.
 *
 * Errors: every entry returns a ch_status; argument problems are detected
 * on the host before any launch; a HIP error reports CH_ERR_HIP; the text of
 * the last error is available from ch_last_error().  No entry point throws.
 * A context is not thread-safe; distinct contexts are independent.
 */
#ifndef CH_H
#define CH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ch_status {
  CH_OK = 0,
  CH_ERR_ARG = 1,          /* invalid argument or layout                      */
  CH_ERR_HIP = 2,          /* a HIP runtime call or kernel launch failed       */
  CH_ERR_UNSUPPORTED = 3,  /* valid problem the kernels do not cover (n, dim) */
  CH_ERR_NOCONV = 4,       /* Newton or Krylov iteration cap, or non-finite   */
  CH_ERR_STATE = 5,        /* call order violated (e.g. workspace not bound)  */
  CH_ERR_TIMEOUT = 6       /* a workgroup of a group launch waited past its
                              limit for the others (device oversubscribed):
                              the states that launch wrote are invalid       */
} ch_status;

/* fine propagator (Section 2.1): the linear stabilised step (scheme (2.5)
 * for s = 2; PA-II, PA-III), the implicit step solved by Newton's method
 * (scheme (2.3), or backward Euler; NPA-I, NPA-II), or scheme (2.4) with
 * tau = dt (PA-I: a variable-coefficient linear solve every fine step), the
 * latter also solved by the Neumann-Neumann domain decomposition of
 * Section 4 (1D; subdomain count, relaxation and stop in ch_problem) */
enum { CH_FINE_LINEAR = 0, CH_FINE_NONLINEAR = 1, CH_FINE_APPROX2 = 2, CH_FINE_APPROX2_DD = 3 };
enum { CH_NL_EYRE = 0, CH_NL_FULL_BE = 1 };
/* coarse propagator: scheme (2.4) (default; PA-I, PA-III, NPA-I), the
 * stabilised step (PA-II), the learned surrogate (weights bound with
 * ch_nn_bind), or scheme (2.3) solved by Newton's method (NPA-II; 2D, the
 * Newton parameters of the problem, one workgroup per instance) */
enum { CH_COARSE_APPROX2 = 0, CH_COARSE_STAB = 1, CH_COARSE_NEURAL = 2, CH_COARSE_EYRE = 3 };
/* arithmetic of the sine transforms of the linear fine step */
enum { CH_PREC_FP64 = 0, CH_PREC_SPLIT_BF16 = 1 };

typedef struct ch_problem {
  int32_t dim;          /* 1 or 2                                              */
  int32_t n;            /* interior points per dimension, h = 1/(n+1)          */
  double eps;           /* interface width                                     */
  double T;             /* final time                                          */
  int32_t n_slices;     /* Parareal slices N (dT = T/N)                        */
  int32_t j_fine;       /* fine steps per slice J (dt = dT/J), Section 2       */
  int32_t m_coarse;     /* coarse sub-steps per slice (paper: 1)               */
  double s_fine;        /* stabilisation constant s of the linear step (2.0)   */
  int32_t fine_kind;    /* CH_FINE_*                                           */
  int32_t nl_variant;   /* CH_NL_*                                             */
  int32_t coarse_kind;  /* CH_COARSE_*                                         */
  int32_t precision;    /* CH_PREC_*                                           */
  double newton_tol;    /* Newton stop: ||Y_{m+1}-Y_m||_h <= tol (1e-10)       */
  int32_t newton_max;   /* Newton iteration cap (20)                           */
  double krylov_rtol;   /* relative residual target of the CG solves of (2.4)
                           (coarse step, and the PA-I fine step) in 2D; 0 =
                           default: 1e-12 with the linear fine step, 1e-13
                           otherwise.  In 1D the (2.4) steps are solved
                           directly (block-tridiagonal elimination)            */
  int32_t krylov_max;   /* CG iteration cap                                    */
  int32_t f_zero;       /* test hook: f(u) == 0                                */
  double nl_krylov_rtol;/* relative residual target of the CG inside Newton    */
  int32_t nn_base;      /* learned coarse propagator: 0 = clip(u + net(u)); 1 =
                           clip(G_plain(u) + net(u)), the network learns the
                           plain propagator's defect F - G_plain                 */
  /* CH_FINE_APPROX2_DD (1D only): each fine step (2.4) solved by the
   * Neumann-Neumann iteration of Section 4 on equal subdomains; 0 picks the
   * default in brackets                                                      */
  int32_t dd_subdomains;/* N0, with (n + 1) divisible by N0 and (n+1)/N0 >= 2 (8) */
  double dd_theta;      /* relaxation theta of the trace update, 0 < theta < 1 (1/4) */
  double dd_tol;        /* stop: every interface trace (u and v) changed by at
                           most dd_tol in the last iteration (1e-10)            */
  int32_t dd_max;       /* iteration cap per step; reaching it is status bit 1
                           (100)                                                */
} ch_problem;

typedef struct ch_ctx ch_ctx;
typedef void* ch_stream; /* a hipStream_t (NULL = default stream) */

/* Iterate state of ch_parareal_iterate; every pointer is device memory owned
 * by the caller, sized from ch_layout().  U_0 of each instance holds u0. */
typedef struct ch_pr_state {
  double* U;          /* iterate layout: U_n^k, n = 0..N_i                      */
  double* F;          /* slice layout: F(U_n^k) of the latest fine sweep        */
  double* G_old;      /* slice layout: G(U_n^k) kept for the correction         */
  double* delta;      /* [n_inst]: update norm max_n ||U_n^{k+1}-U_n^k||_h      */
  int32_t* status;    /* [n_inst]: flags of every call since the prediction
                         (cleared there): bit 1 = Newton/Krylov cap hit,
                         bit 2 = non-finite update norm, bit 4 = a group wait
                         timed out (states invalid); ch_check_status reads it */
  int32_t k;          /* host: corrections done so far                          */
  int32_t predicted;  /* host: 1 once the coarse prediction U^0 has been formed */
} ch_pr_state;

/* Validate the problems and plan the device work.  Host-only. */
ch_status ch_create(const ch_problem* probs, int32_t n_inst, ch_ctx** out);
ch_status ch_destroy(ch_ctx* ctx);

/* Bytes of device workspace the context needs (tables and solver scratch). */
ch_status ch_workspace_size(const ch_ctx* ctx, size_t* bytes);
/* Hand the context its workspace (256-byte aligned device pointer) and upload
 * its tables on `stream`.  Must precede every compute call. */
ch_status ch_bind_workspace(ch_ctx* ctx, void* dptr, size_t bytes, ch_stream stream);

/* Element counts of the slice layout and the iterate layout, and the offsets
 * of instance `inst` in both (in float64 elements). */
ch_status ch_layout(const ch_ctx* ctx, int32_t inst, int64_t* slice_total, int64_t* iter_total,
                    int64_t* slice_off, int64_t* iter_off);

/* F(T_{n+1}, T_n, U_n) for every slice whose mask byte is non-zero (all if
 * mask is NULL): J fine steps of dt = dT/J (Section 2).  U_in and F_out use
 * the slice layout and must not overlap; mask is device memory, one byte per
 * slice in slice-layout order. */
ch_status ch_fine_propagate(ch_ctx* ctx, const double* U_in, double* F_out,
                            const uint8_t* slice_mask, ch_stream stream);

/* G(T_{n+1}, T_n, U_n), independently for every masked slice (same layout
 * and rules as ch_fine_propagate). */
ch_status ch_coarse_propagate(ch_ctx* ctx, const double* U_in, double* G_out,
                              const uint8_t* slice_mask, ch_stream stream);

/* One step of the Parareal iteration (2.2) for every instance.
 * First call (st->predicted == 0): the coarse prediction U_{n+1}^0 = G(U_n^0),
 * G_old_n = U_{n+1}^0.  Later calls: the fine sweep F_n = F(U_n^k) over the
 * slices n >= k (earlier ones are final, finite termination), then the
 * sequential correction U_{n+1}^{k+1} = F_n + (G(U_n^{k+1}) - G_old_n) and
 * the update norm into st->delta.  Instances whose previous delta was below
 * tol are left unchanged.  No host synchronisation inside. */
ch_status ch_parareal_iterate(ch_ctx* ctx, ch_pr_state* st, double tol, ch_stream stream);

/* The second half of ch_parareal_iterate alone (after the prediction): with
 * st->F already holding F(U_n^k) for n >= k, run the sequential coarse sweep
 * and correction of (2.2) and the update norm, and advance st->k.  For a
 * single instance the slice inputs U_0..U_{N-1} are the first N states of
 * the iterate layout, so ch_fine_propagate(st->U, st->F) followed by this
 * call equals one ch_parareal_iterate. */
ch_status ch_parareal_correct(ch_ctx* ctx, ch_pr_state* st, double tol, ch_stream stream);

/* out[i] = ||A_i - B_i||_h (h^d-weighted L2 norm, the norm of the update norm,
 * Section 4) for every slice i of the slice layout, in slice order over all
 * instances (out holds the total slice count).  A, B and out are device
 * memory; A and B use the slice layout.  Used to judge a coarse propagator's
 * error against F slice by slice (the learned propagator's Parareal loop). */
ch_status ch_slice_distance(ch_ctx* ctx, const double* A, const double* B, double* out,
                            ch_stream stream);

/* Up to max_iters steps of the Parareal iteration (2.2) in one launch, each
 * equal to one ch_parareal_iterate call: iteration k sweeps the slices n >= k
 * (finite termination) and the run stops after the first iteration whose
 * update norm is below tol (the rule that ends an instance's iterations in
 * ch_parareal_iterate), or once k reaches N.  Same states,
 * update norms and G_old as that many ch_parareal_iterate calls, bit for bit;
 * only the schedule differs: the fine solve of slice n for iteration k + 1
 * starts as soon as the coarse sweep of iteration k has corrected slice n - 1,
 * so fine solves and coarse sweeps of consecutive iterations overlap (one
 * group of workgroups runs the sweeps, the others the fine solves; they hand
 * states over through device memory).
 * flags: CH_RUN_SWEEP_ALL sweeps every slice from the current k in every
 * iteration (nothing skipped as final: the same iterates, equal work per
 * iteration, used for timing).
 * If the coarse prediction has not been formed, it is formed first (not
 * counted).  The device iteration counter advances by the iterations done;
 * st->k is not updated (ch_iteration_count reads it).  st->F is used as a
 * buffer for the fine results of even iterations; its contents afterwards are
 * unspecified.  No host synchronisation inside.
 * Covers a context of one instance, 2D n = 128, linear FP64 fine step, coarse
 * scheme (2.4), N >= 2; CH_ERR_UNSUPPORTED otherwise, and when the device
 * cannot hold all workgroups of the launch at once (the launch needs one
 * group of eight workgroups per slice, up to 64 groups at two per CU).  The
 * groups wait for each other at device-memory counters, each wait bounded by
 * a limit (ch_set_wait_limit, 10 s by default); a failure sets status bit 4
 * (ch_check_status: CH_ERR_TIMEOUT) and the states of that call are
 * invalid. */
#define CH_RUN_SWEEP_ALL 1
ch_status ch_parareal_run(ch_ctx* ctx, ch_pr_state* st, double tol, int32_t max_iters,
                          int32_t flags, ch_stream stream);

/* Autotuner of the FP64 linear fine sweep (2D): for each grid-size class it
 * times every launch configuration over `steps` fine steps of all slices of
 * the class on the given inputs (slice layout; F_out is overwritten) and
 * keeps the fastest: one workgroup per slice with each wave count
 * (ch_fine_variant), and groups of workgroups per slice with each group size
 * the class has (ch_fine_groups: 4 or 8 at n = 128, 8 at n = 256).
 * Synchronous. */
ch_status ch_autotune(ch_ctx* ctx, const double* U_in, double* F_out, int32_t steps,
                      ch_stream stream);
/* Query (set = 0) or set (set = 1) the waves per workgroup of the fine
 * kernel for grid size n (e.g. from a cached tuning result). */
ch_status ch_fine_variant(ch_ctx* ctx, int32_t n, int32_t* waves, int32_t set);

/* Query (set = 0) or set (set = 1) how many workgroups run each slice of the
 * FP64 fine sweep for the 2D class of grid size n and fine step fine_kind
 * (CH_FINE_LINEAR or CH_FINE_NONLINEAR):
 * 1, or a group that splits the sine transforms of every step and meets at
 * device-memory barriers.  Linear step (2.5), with the Laplacian applied in
 * the sine basis where it is diagonal: 4 or 8 at n = 128, 8 at n = 256.
 * Implicit steps (Newton, the Krylov solves on the group): 8 at n = 128, 16
 * at n = 256.  The group kernels are persistent over the slices.  Defaults:
 * linear 8 at n = 128 with at most 64 slices in the class, 8 at n = 256;
 * implicit 8 at n = 128 with at most 32 slices, 16 at n = 256; else 1.  A
 * device that cannot hold a group falls back to 1.  All give the same states
 * to rounding.  CH_ERR_UNSUPPORTED for a group size without a kernel.
 * The members of a group wait for each other at device-memory barriers, so
 * the group kernels need every workgroup resident at once: the launch checks
 * the device's capacity, but kernels of other streams that hold CUs at the
 * same time can delay members.  A member that waits longer than the limit
 * (ch_set_wait_limit, 0.2 s by default) gives up.  The instance's status
 * word then gets bit 4 (ch_check_status reports CH_ERR_TIMEOUT), and the
 * states of that launch are invalid. */
ch_status ch_fine_groups(ch_ctx* ctx, int32_t n, int32_t fine_kind, int32_t* groups, int32_t set);

/* Query (set = 0) or set (set = 1) how many workgroups run each instance's
 * sequential coarse sweep of (2.2) for the 2D grid-size class n: 1 (one
 * workgroup per instance), 4 or 8 (the 2D sine transforms of every solve of
 * (2.4) split over that many workgroups that meet at device-memory barriers;
 * n = 128, at most 256 workgroups in all, i.e. 64 instances with 4 or 32
 * with 8; the default is 8 up to 32 instances and 4 up to 64, and a device
 * that cannot hold all workgroups at once falls back to 1).  All give the same iterates to rounding.  Instances with the
 * stabilised coarse step always use one workgroup.  Residency and time-out
 * as for ch_fine_groups (status bit 4). */
ch_status ch_chain_variant(ch_ctx* ctx, int32_t n, int32_t* groups, int32_t set);

/* hipGraph of one Parareal iteration (after the prediction): captured on
 * the non-default `stream`, replayable with ch_graph_launch; each replay
 * performs the next iteration (the iteration index, the judge of a learned
 * propagator and its fallback live in device memory).  After replays,
 * ch_iteration_count refreshes st->k from the device.  The caller owns the
 * handle. */
ch_status ch_parareal_graph_create(ch_ctx* ctx, ch_pr_state* st, double tol, ch_stream stream,
                                   void** graph_exec);
ch_status ch_graph_launch(void* graph_exec, ch_stream stream);
ch_status ch_graph_destroy(void* graph_exec);
/* Synchronous: copy the device iteration counter into st->k. */
ch_status ch_iteration_count(ch_ctx* ctx, ch_pr_state* st, ch_stream stream);
/* Set the iteration counter (device and st->k), e.g. to repeat an iteration. */
ch_status ch_set_iteration(ch_ctx* ctx, ch_pr_state* st, int32_t k, ch_stream stream);

/* Synchronous check of the flags the device raised.  Reads, for every
 * instance, the flags of the latest call that launched fine or coarse kernels
 * (ch_fine_propagate, ch_coarse_propagate, ch_parareal_iterate,
 * ch_parareal_run; ch_parareal_correct adds to those of the preceding call)
 * and, when st is given, st->status (the whole run).  bits (host memory,
 * n_inst values, may be NULL) receives their OR per instance.  Returns
 * CH_ERR_TIMEOUT if any bit 4 is set, else CH_ERR_NOCONV if any bit 1 or 2
 * is set (cap reached or non-finite), else CH_OK; ch_last_error names the
 * first instance.  Compute calls never synchronise, so this is how a caller
 * learns of device-side failures. */
ch_status ch_check_status(ch_ctx* ctx, const ch_pr_state* st, int32_t* bits, ch_stream stream);

/* Bounds of the inter-workgroup waits of this context's group kernels: a
 * group barrier gives up after group_seconds (default 0.2) and a hand-off of
 * the pipelined launch after pipe_seconds (default 10); both in [0, 60].  A
 * wait that gives up sets status bit 4 and lets its kernel run to its end, so
 * a limit of 0 forces the failure path (for tests of error reporting).
 * Synchronous. */
ch_status ch_set_wait_limit(ch_ctx* ctx, double group_seconds, double pipe_seconds,
                            ch_stream stream);

/* Constants of the convergence theorems for the linear pairings (Section 3,
 * Theorems 3.7, 3.9, 3.11): with diag(u^2) ~ I the fine and coarse steps
 * become P_i = (I - i tau D_h + eps^2 tau D_h^2)^{-1} (I - i tau D_h), i = 1
 * for scheme (2.4) and i = 2 for (2.5); alpha = ||P_{J,i_fine} - P_{i_coarse}||,
 * beta = ||P_{i_coarse}|| (2-norms), where the fine operator is J steps of
 * dT/J and the coarse one m_coarse steps of dT/m_coarse.  The Parareal error
 * then obeys max_n ||E_n^k|| <= alpha^k min{((1 - beta^{N-1})/(1 - beta))^k,
 * binom(N-1, k)} max_n ||E_n^0||.  Host-only; dim 1 or 2, n interior points
 * per dimension. */
ch_status ch_linear_bound(int32_t dim, int32_t n, double eps, double dT, int32_t J,
                          int32_t m_coarse, double i_fine, double i_coarse, double* alpha,
                          double* beta);

/* Discrete energy (Section 1, (1.2)) of `count` states of instance `inst`:
 * E_h = h^d sum (u^2-1)^2/4 + (eps^2/2) h^d sum u (-Lap_h u).  E_out is
 * device memory of `count` doubles. */
ch_status ch_energy(ch_ctx* ctx, int32_t inst, const double* u, int32_t count, double* E_out,
                    ch_stream stream);

/* ------------------------------------------------------------------------
 * Learned coarse propagator (G_nn(u) = u + net(u)): a 4-level convolutional
 * encoder-decoder with BF16 weights and FP32 accumulation on n x n grids
 * (n divisible by 8).  Parameter vector: for each layer, W[c_out][c_in][k][k]
 * then b[c_out]; ch_nn_layer describes the layers.  Activation workspaces
 * are caller device memory of ch_nn_workspace_bytes(batch, n) bytes.  These
 * calls need no context.  States u/out/target are float64 (batch, n, n).
 * ---------------------------------------------------------------------- */
int64_t ch_nn_param_count(void);
ch_status ch_nn_layer(int32_t layer, int32_t* c_in, int32_t* c_out, int32_t* k, int32_t* stride,
                      int32_t* act, int32_t* cat);
size_t ch_nn_workspace_bytes(int32_t batch, int32_t n);
/* out = clip(u + net(u), -1.5, 1.5) (the clip bounds repeated application on
 * states far from the training data; ch_nn_train_step uses the unclipped
 * output) */
ch_status ch_nn_forward(const uint16_t* w_bf16, const double* u, int32_t batch, int32_t n,
                        void* ws, double* out, ch_stream stream);
/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): the same forward pass as
 * ch_nn_forward, same kernels and results, with no workspace argument.  The
 * activations and the weights copied into the forward pass's layout (0.25 Mi
 * floats) live in a static device array of 32 MiB (8 Mi floats) that each
 * GPU the library runs on holds until the process ends; the call allocates
 * nothing.  Limit: batch * (activation floats per sample) + 0.25 Mi <= 8 Mi,
 * i.e. batch <= 5 at n = 128, 1 at n = 256, 22 at n = 64; larger requests
 * return CH_ERR_ARG (with a message on stderr) before any launch.  Every
 * call on one GPU shares that array, which keeps the last call's contents
 * (nothing in it needs clearing: each value is written before it is read),
 * so calls that overlap on one GPU (different streams, or threads) race and
 * must be serialised by the caller. */
ch_status ch_nn_forward_static(const uint16_t* w_bf16, const double* u, int32_t batch, int32_t n,
                               double* out, ch_stream stream);
/* forward, loss = mean((u + net(u) - target)^2) (device float), gradient of
 * the loss w.r.t. every parameter into grad (float32, overwritten);
 * batch * n * n <= 2^20 */
ch_status ch_nn_train_step(const uint16_t* w_bf16, const double* u, const double* target,
                           int32_t batch, int32_t n, void* ws, float* grad, float* loss,
                           ch_stream stream);
/* Adam on the FP32 master weights (bias-corrected, step >= 1), then the BF16
 * copy rounded to nearest even */
ch_status ch_nn_adam(float* w_master, uint16_t* w_bf16, float* m, float* v, const float* grad,
                     int64_t count, float lr, float beta1, float beta2, float eps, int32_t step,
                     ch_stream stream);
ch_status ch_nn_to_bf16(const float* w_master, uint16_t* w_bf16, int64_t count, ch_stream stream);
/* weights used by instances whose coarse kind is CH_COARSE_NEURAL */
ch_status ch_nn_bind(ch_ctx* ctx, const uint16_t* w_bf16);
/* switch the coarse propagator of one instance; the context must have been
 * created with a learned-propagator instance to switch one to it.  (The
 * fallback of a Parareal run needs no call: see ch_judge_read.) */
ch_status ch_set_coarse_kind(ch_ctx* ctx, int32_t inst, int32_t kind, ch_stream stream);

/* The plain coarse propagator (2.4) is the learned one's fallback and judge,
 * inside ch_parareal_iterate (and its graph), on the device.  Before each
 * correction of an instance still on the learned propagator it computes
 * G_plain(U_n^k) for every slice and the ratio r^k = mean over the slices
 * n >= k with ||G_plain(U_n^k) - F_n||_h > 0 of ||G(U_n^k) - F_n||_h /
 * ||G_plain(U_n^k) - F_n||_h (G(U_n^k) = G_old_n).  After the correction the
 * instance falls back to the plain propagator for the rest of the run when
 * the update norm is not finite, or not smaller than the previous one, or r
 * exceeded 1 in this and the previous iteration (unless the norm is already
 * below tol); G_old is then recomputed with the plain propagator at the new
 * iterate.  A new run (the prediction) starts on the learned propagator
 * again.  This call reads, synchronously, instance inst's ratios (ratios:
 * host memory of N doubles, NaN for iterations not judged; may be NULL),
 * the number of corrections done when it fell back (-1: it has not), and
 * whether it still uses the learned propagator.  CH_ERR_ARG for an
 * instance created with another coarse propagator. */
ch_status ch_judge_read(ch_ctx* ctx, int32_t inst, double* ratios, int32_t* fallback_at,
                        int32_t* learned_now, ch_stream stream);

/* Neumann-Neumann fine step (Section 4): the number of iterations the J
 * steps of each slice of instance inst took in the latest fine sweep that
 * processed that slice (slices a sweep skipped keep their earlier count; 0
 * before any).  iters: host memory of N int32, written synchronously after
 * `stream` drains.  CH_ERR_ARG for an instance of another fine kind. */
ch_status ch_dd_iterations(ch_ctx* ctx, int32_t inst, int32_t* iters, ch_stream stream);

/* Implicit fine step (2.3) or backward Euler solved by Newton's method with
 * spectral CG (Section 3, the Newton iteration of NPA-II), on groups of
 * workgroups: per slice of instance inst, the Newton iterations and the
 * applications of the CG operator (one per CG iteration, plus one to start
 * each solve) that its J steps took in the latest fine sweep that processed
 * it.  They give the sweep's executed matrix-core work: n^3 flops per sine
 * transform stage, four stages per Newton iteration (the state and its cube
 * to physical space and back) and four per operator application, plus four
 * per slice to enter and leave the sine basis.  newton,
 * krylov: host memory of N int32 each, written synchronously after `stream`
 * drains.  CH_ERR_ARG for another fine kind; CH_ERR_UNSUPPORTED when the
 * instance's class runs one workgroup per slice (those kernels do not
 * count). */
ch_status ch_solver_counts(ch_ctx* ctx, int32_t inst, int32_t* newton, int32_t* krylov,
                           ch_stream stream);

const char* ch_status_str(ch_status s);
const char* ch_last_error(const ch_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* CH_H */
