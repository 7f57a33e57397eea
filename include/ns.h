/*
 * ns.h -- C ABI of the MI355X (gfx950) Fourier pseudo-spectral Navier--Stokes
 * time integrator.
 *
 * The library integrates the ODE system that the Fourier pseudo-spectral
 * discretisation turns the incompressible Navier--Stokes equations into
 * (Sec. 2.1, Eq. (2)):  d u_hat / dt = f(u_hat), with
 *
 *   f(u_hat) = N_hat - k (k . N_hat) / |k|^2 - nu |k|^2 u_hat,
 *   N_hat    = dealiased DFT of u x omega evaluated in physical space
 *              (2/3 rule, or the 3/2-rule padding of Sec. 2.1.1),
 *
 * and, in two dimensions, the Boussinesq system of Sec. 3.2, Eqs. (3a-c),
 * (4a-b).  Steppers: classical RK4 with a fixed step and the Bogacki--Shampine
 * 5(4) pair (Appendix A.3, Eq. (8)) with the error estimate and step-size
 * controller of Sec. 2.2.1.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * State layout (device memory, complex128 = two doubles, re then im):
 *   3D: [batch][3][n][n][n/2+1]  index [kz][ky][kx], components (u, v, w)
 *   2D: [batch][c][n][n/2+1]     index [ky][kx],     components (u, v[, rho])
 * i.e. numpy.fft.rfftn of the physical field over its spatial axes divided by
 * n^dim (the normalised transform; physical values are sum_k u_hat e^{ik.x}).
 * Full axes hold wavenumbers 0..n/2-1, -n/2..-1; the last axis 0..n/2.  Only
 * modes with every |k_j| <= K are read; the library writes zeros everywhere
 * else.  K = (n-1)/3 under the 2/3 rule (NS_DEALIAS_23); K = n/2 - 1 under
 * the 3/2 rule (NS_DEALIAS_32), whose products are formed on the zero-padded
 * (3n/2)^dim grid.  The kx = 0 plane must be Hermitian (a real field).
 * Internally the solver keeps only the retained modes.
 *
 * Memory ownership: the caller owns every device buffer (state, f, the
 * workspace); the solver keeps non-owning pointers and never frees caller
 * memory.  The library itself allocates no device memory.  Host pointers are
 * marked "host"; all others are device pointers.
 *
 * Streams: every call is enqueued on the stream given to ns_init (a
 * hipStream_t passed as void*; NULL = the default stream) and is
 * asynchronous, except calls that return values in host memory, which
 * synchronise that stream before returning.
 *
 * Errors: functions return an int status; 0 = NS_OK, 1 = NS_STEP_REJECTED
 * (informational), negative = error.  No C++ exception crosses the ABI.  A
 * failed call leaves the committed state unchanged unless stated otherwise.
 */
#ifndef NS_H
#define NS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NS_OK 0
#define NS_STEP_REJECTED 1
#define NS_ERR_ARG (-1)         /* invalid argument or configuration */
#define NS_ERR_HIP (-2)         /* a HIP runtime call failed */
#define NS_ERR_NOMEM (-3)       /* workspace too small */
#define NS_ERR_NONFINITE (-4)   /* a non-finite value reached a reduction */
#define NS_ERR_STEPFAIL (-5)    /* too many consecutive rejected steps */
#define NS_ERR_UNSUPPORTED (-6) /* size or mode not built */
#define NS_ERR_STATE (-7)       /* call out of order (e.g. no state set) */
#define NS_ERR_SCRATCH (-8)     /* ns_rhs_static: the problem exceeds its static scratch */

#define NS_DEALIAS_23 0         /* 2/3 rule: |k_j| <= (n-1)/3, products on the n grid */
#define NS_DEALIAS_32 1         /* 3/2 rule (Sec. 2.1.1): |k_j| <= n/2-1, products on
                                   the zero-padded 3n/2 grid, truncated back */

#define NS_FP32 0               /* FFTs and nonlinear term in float */
#define NS_FP64 1               /* FFTs and nonlinear term in double */

#define NS_CTRL_PI 0            /* Sec. 2.2.1 controller (optionally PI) */
#define NS_CTRL_MLP 1           /* learned proposer with the PI fallback */

#define NS_FORCE_COMMIT 1       /* ns_step_bs5: commit whatever err is */
#define NS_INTEGRATE_HOST 0x100 /* ns_integrate: launch each attempt's kernels
                                   individually instead of replaying a graph */
#define NS_METHOD_DP5 0x200     /* ns_integrate: the DP5 pair instead of BS5 */
#define NS_INTEGRATE_RESUME 0x400 /* ns_integrate: continue the controller (step,
                                   rejection flag, error history) of the last
                                   ns_integrate or ns_checkpoint_load; h0 is
                                   used only when there is none */

#define NS_MLP_NPARAM 5569      /* W1 64x20, b1 64, W2 64x64, b2 64, W3 1x64, b3 1 */
#define NS_MLP_NWEIGHTS 5609    /* parameters + feature mean [20] + feature scale [20] */

typedef struct ns_config {
  int dim;              /* 3, or 2 */
  int n;                /* points per direction: power of two, 8..1024 (3D at 1024:
                           about 175 GB of workspace with an FP32 right-hand side) */
  int batch;            /* ensemble members B >= 1, stepped together */
  int rhs_precision;    /* NS_FP32 or NS_FP64; state and reductions are always FP64 */
  int scalar;           /* 2D only: 1 = Boussinesq density as third component */
  double ri;            /* Boussinesq buoyancy coefficient (Atwood x gravity) */
  double kappa;         /* Boussinesq scalar diffusivity */
  double force_kf;      /* 3D: forcing band 0 < |k| <= kf after each accepted step; <= 0 off */
  double force_e0;      /* energy the forcing restores */
  int dealias;          /* NS_DEALIAS_23, or NS_DEALIAS_32 (n >= 16; 3D n <= 512) */
} ns_config;

typedef struct ns_solver ns_solver;

/* Per-member counters of ns_integrate. */
typedef struct ns_stats {
  double t;             /* time reached */
  double h_next;        /* step size the controller proposes next */
  double last_err;      /* error estimate of the last attempt */
  long long n_rhs;      /* right-hand-side evaluations, rejected attempts included */
  long long n_accept;
  long long n_reject;
} ns_stats;

/* Bytes of device workspace ns_init needs for cfg (0 if cfg is invalid). */
size_t ns_workspace_bytes(const ns_config* cfg);

/* Create a solver for `batch` independent members of the problem of Sec. 2
 * (the periodic box of Eq. (1), discretised as Eq. (2); in 2D, Sec. 3.2).
 * nu_host[batch]: viscosity (1/Re, Sec. 2) per member.  workspace: device
 * buffer of at least ns_workspace_bytes(cfg) bytes, 256-byte aligned, owned by
 * the caller and kept until ns_free.  stream: hipStream_t or NULL.  On success
 * *out receives the solver; the state is unset until ns_set_state.  Errors:
 * NS_ERR_ARG (invalid cfg, null pointers, workspace too small or misaligned),
 * NS_ERR_HIP. */
int ns_init(const ns_config* cfg, const double* nu_host, void* workspace,
            size_t workspace_bytes, void* stream, ns_solver** out);

/* Copy in / out the state u_hat of Eq. (2) (layout above; the transform of
 * Sec. 2.1).  set_state drops non-retained modes, invalidates the cached first
 * stage f(u_n) and leaves no controller to resume; it does not check that the
 * field is divergence-free (the projection of every right-hand side keeps the
 * divergence-free part's evolution exact).  Device buffers, may be freed after
 * the call returns (the copy is ordered on the solver's stream). */
int ns_set_state(ns_solver* s, const void* uhat);
int ns_get_state(ns_solver* s, void* uhat);

/* Per-member viscosity (host array of batch values). */
int ns_set_nu(ns_solver* s, const double* nu_host);

/* f(u_hat) of Eq. (2) (or Eqs. (4a-b)) for every member: uhat and f in the
 * state layout, may not alias.  Does not touch the solver's state. */
int ns_rhs(ns_solver* s, const void* uhat, void* f);

/* Allocation-free right-hand side, for callers that cannot allocate device
 * memory or create a solver: code under HIP stream capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Computes what ns_rhs computes,
 * f(u_hat) for every member of cfg, with the same pass kernels (default
 * launch variants, one stream), but takes no solver and no workspace: the
 * compact state, f, the transform intermediates, the twiddle table and the
 * viscosities live in one file-scope device array of NS_STATIC_SCRATCH_BYTES
 * that each GPU the library runs on holds until the process ends.
 *   cfg      configuration as for ns_init (forcing fields are ignored), with
 *            batch <= NS_STATIC_MAX_BATCH
 *   nu_host  [batch] viscosities (host memory, read before the call returns)
 *   uhat, f  device buffers in the state layout; may not alias
 *   stream   hipStream_t or NULL; the work is stream-ordered and asynchronous
 * Returns NS_ERR_ARG for an invalid cfg, batch or pointer, NS_ERR_SCRATCH
 * (nothing launched) when the problem's buffers exceed the array, e.g. a 3D
 * grid above 64^3 (the sizes that fit are those ns_rhs_static_bytes accepts),
 * NS_ERR_HIP on a failed launch.  Calls no allocating routine.  Every call on
 * one GPU uses that GPU's array: calls that overlap on one GPU (other streams,
 * other host threads) race and must be serialised by the caller; nothing in
 * the array needs to start at zero (every buffer is written before it is
 * read within the call). */
#define NS_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
#define NS_STATIC_MAX_BATCH 64
int ns_rhs_static(const ns_config* cfg, const double* nu_host, const void* uhat, void* f,
                  void* stream);

/* Bytes of the static array ns_rhs_static would use for cfg (0 if cfg is
 * invalid); the call is accepted iff 0 < bytes <= NS_STATIC_SCRATCH_BYTES. */
size_t ns_rhs_static_bytes(const ns_config* cfg);

/* One classical RK4 step of size h for every member (committed). */
int ns_step_rk4(ns_solver* s, double h);

/* One attempt of the BS5 pair with step h for every member (Sec. 2.2,
 * Sec. 2.2.1).  err_host[batch] (host, may be NULL) receives
 * err = max_j sqrt(mean_k |(u - v)_j / sc_j|^2) with
 * sc = atol + rtol max(|u_n|, |u_{n+1}|).  A member commits iff its err <= 1,
 * or always with flags & NS_FORCE_COMMIT (fixed-step BS5).  Returns
 * NS_STEP_REJECTED if any member did not commit. */
int ns_step_bs5(ns_solver* s, double h, double atol, double rtol, int flags,
                double* err_host);

/* The same with the Dormand--Prince 5(4) pair of Appendix A.1, Eq. (7): seven
 * stages, FSAL (six new right-hand sides per attempt), embedded b_hat of
 * order 4, so the controller's exponent is again 1/5.  Arguments, error norm
 * and commit rule as ns_step_bs5. */
int ns_step_dp5(ns_solver* s, double h, double atol, double rtol, int flags,
                double* err_host);

/* Adaptive BS5 integration of every member from its current time to t_end
 * (Sec. 2.2.1): h0 is the first trial step, the factor
 * 0.8 err^(-1/5) clamped to [0.01, 2] (1 right after a rejection) sets the
 * next step, a step is accepted iff err <= 1, the last step is clipped to land
 * on t_end.  Each member is controlled on the device (own step, time and
 * counters); one attempt -- stages, error norm, decision, commit, forcing --
 * is captured once as a HIP graph and replayed until every member is done.
 * controller: NS_CTRL_PI or NS_CTRL_MLP (needs weights, see
 * ns_mlp_set_weights: after an accepted step the network's proposal exp(y)
 * replaces the Sec. 2.2.1 factor fac, clamped to [0.7 fac, fac]: it can only
 * shorten a step, by at most 30%, so the controller stays the fallback; after
 * a rejection, or if the proposal is not finite, fac is used),
 * optionally or-ed with NS_INTEGRATE_HOST and with NS_METHOD_DP5 (the DP5 pair
 * of ns_step_dp5 instead of BS5).  stats_host[batch] (host, may be NULL)
 * receives the counters.  Returns NS_ERR_STEPFAIL after 50 consecutive
 * rejections of a member (that member keeps its last accepted state). */
int ns_integrate(ns_solver* s, double t_end, double h0, double atol,
                 double rtol, int controller, ns_stats* stats_host);

/* Checkpoint and resume (a long run restarted from a saved time, as the
 * paper's forced-turbulence runs are).  The checkpoint is one host buffer of
 * ns_checkpoint_bytes(s) bytes holding: a header with the configuration, the
 * per-member viscosity and time, the controller's continuation state (next
 * step, rejection flag, consecutive rejections, last three accepted errors),
 * the retained-mode state u_n, the cached first stage f(u_n) when valid
 * (with its FP32 copy, FP32 right-hand side) and the proposer's weights.
 * Not included: the proposer's training rows and optimiser moments, the
 * autotuner's choice.  save: host buffer owned by the caller, written
 * synchronously.  load: into a solver created with the same configuration
 * (dim, n, batch, precision, scalar, dealias; else NS_ERR_ARG) -- a run
 * continued with ns_integrate(..., controller | NS_INTEGRATE_RESUME, ...) is
 * then bitwise equal to the same calls made without the checkpoint.
 * ns_set_state and the single-step calls leave no controller to resume. */
size_t ns_checkpoint_bytes(const ns_solver* s);
int ns_checkpoint_save(ns_solver* s, void* host_buf, size_t bytes);
int ns_checkpoint_load(ns_solver* s, const void* host_buf, size_t bytes);
/* The same in one pair of calls: ns_save with host_blob NULL writes the size
 * a checkpoint needs to *bytes (host); with a buffer of *bytes bytes it saves
 * and sets *bytes to the size written.  ns_load is ns_checkpoint_load. */
int ns_save(ns_solver* s, void* host_blob, size_t* bytes);
int ns_load(ns_solver* s, const void* host_blob, size_t bytes);

/* Time of each member (host array of batch values); set_time resets it. */
int ns_get_time(ns_solver* s, double* t_host);
int ns_set_time(ns_solver* s, const double* t_host);

/* Diagnostics of the current state (Sec. 3.1): kinetic energy
 * E = 1/2 sum w |u_hat|^2, dissipation rate eps = -sum w Re(conj(u_hat).f)
 * and the 16 shell energies (bin b: floor(16 |k| / K) = b, last bin open),
 * w = 1 on the kx = 0 plane and 2 elsewhere.  Host arrays of batch, batch
 * and 16*batch doubles; any may be NULL. */
int ns_diagnostics(ns_solver* s, double* energy_host, double* dissipation_host,
                   double* shells_host);

/* Evaluate f(u_n) into the solver's cached first stage (used by the next BS5
 * attempt and by ns_diagnostics).  Asynchronous. */
int ns_refresh_rhs(ns_solver* s);

/* ---- learned step-size proposer (20-64-64-1 tanh network, FP32) ----
 * Features of an accepted state: log10(E_b / E + 1e-30) of the 16 shell
 * energies, then log10 of the last four accepted error estimates (oldest
 * first, padded with 1.0); normalised by the stored mean and scale.  Output:
 * y = log(h_next / h).  Weights live in the solver's workspace. */
/* Copy the NS_MLP_NWEIGHTS weights in / out.  Host arrays: the weights are a
 * 22 KB vector that callers keep in files and checkpoints, so the host is their
 * natural home; the copy is synchronous and the library keeps its own device
 * copy in the workspace. */
int ns_mlp_set_weights(ns_solver* s, const float* w_host);   /* NS_MLP_NWEIGHTS */
int ns_mlp_get_weights(ns_solver* s, float* w_host);
/* y_dev[n] = network(x_dev[n][20]) for raw (unnormalised) feature rows. */
int ns_mlp_forward(ns_solver* s, const float* x_dev, int n, float* y_dev);
/* Mean-squared-error loss over (x_dev[n][20], t_dev[n]) and its gradient
 * w.r.t. the NS_MLP_NPARAM parameters (host array), 1 <= n <= 1024. */
int ns_mlp_grad(ns_solver* s, const float* x_dev, const float* t_dev, int n,
                float* grad_host, float* loss_host);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on that batch. */
int ns_mlp_train_batch(ns_solver* s, const float* x_dev, const float* t_dev, int n,
                       float lr, float* loss_host);
/* Zero Adam's moments and step count. */
int ns_mlp_reset_optimizer(ns_solver* s);
/* While enabled, ns_integrate records a training row (features after an
 * accepted step, label log(h_next_accepted / h)) for every accepted step that
 * follows an accepted step, into a ring of 65536 rows. */
int ns_mlp_collect(ns_solver* s, int enable);
/* Number of rows recorded (host); copies min(count, capacity, max_rows) rows
 * to x_host[.][20] / y_host[.] when they are not NULL. */
int ns_mlp_rows(ns_solver* s, float* x_host, float* y_host, int max_rows, long long* count_host);
/* Append n rows (host x_host[n][20], y_host[n]) to the ring, e.g. rows
 * recorded by other solvers. */
int ns_mlp_push_rows(ns_solver* s, const float* x_host, const float* y_host, int n);
/* Set the feature mean and scale from the recorded rows. */
int ns_mlp_fit_stats(ns_solver* s);
/* iters Adam steps on minibatches of `batch` recorded rows drawn with
 * splitmix64(seed + iteration * batch + sample); loss_host (may be NULL)
 * receives the last minibatch loss.  The seed is this library's addition to
 * the training call: with it a run's minibatches are reproducible and a test
 * can replay them on the host. */
int ns_mlp_train(ns_solver* s, int iters, int batch, float lr, unsigned long long seed,
                 float* loss_host);

/* Kernel timing with HIP events recorded around kernel launches while
 * profiling is on (a tracing aid; timing-only events without the system-scope
 * cache fence, which still add a few microseconds of packet time per
 * launch).  Index: 0..4 the five right-hand-side passes (z-inverse,
 * y-inverse, x-pass, y-forward, z-forward; in 3D the y/x/y launches are not
 * timed one by one), 5 stage combinations, 6 reductions, 7 other, 8 the
 * whole y/x/y slab phase of a 3D evaluation (wall time on the solver's
 * stream; its launches may overlap on two streams), 9 whole right-hand-side
 * evaluations (mode 2 only).  stop synchronises and fills total milliseconds
 * and launch counts per index. */
#define NS_NPROF 10
typedef struct ns_kernel_times {
  double ms[NS_NPROF];
  long long count[NS_NPROF];
} ns_kernel_times;
int ns_profile_start(ns_solver* s);
int ns_profile_stop(ns_solver* s, ns_kernel_times* out_host);
/* What profiling brackets.  mode 0 (the default): the passes, with the 3D
 * y/x/y phase as one unit (index 8).  1: also each y-inverse, x-pass and
 * y-forward launch, on its own stream (indices 1..3; with the two-stream slab
 * schedule a launch's time then includes what overlaps it on the other
 * stream).  2: only each whole right-hand-side evaluation, first pass start to
 * last pass end (index 9), so that the evaluation runs with two events instead
 * of one pair per pass; combinations and reductions keep their brackets.
 * Other values: NS_ERR_ARG. */
int ns_profile_mode(ns_solver* s, int mode);

/* Autotuner of the right-hand side.  3D: parameters 0-4 are launch variants of
 * the five passes (z-inverse, y-inverse, x-pass, y-forward, z-forward): radix
 * plan (wide = few passes, narrow = fewer values per thread) and column
 * tile (16, 32 or 64 columns per block).  Parameter 5 is the slab schedule of
 * the y/x/y passes: variant v < 5 runs them over slabs of n >> v planes of z
 * (at least 1) through slab buffers that are reused, so that small slabs stay
 * in the memory-side cache; 5 <= v < 9 uses slabs of n >> (v - 4) planes that
 * alternate between two streams and two buffers, so that one slab's passes
 * overlap the next one's; 9, 10 (one stream) and 11, 12 (two streams) use
 * the finer slabs n >> 5 and n >> 6.  ns_autotune times every variant of every
 * parameter on the current state (reps evaluations each, HIP events: the z
 * passes per launch, the y/x/y passes and the slab schedule by the wall time
 * of the y/x/y phase per evaluation) and keeps the fastest; then, for each
 * parameter with several variants within 3% of its fastest, it times those on
 * whole evaluations (2 x reps each, one event pair per evaluation) and keeps the
 * lowest-numbered of them within 1% of the fastest (variants are numbered from
 * the plainest launch up; closer timings are within the scatter), since a
 * pass's variant also changes what the caches hold for its neighbours.  ms_host (NS_NTUNE x NS_TUNE_MAXV doubles, may be NULL)
 * receives the per-parameter averages of the first round in milliseconds (0
 * for variants a parameter lacks).  tune_get /
 * tune_set read or restore the choice (e.g. from a cache).  2D (n >= 256):
 * parameter 0 is the y-inverse's (0-4) and parameter 4 the y-forward's (0-6)
 * variant (radix plan and column tile; with the Boussinesq scalar, y-forward
 * variants 2, 4, 5 and 6 split the four fields over two blocks, 5 and 6 with
 * tiles of at most two and four columns), timed per launch;
 * parameter 2 the x-pass: bit 0 the layout it hands to the y-forward (0
 * row-major, 1 column-major), 2 and 3 the same layouts with one row per
 * block and one wavefront per transform (at 512, 1024 and the padded 1536
 * points; elsewhere as 0 and 1), timed over the whole right-hand side; the
 * other parameters are accepted and ignored, as are all of them below 256
 * points. */
#define NS_NTUNE 6
#define NS_TUNE_MAXV 13
int ns_autotune(ns_solver* s, int reps, double* ms_host);
int ns_tune_get(ns_solver* s, int* variant_host);
int ns_tune_set(ns_solver* s, const int* variant_host);

/* Static description of a status code. */
const char* ns_strerror(int status);

/* Release the solver (no passage of the paper: resource bookkeeping).  Frees
 * its streams, events, graph and the small pinned host buffer ns_integrate
 * reads the done flags through; caller memory is untouched.  NULL is a no-op. */
void ns_free(ns_solver* s);

#ifdef __cplusplus
}
#endif

#endif /* NS_H */
