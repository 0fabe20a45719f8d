/*
 * ensode.h -- C ABI of the ODE-ensemble record-and-replay gradient library.
 *
 * An ensemble is n independent trajectories of one autonomous system
 * y' = f(y, theta), y in R^d, integrated from t0 to t1, with theta per
 * trajectory or shared by all (paper, Section 2).  The library exposes the
 * paper's two user-facing operations (Section 3.4): a forward solve, and a
 * gradient of a scalar loss formed from sampled states.  The gradient is the
 * record-and-replay construction of Section 3.1:
 *
 *   ensemble_record   runs the adaptive solve (embedded-pair error estimate,
 *                     RMS acceptance test and step-size controller of
 *                     Section 2.1) and keeps each trajectory's accepted step
 *                     sizes h_1..h_S -- its mesh -- together with the state
 *                     before each accepted step (the "tape").
 *   ensemble_adjoint  sweeps backward over the recorded mesh: the exact
 *                     reverse-mode derivative of the fixed chain
 *                     y_i = Phi(y_{i-1}; h_i, theta) (eq. replay) with the
 *                     mesh held constant (the stop-gradient sg[h] of
 *                     Section 3.1).  It recomputes the stages of each step
 *                     from the taped state and takes vector-Jacobian
 *                     products through every stage.
 *
 * States at requested save times are integrated, not interpolated: each is
 * one extra step of the method from the last mesh point at or before it
 * (Section 3.4).  The loss is a function of those save states.
 *
 * Device layouts are structure-of-arrays with the trajectory index fastest:
 *   y0 [dim][n], params [P][n] (or [P] when shared), y_save [n_save][dim][n],
 *   grad_params [P][n] (or [P] when shared), grad_y0 [dim][n].
 * Element type is double (ENS_F64) or float (ENS_F32) for states, params
 * and their gradients; times, step sizes, the error norm and the controller
 * are always double.
 *
 * Ownership.  Every device buffer is allocated by the caller.  The library
 * allocates no device memory in ensemble_solve / ensemble_record /
 * ensemble_adjoint: a record lives inside a caller-owned pool whose size
 * ensemble_record_bytes plans.  A record stays valid, and can serve any
 * number of adjoints, while its pool is alive and unmodified.
 *
 * Streams.  Each call enqueues its work on `stream` (a hipStream_t; NULL is
 * the default stream) and returns without waiting.  The return code covers
 * argument validation and launch only.  Per-trajectory outcomes land in
 * lane_status [n] (ENS_LANE_*), valid once the stream has completed; a
 * failing trajectory never aborts the others.
 *
 * Errors.  Functions return 0 on success or a negative ENS_E* code; the
 * calling thread's last error text is available from ensemble_last_error().
 */
#ifndef ENSODE_H
#define ENSODE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define ENS_OK 0
#define ENS_EINVAL (-1)       /* null pointer, n <= 0, t1 <= t0, bad tolerance, size mismatch */
#define ENS_EUNSUPPORTED (-2) /* system x method x dtype combination not built */
#define ENS_ENOSPACE (-3)     /* pool smaller than the fixed part of a record */
#define ENS_EHIP (-4)         /* HIP runtime or launch error (text has details) */

/* ---- per-trajectory status (lane_status) ------------------------------- */
#define ENS_LANE_OK 0
#define ENS_LANE_MAX_STEPS 1   /* trial budget max_steps exhausted before t1 */
#define ENS_LANE_DT_UNDERFLOW 2 /* proposed h below 16 eps max(|t|, 1) */
#define ENS_LANE_NONFINITE 3   /* non-finite initial state or slope */
#define ENS_LANE_NOSPACE 4     /* the pool ran out of tape pages */

/* ---- problem description ----------------------------------------------- */
/* Built-in systems (paper, Appendix A; the linear system is the damped
 * rotation y' = [[-a, -w], [w, -a]] y used for closed-form checks). */
#define ENS_SYS_LORENZ 1    /* d = 3, P = 3: (sigma, rho, beta) */
#define ENS_SYS_VDP 2       /* d = 2, P = 1: (mu) */
#define ENS_SYS_ROBERTSON 3 /* d = 3, P = 3: (k1, k2, k3); stiff */
#define ENS_SYS_HIRES 4     /* d = 8, P = 12: the rate constants in order of
                               first appearance; stiff */
#define ENS_SYS_LV_UDE 5    /* d = 2, P = 1218: Lotka-Volterra (1.5, 1, 3, 1) plus a
                               2-32-32-2 tanh MLP, weights W1 [32][2], b1, W2 [32][32],
                               b2, W3 [2][32], b3; shared by all trajectories
                               (params_shared = 1), Tsit5, F32 */
#define ENS_SYS_LINEAR 6    /* d = 2, P = 2: (a, w) */

/* Methods (paper, Section 3.2).  The explicit pairs run on LORENZ, VDP and
 * LINEAR in F64 or F32, Tsit5 also on LV_UDE in F32; the Rosenbrock methods
 * (Rodas4, Rosenbrock23) on ROBERTSON, HIRES and LINEAR in F64.  Other
 * combinations return ENS_EUNSUPPORTED. */
/* Systems registered at run time (ensemble_system_register) get the ids
 * ENS_SYS_USER_BASE, ENS_SYS_USER_BASE + 1, ... */
#define ENS_SYS_USER_BASE 1000
#define ENS_USER_MAX_SYSTEMS 64
#define ENS_USER_MAX_DIM 16     /* 8 with a Jacobian (Rosenbrock methods) */
#define ENS_USER_MAX_PARAMS 64

#define ENS_TSIT5 1  /* Tsitouras 5(4), 7 stages, first-same-as-last */
#define ENS_VERN7 2  /* Verner 7(6), 10 stages */
#define ENS_RODAS4 3 /* Rosenbrock-Wanner Rodas4 (Hairer-Wanner IV.7), order
                        4(3), 6 stages, one LU of I/(gamma h) - J per step */
#define ENS_ROS23 4  /* Rosenbrock23 (Shampine-Reichelt, the paper's default
                        stiff method for fused fields, Section 3.2): order 2
                        with an O(h^3) error estimate, 3 stages in a trial
                        step and 2 in a replay, one LU per step; autonomous
                        fields only (all built-in stiff systems are) */

#define ENS_F64 1
#define ENS_F32 2

#define ENS_MAX_SAVE 64

typedef struct {
  int32_t system;        /* ENS_SYS_* */
  int32_t method;        /* ENS_TSIT5 / ENS_VERN7 / ENS_RODAS4 / ENS_ROS23 */
  int32_t dtype;         /* ENS_F64 / ENS_F32 */
  int32_t dim;           /* must equal the system's state dimension */
  int32_t nparams;       /* must equal the system's parameter count */
  int32_t params_shared; /* 0: params [P][n]; 1: params [P] for all trajectories */
} ens_problem;

typedef struct {
  int64_t n;                /* trajectories, >= 1 */
  const void* y0;           /* device [dim][n] */
  const void* params;       /* device [P][n] or [P] */
  double t0, t1;            /* t1 > t0 */
  double rtol, atol;        /* rtol >= 0, atol > 0 (or rtol > 0) */
  double h0;                /* first trial step; 0 = automatic (Hairer-Norsett-Wanner) */
  int64_t max_steps;        /* trial budget per trajectory; 0 = 100000 */
  int32_t n_save;           /* 0: the only save time is t1 */
  const double* save_times; /* host [n_save], nondecreasing, each in [t0, t1] */
  int32_t dense;            /* 0: each save state by one extra step from the last
                               mesh point before it (Section 3.4); 1: by the
                               continuous extension of the accepted step that
                               holds it (dense output, Section 3.2): the cubic
                               Hermite interpolant of the step's end states and
                               slopes, no extra step.  Explicit pairs and
                               Rosenbrock methods on the built-in systems except
                               the UDE, in ensemble_solve, ensemble_record,
                               ensemble_replay_mesh and ensemble_adjoint;
                               elsewhere ENS_EUNSUPPORTED */
} ens_ivp;

/* ---- records ------------------------------------------------------------ */
/* Pool configuration.
 *   ckpt_every = 0: full tape -- the state before every accepted step is kept
 *     with its step size (16 steps per page).
 *   ckpt_every in {16, 32, 64, 128, 256}: checkpointed tape -- one page per
 *     segment of ckpt_every accepted steps holds the state at the segment's
 *     start and the segment's step sizes; the reverse sweep replays each
 *     segment forward (the same arithmetic, so the same gradient bits) before
 *     sweeping it backward.  About 8.5 instead of 32 bytes per Lorenz step.
 * Each trajectory reserves steps_per_traj taped steps up front (rounded up
 * to whole pages); steps beyond that come from a shared overflow area of the
 * pool, handed out on demand.  steps_per_traj = 0 reserves 7/8 of the pool
 * evenly. */
typedef struct {
  void* pool;        /* device, 256-byte aligned */
  size_t pool_bytes;
  int32_t ckpt_every;
  int32_t steps_per_traj;
} ens_tape_cfg;

/* A record: plain data describing what ensemble_record wrote into a pool.
 * Filled by ensemble_record / ensemble_replay_mesh; read by the others. */
typedef struct {
  int64_t n;
  int32_t system, method, dtype, dim, nparams, params_shared;
  int32_t n_save;
  int32_t page_steps;   /* accepted steps per tape page */
  int32_t rec_bytes;    /* bytes per taped step: h (double) + state */
  int64_t n_pages;      /* pages the pool holds (reserved + overflow) */
  int64_t page_bytes;
  int32_t static_pages; /* pages reserved per trajectory */
  int32_t ckpt_every;   /* 0: full tape; else steps per checkpoint segment */
  double t0, t1;
  void* pool;
  size_t pool_bytes;
  /* device pointers into the pool */
  int32_t* steps;       /* [n] accepted steps S */
  int32_t* n_trial;     /* [n] trials (accepted + rejected) */
  int32_t* first_page;  /* [n] first overflow page, -1 if none */
  int32_t* last_page;   /* [n] page holding the last taped step */
  int32_t* status;      /* [n] copy of lane_status */
  int32_t* save_idx;    /* [n_save][n] mesh index of each save's base state */
  double* save_dt;      /* [n_save][n] side-step size t_s - t_base */
  double* save_times;   /* [max(n_save,1)] */
  void* y_final;        /* [dim][n] y_S */
  int32_t* links;       /* [overflow pages][2] previous / next page */
  unsigned long long* counters; /* [8] page counter and step totals */
  void* pages;          /* [n_pages][page_bytes] */
  void* save_base;      /* [n_save][dim][n] state each save's side step starts from
                           (the record writes it; the reverse sweep reads it) */
  int32_t dense;        /* the save states are the dense output (ens_ivp.dense) */
  void* save_base_hi;   /* dense: [n_save][dim][n] end state of the step holding
                           each save; NULL otherwise */
  double* save_h;       /* dense: [n_save][n] size of that step (0 for a save at
                           the last mesh point); NULL otherwise */
} ens_record;

typedef struct {
  unsigned long long overflow_pages_used;
  unsigned long long steps_accepted; /* summed over trajectories */
  unsigned long long trials;         /* accepted + rejected, summed */
  unsigned long long side_steps;     /* save-time steps with nonzero size */
} ens_stats;

/* Loss on the save states (paper, eq. loss, with the states at the save
 * times in place of the final state):
 *   ENS_LOSS_SUMSQ       L = scale * sum ||y(t_s)||^2
 *   ENS_LOSS_MSE_TARGET  L = scale * sum ||y(t_s) - target_s||^2, data = targets
 *   ENS_LOSS_COTANGENT   dL/dy(t_s) = data (L itself is not formed)
 * data is device [n_save][dim][n] (n_save = 0 counts as 1). */
#define ENS_LOSS_SUMSQ 0
#define ENS_LOSS_MSE_TARGET 1
#define ENS_LOSS_COTANGENT 2
typedef struct {
  int32_t kind;
  const void* data;
  double scale;
} ens_loss;

/* ---- entry points -------------------------------------------------------- */

/* Forward solve only (paper, Sections 3.3-3.4, the forward-only kernel):
 * adaptive integration of every trajectory with no record.
 * y_out: device [max(n_save,1)][dim][n], the states at the save times (t1
 * when n_save = 0).  lane_status: device [n]. */
int ensemble_solve(const ens_problem* prob, const ens_ivp* ivp, void* y_out,
                   int32_t* lane_status, void* stream);

/* Pool bytes for a record of `ivp` that reserves steps_hint taped steps per
 * trajectory plus an overflow area of 1/8 of that for trajectories that
 * need more; pass steps_hint as ens_tape_cfg.steps_per_traj. */
int ensemble_record_bytes(const ens_problem* prob, const ens_ivp* ivp,
                          int64_t steps_hint, int32_t ckpt_every,
                          size_t* bytes);

/* Record (paper, Section 3.1): adaptive solve keeping the accepted mesh and
 * the state before each accepted step.  y_save as y_out above. */
int ensemble_record(const ens_problem* prob, const ens_ivp* ivp,
                    const ens_tape_cfg* tape, ens_record* out, void* y_save,
                    int32_t* lane_status, void* stream);

/* Replay a given mesh (paper, eq. replay; the zero-padded rectangle of
 * Section 3.1): h device [cap][n] with S device [n] steps per trajectory
 * (entries past S are ignored).  Produces a record as ensemble_record does,
 * with the mesh held fixed -- the reuse of one record while theta or y0
 * moves (Section 3.1) and the frozen-mesh finite-difference checks
 * (Appendix B.6).  The mesh must reach t1: sum of the steps with the last
 * point set to t1, as the record makes it. */
int ensemble_replay_mesh(const ens_problem* prob, const ens_ivp* ivp,
                         const ens_tape_cfg* tape, const double* h,
                         const int32_t* steps, int64_t cap, ens_record* out,
                         void* y_save, int32_t* lane_status, void* stream);

/* Refresh an old mesh at new inputs: the mesh-drift policy, re-recording
 * only what drifted (the paper's future work for long fits, Section 5).
 * h [cap][n] and steps [n] (device) are an old mesh, as from
 * ensemble_mesh_export; ivp carries the new y0 and parameters with the
 * tolerances and save times.  Each trajectory takes its old steps while
 * each one's error estimate at the new inputs (the record's scaled RMS norm)
 * is <= slack; the first that fails counts as a rejected trial, and the
 * trajectory goes on with the adaptive controller from there, as
 * ensemble_record would.  A trajectory whose old steps all pass keeps its
 * old mesh bit for bit; one with steps = 0 is recorded afresh.  Produces a
 * record as ensemble_record does (same pool rules, lane_status, y_save);
 * drift_at (device [n], nullable) receives the number of old steps kept
 * (= steps[i] when none failed).  slack >= 0 (1 is the record's own test;
 * larger keeps more old steps).  Tsit5, Vern7, Rodas4 and Rosenbrock23 on
 * the built-in systems except the UDE; registered systems: ENS_EUNSUPPORTED. */
int ensemble_refresh(const ens_problem* prob, const ens_ivp* ivp, const ens_tape_cfg* tape,
                     const double* h, const int32_t* steps, int64_t cap, double slack,
                     ens_record* out, void* y_save, int32_t* lane_status, int32_t* drift_at,
                     void* stream);

/* Export a record's mesh as the zero-padded rectangle h [cap][n] and S [n]
 * (device).  Trajectories with more than cap steps are truncated and their
 * S reports the full count. */
int ensemble_mesh_export(const ens_record* rec, double* h, int32_t* steps,
                         int64_t cap, void* stream);

/* Reverse sweep (paper, Section 3.1): gradient of the loss with respect to
 * the parameters (grad_params) and, if grad_y0 is not NULL, the initial
 * states.  loss_out (device [n], nullable) receives each trajectory's loss.
 * Trajectories whose record status is not ENS_LANE_OK get NaN per-trajectory
 * gradients and loss; with shared parameters they contribute nothing to the
 * sum.  Shared parameters (problem.params_shared) give grad_params [P],
 * summed over trajectories in a fixed order (run-to-run identical).  The
 * sweep needs a caller-owned, 256-byte aligned device workspace of at least
 * ensemble_adjoint_workspace_bytes bytes, not used by a concurrent call (NULL
 * only where that size is 0; a missing, too small or misaligned workspace is
 * ENS_EINVAL).  The sweep takes the save steps first, then the mesh steps from
 * the last; that order fixes the rounding of the parameter gradient.  The ivp
 * must describe the same ensemble as the record. */
int ensemble_adjoint(const ens_problem* prob, const ens_ivp* ivp,
                     const ens_record* rec, const ens_loss* loss,
                     void* grad_params, void* grad_y0, double* loss_out,
                     void* workspace, size_t workspace_bytes, void* stream);

/* Forward mode on the recorded mesh (paper, Section 4, forward mode for few
 * inputs; the mesh held fixed as in Section 3.1): the directional derivative
 * of each trajectory's save states, and of its loss, along the tangent
 * (dy0 [dim][n], dparams [P][n]) of its initial state and parameters, by a
 * dual-number replay.  dy0 and dparams may be NULL (zero tangent); y_save_dot
 * [n_save][dim][n] (device, dtype) and loss_dot [n] (device, double) may be
 * NULL.  With the same unit tangent in every trajectory, one call gives every
 * trajectory's derivative with respect to that input: P calls give the full
 * per-trajectory gradient.  loss_dot needs loss (same kinds as
 * ensemble_adjoint): 2 scale sum y . ydot (SUMSQ), 2 scale sum (y - target)
 * . ydot (MSE_TARGET), sum c . ydot (COTANGENT).  Per-trajectory parameters
 * only; built for Lorenz, Van der Pol and the damped rotation (Tsit5, Vern7;
 * F64, F32) and Robertson and the damped rotation (Rodas4, Rosenbrock23;
 * F64); otherwise
 * ENS_EUNSUPPORTED.  Trajectories whose record failed get NaN.  Full and
 * checkpointed tapes alike (only the mesh is read). */
int ensemble_jvp(const ens_problem* prob, const ens_ivp* ivp, const ens_record* rec,
                 const void* dy0, const void* dparams, const ens_loss* loss,
                 void* y_save_dot, double* loss_dot, void* stream);

/* Register a system given as source text (the paper's user-supplied
 * right-hand side and its vector-Jacobian product, Section 3.4), compiled at
 * run time with hipRTC against the library's own kernels, so that it runs
 * the same record, reverse sweep and forward mode as a built-in system.  The
 * source defines a struct named System with static member templates on the
 * element type T, writing results through pointers:
 *   rhs(const T* y, const T* p, T* f)                 f = f(y, p)
 *   vjp(const T* y, const T* p, const T* w, T* gy, T* gp)
 *                    gy = (df/dy)^T w (overwrite), gp += (df/dp)^T w
 * and, with has_jacobian != 0 (needed for the Rosenbrock methods, dim <= 8),
 *   jac(const T* y, const T* p, T* J)                 J = df/dy, row-major
 *   jac_vjp(const T* y, const T* p, const T* u, const T* v, T* gy, T* gp)
 *                    gy, gp += d/d(y, p) of u^T J(y, p) v
 * each declared `template <class T> __device__ static void ...`.  The code
 * may use + - * / and fmaT(a, b, c) (a fused multiply-add; the library's
 * build never fuses a product and a sum by itself, so the written operations
 * fix the rounding), constants, and T(c).  It must be straight-line: no
 * branches, loops, '?', '&&', '||', preprocessor directives, inline
 * assembly, compiler intrinsics (identifiers that begin with two
 * underscores, other than __device__ and __forceinline__), shared memory,
 * synchronisation, atomics or thread and block indices -- data-dependent
 * control flow is refused (ENS_EINVAL, as is a source that does not
 * compile; ensemble_last_error gives the reason and the compiler's log).
 * A system with a Jacobian may also declare
 *   static constexpr unsigned JAC_ROWS[dim] = {...};
 * bit j of row i set where dF_i/dy_j can be nonzero: the Rosenbrock
 * factorisation and solves then leave out the structural zeros (the fill over
 * every pivot order is found at compile time; the results are the dense
 * factorisation's).  A bit declared zero must be zero for every input, or the
 * results are wrong; without the declaration the pattern is dense.
 * dim in [1, ENS_USER_MAX_DIM], nparams in [1, ENS_USER_MAX_PARAMS].  On
 * success *system receives the id to use in ens_problem.system.  The Tsit5
 * kernels in F64 (and Rodas4 with a Jacobian) are compiled here; the others
 * (Rosenbrock23 among them)
 * on first use.  Registered systems are not served by ensemble_server_*.
 * Thread-safe; a registration lasts until the process ends. */
int ensemble_system_register(const char* source, int dim, int nparams, int has_jacobian,
                             int* system);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc:
 * ensemble_adjoint with its workspace taken from a library-owned device array
 * of ENS_STATIC_WORKSPACE_BYTES on each GPU (a file-scope static; each GPU
 * the library runs on holds one until the process ends) instead of a caller
 * buffer.  Arguments and results as ensemble_adjoint; the caller still
 * provides every input and output.  A record whose
 * ensemble_adjoint_workspace_bytes exceeds ENS_STATIC_WORKSPACE_BYTES is
 * refused (ENS_EINVAL, with the sizes in the message): at 20 save times that
 * is about 2^17 FP64 Lorenz trajectories.  Calls no allocating routine.  The
 * array is shared by every call on a GPU and keeps the last call's contents
 * (nothing in it must start at zero): calls that overlap on one GPU -- on
 * different streams, or from different host threads without ordering --
 * race and give wrong results. */
#define ENS_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
int ensemble_adjoint_static(const ens_problem* prob, const ens_ivp* ivp,
                            const ens_record* rec, const ens_loss* loss,
                            void* grad_params, void* grad_y0, double* loss_out,
                            void* stream);

/* Workspace ensemble_adjoint needs for this record: per-block partial sums
 * for shared parameters, one segment of step records per trajectory for a
 * checkpointed tape, and each save's cotangent for the state its side step
 * starts from ([n_save][dim][n] elements, twice that for dense output,
 * whose saves reach both end states of their step; not for the UDE). */
int ensemble_adjoint_workspace_bytes(const ens_record* rec, size_t* bytes);

/* Totals of a finished record (synchronizes the stream). */
int ensemble_record_stats(const ens_record* rec, ens_stats* out, void* stream);

/* Text of the calling thread's last error. */
const char* ensemble_last_error(void);

/* ---- serving: continuous batching of ensemble-gradient jobs ------------
 * A server owns a caller-provided device pool and runs submitted jobs -- each
 * one ensemble_record + ensemble_adjoint on its own trajectories -- on the
 * GPU as they arrive.  Admission is by memory: a job is admitted when its
 * record (planned from steps_hint) fits in the free part of the pool; until
 * then it waits in FIFO order.  Admitted jobs of one (system, method,
 * dtype) family are packed into one launch of a persistent kernel: a grid
 * sized to the GPU whose blocks pull 256-trajectory tiles of any packed job
 * from a device-resident queue and run the record and the reverse sweep of
 * that tile back to back.  Up to n_slots launches are in flight on separate
 * streams, so jobs that arrive while others run are admitted as memory and
 * slots free up and their work overlaps on the device.
 *
 * A job's results are those of ensemble_record + ensemble_adjoint run alone
 * on it, to the bit: no arithmetic depends on the co-scheduled jobs.  A job
 * whose record runs out of pages (a lane reports ENS_LANE_NOSPACE) is run
 * again with twice the steps_hint (at most 3 times) before it fails.
 *
 * Per-trajectory parameters only (params_shared = 0); the UDE is not served.
 * A server is used from one host thread at a time.  Every device pointer of a
 * job must stay valid until the job is done or failed. */
typedef struct ens_server ens_server; /* opaque */

typedef struct {
  ens_problem prob;      /* params_shared must be 0 */
  ens_ivp ivp;           /* y0, params: device; save_times: host (copied at submit) */
  ens_loss loss;         /* loss.data: device, or NULL for ENS_LOSS_SUMSQ */
  int64_t steps_hint;    /* expected accepted steps per trajectory; 0 = 512 */
  void* y_save;          /* out [n_save][dim][n] (n_save = 1 when ivp.n_save = 0) */
  int32_t* lane_status;  /* out [n] or NULL */
  void* grad_params;     /* out [P][n] */
  void* grad_y0;         /* out [dim][n] or NULL */
  double* loss_out;      /* out [n] or NULL */
} ens_job;

#define ENS_JOB_WAITING 0
#define ENS_JOB_RUNNING 1
#define ENS_JOB_DONE 2
#define ENS_JOB_FAILED (-1)

typedef struct {
  int64_t submitted, completed, failed, retried, running, waiting;
  int64_t lanes_completed;   /* trajectory-gradients delivered */
  double p50_latency_s;      /* submission to completion, completed jobs */
  double p99_latency_s;
  double mean_latency_s;
  double busy_s;             /* first submission to last completion */
  double throughput;         /* lanes_completed / busy_s */
  size_t pool_in_use, pool_peak, pool_arena;
} ens_server_stats;

/* Create a server over the device pool [pool, pool + pool_bytes) (256-byte
 * aligned; the caller keeps it alive until destroy).  n_slots in [1, 8]
 * launches may be in flight.  Creates its streams and pinned staging
 * buffers; allocates no device memory.  EINVAL: bad arguments or a pool too
 * small for the control area (n_slots x about 1 MiB). */
int ensemble_server_create(void* pool, size_t pool_bytes, int32_t n_slots, ens_server** out);

/* Queue a job (validated here: EINVAL / EUNSUPPORTED as ensemble_record and
 * ensemble_adjoint would return) and start it if it fits.  *id names it. */
int ensemble_server_submit(ens_server* s, const ens_job* job, int64_t* id);

/* Retire finished launches and start waiting jobs; never blocks.
 * *n_active (may be NULL) = jobs waiting or running. */
int ensemble_server_progress(ens_server* s, int32_t* n_active);

/* State of a job (ENS_JOB_*); EINVAL for an unknown id. */
int ensemble_server_poll(ens_server* s, int64_t id, int32_t* state);

/* Make progress until job `id` (or, for ensemble_server_drain, every job)
 * is done or failed. */
int ensemble_server_wait(ens_server* s, int64_t id);
int ensemble_server_drain(ens_server* s);

int ensemble_server_stats(const ens_server* s, ens_server_stats* out);

/* Waits for in-flight work, then frees the server's streams and buffers. */
int ensemble_server_destroy(ens_server* s);

#ifdef __cplusplus
}
#endif

#endif /* ENSODE_H */
