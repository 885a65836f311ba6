/*
 * rte.h -- C ABI of the MI355X FC-DOM time-domain radiative-transfer library.
 *
 * The library time-steps the 2-D discrete-ordinates RTE of Gaggioli & Bruno,
 * "Parallel inverse-problem solver for time-domain optical tomography with
 * perfect parallel scaling" (arXiv:2202.09421):
 *
 *   transport operator, inflow/Fresnel condition ... Sec. 2, eqs. (Toper), (RTE)
 *   beams, generalised (MSS) sources, detectors ... Sec. 3.1, eqs. (RTEsources),
 *                                                  (RTEsources2), (OpMed)
 *   misfit .......................................... Sec. 3.2, eqs. (FObj), (FObjpr)
 *   adjoint and gradient ............................ Sec. 3.4-3.6, eqs. (AdjointProblem),
 *                                                  (FDwin22)
 *   DOM ordinates, normalised HG scattering ......... Sec. 4.1, eq. (RTETrapz)
 *   AB4 time stepping ............................... Sec. 4.2, eq. (RTEAB4)
 *   FC-Gram continuation + filtered derivative ...... Sec. 4.3, eqs. (RTEFCSum),
 *                                                  (FFilter), (RTEFCSumder)
 *   step loop ....................................... Algorithm 1
 *
 * Conventions
 *   - Units: cm, ps, 1/cm.  The grid has Nx (Ny) intervals, i.e. Nx+1 (Ny+1)
 *     nodes; node (j, i) sits at (xmin + i*dx, ymin + j*dy).
 *   - Ordinate m = 0..M-1 has angle 2*pi*m/M.  M must be a multiple of 4.
 *   - Step n = 0..K-1 advances u^n to u^{n+1} at time t_{n+1} = (n+1)*dt from
 *     u^0 = 0 with zero AB4 history.
 *   - Nq generalised sources (MSS combinations, Sec. 3.1) are solved together;
 *     beam.group selects the combination a beam belongs to.
 *   - "device" pointers are HIP device memory on the current device; "host"
 *     pointers are ordinary memory.  All buffers are owned by the caller; the
 *     plan owns only its immutable tables (allocated in rte_plan_create,
 *     released in rte_plan_destroy).
 *   - Every call returns an rte_status.  No C++ exception crosses this ABI.
 *     On failure rte_last_error() returns a message (thread-local, valid until
 *     the next call on the same thread).
 *   - Calls are enqueued on the given hipStream_t (NULL = default stream) and
 *     return before the GPU finishes unless stated otherwise.  Calls that share
 *     a plan must not overlap.
 */
#ifndef RTE_H
#define RTE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RTE_OK = 0,
  RTE_EINVAL = -1,       /* invalid argument or problem description          */
  RTE_ENOMEM = -2,       /* workspace too small / allocation failed          */
  RTE_EDEVICE = -3,      /* HIP runtime error                                */
  RTE_EUNSTABLE = -4,    /* non-finite outputs seen by the guard (see
                            rte_plan_set_guard)                              */
  RTE_EUNSUPPORTED = -5, /* valid request outside what the library implements */
  RTE_ESTATE = -6        /* call order violated (e.g. adjoint before forward)*/
} rte_status;

typedef enum { RTE_F64 = 0, RTE_F32 = 1 } rte_dtype;

/* One problem instance (plain data, host memory, copied by rte_plan_create). */
typedef struct {
  int32_t dtype;            /* rte_dtype: precision of states and medium maps      */
  int32_t reserved0;
  int64_t Nx, Ny;           /* intervals per side; each side needs >= 2*fc_d nodes */
  int64_t M;                /* ordinates, multiple of 4                            */
  int64_t K;                /* time steps                                          */
  double xmin, xmax, ymin, ymax;
  double c;                 /* speed of light in the medium, cm/ps                 */
  double dt;                /* time step, ps                                       */
  double g;                 /* HG anisotropy, |g| < 1                              */
  double hg_exponent;       /* 1.5 as printed in eq. (Henyey-Greeinstein)          */
  double n_in, n_out;       /* refractive indices inside / outside (Fresnel law)   */
  int64_t fc_d, fc_C;       /* matching points d and blend length C (Sec. 4.3)     */
  double filt_alpha, filt_beta; /* filter exp(-alpha |2k/Np|^(2 beta)), eq. (FFilter) */
  const double* fc_Q;       /* host, d*d row-major: Q[k*d+j] = P_j(k), the Gram
                               basis on the d matching points; NULL (with fc_A
                               NULL): the built-in table, available for
                               (fc_d, fc_C) = (5, 25), RTE_EUNSUPPORTED for
                               other sizes                                        */
  const double* fc_A;       /* host, C*d row-major: A[p*d+j] = blend of P_j at the
                               p-th continuation point (Sec. 4.3 step 2); NULL
                               together with fc_Q                                 */
  int64_t ckpt_every;       /* 0: keep every state u^0..u^K for the adjoint;
                               s > 0: keep checkpoints every s steps and replay
                               segments of s steps during the adjoint              */
  int64_t combo_chunk;      /* generalised sources solved together (0: all Nq).
                               With c < Nq the workspace holds the states of c
                               sources; rte_gradient runs forward, misfit and
                               adjoint chunk by chunk (the misfit and the
                               gradient are sums over sources), and rte_adjoint
                               recomputes the forward of every chunk but the
                               last one rte_forward left in the workspace.       */
} rte_problem;

/* Temporal profile T of a beam (eq. RTEsources2 leaves it general). */
typedef enum {
  RTE_PROFILE_GAUSSIAN = 0, /* exp(-(t - tau - t0)^2 / (2 sigma_t^2))                  */
  RTE_PROFILE_WINDOW = 1    /* w(|t - tau - t0| / sigma_t), the window of
                               eq. (sourcelabwind) as in eq. (sourcelab), t_s = tau+t0 */
} rte_profile;

/* A laser beam, eq. (RTEsources2)/(sourcelab):
 *   s(x, theta, t) = exp(-|x - (x,y)|^2 / (2 sigma_x^2))
 *                  * w(d(theta, theta_b) / sigma_theta) * T(t)
 * with w the window of eq. (sourcelabwind), d the circular angular distance
 * and T the temporal profile selected by `profile`.  It enters through the
 * inflow condition on the boundary.                                         */
typedef struct {
  double x, y, theta, sigma_x, sigma_theta, tau, sigma_t, t0;
  int32_t group;            /* generalised source q (0..Nq-1) this beam fires in */
  int32_t profile;          /* rte_profile; RTE_EINVAL for other values          */
} rte_beam;

/* A detector, eq. (OpMed): boundary point and footprint sigma_d (cm). */
typedef struct { double x, y, sigma_d; } rte_detector;

typedef struct rte_plan rte_plan;

/* Build host tables (ordinates, HG matrix, Fresnel/boundary map, beam and
 * detector tables, FC multipliers and FFT twiddles) and upload them.
 * Nq = 1 + max(beam.group).  Errors: RTE_EINVAL for an invalid description
 * (message says which field), among them a beam or detector off the
 * boundary (Sec. 2.1) and a dt beyond the AB4 stability limit of the
 * spectral advection, c dt pi sqrt(1/dx^2 + 1/dy^2) > 0.43 (the stiff
 * limit c dt max(a + b) <~ 0.3 depends on the maps of each call and is the
 * caller's); RTE_EDEVICE if the upload fails.                            */
int rte_plan_create(const rte_problem* prob, const rte_beam* beams, int64_t n_beams,
                    const rte_detector* dets, int64_t n_det, rte_plan** out);
int rte_plan_destroy(rte_plan* plan);

/* Queries: Nq, number of detectors, FC extended lengths (x and y lines). */
int rte_plan_info(const rte_plan* plan, int64_t* Nq, int64_t* Nd, int64_t* Np_x, int64_t* Np_y);

/* Bytes of device workspace needed by rte_forward (+ rte_adjoint when
 * with_adjoint != 0).  The workspace carries the stored states between a
 * forward and its adjoint, so the same buffer must be passed to both.  Every
 * call that takes a workspace requires its base address to be 256-byte
 * aligned (RTE_EINVAL otherwise, before any device work); hipMalloc and
 * torch allocations are.                                                   */
int rte_workspace_bytes(const rte_plan* plan, int with_adjoint, int64_t* bytes);

/* Forward solve, Algorithm 1 for all Nq sources.
 *   mu_a, mu_s : device, [Ny+1][Nx+1] in the plan dtype: a(x), b(x)
 *   G          : device out, double [Nq][Nd][K]; G[q][j][n-1] = G_j[u_q](t_n)
 *   u_final    : device out or NULL, plan dtype [Nq][Ny+1][Nx+1][M] = u^K
 *   save_states: nonzero keeps what rte_adjoint needs in the workspace
 *   workspace  : device, >= rte_workspace_bytes(plan, save_states) bytes   */
int rte_forward(rte_plan* plan, const void* mu_a, const void* mu_s, double* G, void* u_final,
                int save_states, void* workspace, int64_t workspace_bytes, void* stream);

/* rte_forward (no kept states) without a workspace argument, for callers
 * that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation.  The workspace lives in a
 * static device array of 128 MiB that each GPU the library runs on holds
 * until the process ends; its address is resolved once per device on the
 * first call there.  The call allocates nothing (no hipMalloc, no events);
 * everything the forward needs at zero is cleared by the call itself, the
 * rest keeps the previous call's contents.  Calls that overlap on one GPU
 * (two streams, or two threads) share the array and race: serialize them.
 * A forward saved by rte_forward / rte_gradient in a caller workspace stays
 * valid.  Same arguments and outputs as rte_forward with save_states = 0.
 * RTE_ENOMEM when rte_workspace_bytes(plan, 0) exceeds 128 MiB, before any
 * device work (the 257 x 257-node, 32-ordinate, 2000-step FP64 forward needs
 * 136 MB; with 28 ordinates it fits).                                      */
int rte_forward_noalloc(rte_plan* plan, const void* mu_a, const void* mu_s, double* G, void* u_final, void* stream);

/* Exact discrete adjoint of the last rte_forward(save_states=1) made with the
 * same workspace and medium (discrete image of eq. (AdjointProblem)).
 *   G_bar      : device, double [Nq][Nd][K], the cotangent dJ/dG
 *   dmu_a/dmu_s: device out, double [Ny+1][Nx+1]: dJ/da_ij, dJ/db_ij summed over
 *                the Nq sources (discrete eq. (FDwin22) and its b analogue).
 * RTE_ESTATE if no saved forward is in the workspace: none was made, a later
 * call on the plan overwrote it (rte_forward without saving, rte_forward_ex,
 * rte_plan_autotune, rte_plan_time_kernels), or `workspace` is not the buffer
 * the saving call (rte_forward, rte_gradient, rte_gradient_continuous, a
 * batch gradient) used.  The medium must be the one of that call (not
 * checked).                                                                */
int rte_adjoint(rte_plan* plan, const void* mu_a, const void* mu_s, const double* G_bar,
                double* dmu_a, double* dmu_s, void* workspace, int64_t workspace_bytes, void* stream);

/* Misfit and gradient, eqs. (FObj)/(FObjpr) with the rectangle rule in time:
 *   J = 1/2 dt sum_q sum_j sum_{n=1..K} (G - G_meas)^2,
 * followed by the adjoint with G_bar = dt (G - G_meas).
 *   G_meas : device, double [Nq][Nd][K]
 *   J      : device out, one double
 *   G      : device out, double [Nq][Nd][K] (the forward traces)           */
int rte_gradient(rte_plan* plan, const void* mu_a, const void* mu_s, const double* G_meas,
                 double* J, double* dmu_a, double* dmu_s, double* G, void* workspace,
                 int64_t workspace_bytes, void* stream);

/* Staged gradient.  rte_gradient enqueues a fixed sequence of n_ops
 * operations (rte_gradient_ops): one that zeroes the accumulators; per
 * combination chunk the forward start, K forward steps, the misfit, the
 * adjoint start and then K adjoint steps (every state kept) or, per
 * checkpoint segment from the last, the checkpoint restore, the replayed
 * forward steps and the adjoint steps; and a final reduction of the gradient
 * over the sources.  rte_gradient_range enqueues the operations with index
 * in [first, last), with the arguments of rte_gradient.  The ranges of one
 * gradient must be enqueued in order from first = 0 with identical
 * arguments (RTE_ESTATE otherwise); consecutive ranges that cover
 * [0, n_ops) compute exactly what one rte_gradient call computes, bit for
 * bit.  J, dmu_a, dmu_s and G are complete once the range holding the last
 * operation has run; the guard (if enabled) checks them then.  For
 * long solves that must be interleaved with other work, bounded in time per
 * call, or progress-reported.  Always eager (graph mode does not apply).
 * RTE_EINVAL for a range outside [0, n_ops].                               */
int rte_gradient_ops(const rte_plan* plan, int64_t* n_ops);
int rte_gradient_range(rte_plan* plan, const void* mu_a, const void* mu_s, const double* G_meas, double* J,
                       double* dmu_a, double* dmu_s, double* G, void* workspace, int64_t workspace_bytes,
                       int64_t first, int64_t last, void* stream);

/* A space-time-angle field given as a sum of separable products
 *   f(x_i, y_j, theta_m, t_n) = sum_k X[k][n+3][i] * Y[k][n+3][j] * Th[k][m]
 * on the time levels n = -3 .. K (row n+3 of X and Y), nodes i, j and
 * ordinates m = 0..M-1 in natural order (theta_m = 2 pi m / M).  Device
 * arrays, FP64: X [rank][K+4][Nx+1], Y [rank][K+4][Ny+1], Th [rank][M].
 * rank = 0: absent.                                                        */
typedef struct {
  int32_t rank;
  int32_t reserved0;
  const double* X;
  const double* Y;
  const double* Th;
} rte_separable;

/* Extra data of a forward solve beyond the paper's laser-beam problem, as in
 * the manufactured-solution problem eq. (RTEdisp) of Sec. 5, and scalar-flux
 * snapshots as in the laboratory simulation of Sec. 5 (Fig. 6):
 *   u0      : device [Nq][Ny+1][Nx+1][M] (plan dtype), initial state (NULL: 0)
 *   u_hist  : device [3][Nq][Ny+1][Nx+1][M], the states at t_{-1}, t_{-2},
 *             t_{-3}; the AB4 history starts from L^{-k} = L(u_hist[k-1]) +
 *             q(t_{-k}) (NULL: zero history, as for the beam problem)
 *   source  : volumetric source q added to the right-hand side,
 *             u_t = c (L(u) + q)
 *   inflow  : data u_b on Gamma_- after every update (with the plan's Fresnel
 *             reflection, which vanishes for n_in = n_out), replacing the
 *             beams; rank 0 keeps the beams.
 *   n_snap, snap_steps, snap_flux : scalar flux (eq. photondensity with the
 *             trapezoid rule on the uniform ordinates, dtheta sum_m u_m) of the
 *             states u^n for the n_snap time levels snap_steps[k] in [0, K]
 *             (host array, any order, repeats allowed), written to the device
 *             array snap_flux [Nq][n_snap][Ny+1][Nx+1] (FP64, summed in FP64);
 *             n_snap = 0: none.  RTE_EINVAL for n_snap < 0, a NULL array with
 *             n_snap > 0, or a level outside [0, K].
 * The same fields apply to every generalised source.                       */
typedef struct {
  const void* u0;
  const void* u_hist;
  rte_separable source;
  rte_separable inflow;
  int32_t n_snap;
  int32_t reserved1;
  const int32_t* snap_steps;
  double* snap_flux;
} rte_forward_extra;

/* Forward solve with the extra data (Algorithm 1 with q, u0, u_b): outputs
 * as rte_forward (G, optional u_final); no states are kept.  Workspace:
 * rte_workspace_bytes(plan, 0).  RTE_EINVAL for a negative rank or a NULL
 * table of a positive-rank field.                                          */
int rte_forward_ex(rte_plan* plan, const void* mu_a, const void* mu_s, const rte_forward_extra* extra,
                   double* G, void* u_final, void* workspace, int64_t workspace_bytes, void* stream);

/* The paper's own gradient (Sec. 3.3): the continuous adjoint problem
 * eq. (AdjointProblem) solved by the forward machinery, then eq. (FDwin22).
 * With s = T - t and reversed ordinates, psi(x, theta, s) = lambda(x,
 * theta + pi, T - s) satisfies the forward equation with zero initial data;
 * its inflow condition is the forward one (Fresnel reflection) plus the
 * detector residual (1 - f) sum_j (G_j - G~_j) w(|x - x_j| / sigma_d) at
 * t = T - s.  Each psi step is a forward step (line pass, node pass), and
 * the node pass adds, with psi^k = lambda(t_{K-k}) paired with u^{K-k},
 *   dmu_a -= dtheta dx dy dt sum_m lambda_m u_m,
 *   dmu_s += dtheta dx dy dt sum_m lambda_m ((W u)_m - u_m).
 * Same arguments, outputs and workspace as rte_gradient (J and G identical
 * to it); the gradient approximates the exact discrete one of rte_gradient
 * to discretisation error (first order under refinement), not to rounding.
 * Always launched eagerly (graph mode does not apply).  Leaves the forward
 * states in the workspace like rte_gradient.                              */
int rte_gradient_continuous(rte_plan* plan, const void* mu_a, const void* mu_s, const double* G_meas,
                            double* J, double* dmu_a, double* dmu_s, double* G, void* workspace,
                            int64_t workspace_bytes, void* stream);

/* Non-finite guard.  With enable != 0, rte_forward, rte_forward_ex,
 * rte_adjoint, rte_gradient, rte_gradient_continuous and rte_batch_gradient
 * scan their FP64 outputs (G, snapshots, J, dmu_a, dmu_s) on the device after
 * the solve, wait for the stream, and return RTE_EUNSTABLE when any value is
 * NaN or infinite: a time step beyond the stiff limit c dt max(a + b) ~ 0.3
 * or a non-finite medium map (one bad node reaches every detector within
 * two steps, the spectral derivative being global along a line).  The
 * outputs are still written.  Off by default (no synchronisation).         */
int rte_plan_set_guard(rte_plan* plan, int enable);

/* Graph mode.  With enable != 0, rte_gradient records its whole launch
 * sequence (forward, misfit, adjoint: ~6 kernels per time step) into one HIP
 * graph on first use and replays it while the argument pointers and the
 * workspace size stay the same; any change re-records.  Profiling events are
 * not recorded into the graph.  enable == 0 frees the graph.              */
int rte_plan_set_graph(rte_plan* plan, int enable);

/* A batch of independent plans of any sizes (uneven grids, ordinate counts,
 * step counts; multiple-staggered-source combinations or separate
 * instances).  The batch refers to the plans; they must outlive it.       */
typedef struct rte_batch rte_batch;
int rte_batch_create(rte_plan* const* plans, int64_t n, rte_batch** out);
int rte_batch_destroy(rte_batch* batch);

/* rte_gradient of every plan of the batch in ONE graph launch on `stream`:
 * each instance is a branch of the graph, so small instances run alongside
 * large ones.  Every argument is an array of n entries with the meaning of
 * the rte_gradient argument of the same name; each instance needs its own
 * workspace.  The graph is recorded on the first call and replayed while all
 * pointers stay the same.                                                  */
int rte_batch_gradient(rte_batch* batch, const void* const* mu_a, const void* const* mu_s,
                       const double* const* G_meas, double* const* J, double* const* dmu_a,
                       double* const* dmu_s, double* const* G, void* const* workspaces,
                       const int64_t* workspace_bytes, void* stream);

/* Launch schedule of the per-step kernels.  The units-per-wave and
 * tiles-per-block choices compute the same result bit for bit; the generic
 * line kernel computes the same operator with another FFT factorisation
 * (equal to rounding).  Zero fields mean the default (one unit per
 * workgroup, two waves per unit, tables staged unless set, the node tiling
 * of the plan).  The waves-per-unit and table-placement choices are bitwise
 * neutral as well.  Extended lengths outside {90, 160, 288, 540} have one
 * four-step variant (one unit, two waves, global tables) whatever is set.
 *   line_units_per_wave : 1 or 2 work units (two lines x four slots of one
 *                         ordinate group) per workgroup of the four-step line
 *                         kernel, transformed one after the other
 *   line_waves_per_unit : 1 or 2 waves sharing the transforms of one unit
 *   line_global_tables  : 1 = the FFT twiddles and derivative multipliers are
 *                         read from global memory (cached) instead of being
 *                         staged in LDS (smaller LDS footprint)
 *   line_generic        : 1 = use the generic Stockham line kernel even where
 *                         the extended length has a four-step split
 *   node_tiles_per_block: 16-node tiles per workgroup of the node passes
 *                         (1, 2 or 4; times the 16-slot row tiles, at most 8
 *                         waves; plans with M > 64 always use 1)          */
typedef struct {
  int32_t line_units_per_wave;
  int32_t line_generic;
  int32_t node_tiles_per_block;
  int32_t line_waves_per_unit;
  int32_t line_global_tables;
  int32_t reserved;          /* 0 */
} rte_schedule;

/* Current schedule of the plan (defaults resolved). */
int rte_plan_get_schedule(const rte_plan* plan, rte_schedule* out);

/* Sets the schedule; RTE_EINVAL for values outside the ranges above.  A
 * recorded graph is dropped (the next graph-mode call re-records).      */
int rte_plan_set_schedule(rte_plan* plan, const rte_schedule* sched);

/* Autotuner: times every admissible schedule of the four per-step kernel
 * classes on this plan's shapes (a few launches each, on `stream`, with
 * HIP events; the call synchronizes the stream), keeps the fastest choice
 * per class and stores it in the plan; `chosen` (host, may be NULL)
 * receives it.  Uses the gradient workspace (>= rte_workspace_bytes(plan,
 * 1)) as scratch: any saved forward is invalidated.  mu_a, mu_s as in
 * rte_forward.  Not for use under stream capture.                         */
int rte_plan_autotune(rte_plan* plan, const void* mu_a, const void* mu_s, void* workspace,
                      int64_t workspace_bytes, void* stream, rte_schedule* chosen);

/* Instrumentation.  Kernel classes of one time step: */
typedef enum {
  RTE_K_LINES_FWD = 0, /* FC derivatives along x and y lines          */
  RTE_K_NODE_FWD = 1,  /* scattering, AB4, inflow condition, flux     */
  RTE_K_NODE_ADJ = 2,  /* adjoint node pass and gradient accumulation  */
  RTE_K_LINES_ADJ = 3, /* transposed FC derivatives along x and y     */
  RTE_K_COUNT = 4
} rte_kernel_class;

/* enable != 0: every later launch of a time-step kernel on this plan is
 * bracketed by two hipEvents recorded on the call's stream (they add a few
 * microseconds per launch).  enable == 0 stops recording and drops pending
 * records.                                                                 */
int rte_profile_enable(rte_plan* plan, int enable);

/* Waits for the recorded events and returns, per kernel class, the summed
 * GPU time (ms) and the number of launches since the last read; then clears
 * the records.  total_ms and launches point to RTE_K_COUNT entries (host). */
int rte_profile_read(rte_plan* plan, double* total_ms, int64_t* launches);

/* Per-launch duration (microseconds) of each per-step kernel class with the
 * plan's current schedule: `reps` (1..10000) back-to-back launches of the
 * class on the plan's shapes are recorded as one HIP graph, replayed on
 * `stream` between two HIP events, and the time is divided by `reps`.  The
 * launches work on zeroed state arrays of `workspace` (>= rte_workspace_bytes
 * (plan, 1)), which this call overwrites (a saved forward is invalidated).
 * us points to RTE_K_COUNT doubles (host).  Synchronizes the stream; not for
 * use under stream capture.                                              */
int rte_plan_time_kernels(rte_plan* plan, const void* mu_a, const void* mu_s, void* workspace,
                          int64_t workspace_bytes, void* stream, int reps, double* us);

/* Thread-local message of the last failed call ("" if none). */
const char* rte_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RTE_H */
