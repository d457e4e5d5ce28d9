/*
 * scp_batch.h -- C ABI of the batched 6-DoF SCP solver for AMD MI355X (gfx950).
 *
 * The library solves many independent free-final-time 6-DoF powered-descent guidance
 * problems at once with the prox-linear sequential convex programming method, the
 * continuous-time constraint satisfaction (CTCS) reformulation and the customized PIPG
 * solver of Chari, Kamath, Elango and Acikmese, "Fast Monte Carlo Analysis for 6-DoF
 * Powered-Descent Guidance via GPU-Accelerated Sequential Convex Programming"
 * (sections "Problem Formulation", "Sequential Convex Programming", "Convex Optimization
 * Solver", "6-DoF Powered Descent Guidance").
 *
 * Conventions
 *   state   x = (m, r[3], v[3], q[4], w[3], y)  n_x = 15, q a Hamilton quaternion, scalar
 *           first, body to inertial; y the CTCS constraint-violation integrator.
 *   control u = (T[3], s)                         n_u = 4, T body-frame thrust, s dilation;
 *           or u = (T[3], gamma[3], s)            n_u = 7 with the reaction-control torque
 *           gamma (body frame) of the paper's full control set (scp_settings.n_u).
 *   "real"  is float when scp_settings.dtype == SCP_F32 and double when SCP_F64.
 *   All arrays are dense, row-major, device-resident (allocated by the caller on the
 *   device the handle was created for), and 16-byte aligned.
 *
 * Shapes
 *   The structs below pass bare pointers, so the library cannot see an array's shape or
 *   element type: it trusts the caller to pass arrays of the documented shapes and of the
 *   handle's dtype.  Before anything is launched it checks what it can see -- null pointers,
 *   16-byte alignment, the batch against max_batch -- and an instance whose K is outside
 *   [2, k_max] is not solved (status 3).  The Python binding checks every array's shape,
 *   dtype, device and contiguity before it calls in.
 *
 * Threading and ordering
 *   Every call that takes device memory only enqueues work on the handle's HIP stream and
 *   returns; outputs are valid after the stream is synchronized.  A handle is not
 *   thread-safe: use one handle per stream.  Nothing throws across this interface; every
 *   entry point returns an scp_status and, on failure, scp_batch_last_error() describes it.
 *
 * Ownership
 *   The caller owns every problem, solution and workspace buffer.  The library allocates no
 *   device memory in scp_batch_solve; its workspace is the caller's buffer handed to
 *   scp_batch_create.  The handle owns host-side state only.
 */
#ifndef SCP_BATCH_H
#define SCP_BATCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct scp_batch_s *scp_batch;

typedef enum {
    SCP_OK = 0,
    SCP_ERR_ARG = 1,          /* a null pointer or an out-of-range setting                */
    SCP_ERR_SHAPE = 2,        /* batch larger than max_batch, node count out of range     */
    SCP_ERR_DTYPE = 3,        /* unknown dtype                                            */
    SCP_ERR_DEVICE = 4,       /* no such device, or not a gfx950 device                   */
    SCP_ERR_HIP = 5,          /* a HIP runtime call failed (message has the HIP error)    */
    SCP_ERR_WORKSPACE = 6,    /* workspace missing, misaligned or smaller than required   */
    SCP_ERR_STATE = 7,        /* the call needs state the handle does not have            */
    SCP_ERR_UNSUPPORTED = 8   /* a setting the library does not implement                 */
} scp_status;

typedef enum { SCP_F32 = 0, SCP_F64 = 1 } scp_dtype;

/* Solver settings; copied at scp_batch_create.  The weights, scalings and tolerances are the
 * quantities the paper leaves as inputs: w_cost, w_prox and w_ep weigh the terminal cost,
 * the proximal term and the exact l1 penalty of the subproblem (eq. cvx-subproblem-custom);
 * px, pu are the diagonal prescaling P_x, P_u; omega, rho, pipg_eps_* and pipg_check_every
 * are the PIPG step-size ratio, extrapolation, tolerances and check period (Algorithms
 * "PIPG_custom" and "Customized stopping criterion"); power_* are those of the customized
 * power iteration. */
typedef struct {
    int32_t dtype;              /* scp_dtype of the bulk arithmetic and of "real" arrays   */
    int32_t k_max;              /* largest node count K of any instance (2..50)            */
    int32_t max_batch;          /* largest batch passed to scp_batch_solve                 */
    int32_t scp_iters_max;      /* maximum convex subproblems per instance                 */
    int32_t pipg_iters_max;     /* PIPG iterations per subproblem (j_max)                  */
    int32_t pipg_check_every;   /* j_check                                                 */
    int32_t rk4_substeps;       /* RK4 steps per discretization interval                   */
    int32_t power_iters_max;    /* power-iteration limit                                   */
    int32_t early_exit;         /* 1: SCP and PIPG stop on their tolerances; 0: fixed work */
    int32_t node_projections;   /* bitmask of node-wise convex path-constraint sets the
                                   PIPG projection also enforces: 1 dry mass, 2 glide slope,
                                   4 tilt, 8 rate, 16 thrust (gimbal cone and T_max);
                                   0 = the paper's set only (boundary values, s box)       */
    int32_t mode;               /* 0: kernel launches per solve, workgroup b <-> instance b;
                                   1: the launch sequence is captured once into a HIP graph
                                   (per set of arguments) and replayed;
                                   2: as 1, and subproblem workgroups take instances by node
                                   count, descending (hardware dispatch as the work queue);
                                   3: as 1, with a persistent subproblem grid (resident
                                   workgroups pop instances from an atomic queue in that
                                   order);
                                   4: as 2, and when k_max > 12 the subproblem launch is
                                   split by node count: K <= 12 in 192-lane workgroups,
                                   12 < K <= 20 in 320-lane ones, the rest in the
                                   k_max-sized kernel (up to three launches per SCP
                                   iteration, on two streams) */
    int32_t grad_pipg_steps;    /* PIPG steps of the differentiated last iteration (0: the
                                   handle computes no gradients and carves no scratch)     */
    int32_t grad_ckpt_every;    /* checkpoint period of the reverse sweep (1..steps)       */
    int32_t occupancy;          /* FP32 subproblem kernel variant: 0 = the compiler's
                                   register budget, 4, 5 or 6 = registers bounded for that
                                   many waves per SIMD; FP64 always uses 0                */
    int32_t grad_rk4_tangent;   /* how scp_batch_grad differentiates the discretization:
                                   0 = reverse (adjoint) sweep through the RK4 stages,
                                   1 = forward tangents along (alpha_mdot, T_max); the
                                   two agree to rounding, 1 is the faster here            */
    int32_t scalar_dilation;    /* 0: the dilation s is a first-order-hold control with one
                                   value per node (section "Free-Final-Time Problem");
                                   1: one dilation value over the horizon, i.e. each
                                   subproblem restricted to s_1 = ... = s_K (its dynamics
                                   column in interval k is B^-_k[:, s] + B^+_k[:, s]); PIPG
                                   projects the dilation values onto their mean clamped to
                                   the s box.  The initial guess must hold one value (it does:
                                   s_init).  Not with mode 3 or grad_pipg_steps > 0
                                   (SCP_ERR_UNSUPPORTED at scp_batch_create); occupancy is
                                   ignored (the FP32 variant is bounded to six waves per
                                   SIMD) and scp_batch_autotune times modes 1, 2 and 4
                                   only (the other entries of ms_out stay -1)             */
    int32_t n_u;                /* controls per node: 4 = (T, s); 7 = (T, gamma, s), the
                                   reaction-control torque gamma of section "6-DoF Powered
                                   Descent Guidance" adding J^-1 gamma to w_dot and the
                                   path constraint ||gamma||^2 <= gamma_max^2 (params
                                   column 23) to the CTCS integrand.  With 7: not with
                                   scalar_dilation or grad_pipg_steps > 0
                                   (SCP_ERR_UNSUPPORTED)                                  */
    int32_t power_fp32;         /* precision of the customized power iteration (Algorithm
                                   "Customized power iteration") on the FP32 path: 0 = the
                                   iterate and the block products in FP64 over the FP32
                                   blocks (default); 1 = in FP32, sigma and the stopping
                                   test still FP64 (faster, a variant).  Ignored with
                                   SCP_F64.  Must be 0 or 1                               */
    double scp_tol;             /* converged: scaled step inf-norm <= scp_tol ...          */
    double feas_tol;            /* ... and scaled defect, scaled CTCS excess <= feas_tol   */
    double pipg_eps_abs, pipg_eps_rel;
    double power_eps_abs, power_eps_rel, power_buff;
    double w_cost, w_prox, w_ep, omega, rho;
    double px[15], pu[7];       /* pu: the first n_u entries are read                       */
} scp_settings;

/* A batch of B problems.  params columns (24): m_wet, m_dry, alpha_mdot, g[3], J_diag[3],
 * r_T[3], T_min, T_max, delta_max, gamma_gs, theta_max, omega_max, s_min, s_max, eps_ctcs,
 * s_init, v_max, gamma_max (angles in radians; v_max = +inf for no speed bound, otherwise the
 * path constraint ||v||^2 <= v_max^2 of section "6-DoF Powered Descent Guidance" joins the
 * CTCS integrand; gamma_max bounds the torque likewise and is read only with n_u = 7, +inf
 * for no bound).  x0 is the initial state (its y entry is ignored: y(0) = 0);
 * xf = (r, v, q, w) is the landing condition, of which r, v, the tilt part (q2, q3) of q and
 * the transverse rates (w2, w3) are imposed (the roll angle and rate are free: thrust alone
 * exerts no torque about the thrust axis).  An instance whose K is outside [2, k_max] is not
 * solved (status 3). */
typedef struct {
    int32_t batch;              /* B >= 0                                                  */
    const void *x0;             /* real [B][15]                                            */
    const void *xf;             /* real [B][13]                                            */
    const void *params;         /* real [B][24]                                            */
    const int32_t *K;           /* int32 [B] node counts                                   */
    /* Optional first reference trajectory of the SCP iteration (NULL: the built-in guess,
     * straight-line r, v, w, interpolated q, constant m, y = 0, hover thrust, s = s_init).
     * Rows k < K_b of instance b are taken as given, all 15 state entries (y too) and all
     * n_u controls; e.g. an earlier solution warm-starts the solve.  Either may be NULL
     * independently; 16-byte aligned like the other arrays. */
    const void *x_init;         /* real [B][k_max][15] or NULL                             */
    const void *u_init;         /* real [B][k_max][n_u] or NULL                            */
} scp_problem;

/* Per-instance results.  x, u hold the trajectory on the K nodes (rows >= K are zero).
 * status: 0 converged, 1 iteration limit reached, 2 non-finite value met (the instance is
 * frozen, the others are unaffected), 3 invalid instance (K out of range). */
typedef struct {
    void *x;                    /* real [B][k_max][15]                                     */
    void *u;                    /* real [B][k_max][n_u]                                    */
    void *t_f;                  /* real [B] time of flight = integral of s                 */
    void *m_f;                  /* real [B] final mass                                     */
    int32_t *status;            /* int32 [B]                                               */
    int32_t *scp_iters;         /* int32 [B] convex subproblems solved                     */
    int32_t *pipg_iters;        /* int32 [B] PIPG iterations summed over subproblems       */
    double *defect_inf;         /* f64 [B] scaled dynamics defect (inf-norm) at the end    */
    double *ctcs_viol;          /* f64 [B] largest per-interval CTCS increment y_k+1 - y_k */
    double *objective;          /* f64 [B] -m_f + w_ep * sum |scaled defect|               */
} scp_solution;

/* Bytes of device workspace a handle with these settings needs (0 on invalid settings). */
size_t scp_batch_workspace_bytes(const scp_settings *settings);

/* Create a handle on HIP device `device`, enqueuing on `hip_stream` (a hipStream_t, NULL
 * for the default stream).  `workspace` is caller-owned device memory of at least
 * scp_batch_workspace_bytes() bytes, 256-byte aligned, that must outlive the handle. */
scp_status scp_batch_create(const scp_settings *settings, int device, void *hip_stream,
                            void *workspace, size_t workspace_bytes, scp_batch *out);

/* Solve every instance of `problem`, writing `solution` (prox-linear SCP, section
 * "Sequential Convex Programming"; each subproblem is discretized by RK4 on the state and
 * variational equations, scaled as in "Convex Subproblem with Prescaling and
 * Preconditioning", and solved by the customized power iteration and PIPG).  Enqueued on the
 * handle's stream.  Inputs are validated before anything is enqueued. */
scp_status scp_batch_solve(scp_batch h, const scp_problem *problem, scp_solution *solution);

/* Change the stream later calls enqueue on. */
scp_status scp_batch_set_stream(scp_batch h, void *hip_stream);

/* Message for the last failed call on this handle ("" if none); valid until the next call. */
const char *scp_batch_last_error(scp_batch h);

/* Message for the last failed call without a handle in this process (scp_batch_create,
 * scp_batch_solve_noalloc). */
const char *scp_batch_create_error(void);

/* Launch timing, for measurement tools.  With profiling enabled, every kernel launch of a
 * solve is bracketed by two HIP events recorded on the handle's stream (created here, once;
 * no device memory is allocated).  scp_batch_profile_read() waits for the last solve and
 * returns, per kernel class (0 initial guess, 1 discretization, 2 subproblem PIPG iteration,
 * 3 preparation: convergence test of the reference and power iteration), the summed launch
 * durations in milliseconds (ms[SCP_KERNEL_CLASSES]) and the number of launches
 * (launches[SCP_KERNEL_CLASSES]).  Reading without profiling enabled is SCP_ERR_STATE. */
#define SCP_KERNEL_CLASSES 4
scp_status scp_batch_profile(scp_batch h, int enable);
scp_status scp_batch_profile_read(scp_batch h, double *ms, int32_t *launches);

/* Autotuner.  Times the launch variants (mode, occupancy) = (1, 0), (2, 0), (3, 0), (1, 5),
 * (2, 5), (1, 6), (2, 6), (4, 0), (4, 5), (4, 6) -- variant v is entry v of that list; see
 * scp_settings.mode and .occupancy -- with
 * HIP events, solving `problem` into `solution` (whose contents are overwritten), and keeps
 * the fastest for later solves on this handle.  *variant_out receives its index and
 * ms_out[SCP_TUNE_VARIANTS] the measured milliseconds per variant (-1 where not timed).
 * With a non-NULL cache_path, a JSON-lines file keyed by (GPU arch, k_max, dtype,
 * early_exit, node_projections, batch) is consulted first -- a hit skips the timing -- and
 * the new result is appended.  Synchronizes the handle's stream. */
#define SCP_TUNE_VARIANTS 10
scp_status scp_batch_autotune(scp_batch h, const scp_problem *problem, scp_solution *solution,
                              const char *cache_path, int32_t *variant_out, double *ms_out);

/* The dispatch mode and occupancy variant the handle currently uses. */
scp_status scp_batch_mode(scp_batch h, int32_t *mode_out, int32_t *occupancy_out);

/* Starting point of the last convex subproblem an instance solved: the reference trajectory
 * it linearized about, the warm-start duals (mu+, mu-, the dynamics dual phi and the CTCS
 * dual theta; x^ and u^ start at zero) and the buffered power-iteration estimate sigma.
 * Caller-owned device arrays; rows beyond an instance's K are not written.  Real arrays have
 * the handle's dtype. */
typedef struct {
    void *xbar;                 /* real [B][k_max][15]                                     */
    void *ubar;                 /* real [B][k_max][4] (n_u = 4)                            */
    void *mup, *mum, *phi;      /* real [B][k_max-1][15]                                   */
    void *th;                   /* real [B][k_max-1]                                       */
    double *sigma;              /* f64  [B]                                                */
} scp_lastiter;

/* As scp_batch_solve, and every subproblem also writes its starting point into `last`, so
 * that after the solve `last` holds each instance's last subproblem (the input of
 * scp_batch_grad).  Asynchronous on the handle's stream. */
scp_status scp_batch_solve_record(scp_batch h, const scp_problem *problem,
                                  scp_solution *solution, const scp_lastiter *last);

/* Vector-Jacobian product of the last SCP iteration (not the full [B][2][18] Jacobian: a
 * caller that wants both rows calls it twice, with cotangents (1, 0) and (0, 1), as the Python
 * binding's autograd function does for a general cotangent in one call).  The differentiated
 * map, an extension
 * (the paper does not differentiate its solver), takes
 *     theta = (x0[15], m_wet, alpha_mdot, T_max)
 * to (m_f, t_f) through one SCP iteration started from `last`: the discretization at
 * last->xbar/ubar (section "Discretization" with the variational equations of "Gradient of
 * Discretized Dynamics"), the prescaled subproblem ("Convex Subproblem with Prescaling and
 * Preconditioning"), settings.grad_pipg_steps steps of PIPG_custom (Algorithm "PIPG_custom",
 * no early exit) from last's warm start with step sizes from last->sigma, and the reference
 * update; m_f = m at the last node, t_f the integral of s.  m_wet is the initial-mass
 * boundary value, so a change of m_wet moves x0[0] with it.
 *   cotangent  real [B][2]  (c_m, c_t)
 *   grad       real [B][18] c_m dm_f/dtheta + c_t dt_f/dtheta (zero for invalid instances)
 *   value      real [B][2]  (m_f, t_f) of the map, or NULL
 * The reverse sweep recomputes the PIPG steps from checkpoints every grad_ckpt_every steps.
 * Needs a handle created with grad_pipg_steps > 0 (SCP_ERR_STATE otherwise).  Uses the
 * handle's workspace: do not overlap with a solve on the same handle.  Asynchronous. */
scp_status scp_batch_grad(scp_batch h, const scp_problem *problem, const scp_lastiter *last,
                          const void *cotangent, void *grad, void *value);

/* Multi-start choice (the paper's Conclusion names multi-start as future work): after one
 * batched solve of every start of every problem, pick for each problem its cheapest converged
 * start.  `solution` holds a batch solved by this handle of problems * starts instances in
 * which the starts of problem p are instances p*starts .. p*starts + starts - 1 (they differ
 * only in their initial guess, e.g. the dilation guess s_init in params).  For each problem:
 *   best  int32 [problems]  the start with status 0 and the smallest objective (ties: the
 *                           smallest start index), or -1 when no start converged;
 *   out   a solution of `problems` instances (this handle's dtype and k_max) that receives
 *         that start's results -- start 0's when none converged, so out->status says why.
 * problems * starts must not exceed max_batch; out and best may not overlap the solution or
 * each other (SCP_ERR_ARG); every array is device memory, 16-byte aligned (best: 4); with
 * problems = 0 nothing is read or written.  Reads nothing but `solution`, so it may follow
 * the solve on the same stream.  Asynchronous on the handle's stream. */
scp_status scp_batch_select_best(scp_batch h, const scp_solution *solution, int32_t problems,
                                 int32_t starts, int32_t *best, scp_solution *out);

/* Solve without allocating anything: for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid allocation).  As
 * scp_batch_solve for a handle created with `settings`, with plain kernel launches (workgroup
 * b <-> instance b, whatever settings->mode says; gradients are not available here), but
 * with no handle and no caller workspace: the workspace is a fixed device array inside the
 * library, of SCP_NOALLOC_SCRATCH_BYTES (64 MiB) per device, which each device holds from the
 * library's load until the process ends.  A batch whose workspace (scp_batch_workspace_bytes
 * of these settings with max_batch = batch and no gradients) exceeds it is rejected with
 * SCP_ERR_WORKSPACE before anything is launched: about 1,300 instances at k_max = 30 and
 * 2,000 at k_max = 20 in FP32.  Every such call on a device shares that device's array, so
 * calls that overlap on one device race (they must be ordered, e.g. on one stream); the
 * kernels rewrite every part of the array they read, so no clearing is needed between calls.
 * Enqueued on `hip_stream` (NULL: the default stream) of `device`, which becomes current for
 * the call and is restored.  Errors as scp_batch_create (message: scp_batch_create_error). */
#define SCP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
scp_status scp_batch_solve_noalloc(const scp_settings *settings, int device, void *hip_stream,
                                   const scp_problem *problem, scp_solution *solution);

/* Release the handle (not the caller's workspace).  Synchronizes its stream first. */
scp_status scp_batch_destroy(scp_batch h);

#ifdef __cplusplus
}
#endif
#endif /* SCP_BATCH_H */
