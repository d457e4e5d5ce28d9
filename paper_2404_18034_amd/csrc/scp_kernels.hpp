// scp_kernels.hpp -- launch interface between the C ABI layer and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scp {

// Device workspace carved by the host (all pointers device-resident).  R-typed regions are
// allocated for the dtype of the handle; the blocks of one interval are stored column by
// column, 23 columns [A^- | B^- | B^+] of 16 entries (15 rows + 1 pad).
struct Workspace {
    void *blocks;       // R  [B][kmax-1][15 + 2 nu][16]  scaled A^-_k, B^-_k, B^+_k
    void *what;         // R  [B][kmax-1][16]      scaled defect w^_k
    double *dy;         // f64 [B][kmax-1]          CTCS increment y^k(tau_k+1) - y_k
    void *mup;          // R  [B][kmax-1][16]      warm start mu+
    void *mum;          // R  [B][kmax-1][16]      warm start mu-
    void *phi;          // R  [B][kmax-1][16]      warm start dual of the dynamics
    void *th;           // R  [B][kmax]            warm start dual of the CTCS rows
    double *step;       // f64 [B]                  scaled step of the last subproblem
    double *sigma;      // f64 [B]                  buffered spectral estimate of the subproblem
    void *stepsz;       // R  [B][2]                PIPG step sizes (alpha, beta) of the subproblem
    int32_t *pipg_total;// i32 [B]
    int32_t *queue;     // i32 [scp_iters_max + 2]  work-queue heads (persistent form)
    int32_t *bucket;    // i32 [kmax + 1]           node-count buckets
    int32_t *order;     // i32 [B]                  instances by node count, descending
};

struct Config {
    int dtype;          // 0 float, 1 double
    int B, kmax;
    int scp_iters_max, pipg_iters_max, pipg_check_every, rk4_substeps, power_iters_max;
    int early_exit, node_projections;
    int persistent_blocks;  // 0: one workgroup per instance; > 0: persistent grid size
    int ordered;            // 1: workgroups take instances by node count, descending
    int bucketed;           // 1 (with ordered): instances with K <= 20 solved by the 320-lane
                            //   subproblem kernel, the others by the k_max-sized one
    hipStream_t aux_stream; // bucketed: the 320-lane launch runs on this stream, forked from
    hipEvent_t ev_fork;     //   and joined back to the launch stream by these two events
    hipEvent_t ev_join;     //   (null: both launches on the launch stream, one after the other)
    int occupancy;          // 4 / 5: FP32 subproblem variant bounded to 4 / 5 waves per SIMD
    int grad_rk4_tangent;   // 1: the gradient takes the RK4 share by forward tangents
    int scalar_dilation;    // 1: one dilation value over the horizon (PIPG projects the
                            //   dilation controls of all nodes onto their mean)
    int power_fp32;         // 1 (FP32 path): power iteration in FP32 instead of FP64
    int nu;                 // controls per node: 4 (T, s) or 7 (T, gamma, s)
    double scp_tol, feas_tol, pipg_eps_abs, pipg_eps_rel;
    double power_eps_abs, power_eps_rel, power_buff;
    double w_cost, w_prox, w_ep, omega, rho;
    double px[15], pu[7];   // pu: the first nu entries
};

struct Problem {
    const void *x0, *xf, *params;
    const int32_t *K;
    const void *x_init = nullptr, *u_init = nullptr;  // optional first reference
};

struct Solution {
    void *x, *u, *t_f, *m_f;
    int32_t *status, *scp_iters, *pipg_iters;
    double *defect_inf, *ctcs_viol, *objective;
};

// Starting point of a subproblem, recorded by a solve and consumed by the gradient: the
// reference (x^, u^ are zero there), the warm-start duals and the buffered spectral estimate.
// Dense layouts: xbar [B][kmax][15], ubar [B][kmax][4], mup/mum/phi [B][kmax-1][15],
// th [B][kmax-1] (R-typed), sigma [B] (double).
struct Record {
    void *xbar, *ubar, *mup, *mum, *phi, *th;
    double *sigma;
};

// Device scratch of the gradient (carved by the host when gradients are enabled).
struct GradWorkspace {
    void *dblk;      // R [B][kmax-1][2][23][16]  tangents of the scaled blocks along
                     //   (alpha_mdot, T_max), or (first half) the adjoint of the blocks
    void *dwhat;     // R [B][kmax-1][2][16]      likewise for the scaled defect
    void *tape;      // R [B][n_ckpt + ckpt][grad_state_len(kmax)]  checkpoints and segment
    int32_t *gstat;  // i32 [B] -1 for a valid instance, 3 otherwise
    double *pbar;    // f64 [B][kmax-1][2] RK4 share of d/d(alpha_mdot, T_max) per interval
};

// Optional per-launch timing: when `events` is non-null, launch i is bracketed by
// events[2i] and events[2i+1] (recorded on `stream`) and kinds[i] receives its kernel class
// (0 init, 1 discretize, 2 subproblem PIPG, 3 preparation: convergence test and power
// iteration); *n_launches receives the number of launches.
struct LaunchTimer {
    hipEvent_t *events;
    int *kinds;
    int capacity;
    int n_launches;
};

// Enqueue one whole solve on `stream`; returns the first HIP error met while launching.
// With `rec` non-null every subproblem writes its starting point there (the last one
// solved by each instance remains).
hipError_t launch_solve(const Config &cfg, const Problem &prob, const Solution &sol,
                        const Workspace &ws, const Record *rec, hipStream_t stream,
                        LaunchTimer *timer);

// Discretization at the reference (x, u) into ws.blocks / ws.what / ws.dy for every
// instance whose status entry is negative.
hipError_t launch_discretize_at(const Config &cfg, const void *x, const void *u,
                                const Problem &prob, const int32_t *status, const Workspace &ws,
                                hipStream_t stream);

// Multi-start selection: the solution `in` holds problems * starts instances, the starts of
// problem p at p*starts .. p*starts + starts - 1.  best[p] = the start with status 0 and the
// smallest objective (ties: the smallest index), -1 if none converged; `out` (problems
// instances) receives that start's results, start 0's when none converged.
hipError_t launch_select_best(int dtype, int kmax, int nu, const Solution &in,
                              const Solution &out, int problems, int starts, int32_t *best,
                              hipStream_t stream);

// Gradient of (m_f, t_f) of the truncated last-iteration map (discretization at the
// recorded reference, QP build, `nsteps` PIPG steps from the recorded warm start) with
// respect to theta = (x0[15], m_wet, alpha_mdot, T_max), contracted with the cotangent
// cot [B][2]: grad [B][18] = cot_m dm_f/dtheta + cot_t dt_f/dtheta.  fval [B][2] (optional)
// receives (m_f, t_f) of the map.  Checkpoints every `ckpt` steps.
hipError_t launch_grad(const Config &cfg, int nsteps, int ckpt, const Problem &prob,
                       const Record &rec, const void *cot, void *grad, void *fval,
                       const Workspace &ws, const GradWorkspace &gw, hipStream_t stream);

// Values per instance of one saved PIPG state in the gradient tape.
int grad_state_len(int kmax);

// LDS bytes of the gradient kernel (0 if it does not fit a workgroup).
size_t grad_smem_bytes(int dtype, int kmax);

// Workgroup size of the subproblem kernel for node count kmax.
int qp_block_threads(int kmax);
// dynamic LDS bytes of one subproblem workgroup (rsize = 4 for FP32, 8 for FP64)
size_t qp_smem_bytes(int kmax, size_t rsize);

// Resident workgroups per compute unit of the persistent subproblem kernel (occupancy query).
int qp_blocks_per_cu(int dtype, int kmax, int nu);

// Bytes of the library's fixed device scratch array (the workspace of the allocation-free
// solve).
constexpr size_t SCRATCH_BYTES = size_t(64) << 20;

// Device address of the fixed scratch array on `device`, which must be the current device.
// Looked up once per device (the array's name is a host-side stand-in, not an address) and
// kept until the process ends.
hipError_t scratch_address(int device, void **out);

}  // namespace scp
