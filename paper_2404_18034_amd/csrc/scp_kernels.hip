// scp_kernels.hip -- HIP kernels of the batched prox-linear SCP solver for gfx950.
//
// One SCP iteration is three launches:
//   discretize_kernel  one lane per (instance, interval, column of [A | B- | B+]): RK4 on the
//                      state and on one column of the variational equations (section
//                      "Gradient of Discretized Dynamics"), then the prescaling of that
//                      column (subsection "Convex Subproblem with Prescaling and
//                      Preconditioning"); separate state lanes, one per interval, write the
//                      scaled defect w^_k, the CTCS increment and the y column of A^- (e_y:
//                      no entry of f reads y, so that column is not integrated).
//   prepare_kernel     one workgroup per instance, one 16-lane row per node: convergence
//                      test of the current reference and the customized power iteration
//                      (FP64), which sets the PIPG step sizes.
//   subproblem_kernel  one workgroup per instance, one 16-lane row per node: PIPG_custom
//                      with its projections and stopping rule, and the reference update.  The instance's blocks stay in registers for all
//                      PIPG iterations; products inside an interval use DPP row
//                      broadcasts, and only values exchanged between neighbouring nodes
//                      pass through LDS.
// Per-instance results never depend on other instances, and every reduction has a fixed
// order, so repeated runs are bitwise identical.
#include <math.h>

#include <mutex>
#include <type_traits>
#include <utility>

#include "lander_model.hpp"
#include "scp_common.hpp"
#include "scp_dpp.hpp"
#include "scp_kernels.hpp"

namespace scp {

template <typename R>
struct Args {
    int B, kmax, j;  // j: 1-based SCP iteration of this launch
    int scp_iters_max, pipg_iters_max, pipg_check_every, rk4_substeps, power_iters_max;
    int early_exit, node_projections;
    int scalar_dilation;  // 1: one dilation value over the horizon
    double scp_tol, feas_tol, pipg_eps_abs, pipg_eps_rel;
    double power_eps_abs, power_eps_rel, power_buff;
    double w_cost, w_prox, w_ep, omega, rho;
    double px[NX], pu[NU_MAX];
    double ipx[NX];  // 1 / px
    const R *x0, *xf, *params;
    const R *x_init, *u_init;  // optional first reference ([B][kmax][NX], [B][kmax][NUC])
    const int32_t *K;
    R *x, *u, *t_f, *m_f;
    int32_t *status, *scp_iters, *pipg_iters;
    double *defect_inf, *ctcs_viol, *objective;
    R *blocks, *what, *mup, *mum, *phi, *th;
    double *dy, *step;
    double *sigma;    // [B] buffered power-iteration estimate of the current subproblem
    R *stepsz;        // [B][2] PIPG step sizes (alpha, beta) of the current subproblem
    // PIPG weights in the working precision (kernel arguments, so scalar registers)
    R rho_r, wprox_r, wep_r;
    int32_t *pipg_total;
    int32_t *queue;   // [scp_iters_max + 2] work-queue heads (persistent form)
    int32_t *bucket;  // [kmax + 1] counting-sort buckets
    int32_t *order;   // [B] instances by node count, descending
    int use_order;    // subproblem workgroup w solves instance order[w]
    int split;        // 0: every instance; K-bucketed launches: 1 K > 20, 2 12 < K <= 20, 3 the rest
    // optional record of each subproblem's starting point (the last one solved remains):
    // reference [B][kmax][15], [B][kmax][4]; warm-start duals [B][kmax-1][15], [B][kmax-1];
    // buffered power-iteration estimate [B]
    R *rec_x, *rec_u, *rec_mup, *rec_mum, *rec_phi, *rec_th;
    double *rec_sigma;
};

// ------------------------------------------------------------------------------------------
// Initial guess (straight-line interpolation of r, v, w, normalized interpolation of q,
// constant mass, hover thrust along the body axis, s = s_init) and state reset.
// ------------------------------------------------------------------------------------------
template <typename R, int NUC = NU>
__global__ void __launch_bounds__(256) init_kernel(Args<R> a)
{
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int b = (int)(gid / a.kmax), k = (int)(gid % a.kmax);
    if (b >= a.B) return;
    const int K = a.K[b];
    const bool valid = K >= 2 && K <= a.kmax;
    R *x = a.x + ((long)b * a.kmax + k) * NX;
    R *u = a.u + ((long)b * a.kmax + k) * NUC;
    if (k < a.kmax - 1) {
        const long o = ((long)b * (a.kmax - 1) + k) * DST;
        for (int i = 0; i < DST; ++i) a.mup[o + i] = a.mum[o + i] = a.phi[o + i] = R(0);
    }
    a.th[(long)b * a.kmax + k] = R(0);
    if (b == 0) {
        for (int q = k; q < a.scp_iters_max + 2; q += a.kmax) a.queue[q] = 0;
        for (int q = k; q <= a.kmax; q += a.kmax) a.bucket[q] = 0;
    }
    if (k == 0) {
        a.status[b] = valid ? -1 : 3;
        a.scp_iters[b] = 0;
        a.pipg_iters[b] = 0;
        a.pipg_total[b] = 0;
        a.step[b] = INFINITY;
        if (!valid) {
            a.t_f[b] = R(0);
            a.m_f[b] = R(0);
            a.defect_inf[b] = 0.0;
            a.ctcs_viol[b] = 0.0;
            a.objective[b] = 0.0;
        }
    }
    if (!valid || k >= K) {
        for (int i = 0; i < NX; ++i) x[i] = R(0);
        for (int i = 0; i < NUC; ++i) u[i] = R(0);
        return;
    }
    const R *x0 = a.x0 + (long)b * NX, *xf = a.xf + (long)b * NXF, *p = a.params + (long)b * NP;
    const double al = (double)k / (K - 1), be = 1.0 - al;
    double xd[NX];
    xd[0] = double(x0[0]);
    for (int i = 1; i < 14; ++i) xd[i] = be * double(x0[i]) + al * double(xf[i - 1]);
    double qn = 0.0;
    for (int i = 7; i < 11; ++i) qn += xd[i] * xd[i];
    qn = sqrt(qn);
    for (int i = 7; i < 11; ++i) xd[i] /= qn;
    xd[IY] = 0.0;
    for (int i = 0; i < NX; ++i) x[i] = R(xd[i]);
    const double g0 = p[3], g1 = p[4], g2 = p[5];
    for (int i = 1; i < NUC - 1; ++i) u[i] = R(0);  // the torque guess is zero
    u[0] = R(double(x0[0]) * sqrt(g0 * g0 + g1 * g1 + g2 * g2));
    u[NUC - 1] = p[21];
    // a caller-supplied first reference replaces the guess on the instance's nodes
    if (a.x_init) {
        const R *xi = a.x_init + ((long)b * a.kmax + k) * NX;
        for (int i = 0; i < NX; ++i) x[i] = xi[i];
    }
    if (a.u_init) {
        const R *ui = a.u_init + ((long)b * a.kmax + k) * NUC;
        for (int i = 0; i < NUC; ++i) u[i] = ui[i];
    }
}

// ------------------------------------------------------------------------------------------
// Discretization over interval k with rk4_substeps RK4 steps, in two kinds of workgroup.
// Column workgroups (the first `col_blocks`): lane (b, k, c) integrates x and column c of
// [Phi_x | Phi_u- | Phi_u+] in the working precision R and writes the prescaled column.
// State workgroups (the rest): lane (b, k) integrates x alone with the state accumulated in
// double (the model still in R), which keeps the propagated endpoint -- and so the defect
// w^_k and the CTCS increment it writes -- free of R-rounding accumulated over the RK4
// stages.  In FP32 the columns thus linearize along an FP32 copy of the state (a relative
// difference of order 1e-7 in the linearization point), and the column lanes carry no FP64
// arithmetic.  Every lane of an interval's columns integrates the same x (identical
// instruction stream, so identical bits).
// ------------------------------------------------------------------------------------------
template <typename R, int NUC = NU>
__global__ void __launch_bounds__(128) discretize_kernel(Args<R> a, int col_blocks)
{
    constexpr int BLK = Blk<NUC>::SIZE;
    // integrated columns: all but the y column of A^- (no entry of f reads y, so that column
    // of the transition matrix stays e_y; the state lane writes it)
    constexpr int ICOLS = Blk<NUC>::COLS - 1;
    const bool column = (int)blockIdx.x < col_blocks;  // uniform over the workgroup
    const long gid = (long)(column ? blockIdx.x : blockIdx.x - col_blocks) * blockDim.x + threadIdx.x;
    const long per_b = (long)(a.kmax - 1) * (column ? ICOLS : 1);
    const int b = (int)(gid / per_b);
    if (b >= a.B) return;
    const int rem = (int)(gid % per_b), k = column ? rem / ICOLS : rem;
    const int ci = column ? rem % ICOLS : 0, c = ci < IY ? ci : ci + 1;
    if (a.status[b] >= 0) return;
    const int K = a.K[b];
    if (k >= K - 1) return;

    const R *p = a.params + (long)b * NP;
    const Vehicle<R> V = load_vehicle<R>(p);
    const R *xk = a.x + ((long)b * a.kmax + k) * NX;
    const R *xk1 = xk + NX;
    const R *uk = a.u + ((long)b * a.kmax + k) * NUC;
    const R *uk1 = uk + NUC;
    R ua[NUC], ub[NUC];
    for (int i = 0; i < NUC; ++i) {
        ua[i] = uk[i];
        ub[i] = uk1[i];
    }
    // direction of the control perturbation: e_j scaled by lambda- (B- columns) or lambda+
    const int uj = c < NX ? -1 : (c - NX) % NUC;
    const bool plus = c >= NX + NUC;

    const R dtau = R(1.0 / double(K - 1));
    const R km1 = R(K - 1);
    const int nsub = a.rk4_substeps;
    const R h = dtau / R(nsub);
    const R hh = R(0.5) * h;
    const R h6 = h / R(6);
    const long ib = (long)b * (a.kmax - 1) + k;
    R u[NUC], du[NUC], fx[NX], fc[NX];
    double fy;

    if (column) {
        R x[NX], col[NX], xin[NX], cs[NX], accx[NX], accc[NX];
        for (int i = 0; i < NX; ++i) {
            x[i] = xk[i];
            col[i] = (c < NX && i == c) ? R(1) : R(0);
        }
        for (int n = 0; n < nsub; ++n) {
            const R sig = R(n) * h;
            for (int st = 0; st < 4; ++st) {
                const R sg = st == 0 ? sig : (st == 3 ? sig + h : sig + hh);
                const R lp = sg * km1, lm = R(1) - lp;
                for (int i = 0; i < NUC; ++i) {
                    u[i] = lm * ua[i] + lp * ub[i];
                    du[i] = (i == uj) ? (plus ? lp : lm) : R(0);
                }
                f_jvp<R, true, NUC>(V, st == 0 ? x : xin, u, st == 0 ? col : cs, du, fx, fy, fc);
                const R wgt = (st == 0 || st == 3) ? R(1) : R(2);
                for (int i = 0; i < NX; ++i) {
                    accx[i] = st == 0 ? fx[i] : accx[i] + wgt * fx[i];
                    accc[i] = st == 0 ? fc[i] : accc[i] + wgt * fc[i];
                }
                if (st < 3) {
                    const R hs = st == 2 ? h : hh;
                    for (int i = 0; i < NX; ++i) {
                        xin[i] = x[i] + hs * fx[i];
                        cs[i] = col[i] + hs * fc[i];
                    }
                }
            }
            for (int i = 0; i < NX; ++i) {
                x[i] = x[i] + h6 * accx[i];
                col[i] = col[i] + h6 * accc[i];
            }
        }
        R *dst = a.blocks + ib * BLK + c * CST;
        const double pc = c < NX ? a.px[c] : a.pu[(c - NX) % NUC];
        for (int i = 0; i < NX; ++i) dst[i] = R(double(col[i]) * pc * a.ipx[i]);
        dst[NX] = R(0);
        return;
    }

    // state lane: the stage input is only taken in R (formed in double, rounded once)
    double x[NX], accx[NX];
    R xin[NX];
    for (int i = 0; i < NX; ++i) x[i] = double(xk[i]);
    const double hd = double(h), hhd = double(hh), h6d = double(h6);
    for (int n = 0; n < nsub; ++n) {
        const R sig = R(n) * h;
        for (int st = 0; st < 4; ++st) {
            const R sg = st == 0 ? sig : (st == 3 ? sig + h : sig + hh);
            const R lp = sg * km1, lm = R(1) - lp;
            for (int i = 0; i < NUC; ++i) u[i] = lm * ua[i] + lp * ub[i];
            if (st == 0)
                for (int i = 0; i < NX; ++i) xin[i] = R(x[i]);
            f_jvp<R, false, NUC>(V, xin, u, xin, u, fx, fy, fc);
            fx[IY] = R(0);  // y is advanced with the double-precision fy below
            if (st == 0) {
                for (int i = 0; i < IY; ++i) accx[i] = double(fx[i]);
                accx[IY] = fy;
            } else {
                const double wgt = st == 3 ? 1.0 : 2.0;
                for (int i = 0; i < IY; ++i) accx[i] += wgt * double(fx[i]);
                accx[IY] += wgt * fy;
            }
            if (st < 3) {
                const double hsd = st == 2 ? hd : hhd;
                for (int i = 0; i < IY; ++i) xin[i] = R(x[i] + hsd * double(fx[i]));
                xin[IY] = R(x[IY] + hsd * fy);
            }
        }
        for (int i = 0; i < NX; ++i) x[i] = x[i] + h6d * accx[i];
    }
    R *w = a.what + ib * DST;
    for (int i = 0; i < NX; ++i) w[i] = R((x[i] - double(xk1[i])) * a.ipx[i]);
    w[NX] = R(0);
    a.dy[ib] = x[IY] - double(xk[IY]);
    // the y column of the prescaled A^-: e_y, scaled as the integrated columns are
    R *ycol = a.blocks + ib * BLK + IY * CST;
    for (int i = 0; i < NX; ++i) ycol[i] = R(double(i == IY ? R(1) : R(0)) * a.px[IY] * a.ipx[i]);
    ycol[NX] = R(0);
}

// Square root and reciprocal of the generic (FP64) projection: IEEE arithmetic.  The FP32
// specialization below uses the hardware reciprocal square root (about 1 ulp).
__device__ __forceinline__ double proj_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ double proj_rcp(double x) { return 1.0 / x; }

// Node-wise convex sets, branch-free: project v = (t, z0, z1) onto the second-order cone
// {||z|| <= a t} (when `cone`), then onto the ball of radius `rad` centred at the cone's apex
// (rad = +inf for none); for a cone and a ball sharing that centre the composition is the
// projection onto their intersection.  inv1a2 = 1 / (1 + a^2).
template <typename R>
__device__ __forceinline__ void proj_cone_ball(R &t, R &z0, R &z1, bool cone, R a, R inv1a2, R rad)
{
    const R nz = proj_sqrt(z0 * z0 + z1 * z1);
    const bool inside = !cone || nz <= a * t;
    const bool polar = a * nz <= -t;
    const R tp = (t + a * nz) * inv1a2;
    const R zs = nz > R(0) ? a * tp * proj_rcp(nz) : R(0);
    const R t1 = inside ? t : (polar ? R(0) : tp);
    const R s1 = inside ? R(1) : (polar ? R(0) : zs);
    const R a0 = z0 * s1, a1 = z1 * s1;
    const R n = proj_sqrt(t1 * t1 + a0 * a0 + a1 * a1);
    const R bs = n > rad ? rad * proj_rcp(n) : R(1);
    t = t1 * bs;
    z0 = a0 * bs;
    z1 = a1 * bs;
}
// FP32: one reciprocal square root per norm (v_rsq_f32) gives both the norm and its inverse.
// A bias of 1e-30 under the first root keeps it finite at z = 0 (its relative effect on a norm
// is below 1e-30 / ||z||^2).  Outside the cone the projected t is (t + a ||z||) / (1 + a^2),
// clamped at zero, which also covers the polar cone; the ball scale is min(1, rad / ||.||).
template <>
__device__ __forceinline__ void proj_cone_ball<float>(float &t, float &z0, float &z1, bool cone,
                                                      float a, float inv1a2, float rad)
{
    const float s2 = fmaf(z0, z0, fmaf(z1, z1, 1e-30f));
    const float rs = __builtin_amdgcn_rsqf(s2);
    const float nz = s2 * rs;
    const bool inside = !cone || nz <= a * t;
    const float tp = fmaxf((t + a * nz) * inv1a2, 0.0f);
    const float t1 = inside ? t : tp;
    const float s1 = inside ? 1.0f : a * tp * rs;
    const float n2 = fmaf(t1, t1, (s1 * s1) * s2);
    const float bs = fminf(1.0f, rad * __builtin_amdgcn_rsqf(n2));
    const float sb = s1 * bs;
    t = t1 * bs;
    z0 = z0 * sb;
    z1 = z1 * sb;
}

// Column i of A^-_k for the transposed product.  FP32: a per-lane LDS slot of 20 floats
// (80 bytes), read back in two halves of two 16-byte loads each, one half per part of the
// product (at that stride eight consecutive lanes cover all 32 banks once); keeping these 15
// values out of registers is what lets four 5-wave workgroups share a CU.  FP64: registers.
template <typename R> struct ColStore;
template <>
struct ColStore<float> {
    static constexpr int LDS_STRIDE = 20;
    float *slot;
    __device__ __forceinline__ void put(int q, float v) { slot[q] = v; }
    // entries 0..7 and 8..15
    __device__ __forceinline__ void get_lo(float (&c)[8]) const
    {
        const float4 *p = reinterpret_cast<const float4 *>(slot);
        float4 *o = reinterpret_cast<float4 *>(c);
        o[0] = p[0];
        o[1] = p[1];
    }
    __device__ __forceinline__ void get_hi(float (&c)[8]) const
    {
        const float4 *p = reinterpret_cast<const float4 *>(slot);
        float4 *o = reinterpret_cast<float4 *>(c);
        o[0] = p[2];
        o[1] = p[3];
    }
};
// the same column kept in registers (the preparation kernel's FP32 thrust-only form)
template <typename R>
struct ColRegs {
    R *unused;
    R c[16];
    __device__ __forceinline__ void put(int q, R v) { c[q] = v; }
    __device__ __forceinline__ void get_lo(R (&o)[8]) const
    {
        for (int q = 0; q < 8; ++q) o[q] = c[q];
    }
    __device__ __forceinline__ void get_hi(R (&o)[8]) const
    {
        for (int q = 0; q < 8; ++q) o[q] = c[8 + q];
    }
};
template <>
struct ColStore<double> {
    static constexpr int LDS_STRIDE = 0;
    double *unused;
    double c[16];
    __device__ __forceinline__ void put(int q, double v) { c[q] = v; }
    __device__ __forceinline__ void get_lo(double (&o)[8]) const
    {
        for (int q = 0; q < 8; ++q) o[q] = c[q];
    }
    __device__ __forceinline__ void get_hi(double (&o)[8]) const
    {
        for (int q = 0; q < 8; ++q) o[q] = c[8 + q];
    }
};

// FP64 subproblem kernel of 512 lanes (K = 21..32): the column in LDS, transposed ([16][MAXT]:
// entry q of every lane's column in one row, so that an entry is read by consecutive lanes
// from consecutive 8-byte words, free of bank conflicts), which frees its 32 VGPRs for a
// second workgroup per CU (the smaller workgroups keep it in registers: measured faster)
template <int MAXT>
struct ColLdsT {
    double *slot;  // this lane's word of row 0
    __device__ __forceinline__ void put(int q, double v) { slot[q * MAXT] = v; }
    __device__ __forceinline__ void get_lo(double (&o)[8]) const
    {
        for (int q = 0; q < 8; ++q) o[q] = slot[q * MAXT];
    }
    __device__ __forceinline__ void get_hi(double (&o)[8]) const
    {
        for (int q = 0; q < 8; ++q) o[q] = slot[(8 + q) * MAXT];
    }
};
template <typename R, int MAXT>
constexpr bool col_in_lds_t = sizeof(R) == 8 && MAXT == 512;

// Exchange arrays of the PIPG iteration for a workgroup of at most MAXT lanes, one value per
// lane (row stride 16), so that every access of the iteration is this lane's slot or a slot
// of the row above or below, at a compile-time offset from a per-lane address register:
// the duals (phi on lanes 0..14, -theta on lane 15; rows -1 .. ROWS-1, row -1 zero), the
// extrapolated primal values 2x^ - x~ and 2u^ - u~ (rows 0 .. ROWS, the row after the last
// workgroup row zero).
// LEAN (no node-wise sets, no stopping test): the exchange arrays only.
template <typename R, int MAXT, bool LEAN = false>
struct QpLds {
    static constexpr int SLOTS = (MAXT / 16 + 1) * 16;
    static constexpr int PHI = 0, VX = SLOTS, VU = 2 * SLOTS;
    // previous fresh iterate (x^, u^, mu+, mu-, phi and -theta), this lane's slot only
    static constexpr int PX = 3 * SLOTS, PU = 4 * SLOTS, PMP = 5 * SLOTS, PMM = 6 * SLOTS,
                         PPH = 7 * SLOTS;
    static constexpr int ARRAYS = LEAN ? 3 : 8;
    static constexpr size_t BYTES = (ARRAYS * SLOTS * sizeof(R) + 15) / 16 * 16;
};
// workgroup size bound of the subproblem kernel variant that runs k_max nodes
__host__ __device__ inline int qp_maxt(int kmax)
{
    const int threads = (kmax + 3) / 4 * 64;
    return threads <= 320 ? 320 : (threads <= 512 ? 512 : 1024);
}
// clamp to [lo, hi] (lo <= hi), one median-of-three in FP32
__device__ __forceinline__ float clampbox(float v, float lo, float hi)
{
    return __builtin_amdgcn_fmed3f(v, lo, hi);
}
__device__ __forceinline__ double clampbox(double v, double lo, double hi)
{
    return fmin(fmax(v, lo), hi);
}
// upper bound: min(v, hi) for hi >= v or hi = 0 on the lanes it binds; FP32 as one v_min
// (fminf would canonicalize hi on every call)
__device__ __forceinline__ float upper(float v, float hi)
{
    float r;
    asm("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(v), "v"(hi));
    return r;
}
__device__ __forceinline__ double upper(double v, double hi) { return fmin(v, hi); }
// maximum over the 16 lanes of a row, on every lane (max is exact in any order)
template <typename R>
__device__ __forceinline__ R row_max(R v)
{
    v = fmax(v, dppmov<0xB1>(v));   // quad_perm [1,0,3,2]
    v = fmax(v, dppmov<0x4E>(v));   // quad_perm [2,3,0,1]
    v = fmax(v, dppmov<0x141>(v));  // row_half_mirror
    v = fmax(v, dppmov<0x140>(v));  // row_mirror
    return v;
}
// bit patterns of non-negative values, ordered as unsigned integers like the values
__device__ __forceinline__ unsigned int max_bits(float v) { return __float_as_uint(v); }
__device__ __forceinline__ unsigned long long max_bits(double v)
{
    return (unsigned long long)__double_as_longlong(v);
}
// Maximum over a wave of non-negative values, as its bit pattern.  FP32: unsigned maxima of
// the patterns (monotone for non-negative values) over the row by DPP (every lane of a row ends
// with the row's), then row 0 into row 1 and row 2 into row 3 (row_bcast:15), rows 0-1 into
// rows 2-3 (row_bcast:31): lane 63 holds the wave's.  FP64: the row maxima, then the four
// rows' through scalar registers (uniform).  Every lane of the wave must be active.
__device__ __forceinline__ double lane_value(double v, int l)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}
__device__ __forceinline__ unsigned long long wave_max_bits(double v)
{
    v = row_max<double>(v);
    return max_bits(fmax(fmax(lane_value(v, 0), lane_value(v, 16)),
                         fmax(lane_value(v, 32), lane_value(v, 48))));
}
// Four such maxima at once, added to dst[0..3] (LDS, bit patterns) by atomic maxima from the
// wave's lane 63 (`leader`).  The four DPP chains are interleaved: three instructions separate
// each result from its next read, more than the two wait states a DPP read needs.  The atomics
// complete before the block ends (the barrier after them must see them).
__device__ __forceinline__ void wave_max_to_lds(float m0, float m1, float m2, float m3,
                                                unsigned int *dst, bool leader)
{
    unsigned u0 = __float_as_uint(m0), u1 = __float_as_uint(m1), u2 = __float_as_uint(m2),
             u3 = __float_as_uint(m3);
#define SCP_DPP_MAX4(CTRL, MASK)                                                            \
    "v_max_u32_dpp %0, %0, %0 " CTRL " row_mask:" MASK " bank_mask:0xf\n\t"               \
    "v_max_u32_dpp %1, %1, %1 " CTRL " row_mask:" MASK " bank_mask:0xf\n\t"               \
    "v_max_u32_dpp %2, %2, %2 " CTRL " row_mask:" MASK " bank_mask:0xf\n\t"               \
    "v_max_u32_dpp %3, %3, %3 " CTRL " row_mask:" MASK " bank_mask:0xf\n\t"
    asm("s_nop 1\n\t"
        SCP_DPP_MAX4("quad_perm:[1,0,3,2]", "0xf")
        SCP_DPP_MAX4("quad_perm:[2,3,0,1]", "0xf")
        SCP_DPP_MAX4("row_half_mirror", "0xf")
        SCP_DPP_MAX4("row_mirror", "0xf")
        SCP_DPP_MAX4("row_bcast:15", "0xa")
        SCP_DPP_MAX4("row_bcast:31", "0xc")
        : "+v"(u0), "+v"(u1), "+v"(u2), "+v"(u3));
#undef SCP_DPP_MAX4
    if (leader) {
        // the low 32 bits of a generic pointer into LDS are its LDS address
        const unsigned a = (unsigned)(uintptr_t)dst;
        asm volatile("ds_max_u32 %0, %1\n\t"
                     "ds_max_u32 %0, %2 offset:4\n\t"
                     "ds_max_u32 %0, %3 offset:8\n\t"
                     "ds_max_u32 %0, %4 offset:12\n\t"
                     "s_waitcnt lgkmcnt(0)"
                     :
                     : "v"(a), "v"(u0), "v"(u1), "v"(u2), "v"(u3)
                     : "memory");
    }
}
__device__ __forceinline__ void wave_max_to_lds(double m0, double m1, double m2, double m3,
                                                unsigned long long *dst, bool)
{
    const unsigned long long w0 = wave_max_bits(m0), w1 = wave_max_bits(m1),
                             w2 = wave_max_bits(m2), w3 = wave_max_bits(m3);
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&dst[0], w0);
        atomicMax(&dst[1], w1);
        atomicMax(&dst[2], w2);
        atomicMax(&dst[3], w3);
    }
}
// max(|a|, |b|, |c|): one instruction in FP32 (the operands are finite)
__device__ __forceinline__ float absmax3(float a, float b, float c)
{
    float r;
    asm("v_max3_f32 %0, |%1|, |%2|, |%3|" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}
__device__ __forceinline__ double absmax3(double a, double b, double c)
{
    return fmax(fmax(fabs(a), fabs(b)), fabs(c));
}
__device__ __forceinline__ unsigned int uniform(unsigned int v)
{
    return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ unsigned long long uniform(unsigned long long v)
{
    return (unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(v >> 32)) << 32 |
           (unsigned)__builtin_amdgcn_readfirstlane((unsigned)v);
}
template <typename R>
__device__ __forceinline__ double from_max_bits(unsigned int b) { return double(__uint_as_float(b)); }
template <typename R>
__device__ __forceinline__ double from_max_bits(unsigned long long b)
{
    return __longlong_as_double((long long)b);
}

// ------------------------------------------------------------------------------------------
// Power-iteration products in FP64 over FP32 blocks (the FP32 path's default): each term
// widens its block entry and multiplies it by the FP64 iterate of lane L of the row, read
// through a DPP row broadcast.
// ------------------------------------------------------------------------------------------
// marks the values of c as redefined at this point (no instruction is emitted), so that a
// conversion of them is not hoisted out of the enclosing loop: widening the blocks once
// would take twice their registers
template <typename T, int N>
__device__ __forceinline__ void keep_narrow(T (&c)[N])
{
    for (int n = 0; n < N; ++n) asm volatile("" : "+v"(c[n]));
}
// sum_{j<N} c[j] * (lane J0 + S*j of this row's v), in the order j = 0, 1, ...; generic form
template <typename C, typename P, int J0, int S, int... J>
__device__ __forceinline__ P pw_dot_impl(const C *c, P v, P acc, std::integer_sequence<int, J...>)
{
    ((acc = acc + P(c[J]) * rowb<J0 + S * J>(v)), ...);
    return acc;
}
template <typename C, typename P, int J0, int S, int N>
__device__ __forceinline__ P pw_dot(const C *c, P v, P acc)
{
    if constexpr (sizeof(C) == sizeof(P)) {
        if constexpr (J0 == 0 && S == 1 && N == NX) return rowdot15<P>(c, v, acc);
        else if constexpr (J0 == 0 && S == 4 && N == NU) return rowdot4q<P>(c, v, acc);
        else if constexpr (S == 1) return rowdot_part<P, J0, N>(c, v, acc);
    }
    return pw_dot_impl<C, P, J0, S>(c, v, acc, std::make_integer_sequence<int, N>{});
}
// FP32 coefficients, FP64 iterate: one v_cvt_f64_f32 and one v_fmac_f64 with a DPP
// row_newbcast source per term (the leading s_nop covers the DPP read of v)
#define SCP_PW_TERM(T, C, L) \
    "v_cvt_f64_f32 %[" #T "], %[" #C "]\n\t" \
    "v_fmac_f64_dpp %[acc], %[v], %[" #T "] row_newbcast:" #L " row_mask:0xf bank_mask:0xf\n\t"
template <>
__device__ __forceinline__ double pw_dot<float, double, 0, 1, NX>(const float *c, double v, double acc)
{
    double t0, t1;
    asm volatile("s_nop 4\n\t"
                 SCP_PW_TERM(t0, c0, 0) SCP_PW_TERM(t1, c1, 1) SCP_PW_TERM(t0, c2, 2)
                 SCP_PW_TERM(t1, c3, 3) SCP_PW_TERM(t0, c4, 4) SCP_PW_TERM(t1, c5, 5)
                 SCP_PW_TERM(t0, c6, 6) SCP_PW_TERM(t1, c7, 7) SCP_PW_TERM(t0, c8, 8)
                 SCP_PW_TERM(t1, c9, 9) SCP_PW_TERM(t0, c10, 10) SCP_PW_TERM(t1, c11, 11)
                 SCP_PW_TERM(t0, c12, 12) SCP_PW_TERM(t1, c13, 13) SCP_PW_TERM(t0, c14, 14)
                 : [acc] "+v"(acc), [t0] "=&v"(t0), [t1] "=&v"(t1)
                 : [v] "v"(v), [c0] "v"(c[0]), [c1] "v"(c[1]), [c2] "v"(c[2]), [c3] "v"(c[3]),
                   [c4] "v"(c[4]), [c5] "v"(c[5]), [c6] "v"(c[6]), [c7] "v"(c[7]),
                   [c8] "v"(c[8]), [c9] "v"(c[9]), [c10] "v"(c[10]), [c11] "v"(c[11]),
                   [c12] "v"(c[12]), [c13] "v"(c[13]), [c14] "v"(c[14]));
    return acc;
}
template <>
__device__ __forceinline__ double pw_dot<float, double, 0, 1, 8>(const float *c, double v, double acc)
{
    double t0, t1;
    asm volatile("s_nop 4\n\t"
                 SCP_PW_TERM(t0, c0, 0) SCP_PW_TERM(t1, c1, 1) SCP_PW_TERM(t0, c2, 2)
                 SCP_PW_TERM(t1, c3, 3) SCP_PW_TERM(t0, c4, 4) SCP_PW_TERM(t1, c5, 5)
                 SCP_PW_TERM(t0, c6, 6) SCP_PW_TERM(t1, c7, 7)
                 : [acc] "+v"(acc), [t0] "=&v"(t0), [t1] "=&v"(t1)
                 : [v] "v"(v), [c0] "v"(c[0]), [c1] "v"(c[1]), [c2] "v"(c[2]), [c3] "v"(c[3]),
                   [c4] "v"(c[4]), [c5] "v"(c[5]), [c6] "v"(c[6]), [c7] "v"(c[7]));
    return acc;
}
template <>
__device__ __forceinline__ double pw_dot<float, double, 8, 1, 7>(const float *c, double v, double acc)
{
    double t0, t1;
    asm volatile("s_nop 4\n\t"
                 SCP_PW_TERM(t0, c0, 8) SCP_PW_TERM(t1, c1, 9) SCP_PW_TERM(t0, c2, 10)
                 SCP_PW_TERM(t1, c3, 11) SCP_PW_TERM(t0, c4, 12) SCP_PW_TERM(t1, c5, 13)
                 SCP_PW_TERM(t0, c6, 14)
                 : [acc] "+v"(acc), [t0] "=&v"(t0), [t1] "=&v"(t1)
                 : [v] "v"(v), [c0] "v"(c[0]), [c1] "v"(c[1]), [c2] "v"(c[2]), [c3] "v"(c[3]),
                   [c4] "v"(c[4]), [c5] "v"(c[5]), [c6] "v"(c[6]));
    return acc;
}
template <>
__device__ __forceinline__ double pw_dot<float, double, 0, 4, NU>(const float *c, double v, double acc)
{
    double t0, t1;
    asm volatile("s_nop 4\n\t"
                 SCP_PW_TERM(t0, c0, 0) SCP_PW_TERM(t1, c1, 4) SCP_PW_TERM(t0, c2, 8)
                 SCP_PW_TERM(t1, c3, 12)
                 : [acc] "+v"(acc), [t0] "=&v"(t0), [t1] "=&v"(t1)
                 : [v] "v"(v), [c0] "v"(c[0]), [c1] "v"(c[1]), [c2] "v"(c[2]), [c3] "v"(c[3]));
    return acc;
}
#undef SCP_PW_TERM

// LDS of the preparation kernel for a workgroup of at most MAXT lanes: per-lane slots, in the
// power iteration's precision R, of the power iterate (x part Z and u part U, rows 0 .. ROWS,
// the row after the last workgroup row zero) and of phi and theta (rows -1 .. ROWS-1, row -1
// zero), then the FP64 reduction scratch.
template <typename R, int MAXT>
struct PrepLds {
    static constexpr int SLOTS = (MAXT / 16 + 1) * 16;
    static constexpr int Z = 0, U = SLOTS, P = 2 * SLOTS, T = 3 * SLOTS;
    static constexpr size_t RED_BYTES = (4 * SLOTS * sizeof(R) + 15) / 16 * 16;
    static constexpr size_t BYTES = RED_BYTES + 128 * sizeof(double);
};
// sum over the 64 lanes of a wave, on every lane: row sums in the working precision
// (symmetric exchanges), then the four row sums added in FP64 in row order
template <typename R>
__device__ __forceinline__ double wave_sum(R v)
{
    v = row_allreduce<R>(v);
    auto lane = [&](int l) -> double {
        if constexpr (sizeof(R) == 4) {
            return double(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)));
        } else {
            const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
            const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
            return __hiloint2double(hi, lo);
        }
    };
    return ((lane(0) + lane(16)) + lane(32)) + lane(48);
}

// ------------------------------------------------------------------------------------------
// Preparation kernel, one workgroup per instance in the subproblem kernel's lane layout: the
// convergence test of the current reference (an instance that has finished gets its outputs
// and final status here), then the customized power iteration that bounds the spectral norm
// of the subproblem's constraint operator; the buffered estimate goes to the workspace.  It
// is a kernel of its own so that its registers (the FP64 reductions of the test, the
// power-iteration blocks) do not count against the register budget of the PIPG iteration.
// ------------------------------------------------------------------------------------------
// P: precision of the power iteration (iterate and block products); FP64 unless the FP32
// variant is selected on the FP32 path.  NUC: controls per node (4, or 7 with the torque).
template <typename R, typename P, int MAXT, int NUC = NU>
__device__ __forceinline__ void prepare_body(const Args<R> &a, const int b, unsigned char *smem_raw)
{
    constexpr int BLK = Blk<NUC>::SIZE;
    if (b >= a.B) return;
    if (a.status[b] >= 0) return;  // uniform over the workgroup
    const int K = a.K[b], M = K - 1, kmax = a.kmax;
    const int t = threadIdx.x;
    const int k = t >> 4, i = t & 15;
    const bool wact = ((t >> 6) << 2) < K;
    using Lds = PrepLds<P, MAXT>;
    P *sl = reinterpret_cast<P *>(smem_raw) + t;                            // exchange slots
    double *red = reinterpret_cast<double *>(smem_raw + Lds::RED_BYTES);  // [16 waves * 8]

    const bool node = k < K;               // row holds a node
    const bool isx = node && i < NX;       // lane holds a state variable
    const bool dual = k < M && i < NX;     // lane holds a dynamics row
    const long xoff = ((long)b * kmax + (node ? k : 0)) * NX;
    const long uoff = ((long)b * kmax + (node ? k : 0)) * NUC;
    const R *p = a.params + (long)b * NP;

    // -------------------- convergence test of the current reference --------------------
    {
        double mx[2] = {0.0, -INFINITY};
        double sm[2] = {0.0, 0.0};
        if (dual) {
            const R w = a.what[((long)b * (kmax - 1) + k) * DST + i];
            const double e = fabs(double(w));
            mx[0] = isfinite(e) ? e : INFINITY;
            sm[0] = e;
            if (i == 0) mx[1] = a.dy[(long)b * (kmax - 1) + k];
            if (!isfinite(e)) sm[1] = 1.0;
        }
        if (isx && !isfinite(double(a.x[xoff + i]))) sm[1] = 1.0;
        if (node && i < NUC && !isfinite(double(a.u[uoff + i]))) sm[1] = 1.0;
        block_reduce<2, true>(mx, red);
        block_reduce<2, false>(sm, red);
        const double d = mx[0], c = mx[1];
        const double step = a.step[b];
        const bool bad = sm[1] > 0.0 || !isfinite(d) || (a.j > 1 && !isfinite(step));
        const double eps = double(p[20]);
        const bool conv = a.j > 1 && step <= a.scp_tol && d <= a.feas_tol &&
                          (c - eps) / a.px[IY] <= a.feas_tol;
        if (bad || a.j > a.scp_iters_max || (a.early_exit && conv)) {
            if (t == 0) {
                a.status[b] = bad ? 2 : (conv ? 0 : 1);
                a.scp_iters[b] = a.j - 1;
                a.pipg_iters[b] = a.pipg_total[b];
                a.defect_inf[b] = d;
                a.ctcs_viol[b] = c;
                const double mN = double(a.x[((long)b * kmax + K - 1) * NX + 0]);
                a.objective[b] = -mN + a.w_ep * sm[0];
                double tf = 0.0;
                const double dtau = 1.0 / M;
                for (int q = 0; q < M; ++q)
                    tf += dtau * 0.5 *
                          (double(a.u[((long)b * kmax + q) * NUC + NUC - 1]) +
                           double(a.u[((long)b * kmax + q + 1) * NUC + NUC - 1]));
                a.t_f[b] = R(tf);
                a.m_f[b] = R(mN);
            }
            return;
        }
    }

    // -------------------- load the subproblem's blocks --------------------
    const R *blk = a.blocks + (long)b * (kmax - 1) * BLK;
    R rowA[NX], rowBm[NUC], rowBp[NUC], rowBq[NUC];
    // FP32 with thrust only: the column in registers (76 VGPRs, no LDS for it, so three 8-wave
    // workgroups share a CU); otherwise in LDS as in the subproblem kernel
    constexpr bool COLREG = sizeof(R) == 4 && NUC == NU;
    using ColT = std::conditional_t<COLREG, ColRegs<R>, ColStore<R>>;
    ColT colA{reinterpret_cast<R *>(smem_raw + Lds::BYTES) + t * ColStore<R>::LDS_STRIDE};
    // colA: column i of A^-_k (transposed product); row*: row i of [A^-_k | B^-_k | B^+_k]
    // (forward product); rowBq: row i of B^+_{k-1} (control part of the transposed product)
    for (int q = 0; q < NX; ++q) {
        colA.put(q, dual ? blk[(long)k * BLK + i * CST + q] : R(0));
        rowA[q] = dual ? blk[(long)k * BLK + q * CST + i] : R(0);
    }
    for (int q = 0; q < NUC; ++q) {
        rowBm[q] = dual ? blk[(long)k * BLK + (NX + q) * CST + i] : R(0);
        rowBp[q] = dual ? blk[(long)k * BLK + (NX + NUC + q) * CST + i] : R(0);
        rowBq[q] = (node && k > 0 && i < NX) ? blk[(long)(k - 1) * BLK + (NX + NUC + q) * CST + i]
                                             : R(0);
    }
    // with the torque (NUC = 7) the controls of node k sit as in the subproblem kernel: lane i
    // holds component ci = (i & 3) + 4 (i >> 3) (component 7 is padding), read copies on lanes
    // 4..7 (components 0..3) and 8..10 (4..6); the transposed product gathers them by two
    // interleaved reduce-scatters, whose addends are the B entries in exchange order
    const int ci = (i & 3) + ((i >> 3) << 2);
    const bool uval = node && (NUC == NU || ci < NUC);  // lane holds a control component
    R rowBmXA[4], rowBqXA[4], rowBmXB[4], rowBqXB[4];
    if constexpr (NUC == NU_MAX) {
        for (int s = 0; s < 4; ++s) {
            const int qa = xpermi(i, s), qb = 4 + xpermi(i, s);
            const bool bq = node && k > 0 && i < NX;
            rowBmXA[s] = dual ? blk[(long)k * BLK + (NX + qa) * CST + i] : R(0);
            rowBqXA[s] = bq ? blk[(long)(k - 1) * BLK + (NX + NUC + qa) * CST + i] : R(0);
            rowBmXB[s] = (dual && qb < NUC) ? blk[(long)k * BLK + (NX + qb) * CST + i] : R(0);
            rowBqXB[s] = (bq && qb < NUC) ? blk[(long)(k - 1) * BLK + (NX + NUC + qb) * CST + i]
                                          : R(0);
        }
    }

    // -------------------- customized power iteration --------------------
    // z = (x, u, mu+, mu-) starts at all ones: x_k on lane i of row k, u_k[q] on lanes
    // 4q..4q+3 of row k, mu+- of dynamics row (k, i) on the dual lanes.  Each step forms
    // phi = H z / sigma (dynamics rows; theta for the CTCS rows) and z' = H^T phi, where
    // mu+' = phi and mu-' = -phi; the block products use row broadcasts of the iterate, the
    // neighbouring rows pass through this lane's LDS slots.  Two barriers per step.  The
    // iterate and the products are in P (FP64 by default: the blocks are widened term by
    // term); the squared norm is summed over each row in P and over the rows in FP64; sigma
    // and the stopping test are FP64.  Each step takes sqrt and 1/sqrt of the squared norm from
    // the hardware reciprocal square root refined by two Newton steps (a few ulp, about a third
    // of the instructions of a correctly rounded square root and division); 1/sigma multiplies.
    const int KR = (kmax + 3) / 4 * 4;
    const bool thlane = dual && i == IY;
    P zx = isx ? P(1) : P(0), zu = uval ? P(1) : P(0);
    P dmu = P(0);  // mu+ - mu- of this dynamics row
    double sigma, isig;
    {
        double acc[1] = {(isx ? 1.0 : 0.0) + ((node && i < NUC) ? 1.0 : 0.0) + (dual ? 2.0 : 0.0)};
        block_reduce<1, false>(acc, red);
        sigma = sqrt(acc[0]);
        isig = 1.0 / sigma;
    }
    sl[Lds::Z] = zx;
    sl[Lds::U] = zu;
    if (t < 16) {
        sl[Lds::Z + KR * 16] = P(0);  // row after the last workgroup row
        sl[Lds::U + KR * 16] = P(0);
        sl[Lds::P] = P(0);            // row -1
        sl[Lds::T] = P(0);
    }
    __syncthreads();
    double sstar = sigma;
    const int nw = (blockDim.x + 63) >> 6;
    for (int it = 1; it <= a.power_iters_max; ++it) {
        if constexpr (sizeof(R) < sizeof(P)) {
            keep_narrow(rowA);
            keep_narrow(rowBm);
            keep_narrow(rowBp);
            keep_narrow(rowBq);
            if constexpr (NUC == NU_MAX) {
                keep_narrow(rowBmXA);
                keep_narrow(rowBqXA);
                keep_narrow(rowBmXB);
                keep_narrow(rowBqXB);
            }
        }
        P ph = P(0), thv = P(0);
        if (wact) {
            // A^-_k z_k - z_{k+1} + B^-_k u_k + B^+_k u_{k+1} + (mu+ - mu-), divided by sigma
            const P zxn = sl[Lds::Z + 16], zun = sl[Lds::U + 16];
            P r = pw_dot<R, P, 0, 1, NX>(rowA, zx, P(0));
            r -= zxn;
            if constexpr (NUC == NU) {
                r = pw_dot<R, P, 0, 4, NU>(rowBm, zu, r);
                r = pw_dot<R, P, 0, 4, NU>(rowBp, zun, r);
            } else {
                r = pw_dot<R, P, 4, 1, 4>(rowBm, zu, r);
                r = pw_dot<R, P, 8, 1, 3>(rowBm + 4, zu, r);
                r = pw_dot<R, P, 4, 1, 4>(rowBp, zun, r);
                r = pw_dot<R, P, 8, 1, 3>(rowBp + 4, zun, r);
            }
            r += dmu;
            // 1/sigma once per step (uniform), rounded to P
            const P isg = P(isig);
            ph = dual ? r * isg : P(0);
            thv = thlane ? (zxn - zx) * isg : P(0);
        }
        sl[Lds::P + 16] = ph;
        sl[Lds::T + 16] = thv;
        __syncthreads();
        P q2 = P(0);
        if (wact) {
            const P phm = sl[Lds::P], thm = sl[Lds::T];  // row k-1 (zero above node 0)
            // x part: (A^-_k)^T phi_k - phi_{k-1}, and theta_{k-1} - theta_k on the y lane
            P r;
            {
                R c[8];
                colA.get_lo(c);
                r = pw_dot<R, P, 0, 1, 8>(c, ph, P(0));
            }
            {
                R c[8];
                colA.get_hi(c);
                r = pw_dot<R, P, 8, 1, 7>(c, ph, r);
            }
            r -= phm;
            r -= thv;
            r += thm;
            zx = isx ? r : P(0);
            // u part: sum over rows i of B^-_k[i][q] phi_k[i] + B^+_{k-1}[i][q] phi_{k-1}[i]
            if constexpr (NUC == NU) {
                P gq[NU];
                for (int q = 0; q < NU; ++q) gq[q] = P(rowBm[q]) * ph + P(rowBq[q]) * phm;
                const P zq = row_reduce_scatter4<P>(gq, i);
                zu = node ? zq : P(0);
            } else {
                P ga[4], gb[4];
                for (int q = 0; q < 4; ++q) {
                    ga[q] = P(rowBmXA[q]) * ph + P(rowBqXA[q]) * phm;
                    gb[q] = P(rowBmXB[q]) * ph + P(rowBqXB[q]) * phm;
                }
                const P za = row_reduce_scatter4i<P>(ga), zb = row_reduce_scatter4i<P>(gb);
                zu = uval ? (i >= 8 ? zb : za) : P(0);
            }
            dmu = ph + ph;
            // each control component counted once: lanes 4q of the 4-copy layout, the read
            // copies of the torque layout
            const bool ucount = NUC == NU ? (i & 3) == 0 : (uval && (i >> 2) >= 1 && (i >> 2) <= 2);
            q2 = zx * zx + (ucount ? zu * zu : P(0)) + (ph * ph + ph * ph);
        }
        sl[Lds::Z] = zx;
        sl[Lds::U] = zu;
        const double wsum = wave_sum<P>(q2);
        if ((t & 63) == 0) red[t >> 6] = wsum;
        __syncthreads();
        double s2 = red[0];
        for (int w = 1; w < nw; ++w) s2 += red[w];
        // s2 > 0: the dynamics rows hold -I on x_{k+1}, so H^T is injective and z' != 0
        double y = __builtin_amdgcn_rsq(s2);  // approximate; two Newton steps reach rounding level
        for (int nwt = 0; nwt < 2; ++nwt) y = fma(0.5 * y, fma(-s2 * y, y, 1.0), y);
        sstar = s2 * y;
        if (fabs(sstar - sigma) <= a.power_eps_abs + a.power_eps_rel * fmax(sstar, sigma))
            break;
        else if (it < a.power_iters_max) {
            sigma = sstar;
            isig = y;
        }
    }
    sigma = (1.0 + a.power_buff) * sstar;
    if (t == 0) {
        a.sigma[b] = sigma;
        // PIPG step sizes from the buffered estimate
        const double alpha = 2.0 / (a.w_prox + sqrt(a.w_prox * a.w_prox + 4.0 * a.omega * sigma));
        a.stepsz[2 * b] = R(alpha);
        a.stepsz[2 * b + 1] = R(a.omega * alpha);
    }
}

// FP32: registers bounded for six waves per SIMD with thrust only (three 8-wave workgroups per
// CU), five with the torque
template <typename R, typename P, int MAXT, int NUC = NU>
__global__ void __launch_bounds__(MAXT)
    __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? (NUC == NU ? 6 : 5) : 1)))
prepare_kernel(Args<R> a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    prepare_body<R, P, MAXT, NUC>(a, blockIdx.x, smem_raw);
}

// ------------------------------------------------------------------------------------------
// Subproblem kernel: one workgroup per instance, 16 lanes (one DPP row) per node.
//   lane i of row k:  state variable (k, i) for i < 15 (primal step), dynamics row (k, i)
//                     of interval k for i < 15, k < K-1, and the CTCS row of interval k on
//                     lane 15 (dual step); each control of node k is held, bitwise
//                     identical, by four lanes of the row.
// The block products inside an interval use row broadcasts of register values (DPP);
// only the values a row needs from its neighbouring rows pass through LDS.
// ------------------------------------------------------------------------------------------
// SD: one dilation value over the horizon.  The subproblem is the per-node one restricted
// to s_1 = ... = s_K; the Euclidean projection of the fresh dilation values onto that set
// and the s box is their mean, clamped to the box (every node holds the same reference s
// and so the same box).  Each wave publishes the sum of its rows' values through LDS before
// the step's barrier; after it every lane adds the partials in wave order, so all nodes take
// a bit-identical mean, and the s lanes finish their primal update there.
// NUC: controls per node.  With the reaction-control torque (NUC = 7) lane i of a node row
// holds control component ci = (i & 3) + 4 (i >> 3) (component 7 is padding, zero): the thrust
// and the first torque component on lanes 0..7 (read copy 4..7, as with thrust alone), the rest
// of the torque and the dilation on lanes 8..15 (read copy 8..10).
// LEAN: the variant for the paper's constraint set without a PIPG stopping test (node-wise
// sets off; no early exit, or a check period beyond the iteration budget), bit for bit the
// general one there: the projection and stopping-test code and their LDS slots are compiled
// out, which takes the FP32 kernel from 95 to 79 VGPRs and its LDS from 59 to 48 KB at
// K = 30, three workgroups per CU instead of two.
template <typename R, int MAXT, bool FAIR = false, bool SD = false, int NUC = NU,
          int LEAN = 0>
__device__ __forceinline__ void subproblem_body(const Args<R> &a, const int b,
                                                unsigned char *smem_raw)
{
    static_assert(NUC == NU || !SD, "one dilation value with thrust and dilation only");
    constexpr int BLK = Blk<NUC>::SIZE;
    if (b >= a.B) return;
    if (a.status[b] >= 0) return;  // uniform over the workgroup
    const int K = a.K[b], M = K - 1, kmax = a.kmax;
    const int t = threadIdx.x;
    const int k = t >> 4, i = t & 15;
    // waves whose four rows all lie beyond the instance's last node skip the arithmetic
    // (they only take part in the barriers)
    const bool wact = ((t >> 6) << 2) < K;

    // LDS: the PIPG exchange arrays at fixed offsets, the reduction scratch, the column slots
    using Lds = QpLds<R, MAXT, (LEAN > 0)>;
    const int KR = blockDim.x >> 4;  // rows of this workgroup (a multiple of 4)
    double *red = reinterpret_cast<double *>(smem_raw + Lds::BYTES);  // [16 waves * 8]
    // stopping-test maxima: two sets of six bit patterns (32-bit for FP32, 64-bit for FP64)
    using Bits = decltype(max_bits(R(0)));
    Bits *chk = reinterpret_cast<Bits *>(red + 128);               // [2][8]
    // the column of A^-: FP32 [KR * 16][20]; FP64 at 512 lanes [16][MAXT]
    R *myCol = reinterpret_cast<R *>(red + 144) +
               (col_in_lds_t<R, MAXT> ? t : t * ColStore<R>::LDS_STRIDE);
    // SD: partial sums of the fresh dilation values, one per wave (the reduction scratch is
    // idle during PIPG)
    R *sdil = reinterpret_cast<R *>(red);  // [KR / 4]
    const R invK = R(1.0 / K);

    const bool node = k < K;               // row holds a node
    const bool isx = node && i < NX;       // lane holds a state variable
    const bool dual = k < M && i < NX;     // lane holds a dynamics row
    // lane 15 of interval k holds the CTCS dual theta_k, negated, in the phi registers: its
    // constraint y^_{k+1} - y^_k <= eps^_k enters the dual step as one more row of the block
    // product (coefficient +1 on y^_k, the row's "w" the bound, y^_{k+1} from node k+1's y
    // lane) and its projection onto theta >= 0 is a bound on phi
    const bool thl = k < M && i == 15;
    const long xoff = ((long)b * kmax + (node ? k : 0)) * NX;
    const long uoff = ((long)b * kmax + (node ? k : 0)) * NUC;
    const R *p = a.params + (long)b * NP;

    // -------------------- load the subproblem into registers --------------------
    const R *blk = a.blocks + (long)b * (kmax - 1) * BLK;
    R rowA[NX], rowBm[NUC], rowBp[NUC];
    using ColT = std::conditional_t<col_in_lds_t<R, MAXT>, ColLdsT<MAXT>, ColStore<R>>;
    ColT colA{myCol};
    // colA: column i of [A^-_k ; e_y^T] (transposed product: entry 15 is the coefficient of
    // -theta_k in the y lane's gradient); row*: row i of [A^-_k | B^-_k | B^+_k] (forward
    // product; on lane 15 the CTCS row)
    for (int q = 0; q < NX; ++q) {
        colA.put(q, dual ? blk[(long)k * BLK + i * CST + q] : R(0));
        rowA[q] = dual ? blk[(long)k * BLK + q * CST + i] : ((thl && q == IY) ? R(1) : R(0));
    }
    colA.put(15, (dual && i == IY) ? R(1) : R(0));
    for (int q = 0; q < NUC; ++q) {
        rowBm[q] = dual ? blk[(long)k * BLK + (NX + q) * CST + i] : R(0);
        rowBp[q] = dual ? blk[(long)k * BLK + (NX + NUC + q) * CST + i] : R(0);
    }
    // coefficients of the control gradient (row i of B^-_k and of B^+_{k-1}) in this lane's
    // exchange order (see row_reduce_scatter4i): slot s holds control component xpermi(i, s)
    // (with the torque a second set for components 4 + xpermi(i, s))
    R rowBmX[4], rowBqX[4], rowBmY[4], rowBqY[4];
    for (int s = 0; s < 4; ++s) {
        const int q = xpermi(i, s);
        const bool bq = node && k > 0 && i < NX;
        rowBmX[s] = dual ? blk[(long)k * BLK + (NX + q) * CST + i] : R(0);
        rowBqX[s] = bq ? blk[(long)(k - 1) * BLK + (NX + NUC + q) * CST + i] : R(0);
        if constexpr (NUC == NU_MAX) {
            const int qb = 4 + q;
            rowBmY[s] = (dual && qb < NUC) ? blk[(long)k * BLK + (NX + qb) * CST + i] : R(0);
            rowBqY[s] = (bq && qb < NUC) ? blk[(long)(k - 1) * BLK + (NX + NUC + qb) * CST + i]
                                         : R(0);
        }
    }

    const double sigma = a.sigma[b];  // buffered spectral estimate (preparation kernel)

    // boundary values, bounds, reference values
    const R xb = isx ? a.x[xoff + i] : R(0);
    // control component of this lane (interleaved: lanes q, q+4, q+8, q+12 hold u_q; the
    // copy on lanes 4..7 is the one the products, the projections and the outputs use; with
    // the torque lanes 8..15 hold components 4..7 and the copy on lanes 8..10 is read)
    const int qi = NUC == NU ? (i & 3) : (i & 3) + ((i >> 3) << 2);
    const bool uval = node && qi < NUC;  // lane holds a control component
    const bool uread = uval && ((i >> 2) == 1 || (NUC == NU_MAX && (i >> 2) == 2));
    const R ubq = uval ? a.u[uoff + qi] : R(0);
    const R ub3 = node ? a.u[uoff + NUC - 1] : R(0);  // dilation of the reference
    bool fixed = false;
    R fixv = R(0);
    if (isx) {
        if (k == 0) {
            fixed = true;
            const double zi = i < IY ? double(a.x0[(long)b * NX + i]) : 0.0;
            fixv = R((zi - double(xb)) / a.px[i]);
        } else if (k == K - 1 && final_fixed(i)) {
            fixed = true;
            fixv = R((double(a.xf[(long)b * NXF + i - 1]) - double(xb)) / a.px[i]);
        }
    }
    const R slo = R((double(p[18]) - double(ub3)) / a.pu[NUC - 1]);
    const R shi = R((double(p[19]) - double(ub3)) / a.pu[NUC - 1]);
    // the row's constant: the defect w^_k on the dynamics lanes, the scaled CTCS bound
    // eps^_k = (eps - (y_{k+1} - y_k)) / p_y on lane 15
    R wk = R(0);
    if (dual) {
        wk = a.what[((long)b * (kmax - 1) + k) * DST + i];
    } else if (thl) {
        const double y0 = double(a.x[((long)b * kmax + k) * NX + IY]);
        const double y1 = double(a.x[((long)b * kmax + k + 1) * NX + IY]);
        wk = R((double(p[20]) - (y1 - y0)) / a.px[IY]);
    }

    // workgroup-uniform step sizes (from the preparation kernel) and weights: scalar registers
    const R alpha = a.stepsz[2 * b], beta = a.stepsz[2 * b + 1];
    const R rho = a.rho_r, wprox = a.wprox_r, wep = a.wep_r;
    // mu+- of lane 15 stay zero (an infinite penalty), its phi (-theta) stays <= 0
    const R wepv = thl ? R(INFINITY) : wep;
    const R phhi = thl ? R(0) : R(INFINITY);
    const R cost = (isx && k == K - 1 && i == 0) ? R(-a.w_cost) : R(0);  // e_cost = -e_m

    // -------------------- PIPG_custom --------------------
    // warm start: x^, u^ = 0; mu+-, phi, theta from the previous subproblem
    // fresh iterates (x^, u^, mu, phi, theta) double as the previous iterate of the stopping
    // test; the extrapolated ones are x~, u~, nu, varphi, vartheta.  Lanes that hold no
    // dynamics row start at zero and, with zero blocks and zero neighbour values, stay there.
    R xt = R(0), ut = R(0);  // ut: control component qi of node k
    R vphi = R(0), nup = R(0), num = R(0);  // vphi: phi_k[i], or -theta_k on lane 15
    const long doff = ((long)b * (kmax - 1) + (dual ? k : 0)) * DST + i;
    if (dual) {
        nup = a.mup[doff];
        num = a.mum[doff];
        vphi = a.phi[doff];
    } else if (thl) {
        vphi = -a.th[(long)b * kmax + k];
    }
    // this lane's exchange slots; row -1 of the duals and row KR of the extrapolated primal
    // values are zero rows.  The fresh iterate of the step before a stopping test, and of the
    // last step, goes to this lane's previous-iterate slots; they start with the warm start.
    R *sl = reinterpret_cast<R *>(smem_raw) + t;
    // -theta_{k-1} for the y lane (lane 15 of the row above), a zero slot of row -1 for the
    // other lanes (lane i's, lane 15 taking lane 14's: they stay clear of the LDS banks of the
    // y lanes' reads); y of node k+1 for lane 15 of a CTCS row (the y lane of the row below)
    const R *slth = i == IY ? sl + 1
                            : reinterpret_cast<R *>(smem_raw) + Lds::PHI + (i == 15 ? IY : i);
    const R *slv = thl ? sl - 1 : sl;
    // LEAN keeps the last step's fresh iterate in registers
    R fxh = R(0), fuh = R(0), fmup = nup, fmum = num, fph = vphi;
    if constexpr (!LEAN) {
        sl[Lds::PX] = R(0);
        sl[Lds::PU] = R(0);
        sl[Lds::PMP] = nup;
        sl[Lds::PMM] = num;
        sl[Lds::PPH] = vphi;
    }
    sl[Lds::PHI + 16] = vphi;
    sl[Lds::VX] = R(0);
    sl[Lds::VU] = R(0);
    if (t < 16) {
        reinterpret_cast<uint64_t *>(chk)[t] = 0;
        sl[Lds::PHI] = R(0);
        sl[Lds::VX + KR * 16] = R(0);
        sl[Lds::VU + KR * 16] = R(0);
    }
    if (a.rec_x) {
        if (isx) a.rec_x[xoff + i] = xb;
        if (node && i < NUC) a.rec_u[uoff + i] = a.u[uoff + i];
        if (dual) {
            const long ro = ((long)b * (kmax - 1) + k) * NX + i;
            a.rec_mup[ro] = nup;
            a.rec_mum[ro] = num;
            a.rec_phi[ro] = vphi;
        }
        if (thl) a.rec_th[(long)b * (kmax - 1) + k] = -vphi;
        if (t == 0) a.rec_sigma[b] = sigma;
    }
    __syncthreads();

    const int jmax = a.pipg_iters_max;
    const int check = LEAN == 1 ? 0 : (a.early_exit ? a.pipg_check_every : 0);
    const int pmask = LEAN ? 0 : a.node_projections;
    // state set of this lane: 1 dry mass (lane 0), 2 glide-slope cone (lanes 1-3),
    // 3 tilt disk (lanes 9-10), 4 rate ball (lanes 11-13); groups are masked by pmask
    // Each set is projected once, by its leader lane: glide slope by lane 1 (r), tilt by lane
    // 9 (q2, q3), rate by lane 11 (w), and thrust by lane 4, which with lanes 5 and 6 holds
    // the read copy of T (velocity lanes, in no state set, stand in for it during the
    // projection).  Each leader receives its members from lanes +1, +2 and the members read
    // their component back.  Members that are fixed boundary values keep them.
    int grp = 0, gw = 0;  // member group of this lane (1 mass, 2 glide, 3 tilt, 4 rate), slot
    if (isx && !fixed) {
        if (i == 0) grp = (pmask & 1) ? 1 : 0;
        else if (i <= 3) { grp = (pmask & 2) ? 2 : 0; gw = i - 1; }
        else if (i == 9 || i == 10) { grp = (pmask & 4) ? 3 : 0; gw = i - 9; }
        else if (i >= 11 && i <= 13) { grp = (pmask & 8) ? 4 : 0; gw = i - 11; }
    }
    const bool tmem = node && (pmask & 16) && i >= 4 && i <= 6;  // thrust member, slot i - 4
    if (tmem) gw = i - 4;
    const int role = (i == 1 && (pmask & 2)) ? 2 : (i == 9 && (pmask & 4)) ? 3
                   : (i == 11 && (pmask & 8)) ? 4 : (i == 4 && (pmask & 16)) ? 5 : 0;
    const R INF = R(INFINITY);
    const double tan_g = tan(double(p[15])), tan_d = tan(double(p[14]));
    const R g_a = role == 2 ? R(1.0 / tan_g) : (role == 5 ? R(tan_d) : R(0));
    const R g_inv = role == 2 ? R(1.0 / (1.0 + 1.0 / (tan_g * tan_g)))
                              : (role == 5 ? R(1.0 / (1.0 + tan_d * tan_d)) : R(1));
    // rate ball at the last node: the transverse rates are fixed boundary values, so the roll
    // rate is projected onto the ball's slice through them (radius sqrt(w_max^2 - w2^2 - w3^2),
    // zero when they alone leave the ball); the fixed members then contribute zero below
    double w_rad = double(p[17]);
    if (role == 4 && k == K - 1) {
        const double c2 = double(a.xf[(long)b * NXF + 11]), c3 = double(a.xf[(long)b * NXF + 12]);
        const double r2 = w_rad * w_rad - c2 * c2 - c3 * c3;
        w_rad = r2 > 0.0 ? sqrt(r2) : 0.0;
    }
    const R g_rad = role == 3 ? R(sqrt(0.5 * (1.0 - cos(double(p[16])))))
                              : (role == 4 ? R(w_rad) : (role == 5 ? p[13] : INF));
    const bool g_cone = role == 2 || role == 5;
    const R mdry = p[1];
    const R ipxi = R(1.0 / a.px[isx ? i : 0]);
    const bool tilt = role == 3;
    // affine map between this lane's scaled iterate and the physical value the projections
    // act on: x = x_ref + p_x x^ (state lanes), T = u_ref + p_u u^ (thrust lanes 4..6)
    const R mb = tmem ? ubq : xb;
    const R msc = tmem ? R(a.pu[qi]) : R(a.px[isx ? i : 0]);
    const R imsc = tmem ? R(1.0 / a.pu[qi]) : ipxi;
    // box applied to the fresh iterate after the set projections: fixed boundary values
    // (lo = hi), the dry-mass bound, zero on lanes without a state variable; the dilation
    // bounds on the s lanes, zero on rows without a node
    R xlo = -INF, xhi = INF, ulo = -INF, uhi = INF;
    if (!isx) xlo = xhi = R(0);
    else if (fixed) xlo = xhi = fixv;
    else if (grp == 1) xlo = (mdry - xb) * ipxi;
    if (!uval) ulo = uhi = R(0);
    else if (qi == NUC - 1) { ulo = slo; uhi = shi; }

    int iters = 0;
    int since = 0;  // steps since the last stopping test
    int cset = 0;   // stopping-test slot set of the next test
    for (int it = 1; it <= jmax; ++it) {
        ++since;
        if constexpr (FAIR) {
            // rotate the wave priority every 16 steps: the workgroups sharing a CU then take
            // turns at the head of the issue order instead of the oldest one running ahead and
            // the last one finishing alone
            switch ((it >> 4) & 3) {
            case 0: __builtin_amdgcn_s_setprio(0); break;
            case 1: __builtin_amdgcn_s_setprio(2); break;
            case 2: __builtin_amdgcn_s_setprio(1); break;
            default: __builtin_amdgcn_s_setprio(3); break;
            }
        }
        const bool test = check > 0 && since == check;
        const bool before_test = check > 1 && since == check - 1;
        // fresh iterate of this step (waves beyond the last node compute nothing and store
        // nothing: their slots keep the zeros they started with)
        R xn, un, vx, vu;
        if (wact) {
        // ---- projected gradient step on the primal variables ----
        const R phm1 = sl[Lds::PHI];    // phi_{k-1}[i] (zero row above the first node)
        const R thm1 = slth[Lds::PHI];  // -theta_{k-1} on the y lane, zero elsewhere
        // control gradient: sum over rows i of B^-_k[i][j] phi_k[i] + B^+_{k-1}[i][j] phi_{k-1}[i],
        // with the coefficients in this lane's exchange order (computed while the column of
        // A^-_k is on its way from LDS)
        {
            R gq[4];
            for (int q = 0; q < 4; ++q) gq[q] = rowBmX[q] * vphi + rowBqX[q] * phm1;
            R gs = row_reduce_scatter4i<R>(gq);
            if constexpr (NUC == NU_MAX) {
                R gy[4];
                for (int q = 0; q < 4; ++q) gy[q] = rowBmY[q] * vphi + rowBqY[q] * phm1;
                const R gsy = row_reduce_scatter4i<R>(gy);
                gs = i >= 8 ? gsy : gs;
            }
            const R gu = wprox * ut + gs;
            un = ut - alpha * gu;
        }
        // (A^-_k)^T phi_k, column i, in two halves of the column (fewer live registers); the
        // y lane also gathers -theta_k from lane 15 (the CTCS rows give it theta_{k-1} -
        // theta_k; theta is zero beyond the last interval)
        R g = wprox * xt + cost;
        {
            R c[8];
            colA.get_lo(c);
            g = rowdot_part<R, 0, 8>(c, vphi, g);
        }
        {
            R c[8];
            colA.get_hi(c);
            g = rowdot_part<R, 8, 8>(c, vphi, g);
        }
        g -= phm1;
        g -= thm1;
        xn = xt - alpha * g;
        if (pmask) {
            // every lane forms its physical value (the thrust lanes 4..6 that of their control
            // component, the others that of their state variable); each leader gathers its
            // set from itself and lanes +1, +2 (row_shl).  Every DPP exchange is evaluated by
            // all lanes before any selection (a lane-dependent condition around it would mask
            // out the lanes it reads from).
            // (members that are fixed boundary values enter as zero: see the rate ball above)
            const R s0 = (fixed && !tmem) ? R(0) : mb + msc * (tmem ? un : xn);
            const R s1 = dppmov<0x101>(s0), s2 = dppmov<0x102>(s0);
            R t0 = s0, t1 = s1;
            R t2 = tilt ? R(0) : s2;
            // glide-slope cone; tilt disk; rate ball; thrust: gimbal cone, then the ball
            // ||T|| <= T_max centred at its apex
            proj_cone_ball<R>(t0, t1, t2, g_cone, g_a, g_inv, g_rad);
            // members read their component from the leader (row_shr by their slot)
            const R t1_m1 = dppmov<0x111>(t1), t2_m2 = dppmov<0x112>(t2);
            const R o = gw == 0 ? t0 : (gw == 1 ? t1_m1 : t2_m2);
            const R v = (o - mb) * imsc;
            if (grp >= 2 && grp <= 4) xn = v;
            if (tmem) un = v;
        }
        xn = clampbox(xn, xlo, xhi);
        if constexpr (SD) {
            // the read copies of s (lane 7 of each node row) summed over the wave's four rows
            // by two butterfly exchanges (each adds the same pair on both lanes, so the wave
            // agrees bit for bit); lane 7 publishes the wave's partial.  The s lanes finish
            // their update after the barrier; their values stored here are never read.
            R sv = (node && i == 7) ? un : R(0);
            sv += __shfl_xor(sv, 16);
            sv += __shfl_xor(sv, 32);
            if ((t & 63) == 7) sdil[t >> 6] = sv;
        }
        un = clampbox(un, ulo, uhi);  // lanes without a control: ulo = uhi = 0
        // extrapolation 2z^ - z~ and relaxation z~ += rho (z^ - z~), in place
        vx = R(2) * xn - xt;
        xt += rho * (xn - xt);
        vu = R(2) * un - ut;
        if (!SD || qi != 3) ut += rho * (un - ut);
        sl[Lds::VX] = vx;
        sl[Lds::VU] = vu;
        }  // wact
        __syncthreads();
        if (wact) {
        // ---- dual (proportional-integral) step ----
        const R vnext = slv[Lds::VX + 16];  // 2x^ - x~ of node k+1 (zero beyond the last node)
        R vunext = sl[Lds::VU + 16];        // 2u^ - u~ of node k+1
        if constexpr (SD) {
            // the mean of the active waves' partials, then the box, the extrapolation and the
            // relaxation of s; every node holds the same s, so node k+1's 2u^ - u~ of s is
            // this lane's
            if (qi == 3) {
                R s = R(0);
                for (int q = 0; q < ((K + 3) >> 2); ++q) s += sdil[q];
                un = clampbox(s * invK, ulo, uhi);
                vu = R(2) * un - ut;
                ut += rho * (un - ut);
                vunext = vu;
            }
        }
        R mupn = nup - alpha * (wepv + vphi);
        R mumn = num - alpha * (wepv - vphi);
        mupn = mupn > R(0) ? mupn : R(0);
        mumn = mumn > R(0) ? mumn : R(0);
        // (2 mu+^ - nu+) - (2 mu-^ - nu-) + w^_k, then + A^-_k (2x^ - x~)_k - (2x^ - x~)_{k+1};
        // on lane 15: eps^_k + (2y^ - y~)_k - (2y^ - y~)_{k+1}
        R r = R(2) * (mupn - mumn) - (nup - num) + wk;
        r = rowdot15<R>(rowA, vx, r);
        r -= vnext;
        r = rowdot4c<R>(rowBm, vu, r);      // B^-_k (2u^ - u~)_k
        r = rowdot4c<R>(rowBp, vunext, r);  // B^+_k (2u^ - u~)_{k+1}
        if constexpr (NUC == NU_MAX) {      // torque components 1, 2 and the dilation
            r = rowdot_part<R, 8, 3>(rowBm + 4, vu, r);
            r = rowdot_part<R, 8, 3>(rowBp + 4, vunext, r);
        }
        const R phn = upper(vphi + beta * r, phhi);  // lane 15: theta >= 0
        vphi += rho * (phn - vphi);
        nup += rho * (mupn - nup);
        num += rho * (mumn - num);
        sl[Lds::PHI + 16] = vphi;
        // stopping test every `check` steps: infinity norms of (x, u, mu+, mu-) and of
        // (phi, theta) at j+1 and j and of their differences.  Lanes without a variable hold
        // zeros; the controls enter from their read copy (lanes 4..7) only, the other copies
        // are not projected.  Row maxima by DPP, then one LDS atomic max per row on the bit
        // patterns (monotone for non-negative values); the slot set alternates between tests,
        // the other set is cleared for the next one.
        if (test) {
            const bool ucopy = uread;
            const R xh = LEAN ? fxh : sl[Lds::PX], mup = LEAN ? fmup : sl[Lds::PMP];
            const R mum = LEAN ? fmum : sl[Lds::PMM];
            const R uh = ucopy ? (LEAN ? fuh : sl[Lds::PU]) : R(0), unr = ucopy ? un : R(0);
            const R ph = LEAN ? fph : sl[Lds::PPH];
            // the test takes the larger of the norms at j+1 and j, so each lane contributes
            // the larger of its two magnitudes
            const R m0 = absmax3(absmax3(absmax3(xn, unr, mupn), mumn, xh), uh, absmax3(mup, mum, R(0)));
            const R m1 = absmax3(absmax3(xn - xh, unr - uh, mupn - mup), mumn - mum, R(0));
            const R m2 = absmax3(phn, ph, R(0)), m3 = fabs(phn - ph);
            wave_max_to_lds(m0, m1, m2, m3, &chk[8 * cset], (t & 63) == 63);
            if (t == 0)
                for (int q = 0; q < 4; ++q) chk[8 * (cset ^ 1) + q] = 0;
        }
        if constexpr (LEAN) {
            if (test || before_test || it == jmax) {
                fxh = xn;
                fuh = un;
                fmup = mupn;
                fmum = mumn;
                fph = phn;
            }
        } else if (test || before_test || it == jmax) {
            sl[Lds::PX] = xn;
            sl[Lds::PU] = un;
            sl[Lds::PMP] = mupn;
            sl[Lds::PMM] = mumn;
            sl[Lds::PPH] = phn;
        }
        }  // wact
        __syncthreads();
        iters = it;
        if (test) {
            // the workgroup's norms are uniform: scalar registers
            double n[4];
            for (int q = 0; q < 4; ++q) n[q] = from_max_bits<R>(uniform(chk[8 * cset + q]));
            since = 0;
            cset ^= 1;
            if (n[1] <= a.pipg_eps_abs + a.pipg_eps_rel * n[0] &&
                n[3] <= a.pipg_eps_abs + a.pipg_eps_rel * n[2])
                break;
        }
    }

    // -------------------- reference update and warm start --------------------
    // the subproblem's solution: the fresh iterate of the last step
    if constexpr (!LEAN) {
        fxh = sl[Lds::PX];
        fuh = sl[Lds::PU];
        fmup = sl[Lds::PMP];
        fmum = sl[Lds::PMM];
        fph = sl[Lds::PPH];
    }
    const R xh = fxh, uh = fuh, mup = fmup, mum = fmum, ph = fph;
    double st[1] = {0.0};
    if (isx) {
        st[0] = fabs(double(xh));
        a.x[xoff + i] = R(double(a.x[xoff + i]) + a.px[i] * double(xh));
    }
    if (uread) {  // the read copy of the controls
        st[0] = fmax(st[0], fabs(double(uh)));
        a.u[uoff + qi] = R(double(ubq) + a.pu[qi] * double(uh));
    }
    if (dual) {
        a.mup[doff] = mup;
        a.mum[doff] = mum;
        a.phi[doff] = ph;
    } else if (thl) {
        a.th[(long)b * kmax + k] = -ph;
    }
    block_reduce<1, true>(st, red);
    if (t == 0) {
        a.step[b] = st[0];
        a.pipg_total[b] += iters;
    }
}

// ------------------------------------------------------------------------------------------

// WPE: minimum waves per SIMD the register allocation must allow (1: no constraint).
template <typename R, int MAXT, int WPE, bool SD = false, int NUC = NU, int LEAN = 0>
__global__ void __launch_bounds__(MAXT) __attribute__((amdgpu_waves_per_eu(WPE)))
subproblem_kernel(Args<R> a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    // with ordered dispatch, workgroup w takes the w-th instance by node count (descending):
    // the hardware issues workgroups as earlier ones retire, so the longest instances start
    // first and the short ones fill in behind them
    // with bucketed launches the K-descending order is cut after the instances with K > 20
    // and after those with K > 12 (the ends of the K = 21 and K = 13 buckets once the order is
    // built): the k_max-sized kernel takes the first part, the 320-lane kernel the second, the
    // 192-lane kernel the rest
    int idx = blockIdx.x;
    if (a.split) {
        const int n20 = a.kmax > 20 ? a.bucket[a.kmax - 21] : 0;
        const int n12 = a.kmax > 12 ? a.bucket[a.kmax - 13] : 0;
        const int lo = a.split == 1 ? 0 : (a.split == 2 ? n20 : n12);
        const int hi = a.split == 1 ? n20 : (a.split == 2 ? n12 : a.B);
        idx += lo;
        if (idx >= hi) return;
    }
    const int b = a.use_order ? __builtin_amdgcn_readfirstlane(a.order[idx]) : idx;
    // with four 5-wave workgroups per CU (WPE >= 6) the priority rotation keeps them abreast
    // (not in the lean variant with the stopping test: measured slower there)
    subproblem_body<R, MAXT, (WPE >= 6 && LEAN != 2), SD, NUC, LEAN>(a, b, smem_raw);
}

// Persistent form: a fixed grid whose workgroups pop instances from a queue (one int32
// counter per SCP iteration, the only atomic) in the order of `order` (node count
// descending, so the longest instances start first).  Which workgroup solves which instance
// does not change any result.
template <typename R, int MAXT, int NUC = NU>
__global__ void __launch_bounds__(MAXT) subproblem_persistent(Args<R> a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int s_next;
    if (threadIdx.x == 0) s_next = atomicAdd(&a.queue[a.j], 1);
    __syncthreads();
    int idx = s_next;
    while (idx < a.B) {
        subproblem_body<R, MAXT, false, false, NUC>(a, __builtin_amdgcn_readfirstlane(a.order[idx]),
                                                    smem_raw);
        __syncthreads();
        if (threadIdx.x == 0) s_next = atomicAdd(&a.queue[a.j], 1);
        __syncthreads();
        idx = __builtin_amdgcn_readfirstlane(s_next);
    }
}

// Order instances by node count, descending (counting sort; equal counts in any order).
template <typename R>
__global__ void order_histogram(Args<R> a)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.B) return;
    const int K = a.K[b];
    const int key = (K >= 2 && K <= a.kmax) ? a.kmax - K : a.kmax;  // invalid last
    atomicAdd(&a.bucket[key], 1);
}
template <typename R>
__global__ void order_scan(Args<R> a)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int acc = 0;
    for (int q = 0; q <= a.kmax; ++q) {
        const int c = a.bucket[q];
        a.bucket[q] = acc;
        acc += c;
    }
}
template <typename R>
__global__ void order_scatter(Args<R> a)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.B) return;
    const int K = a.K[b];
    const int key = (K >= 2 && K <= a.kmax) ? a.kmax - K : a.kmax;
    a.order[atomicAdd(&a.bucket[key], 1)] = b;
}

// ------------------------------------------------------------------------------------------
int qp_block_threads(int kmax) { return (kmax + 3) / 4 * 64; }

// dynamic LDS bytes of the subproblem kernel variant `maxt` running k_max nodes
template <bool LEAN>
static size_t qp_stage_bytes(int maxt, size_t rsize)
{
    if (rsize == 4)
        return maxt == 192 ? QpLds<float, 192, LEAN>::BYTES
             : maxt == 320 ? QpLds<float, 320, LEAN>::BYTES
             : maxt == 512 ? QpLds<float, 512, LEAN>::BYTES : QpLds<float, 1024, LEAN>::BYTES;
    return maxt == 192 ? QpLds<double, 192, LEAN>::BYTES
         : maxt == 320 ? QpLds<double, 320, LEAN>::BYTES
         : maxt == 512 ? QpLds<double, 512, LEAN>::BYTES : QpLds<double, 1024, LEAN>::BYTES;
}
static size_t qp_smem_bytes_at(int maxt, int kmax, size_t rsize, bool lean = false)
{
    const size_t KR = (size_t)(kmax + 3) / 4 * 4;
    const size_t stage = lean ? qp_stage_bytes<true>(maxt, rsize) : qp_stage_bytes<false>(maxt, rsize);
    // the column of A^-: FP32 [KR * 16][20]; FP64 [16][maxt] at 512 lanes, else registers
    const size_t col = rsize == 4 ? sizeof(float) * KR * 16 * ColStore<float>::LDS_STRIDE
                                  : (maxt == 512 ? sizeof(double) * 16 * (size_t)maxt : 0);
    return stage + sizeof(double) * 144 + col;
}
size_t qp_smem_bytes(int kmax, size_t rsize) { return qp_smem_bytes_at(qp_maxt(kmax), kmax, rsize); }
// dynamic LDS bytes of the preparation kernel (rsize: the working precision, psize: that of
// the power iteration)
static size_t prep_smem_bytes(int kmax, size_t rsize, size_t psize, int nu)
{
    const int maxt = qp_maxt(kmax);
    const size_t KR = (size_t)(kmax + 3) / 4 * 4;
    const size_t col = rsize == 4 ? ColStore<float>::LDS_STRIDE : ColStore<double>::LDS_STRIDE;
    const size_t stage = psize == 4 ? (maxt == 320 ? PrepLds<float, 320>::BYTES
                                                   : (maxt == 512 ? PrepLds<float, 512>::BYTES
                                                                  : PrepLds<float, 1024>::BYTES))
                                    : (maxt == 320 ? PrepLds<double, 320>::BYTES
                                                   : (maxt == 512 ? PrepLds<double, 512>::BYTES
                                                                  : PrepLds<double, 1024>::BYTES));
    if (rsize == 4 && nu == NU) return stage;  // the column in registers
    return stage + rsize * KR * 16 * col;
}

template <typename R, typename P, int NUC = NU>
static void launch_prepare(int maxt, int B, int threads, size_t smem, hipStream_t stream,
                           const Args<R> &a)
{
    if (maxt == 320)
        prepare_kernel<R, P, 320, NUC><<<dim3(B), dim3(threads), smem, stream>>>(a);
    else if (maxt == 512)
        prepare_kernel<R, P, 512, NUC><<<dim3(B), dim3(threads), smem, stream>>>(a);
    else
        prepare_kernel<R, P, 1024, NUC><<<dim3(B), dim3(threads), smem, stream>>>(a);
}

// Subproblem launch with the register-budget variant: occupancy 4, 5 or 6 bounds the kernel
// to that many waves per SIMD (FP32 only; FP64 always uses the compiler's choice).
template <typename R, int MAXT, int NUC, int LEAN>
static void launch_subproblem_v(int occupancy, int B, int threads, size_t smem, hipStream_t stream,
                                const Args<R> &a)
{
    if constexpr (sizeof(R) == 4) {
        if (occupancy == 6) {
            subproblem_kernel<R, MAXT, 6, false, NUC, LEAN><<<dim3(B), dim3(threads), smem, stream>>>(a);
            return;
        }
        if (occupancy == 5) {
            subproblem_kernel<R, MAXT, 5, false, NUC, LEAN><<<dim3(B), dim3(threads), smem, stream>>>(a);
            return;
        }
        if constexpr (MAXT < 1024) {
            if (occupancy == 4) {
                subproblem_kernel<R, MAXT, 4, false, NUC, LEAN>
                    <<<dim3(B), dim3(threads), smem, stream>>>(a);
                return;
            }
        }
    }
    // FP64, thrust only, 512 lanes, lean without a test: bounded for four waves per SIMD (128
    // VGPRs, a few spills; the column sits in LDS), two 8-wave workgroups per CU at K = 30
    // where the compiler's 138 VGPRs hold one
    constexpr int W64 = (sizeof(R) == 8 && LEAN == 1 && MAXT == 512 && NUC == NU) ? 4 : 1;
    subproblem_kernel<R, MAXT, W64, false, NUC, LEAN><<<dim3(B), dim3(threads), smem, stream>>>(a);
}
// smem must be the dynamic LDS of the variant launched (qp_smem_bytes_at with `lean` > 0);
// lean: 0 the general kernel, 1 the lean one without a stopping test, 2 with it (FP32,
// thrust and dilation only)
template <typename R, int MAXT, int NUC = NU>
static void launch_subproblem(int occupancy, int B, int threads, size_t smem, hipStream_t stream,
                              const Args<R> &a, int lean)
{
    if (NUC == NU && a.scalar_dilation) {
        // one variant: FP32 bounded to six waves per SIMD (with the priority rotation), FP64
        // the compiler's choice
        subproblem_kernel<R, MAXT, (sizeof(R) == 4 ? 6 : 1), true>
            <<<dim3(B), dim3(threads), smem, stream>>>(a);
        return;
    }
    if constexpr (sizeof(R) == 4 && NUC == NU) {
        if (lean == 2) {
            launch_subproblem_v<R, MAXT, NUC, 2>(occupancy, B, threads, smem, stream, a);
            return;
        }
    }
    if (lean)
        launch_subproblem_v<R, MAXT, NUC, 1>(occupancy, B, threads, smem, stream, a);
    else
        launch_subproblem_v<R, MAXT, NUC, 0>(occupancy, B, threads, smem, stream, a);
}

template <typename R, int NUC = NU>
static hipError_t launch_typed(const Config &cfg, const Problem &prob, const Solution &sol,
                               const Workspace &ws, const Record *rec, hipStream_t stream,
                               LaunchTimer *timer)
{
    Args<R> a;
    a.B = cfg.B;
    a.kmax = cfg.kmax;
    a.j = 0;
    a.scp_iters_max = cfg.scp_iters_max;
    a.pipg_iters_max = cfg.pipg_iters_max;
    a.pipg_check_every = cfg.pipg_check_every;
    a.rk4_substeps = cfg.rk4_substeps;
    a.power_iters_max = cfg.power_iters_max;
    a.early_exit = cfg.early_exit;
    a.node_projections = cfg.node_projections;
    a.scalar_dilation = cfg.scalar_dilation;
    a.scp_tol = cfg.scp_tol;
    a.feas_tol = cfg.feas_tol;
    a.pipg_eps_abs = cfg.pipg_eps_abs;
    a.pipg_eps_rel = cfg.pipg_eps_rel;
    a.power_eps_abs = cfg.power_eps_abs;
    a.power_eps_rel = cfg.power_eps_rel;
    a.power_buff = cfg.power_buff;
    a.w_cost = cfg.w_cost;
    a.w_prox = cfg.w_prox;
    a.w_ep = cfg.w_ep;
    a.omega = cfg.omega;
    a.rho = cfg.rho;
    for (int i = 0; i < NX; ++i) {
        a.px[i] = cfg.px[i];
        a.ipx[i] = 1.0 / cfg.px[i];
    }
    for (int i = 0; i < NU_MAX; ++i) a.pu[i] = i < NUC ? cfg.pu[i] : 1.0;
    a.x0 = static_cast<const R *>(prob.x0);
    a.x_init = static_cast<const R *>(prob.x_init);
    a.u_init = static_cast<const R *>(prob.u_init);
    a.xf = static_cast<const R *>(prob.xf);
    a.params = static_cast<const R *>(prob.params);
    a.K = prob.K;
    a.x = static_cast<R *>(sol.x);
    a.u = static_cast<R *>(sol.u);
    a.t_f = static_cast<R *>(sol.t_f);
    a.m_f = static_cast<R *>(sol.m_f);
    a.status = sol.status;
    a.scp_iters = sol.scp_iters;
    a.pipg_iters = sol.pipg_iters;
    a.defect_inf = sol.defect_inf;
    a.ctcs_viol = sol.ctcs_viol;
    a.objective = sol.objective;
    a.blocks = static_cast<R *>(ws.blocks);
    a.what = static_cast<R *>(ws.what);
    a.mup = static_cast<R *>(ws.mup);
    a.mum = static_cast<R *>(ws.mum);
    a.phi = static_cast<R *>(ws.phi);
    a.th = static_cast<R *>(ws.th);
    a.dy = ws.dy;
    a.step = ws.step;
    a.sigma = ws.sigma;
    a.stepsz = static_cast<R *>(ws.stepsz);
    a.rho_r = R(cfg.rho);
    a.wprox_r = R(cfg.w_prox);
    a.wep_r = R(cfg.w_ep);
    a.pipg_total = ws.pipg_total;
    a.queue = ws.queue;
    a.bucket = ws.bucket;
    a.order = ws.order;
    a.rec_x = rec ? static_cast<R *>(rec->xbar) : nullptr;
    a.rec_u = rec ? static_cast<R *>(rec->ubar) : nullptr;
    a.rec_mup = rec ? static_cast<R *>(rec->mup) : nullptr;
    a.rec_mum = rec ? static_cast<R *>(rec->mum) : nullptr;
    a.rec_phi = rec ? static_cast<R *>(rec->phi) : nullptr;
    a.rec_th = rec ? static_cast<R *>(rec->th) : nullptr;
    a.rec_sigma = rec ? rec->sigma : nullptr;

    if (cfg.B == 0) return hipSuccess;
    int nl = 0;
    auto mark = [&](int kind, bool begin) -> hipError_t {
        if (!timer || nl >= timer->capacity) return hipSuccess;
        if (begin) timer->kinds[nl] = kind;
        hipError_t e = hipEventRecord(timer->events[2 * nl + (begin ? 0 : 1)], stream);
        if (!begin) timer->n_launches = ++nl;
        return e;
    };
    hipError_t e;
    if (timer) timer->n_launches = 0;
    {
        const long n = (long)cfg.B * cfg.kmax;
        if ((e = mark(0, true)) != hipSuccess) return e;
        init_kernel<R, NUC><<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream>>>(a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = mark(0, false)) != hipSuccess) return e;
    }
    // discretization grid: column workgroups (when the blocks are needed), then state ones
    const unsigned dcol = (unsigned)(((long)cfg.B * (cfg.kmax - 1) * (Blk<NUC>::COLS - 1) + 127) / 128);
    const unsigned dstate = (unsigned)(((long)cfg.B * (cfg.kmax - 1) + 127) / 128);
    const int qthreads = qp_block_threads(cfg.kmax);
    const int maxt = qp_maxt(cfg.kmax);
    // the lean variants where the node-wise sets are off: no stopping test can fire
    // (variant 1), or where a test can fire, FP32 with thrust and dilation (variant 2)
    const bool no_test = !cfg.early_exit || cfg.pipg_check_every > cfg.pipg_iters_max;
    const int lean = (cfg.scalar_dilation || cfg.node_projections != 0) ? 0
                   : no_test ? 1 : (sizeof(R) == 4 && NUC == NU) ? 2 : 0;
    const size_t smem = qp_smem_bytes_at(maxt, cfg.kmax, sizeof(R), lean > 0);
    const size_t smem_full = qp_smem_bytes(cfg.kmax, sizeof(R));
    // power iteration in FP64 unless the FP32 variant is selected (FP32 path only)
    const bool pw32 = sizeof(R) == 4 && cfg.power_fp32;
    const size_t psmem = prep_smem_bytes(cfg.kmax, sizeof(R), pw32 ? 4 : 8, NUC);
    const bool persistent = cfg.persistent_blocks > 0;
    a.use_order = cfg.ordered ? 1 : 0;
    a.split = 0;
    const bool bucketed = cfg.bucketed && cfg.ordered && cfg.kmax > 12;
    const size_t smem20 = qp_smem_bytes_at(320, 20, sizeof(R), lean > 0);
    const size_t smem12 = qp_smem_bytes_at(192, 12, sizeof(R), lean > 0);
    if (persistent || cfg.ordered) {
        const unsigned nb = (unsigned)((cfg.B + 255) / 256);
        order_histogram<R><<<dim3(nb), dim3(256), 0, stream>>>(a);
        order_scan<R><<<dim3(1), dim3(64), 0, stream>>>(a);
        order_scatter<R><<<dim3(nb), dim3(256), 0, stream>>>(a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const unsigned pgrid = (unsigned)(cfg.persistent_blocks < cfg.B ? cfg.persistent_blocks : cfg.B);
    for (int j = 1; j <= cfg.scp_iters_max + 1; ++j) {
        a.j = j;
        // the last launch only tests the final reference: no blocks
        const unsigned ncol = j <= cfg.scp_iters_max ? dcol : 0;
        if ((e = mark(1, true)) != hipSuccess) return e;
        discretize_kernel<R, NUC><<<dim3(ncol + dstate), dim3(128), 0, stream>>>(a, (int)ncol);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = mark(1, false)) != hipSuccess) return e;
        if ((e = mark(3, true)) != hipSuccess) return e;
        if (pw32)
            launch_prepare<R, R, NUC>(maxt, cfg.B, qthreads, psmem, stream, a);
        else
            launch_prepare<R, double, NUC>(maxt, cfg.B, qthreads, psmem, stream, a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = mark(3, false)) != hipSuccess) return e;
        if (j > cfg.scp_iters_max) break;  // the last test has set every remaining status
        if ((e = mark(2, true)) != hipSuccess) return e;
        if (persistent) {
            if (maxt == 320)
                subproblem_persistent<R, 320, NUC><<<dim3(pgrid), dim3(qthreads), smem_full, stream>>>(a);
            else if (maxt == 512)
                subproblem_persistent<R, 512, NUC><<<dim3(pgrid), dim3(qthreads), smem_full, stream>>>(a);
            else
                subproblem_persistent<R, 1024, NUC><<<dim3(pgrid), dim3(qthreads), smem_full, stream>>>(a);
        } else if (bucketed) {
            // the launches touch disjoint instances; on two streams they run side by side
            hipStream_t s2 = cfg.aux_stream ? cfg.aux_stream : stream;
            if (cfg.aux_stream) {
                if ((e = hipEventRecord(cfg.ev_fork, stream)) != hipSuccess) return e;
                if ((e = hipStreamWaitEvent(s2, cfg.ev_fork, 0)) != hipSuccess) return e;
            }
            // K <= 12 in 192-lane workgroups (three waves: six of them fit a CU where the
            // 320-lane kernel holds four with two idle waves each), 12 < K <= 20 in 320-lane
            // ones, the rest in the k_max-sized kernel
            a.split = 3;
            launch_subproblem<R, 192, NUC>(cfg.occupancy, cfg.B, qp_block_threads(12), smem12, s2, a, lean);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            a.split = 2;
            if (cfg.kmax > 20) {
                launch_subproblem<R, 320, NUC>(cfg.occupancy, cfg.B, qp_block_threads(20), smem20, s2, a, lean);
                if ((e = hipGetLastError()) != hipSuccess) return e;
                a.split = 1;
                if (maxt == 512)
                    launch_subproblem<R, 512, NUC>(cfg.occupancy, cfg.B, qthreads, smem, stream, a, lean);
                else
                    launch_subproblem<R, 1024, NUC>(cfg.occupancy, cfg.B, qthreads, smem, stream, a, lean);
            } else {
                launch_subproblem<R, 320, NUC>(cfg.occupancy, cfg.B, qthreads, smem, stream, a, lean);
            }
            if ((e = hipGetLastError()) != hipSuccess) return e;
            a.split = 0;
            if (cfg.aux_stream) {
                if ((e = hipEventRecord(cfg.ev_join, s2)) != hipSuccess) return e;
                if ((e = hipStreamWaitEvent(stream, cfg.ev_join, 0)) != hipSuccess) return e;
            }
        } else if (maxt == 320) {
            launch_subproblem<R, 320, NUC>(cfg.occupancy, cfg.B, qthreads, smem, stream, a, lean);
        } else if (maxt == 512) {
            launch_subproblem<R, 512, NUC>(cfg.occupancy, cfg.B, qthreads, smem, stream, a, lean);
        } else {
            launch_subproblem<R, 1024, NUC>(cfg.occupancy, cfg.B, qthreads, smem, stream, a, lean);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = mark(2, false)) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_solve(const Config &cfg, const Problem &prob, const Solution &sol,
                        const Workspace &ws, const Record *rec, hipStream_t stream,
                        LaunchTimer *timer)
{
    if (cfg.nu == NU_MAX) {
        if (cfg.dtype == 1)
            return launch_typed<double, NU_MAX>(cfg, prob, sol, ws, rec, stream, timer);
        return launch_typed<float, NU_MAX>(cfg, prob, sol, ws, rec, stream, timer);
    }
    if (cfg.dtype == 1) return launch_typed<double>(cfg, prob, sol, ws, rec, stream, timer);
    return launch_typed<float>(cfg, prob, sol, ws, rec, stream, timer);
}

// Discretization (blocks, scaled defect, CTCS increment) at a given reference, for the
// instances whose status entry is negative.
template <typename R>
static hipError_t discretize_at_typed(const Config &cfg, const void *x, const void *u,
                                      const Problem &prob, const int32_t *status,
                                      const Workspace &ws, hipStream_t stream)
{
    Args<R> a = {};
    a.B = cfg.B;
    a.kmax = cfg.kmax;
    a.rk4_substeps = cfg.rk4_substeps;
    for (int i = 0; i < NX; ++i) {
        a.px[i] = cfg.px[i];
        a.ipx[i] = 1.0 / cfg.px[i];
    }
    for (int i = 0; i < NU_MAX; ++i) a.pu[i] = i < NU ? cfg.pu[i] : 1.0;
    a.params = static_cast<const R *>(prob.params);
    a.K = prob.K;
    a.x = const_cast<R *>(static_cast<const R *>(x));
    a.u = const_cast<R *>(static_cast<const R *>(u));
    a.status = const_cast<int32_t *>(status);
    a.blocks = static_cast<R *>(ws.blocks);
    a.what = static_cast<R *>(ws.what);
    a.dy = ws.dy;
    const unsigned ncol = (unsigned)(((long)cfg.B * (cfg.kmax - 1) * (COLS - 1) + 127) / 128);
    const unsigned nstate = (unsigned)(((long)cfg.B * (cfg.kmax - 1) + 127) / 128);
    discretize_kernel<R><<<dim3(ncol + nstate), dim3(128), 0, stream>>>(a, (int)ncol);
    return hipGetLastError();
}

hipError_t launch_discretize_at(const Config &cfg, const void *x, const void *u,
                                const Problem &prob, const int32_t *status, const Workspace &ws,
                                hipStream_t stream)
{
    if (cfg.B == 0) return hipSuccess;
    if (cfg.dtype == 1) return discretize_at_typed<double>(cfg, x, u, prob, status, ws, stream);
    return discretize_at_typed<float>(cfg, x, u, prob, status, ws, stream);
}

// ------------------------------------------------------------------------------------------
// Multi-start selection (named as future work in the paper's Conclusion): each problem is run
// from several starts and, of the starts that converge, the one of lowest cost is kept.  One 64-lane workgroup per
// problem: every lane scans the problem's starts (the same loads, so every lane reaches the
// same choice without an exchange), lane 0 writes the choice and the scalar outputs, and the
// workgroup copies the chosen trajectory.
// ------------------------------------------------------------------------------------------
template <typename R, int NUC = NU>
__global__ void __launch_bounds__(64) select_best_kernel(Solution in, Solution out, int problems,
                                                          int starts, int kmax, int32_t *best)
{
    const int p = blockIdx.x;
    if (p >= problems) return;
    int pick = -1;
    double cost = 0.0;
    for (int j = 0; j < starts; ++j) {
        const long s = (long)p * starts + j;
        if (in.status[s] == 0 && (pick < 0 || in.objective[s] < cost)) {
            pick = j;
            cost = in.objective[s];
        }
    }
    const long src = (long)p * starts + (pick < 0 ? 0 : pick);
    if (threadIdx.x == 0) {
        best[p] = pick;
        static_cast<R *>(out.t_f)[p] = static_cast<const R *>(in.t_f)[src];
        static_cast<R *>(out.m_f)[p] = static_cast<const R *>(in.m_f)[src];
        out.status[p] = in.status[src];
        out.scp_iters[p] = in.scp_iters[src];
        out.pipg_iters[p] = in.pipg_iters[src];
        out.defect_inf[p] = in.defect_inf[src];
        out.ctcs_viol[p] = in.ctcs_viol[src];
        out.objective[p] = in.objective[src];
    }
    const R *xs = static_cast<const R *>(in.x) + src * kmax * NX;
    const R *us = static_cast<const R *>(in.u) + src * kmax * NUC;
    R *xd = static_cast<R *>(out.x) + (long)p * kmax * NX;
    R *ud = static_cast<R *>(out.u) + (long)p * kmax * NUC;
    for (int e = threadIdx.x; e < kmax * NX; e += blockDim.x) xd[e] = xs[e];
    for (int e = threadIdx.x; e < kmax * NUC; e += blockDim.x) ud[e] = us[e];
}

hipError_t launch_select_best(int dtype, int kmax, int nu, const Solution &in,
                              const Solution &out, int problems, int starts, int32_t *best,
                              hipStream_t stream)
{
    if (problems == 0) return hipSuccess;
    const dim3 g((unsigned)problems), t(64);
    if (dtype == 1 && nu == NU_MAX)
        select_best_kernel<double, NU_MAX><<<g, t, 0, stream>>>(in, out, problems, starts, kmax, best);
    else if (dtype == 1)
        select_best_kernel<double><<<g, t, 0, stream>>>(in, out, problems, starts, kmax, best);
    else if (nu == NU_MAX)
        select_best_kernel<float, NU_MAX><<<g, t, 0, stream>>>(in, out, problems, starts, kmax, best);
    else
        select_best_kernel<float><<<g, t, 0, stream>>>(in, out, problems, starts, kmax, best);
    return hipGetLastError();
}

}  // namespace scp

namespace scp {
template <typename R, int MAXT, int NUC>
static hipError_t persistent_blocks(int *n, int kmax)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, subproblem_persistent<R, MAXT, NUC>,
                                                        qp_block_threads(kmax),
                                                        qp_smem_bytes(kmax, sizeof(R)));
}
template <typename R, int NUC>
static hipError_t persistent_blocks_of(int *n, int kmax)
{
    const int maxt = qp_maxt(kmax);
    return maxt == 320 ? persistent_blocks<R, 320, NUC>(n, kmax)
                       : (maxt == 512 ? persistent_blocks<R, 512, NUC>(n, kmax)
                                      : persistent_blocks<R, 1024, NUC>(n, kmax));
}
int qp_blocks_per_cu(int dtype, int kmax, int nu)
{
    int n = 0;
    hipError_t e;
    if (dtype == 1)
        e = nu == NU_MAX ? persistent_blocks_of<double, NU_MAX>(&n, kmax)
                         : persistent_blocks_of<double, NU>(&n, kmax);
    else
        e = nu == NU_MAX ? persistent_blocks_of<float, NU_MAX>(&n, kmax)
                         : persistent_blocks_of<float, NU>(&n, kmax);
    return (e == hipSuccess && n > 0) ? n : 1;
}
// ------------------------------------------------------------------------------------------
// Fixed device scratch for callers that cannot allocate device memory: every allocation-free
// solve on a device uses this one array as its workspace, so such calls that overlap on a
// device race.  Each device holds its own copy, at its own address.
// ------------------------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

hipError_t scratch_address(int device, void **out)
{
    constexpr int MAX_DEVICES = 64;
    static std::mutex mu;
    static void *addr[MAX_DEVICES] = {};
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = p;
    }
    *out = addr[device];
    return hipSuccess;
}

}  // namespace scp
