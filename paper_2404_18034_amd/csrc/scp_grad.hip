// scp_grad.hip -- derivative of the last SCP iteration with respect to the problem data.
//
// The differentiated map takes theta = (x0[15], m_wet, alpha_mdot, T_max) to (m_f, t_f) through
// one SCP iteration with its starting point frozen: the discretization at the recorded
// reference (section "Discretization", with the variational equations of "Gradient of
// Discretized Dynamics"), the prescaled QP ("Convex Subproblem with Prescaling and
// Preconditioning"), a fixed number of PIPG_custom steps (Algorithm "PIPG_custom") from the
// recorded warm start with the recorded step sizes, and the reference update.  The paper
// does not differentiate its solver; this is an extension.
//
//   grad_kernel     one workgroup per instance, one 16-lane row per node: the PIPG steps
//                   forward with a checkpoint every `ckpt` steps, then the reverse (adjoint)
//                   sweep segment by segment, each segment recomputed from its checkpoint.
//                   The adjoint accumulates the derivative of the output with respect to
//                   the scaled blocks, the defect and the initial boundary value.
//   rk4_adjoint_kernel  one 32-lane group per (instance, interval): the reverse sweep through
//                   the RK4 discretization that carries the block and defect adjoints back to
//                   alpha_mdot and T_max (the only entries of theta the discretization sees;
//                   x0 and m_wet enter through the initial boundary value alone).
//   tangent_kernel  alternative to the reverse sweep (settings.grad_rk4_tangent): the RK4 run
//                   on one-direction dual numbers along alpha_mdot, with two quadratures for
//                   T_max, gives the tangents of the blocks and defect along (alpha_mdot,
//                   T_max) in the working precision, contracted with the adjoints in
//                   grad_kernel.
// Every projection is differentiated on the branch the forward evaluation takes; a kink is
// given the derivative of that branch (the derivative of max(0, .) at 0 is that of the
// clamped side).
#include <math.h>

#include <utility>

#include "dual.hpp"
#include "lander_model.hpp"
#include "scp_common.hpp"
#include "scp_dpp.hpp"
#include "scp_kernels.hpp"

namespace scp {

// acc[q] += w * (value of lane q of this row), q < N: the broadcast form of an outer-product
// accumulation (every lane of the row must take part)
template <typename R, int... Q>
__device__ __forceinline__ void bcast_axpy_impl(R *acc, R w, R v, std::integer_sequence<int, Q...>)
{
    ((acc[Q] = acc[Q] + w * rowb<Q>(v)), ...);
}
template <typename R, int N>
__device__ __forceinline__ void bcast_axpy(R *acc, R w, R v)
{
    bcast_axpy_impl<R>(acc, w, v, std::make_integer_sequence<int, N>{});
}

// Offsets of one saved PIPG iterate (x~, u~, nu+, nu-, varphi, vartheta) in LDS and tape.
struct StateLayout {
    int X, U, MP, MM, PH, TH, len;
};

__host__ __device__ inline StateLayout state_layout(int kmax)
{
    StateLayout L;
    const int M = kmax - 1;
    L.X = 0;
    L.U = kmax * 16;
    L.MP = L.U + kmax * NU;
    L.MM = L.MP + M * DST;
    L.PH = L.MM + M * DST;
    L.TH = L.PH + M * DST;
    L.len = L.TH + kmax;
    return L;
}

int grad_state_len(int kmax) { return state_layout(kmax).len; }

template <typename R>
struct GradArgs {
    int B, kmax, nsteps, ckpt, n_ckpt, rk4_substeps, node_projections;
    double w_cost, w_prox, w_ep, omega, rho;
    double px[NX], pu[NU];
    const R *x0, *xf, *params;
    const int32_t *K;
    const R *xbar, *ubar, *mup, *mum, *phi, *th;
    const double *sigma;
    const R *cot;
    R *grad, *fval;
    const R *blocks, *what;
    R *dblk, *dwhat;
    R *tape;
    int32_t *gstat;
    int rk4_reverse;  // 1: the grad kernel leaves the block adjoints for the RK4 reverse sweep
    double *pbar;     // [B][kmax-1][2] derivative with respect to (alpha_mdot, T_max) per interval
};

__global__ void grad_status_kernel(const int32_t *K, int B, int kmax, int32_t *gstat)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const int k = K[b];
    gstat[b] = (k >= 2 && k <= kmax) ? -1 : 3;
}

// Vehicle data on dual numbers; with `params` the tangents 0 and 1 are seeded on alpha_mdot
// and T_max.
template <int N>
__device__ __forceinline__ Vehicle<Dual<double, N>> lift_vehicle(const Vehicle<double> &W,
                                                                 bool params)
{
    using D = Dual<double, N>;
    Vehicle<D> V;
    V.m_dry = D(W.m_dry);
    V.alpha = params ? seed<double, N>(W.alpha, 0, 1.0) : D(W.alpha);
    for (int q = 0; q < 3; ++q) {
        V.g[q] = D(W.g[q]);
        V.Jinv[q] = D(W.Jinv[q]);
        V.J[q] = D(W.J[q]);
        V.rT[q] = D(W.rT[q]);
    }
    V.T_min = D(W.T_min);
    V.T_max = params ? seed<double, N>(W.T_max, N > 1 ? 1 : 0, 1.0) : D(W.T_max);
    V.sec_delta = D(W.sec_delta);
    V.tan_gamma = D(W.tan_gamma);
    V.tilt_c = D(W.tilt_c);
    V.w_max2 = D(W.w_max2);
    V.v_max2 = D(W.v_max2);
    V.has_vmax = W.has_vmax;
    return V;
}

// ------------------------------------------------------------------------------------------
// Tangents of the discretization with respect to (alpha_mdot, T_max), in the working precision.
//
// alpha_mdot enters the mass rate, so it reaches the whole state and every column: the RK4
// run of (x, column) is carried on one-direction dual numbers along it.  T_max enters only the
// CTCS integrand (the row ||T|| - T_max), which no other component reads, so its tangents
// vanish except in the y entries of the state and of the column, and those obey quadratures:
//     d/dt (dy/dT_max)      = s d([g]_+^2)/dT_max            = -2 s [g]_+
//     d/dt (dcol_y/dT_max)  = d/dT_max of the y row of the column's slope
//                           = -2 ds [g]_+ - 2 s 1{g > 0} dTn,
// with g = ||T|| - T_max, s the dilation, (dT, ds) the column's control direction and dTn the
// derivative of ||T|| along dT; they run with the same RK4 weights.
// ------------------------------------------------------------------------------------------
// Vehicle data on one-direction dual numbers, seeded on alpha_mdot.
template <typename T>
__device__ __forceinline__ Vehicle<Dual<T, 1>> lift_alpha(const Vehicle<T> &W)
{
    using D = Dual<T, 1>;
    Vehicle<D> V;
    V.m_dry = D(double(W.m_dry));
    V.alpha = seed<T, 1>(W.alpha, 0, T(1));
    for (int q = 0; q < 3; ++q) {
        V.g[q] = D(double(W.g[q]));
        V.Jinv[q] = D(double(W.Jinv[q]));
        V.J[q] = D(double(W.J[q]));
        V.rT[q] = D(double(W.rT[q]));
    }
    V.T_min = D(double(W.T_min));
    V.T_max = D(double(W.T_max));
    V.sec_delta = D(double(W.sec_delta));
    V.tan_gamma = D(double(W.tan_gamma));
    V.tilt_c = D(double(W.tilt_c));
    V.w_max2 = D(double(W.w_max2));
    V.v_max2 = D(double(W.v_max2));
    V.has_vmax = W.has_vmax;
    V.g_max2 = D(double(W.g_max2));
    V.has_gmax = W.has_gmax;
    return V;
}

template <typename R>
__global__ void __launch_bounds__(64)
tangent_kernel(GradArgs<R> a)
{
    using D = Dual<R, 1>;
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long per_b = (long)(a.kmax - 1) * COLS;
    const int b = (int)(gid / per_b);
    if (b >= a.B) return;
    const int rem = (int)(gid % per_b), k = rem / COLS, c = rem % COLS;
    if (a.gstat[b] >= 0) return;
    const int K = a.K[b];
    if (k >= K - 1) return;

    const Vehicle<R> W = load_vehicle<R>(a.params + (long)b * NP);
    const Vehicle<D> V = lift_alpha<R>(W);

    const R *xk = a.xbar + ((long)b * a.kmax + k) * NX;
    const R *uk = a.ubar + ((long)b * a.kmax + k) * NU;
    D x[NX], col[NX];
    for (int i = 0; i < NX; ++i) {
        x[i] = D(double(xk[i]));
        col[i] = D((c < NX && i == c) ? 1.0 : 0.0);
    }
    R ua[NU], ub[NU];
    for (int i = 0; i < NU; ++i) {
        ua[i] = uk[i];
        ub[i] = uk[NU + i];
    }
    const int uj = c < NX ? -1 : (c - NX) % NU;
    const bool plus = c >= NX + NU;
    const R dtau = R(1.0 / double(K - 1));
    const int nsub = a.rk4_substeps;
    const R h = dtau / R(nsub), hh = R(0.5) * h, h6 = h / R(6);

    R yT = R(0), cyT = R(0);  // tangents along T_max of y and of the column's y entry
    D xn[NX], cn[NX], xin[NX], cin[NX], fx[NX], fc[NX];
    double fy;
    for (int n = 0; n < nsub; ++n) {
        const R sig = R(n) * h;
        R yTn = yT, cyTn = cyT;
        for (int st = 0; st < 4; ++st) {
            const R sg = st == 0 ? sig : (st == 3 ? sig + h : sig + hh);
            const R lp = sg / dtau, lm = R(1) - lp;
            R u[NU], du[NU];
            D uD[NU], duD[NU];
            for (int i = 0; i < NU; ++i) {
                u[i] = lm * ua[i] + lp * ub[i];
                du[i] = i == uj ? (plus ? lp : lm) : R(0);
                uD[i] = D(double(u[i]));
                duD[i] = D(double(du[i]));
            }
            f_jvp<D, true>(V, st == 0 ? x : xin, uD, st == 0 ? col : cin, duD, fx, fy, fc);
            // the T_max quadratures (the model's thrust norm and its derivative, same forms)
            const R Tn = msqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            const R g5 = Tn - W.T_max, gp5 = g5 > R(0) ? g5 : R(0);
            const R dTn = Tn > R(NORM_EPS) ? mdiv(u[0] * du[0] + u[1] * du[1] + u[2] * du[2], Tn)
                                           : R(0);
            const R s = u[NU - 1], ds = du[NU - 1];
            const R ky = R(-2) * s * gp5;
            const R kc = R(-2) * (ds * gp5 + (g5 > R(0) ? s * dTn : R(0)));
            // RK4: the next value accumulates h/6 (k1 + 2 k2 + 2 k3 + k4)
            const R w = (st == 0 || st == 3) ? h6 : R(2) * h6;
            const D wd = D(double(w));
            for (int i = 0; i < NX; ++i) {
                if (st == 0) {
                    xn[i] = x[i] + wd * fx[i];
                    cn[i] = col[i] + wd * fc[i];
                } else {
                    xn[i] += wd * fx[i];
                    cn[i] += wd * fc[i];
                }
            }
            yTn += w * ky;
            cyTn += w * kc;
            if (st < 3) {
                const D hs = D(double(st == 2 ? h : hh));
                for (int i = 0; i < NX; ++i) {
                    xin[i] = x[i] + hs * fx[i];
                    cin[i] = col[i] + hs * fc[i];
                }
            }
        }
        for (int i = 0; i < NX; ++i) {
            x[i] = xn[i];
            col[i] = cn[i];
        }
        yT = yTn;
        cyT = cyTn;
    }

    const long ib = (long)b * (a.kmax - 1) + k;
    const double pc = c < NX ? a.px[c] : a.pu[(c - NX) % NU];
    R *d0 = a.dblk + (ib * 2) * BLK + c * CST;
    R *d1 = d0 + BLK;
    for (int i = 0; i < NX; ++i) {
        d0[i] = R(double(col[i].d[0]) * pc / a.px[i]);
        d1[i] = i == IY ? R(double(cyT) * pc / a.px[IY]) : R(0);
    }
    d0[NX] = d1[NX] = R(0);
    if (c == 0) {
        R *w0 = a.dwhat + (ib * 2) * DST;
        R *w1 = w0 + DST;
        for (int i = 0; i < NX; ++i) {
            w0[i] = R(double(x[i].d[0]) / a.px[i]);
            w1[i] = i == IY ? R(double(yT) / a.px[IY]) : R(0);
        }
        w0[NX] = w1[NX] = R(0);
    }
}

// ------------------------------------------------------------------------------------------
// Reverse (adjoint) sweep through the RK4 discretization, in double.
//
// One 32-lane group per (instance, interval); lane c < 23 owns column c of the variational
// system [A | B- | B+] (lanes 23..31 carry zero adjoints), and every lane carries the shared
// state x.  The cotangents entering at the end of the interval are the grad kernel's
// derivatives of the output with respect to the scaled column c and the scaled defect.  The
// sweep runs the RK4 substeps and their four stages backwards.  At a stage with input (X, P)
// the local vector-Jacobian products are
//     X^bar = J(X)^T K^bar + sum over columns c of (d/dX <L^bar_c, Df(X)[P_c, du_c]>)
//     P^bar_c = J(X)^T L^bar_c
// where K = f(X) and L_c = Df(X)[P_c, du_c] are the stage slopes of the state and of column c.
// The products with the state Jacobian and with the second derivative are both taken from
// evaluations of the model on one-direction dual numbers along e_i, i = 0..14 (the value part
// of the slope then carries J e_i and the column slope carries the second derivative along
// e_i); the column sum is a 32-lane reduction.  The parameter derivative accumulates
// <K^bar, df/dp> (state part, counted once) + <L^bar_c, d(Df[P_c])/dp> along the way.
// Substep starts and stage inputs are recomputed from the interval start.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ double group_sum32(double v)
{
    for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o, 32);
    return v;
}

// FOH control and the control part of the column direction at stage time sg.
__device__ __forceinline__ void stage_controls(const double *ua, const double *ub, double sg,
                                               double dtau, int uj, bool plus, double *u,
                                               double *du)
{
    const double lp = sg / dtau, lm = 1.0 - lp;
    for (int i = 0; i < NU; ++i) {
        u[i] = lm * ua[i] + lp * ub[i];
        du[i] = i == uj ? (plus ? lp : lm) : 0.0;
    }
}

// Slopes (f, Df[col, du]) of the state and of one column.
__device__ __forceinline__ void slopes(const Vehicle<double> &V, const double *x,
                                       const double *col, const double *u, const double *du,
                                       double *fx, double *fc)
{
    double fy;
    f_jvp<double, true>(V, x, u, col, du, fx, fy, fc);
}

template <typename R>
__global__ void __launch_bounds__(64) rk4_adjoint_kernel(GradArgs<R> a)
{
    using D1 = Dual<double, 1>;
    using D2 = Dual<double, 2>;
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long per_b = (long)(a.kmax - 1) * 32;
    const int b = (int)(gid / per_b);
    const int rem = (int)(gid % per_b), k = rem >> 5, c = rem & 31;
    // whole 32-lane groups leave together (b, k are uniform over a group)
    if (b >= a.B) return;
    if (a.gstat[b] >= 0) return;
    const int K = a.K[b];
    if (k >= K - 1) return;
    const bool col_lane = c < COLS;
    const int cc = col_lane ? c : 0;

    double pd[NP];
    for (int q = 0; q < NP; ++q) pd[q] = double(a.params[(long)b * NP + q]);
    const Vehicle<double> V = load_vehicle<double>(pd);
    const Vehicle<D1> V1 = lift_vehicle<1>(V, false);
    const Vehicle<D2> V2 = lift_vehicle<2>(V, true);

    const R *xk = a.xbar + ((long)b * a.kmax + k) * NX;
    const R *uk = a.ubar + ((long)b * a.kmax + k) * NU;
    double x0[NX], ua[NU], ub[NU];
    for (int i = 0; i < NX; ++i) x0[i] = double(xk[i]);
    for (int i = 0; i < NU; ++i) {
        ua[i] = double(uk[i]);
        ub[i] = double(uk[NU + i]);
    }
    const int uj = cc < NX ? -1 : (cc - NX) % NU;
    const bool plus = cc >= NX + NU;
    const double dtau = 1.0 / double(K - 1);
    const int nsub = a.rk4_substeps;
    const double h = dtau / nsub, hh = 0.5 * h;

    // cotangents at the end of the interval: scaled quantities back to original units
    const long ib = (long)b * (a.kmax - 1) + k;
    const double pc = cc < NX ? a.px[cc] : a.pu[(cc - NX) % NU];
    double xb[NX], cb[NX];
    for (int i = 0; i < NX; ++i) {
        xb[i] = double(a.dwhat[ib * 2 * DST + i]) / a.px[i];
        cb[i] = col_lane ? double(a.dblk[ib * 2 * BLK + cc * CST + i]) * pc / a.px[i] : 0.0;
    }
    double pb0 = 0.0, pb1 = 0.0;

    double xs[NX], cs[NX], X[NX], P[NX], fx[NX], fc[NX], u[NU], du[NU];
    for (int n = nsub - 1; n >= 0; --n) {
        // state and column at the start of substep n
        for (int i = 0; i < NX; ++i) {
            xs[i] = x0[i];
            cs[i] = (col_lane && cc < NX && i == cc) ? 1.0 : 0.0;
        }
        for (int m = 0; m < n; ++m) {
            double ax[NX], ac[NX];
            for (int st = 0; st < 4; ++st) {
                const double sg = m * h + (st == 0 ? 0.0 : (st == 3 ? h : hh));
                stage_controls(ua, ub, sg, dtau, uj, plus, u, du);
                if (st == 0)
                    for (int i = 0; i < NX; ++i) {
                        X[i] = xs[i];
                        P[i] = cs[i];
                    }
                slopes(V, X, P, u, du, fx, fc);
                const double w = (st == 0 || st == 3) ? 1.0 : 2.0;
                for (int i = 0; i < NX; ++i) {
                    ax[i] = st == 0 ? fx[i] : ax[i] + w * fx[i];
                    ac[i] = st == 0 ? fc[i] : ac[i] + w * fc[i];
                }
                if (st < 3) {
                    const double hs = st == 2 ? h : hh;
                    for (int i = 0; i < NX; ++i) {
                        X[i] = xs[i] + hs * fx[i];
                        P[i] = cs[i] + hs * fc[i];
                    }
                }
            }
            for (int i = 0; i < NX; ++i) {
                xs[i] += h / 6.0 * ax[i];
                cs[i] += h / 6.0 * ac[i];
            }
        }
        // stages of substep n, backwards
        double xa[NX], ca[NX], kx[NX], kc[NX];
        for (int i = 0; i < NX; ++i) {
            xa[i] = xb[i];
            ca[i] = cb[i];
            kx[i] = kc[i] = 0.0;
        }
        for (int st = 3; st >= 0; --st) {
            // stage input (X, P): the stages before st, from the substep start
            for (int i = 0; i < NX; ++i) {
                X[i] = xs[i];
                P[i] = cs[i];
            }
            for (int r = 0; r < st; ++r) {
                const double sg = n * h + (r == 0 ? 0.0 : hh);
                stage_controls(ua, ub, sg, dtau, uj, plus, u, du);
                slopes(V, X, P, u, du, fx, fc);
                const double hs = r == 2 ? h : hh;
                for (int i = 0; i < NX; ++i) {
                    X[i] = xs[i] + hs * fx[i];
                    P[i] = cs[i] + hs * fc[i];
                }
            }
            const double sg = n * h + (st == 0 ? 0.0 : (st == 3 ? h : hh));
            stage_controls(ua, ub, sg, dtau, uj, plus, u, du);
            const double w = (st == 0 || st == 3) ? h / 6.0 : h / 3.0;
            double Kb[NX], Lb[NX];
            for (int i = 0; i < NX; ++i) {
                Kb[i] = w * xb[i] + kx[i];
                Lb[i] = w * cb[i] + kc[i];
            }
            // local products along e_i
            double Xb[NX], Pb[NX];
            D1 Xd[NX], Pd[NX], ud[NU], dud[NU], fd[NX], gd[NX];
            for (int i = 0; i < NU; ++i) {
                ud[i] = D1(u[i]);
                dud[i] = D1(du[i]);
            }
            for (int i = 0; i < NX; ++i) Pd[i] = D1(P[i]);
            for (int e = 0; e < NX; ++e) {
                for (int i = 0; i < NX; ++i) Xd[i] = seed<double, 1>(X[i], 0, i == e ? 1.0 : 0.0);
                double fy;
                f_jvp<D1, true>(V1, Xd, ud, Pd, dud, fd, fy, gd);
                double jk = 0.0, jl = 0.0, hl = 0.0;
                for (int r = 0; r < NX; ++r) {
                    jk += Kb[r] * fd[r].d[0];
                    jl += Lb[r] * fd[r].d[0];
                    hl += Lb[r] * gd[r].d[0];
                }
                Xb[e] = jk + group_sum32(hl);
                Pb[e] = jl;
            }
            // parameter derivatives at this stage
            {
                D2 Xp[NX], Pp[NX], up[NU], dup[NU], fp[NX], gp[NX];
                for (int i = 0; i < NX; ++i) {
                    Xp[i] = D2(X[i]);
                    Pp[i] = D2(P[i]);
                }
                for (int i = 0; i < NU; ++i) {
                    up[i] = D2(u[i]);
                    dup[i] = D2(du[i]);
                }
                double fy;
                f_jvp<D2, true>(V2, Xp, up, Pp, dup, fp, fy, gp);
                for (int r = 0; r < NX; ++r) {
                    if (c == 0) {
                        pb0 += Kb[r] * fp[r].d[0];
                        pb1 += Kb[r] * fp[r].d[1];
                    }
                    pb0 += Lb[r] * gp[r].d[0];
                    pb1 += Lb[r] * gp[r].d[1];
                }
            }
            for (int i = 0; i < NX; ++i) {
                xa[i] += Xb[i];
                ca[i] += Pb[i];
            }
            // this stage's input was substep start + coefficient * previous slope
            const double cf = st == 3 ? h : hh;
            for (int i = 0; i < NX; ++i) {
                kx[i] = st > 0 ? cf * Xb[i] : 0.0;
                kc[i] = st > 0 ? cf * Pb[i] : 0.0;
            }
        }
        for (int i = 0; i < NX; ++i) {
            xb[i] = xa[i];
            cb[i] = col_lane ? ca[i] : 0.0;
        }
    }
    pb0 = group_sum32(pb0);
    pb1 = group_sum32(pb1);
    if (c == 0) {
        a.pbar[ib * 2] = pb0;
        a.pbar[ib * 2 + 1] = pb1;
    }
}

// Adds the discretization part of d/d(alpha_mdot, T_max), summed over intervals in order.
template <typename R>
__global__ void grad_finalize_kernel(GradArgs<R> a)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.B || a.gstat[b] >= 0) return;
    const int M = a.K[b] - 1;
    double s0 = 0.0, s1 = 0.0;
    for (int k = 0; k < M; ++k) {
        s0 += a.pbar[((long)b * (a.kmax - 1) + k) * 2];
        s1 += a.pbar[((long)b * (a.kmax - 1) + k) * 2 + 1];
    }
    R *g = a.grad + (long)b * 18;
    g[16] = R(double(g[16]) + s0);
    g[17] = R(double(g[17]) + s1);
}

// ------------------------------------------------------------------------------------------
// Projections and their vector-Jacobian products (recomputed from the projection's input).
// ------------------------------------------------------------------------------------------
// Second-order cone {(t, z) : ||z|| <= a t}, z in R^2.
template <typename R>
__device__ __forceinline__ void soc2_fwd(R &t, R &z0, R &z1, R a)
{
    const R nz = sqrt(z0 * z0 + z1 * z1);
    if (nz <= a * t) return;
    if (a * nz <= -t) {
        t = z0 = z1 = R(0);
        return;
    }
    const R tp = (t + a * nz) / (R(1) + a * a);
    const R s = a * tp / nz;
    z0 *= s;
    z1 *= s;
    t = tp;
}

// (tb, zb) holds the adjoint of the projection's output and receives that of its input
// (t, z).
template <typename R>
__device__ __forceinline__ void soc2_vjp(R t, R z0, R z1, R a, R &tb, R &zb0, R &zb1)
{
    const R nz = sqrt(z0 * z0 + z1 * z1);
    if (nz <= a * t) return;
    if (a * nz <= -t) {
        tb = zb0 = zb1 = R(0);
        return;
    }
    const R den = R(1) + a * a;
    const R tp = (t + a * nz) / den;
    const R n0 = z0 / nz, n1 = z1 / nz;
    const R tpb = tb + a * (n0 * zb0 + n1 * zb1);
    const R nb0 = a * tp * zb0, nb1 = a * tp * zb1;
    const R nn = n0 * nb0 + n1 * nb1;
    const R c = a * tpb / den;
    tb = tpb / den;
    zb0 = c * n0 + (nb0 - n0 * nn) / nz;
    zb1 = c * n1 + (nb1 - n1 * nn) / nz;
}

// Ball ||z|| <= rad in R^N.
template <typename R, int N>
__device__ __forceinline__ void ball_fwd(R *z, R rad)
{
    R s = R(0);
    for (int q = 0; q < N; ++q) s += z[q] * z[q];
    const R nz = sqrt(s);
    if (nz > rad) {
        const R f = rad / nz;
        for (int q = 0; q < N; ++q) z[q] *= f;
    }
}

// zb: adjoint of the output in, of the input z out; returns the adjoint of the radius.
template <typename R, int N>
__device__ __forceinline__ R ball_vjp(const R *z, R rad, R *zb)
{
    R s = R(0);
    for (int q = 0; q < N; ++q) s += z[q] * z[q];
    const R nz = sqrt(s);
    if (!(nz > rad)) return R(0);
    R nzb = R(0);
    for (int q = 0; q < N; ++q) nzb += z[q] * zb[q];
    nzb /= nz;
    for (int q = 0; q < N; ++q) zb[q] = rad / nz * (zb[q] - z[q] / nz * nzb);
    return nzb;
}

// Sets of the node-wise projection in original units, with what the kernel needs of them.
template <typename R>
struct NodeSets {
    int mask;
    R mdry, glide_a, tilt_rad, w_max, gimbal_a, T_max;
};

// State sets of node k (bits 1, 2, 4, 8): pre-projection x^ in XP (scaled), reference xb
// (original units).  Writes the projected non-fixed group members into xh, which holds the
// boundary values of the fixed members already.  At the last node (`last`) the roll rate is
// projected onto the rate ball's slice through the fixed transverse rates.
template <typename R>
__device__ __forceinline__ R roll_rate_radius(const NodeSets<R> &S, const R *xh, const R *xb,
                                              const R *px)
{
    const R c2 = xb[12] + px[12] * xh[12], c3 = xb[13] + px[13] * xh[13];
    const R r2 = S.w_max * S.w_max - c2 * c2 - c3 * c3;
    return r2 > R(0) ? sqrt(r2) : R(0);
}
template <typename R>
__device__ __forceinline__ void xproj_fwd(const NodeSets<R> &S, const R *xp, const R *xb,
                                          const R *px, const bool *fixed, bool last, R *xh)
{
    R xo[NX];
    for (int q = 0; q < NX; ++q) xo[q] = xb[q] + px[q] * xp[q];
    if (S.mask & 1)
        if (!fixed[0] && xo[0] < S.mdry) xh[0] = (S.mdry - xb[0]) / px[0];
    // a group member that is a fixed boundary value keeps that value (the projection acts on
    // the pre-boundary values, then the boundary values overwrite, as in the solve)
    if (S.mask & 2) {
        R z[3] = {xo[1], xo[2], xo[3]};
        soc2_fwd<R>(z[0], z[1], z[2], S.glide_a);
        for (int q = 0; q < 3; ++q)
            if (!fixed[1 + q]) xh[1 + q] = (z[q] - xb[1 + q]) / px[1 + q];
    }
    if (S.mask & 4) {
        R z[2] = {xo[9], xo[10]};
        ball_fwd<R, 2>(z, S.tilt_rad);
        for (int q = 0; q < 2; ++q)
            if (!fixed[9 + q]) xh[9 + q] = (z[q] - xb[9 + q]) / px[9 + q];
    }
    if ((S.mask & 8) && last) {
        const R r = roll_rate_radius<R>(S, xh, xb, px);
        const R w1 = fmin(fmax(xo[11], -r), r);
        xh[11] = (w1 - xb[11]) / px[11];
    } else if (S.mask & 8) {
        R z[3] = {xo[11], xo[12], xo[13]};
        ball_fwd<R, 3>(z, S.w_max);
        for (int q = 0; q < 3; ++q)
            if (!fixed[11 + q]) xh[11 + q] = (z[q] - xb[11 + q]) / px[11 + q];
    }
}

// g: adjoint of the projected (scaled) state in, of the pre-projection state out.  Fixed
// members already carry a zero adjoint.
template <typename R>
__device__ __forceinline__ void xproj_vjp(const NodeSets<R> &S, const R *xp, const R *xb,
                                          const R *px, const R *xh, bool last, R *g)
{
    R xo[NX];
    for (int q = 0; q < NX; ++q) xo[q] = xb[q] + px[q] * xp[q];
    if ((S.mask & 1) && xo[0] < S.mdry) g[0] = R(0);
    if (S.mask & 2) {
        R tb = g[1] / px[1], zb0 = g[2] / px[2], zb1 = g[3] / px[3];
        soc2_vjp<R>(xo[1], xo[2], xo[3], S.glide_a, tb, zb0, zb1);
        g[1] = tb * px[1];
        g[2] = zb0 * px[2];
        g[3] = zb1 * px[3];
    }
    if (S.mask & 4) {
        R zb[2] = {g[9] / px[9], g[10] / px[10]};
        const R z[2] = {xo[9], xo[10]};
        (void)ball_vjp<R, 2>(z, S.tilt_rad, zb);
        g[9] = zb[0] * px[9];
        g[10] = zb[1] * px[10];
    }
    if ((S.mask & 8) && last) {
        const R r = roll_rate_radius<R>(S, xh, xb, px);
        if (!(xo[11] >= -r && xo[11] <= r)) g[11] = R(0);
    } else if (S.mask & 8) {
        R zb[3] = {g[11] / px[11], g[12] / px[12], g[13] / px[13]};
        const R z[3] = {xo[11], xo[12], xo[13]};
        (void)ball_vjp<R, 3>(z, S.w_max, zb);
        for (int q = 0; q < 3; ++q) g[11 + q] = zb[q] * px[11 + q];
    }
}

// Control of node k: the s box, then (bit 16) the gimbal cone and the T_max ball.
template <typename R>
__device__ __forceinline__ void uproj_fwd(const NodeSets<R> &S, const R *up, const R *ub,
                                          const R *pu, R slo, R shi, R *uh)
{
    uh[3] = fmin(fmax(up[3], slo), shi);
    if (S.mask & 16) {
        R T[3];
        for (int q = 0; q < 3; ++q) T[q] = ub[q] + pu[q] * up[q];
        soc2_fwd<R>(T[0], T[1], T[2], S.gimbal_a);
        ball_fwd<R, 3>(T, S.T_max);
        for (int q = 0; q < 3; ++q) uh[q] = (T[q] - ub[q]) / pu[q];
    } else {
        for (int q = 0; q < 3; ++q) uh[q] = up[q];
    }
}

// Returns the adjoint of T_max.
template <typename R>
__device__ __forceinline__ R uproj_vjp(const NodeSets<R> &S, const R *up, const R *ub,
                                       const R *pu, R slo, R shi, R *g)
{
    if (!(up[3] >= slo && up[3] <= shi)) g[3] = R(0);
    if (!(S.mask & 16)) return R(0);
    R T[3], Tc[3], Tb[3];
    for (int q = 0; q < 3; ++q) {
        T[q] = Tc[q] = ub[q] + pu[q] * up[q];
        Tb[q] = g[q] / pu[q];
    }
    soc2_fwd<R>(Tc[0], Tc[1], Tc[2], S.gimbal_a);
    const R radb = ball_vjp<R, 3>(Tc, S.T_max, Tb);
    soc2_vjp<R>(T[0], T[1], T[2], S.gimbal_a, Tb[0], Tb[1], Tb[2]);
    for (int q = 0; q < 3; ++q) g[q] = Tb[q] * pu[q];
    return radb;
}

// ------------------------------------------------------------------------------------------
// Forward steps with checkpoints, then the reverse sweep.
// ------------------------------------------------------------------------------------------
size_t grad_smem_bytes_r(int kmax, size_t rs)
{
    const StateLayout L = state_layout(kmax);
    return 128 * sizeof(double) +
           rs * ((size_t)2 * L.len + 4 * 16 * kmax + 4 * NU * kmax + DST * (kmax - 1) + kmax);
}

template <typename R, int MAXT>
__global__ void __launch_bounds__(MAXT) grad_kernel(GradArgs<R> a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int b = blockIdx.x;
    const int kmax = a.kmax, t = threadIdx.x;
    const int k = t >> 4, i = t & 15;
    R *gout = a.grad + (long)b * 18;
    if (a.gstat[b] >= 0) {
        if (t < 18) gout[t] = R(0);
        if (a.fval && t < 2) a.fval[(long)b * 2 + t] = R(0);
        return;
    }
    const int K = a.K[b], M = K - 1;
    const StateLayout L = state_layout(kmax);

    double *red = reinterpret_cast<double *>(smem_raw);  // [16 waves * 8]
    // the extrapolated iterate S lives in two buffers (each extrapolation writes the other)
    R *S = reinterpret_cast<R *>(red + 128);             // current extrapolated iterate
    R *const S1 = S;
    R *XP = S + L.len;                                    // [kmax][16] x^ before projection
    R *XH = XP + kmax * 16;                               // [kmax][16] fresh x^
    R *XB = XH + kmax * 16;                               // [kmax][16] reference (original)
    R *XHB = XB + kmax * 16;                              // [kmax][16] adjoint of x^
    R *UP = XHB + kmax * 16;                              // [kmax][4]  u^ before projection
    R *UH = UP + kmax * NU;                               // [kmax][4]  fresh u^
    R *UB = UH + kmax * NU;                               // [kmax][4]  reference (original)
    R *UHB = UB + kmax * NU;                              // [kmax][4]  adjoint of u^
    R *RB = UHB + kmax * NU;                              // [kmax-1][16] adjoint of r
    R *PB = RB + (kmax - 1) * DST;                        // [kmax] adjoint of the theta step
    R *const S2 = PB + kmax;                              // [L.len] second buffer of S

    const bool node = k < K;
    const bool isx = node && i < NX;
    const bool isu = node && i < NU;
    const bool dual = k < M && i < NX;
    const R *p = a.params + (long)b * NP;
    const long ib = (long)b * (kmax - 1) + (dual ? k : 0);

    // -------------------- load the recorded starting point and the QP --------------------
    for (int q = t; q < L.len; q += blockDim.x) S2[q] = R(0);
    if (k < kmax) {
        XB[k * 16 + i] = isx ? a.xbar[((long)b * kmax + k) * NX + i] : R(0);
        if (i < NU) UB[k * NU + i] = isu ? a.ubar[((long)b * kmax + k) * NU + i] : R(0);
        S[L.X + k * 16 + i] = R(0);
        if (i < NU) S[L.U + k * NU + i] = R(0);
        if (k < kmax - 1) {
            const long ro = ((long)b * (kmax - 1) + k) * NX + i;
            S[L.MP + k * DST + i] = dual ? a.mup[ro] : R(0);
            S[L.MM + k * DST + i] = dual ? a.mum[ro] : R(0);
            S[L.PH + k * DST + i] = dual ? a.phi[ro] : R(0);
        }
        if (i == IY) S[L.TH + k] = k < M ? a.th[(long)b * (kmax - 1) + k] : R(0);
    }
    R colA[NX], rowA[NX], rowBm[NU], rowBp[NU];
    for (int q = 0; q < NX; ++q) {
        colA[q] = dual ? a.blocks[ib * BLK + i * CST + q] : R(0);
        rowA[q] = dual ? a.blocks[ib * BLK + q * CST + i] : R(0);
    }
    for (int q = 0; q < NU; ++q) {
        rowBm[q] = dual ? a.blocks[ib * BLK + (NX + q) * CST + i] : R(0);
        rowBp[q] = dual ? a.blocks[ib * BLK + (NX + NU + q) * CST + i] : R(0);
    }
    // transposed control products: lane i supplies row i of B^-_k and of B^+_{k-1} with the
    // components in the exchange order of row_reduce_scatter4i, which leaves the row sum of
    // component q on lane q
    R rowBmX[NU], rowBqX[NU];
    {
        const bool bq = node && k > 0 && i < NX;
        const long ibq = (long)b * (kmax - 1) + (bq ? k - 1 : 0);
        for (int s = 0; s < NU; ++s) {
            const int q = xpermi(i, s);
            rowBmX[s] = dual ? a.blocks[ib * BLK + (NX + q) * CST + i] : R(0);
            rowBqX[s] = bq ? a.blocks[ibq * BLK + (NX + NU + q) * CST + i] : R(0);
        }
    }
    const R wk = dual ? a.what[ib * DST + i] : R(0);
    R epsk = R(0);
    if (dual && i == IY) {
        const double y0 = double(a.xbar[((long)b * kmax + k) * NX + IY]);
        const double y1 = double(a.xbar[((long)b * kmax + k + 1) * NX + IY]);
        epsk = R((double(p[20]) - (y1 - y0)) / a.px[IY]);
    }
    bool fixed = false;
    R fixv = R(0);
    if (isx) {
        const double xb = double(a.xbar[((long)b * kmax + k) * NX + i]);
        if (k == 0) {
            fixed = true;
            const double zi = i < IY ? double(a.x0[(long)b * NX + i]) : 0.0;
            fixv = R((zi - xb) / a.px[i]);
        } else if (k == K - 1 && final_fixed(i)) {
            fixed = true;
            fixv = R((double(a.xf[(long)b * NXF + i - 1]) - xb) / a.px[i]);
        }
    }
    R slo = R(0), shi = R(0);
    if (node) {
        const double s0 = double(a.ubar[((long)b * kmax + k) * NU + 3]);
        slo = R((double(p[18]) - s0) / a.pu[3]);
        shi = R((double(p[19]) - s0) / a.pu[3]);
    }
    NodeSets<R> sets;
    sets.mask = a.node_projections;
    sets.mdry = p[1];
    sets.glide_a = R(1.0 / tan(double(p[15])));
    sets.tilt_rad = R(sqrt(0.5 * (1.0 - cos(double(p[16])))));
    sets.w_max = p[17];
    sets.gimbal_a = R(tan(double(p[14])));
    sets.T_max = p[13];
    R pxr[NX], pur[NU];
    for (int q = 0; q < NX; ++q) pxr[q] = R(a.px[q]);
    for (int q = 0; q < NU; ++q) pur[q] = R(a.pu[q]);
    bool fixed_node[NX];
    for (int q = 0; q < NX; ++q) fixed_node[q] = k == 0 || (k == K - 1 && final_fixed(q));

    const double sig = a.sigma[b];
    const double alpha_d = 2.0 / (a.w_prox + sqrt(a.w_prox * a.w_prox + 4.0 * a.omega * sig));
    const R alpha = R(alpha_d), beta = R(a.omega * alpha_d), rho = R(a.rho), omr = R(1) - rho;
    const R wprox = R(a.w_prox), wep = R(a.w_ep);
    const R cost = (isx && k == K - 1 && i == 0) ? R(-a.w_cost) : R(0);  // e_cost = -e_m
    __syncthreads();

    // per-lane values of the step last evaluated
    R a_mu = R(0), b_mu = R(0), mupn = R(0), mumn = R(0), phn = R(0), thp = R(0), thn = R(0);

    // projected gradient step on the primal variables: XP/UP (pre-projection), XH/UH
    // (the row products below run on every lane of a row, with zeros where a lane holds no
    // variable: a DPP exchange reads lanes that a branch would have switched off)
    auto primal = [&]() {
        // phi_k of this lane's dynamics row and phi_{k-1} of the row above
        const R vph = dual ? S[L.PH + k * DST + i] : R(0);
        const R vphm = (node && k > 0 && i < NX) ? S[L.PH + (k - 1) * DST + i] : R(0);
        // x: wprox x~ + cost + (A^-_k)^T phi_k, by row broadcasts of phi_k
        const R xt = isx ? S[L.X + k * 16 + i] : R(0);
        R g = rowdot15<R>(colA, vph, wprox * xt + cost);
        // u: (B^-_k)^T phi_k + (B^+_{k-1})^T phi_{k-1}, reduced onto lane q
        R gq[NU];
        for (int s = 0; s < NU; ++s) gq[s] = rowBmX[s] * vph + rowBqX[s] * vphm;
        const R gu = row_reduce_scatter4i<R>(gq);
        if (isx) {
            if (k > 0) g -= vphm;
            if (i == IY) {
                if (k < M) g -= S[L.TH + k];
                if (k > 0) g += S[L.TH + k - 1];
            }
            const R xp = xt - alpha * g;
            XP[k * 16 + i] = xp;
            XH[k * 16 + i] = fixed ? fixv : xp;
        }
        if (isu) {
            const R ut = S[L.U + k * NU + i];
            const R up = ut - alpha * (wprox * ut + gu);
            UP[k * NU + i] = up;
            // the paper's set: the s box is the only control projection, taken in place
            if (!sets.mask) UH[k * NU + i] = i == 3 ? fmin(fmax(up, slo), shi) : up;
        }
        if (sets.mask) {
            __syncthreads();
            if (node && i == 0 && (sets.mask & 15))
                xproj_fwd<R>(sets, XP + k * 16, XB + k * 16, pxr, fixed_node,
                             k == K - 1 && k > 0, XH + k * 16);
            if (node && i == 1)
                uproj_fwd<R>(sets, UP + k * NU, UB + k * NU, pur, slo, shi, UH + k * NU);
        }
        __syncthreads();
    };

    // dual step (needs XH, UH)
    // extrapolated primal values 2 z^ - z~: this node's x (lane i), its u and node k+1's u
    // (lanes q < 4)
    auto vx_own = [&]() { return isx ? R(2) * XH[k * 16 + i] - S[L.X + k * 16 + i] : R(0); };
    auto vu_own = [&]() { return isu ? R(2) * UH[k * NU + i] - S[L.U + k * NU + i] : R(0); };
    auto vu_next = [&]() {
        return (dual && i < NU) ? R(2) * UH[(k + 1) * NU + i] - S[L.U + (k + 1) * NU + i] : R(0);
    };
    auto dual_step = [&]() {
        // A^-_k, B^-_k, B^+_k times the extrapolated values, by row broadcasts
        R r = rowdot15<R>(rowA, vx_own(), R(0));
        r = rowdot_part<R, 0, NU>(rowBm, vu_own(), r);
        r = rowdot_part<R, 0, NU>(rowBp, vu_next(), r);
        if (!dual) return;
        const R vph = S[L.PH + k * DST + i];
        const R np = S[L.MP + k * DST + i], nm = S[L.MM + k * DST + i];
        a_mu = np - alpha * (wep + vph);
        b_mu = nm - alpha * (wep - vph);
        mupn = a_mu > R(0) ? a_mu : R(0);
        mumn = b_mu > R(0) ? b_mu : R(0);
        r -= R(2) * XH[(k + 1) * 16 + i] - S[L.X + (k + 1) * 16 + i];
        r += (R(2) * mupn - np) - (R(2) * mumn - nm) + wk;
        phn = vph + beta * r;
        if (i == IY) {
            const R vy1 = R(2) * XH[(k + 1) * 16 + IY] - S[L.X + (k + 1) * 16 + IY];
            const R vy0 = R(2) * XH[k * 16 + IY] - S[L.X + k * 16 + IY];
            thp = S[L.TH + k] + beta * (vy1 - vy0 - epsk);
            thn = thp > R(0) ? thp : R(0);
        }
    };

    // extrapolation: S <- (1 - rho) S + rho (fresh iterate)
    // into the other buffer, so that no lane still reading this step's S is overtaken; the
    // entries no lane writes (no variable) are zero in both buffers
    auto extrapolate = [&]() {
        R *const Sn = S == S1 ? S2 : S1;
        if (isx) Sn[L.X + k * 16 + i] = omr * S[L.X + k * 16 + i] + rho * XH[k * 16 + i];
        if (isu) Sn[L.U + k * NU + i] = omr * S[L.U + k * NU + i] + rho * UH[k * NU + i];
        if (dual) {
            Sn[L.MP + k * DST + i] = omr * S[L.MP + k * DST + i] + rho * mupn;
            Sn[L.MM + k * DST + i] = omr * S[L.MM + k * DST + i] + rho * mumn;
            Sn[L.PH + k * DST + i] = omr * S[L.PH + k * DST + i] + rho * phn;
            if (i == IY) Sn[L.TH + k] = omr * S[L.TH + k] + rho * thn;
        }
        __syncthreads();
        S = Sn;
    };

    R *tape = a.tape + (long)b * (a.n_ckpt + a.ckpt) * L.len;
    auto save = [&](int slot) {
        __syncthreads();
        for (int q = t; q < L.len; q += blockDim.x) tape[(long)slot * L.len + q] = S[q];
    };
    auto load = [&](int slot) {
        __syncthreads();
        for (int q = t; q < L.len; q += blockDim.x) S[q] = tape[(long)slot * L.len + q];
        __syncthreads();
    };

    // -------------------- forward: n steps with checkpoints --------------------
    const int n = a.nsteps;
    for (int j = 1; j <= n; ++j) {
        if ((j - 1) % a.ckpt == 0) save((j - 1) / a.ckpt);
        primal();
        dual_step();
        if (j == n && a.fval && t == 0) {
            const double mf = double(XB[(K - 1) * 16]) + a.px[0] * double(XH[(K - 1) * 16]);
            double tf = 0.0;
            const double dtau = 1.0 / M;
            for (int q = 0; q < M; ++q)
                tf += dtau * 0.5 *
                      (double(UB[q * NU + 3]) + a.pu[3] * double(UH[q * NU + 3]) +
                       double(UB[(q + 1) * NU + 3]) + a.pu[3] * double(UH[(q + 1) * NU + 3]));
            a.fval[(long)b * 2] = R(mf);
            a.fval[(long)b * 2 + 1] = R(tf);
        }
        extrapolate();
    }

    // -------------------- reverse sweep --------------------
    const R cm = a.cot[(long)b * 2], ct = a.cot[(long)b * 2 + 1];
    const R dtau = R(1.0 / M);
    // adjoints of the extrapolated iterate owned by this lane
    R tbx = R(0), tbu = R(0), tbmp = R(0), tbmm = R(0), tbph = R(0), tbth = R(0);
    // accumulated derivatives: scaled blocks (row i of interval k), defect, boundary value,
    // and T_max through the thrust ball
    R accA[NX], accBm[NU], accBp[NU];
    for (int q = 0; q < NX; ++q) accA[q] = R(0);
    for (int q = 0; q < NU; ++q) accBm[q] = accBp[q] = R(0);
    R accW = R(0), accZ = R(0), accT = R(0);

    for (int m = a.n_ckpt - 1; m >= 0; --m) {
        const int j0 = m * a.ckpt;
        const int j1 = (j0 + a.ckpt < n) ? j0 + a.ckpt : n;
        load(m);
        for (int j = j0 + 1; j <= j1; ++j) {
            save(a.n_ckpt + (j - j0 - 1));
            if (j < j1) {
                primal();
                dual_step();
                extrapolate();
            }
        }
        for (int j = j1; j > j0; --j) {
            load(a.n_ckpt + (j - j0 - 1));
            primal();
            dual_step();
            // adjoints of the fresh iterate: the extrapolation passes rho of the adjoint on,
            // the last step also receives the output's cotangent
            R hxb = rho * tbx, hub = rho * tbu, hmpb = rho * tbmp, hmmb = rho * tbmm;
            R hphb = rho * tbph, hthb = rho * tbth;
            if (j == n) {
                if (isx && k == K - 1 && i == 0) hxb += cm * pxr[0];
                if (isu && i == 3) hub += ct * pur[3] * dtau * ((k == 0 || k == K - 1) ? R(0.5) : R(1));
            }
            R nbx = omr * tbx, nbu = omr * tbu, nbmp = omr * tbmp, nbmm = omr * tbmm;
            R nbph = omr * tbph, nbth = omr * tbth;
            // dual step: phi = varphi + beta r, theta = max(0, vartheta + beta (...))
            R rb = R(0);
            if (dual) {
                rb = beta * hphb;
                RB[k * DST + i] = rb;
                nbph += hphb;
                if (i == IY) {
                    const R pb = thp > R(0) ? hthb : R(0);
                    PB[k] = pb;
                    nbth += pb;
                }
            }
            __syncthreads();
            // (A^-_k)^T rb_k and (B^-_k)^T rb_k + (B^+_{k-1})^T rb_{k-1}, by row broadcasts
            const R rbm = (node && k > 0 && i < NX) ? RB[(k - 1) * DST + i] : R(0);
            const R vbA = rowdot15<R>(colA, rb, R(0));
            R gq[NU];
            for (int s = 0; s < NU; ++s) gq[s] = rowBmX[s] * rb + rowBqX[s] * rbm;
            const R vub = row_reduce_scatter4i<R>(gq);
            if (isx) {
                R vb = vbA;
                if (k > 0) vb -= rbm;
                if (i == IY) vb += beta * ((k > 0 ? PB[k - 1] : R(0)) - (k < M ? PB[k] : R(0)));
                R xb_ = hxb + R(2) * vb;
                nbx -= vb;
                if (fixed) {
                    if (k == 0) accZ += xb_;
                    xb_ = R(0);
                }
                XHB[k * 16 + i] = xb_;
            }
            if (isu) {
                R ub_ = hub + R(2) * vub;
                // the paper's set: the s box's derivative, taken in place (zero where it clamps)
                if (!sets.mask && i == 3 && !(UP[k * NU + 3] >= slo && UP[k * NU + 3] <= shi))
                    ub_ = R(0);
                UHB[k * NU + i] = ub_;
                nbu -= vub;
            }
            // derivative of the blocks: rb_k times the extrapolated values (zero rb off the
            // dynamics rows)
            bcast_axpy<R, NX>(accA, rb, vx_own());
            bcast_axpy<R, NU>(accBm, rb, vu_own());
            bcast_axpy<R, NU>(accBp, rb, vu_next());
            if (dual) {
                const R mpb = hmpb + R(2) * rb, mmb = hmmb - R(2) * rb;
                nbmp -= rb;
                nbmm += rb;
                accW += rb;
                const R ab = a_mu > R(0) ? mpb : R(0), bb = b_mu > R(0) ? mmb : R(0);
                nbmp += ab;
                nbph -= alpha * ab;
                nbmm += bb;
                nbph += alpha * bb;
            }
            // projections (the node-wise sets; with the paper's set only the s box, above)
            if (sets.mask) {
                __syncthreads();
                if (node && i == 0 && (sets.mask & 15))
                    xproj_vjp<R>(sets, XP + k * 16, XB + k * 16, pxr, XH + k * 16,
                                 k == K - 1 && k > 0, XHB + k * 16);
                if (node && i == 1)
                    accT += uproj_vjp<R>(sets, UP + k * NU, UB + k * NU, pur, slo, shi,
                                         UHB + k * NU);
            }
            __syncthreads();
            // gradient step: x^pre = x~ - alpha g(x~, varphi, vartheta), likewise u
            if (isx) nbx += XHB[k * 16 + i] * (R(1) - alpha * wprox);
            if (isu) nbu += UHB[k * NU + i] * (R(1) - alpha * wprox);
            {
                // -alpha times the adjoints of this node's x^, u^ and of node k+1's u^
                const R gxo = isx ? -alpha * XHB[k * 16 + i] : R(0);
                const R guo = isu ? -alpha * UHB[k * NU + i] : R(0);
                const R gun = (dual && i < NU) ? -alpha * UHB[(k + 1) * NU + i] : R(0);
                const R ph = dual ? S[L.PH + k * DST + i] : R(0);
                R s = dual ? alpha * XHB[(k + 1) * 16 + i] : R(0);
                s = rowdot15<R>(rowA, gxo, s);
                s = rowdot_part<R, 0, NU>(rowBm, guo, s);
                s = rowdot_part<R, 0, NU>(rowBp, gun, s);
                bcast_axpy<R, NX>(accA, ph, gxo);
                bcast_axpy<R, NU>(accBm, ph, guo);
                bcast_axpy<R, NU>(accBp, ph, gun);
                if (dual) nbph += s;
            }
            if (dual) {
                if (i == IY) nbth += alpha * (XHB[k * 16 + IY] - XHB[(k + 1) * 16 + IY]);
            }
            tbx = nbx;
            tbu = nbu;
            tbmp = nbmp;
            tbmm = nbmm;
            tbph = nbph;
            tbth = nbth;
            __syncthreads();
        }
    }

    // -------------------- the discretization's share --------------------
    // reverse mode: hand the block and defect adjoints (scaled) to the RK4 reverse sweep,
    // stored where the tangents would be; tangent mode: contract with the tangents here
    double part[3] = {0.0, 0.0, 0.0};
    if (a.rk4_reverse && dual) {
        R *ab = a.dblk + (ib * 2) * BLK;
        for (int q = 0; q < NX; ++q) ab[q * CST + i] = accA[q];
        for (int q = 0; q < NU; ++q) {
            ab[(NX + q) * CST + i] = accBm[q];
            ab[(NX + NU + q) * CST + i] = accBp[q];
        }
        a.dwhat[(ib * 2) * DST + i] = accW;
    }
    if (!a.rk4_reverse && dual) {
        const R *d0 = a.dblk + (ib * 2) * BLK;
        const R *d1 = d0 + BLK;
        const R *w0 = a.dwhat + (ib * 2) * DST;
        const R *w1 = w0 + DST;
        for (int q = 0; q < NX; ++q) {
            part[0] += double(accA[q]) * double(d0[q * CST + i]);
            part[1] += double(accA[q]) * double(d1[q * CST + i]);
        }
        for (int q = 0; q < NU; ++q) {
            part[0] += double(accBm[q]) * double(d0[(NX + q) * CST + i]) +
                       double(accBp[q]) * double(d0[(NX + NU + q) * CST + i]);
            part[1] += double(accBm[q]) * double(d1[(NX + q) * CST + i]) +
                       double(accBp[q]) * double(d1[(NX + NU + q) * CST + i]);
        }
        part[0] += double(accW) * double(w0[i]);
        part[1] += double(accW) * double(w1[i]);
    }
    if (node && i == 1) part[2] = double(accT);
    block_reduce<3, false>(part, red);
    if (k == 0 && i < NX) {
        gout[i] = i < IY ? R(double(accZ) / a.px[i]) : R(0);
        if (i == 0) gout[15] = R(double(accZ) / a.px[0]);  // m_wet is the initial mass
    }
    if (t == 0) {
        gout[16] = R(part[0]);
        gout[17] = R(part[1] + part[2]);
    }
}

// ------------------------------------------------------------------------------------------
template <typename R>
static hipError_t launch_grad_typed(const Config &cfg, int nsteps, int ckpt, const Problem &prob,
                                    const Record &rec, const void *cot, void *grad, void *fval,
                                    const Workspace &ws, const GradWorkspace &gw,
                                    hipStream_t stream)
{
    GradArgs<R> a;
    a.B = cfg.B;
    a.kmax = cfg.kmax;
    a.nsteps = nsteps;
    a.ckpt = ckpt;
    a.n_ckpt = (nsteps + ckpt - 1) / ckpt;
    a.rk4_substeps = cfg.rk4_substeps;
    a.node_projections = cfg.node_projections;
    a.w_cost = cfg.w_cost;
    a.w_prox = cfg.w_prox;
    a.w_ep = cfg.w_ep;
    a.omega = cfg.omega;
    a.rho = cfg.rho;
    for (int q = 0; q < NX; ++q) a.px[q] = cfg.px[q];
    for (int q = 0; q < NU; ++q) a.pu[q] = cfg.pu[q];
    a.x0 = static_cast<const R *>(prob.x0);
    a.xf = static_cast<const R *>(prob.xf);
    a.params = static_cast<const R *>(prob.params);
    a.K = prob.K;
    a.xbar = static_cast<const R *>(rec.xbar);
    a.ubar = static_cast<const R *>(rec.ubar);
    a.mup = static_cast<const R *>(rec.mup);
    a.mum = static_cast<const R *>(rec.mum);
    a.phi = static_cast<const R *>(rec.phi);
    a.th = static_cast<const R *>(rec.th);
    a.sigma = rec.sigma;
    a.cot = static_cast<const R *>(cot);
    a.grad = static_cast<R *>(grad);
    a.fval = static_cast<R *>(fval);
    a.blocks = static_cast<const R *>(ws.blocks);
    a.what = static_cast<const R *>(ws.what);
    a.dblk = static_cast<R *>(gw.dblk);
    a.dwhat = static_cast<R *>(gw.dwhat);
    a.tape = static_cast<R *>(gw.tape);
    a.gstat = gw.gstat;
    a.rk4_reverse = cfg.grad_rk4_tangent ? 0 : 1;
    a.pbar = gw.pbar;
    if (cfg.B == 0) return hipSuccess;

    hipError_t e;
    grad_status_kernel<<<dim3((unsigned)((cfg.B + 255) / 256)), dim3(256), 0, stream>>>(
        prob.K, cfg.B, cfg.kmax, gw.gstat);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_discretize_at(cfg, rec.xbar, rec.ubar, prob, gw.gstat, ws, stream)) !=
        hipSuccess)
        return e;
    if (!a.rk4_reverse) {
        const long nd = (long)cfg.B * (cfg.kmax - 1) * COLS;
        tangent_kernel<R><<<dim3((unsigned)((nd + 63) / 64)), dim3(64), 0, stream>>>(a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const int threads = qp_block_threads(cfg.kmax);
    const size_t smem = grad_smem_bytes_r(cfg.kmax, sizeof(R));
    // the workgroup-size bound sets the register budget: the 320- and 512-lane bounds (k_max <=
    // 20, <= 32) leave room for the kernel's per-lane state without spilling (FP32)
    if (threads <= 320)
        grad_kernel<R, 320><<<dim3(cfg.B), dim3(threads), smem, stream>>>(a);
    else if (threads <= 512)
        grad_kernel<R, 512><<<dim3(cfg.B), dim3(threads), smem, stream>>>(a);
    else if (threads <= 640)
        grad_kernel<R, 640><<<dim3(cfg.B), dim3(threads), smem, stream>>>(a);
    else
        grad_kernel<R, 1024><<<dim3(cfg.B), dim3(threads), smem, stream>>>(a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (a.rk4_reverse) {
        const long nl = (long)cfg.B * (cfg.kmax - 1) * 32;
        rk4_adjoint_kernel<R><<<dim3((unsigned)((nl + 63) / 64)), dim3(64), 0, stream>>>(a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        grad_finalize_kernel<R><<<dim3((unsigned)((cfg.B + 255) / 256)), dim3(256), 0, stream>>>(a);
    }
    return hipGetLastError();
}

hipError_t launch_grad(const Config &cfg, int nsteps, int ckpt, const Problem &prob,
                       const Record &rec, const void *cot, void *grad, void *fval,
                       const Workspace &ws, const GradWorkspace &gw, hipStream_t stream)
{
    if (cfg.dtype == 1)
        return launch_grad_typed<double>(cfg, nsteps, ckpt, prob, rec, cot, grad, fval, ws, gw,
                                         stream);
    return launch_grad_typed<float>(cfg, nsteps, ckpt, prob, rec, cot, grad, fval, ws, gw, stream);
}

size_t grad_smem_bytes(int dtype, int kmax)
{
    const size_t b = grad_smem_bytes_r(kmax, dtype == 1 ? 8 : 4);
    return b <= 65536 ? b : 0;
}

}  // namespace scp
