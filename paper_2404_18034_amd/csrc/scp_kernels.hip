// scp_kernels.hip -- HIP kernels of the batched prox-linear SCP solver for gfx950.
//
// One SCP iteration is two launches:
//   discretize_kernel  one lane per (instance, interval, column of [A | B- | B+]): RK4 on the
//                      state and on one column of the variational equations (section
//                      "Gradient of Discretized Dynamics"), then the prescaling of that
//                      column (subsection "Convex Subproblem with Prescaling and
//                      Preconditioning"); lane 0 of each interval also writes the scaled
//                      defect w^_k and the CTCS increment.
//   subproblem_kernel  one workgroup per instance: convergence test of the current
//                      reference, the customized power iteration (FP64), PIPG_custom with
//                      its projections and stopping rule, and the reference update.  The
//                      instance's blocks stay in registers for all PIPG iterations; the
//                      iterates that neighbouring nodes exchange live in LDS.
// Per-instance results never depend on other instances, and every reduction has a fixed
// order, so repeated runs are bitwise identical.
#include <math.h>

#include "lander_model.hpp"
#include "scp_kernels.hpp"

namespace scp {

constexpr int COLS = 23;         // columns of [A^- | B^- | B^+]
constexpr int CST = 16;          // stride of one column (15 rows + pad)
constexpr int BLK = COLS * CST;  // entries per interval
constexpr int VST = 20;          // node stride of (x, u) vectors in LDS (15 + 4 + pad)
constexpr int DST = 16;          // interval stride of dual vectors

// Final boundary condition: r, v, (q2, q3) and w are imposed; m, (q0, q1) and y are free.
__device__ __forceinline__ bool final_fixed(int i) { return i >= 1 && i <= 13 && i != 7 && i != 8; }

template <typename R>
struct Args {
    int B, kmax, j;  // j: 1-based SCP iteration of this launch
    int scp_iters_max, pipg_iters_max, pipg_check_every, rk4_substeps, power_iters_max;
    int early_exit, node_projections;
    double scp_tol, feas_tol, pipg_eps_abs, pipg_eps_rel;
    double power_eps_abs, power_eps_rel, power_buff;
    double w_cost, w_prox, w_ep, omega, rho;
    double px[NX], pu[NU];
    const R *x0, *xf, *params;
    const int32_t *K;
    R *x, *u, *t_f, *m_f;
    int32_t *status, *scp_iters, *pipg_iters;
    double *defect_inf, *ctcs_viol, *objective;
    R *blocks, *what, *mup, *mum, *phi, *th;
    double *dy, *step;
    int32_t *pipg_total;
};

// ------------------------------------------------------------------------------------------
// Initial guess (straight-line interpolation of r, v, w, normalized interpolation of q,
// constant mass, hover thrust along the body axis, s = s_init) and state reset.
// ------------------------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(256) init_kernel(Args<R> a)
{
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int b = (int)(gid / a.kmax), k = (int)(gid % a.kmax);
    if (b >= a.B) return;
    const int K = a.K[b];
    const bool valid = K >= 2 && K <= a.kmax;
    R *x = a.x + ((long)b * a.kmax + k) * NX;
    R *u = a.u + ((long)b * a.kmax + k) * NU;
    if (k < a.kmax - 1) {
        const long o = ((long)b * (a.kmax - 1) + k) * DST;
        for (int i = 0; i < DST; ++i) a.mup[o + i] = a.mum[o + i] = a.phi[o + i] = R(0);
    }
    a.th[(long)b * a.kmax + k] = R(0);
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
        for (int i = 0; i < NU; ++i) u[i] = R(0);
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
    u[0] = R(double(x0[0]) * sqrt(g0 * g0 + g1 * g1 + g2 * g2));
    u[1] = R(0);
    u[2] = R(0);
    u[3] = p[21];
}

// ------------------------------------------------------------------------------------------
// Discretization: lane (b, k, c) integrates x and column c of [Phi_x | Phi_u- | Phi_u+] over
// interval k with rk4_substeps RK4 steps; every lane of an interval integrates the same x
// (identical instruction stream, so identical bits).
// ------------------------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(128) discretize_kernel(Args<R> a, int need_blocks)
{
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long per_b = (long)(a.kmax - 1) * COLS;
    const int b = (int)(gid / per_b);
    if (b >= a.B) return;
    const int rem = (int)(gid % per_b), k = rem / COLS, c = rem % COLS;
    if (a.status[b] >= 0) return;
    const int K = a.K[b];
    if (k >= K - 1) return;
    if (!need_blocks && c != 0) return;

    const R *p = a.params + (long)b * NP;
    const Vehicle<R> V = load_vehicle<R>(p);
    const R *xk = a.x + ((long)b * a.kmax + k) * NX;
    const R *xk1 = xk + NX;
    const R *uk = a.u + ((long)b * a.kmax + k) * NU;
    const R *uk1 = uk + NU;

    // the state is accumulated in double (the model and the variational columns run in R),
    // which keeps the propagated endpoint -- and so the defect w^_k -- free of R-rounding
    // accumulated over the RK4 stages
    double x[NX];
    R col[NX];
    for (int i = 0; i < NX; ++i) {
        x[i] = double(xk[i]);
        col[i] = (c < NX && i == c) ? R(1) : R(0);
    }
    R ua[NU], ub[NU];
    for (int i = 0; i < NU; ++i) {
        ua[i] = uk[i];
        ub[i] = uk1[i];
    }
    // direction of the control perturbation: e_j scaled by lambda- (B- columns) or lambda+
    const int uj = c < NX ? -1 : (c - NX) % NU;
    const bool plus = c >= NX + NU;

    const R dtau = R(1.0 / double(K - 1));
    const int nsub = a.rk4_substeps;
    const R h = dtau / R(nsub);
    const R hh = R(0.5) * h;
    const R h6 = h / R(6);
    const double hd = double(h), hhd = double(hh), h6d = double(h6);

    double xs[NX], accx[NX];
    R xin[NX], cs[NX], accc[NX], fx[NX], fc[NX], u[NU], du[NU];
    double fy;

    for (int n = 0; n < nsub; ++n) {
        const R sig = R(n) * h;
        for (int st = 0; st < 4; ++st) {
            const R sg = st == 0 ? sig : (st == 3 ? sig + h : sig + hh);
            const R lp = sg / dtau, lm = R(1) - lp;
            for (int i = 0; i < NU; ++i) {
                u[i] = lm * ua[i] + lp * ub[i];
                du[i] = (i == uj) ? (plus ? lp : lm) : R(0);
            }
            for (int i = 0; i < NX; ++i) xin[i] = R(st == 0 ? x[i] : xs[i]);
            const R *cin = st == 0 ? col : cs;
            f_jvp<R, true>(V, xin, u, cin, du, fx, fy, fc);
            fx[IY] = R(0);  // y is advanced with the double-precision fy below
            if (st == 0) {
                for (int i = 0; i < IY; ++i) accx[i] = double(fx[i]);
                accx[IY] = fy;
                for (int i = 0; i < NX; ++i) accc[i] = fc[i];
            } else {
                const R wgt = st == 3 ? R(1) : R(2);
                for (int i = 0; i < IY; ++i) accx[i] += double(wgt) * double(fx[i]);
                accx[IY] += double(wgt) * fy;
                for (int i = 0; i < NX; ++i) accc[i] += wgt * fc[i];
            }
            if (st < 3) {
                const R hs = st == 2 ? h : hh;
                const double hsd = st == 2 ? hd : hhd;
                for (int i = 0; i < IY; ++i) xs[i] = x[i] + hsd * double(fx[i]);
                xs[IY] = x[IY] + hsd * fy;
                for (int i = 0; i < NX; ++i) cs[i] = col[i] + hs * fc[i];
            }
        }
        for (int i = 0; i < NX; ++i) {
            x[i] = x[i] + h6d * accx[i];
            col[i] = col[i] + h6 * accc[i];
        }
    }

    const long ib = (long)b * (a.kmax - 1) + k;
    if (need_blocks) {
        R *dst = a.blocks + ib * BLK + c * CST;
        const double pc = c < NX ? a.px[c] : a.pu[(c - NX) % NU];
        for (int i = 0; i < NX; ++i) dst[i] = R(double(col[i]) * pc / a.px[i]);
        dst[NX] = R(0);
    }
    if (c == 0) {
        R *w = a.what + ib * DST;
        for (int i = 0; i < NX; ++i) w[i] = R((x[i] - double(xk1[i])) / a.px[i]);
        w[NX] = R(0);
        a.dy[ib] = x[IY] - double(xk[IY]);
    }
}

// ------------------------------------------------------------------------------------------
// Workgroup reductions with a fixed combination order (deterministic).
// ------------------------------------------------------------------------------------------
template <int N, bool MAX>
__device__ __forceinline__ void block_reduce(double (&v)[N], double *red)
{
    for (int o = 32; o > 0; o >>= 1)
        for (int q = 0; q < N; ++q) {
            const double w = __shfl_xor(v[q], o, 64);
            v[q] = MAX ? fmax(v[q], w) : v[q] + w;
        }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0)
        for (int q = 0; q < N; ++q) red[wave * N + q] = v[q];
    __syncthreads();
    for (int q = 0; q < N; ++q) {
        double r = red[q];
        for (int w = 1; w < nw; ++w) r = MAX ? fmax(r, red[w * N + q]) : r + red[w * N + q];
        v[q] = r;
    }
}

// Node-wise convex sets (original units); component `j` of group member `which`.
template <typename R>
__device__ __forceinline__ R proj_soc_comp(R t, R z0, R z1, R a, int which)
{
    // second-order cone {(t, z) : ||z|| <= a t}; returns component 0 (t), 1 or 2 (z)
    const R nz = sqrt(z0 * z0 + z1 * z1);
    if (nz <= a * t) return which == 0 ? t : (which == 1 ? z0 : z1);
    if (a * nz <= -t) return R(0);
    const R tp = (t + a * nz) / (R(1) + a * a);
    if (which == 0) return tp;
    return a * tp * (which == 1 ? z0 : z1) / nz;
}

// ------------------------------------------------------------------------------------------
// Subproblem kernel.  Thread t of the workgroup of instance b:
//   t < 15K:          state variable (k, i) = (t / 15, t % 15) of node k for the primal
//                     step; for k < K-1 also dynamics row (k, i) for the dual step.
//   15K <= t < 19K:   control variable (k, j) = ((t - 15K) / 4, (t - 15K) % 4).
// ------------------------------------------------------------------------------------------
template <typename R, int MAXT>
__global__ void __launch_bounds__(MAXT) subproblem_kernel(Args<R> a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int b = blockIdx.x;
    if (b >= a.B) return;
    if (a.status[b] >= 0) return;  // uniform over the workgroup
    const int K = a.K[b], M = K - 1, kmax = a.kmax;
    const int t = threadIdx.x;

    // LDS carve (doubles first for alignment)
    double *red = reinterpret_cast<double *>(smem_raw);           // [16 waves * 8]
    double *dZ = red + 128;                                        // [kmax][VST]
    double *dPhi = dZ + kmax * VST;                                // [kmax-1][DST]
    double *dTh = dPhi + (kmax - 1) * DST;                         // [kmax]
    R *sPhi = reinterpret_cast<R *>(dTh + kmax);                   // [kmax-1][DST]
    R *sTh = sPhi + (kmax - 1) * DST;                              // [kmax]
    R *sV = sTh + kmax;                                            // [kmax][VST]
    R *sPre = sV + kmax * VST;                                     // [kmax][VST]

    const bool isx = t < NX * K;
    const bool isu = !isx && t < (NX + NU) * K;
    const bool prim = isx || isu;
    const int pk = isx ? t / NX : (isu ? (t - NX * K) / NU : 0);
    const int pj = isx ? t % NX : (isu ? NX + (t - NX * K) % NU : 0);  // 0..18 within node
    const bool dual = t < NX * M;
    const int dk = t / NX, di = t % NX;
    const long xoff = ((long)b * kmax + pk) * NX;
    const long uoff = ((long)b * kmax + pk) * NU;
    const double pscale = isx ? a.px[pj] : (isu ? a.pu[pj - NX] : 1.0);

    // -------------------- convergence test of the current reference --------------------
    // (scaled defect, CTCS increment, objective; status and outputs when the instance ends)
    {
        double mx[2] = {0.0, -INFINITY};
        double sm[2] = {0.0, 0.0};
        if (dual) {
            const R w = a.what[((long)b * (kmax - 1) + dk) * DST + di];
            const double e = fabs(double(w));
            mx[0] = isfinite(e) ? e : INFINITY;
            sm[0] = e;
            if (di == 0) mx[1] = a.dy[(long)b * (kmax - 1) + dk];
        }
        if (prim) {
            const R v = isx ? a.x[xoff + pj] : a.u[uoff + pj - NX];
            if (!isfinite(double(v))) sm[1] = 1.0;
        }
        if (dual && !isfinite(mx[0])) sm[1] = 1.0;
        block_reduce<2, true>(mx, red);
        block_reduce<2, false>(sm, red);
        const double d = mx[0], c = mx[1];
        const double step = a.step[b];
        const bool bad = sm[1] > 0.0 || !isfinite(d) || (a.j > 1 && !isfinite(step));
        const double eps = double(a.params[(long)b * NP + 20]);
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
                for (int k = 0; k < M; ++k)
                    tf += dtau * 0.5 *
                          (double(a.u[((long)b * kmax + k) * NU + 3]) +
                           double(a.u[((long)b * kmax + k + 1) * NU + 3]));
                a.t_f[b] = R(tf);
                a.m_f[b] = R(mN);
            }
            return;
        }
    }

    // -------------------- load the subproblem into registers --------------------
    const R *blk = a.blocks + (long)b * (kmax - 1) * BLK;
    R c1[NX], c2[NX], row[COLS];
    // primal: c1 = column pj of A^-_k (state) or of B^-_k (control); c2 = column of B^+_{k-1}
    for (int i = 0; i < NX; ++i) {
        c1[i] = R(0);
        c2[i] = R(0);
    }
    if (prim && pk < M)
        for (int i = 0; i < NX; ++i) c1[i] = blk[(long)pk * BLK + pj * CST + i];
    if (isu && pk > 0)
        for (int i = 0; i < NX; ++i) c2[i] = blk[(long)(pk - 1) * BLK + (pj + NU) * CST + i];
    // dual: row di of [A^-_k | B^-_k | B^+_k]
    for (int j = 0; j < COLS; ++j) row[j] = dual ? blk[(long)dk * BLK + j * CST + di] : R(0);

    const R *p = a.params + (long)b * NP;
    // boundary values and bounds of this primal variable
    bool fixed = false;
    R fixv = R(0), lo = R(-INFINITY), hi = R(INFINITY), xb = R(0);
    if (isx) {
        xb = a.x[xoff + pj];
        if (pk == 0) {
            fixed = true;
            const double zi = pj < IY ? double(a.x0[(long)b * NX + pj]) : 0.0;
            fixv = R((zi - double(xb)) / a.px[pj]);
        } else if (pk == K - 1 && final_fixed(pj)) {
            fixed = true;
            fixv = R((double(a.xf[(long)b * NXF + pj - 1]) - double(xb)) / a.px[pj]);
        }
    } else if (isu) {
        xb = a.u[uoff + pj - NX];
        if (pj == NX + 3) {
            lo = R((double(p[18]) - double(xb)) / a.pu[3]);
            hi = R((double(p[19]) - double(xb)) / a.pu[3]);
        }
    }
    R wk = R(0), epsk = R(0);
    if (dual) {
        wk = a.what[((long)b * (kmax - 1) + dk) * DST + di];
        if (di == IY) {
            const double y0 = double(a.x[((long)b * kmax + dk) * NX + IY]);
            const double y1 = double(a.x[((long)b * kmax + dk + 1) * NX + IY]);
            epsk = R((double(p[20]) - (y1 - y0)) / a.px[IY]);
        }
    }

    // -------------------- customized power iteration (FP64) --------------------
    double sigma;
    {
        double z = 1.0, mp = 1.0, mm = 1.0;
        double acc[1] = {(prim ? 1.0 : 0.0) + (dual ? 2.0 : 0.0)};
        block_reduce<1, false>(acc, red);
        sigma = sqrt(acc[0]);
        double sstar = sigma;
        for (int it = 1; it <= a.power_iters_max; ++it) {
            if (prim) dZ[pk * VST + pj] = z;
            __syncthreads();
            double ph = 0.0;
            if (dual) {
                double r = 0.0;
                for (int j = 0; j < NX; ++j) r += double(row[j]) * dZ[dk * VST + j];
                r -= dZ[(dk + 1) * VST + di];
                for (int j = 0; j < NU; ++j) {
                    r += double(row[NX + j]) * dZ[dk * VST + NX + j];
                    r += double(row[NX + NU + j]) * dZ[(dk + 1) * VST + NX + j];
                }
                r += mp - mm;
                ph = r / sigma;
                dPhi[dk * DST + di] = ph;
                if (di == IY) dTh[dk] = (dZ[(dk + 1) * VST + IY] - dZ[dk * VST + IY]) / sigma;
            }
            __syncthreads();
            if (prim) {
                double r = 0.0;
                if (pk < M)
                    for (int i = 0; i < NX; ++i) r += double(c1[i]) * dPhi[pk * DST + i];
                if (isx) {
                    if (pk > 0) r -= dPhi[(pk - 1) * DST + pj];
                    if (pj == IY) {
                        if (pk < M) r -= dTh[pk];
                        if (pk > 0) r += dTh[pk - 1];
                    }
                } else if (pk > 0) {
                    for (int i = 0; i < NX; ++i) r += double(c2[i]) * dPhi[(pk - 1) * DST + i];
                }
                z = r;
            }
            if (dual) {
                mp = ph;
                mm = -ph;
            }
            double sq[1] = {(prim ? z * z : 0.0) + (dual ? mp * mp + mm * mm : 0.0)};
            block_reduce<1, false>(sq, red);
            sstar = sqrt(sq[0]);
            if (fabs(sstar - sigma) <= a.power_eps_abs + a.power_eps_rel * fmax(sstar, sigma))
                break;
            else if (it < a.power_iters_max)
                sigma = sstar;
        }
        sigma = (1.0 + a.power_buff) * sstar;
    }
    const double alpha_d = 2.0 / (a.w_prox + sqrt(a.w_prox * a.w_prox + 4.0 * a.omega * sigma));
    const R alpha = R(alpha_d), beta = R(a.omega * alpha_d), rho = R(a.rho);
    const R omr = R(1) - rho;
    const R wprox = R(a.w_prox), wep = R(a.w_ep);
    const R cost = (isx && pk == K - 1 && pj == 0) ? R(-a.w_cost) : R(0);  // e_cost = -e_m

    // -------------------- PIPG_custom --------------------
    // warm start: x^, u^ = 0; mu+-, phi, theta from the previous subproblem
    R xt = R(0), xh = R(0), xprev = R(0);
    R vphi = R(0), ph = R(0), phprev = R(0);
    R nup = R(0), num = R(0), mup = R(0), mum = R(0), mupprev = R(0), mumprev = R(0);
    R vth = R(0), th = R(0), thprev = R(0);
    const long doff = ((long)b * (kmax - 1) + dk) * DST + di;
    if (dual) {
        mup = nup = mupprev = a.mup[doff];
        mum = num = mumprev = a.mum[doff];
        ph = vphi = phprev = a.phi[doff];
        sPhi[dk * DST + di] = vphi;
        if (di == IY) {
            th = vth = thprev = a.th[(long)b * kmax + dk];
            sTh[dk] = vth;
        }
    }
    __syncthreads();

    const int jmax = a.pipg_iters_max;
    const int check = a.early_exit ? a.pipg_check_every : 0;
    const bool nodeproj = a.node_projections != 0;
    // projection group of this primal variable: 0 none, 1 mass, 2 glide-slope cone on r,
    // 3 tilt disk on (q2, q3), 4 rate ball on w, 5 thrust cone and ball on T
    int grp = 0, gbase = 0;
    const int pmask = a.node_projections;
    if (nodeproj && prim && !fixed) {
        if (isx) {
            if (pj == 0) grp = (pmask & 1) ? 1 : 0;
            else if (pj <= 3) { grp = (pmask & 2) ? 2 : 0; gbase = 1; }
            else if (pj == 9 || pj == 10) { grp = (pmask & 4) ? 3 : 0; gbase = 9; }
            else if (pj >= 11 && pj <= 13) { grp = (pmask & 8) ? 4 : 0; gbase = 11; }
        } else if (pj < NX + 3) {
            grp = (pmask & 16) ? 5 : 0;
            gbase = NX;
        }
    }
    // reference values of the group (original units) and its scale
    R gref[3] = {R(0), R(0), R(0)};
    if (grp >= 2) {
        const R *src = grp == 5 ? a.u + uoff : a.x + xoff + gbase;
        gref[0] = src[0];
        gref[1] = src[1];
        gref[2] = grp == 3 ? R(0) : src[2];
    }
    const R gsc = R(pscale);
    const R tan_g = R(tan(double(p[15]))), tan_d = R(tan(double(p[14])));
    const R disk = R(sqrt(0.5 * (1.0 - cos(double(p[16]))))), wmax = p[17], Tmax = p[13];
    const R mdry = p[1];

    int it = 1;
    for (; it <= jmax; ++it) {
        // ---- projected gradient step on the primal variables ----
        R xn = R(0);
        if (prim) {
            R g = wprox * xt + cost;
            if (pk < M)
                for (int i = 0; i < NX; ++i) g += c1[i] * sPhi[pk * DST + i];
            if (isx) {
                if (pk > 0) g -= sPhi[(pk - 1) * DST + pj];
                if (pj == IY) {
                    if (pk < M) g -= sTh[pk];
                    if (pk > 0) g += sTh[pk - 1];
                }
                xn = xt - alpha * g;
            } else {
                if (pk > 0)
                    for (int i = 0; i < NX; ++i) g += c2[i] * sPhi[(pk - 1) * DST + i];
                xn = fmin(fmax(xt - alpha * g, lo), hi);
            }
        }
        if (nodeproj) {
            if (prim) sPre[pk * VST + pj] = xn;
            __syncthreads();
            if (grp == 1) {
                R m = xb + gsc * xn;
                m = m < mdry ? mdry : m;
                xn = (m - xb) / gsc;
            } else if (grp >= 2) {
                const int w = pj - gbase;
                R o0 = gref[0] + gsc * sPre[pk * VST + gbase];
                R o1 = gref[1] + gsc * sPre[pk * VST + gbase + 1];
                R o2 = grp == 3 ? R(0) : gref[2] + gsc * sPre[pk * VST + gbase + 2];
                R o;
                if (grp == 2) {
                    o = proj_soc_comp<R>(o0, o1, o2, R(1) / tan_g, w);
                } else if (grp == 5) {
                    // cone {||(T1,T2)|| <= tan(delta) T0}, then the ball ||T|| <= T_max
                    const R t0 = proj_soc_comp<R>(o0, o1, o2, tan_d, 0);
                    const R t1 = proj_soc_comp<R>(o0, o1, o2, tan_d, 1);
                    const R t2 = proj_soc_comp<R>(o0, o1, o2, tan_d, 2);
                    const R n = sqrt(t0 * t0 + t1 * t1 + t2 * t2);
                    const R sc = n > Tmax ? Tmax / n : R(1);
                    o = (w == 0 ? t0 : (w == 1 ? t1 : t2)) * sc;
                } else {
                    const R n = grp == 3 ? sqrt(o0 * o0 + o1 * o1) : sqrt(o0 * o0 + o1 * o1 + o2 * o2);
                    const R rad = grp == 3 ? disk : wmax;
                    const R sc = n > rad ? rad / n : R(1);
                    o = (w == 0 ? o0 : (w == 1 ? o1 : o2)) * sc;
                }
                const R gw = w == 0 ? gref[0] : (w == 1 ? gref[1] : gref[2]);
                xn = (o - gw) / gsc;
            }
        }
        if (fixed) xn = fixv;
        if (prim) {
            sV[pk * VST + pj] = R(2) * xn - xt;
            xt = omr * xt + rho * xn;
        }
        __syncthreads();
        // ---- dual (proportional-integral) step ----
        R phn = R(0), thn = R(0), mupn = R(0), mumn = R(0);
        if (dual) {
            mupn = nup - alpha * (wep + vphi);
            mumn = num - alpha * (wep - vphi);
            mupn = mupn > R(0) ? mupn : R(0);
            mumn = mumn > R(0) ? mumn : R(0);
            R r = R(0);
            for (int j = 0; j < NX; ++j) r += row[j] * sV[dk * VST + j];
            r -= sV[(dk + 1) * VST + di];
            for (int j = 0; j < NU; ++j) {
                r += row[NX + j] * sV[dk * VST + NX + j];
                r += row[NX + NU + j] * sV[(dk + 1) * VST + NX + j];
            }
            r += (R(2) * mupn - nup) - (R(2) * mumn - num);
            r += wk;
            phn = vphi + beta * r;
            if (di == IY) {
                const R tt = vth + beta * (sV[(dk + 1) * VST + IY] - sV[dk * VST + IY] - epsk);
                thn = tt > R(0) ? tt : R(0);
            }
            vphi = omr * vphi + rho * phn;
            nup = omr * nup + rho * mupn;
            num = omr * num + rho * mumn;
            sPhi[dk * DST + di] = vphi;
            if (di == IY) {
                vth = omr * vth + rho * thn;
                sTh[dk] = vth;
            }
        }
        bool done = false;
        if (check > 0 && it % check == 0) {
            // infinity norms of (x, u, mu+, mu-) and of (phi, theta) at j+1 and j
            double nz[6] = {0, 0, 0, 0, 0, 0};
            if (prim) {
                nz[0] = fabs(double(xn));
                nz[1] = fabs(double(xprev));
                nz[2] = fabs(double(xn) - double(xprev));
            }
            if (dual) {
                nz[0] = fmax(nz[0], fmax(fabs(double(mupn)), fabs(double(mumn))));
                nz[1] = fmax(nz[1], fmax(fabs(double(mupprev)), fabs(double(mumprev))));
                nz[2] = fmax(nz[2], fmax(fabs(double(mupn) - double(mupprev)),
                                         fabs(double(mumn) - double(mumprev))));
                nz[3] = fabs(double(phn));
                nz[4] = fabs(double(phprev));
                nz[5] = fabs(double(phn) - double(phprev));
                if (di == IY) {
                    nz[3] = fmax(nz[3], fabs(double(thn)));
                    nz[4] = fmax(nz[4], fabs(double(thprev)));
                    nz[5] = fmax(nz[5], fabs(double(thn) - double(thprev)));
                }
            }
            block_reduce<6, true>(nz, red);
            done = nz[2] <= a.pipg_eps_abs + a.pipg_eps_rel * fmax(nz[0], nz[1]) &&
                   nz[5] <= a.pipg_eps_abs + a.pipg_eps_rel * fmax(nz[3], nz[4]);
        }
        xprev = xn;
        xh = xn;
        if (dual) {
            mupprev = mupn;
            mumprev = mumn;
            phprev = phn;
            mup = mupn;
            mum = mumn;
            ph = phn;
            if (di == IY) {
                thprev = thn;
                th = thn;
            }
        }
        __syncthreads();
        if (done) {
            ++it;
            break;
        }
    }
    const int iters = it - 1;

    // -------------------- reference update and warm start --------------------
    double st[1] = {prim ? fabs(double(xh)) : 0.0};
    if (isx) a.x[xoff + pj] = R(double(xb) + a.px[pj] * double(xh));
    if (isu) a.u[uoff + pj - NX] = R(double(xb) + a.pu[pj - NX] * double(xh));
    if (dual) {
        a.mup[doff] = mup;
        a.mum[doff] = mum;
        a.phi[doff] = ph;
        if (di == IY) a.th[(long)b * kmax + dk] = th;
    }
    block_reduce<1, true>(st, red);
    if (t == 0) {
        a.step[b] = st[0];
        a.pipg_total[b] += iters;
    }
}

// ------------------------------------------------------------------------------------------
int qp_block_threads(int kmax) { return ((NX + NU) * kmax + 63) / 64 * 64; }

static size_t qp_smem_bytes(int kmax, size_t rsize)
{
    return sizeof(double) * (128 + kmax * VST + (kmax - 1) * DST + kmax) +
           rsize * ((kmax - 1) * DST + kmax + 2 * kmax * VST);
}

template <typename R>
static hipError_t launch_typed(const Config &cfg, const Problem &prob, const Solution &sol,
                               const Workspace &ws, hipStream_t stream, LaunchTimer *timer)
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
    for (int i = 0; i < NX; ++i) a.px[i] = cfg.px[i];
    for (int i = 0; i < NU; ++i) a.pu[i] = cfg.pu[i];
    a.x0 = static_cast<const R *>(prob.x0);
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
    a.pipg_total = ws.pipg_total;

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
        init_kernel<R><<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream>>>(a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = mark(0, false)) != hipSuccess) return e;
    }
    const long nd = (long)cfg.B * (cfg.kmax - 1) * COLS;
    const int qthreads = qp_block_threads(cfg.kmax);
    const size_t smem = qp_smem_bytes(cfg.kmax, sizeof(R));
    for (int j = 1; j <= cfg.scp_iters_max + 1; ++j) {
        a.j = j;
        const int need_blocks = j <= cfg.scp_iters_max ? 1 : 0;
        if ((e = mark(1, true)) != hipSuccess) return e;
        discretize_kernel<R><<<dim3((unsigned)((nd + 127) / 128)), dim3(128), 0, stream>>>(
            a, need_blocks);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = mark(1, false)) != hipSuccess) return e;
        if ((e = mark(2, true)) != hipSuccess) return e;
        if (qthreads <= 640)
            subproblem_kernel<R, 640><<<dim3(cfg.B), dim3(qthreads), smem, stream>>>(a);
        else
            subproblem_kernel<R, 1024><<<dim3(cfg.B), dim3(qthreads), smem, stream>>>(a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = mark(2, false)) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_solve(const Config &cfg, const Problem &prob, const Solution &sol,
                        const Workspace &ws, hipStream_t stream, LaunchTimer *timer)
{
    if (cfg.dtype == 1) return launch_typed<double>(cfg, prob, sol, ws, stream, timer);
    return launch_typed<float>(cfg, prob, sol, ws, stream, timer);
}

}  // namespace scp
