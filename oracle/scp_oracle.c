/*
 * scp_oracle.c -- plain FP64 CPU oracle for batched prox-linear SCP with CTCS and the
 * customized PIPG solver, applied to free-final-time 6-DoF powered-descent guidance
 * (Chari, Kamath, Elango, Acikmese: "Fast Monte Carlo Analysis for 6-DoF Powered-Descent
 * Guidance via GPU-Accelerated Sequential Convex Programming").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference that the
 * GPU library is checked against.  It shares no code, header, table or helper with the
 * GPU library and must never be linked into it or called from its product path; only the
 * test-suite, the smoke check and the CPU-baseline leg of the benchmark may use it.
 *
 * Conventions (the paper's notation, 0-based indices in code):
 *   state  x = (m, r[3], v[3], q[4], w[3], y)   n_x = 15   (q Hamilton, scalar first)
 *   control u = (T[3], s)                       n_u = 4    (s = dilation factor), or with
 *           the reaction-control torque (built with -DNU=7) u = (T[3], gamma[3], s)
 *   nodes k = 0..N-1 (paper's 1..N), intervals k = 0..N-2.
 *   params p[24] = m_wet, m_dry, alpha_mdot, g[3], J_diag[3], r_T[3], T_min, T_max,
 *                  delta_max, gamma_gs, theta_max, omega_max, s_min, s_max, eps_ctcs, s_init,
 *                  v_max (+inf: no speed bound), gamma_max (torque bound; n_u = 7 only)
 *
 * Every floating-point operation is written out in double precision, compiled without
 * fast-math and without FMA contraction.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NX 15
#ifndef NU
#define NU 4 /* thrust and dilation; 7 adds the reaction-control torque */
#endif
#if NU != 4 && NU != 7
#error "NU must be 4 or 7"
#endif
#define IS (NU - 1) /* index of the dilation s in u */
#define NP 24
#define NG 9 /* rows of the path-constraint function g (the torque row is -1 when n_u = 4) */
#define NXF 13
#define IY 14 /* index of the CTCS integrator state y */

/* Below this norm a thrust vector (or the lateral position) is treated as zero when
 * differentiating ||.||: the derivative of the norm is taken as 0 there.  The node-wise
 * thrust projection can land exactly on T = 0, and a reference rebuilt from the scaled step
 * then holds T at rounding level; the threshold keeps the linearization continuous across
 * that rounding. */
#define NORM_EPS 1e-4

/* Final boundary condition E_f: r, v, the tilt part (q2, q3) of the attitude and the
 * transverse rates (w2, w3) are fixed; the roll angle part (q0, q1), the roll rate w1, the
 * mass and y are free.  Reading of "land upright at rest": with thrust as the only input the
 * torque r_T x T has no component about the thrust axis, so roll is not controllable and
 * neither its angle nor its rate can be prescribed (with unequal transverse inertias the
 * gyroscopic coupling drives w1, and a fixed w1 = 0 leaves a defect no iteration removes). */
static int final_fixed(int i) { return i >= 1 && i <= 13 && i != 7 && i != 8 && i != 11; }

enum {
    P_MWET = 0, P_MDRY = 1, P_ALPHA = 2, P_G = 3, P_J = 6, P_RT = 9, P_TMIN = 12, P_TMAX = 13,
    P_DELTA = 14, P_GAMMA = 15, P_THETA = 16, P_OMEGA = 17, P_SMIN = 18, P_SMAX = 19,
    P_EPS = 20, P_SINIT = 21, P_VMAX = 22, P_GMAX = 23
};

/* Solver settings; the same fields (in the same order) as the Python wrapper's struct. */
typedef struct {
    int32_t scp_iters_max;     /* maximum number of convex subproblems per solve        */
    int32_t pipg_iters_max;    /* j_max of the PIPG solver                               */
    int32_t pipg_check_every;  /* j_check of the stopping criterion                      */
    int32_t rk4_substeps;      /* RK4 steps per discretization interval                  */
    int32_t power_iters_max;   /* j_max of the power iteration                           */
    int32_t early_exit;        /* 1: SCP and PIPG stop on their tolerances; 0: fixed work */
    int32_t node_projections;  /* bitmask of node-wise convex sets: 1 dry mass, 2 glide slope,
                                  4 tilt, 8 rate, 16 thrust (gimbal cone and T_max); 0 none */
    int32_t scalar_dilation;   /* 1: one dilation value over the whole horizon (the per-node
                                  dilation controls of a subproblem constrained equal)   */
    double scp_tol, feas_tol;
    double pipg_eps_abs, pipg_eps_rel;
    double power_eps_abs, power_eps_rel, power_buff;
    double w_cost, w_prox, w_ep, omega, rho;
    double px[NX], pu[NU];
} orc_settings;

/* ------------------------------------------------------------------------------------------
 * 6-DoF model (section "6-DoF Powered Descent Guidance"): dynamics F and path constraints g,
 * augmented with the CTCS integrator (eq. sys-dyn-dil-aug): f(x,u) = s (F, sum [g]_+^2).
 * Readings: the torque input and the v_max row are dropped (the C0 vehicle has thrust only);
 * glide slope is tan(gamma_gs)*||(r2,r3)|| <= r1 with r1 the altitude; tilt is written as
 * 2(q2^2+q3^2) - (1 - cos theta_max) <= 0, i.e. C11(q) >= cos theta_max.
 * ------------------------------------------------------------------------------------------ */

/* Direction cosine matrix C_{I<-B}(q) for a unit Hamilton quaternion, scalar first. */
static void dcm(const double *q, double C[3][3])
{
    double q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3];
    C[0][0] = q0 * q0 + q1 * q1 - q2 * q2 - q3 * q3;
    C[0][1] = 2.0 * (q1 * q2 - q0 * q3);
    C[0][2] = 2.0 * (q1 * q3 + q0 * q2);
    C[1][0] = 2.0 * (q1 * q2 + q0 * q3);
    C[1][1] = q0 * q0 - q1 * q1 + q2 * q2 - q3 * q3;
    C[1][2] = 2.0 * (q2 * q3 - q0 * q1);
    C[2][0] = 2.0 * (q1 * q3 - q0 * q2);
    C[2][1] = 2.0 * (q2 * q3 + q0 * q1);
    C[2][2] = q0 * q0 - q1 * q1 - q2 * q2 + q3 * q3;
}

/* Omega(w): q_dot = 0.5 * Omega(w) q  (body rates, q_dot = 0.5 q (x) (0, w)). */
static void omega_mat(const double *w, double Om[4][4])
{
    double a = w[0], b = w[1], c = w[2];
    double M[4][4] = {{0, -a, -b, -c}, {a, 0, c, -b}, {b, -c, 0, a}, {c, b, -a, 0}};
    memcpy(Om, M, sizeof(M));
}

static double norm3(const double *a) { return sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]); }

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Path constraints g (9 rows: mass, glide slope, tilt, rate, gimbal, T_max, T_min, speed,
 * torque; the speed row ||v||^2 - v_max^2 of section "6-DoF Powered Descent Guidance" is the
 * constant -1 when v_max is not finite, i.e. there is no speed bound, and the torque row
 * ||gamma||^2 - gamma_max^2 likewise without a finite bound or without the torque input). */
static void constraints(const double *x, const double *u, const double *p, double *g)
{
    const double *r = x + 1, *v = x + 4, *q = x + 7, *w = x + 11;
    double Tn = norm3(u);
    double lat = sqrt(r[1] * r[1] + r[2] * r[2]);
    g[0] = p[P_MDRY] - x[0];
    g[1] = tan(p[P_GAMMA]) * lat - r[0];
    g[2] = 2.0 * (q[2] * q[2] + q[3] * q[3]) - (1.0 - cos(p[P_THETA]));
    g[3] = w[0] * w[0] + w[1] * w[1] + w[2] * w[2] - p[P_OMEGA] * p[P_OMEGA];
    g[4] = Tn - u[0] / cos(p[P_DELTA]);
    g[5] = Tn - p[P_TMAX];
    g[6] = p[P_TMIN] - Tn;
    g[7] = isfinite(p[P_VMAX]) ? v[0] * v[0] + v[1] * v[1] + v[2] * v[2] - p[P_VMAX] * p[P_VMAX]
                               : -1.0;
#if NU == 7
    g[8] = isfinite(p[P_GMAX]) ? u[3] * u[3] + u[4] * u[4] + u[5] * u[5] - p[P_GMAX] * p[P_GMAX]
                               : -1.0;
#else
    g[8] = -1.0;
#endif
}

/* Gradients of g w.r.t. x (9 x 15) and w.r.t. T (9 x 3).  d||v||/dv := 0 for ||v|| <= NORM_EPS.
 * The torque row's gradient w.r.t. gamma (2 gamma) is formed where it is used. */
static void constraint_grads(const double *x, const double *u, const double *p, double Gx[NG][NX],
                             double Gt[NG][3])
{
    const double *r = x + 1, *v = x + 4, *q = x + 7, *w = x + 11;
    double Tn = norm3(u);
    double lat = sqrt(r[1] * r[1] + r[2] * r[2]);
    double tg = tan(p[P_GAMMA]);
    double dT[3] = {0, 0, 0};
    int i;
    memset(Gx, 0, sizeof(double) * NG * NX);
    memset(Gt, 0, sizeof(double) * NG * 3);
    if (Tn > NORM_EPS)
        for (i = 0; i < 3; i++) dT[i] = u[i] / Tn;
    Gx[0][0] = -1.0;
    Gx[1][1] = -1.0;
    if (lat > NORM_EPS) {
        Gx[1][2] = tg * r[1] / lat;
        Gx[1][3] = tg * r[2] / lat;
    }
    Gx[2][9] = 4.0 * q[2];
    Gx[2][10] = 4.0 * q[3];
    for (i = 0; i < 3; i++) Gx[3][11 + i] = 2.0 * w[i];
    for (i = 0; i < 3; i++) {
        Gt[4][i] = dT[i];
        Gt[5][i] = dT[i];
        Gt[6][i] = -dT[i];
    }
    Gt[4][0] -= 1.0 / cos(p[P_DELTA]);
    if (isfinite(p[P_VMAX]))
        for (i = 0; i < 3; i++) Gx[7][4 + i] = 2.0 * v[i];
}

/* Augmented, time-dilated dynamics f(x,u) = s * (F(xi,zeta), sum_i [g_i]_+^2). */
void orc_dynamics(const double *x, const double *u, const double *p, double *f)
{
    const double *v = x + 4, *q = x + 7, *w = x + 11;
    const double *J = p + P_J, *rT = p + P_RT, *gI = p + P_G;
    double s = u[IS], m = x[0];
    double C[3][3], Om[4][4], g[NG];
    double Jw[3], wxJw[3], rxT[3];
    double F[NX];
    int i, j;

    dcm(q, C);
    omega_mat(w, Om);
    F[0] = -p[P_ALPHA] * norm3(u);
    for (i = 0; i < 3; i++) F[1 + i] = v[i];
    for (i = 0; i < 3; i++) {
        double a = 0.0;
        for (j = 0; j < 3; j++) a += C[i][j] * u[j];
        F[4 + i] = a / m + gI[i];
    }
    for (i = 0; i < 4; i++) {
        double a = 0.0;
        for (j = 0; j < 4; j++) a += Om[i][j] * q[j];
        F[7 + i] = 0.5 * a;
    }
    for (i = 0; i < 3; i++) Jw[i] = J[i] * w[i];
    cross3(w, Jw, wxJw);
    cross3(rT, u, rxT);
#if NU == 7
    /* the reaction-control torque gamma (body frame) joins the thrust torque */
    for (i = 0; i < 3; i++) F[11 + i] = (rxT[i] - wxJw[i] + u[3 + i]) / J[i];
#else
    for (i = 0; i < 3; i++) F[11 + i] = (rxT[i] - wxJw[i]) / J[i];
#endif
    constraints(x, u, p, g);
    F[IY] = 0.0;
    for (i = 0; i < NG; i++) {
        double gp = g[i] > 0.0 ? g[i] : 0.0;
        F[IY] += gp * gp;
    }
    for (i = 0; i < NX; i++) f[i] = s * F[i];
}

/* Analytic Jacobians A = df/dx (15x15, row-major) and B = df/du (15 x NU, row-major). */
void orc_jacobians(const double *x, const double *u, const double *p, double *A, double *B)
{
    const double *q = x + 7, *w = x + 11;
    const double *J = p + P_J, *rT = p + P_RT;
    double s = u[IS], m = x[0];
    double C[3][3], Om[4][4], g[NG], Gx[NG][NX], Gt[NG][3];
    double CT[3], dCT_dq[3][4], Xi[4][3];
    double F[NX], f[NX];
    double Tn = norm3(u);
    double qv_dot_T;
    int i, j;

    memset(A, 0, sizeof(double) * NX * NX);
    memset(B, 0, sizeof(double) * NX * NU);
    dcm(q, C);
    omega_mat(w, Om);
    for (i = 0; i < 3; i++) {
        CT[i] = 0.0;
        for (j = 0; j < 3; j++) CT[i] += C[i][j] * u[j];
    }
    /* d(C(q) T)/dq: column 0 = 2 q0 T + 2 qv x T; columns 1..3 =
       -2 T qv^T + 2 (qv.T) I + 2 qv T^T - 2 q0 [T x]. */
    {
        double qv[3] = {q[1], q[2], q[3]}, c[3], Tx[3][3];
        cross3(qv, u, c);
        qv_dot_T = qv[0] * u[0] + qv[1] * u[1] + qv[2] * u[2];
        Tx[0][0] = 0; Tx[0][1] = -u[2]; Tx[0][2] = u[1];
        Tx[1][0] = u[2]; Tx[1][1] = 0; Tx[1][2] = -u[0];
        Tx[2][0] = -u[1]; Tx[2][1] = u[0]; Tx[2][2] = 0;
        for (i = 0; i < 3; i++) {
            dCT_dq[i][0] = 2.0 * q[0] * u[i] + 2.0 * c[i];
            for (j = 0; j < 3; j++)
                dCT_dq[i][1 + j] = -2.0 * u[i] * qv[j] + (i == j ? 2.0 * qv_dot_T : 0.0) +
                                   2.0 * qv[i] * u[j] - 2.0 * q[0] * Tx[i][j];
        }
    }
    /* Xi(q): Omega(w) q = Xi(q) w. */
    Xi[0][0] = -q[1]; Xi[0][1] = -q[2]; Xi[0][2] = -q[3];
    Xi[1][0] = q[0];  Xi[1][1] = -q[3]; Xi[1][2] = q[2];
    Xi[2][0] = q[3];  Xi[2][1] = q[0];  Xi[2][2] = -q[1];
    Xi[3][0] = -q[2]; Xi[3][1] = q[1];  Xi[3][2] = q[0];

    /* Rows of dF/dx (multiplied by s below). */
    /* r_dot = v */
    for (i = 0; i < 3; i++) A[(1 + i) * NX + 4 + i] = 1.0;
    /* v_dot = C T / m + g */
    for (i = 0; i < 3; i++) {
        A[(4 + i) * NX + 0] = -CT[i] / (m * m);
        for (j = 0; j < 4; j++) A[(4 + i) * NX + 7 + j] = dCT_dq[i][j] / m;
    }
    /* q_dot = 0.5 Omega(w) q */
    for (i = 0; i < 4; i++) {
        for (j = 0; j < 4; j++) A[(7 + i) * NX + 7 + j] = 0.5 * Om[i][j];
        for (j = 0; j < 3; j++) A[(7 + i) * NX + 11 + j] = 0.5 * Xi[i][j];
    }
    /* w_dot = J^-1 (rT x T - w x J w):  d/dw = -J^-1 ([w x] J - [(J w) x]) */
    {
        double Jw[3] = {J[0] * w[0], J[1] * w[1], J[2] * w[2]};
        double Wx[3][3] = {{0, -w[2], w[1]}, {w[2], 0, -w[0]}, {-w[1], w[0], 0}};
        double JWx[3][3] = {{0, -Jw[2], Jw[1]}, {Jw[2], 0, -Jw[0]}, {-Jw[1], Jw[0], 0}};
        for (i = 0; i < 3; i++)
            for (j = 0; j < 3; j++)
                A[(11 + i) * NX + 11 + j] = -(Wx[i][j] * J[j] - JWx[i][j]) / J[i];
    }
    /* y_dot = sum_i [g_i]_+^2:  d/dx = sum_i 2 [g_i]_+ dg_i/dx */
    constraints(x, u, p, g);
    constraint_grads(x, u, p, Gx, Gt);
    for (i = 0; i < NG; i++) {
        double gp = g[i] > 0.0 ? g[i] : 0.0;
        for (j = 0; j < NX; j++) A[IY * NX + j] += 2.0 * gp * Gx[i][j];
    }
    for (i = 0; i < NX * NX; i++) A[i] *= s;

    /* dF/dT */
    if (Tn > NORM_EPS)
        for (j = 0; j < 3; j++) B[0 * NU + j] = -p[P_ALPHA] * u[j] / Tn;
    for (i = 0; i < 3; i++)
        for (j = 0; j < 3; j++) B[(4 + i) * NU + j] = C[i][j] / m;
    /* d(rT x T)/dT = [rT x] */
    {
        double Rx[3][3] = {{0, -rT[2], rT[1]}, {rT[2], 0, -rT[0]}, {-rT[1], rT[0], 0}};
        for (i = 0; i < 3; i++)
            for (j = 0; j < 3; j++) B[(11 + i) * NU + j] = Rx[i][j] / J[i];
    }
    for (i = 0; i < NG; i++) {
        double gp = g[i] > 0.0 ? g[i] : 0.0;
        for (j = 0; j < 3; j++) B[IY * NU + j] += 2.0 * gp * Gt[i][j];
    }
#if NU == 7
    /* the torque enters w_dot through J^-1, and the CTCS integrand through its bound row */
    for (i = 0; i < 3; i++) B[(11 + i) * NU + 3 + i] = 1.0 / J[i];
    {
        double gp = g[8] > 0.0 ? g[8] : 0.0;
        for (j = 0; j < 3; j++) B[IY * NU + 3 + j] += 2.0 * gp * (2.0 * u[3 + j]);
    }
#endif
    for (i = 0; i < NX; i++)
        for (j = 0; j < IS; j++) B[i * NU + j] *= s;
    /* df/ds = F */
    orc_dynamics(x, u, p, f);
    for (i = 0; i < NX; i++) F[i] = (s != 0.0) ? f[i] / s : 0.0;
    if (s == 0.0) { /* evaluate F directly when s = 0 */
        double u1[NU];
        for (j = 0; j < NU; j++) u1[j] = u[j];
        u1[IS] = 1.0;
        orc_dynamics(x, u1, p, F);
    }
    for (i = 0; i < NX; i++) B[i * NU + IS] = F[i];
}

void orc_constraints(const double *x, const double *u, const double *p, double *g)
{
    constraints(x, u, p, g);
}

/* ------------------------------------------------------------------------------------------
 * Linear time-invariant test model f = A0 x + B0 u (used only to pin the integrator against
 * closed forms).  The model is selected per call of orc_discretize_interval.
 * ------------------------------------------------------------------------------------------ */
typedef struct {
    int linear;        /* 0: 6-DoF lander; 1: linear test model */
    const double *p;   /* lander parameters                      */
    const double *A0;  /* linear model, 15x15 row-major          */
    const double *B0;  /* linear model, 15xNU row-major          */
} model_t;

static void model_f(const model_t *md, const double *x, const double *u, double *f)
{
    int i, j;
    if (!md->linear) {
        orc_dynamics(x, u, md->p, f);
        return;
    }
    for (i = 0; i < NX; i++) {
        double a = 0.0;
        for (j = 0; j < NX; j++) a += md->A0[i * NX + j] * x[j];
        for (j = 0; j < NU; j++) a += md->B0[i * NU + j] * u[j];
        f[i] = a;
    }
}

static void model_jac(const model_t *md, const double *x, const double *u, double *A, double *B)
{
    if (!md->linear) {
        orc_jacobians(x, u, md->p, A, B);
        return;
    }
    memcpy(A, md->A0, sizeof(double) * NX * NX);
    memcpy(B, md->B0, sizeof(double) * NX * NU);
}

/* ------------------------------------------------------------------------------------------
 * Discretization of one interval [tau_k, tau_k+1] (section "Gradient of Discretized
 * Dynamics"): the state and the variational equations
 *   Phi_x' = A Phi_x,  Phi_u-' = A Phi_u- + B lambda-,  Phi_u+' = A Phi_u+ + B lambda+,
 * with Phi_x(tau_k) = I, Phi_u+-(tau_k) = 0, a first-order-hold control, integrated jointly
 * with n_sub classical RK4 steps.  Output: x^k(tau_k+1), A_k, B_k-, B_k+.
 * The augmented state is X = (x[15], Phi_x[15x15], Phi_u-[15xNU], Phi_u+[15xNU]) (360 values for n_u = 4, 450 for 7).
 * ------------------------------------------------------------------------------------------ */
#define NAUG (NX + NX * NX + 2 * NX * NU)

static void aug_rhs(const model_t *md, double sig, double dtau, const double *uk, const double *uk1,
                    const double *X, double *dX)
{
    double lp = sig / dtau, lm = 1.0 - lp; /* FOH weights lambda+ and lambda- */
    double u[NU], A[NX * NX], B[NX * NU];
    const double *x = X, *Px = X + NX, *Pm = X + NX + NX * NX, *Pp = Pm + NX * NU;
    double *dx = dX, *dPx = dX + NX, *dPm = dX + NX + NX * NX, *dPp = dPm + NX * NU;
    int i, j, l;
    for (i = 0; i < NU; i++) u[i] = lm * uk[i] + lp * uk1[i];
    model_f(md, x, u, dx);
    model_jac(md, x, u, A, B);
    for (i = 0; i < NX; i++)
        for (j = 0; j < NX; j++) {
            double a = 0.0;
            for (l = 0; l < NX; l++) a += A[i * NX + l] * Px[l * NX + j];
            dPx[i * NX + j] = a;
        }
    for (i = 0; i < NX; i++)
        for (j = 0; j < NU; j++) {
            double am = 0.0, ap = 0.0;
            for (l = 0; l < NX; l++) {
                am += A[i * NX + l] * Pm[l * NU + j];
                ap += A[i * NX + l] * Pp[l * NU + j];
            }
            dPm[i * NU + j] = am + B[i * NU + j] * lm;
            dPp[i * NU + j] = ap + B[i * NU + j] * lp;
        }
}

static void discretize_interval(const model_t *md, const double *xk, const double *uk,
                                const double *uk1, double dtau, int nsub, double *xend, double *Ak,
                                double *Bmk, double *Bpk)
{
    double X[NAUG], Xs[NAUG], k1[NAUG], k2[NAUG], k3[NAUG], k4[NAUG];
    double h = dtau / nsub;
    int i, n;
    memset(X, 0, sizeof(X));
    memcpy(X, xk, sizeof(double) * NX);
    for (i = 0; i < NX; i++) X[NX + i * NX + i] = 1.0;
    for (n = 0; n < nsub; n++) {
        double sig = n * h;
        aug_rhs(md, sig, dtau, uk, uk1, X, k1);
        for (i = 0; i < NAUG; i++) Xs[i] = X[i] + 0.5 * h * k1[i];
        aug_rhs(md, sig + 0.5 * h, dtau, uk, uk1, Xs, k2);
        for (i = 0; i < NAUG; i++) Xs[i] = X[i] + 0.5 * h * k2[i];
        aug_rhs(md, sig + 0.5 * h, dtau, uk, uk1, Xs, k3);
        for (i = 0; i < NAUG; i++) Xs[i] = X[i] + h * k3[i];
        aug_rhs(md, sig + h, dtau, uk, uk1, Xs, k4);
        for (i = 0; i < NAUG; i++) X[i] = X[i] + (h / 6.0) * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    }
    memcpy(xend, X, sizeof(double) * NX);
    memcpy(Ak, X + NX, sizeof(double) * NX * NX);
    memcpy(Bmk, X + NX + NX * NX, sizeof(double) * NX * NU);
    memcpy(Bpk, X + NX + NX * NX + NX * NU, sizeof(double) * NX * NU);
}

/* Exported: one interval, lander (A0 == NULL) or linear test model (A0, B0 given). */
void orc_discretize_interval(const double *xk, const double *uk, const double *uk1,
                             const double *p, const double *A0, const double *B0, double dtau,
                             int nsub, double *xend, double *Ak, double *Bmk, double *Bpk)
{
    model_t md = {A0 != NULL, p, A0, B0};
    discretize_interval(&md, xk, uk, uk1, dtau, nsub, xend, Ak, Bmk, Bpk);
}

/* Exported: all K-1 intervals of one instance on the uniform grid tau_k = k/(K-1). */
void orc_discretize(int K, const double *xbar, const double *ubar, const double *p, int nsub,
                    double *xend, double *A, double *Bm, double *Bp)
{
    model_t md = {0, p, NULL, NULL};
    double dtau = 1.0 / (K - 1);
    int k;
    for (k = 0; k < K - 1; k++)
        discretize_interval(&md, xbar + k * NX, ubar + k * NU, ubar + (k + 1) * NU, dtau, nsub,
                            xend + k * NX, A + k * NX * NX, Bm + k * NX * NU, Bp + k * NX * NU);
}

/* ------------------------------------------------------------------------------------------
 * Initial guess (the paper leaves it open; reading): straight-line interpolation of r, v, w
 * from the initial to the final condition, normalized interpolation of q, constant mass m0,
 * y = 0, hover thrust along the body x axis T = (m0 ||g||, 0, 0), dilation s = s_init.
 * ------------------------------------------------------------------------------------------ */
void orc_init_guess(int K, const double *x0, const double *xf, const double *p, double *xbar,
                    double *ubar)
{
    double gn = norm3(p + P_G);
    int k, i;
    for (k = 0; k < K; k++) {
        double a = (double)k / (K - 1), b = 1.0 - a, qn = 0.0;
        double *x = xbar + k * NX, *u = ubar + k * NU;
        x[0] = x0[0];
        for (i = 1; i < 14; i++) x[i] = b * x0[i] + a * xf[i - 1];
        for (i = 7; i < 11; i++) qn += x[i] * x[i];
        qn = sqrt(qn);
        for (i = 7; i < 11; i++) x[i] /= qn;
        x[IY] = 0.0;
        for (i = 0; i < NU; i++) u[i] = 0.0;  /* the torque guess is zero */
        u[0] = x0[0] * gn;
        u[IS] = p[P_SINIT];
    }
}

/* ------------------------------------------------------------------------------------------
 * Scaled convex subproblem (eq. cvx-subproblem-custom) for one instance.
 * ------------------------------------------------------------------------------------------ */
typedef struct {
    int K;                 /* number of nodes N                                   */
    double *Am;            /* [K-1][15][15]  A_hat^-_k = Px^-1 A_k Px               */
    double *Bm, *Bp;       /* [K-1][15][NU]  B_hat^-+_k = Px^-1 B^-+_k Pu           */
    double *w;             /* [K-1][15]      w_hat_k = Px^-1 (x^k(tau_k+1) - x_k+1) */
    double *eps;           /* [K-1]          eps_hat_k                              */
    double *umin, *umax;   /* [K][NU]        scaled control bounds (+-inf but for s) */
    double zi[NX];         /* scaled initial condition (all 15 components)         */
    double zf[NXF];        /* scaled final condition on r, v, q, w                 */
    const double *xbar;    /* [K][15] reference state (node-wise sets only)         */
    const double *ubar;    /* [K][4]  reference control (node-wise sets only)       */
    const double *p;       /* vehicle parameters (node-wise sets only)              */
} qp_t;

/* Iterates of the customized PIPG solver (also the warm start). */
typedef struct {
    double *x;   /* [K][15] */
    double *u;   /* [K][4]  */
    double *mup; /* [K-1][15] mu^+ */
    double *mum; /* [K-1][15] mu^- */
    double *phi; /* [K-1][15] dual of the dynamics */
    double *th;  /* [K-1]     dual of the CTCS rows */
} iter_t;

static void iter_alloc(iter_t *it, int K)
{
    it->x = calloc((size_t)K * NX, sizeof(double));
    it->u = calloc((size_t)K * NU, sizeof(double));
    it->mup = calloc((size_t)(K - 1) * NX, sizeof(double));
    it->mum = calloc((size_t)(K - 1) * NX, sizeof(double));
    it->phi = calloc((size_t)(K - 1) * NX, sizeof(double));
    it->th = calloc((size_t)(K - 1), sizeof(double));
}

static void iter_free(iter_t *it)
{
    free(it->x); free(it->u); free(it->mup); free(it->mum); free(it->phi); free(it->th);
}

static void iter_copy(iter_t *dst, const iter_t *src, int K)
{
    memcpy(dst->x, src->x, sizeof(double) * K * NX);
    memcpy(dst->u, src->u, sizeof(double) * K * NU);
    memcpy(dst->mup, src->mup, sizeof(double) * (K - 1) * NX);
    memcpy(dst->mum, src->mum, sizeof(double) * (K - 1) * NX);
    memcpy(dst->phi, src->phi, sizeof(double) * (K - 1) * NX);
    memcpy(dst->th, src->th, sizeof(double) * (K - 1));
}

static void qp_alloc(qp_t *qp, int K)
{
    int M = K - 1;
    qp->K = K;
    qp->Am = calloc((size_t)M * NX * NX, sizeof(double));
    qp->Bm = calloc((size_t)M * NX * NU, sizeof(double));
    qp->Bp = calloc((size_t)M * NX * NU, sizeof(double));
    qp->w = calloc((size_t)M * NX, sizeof(double));
    qp->eps = calloc((size_t)M, sizeof(double));
    qp->umin = calloc((size_t)K * NU, sizeof(double));
    qp->umax = calloc((size_t)K * NU, sizeof(double));
}

static void qp_free(qp_t *qp)
{
    free(qp->Am); free(qp->Bm); free(qp->Bp); free(qp->w); free(qp->eps);
    free(qp->umin); free(qp->umax);
}

/* Prescaling and preconditioning (subsection "Convex Subproblem with Prescaling and
 * Preconditioning").  A, Bm, Bp, xend come from the discretization at (xbar, ubar). */
static void build_qp(const orc_settings *st, const double *p, int K, const double *x0,
                     const double *xf, const double *xbar, const double *ubar, const double *xend,
                     const double *A, const double *Bm, const double *Bp, qp_t *qp)
{
    const double *px = st->px, *pu = st->pu;
    int M = K - 1, k, i, j;
    for (k = 0; k < M; k++) {
        for (i = 0; i < NX; i++) {
            for (j = 0; j < NX; j++)
                qp->Am[(k * NX + i) * NX + j] = A[(k * NX + i) * NX + j] * px[j] / px[i];
            for (j = 0; j < NU; j++) {
                qp->Bm[(k * NX + i) * NU + j] = Bm[(k * NX + i) * NU + j] * pu[j] / px[i];
                qp->Bp[(k * NX + i) * NU + j] = Bp[(k * NX + i) * NU + j] * pu[j] / px[i];
            }
            qp->w[k * NX + i] = (xend[k * NX + i] - xbar[(k + 1) * NX + i]) / px[i];
        }
        qp->eps[k] = (p[P_EPS] - (xbar[(k + 1) * NX + IY] - xbar[k * NX + IY])) / px[IY];
    }
    for (k = 0; k < K; k++) {
        for (j = 0; j < IS; j++) { /* only the dilation is boxed */
            qp->umin[k * NU + j] = -INFINITY;
            qp->umax[k * NU + j] = INFINITY;
        }
        qp->umin[k * NU + IS] = (p[P_SMIN] - ubar[k * NU + IS]) / pu[IS];
        qp->umax[k * NU + IS] = (p[P_SMAX] - ubar[k * NU + IS]) / pu[IS];
    }
    for (i = 0; i < NX; i++) {
        double zi = (i < IY) ? x0[i] : 0.0; /* (z_i, 0): y(0) = 0 */
        qp->zi[i] = (zi - xbar[i]) / px[i];
    }
    for (i = 0; i < NXF; i++) qp->zf[i] = (xf[i] - xbar[(K - 1) * NX + 1 + i]) / px[1 + i];
    qp->xbar = xbar;
    qp->ubar = ubar;
    qp->p = p;
}

static double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* ------------------------------------------------------------------------------------------
 * Customized power iteration (Algorithm "Customized power iteration method").  It estimates
 * the largest eigenvalue of K^T K with K = [G_hat; H_hat_y] acting on (x, u, mu+, mu-),
 * starting from the all-ones vector.  Readings: the printed v_k in the transpose step is the
 * CTCS dual theta_k, and sigma* accumulates onto itself for the last node.
 * ------------------------------------------------------------------------------------------ */
static double sumsq(const iter_t *z, int K)
{
    double a = 0.0;
    int i;
    for (i = 0; i < K * NX; i++) a += z->x[i] * z->x[i];
    for (i = 0; i < K * NU; i++) a += z->u[i] * z->u[i];
    for (i = 0; i < (K - 1) * NX; i++) a += z->mup[i] * z->mup[i] + z->mum[i] * z->mum[i];
    return a;
}

static double power_iteration(const orc_settings *st, const qp_t *qp, int *iters_out)
{
    int K = qp->K, M = K - 1, k, i, j, it;
    iter_t z;
    double *phi = calloc((size_t)M * NX, sizeof(double));
    double *th = calloc((size_t)M, sizeof(double));
    double sigma, sigma_star = 0.0;
    iter_alloc(&z, K);
    for (i = 0; i < K * NX; i++) z.x[i] = 1.0;
    for (i = 0; i < K * NU; i++) z.u[i] = 1.0;
    for (i = 0; i < M * NX; i++) z.mup[i] = z.mum[i] = 1.0;
    sigma = sqrt(sumsq(&z, K));
    for (it = 1; it <= st->power_iters_max; it++) {
        /* forward: phi_k = (A-_k x_k - x_k+1 + B-_k u_k + B+_k u_k+1 + mu+_k - mu-_k) / sigma */
        for (k = 0; k < M; k++) {
            for (i = 0; i < NX; i++) {
                double a = 0.0;
                for (j = 0; j < NX; j++) a += qp->Am[(k * NX + i) * NX + j] * z.x[k * NX + j];
                a -= z.x[(k + 1) * NX + i];
                for (j = 0; j < NU; j++) {
                    a += qp->Bm[(k * NX + i) * NU + j] * z.u[k * NU + j];
                    a += qp->Bp[(k * NX + i) * NU + j] * z.u[(k + 1) * NU + j];
                }
                a += z.mup[k * NX + i] - z.mum[k * NX + i];
                phi[k * NX + i] = a / sigma;
            }
            th[k] = (z.x[(k + 1) * NX + IY] - z.x[k * NX + IY]) / sigma;
        }
        /* transpose */
        for (k = 0; k < K; k++) {
            for (j = 0; j < NX; j++) {
                double a = 0.0;
                if (k < M)
                    for (i = 0; i < NX; i++) a += qp->Am[(k * NX + i) * NX + j] * phi[k * NX + i];
                if (k > 0) a -= phi[(k - 1) * NX + j]; /* A_hat^+ = -I */
                if (j == IY) {
                    if (k < M) a -= th[k];
                    if (k > 0) a += th[k - 1];
                }
                z.x[k * NX + j] = a;
            }
            for (j = 0; j < NU; j++) {
                double a = 0.0;
                if (k < M)
                    for (i = 0; i < NX; i++) a += qp->Bm[(k * NX + i) * NU + j] * phi[k * NX + i];
                if (k > 0)
                    for (i = 0; i < NX; i++)
                        a += qp->Bp[((k - 1) * NX + i) * NU + j] * phi[(k - 1) * NX + i];
                z.u[k * NU + j] = a;
            }
        }
        for (i = 0; i < M * NX; i++) {
            z.mup[i] = phi[i];
            z.mum[i] = -phi[i];
        }
        sigma_star = sqrt(sumsq(&z, K));
        if (fabs(sigma_star - sigma) <=
            st->power_eps_abs + st->power_eps_rel * (sigma_star > sigma ? sigma_star : sigma))
            break;
        else if (it < st->power_iters_max)
            sigma = sigma_star;
    }
    if (iters_out) *iters_out = it > st->power_iters_max ? st->power_iters_max : it;
    iter_free(&z);
    free(phi);
    free(th);
    return (1.0 + st->power_buff) * sigma_star;
}

/* ------------------------------------------------------------------------------------------
 * Customized stopping criterion (Algorithm "Customized stopping criterion evaluation"):
 * infinity-norm change of the primal (x, u, mu+, mu-) and dual (phi, theta) iterates between
 * iterations j+1 and j, relative to their infinity norms.
 * ------------------------------------------------------------------------------------------ */
static void inf_norms(const double *a, const double *b, int n, double *na, double *nb, double *nd)
{
    int i;
    for (i = 0; i < n; i++) {
        double fa = fabs(a[i]), fb = fabs(b[i]), fd = fabs(a[i] - b[i]);
        if (fa > *na) *na = fa;
        if (fb > *nb) *nb = fb;
        if (fd > *nd) *nd = fd;
    }
}

static int stopping_custom(const iter_t *nw, const iter_t *od, int K, double eabs, double erel)
{
    int M = K - 1;
    double z1 = 0, z0 = 0, zd = 0, r1 = 0, r0 = 0, rd = 0;
    inf_norms(nw->x, od->x, K * NX, &z1, &z0, &zd);
    inf_norms(nw->u, od->u, K * NU, &z1, &z0, &zd);
    inf_norms(nw->mup, od->mup, M * NX, &z1, &z0, &zd);
    inf_norms(nw->mum, od->mum, M * NX, &z1, &z0, &zd);
    inf_norms(nw->phi, od->phi, M * NX, &r1, &r0, &rd);
    inf_norms(nw->th, od->th, M, &r1, &r0, &rd);
    return (zd <= eabs + erel * (z1 > z0 ? z1 : z0)) && (rd <= eabs + erel * (r1 > r0 ? r1 : r0));
}

/* ------------------------------------------------------------------------------------------
 * Optional node-wise convex sets (flag node_projections): Euclidean projections, in the
 * original units, of the node state and control onto convex sets implied by the path
 * constraints.  They are applied to x_hat, u_hat through x = xbar + Px x_hat and
 * u = ubar + Pu u_hat; every set acts on a block whose scale factors are equal, so the
 * projection in scaled coordinates is the same point.  T_min is not convex and stays with
 * the CTCS integrator only.
 * ------------------------------------------------------------------------------------------ */

/* Projection onto the second-order cone {(t, z) : ||z|| <= a t}, z in R^n. */
static void proj_soc(double *t, double *z, int n, double a)
{
    double nz = 0.0;
    int i;
    for (i = 0; i < n; i++) nz += z[i] * z[i];
    nz = sqrt(nz);
    if (nz <= a * *t) return;
    if (a * nz <= -*t) { /* inside the polar cone: the apex */
        *t = 0.0;
        for (i = 0; i < n; i++) z[i] = 0.0;
        return;
    }
    {
        /* closest point on the cone surface: t' = (t + a nz) / (1 + a^2), z' = a t' z/||z|| */
        double tp = (*t + a * nz) / (1.0 + a * a);
        for (i = 0; i < n; i++) z[i] = a * tp * z[i] / nz;
        *t = tp;
    }
}

/* Projection onto the ball ||z|| <= rad. */
static void proj_ball(double *z, int n, double rad)
{
    double nz = 0.0;
    int i;
    for (i = 0; i < n; i++) nz += z[i] * z[i];
    nz = sqrt(nz);
    if (nz > rad)
        for (i = 0; i < n; i++) z[i] *= rad / nz;
}

/* State sets (mask bits 1, 2, 4, 8): m >= m_dry, glide-slope cone on r, tilt disk on
 * (q2, q3), rate ball on w, at an interior node. */
static void project_state(double *xh, const double *xb, const double *px, const double *p,
                          int mask)
{
    double x[NX];
    int i;
    for (i = 0; i < NX; i++) x[i] = xb[i] + px[i] * xh[i];
    if ((mask & 1) && x[0] < p[P_MDRY]) x[0] = p[P_MDRY];
    if (mask & 2) proj_soc(&x[1], &x[2], 2, 1.0 / tan(p[P_GAMMA]));
    if (mask & 4) proj_ball(&x[9], 2, sqrt(0.5 * (1.0 - cos(p[P_THETA]))));
    if (mask & 8) proj_ball(&x[11], 3, p[P_OMEGA]);
    for (i = 0; i < NX; i++) xh[i] = (x[i] - xb[i]) / px[i];
}

/* The same sets at the last node, intersected with the final boundary condition: the fixed
 * components already hold their values (r, v, (q2, q3) and (w2, w3) are fixed), so the
 * glide-slope cone and the tilt disk have nothing left to project; the mass bound acts on
 * the free mass, and the rate ball on the free roll rate w1 through the fixed transverse
 * rates: |w1| <= sqrt(w_max^2 - w2^2 - w3^2) (zero when the fixed rates alone leave the
 * ball), which is the Euclidean projection onto the ball's slice. */
static void project_state_final(double *xh, const double *xb, const double *px,
                                const double *p, int mask)
{
    double x[NX];
    int i;
    for (i = 0; i < NX; i++) x[i] = xb[i] + px[i] * xh[i];
    if ((mask & 1) && x[0] < p[P_MDRY]) x[0] = p[P_MDRY];
    if (mask & 8) {
        double r2 = p[P_OMEGA] * p[P_OMEGA] - x[12] * x[12] - x[13] * x[13];
        double r = r2 > 0.0 ? sqrt(r2) : 0.0;
        x[11] = clampd(x[11], -r, r);
    }
    for (i = 0; i < NX; i++) xh[i] = (x[i] - xb[i]) / px[i];
}

/* Thrust set: gimbal cone ||T|| cos(delta_max) <= T1 intersected with ||T|| <= T_max
 * (cone first, then the ball centred at the cone's apex: exact for this pair). */
static void project_thrust(double *uh, const double *ub, const double *pu, const double *p)
{
    double T[3];
    int i;
    for (i = 0; i < 3; i++) T[i] = ub[i] + pu[i] * uh[i];
    proj_soc(&T[0], &T[1], 2, tan(p[P_DELTA]));
    proj_ball(T, 3, p[P_TMAX]);
    for (i = 0; i < 3; i++) uh[i] = (T[i] - ub[i]) / pu[i];
}

/* ------------------------------------------------------------------------------------------
 * PIPG_custom (Algorithm "PIPG_custom").  Starts from the warm start ws (overwritten with the
 * returned primal-dual solution).  Readings: the u-gradient at interior nodes uses the
 * dynamics dual phi_{k-1}; mu+ descends along w_ep + phi_k and mu- along w_ep - phi_k (the
 * dynamics rows carry +mu+ and -mu-); the cost vector e_cost = -e_m (propellant optimal).
 * Returns the number of iterations performed.
 * ------------------------------------------------------------------------------------------ */
static int pipg_custom(const orc_settings *st, const qp_t *qp, double sigma, int jmax, int check,
                       iter_t *ws)
{
    int K = qp->K, M = K - 1, k, i, j, it, done = 0;
    double alpha = 2.0 / (st->w_prox + sqrt(st->w_prox * st->w_prox + 4.0 * st->omega * sigma));
    double beta = st->omega * alpha, rho = st->rho;
    iter_t tl, hat, prev; /* extrapolated (tilde/nu/varphi/vartheta), fresh, previous fresh */
    double ecost[NX];
    memset(ecost, 0, sizeof(ecost));
    ecost[0] = -1.0;
    iter_alloc(&tl, K);
    iter_alloc(&hat, K);
    iter_alloc(&prev, K);
    iter_copy(&tl, ws, K);
    iter_copy(&prev, ws, K);
    iter_copy(&hat, ws, K);

    for (it = 1; it <= jmax && !done; it++) {
        /* projected gradient step on the primal variables */
        for (k = 0; k < K; k++) {
            for (j = 0; j < NX; j++) {
                double gr = st->w_prox * tl.x[k * NX + j];
                if (k < M)
                    for (i = 0; i < NX; i++) gr += qp->Am[(k * NX + i) * NX + j] * tl.phi[k * NX + i];
                if (k > 0) gr -= tl.phi[(k - 1) * NX + j];
                if (j == IY) {
                    if (k < M) gr -= tl.th[k];
                    if (k > 0) gr += tl.th[k - 1];
                }
                if (k == K - 1) gr += st->w_cost * ecost[j];
                hat.x[k * NX + j] = tl.x[k * NX + j] - alpha * gr;
            }
            /* boundary values (the first node is fixed entirely), then the node-wise state
             * sets on what is left free */
            if (k == 0)
                for (j = 0; j < NX; j++) hat.x[j] = qp->zi[j];
            if (k == K - 1 && k > 0)
                for (j = 0; j < NXF; j++)
                    if (final_fixed(1 + j)) hat.x[k * NX + 1 + j] = qp->zf[j];
            if ((st->node_projections & 15) && k > 0 && k < K - 1)
                project_state(hat.x + k * NX, qp->xbar + k * NX, st->px, qp->p,
                              st->node_projections);
            if ((st->node_projections & 9) && k > 0 && k == K - 1)
                project_state_final(hat.x + k * NX, qp->xbar + k * NX, st->px, qp->p,
                                    st->node_projections);
            for (j = 0; j < NU; j++) {
                double gr = st->w_prox * tl.u[k * NU + j];
                if (k < M)
                    for (i = 0; i < NX; i++) gr += qp->Bm[(k * NX + i) * NU + j] * tl.phi[k * NX + i];
                if (k > 0)
                    for (i = 0; i < NX; i++)
                        gr += qp->Bp[((k - 1) * NX + i) * NU + j] * tl.phi[(k - 1) * NX + i];
                hat.u[k * NU + j] = tl.u[k * NU + j] - alpha * gr;
                if (!(st->scalar_dilation && j == NU - 1))
                    hat.u[k * NU + j] = clampd(hat.u[k * NU + j], qp->umin[k * NU + j],
                                               qp->umax[k * NU + j]);
            }
            if (st->node_projections & 16)
                project_thrust(hat.u + k * NU, qp->ubar + k * NU, st->pu, qp->p);
        }
        if (st->scalar_dilation) {
            /* one dilation value: the Euclidean projection of the K fresh dilation values
             * onto {s_1 = ... = s_K} intersected with every node's box is their mean,
             * clamped to the intersection of the boxes */
            double mean = 0.0, lo = -INFINITY, hi = INFINITY;
            for (k = 0; k < K; k++) {
                mean += hat.u[k * NU + NU - 1];
                lo = fmax(lo, qp->umin[k * NU + NU - 1]);
                hi = fmin(hi, qp->umax[k * NU + NU - 1]);
            }
            mean = clampd(mean / K, lo, hi);
            for (k = 0; k < K; k++) hat.u[k * NU + NU - 1] = mean;
        }
        for (i = 0; i < M * NX; i++) {
            double a = tl.mup[i] - alpha * (st->w_ep + tl.phi[i]);
            double b = tl.mum[i] - alpha * (st->w_ep - tl.phi[i]);
            hat.mup[i] = a > 0.0 ? a : 0.0;
            hat.mum[i] = b > 0.0 ? b : 0.0;
        }
        /* proportional-integral feedback of the constraint violation (dual step) */
        for (k = 0; k < M; k++) {
            for (i = 0; i < NX; i++) {
                double r = 0.0;
                for (j = 0; j < NX; j++)
                    r += qp->Am[(k * NX + i) * NX + j] * (2.0 * hat.x[k * NX + j] - tl.x[k * NX + j]);
                r -= 2.0 * hat.x[(k + 1) * NX + i] - tl.x[(k + 1) * NX + i];
                for (j = 0; j < NU; j++) {
                    r += qp->Bm[(k * NX + i) * NU + j] * (2.0 * hat.u[k * NU + j] - tl.u[k * NU + j]);
                    r += qp->Bp[(k * NX + i) * NU + j] *
                         (2.0 * hat.u[(k + 1) * NU + j] - tl.u[(k + 1) * NU + j]);
                }
                r += (2.0 * hat.mup[k * NX + i] - tl.mup[k * NX + i]) -
                     (2.0 * hat.mum[k * NX + i] - tl.mum[k * NX + i]);
                r += qp->w[k * NX + i];
                hat.phi[k * NX + i] = tl.phi[k * NX + i] + beta * r;
            }
            {
                double y1 = 2.0 * hat.x[(k + 1) * NX + IY] - tl.x[(k + 1) * NX + IY];
                double y0 = 2.0 * hat.x[k * NX + IY] - tl.x[k * NX + IY];
                double t = tl.th[k] + beta * (y1 - y0 - qp->eps[k]);
                hat.th[k] = t > 0.0 ? t : 0.0;
            }
        }
        /* extrapolation */
        for (i = 0; i < K * NX; i++) tl.x[i] = (1.0 - rho) * tl.x[i] + rho * hat.x[i];
        for (i = 0; i < K * NU; i++) tl.u[i] = (1.0 - rho) * tl.u[i] + rho * hat.u[i];
        for (i = 0; i < M * NX; i++) {
            tl.mup[i] = (1.0 - rho) * tl.mup[i] + rho * hat.mup[i];
            tl.mum[i] = (1.0 - rho) * tl.mum[i] + rho * hat.mum[i];
            tl.phi[i] = (1.0 - rho) * tl.phi[i] + rho * hat.phi[i];
        }
        for (i = 0; i < M; i++) tl.th[i] = (1.0 - rho) * tl.th[i] + rho * hat.th[i];
        if (check > 0 && it % check == 0)
            done = stopping_custom(&hat, &prev, K, st->pipg_eps_abs, st->pipg_eps_rel);
        iter_copy(&prev, &hat, K);
    }
    iter_copy(ws, &hat, K);
    iter_free(&tl);
    iter_free(&hat);
    iter_free(&prev);
    return it - 1;
}

/* ------------------------------------------------------------------------------------------
 * Exported single-block entry points used by the tests (QP given in unscaled pieces).
 * ------------------------------------------------------------------------------------------ */

/* Build the scaled QP from a discretization and write its pieces out. */
void orc_build_qp(const orc_settings *st, const double *p, int K, const double *x0,
                  const double *xf, const double *xbar, const double *ubar, const double *xend,
                  const double *A, const double *Bm, const double *Bp, double *Am_o, double *Bm_o,
                  double *Bp_o, double *w_o, double *eps_o, double *umin_o, double *umax_o,
                  double *zi_o, double *zf_o)
{
    qp_t qp;
    int M = K - 1;
    qp_alloc(&qp, K);
    build_qp(st, p, K, x0, xf, xbar, ubar, xend, A, Bm, Bp, &qp);
    memcpy(Am_o, qp.Am, sizeof(double) * M * NX * NX);
    memcpy(Bm_o, qp.Bm, sizeof(double) * M * NX * NU);
    memcpy(Bp_o, qp.Bp, sizeof(double) * M * NX * NU);
    memcpy(w_o, qp.w, sizeof(double) * M * NX);
    memcpy(eps_o, qp.eps, sizeof(double) * M);
    memcpy(umin_o, qp.umin, sizeof(double) * K * NU);
    memcpy(umax_o, qp.umax, sizeof(double) * K * NU);
    memcpy(zi_o, qp.zi, sizeof(double) * NX);
    memcpy(zf_o, qp.zf, sizeof(double) * NXF);
    qp_free(&qp);
}

static void qp_view(qp_t *qp, int K, double *Am, double *Bm, double *Bp, double *w, double *eps,
                    double *umin, double *umax, const double *zi, const double *zf)
{
    qp->xbar = qp->ubar = qp->p = NULL;
    qp->K = K;
    qp->Am = Am; qp->Bm = Bm; qp->Bp = Bp; qp->w = w; qp->eps = eps;
    qp->umin = umin; qp->umax = umax;
    memcpy(qp->zi, zi, sizeof(double) * NX);
    memcpy(qp->zf, zf, sizeof(double) * NXF);
}

double orc_power(const orc_settings *st, int K, double *Am, double *Bm, double *Bp, int *iters)
{
    qp_t qp;
    double zi[NX] = {0}, zf[NXF] = {0};
    qp_view(&qp, K, Am, Bm, Bp, NULL, NULL, NULL, NULL, zi, zf);
    return power_iteration(st, &qp, iters);
}

/* PIPG on given scaled QP data; the warm start arrays are overwritten with the result. */
int orc_pipg(const orc_settings *st, int K, double *Am, double *Bm, double *Bp, double *w,
             double *eps, double *umin, double *umax, const double *zi, const double *zf,
             const double *xbar, const double *ubar, const double *p, double sigma, int jmax,
             int check, double *x, double *u, double *mup, double *mum, double *phi, double *th)
{
    qp_t qp;
    iter_t ws = {x, u, mup, mum, phi, th};
    qp_view(&qp, K, Am, Bm, Bp, w, eps, umin, umax, zi, zf);
    qp.xbar = xbar;
    qp.ubar = ubar;
    qp.p = p;
    if (st->node_projections && (!xbar || !ubar || !p)) return -1;
    return pipg_custom(st, &qp, sigma, jmax, check, &ws);
}

/* ------------------------------------------------------------------------------------------
 * Prox-linear SCP (subsection "Sequential Convex Programming") for one instance.
 * Each pass: discretize at the reference, test convergence, build the scaled QP, run the
 * power iteration and PIPG_custom (warm-started), and move the reference by the scaled step.
 * Readings: uniform grid; x_hat, u_hat warm-start at 0 (the previous solution expressed in
 * the new reference's coordinates) while mu+-, phi, theta carry over; converged when the
 * scaled step, the scaled defect and the scaled CTCS excess are all below tolerance.
 * status: 0 converged, 1 iteration limit, 2 non-finite value.
 * ------------------------------------------------------------------------------------------ */
typedef struct {
    double tf, mf, defect, ctcs, objective, step;
    int32_t status, scp_iters, pipg_iters;
} orc_result;

/* Saved state of the last SCP iteration for the truncated map used by gradient checks. */
typedef struct {
    double *xbar, *ubar;  /* reference before the last subproblem   [K][15], [K][4]         */
    double *ws;           /* warm start before the last subproblem  (packed iter_t layout) */
    double sigma;         /* buffered power-iteration estimate of the last subproblem       */
    int valid;
} orc_lastiter;

static int iter_len(int K) { return K * NX + K * NU + 3 * (K - 1) * NX + (K - 1); }

static void iter_pack(const iter_t *it, int K, double *buf)
{
    int M = K - 1;
    memcpy(buf, it->x, sizeof(double) * K * NX); buf += K * NX;
    memcpy(buf, it->u, sizeof(double) * K * NU); buf += K * NU;
    memcpy(buf, it->mup, sizeof(double) * M * NX); buf += M * NX;
    memcpy(buf, it->mum, sizeof(double) * M * NX); buf += M * NX;
    memcpy(buf, it->phi, sizeof(double) * M * NX); buf += M * NX;
    memcpy(buf, it->th, sizeof(double) * M);
}

static void iter_unpack(iter_t *it, int K, const double *buf)
{
    int M = K - 1;
    memcpy(it->x, buf, sizeof(double) * K * NX); buf += K * NX;
    memcpy(it->u, buf, sizeof(double) * K * NU); buf += K * NU;
    memcpy(it->mup, buf, sizeof(double) * M * NX); buf += M * NX;
    memcpy(it->mum, buf, sizeof(double) * M * NX); buf += M * NX;
    memcpy(it->phi, buf, sizeof(double) * M * NX); buf += M * NX;
    memcpy(it->th, buf, sizeof(double) * M);
}

static int finite_arr(const double *a, int n)
{
    int i;
    for (i = 0; i < n; i++)
        if (!isfinite(a[i])) return 0;
    return 1;
}

/* One instance.  xinit / uinit (NULL: the initial guess of orc_init_guess), when given, are
 * the first reference trajectory, [K][NX] and [K][NU]. */
static void scp_solve_one(const orc_settings *st, int K, const double *x0, const double *xf,
                          const double *p, const double *xinit, const double *uinit,
                          double *xbar, double *ubar, orc_result *res, orc_lastiter *last,
                          int trace_n, double *trace)
{
    int M = K - 1, j, k, i, total_pipg = 0, solves = 0, status = 1;
    double dtau = 1.0 / M, step = INFINITY, d = 0.0, c = 0.0, obj = 0.0;
    double *xend = malloc(sizeof(double) * M * NX);
    double *A = malloc(sizeof(double) * M * NX * NX);
    double *Bm = malloc(sizeof(double) * M * NX * NU);
    double *Bp = malloc(sizeof(double) * M * NX * NU);
    qp_t qp;
    iter_t ws;
    qp_alloc(&qp, K);
    iter_alloc(&ws, K);
    orc_init_guess(K, x0, xf, p, xbar, ubar);
    if (xinit) memcpy(xbar, xinit, sizeof(double) * K * NX);
    if (uinit) memcpy(ubar, uinit, sizeof(double) * K * NU);

    for (j = 1; j <= st->scp_iters_max + 1; j++) {
        int pit, conv;
        orc_discretize(K, xbar, ubar, p, st->rk4_substeps, xend, A, Bm, Bp);
        /* FP64 convergence quantities at the current reference */
        d = 0.0;
        c = -INFINITY;
        obj = -xbar[(K - 1) * NX + 0];
        for (k = 0; k < M; k++) {
            double dy = xend[k * NX + IY] - xbar[k * NX + IY];
            for (i = 0; i < NX; i++) {
                double e = fabs(xend[k * NX + i] - xbar[(k + 1) * NX + i]) / st->px[i];
                if (e > d) d = e;
                obj += st->w_ep * e;
            }
            if (dy > c) c = dy;
        }
        if (!finite_arr(xbar, K * NX) || !finite_arr(ubar, K * NU) || !finite_arr(xend, M * NX) ||
            !isfinite(step) && j > 1) {
            status = 2;
            break;
        }
        conv = (j > 1) && step <= st->scp_tol && d <= st->feas_tol &&
               (c - p[P_EPS]) / st->px[IY] <= st->feas_tol;
        if (j > st->scp_iters_max || (st->early_exit && conv)) {
            status = conv ? 0 : 1;
            break;
        }
        build_qp(st, p, K, x0, xf, xbar, ubar, xend, A, Bm, Bp, &qp);
        {
            double sigma = power_iteration(st, &qp, NULL);
            if (last && j == st->scp_iters_max) {
                memcpy(last->xbar, xbar, sizeof(double) * K * NX);
                memcpy(last->ubar, ubar, sizeof(double) * K * NU);
                iter_pack(&ws, K, last->ws);
                last->sigma = sigma;
                last->valid = 1;
            }
            for (i = 0; i < K * NX; i++) ws.x[i] = 0.0;
            for (i = 0; i < K * NU; i++) ws.u[i] = 0.0;
            pit = pipg_custom(st, &qp, sigma, st->pipg_iters_max,
                              st->early_exit ? st->pipg_check_every : 0, &ws);
        }
        total_pipg += pit;
        solves++;
        step = 0.0;
        for (k = 0; k < K; k++) {
            for (i = 0; i < NX; i++) {
                xbar[k * NX + i] += st->px[i] * ws.x[k * NX + i];
                if (fabs(ws.x[k * NX + i]) > step) step = fabs(ws.x[k * NX + i]);
            }
            for (i = 0; i < NU; i++) {
                ubar[k * NU + i] += st->pu[i] * ws.u[k * NU + i];
                if (fabs(ws.u[k * NU + i]) > step) step = fabs(ws.u[k * NU + i]);
            }
        }
        if (trace && j <= trace_n) {
            trace[(j - 1) * 4 + 0] = step;
            trace[(j - 1) * 4 + 1] = d;
            trace[(j - 1) * 4 + 2] = c;
            trace[(j - 1) * 4 + 3] = (double)pit;
        }
    }
    res->tf = 0.0;
    for (k = 0; k < M; k++) res->tf += dtau * 0.5 * (ubar[k * NU + IS] + ubar[(k + 1) * NU + IS]);
    res->mf = xbar[(K - 1) * NX + 0];
    res->defect = d;
    res->ctcs = c;
    res->objective = obj;
    res->step = step;
    res->status = status;
    res->scp_iters = solves;
    res->pipg_iters = total_pipg;
    free(xend); free(A); free(Bm); free(Bp);
    qp_free(&qp);
    iter_free(&ws);
}

/* ------------------------------------------------------------------------------------------
 * Batch API: instances are independent; a pthread pool takes instance i = t, t+T, ...
 * Output arrays: x[B][kmax][15], u[B][kmax][4] (rows >= K_b are zero); scalars per instance.
 * ------------------------------------------------------------------------------------------ */
typedef struct {
    const orc_settings *st;
    int B, kmax, nthreads, tid;
    const double *x0, *xf, *p;
    const int32_t *K;
    double *x, *u, *tf, *mf, *defect, *ctcs, *objective;
    int32_t *status, *scp_iters, *pipg_iters;
    double *step; /* optional (NULL): scaled step of the last subproblem solved */
    const double *xinit, *uinit; /* optional (NULL): first reference, [B][kmax][NX], [NU] */
} batch_job;

static void *batch_worker(void *arg)
{
    batch_job *jb = (batch_job *)arg;
    int b;
    for (b = jb->tid; b < jb->B; b += jb->nthreads) {
        int K = jb->K[b];
        double *xb = jb->x + (size_t)b * jb->kmax * NX, *ub = jb->u + (size_t)b * jb->kmax * NU;
        orc_result r;
        memset(xb, 0, sizeof(double) * jb->kmax * NX);
        memset(ub, 0, sizeof(double) * jb->kmax * NU);
        scp_solve_one(jb->st, K, jb->x0 + (size_t)b * NX, jb->xf + (size_t)b * NXF,
                      jb->p + (size_t)b * NP,
                      jb->xinit ? jb->xinit + (size_t)b * jb->kmax * NX : NULL,
                      jb->uinit ? jb->uinit + (size_t)b * jb->kmax * NU : NULL, xb, ub, &r, NULL,
                      0, NULL);
        jb->tf[b] = r.tf;
        jb->mf[b] = r.mf;
        jb->defect[b] = r.defect;
        jb->ctcs[b] = r.ctcs;
        jb->objective[b] = r.objective;
        jb->status[b] = r.status;
        jb->scp_iters[b] = r.scp_iters;
        jb->pipg_iters[b] = r.pipg_iters;
        if (jb->step) jb->step[b] = r.step;
    }
    return NULL;
}

int orc_solve_batch(const orc_settings *st, int B, int kmax, const double *x0, const double *xf,
                    const double *p, const int32_t *K, int nthreads, double *x, double *u,
                    double *tf, double *mf, int32_t *status, int32_t *scp_iters,
                    int32_t *pipg_iters, double *defect, double *ctcs, double *objective,
                    double *step, const double *xinit, const double *uinit)
{
    pthread_t th[256];
    batch_job jobs[256];
    int t;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    for (t = 0; t < B; t++)
        if (K[t] < 2 || K[t] > kmax) return -1;
    for (t = 0; t < nthreads; t++) {
        batch_job jb = {st, B, kmax, nthreads, t, x0, xf, p, K, x, u, tf, mf, defect, ctcs,
                        objective, status, scp_iters, pipg_iters, step, xinit, uinit};
        jobs[t] = jb;
    }
    if (nthreads == 1) {
        batch_worker(&jobs[0]);
        return 0;
    }
    for (t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, batch_worker, &jobs[t]);
    for (t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    return 0;
}

/* One instance with a per-iteration trace (step, defect, ctcs, pipg iterations). */
int orc_solve_trace(const orc_settings *st, int K, const double *x0, const double *xf,
                    const double *p, double *xbar, double *ubar, double *scalars,
                    int32_t *ints, int trace_n, double *trace)
{
    orc_result r;
    scp_solve_one(st, K, x0, xf, p, NULL, NULL, xbar, ubar, &r, NULL, trace_n, trace);
    scalars[0] = r.tf; scalars[1] = r.mf; scalars[2] = r.defect; scalars[3] = r.ctcs;
    scalars[4] = r.objective; scalars[5] = r.step;
    ints[0] = r.status; ints[1] = r.scp_iters; ints[2] = r.pipg_iters;
    return 0;
}

/* ------------------------------------------------------------------------------------------
 * Truncated last-iteration map for gradient checks: with the reference, warm start and
 * sigma of the last SCP iteration frozen, map theta = (x0[15], m_wet, alpha_mdot, T_max) to
 * (m_f, t_f) through discretize -> QP build -> n_steps PIPG steps (no early exit) -> update.
 * m_wet is the initial-mass boundary value, so it is applied to x0[0] as well.
 * ------------------------------------------------------------------------------------------ */
int orc_lastiter_state(const orc_settings *st, int K, const double *x0, const double *xf,
                       const double *p, double *xbar_last, double *ubar_last, double *ws_last,
                       double *sigma_last)
{
    orc_lastiter last;
    orc_result r;
    double *xb = malloc(sizeof(double) * K * NX), *ub = malloc(sizeof(double) * K * NU);
    orc_settings s2 = *st;
    s2.early_exit = 0; /* fixed-work forward pass so that the last iteration is well defined */
    last.xbar = xbar_last;
    last.ubar = ubar_last;
    last.ws = ws_last;
    last.valid = 0;
    scp_solve_one(&s2, K, x0, xf, p, NULL, NULL, xb, ub, &r, &last, 0, NULL);
    *sigma_last = last.sigma;
    free(xb);
    free(ub);
    return last.valid ? 0 : -1;
}

int orc_iter_len(int K) { return iter_len(K); }

void orc_truncated_map(const orc_settings *st, int K, const double *x0, const double *xf,
                       const double *p, const double *theta, const double *xbar_last,
                       const double *ubar_last, const double *ws_last, double sigma, int n_steps,
                       double *out)
{
    int M = K - 1, k, i;
    double x0t[NX], pt[NP], dtau = 1.0 / M;
    double *xend = malloc(sizeof(double) * M * NX);
    double *A = malloc(sizeof(double) * M * NX * NX);
    double *Bm = malloc(sizeof(double) * M * NX * NU);
    double *Bp = malloc(sizeof(double) * M * NX * NU);
    qp_t qp;
    iter_t ws;
    memcpy(x0t, x0, sizeof(x0t));
    memcpy(pt, p, sizeof(pt));
    for (i = 0; i < NX; i++) x0t[i] = theta[i];
    /* m_wet (theta[15]) is the initial-mass boundary value: it adds to x0[0]'s perturbation */
    x0t[0] = theta[0] + (theta[15] - p[P_MWET]);
    pt[P_MWET] = theta[15];
    pt[P_ALPHA] = theta[16];
    pt[P_TMAX] = theta[17];
    qp_alloc(&qp, K);
    iter_alloc(&ws, K);
    iter_unpack(&ws, K, ws_last);
    orc_discretize(K, xbar_last, ubar_last, pt, st->rk4_substeps, xend, A, Bm, Bp);
    build_qp(st, pt, K, x0t, xf, xbar_last, ubar_last, xend, A, Bm, Bp, &qp);
    for (i = 0; i < K * NX; i++) ws.x[i] = 0.0;
    for (i = 0; i < K * NU; i++) ws.u[i] = 0.0;
    pipg_custom(st, &qp, sigma, n_steps, 0, &ws);
    out[0] = xbar_last[(K - 1) * NX + 0] + st->px[0] * ws.x[(K - 1) * NX + 0];
    out[1] = 0.0;
    for (k = 0; k < M; k++) {
        double s0 = ubar_last[k * NU + IS] + st->pu[IS] * ws.u[k * NU + IS];
        double s1 = ubar_last[(k + 1) * NU + IS] + st->pu[IS] * ws.u[(k + 1) * NU + IS];
        out[1] += dtau * 0.5 * (s0 + s1);
    }
    free(xend); free(A); free(Bm); free(Bp);
    qp_free(&qp);
    iter_free(&ws);
}

/* ------------------------------------------------------------------------------------------
 * Test-only exports of single steps.
 * ------------------------------------------------------------------------------------------ */
int orc_stopping(int K, const double *x1, const double *u1, const double *mup1,
                 const double *mum1, const double *phi1, const double *th1, const double *x0,
                 const double *u0, const double *mup0, const double *mum0, const double *phi0,
                 const double *th0, double eabs, double erel)
{
    iter_t a = {(double *)x1, (double *)u1, (double *)mup1, (double *)mum1, (double *)phi1,
                (double *)th1};
    iter_t b = {(double *)x0, (double *)u0, (double *)mup0, (double *)mum0, (double *)phi0,
                (double *)th0};
    return stopping_custom(&a, &b, K, eabs, erel);
}

/* Node projections in original units: x (15) and u (4) are projected in place. */
void orc_project_node(const double *p, double *x, double *u)
{
    double zx[NX] = {0}, zu[NU] = {0}, one_x[NX], one_u[NU];
    int i;
    for (i = 0; i < NX; i++) one_x[i] = 1.0;
    for (i = 0; i < NU; i++) one_u[i] = 1.0;
    /* with a zero reference and unit scales the scaled projection is the plain one */
    project_state(x, zx, one_x, p, 15);
    project_thrust(u, zu, one_u, p);
}
