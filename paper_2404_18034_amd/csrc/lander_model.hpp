// lander_model.hpp -- device model of the 6-DoF lander (section "6-DoF Powered Descent
// Guidance"), time-dilated and augmented with the CTCS integrator (eq. sys-dyn-dil-aug):
//     f(x, u) = s * (F(xi, T), sum_i [g_i(xi, T)]_+^2).
// The discretization needs f and its directional derivative (a Jacobian-vector product)
// along (dx, du); both come out of one pass that shares the rotation matrix, the thrust
// norm and the constraint values.  Everything is templated on the arithmetic type R.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

namespace scp {

constexpr int NX = 15;
constexpr int NU = 4;      // controls (T, s); the full control set adds the torque (NU_MAX)
constexpr int NU_MAX = 7;  // (T, gamma, s) with the reaction-control torque gamma
constexpr int NP = 24;
constexpr int NXF = 13;
constexpr int IY = 14;
constexpr double NORM_EPS = 1e-4;  // below this a norm's derivative is taken as 0

// Quotient and square root as the model takes them: in FP32 the hardware reciprocal and square
// root (v_rcp_f32, v_sqrt_f32, about 1 ulp each, one instruction instead of a correctly
// rounded sequence), in every other type the correctly rounded operations.
__device__ __forceinline__ float mdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ float msqrt(float v) { return __builtin_amdgcn_sqrtf(v); }
template <typename T>
__device__ __forceinline__ T mdiv(const T &a, const T &b)
{
    return a / b;
}
template <typename T>
__device__ __forceinline__ T msqrt(const T &v)
{
    return sqrt(v);
}

// Vehicle data used inside the model, with the trigonometric constants folded once.
template <typename R>
struct Vehicle {
    R m_dry, alpha, g[3], Jinv[3], J[3], rT[3], T_min, T_max;
    R sec_delta, tan_gamma, tilt_c, w_max2;
    R v_max2;       // squared speed bound (used when has_vmax)
    bool has_vmax;  // v_max finite: the speed row joins the path constraints
    R g_max2;       // squared torque bound (used when has_gmax, full control set only)
    bool has_gmax;
};

template <typename R>
__device__ __forceinline__ Vehicle<R> load_vehicle(const R *p)
{
    Vehicle<R> v;
    v.m_dry = p[1];
    v.alpha = p[2];
    for (int i = 0; i < 3; ++i) {
        v.g[i] = p[3 + i];
        v.J[i] = p[6 + i];
        v.Jinv[i] = mdiv(R(1), p[6 + i]);
        v.rT[i] = p[9 + i];
    }
    v.T_min = p[12];
    v.T_max = p[13];
    // trigonometric constants: in FP32 directly (a few ulp), otherwise in double, rounded to R
    if constexpr (std::is_same<R, float>::value) {
        v.sec_delta = mdiv(1.0f, cosf(p[14]));
        v.tan_gamma = tanf(p[15]);
        v.tilt_c = 1.0f - cosf(p[16]);
    } else {
        v.sec_delta = R(1.0 / cos(double(p[14])));
        v.tan_gamma = R(tan(double(p[15])));
        v.tilt_c = R(1.0 - cos(double(p[16])));
    }
    v.w_max2 = p[17] * p[17];
    v.has_vmax = isfinite(double(p[22]));
    v.v_max2 = v.has_vmax ? p[22] * p[22] : R(0);
    v.has_gmax = isfinite(double(p[23]));
    v.g_max2 = v.has_gmax ? p[23] * p[23] : R(0);
    return v;
}

// f(x,u) and its derivative along (dx, du).  `want_d` = false skips the derivative.
// The y entry of f is returned in double: it feeds the CTCS accumulator.  NUC controls: 4
// (T, s) or 7 (T, gamma, s), the torque gamma adding J^-1 gamma to w_dot and the row
// ||gamma||^2 - gamma_max^2 to the path constraints.
template <typename R, bool WantD, int NUC = NU>
__device__ __forceinline__ void f_jvp(const Vehicle<R> &V, const R *x, const R *u, const R *dx,
                                      const R *du, R *f, double &fy, R *df)
{
    static_assert(NUC == NU || NUC == NU_MAX, "4 or 7 controls");
    const R m = x[0];
    const R q0 = x[7], q1 = x[8], q2 = x[9], q3 = x[10];
    const R w0 = x[11], w1 = x[12], w2 = x[13];
    const R T0 = u[0], T1 = u[1], T2 = u[2], s = u[NUC - 1];

    // rotation C(q) (body -> inertial) applied to T
    const R C00 = q0 * q0 + q1 * q1 - q2 * q2 - q3 * q3;
    const R C01 = R(2) * (q1 * q2 - q0 * q3);
    const R C02 = R(2) * (q1 * q3 + q0 * q2);
    const R C10 = R(2) * (q1 * q2 + q0 * q3);
    const R C11 = q0 * q0 - q1 * q1 + q2 * q2 - q3 * q3;
    const R C12 = R(2) * (q2 * q3 - q0 * q1);
    const R C20 = R(2) * (q1 * q3 - q0 * q2);
    const R C21 = R(2) * (q2 * q3 + q0 * q1);
    const R C22 = q0 * q0 - q1 * q1 - q2 * q2 + q3 * q3;
    const R a0 = C00 * T0 + C01 * T1 + C02 * T2;
    const R a1 = C10 * T0 + C11 * T1 + C12 * T2;
    const R a2 = C20 * T0 + C21 * T1 + C22 * T2;
    const R im = mdiv(R(1), m);

    const R Tn = msqrt(T0 * T0 + T1 * T1 + T2 * T2);
    const R Jw0 = V.J[0] * w0, Jw1 = V.J[1] * w1, Jw2 = V.J[2] * w2;

    R F[NX];
    F[0] = -V.alpha * Tn;
    F[1] = x[4];
    F[2] = x[5];
    F[3] = x[6];
    F[4] = a0 * im + V.g[0];
    F[5] = a1 * im + V.g[1];
    F[6] = a2 * im + V.g[2];
    // q_dot = 0.5 Omega(w) q
    F[7] = R(0.5) * (-w0 * q1 - w1 * q2 - w2 * q3);
    F[8] = R(0.5) * (w0 * q0 + w2 * q2 - w1 * q3);
    F[9] = R(0.5) * (w1 * q0 - w2 * q1 + w0 * q3);
    F[10] = R(0.5) * (w2 * q0 + w1 * q1 - w0 * q2);
    // w_dot = J^-1 (rT x T - w x J w)
    F[11] = V.Jinv[0] * ((V.rT[1] * T2 - V.rT[2] * T1) - (w1 * Jw2 - w2 * Jw1));
    F[12] = V.Jinv[1] * ((V.rT[2] * T0 - V.rT[0] * T2) - (w2 * Jw0 - w0 * Jw2));
    F[13] = V.Jinv[2] * ((V.rT[0] * T1 - V.rT[1] * T0) - (w0 * Jw1 - w1 * Jw0));
    if constexpr (NUC == NU_MAX)
        for (int i = 0; i < 3; ++i) F[11 + i] += V.Jinv[i] * u[3 + i];

    // path constraints g (mass, glide slope, tilt, rate, gimbal, T_max, T_min, speed; the
    // speed row is the constant -1 without a speed bound)
    const R lat = msqrt(x[2] * x[2] + x[3] * x[3]);
    R g[9];
    g[0] = V.m_dry - m;
    g[1] = V.tan_gamma * lat - x[1];
    g[2] = R(2) * (q2 * q2 + q3 * q3) - V.tilt_c;
    g[3] = w0 * w0 + w1 * w1 + w2 * w2 - V.w_max2;
    g[4] = Tn - T0 * V.sec_delta;
    g[5] = Tn - V.T_max;
    g[6] = V.T_min - Tn;
    g[7] = V.has_vmax ? x[4] * x[4] + x[5] * x[5] + x[6] * x[6] - V.v_max2 : R(-1);
    g[8] = (NUC == NU_MAX && V.has_gmax)
               ? u[3] * u[3] + u[4 % NUC] * u[4 % NUC] + u[5 % NUC] * u[5 % NUC] - V.g_max2
               : R(-1);
    constexpr int NGC = NUC == NU_MAX ? 9 : 8;  // the torque row is -1 without the torque
    R gp[9];
    R Fy = R(0);
#pragma unroll
    for (int i = 0; i < NGC; ++i) {
        gp[i] = g[i] > R(0) ? g[i] : R(0);
        Fy += gp[i] * gp[i];
    }
#pragma unroll
    for (int i = 0; i < 14; ++i) f[i] = s * F[i];
    fy = double(s) * double(Fy);
    f[IY] = s * Fy;

    if (!WantD) return;

    const R ds = du[NUC - 1];
    const R dT0 = du[0], dT1 = du[1], dT2 = du[2];
    const R dq0 = dx[7], dq1 = dx[8], dq2 = dx[9], dq3 = dx[10];
    const R dw0 = dx[11], dw1 = dx[12], dw2 = dx[13];
    const R dm = dx[0];
    // directional derivative of each C entry along dq
    const R dC00 = R(2) * (q0 * dq0 + q1 * dq1 - q2 * dq2 - q3 * dq3);
    const R dC01 = R(2) * (dq1 * q2 + q1 * dq2 - dq0 * q3 - q0 * dq3);
    const R dC02 = R(2) * (dq1 * q3 + q1 * dq3 + dq0 * q2 + q0 * dq2);
    const R dC10 = R(2) * (dq1 * q2 + q1 * dq2 + dq0 * q3 + q0 * dq3);
    const R dC11 = R(2) * (q0 * dq0 - q1 * dq1 + q2 * dq2 - q3 * dq3);
    const R dC12 = R(2) * (dq2 * q3 + q2 * dq3 - dq0 * q1 - q0 * dq1);
    const R dC20 = R(2) * (dq1 * q3 + q1 * dq3 - dq0 * q2 - q0 * dq2);
    const R dC21 = R(2) * (dq2 * q3 + q2 * dq3 + dq0 * q1 + q0 * dq1);
    const R dC22 = R(2) * (q0 * dq0 - q1 * dq1 - q2 * dq2 + q3 * dq3);
    const R da0 = dC00 * T0 + dC01 * T1 + dC02 * T2 + C00 * dT0 + C01 * dT1 + C02 * dT2;
    const R da1 = dC10 * T0 + dC11 * T1 + dC12 * T2 + C10 * dT0 + C11 * dT1 + C12 * dT2;
    const R da2 = dC20 * T0 + dC21 * T1 + dC22 * T2 + C20 * dT0 + C21 * dT1 + C22 * dT2;
    // the derivative of a norm is taken as 0 below NORM_EPS (the thrust projection can put T
    // exactly at the apex of the gimbal cone; its reconstruction carries rounding noise)
    const R dTn = Tn > R(NORM_EPS) ? mdiv(T0 * dT0 + T1 * dT1 + T2 * dT2, Tn) : R(0);
    const R dim = -dm * im * im;

    R dF[NX];
    dF[0] = -V.alpha * dTn;
    dF[1] = dx[4];
    dF[2] = dx[5];
    dF[3] = dx[6];
    dF[4] = da0 * im + a0 * dim;
    dF[5] = da1 * im + a1 * dim;
    dF[6] = da2 * im + a2 * dim;
    dF[7] = R(0.5) * (-dw0 * q1 - dw1 * q2 - dw2 * q3 - w0 * dq1 - w1 * dq2 - w2 * dq3);
    dF[8] = R(0.5) * (dw0 * q0 + dw2 * q2 - dw1 * q3 + w0 * dq0 + w2 * dq2 - w1 * dq3);
    dF[9] = R(0.5) * (dw1 * q0 - dw2 * q1 + dw0 * q3 + w1 * dq0 - w2 * dq1 + w0 * dq3);
    dF[10] = R(0.5) * (dw2 * q0 + dw1 * q1 - dw0 * q2 + w2 * dq0 + w1 * dq1 - w0 * dq2);
    const R dJw0 = V.J[0] * dw0, dJw1 = V.J[1] * dw1, dJw2 = V.J[2] * dw2;
    dF[11] = V.Jinv[0] * ((V.rT[1] * dT2 - V.rT[2] * dT1) -
                          (dw1 * Jw2 + w1 * dJw2 - dw2 * Jw1 - w2 * dJw1));
    dF[12] = V.Jinv[1] * ((V.rT[2] * dT0 - V.rT[0] * dT2) -
                          (dw2 * Jw0 + w2 * dJw0 - dw0 * Jw2 - w0 * dJw2));
    dF[13] = V.Jinv[2] * ((V.rT[0] * dT1 - V.rT[1] * dT0) -
                          (dw0 * Jw1 + w0 * dJw1 - dw1 * Jw0 - w1 * dJw0));
    if constexpr (NUC == NU_MAX)
        for (int i = 0; i < 3; ++i) dF[11 + i] += V.Jinv[i] * du[3 + i];
    R dg[9];
    dg[0] = -dm;
    dg[1] = (lat > R(NORM_EPS) ? mdiv(V.tan_gamma * (x[2] * dx[2] + x[3] * dx[3]), lat) : R(0)) -
            dx[1];
    dg[2] = R(4) * (q2 * dq2 + q3 * dq3);
    dg[3] = R(2) * (w0 * dw0 + w1 * dw1 + w2 * dw2);
    dg[4] = dTn - dT0 * V.sec_delta;
    dg[5] = dTn;
    dg[6] = -dTn;
    dg[7] = V.has_vmax ? R(2) * (x[4] * dx[4] + x[5] * dx[5] + x[6] * dx[6]) : R(0);
    if constexpr (NUC == NU_MAX)
        dg[8] = V.has_gmax ? R(2) * (u[3] * du[3] + u[4] * du[4] + u[5] * du[5]) : R(0);
    R dFy = R(0);
#pragma unroll
    for (int i = 0; i < NGC; ++i) dFy += R(2) * gp[i] * dg[i];
#pragma unroll
    for (int i = 0; i < 14; ++i) df[i] = ds * F[i] + s * dF[i];
    df[IY] = ds * Fy + s * dFy;
}

}  // namespace scp
