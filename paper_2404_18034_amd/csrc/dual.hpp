// dual.hpp -- forward-mode number with N tangent directions: v + sum_n d[n] e_n with
// e_m e_n = 0.  Running the lander model on it gives, besides the value, its first
// derivatives along N directions.  The gradient kernels use it for the directional
// derivatives of the model inside the discretization: with respect to the two differentiated
// vehicle parameters (alpha_mdot, T_max), and with respect to one state direction at a time
// (the local Jacobian-transpose products of the reverse sweep through RK4).  Comparisons look
// at the value only (a branch is taken the way the plain evaluation takes it).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace scp {

using ::sqrt;  // keep the plain overloads visible beside the dual one below

template <typename T, int N>
struct Dual {
    T v, d[N];
    __device__ __forceinline__ Dual() : v(0)
    {
        for (int n = 0; n < N; ++n) d[n] = T(0);
    }
    __device__ __forceinline__ Dual(double c) : v(T(c))
    {
        for (int n = 0; n < N; ++n) d[n] = T(0);
    }
    __device__ __forceinline__ explicit operator double() const { return double(v); }
    __device__ __forceinline__ Dual &operator+=(const Dual &o)
    {
        v += o.v;
        for (int n = 0; n < N; ++n) d[n] += o.d[n];
        return *this;
    }
    __device__ __forceinline__ Dual &operator-=(const Dual &o)
    {
        v -= o.v;
        for (int n = 0; n < N; ++n) d[n] -= o.d[n];
        return *this;
    }
};

// a constant with tangent `t` along direction n
template <typename T, int N>
__device__ __forceinline__ Dual<T, N> seed(T value, int n, T t)
{
    Dual<T, N> r = Dual<T, N>(static_cast<double>(value));
    r.d[n] = t;
    return r;
}

template <typename T, int N>
__device__ __forceinline__ Dual<T, N> operator-(const Dual<T, N> &a)
{
    Dual<T, N> r;
    r.v = -a.v;
    for (int n = 0; n < N; ++n) r.d[n] = -a.d[n];
    return r;
}
template <typename T, int N>
__device__ __forceinline__ Dual<T, N> operator+(const Dual<T, N> &a, const Dual<T, N> &b)
{
    Dual<T, N> r;
    r.v = a.v + b.v;
    for (int n = 0; n < N; ++n) r.d[n] = a.d[n] + b.d[n];
    return r;
}
template <typename T, int N>
__device__ __forceinline__ Dual<T, N> operator-(const Dual<T, N> &a, const Dual<T, N> &b)
{
    Dual<T, N> r;
    r.v = a.v - b.v;
    for (int n = 0; n < N; ++n) r.d[n] = a.d[n] - b.d[n];
    return r;
}
template <typename T, int N>
__device__ __forceinline__ Dual<T, N> operator*(const Dual<T, N> &a, const Dual<T, N> &b)
{
    Dual<T, N> r;
    r.v = a.v * b.v;
    for (int n = 0; n < N; ++n) r.d[n] = a.d[n] * b.v + a.v * b.d[n];
    return r;
}
template <typename T, int N>
__device__ __forceinline__ Dual<T, N> operator/(const Dual<T, N> &a, const Dual<T, N> &b)
{
    Dual<T, N> r;
    r.v = a.v / b.v;
    const T ib = T(1) / b.v;
    for (int n = 0; n < N; ++n) r.d[n] = (a.d[n] - r.v * b.d[n]) * ib;
    return r;
}
template <typename T, int N>
__device__ __forceinline__ Dual<T, N> sqrt(const Dual<T, N> &a)
{
    Dual<T, N> r;
    r.v = ::sqrt(a.v);
    const T h = r.v > T(0) ? T(0.5) / r.v : T(0);
    for (int n = 0; n < N; ++n) r.d[n] = a.d[n] * h;
    return r;
}
template <typename T, int N>
__device__ __forceinline__ bool operator>(const Dual<T, N> &a, const Dual<T, N> &b)
{
    return a.v > b.v;
}
template <typename T, int N>
__device__ __forceinline__ bool operator<(const Dual<T, N> &a, const Dual<T, N> &b)
{
    return a.v < b.v;
}

}  // namespace scp
