// dual2.hpp -- forward-mode number with two tangent directions: v + d0 e0 + d1 e1 with
// e0 e1 = e0^2 = e1^2 = 0.  Running the lander model on it gives, besides the value, its
// first derivatives along two parameter directions (here alpha_mdot and T_max); the
// discretization run on it yields the sensitivities of A_k, B_k^-+ and the propagated
// endpoint to those parameters.  Comparisons look at the value only (a branch is taken the
// way the plain evaluation takes it).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace scp {

using ::sqrt;  // keep the plain overloads visible beside the dual one below

template <typename T>
struct Dual2 {
    T v, d0, d1;
    __device__ __forceinline__ Dual2() : v(0), d0(0), d1(0) {}
    __device__ __forceinline__ Dual2(double c) : v(T(c)), d0(0), d1(0) {}
    __device__ __forceinline__ Dual2(T a, T b, T c) : v(a), d0(b), d1(c) {}
    __device__ __forceinline__ explicit operator double() const { return double(v); }
    __device__ __forceinline__ Dual2 &operator+=(const Dual2 &o)
    {
        v += o.v;
        d0 += o.d0;
        d1 += o.d1;
        return *this;
    }
    __device__ __forceinline__ Dual2 &operator-=(const Dual2 &o)
    {
        v -= o.v;
        d0 -= o.d0;
        d1 -= o.d1;
        return *this;
    }
};

template <typename T>
__device__ __forceinline__ Dual2<T> operator-(const Dual2<T> &a)
{
    return Dual2<T>(-a.v, -a.d0, -a.d1);
}
template <typename T>
__device__ __forceinline__ Dual2<T> operator+(const Dual2<T> &a, const Dual2<T> &b)
{
    return Dual2<T>(a.v + b.v, a.d0 + b.d0, a.d1 + b.d1);
}
template <typename T>
__device__ __forceinline__ Dual2<T> operator-(const Dual2<T> &a, const Dual2<T> &b)
{
    return Dual2<T>(a.v - b.v, a.d0 - b.d0, a.d1 - b.d1);
}
template <typename T>
__device__ __forceinline__ Dual2<T> operator*(const Dual2<T> &a, const Dual2<T> &b)
{
    return Dual2<T>(a.v * b.v, a.d0 * b.v + a.v * b.d0, a.d1 * b.v + a.v * b.d1);
}
template <typename T>
__device__ __forceinline__ Dual2<T> operator/(const Dual2<T> &a, const Dual2<T> &b)
{
    const T q = a.v / b.v;
    const T ib = T(1) / b.v;
    return Dual2<T>(q, (a.d0 - q * b.d0) * ib, (a.d1 - q * b.d1) * ib);
}
template <typename T>
__device__ __forceinline__ Dual2<T> sqrt(const Dual2<T> &a)
{
    const T s = ::sqrt(a.v);
    const T h = s > T(0) ? T(0.5) / s : T(0);
    return Dual2<T>(s, a.d0 * h, a.d1 * h);
}
template <typename T>
__device__ __forceinline__ bool operator>(const Dual2<T> &a, const Dual2<T> &b)
{
    return a.v > b.v;
}
template <typename T>
__device__ __forceinline__ bool operator<(const Dual2<T> &a, const Dual2<T> &b)
{
    return a.v < b.v;
}

}  // namespace scp
