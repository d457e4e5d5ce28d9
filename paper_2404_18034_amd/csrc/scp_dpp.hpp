// scp_dpp.hpp -- cross-lane helpers over the 16-lane DPP rows of a wave, shared by the solve
// kernels and the gradient kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <utility>

#include "lander_model.hpp"

namespace scp {

// ------------------------------------------------------------------------------------------
// Cross-lane helpers.  A workgroup row is 16 lanes (one DPP row); row k of the workgroup
// holds node k (state variable i on lane i) and interval k (dynamics row i on lane i).
// ------------------------------------------------------------------------------------------
template <int L>
__device__ __forceinline__ float rowb(float v)
{
    // row_newbcast: every lane of the 16-lane row receives lane L's value
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x150 + L, 0xf, 0xf, true));
}
template <int L>
__device__ __forceinline__ double rowb(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x150 + L, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x150 + L, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dppmov(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double dppmov(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
// Sum over the 16 lanes of a row, returned to every lane.  Partners are exchanged
// symmetrically at every step (quad xor 1, quad xor 2, row mirror, row rotate by 8), so each
// lane adds the same two operands and all 16 lanes end with bitwise identical sums.
template <typename R>
__device__ __forceinline__ R row_allreduce(R v)
{
    v = v + dppmov<0xB1>(v);   // quad_perm [1,0,3,2]
    v = v + dppmov<0x4E>(v);   // quad_perm [2,3,0,1]
    v = v + dppmov<0x140>(v);  // row_mirror
    v = v + dppmov<0x128>(v);  // row_ror:8
    return v;
}
// Four row sums at once, scattered: lane i receives sum over the row of v[i >> 2], where
// v[q] is this lane's q-th addend.  Three exchange steps (row_mirror pairs lanes differing
// in bit 3, row_half_mirror lanes differing in bit 2, then the two quad swaps) keep half of
// the values each time; the four lanes of a quad end with bitwise identical sums.
template <typename R>
__device__ __forceinline__ R row_reduce_scatter4(const R (&v)[NU], int i)
{
    const bool b3 = (i & 8) != 0, b2 = (i & 4) != 0;
    const R k0 = b3 ? v[2] : v[0], k1 = b3 ? v[3] : v[1];
    const R s0 = b3 ? v[0] : v[2], s1 = b3 ? v[1] : v[3];
    const R a0 = k0 + dppmov<0x140>(s0);  // row_mirror
    const R a1 = k1 + dppmov<0x140>(s1);
    const R kk = b2 ? a1 : a0, ss = b2 ? a0 : a1;
    R w = kk + dppmov<0x141>(ss);         // row_half_mirror
    w = w + dppmov<0xB1>(w);              // quad_perm [1,0,3,2]
    w = w + dppmov<0x4E>(w);              // quad_perm [2,3,0,1]
    return w;
}
// Interleaved control layout of the subproblem kernel: component c of the node's controls on
// lanes c, c+4, c+8 and c+12 of its row; the copy on lanes 4..7 is the one that is read.
// Reduce-scatter onto it: lane i receives the row sum of component i & 3.  Lane i supplies its
// four addends in the order v[s] = addend of component xpermi(i, s), where with b0, b1 the
// bits 0 and 1 of i
//   xpermi(i, 0) = b0 + 2 b1,  xpermi(i, 1) = b0 + 2 (1 - b1),
//   xpermi(i, 2) = (1 - b0) + 2 b1,  xpermi(i, 3) = (1 - b0) + 2 (1 - b1),
// so that the partner across bit 0 sends exactly the two components this lane keeps and the
// partner across bit 1 the one it keeps after that; the four quads are then summed by row
// rotations by 4 and by 8 (the copies may differ in the last bit).
__host__ __device__ constexpr int xpermi(int i, int s)
{
    const int b0 = i & 1, b1 = (i >> 1) & 1;
    return s == 0 ? b0 + 2 * b1 : s == 1 ? b0 + 2 * (1 - b1) : s == 2 ? (1 - b0) + 2 * b1 : (1 - b0) + 2 * (1 - b1);
}
template <typename R>
__device__ __forceinline__ R row_reduce_scatter4i(const R (&v)[NU])
{
    const R a0 = v[0] + dppmov<0xB1>(v[2]);  // quad_perm [1,0,3,2]
    const R a1 = v[1] + dppmov<0xB1>(v[3]);
    R w = a0 + dppmov<0x4E>(a1);             // quad_perm [2,3,0,1]
    w = w + dppmov<0x124>(w);                // row_ror:4
    w = w + dppmov<0x128>(w);                // row_ror:8
    return w;
}
// sum_q c[q] * (value of lane 4 + q of this row), q = 0..3: a control product in the
// interleaved layout
template <typename R>
__device__ __forceinline__ R rowdot4c(const R *c, R v, R acc)
{
    acc = acc + c[0] * rowb<4>(v);
    acc = acc + c[1] * rowb<5>(v);
    acc = acc + c[2] * rowb<6>(v);
    acc = acc + c[3] * rowb<7>(v);
    return acc;
}
// sum_q c[q] * (value of lane 4q of this row), q = 0..3
template <typename R>
__device__ __forceinline__ R rowdot4q(const R *c, R v, R acc)
{
    acc = acc + c[0] * rowb<0>(v);
    acc = acc + c[1] * rowb<4>(v);
    acc = acc + c[2] * rowb<8>(v);
    acc = acc + c[3] * rowb<12>(v);
    return acc;
}
// sum_j c[j] * (value of lane j of this row), j = 0..14, in a fixed order
template <typename R, int... J>
__device__ __forceinline__ R rowdot_impl(const R *c, R v, R acc, std::integer_sequence<int, J...>)
{
    ((acc = acc + c[J] * rowb<J>(v)), ...);
    return acc;
}
template <typename R>
__device__ __forceinline__ R rowdot15(const R *c, R v, R acc)
{
    return rowdot_impl<R>(c, v, acc, std::make_integer_sequence<int, NX>{});
}

// FP32: each broadcast-multiply-add is one v_fmac_f32 whose first source is read through a
// DPP row_newbcast, instead of a DPP move followed by an FMA.  The leading s_nop covers the
// wait states a DPP source read needs after a VALU write of that register or of EXEC.
template <>
__device__ __forceinline__ float rowdot4q<float>(const float *c, float v, float acc)
{
    asm volatile(
        "s_nop 4\n\t"
        "v_fmac_f32_dpp %0, %1, %2 row_newbcast:0 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %3 row_newbcast:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %4 row_newbcast:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %5 row_newbcast:12 row_mask:0xf bank_mask:0xf\n\t"
        : "+v"(acc)
        : "v"(v), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]));
    return acc;
}
template <>
__device__ __forceinline__ float rowdot4c<float>(const float *c, float v, float acc)
{
    asm volatile(
        "s_nop 4\n\t"
        "v_fmac_f32_dpp %0, %1, %2 row_newbcast:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %3 row_newbcast:5 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %4 row_newbcast:6 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %5 row_newbcast:7 row_mask:0xf bank_mask:0xf\n\t"
        : "+v"(acc)
        : "v"(v), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]));
    return acc;
}
template <>
__device__ __forceinline__ float rowdot15<float>(const float *c, float v, float acc)
{
    asm volatile(
        "s_nop 4\n\t"
        "v_fmac_f32_dpp %0, %1, %2 row_newbcast:0 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %3 row_newbcast:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %4 row_newbcast:2 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %5 row_newbcast:3 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %6 row_newbcast:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %7 row_newbcast:5 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %8 row_newbcast:6 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %9 row_newbcast:7 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %10 row_newbcast:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %11 row_newbcast:9 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %12 row_newbcast:10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %13 row_newbcast:11 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %14 row_newbcast:12 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %15 row_newbcast:13 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %16 row_newbcast:14 row_mask:0xf bank_mask:0xf\n\t"
        : "+v"(acc)
        : "v"(v), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]), "v"(c[4]), "v"(c[5]), "v"(c[6]),
          "v"(c[7]), "v"(c[8]), "v"(c[9]), "v"(c[10]), "v"(c[11]), "v"(c[12]), "v"(c[13]),
          "v"(c[14]));
    return acc;
}

// sum_{j<N} c[j] * (value of lane J0 + j of this row), in the order j = 0, 1, ...
template <typename R, int J0, int N, int... J>
__device__ __forceinline__ R rowdot_part_impl(const R *c, R v, R acc, std::integer_sequence<int, J...>)
{
    ((acc = acc + c[J] * rowb<J0 + J>(v)), ...);
    return acc;
}
template <typename R, int J0, int N>
__device__ __forceinline__ R rowdot_part(const R *c, R v, R acc)
{
    return rowdot_part_impl<R, J0, N>(c, v, acc, std::make_integer_sequence<int, N>{});
}
// FP32: lanes 0..7 and 8..15, one v_fmac_f32 with a DPP row_newbcast source each
template <>
__device__ __forceinline__ float rowdot_part<float, 0, 8>(const float *c, float v, float acc)
{
    asm volatile(
        "s_nop 4\n\t"
        "v_fmac_f32_dpp %0, %1, %2 row_newbcast:0 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %3 row_newbcast:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %4 row_newbcast:2 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %5 row_newbcast:3 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %6 row_newbcast:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %7 row_newbcast:5 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %8 row_newbcast:6 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %9 row_newbcast:7 row_mask:0xf bank_mask:0xf\n\t"
        : "+v"(acc)
        : "v"(v), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]), "v"(c[4]), "v"(c[5]), "v"(c[6]),
          "v"(c[7]));
    return acc;
}
template <>
__device__ __forceinline__ float rowdot_part<float, 8, 8>(const float *c, float v, float acc)
{
    asm volatile(
        "s_nop 4\n\t"
        "v_fmac_f32_dpp %0, %1, %2 row_newbcast:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %3 row_newbcast:9 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %4 row_newbcast:10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %5 row_newbcast:11 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %6 row_newbcast:12 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %7 row_newbcast:13 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %8 row_newbcast:14 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %9 row_newbcast:15 row_mask:0xf bank_mask:0xf\n\t"
        : "+v"(acc)
        : "v"(v), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]), "v"(c[4]), "v"(c[5]), "v"(c[6]),
          "v"(c[7]));
    return acc;
}
// FP64 (and the remaining FP32 shapes): the same broadcast chains, one v_fmac_f64 (f32) with a
// DPP row_newbcast source per term instead of two 32-bit DPP moves and an FMA
template <>
__device__ __forceinline__ double rowdot15<double>(const double *c, double v, double acc)
{
    asm volatile(
        "s_nop 4\n\t"
        "v_fmac_f64_dpp %0, %1, %2 row_newbcast:0 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %3 row_newbcast:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %4 row_newbcast:2 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %5 row_newbcast:3 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %6 row_newbcast:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %7 row_newbcast:5 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %8 row_newbcast:6 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %9 row_newbcast:7 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %10 row_newbcast:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %11 row_newbcast:9 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %12 row_newbcast:10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %13 row_newbcast:11 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %14 row_newbcast:12 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %15 row_newbcast:13 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %16 row_newbcast:14 row_mask:0xf bank_mask:0xf\n\t"
        : "+v"(acc)
        : "v"(v), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]), "v"(c[4]), "v"(c[5]), "v"(c[6]),
          "v"(c[7]), "v"(c[8]), "v"(c[9]), "v"(c[10]), "v"(c[11]), "v"(c[12]), "v"(c[13]),
          "v"(c[14]));
    return acc;
}
template <>
__device__ __forceinline__ double rowdot4c<double>(const double *c, double v, double acc)
{
    asm volatile(
        "s_nop 4\n\t"
        "v_fmac_f64_dpp %0, %1, %2 row_newbcast:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %3 row_newbcast:5 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %4 row_newbcast:6 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %5 row_newbcast:7 row_mask:0xf bank_mask:0xf\n\t"
        : "+v"(acc)
        : "v"(v), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]));
    return acc;
}
template <>
__device__ __forceinline__ double rowdot4q<double>(const double *c, double v, double acc)
{
    asm volatile(
        "s_nop 4\n\t"
        "v_fmac_f64_dpp %0, %1, %2 row_newbcast:0 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %3 row_newbcast:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %4 row_newbcast:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %5 row_newbcast:12 row_mask:0xf bank_mask:0xf\n\t"
        : "+v"(acc)
        : "v"(v), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]));
    return acc;
}
template <>
__device__ __forceinline__ double rowdot_part<double, 0, 8>(const double *c, double v, double acc)
{
    asm volatile(
        "s_nop 4\n\t"
        "v_fmac_f64_dpp %0, %1, %2 row_newbcast:0 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %3 row_newbcast:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %4 row_newbcast:2 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %5 row_newbcast:3 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %6 row_newbcast:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %7 row_newbcast:5 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %8 row_newbcast:6 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %9 row_newbcast:7 row_mask:0xf bank_mask:0xf\n\t"
        : "+v"(acc)
        : "v"(v), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]), "v"(c[4]), "v"(c[5]), "v"(c[6]),
          "v"(c[7]));
    return acc;
}
template <>
__device__ __forceinline__ double rowdot_part<double, 8, 8>(const double *c, double v, double acc)
{
    asm volatile(
        "s_nop 4\n\t"
        "v_fmac_f64_dpp %0, %1, %2 row_newbcast:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %3 row_newbcast:9 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %4 row_newbcast:10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %5 row_newbcast:11 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %6 row_newbcast:12 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %7 row_newbcast:13 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %8 row_newbcast:14 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %9 row_newbcast:15 row_mask:0xf bank_mask:0xf\n\t"
        : "+v"(acc)
        : "v"(v), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]), "v"(c[4]), "v"(c[5]), "v"(c[6]),
          "v"(c[7]));
    return acc;
}
template <>
__device__ __forceinline__ double rowdot_part<double, 8, 7>(const double *c, double v, double acc)
{
    asm volatile(
        "s_nop 4\n\t"
        "v_fmac_f64_dpp %0, %1, %2 row_newbcast:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %3 row_newbcast:9 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %4 row_newbcast:10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %5 row_newbcast:11 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %6 row_newbcast:12 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %7 row_newbcast:13 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %8 row_newbcast:14 row_mask:0xf bank_mask:0xf\n\t"
        : "+v"(acc)
        : "v"(v), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]), "v"(c[4]), "v"(c[5]), "v"(c[6]));
    return acc;
}
template <>
__device__ __forceinline__ double rowdot_part<double, 8, 3>(const double *c, double v, double acc)
{
    asm volatile(
        "s_nop 4\n\t"
        "v_fmac_f64_dpp %0, %1, %2 row_newbcast:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %3 row_newbcast:9 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %4 row_newbcast:10 row_mask:0xf bank_mask:0xf\n\t"
        : "+v"(acc)
        : "v"(v), "v"(c[0]), "v"(c[1]), "v"(c[2]));
    return acc;
}
template <>
__device__ __forceinline__ double rowdot_part<double, 4, 4>(const double *c, double v, double acc)
{
    asm volatile(
        "s_nop 4\n\t"
        "v_fmac_f64_dpp %0, %1, %2 row_newbcast:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %3 row_newbcast:5 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %4 row_newbcast:6 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %5 row_newbcast:7 row_mask:0xf bank_mask:0xf\n\t"
        : "+v"(acc)
        : "v"(v), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]));
    return acc;
}
template <>
__device__ __forceinline__ float rowdot_part<float, 8, 3>(const float *c, float v, float acc)
{
    asm volatile(
        "s_nop 4\n\t"
        "v_fmac_f32_dpp %0, %1, %2 row_newbcast:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %3 row_newbcast:9 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %4 row_newbcast:10 row_mask:0xf bank_mask:0xf\n\t"
        : "+v"(acc)
        : "v"(v), "v"(c[0]), "v"(c[1]), "v"(c[2]));
    return acc;
}
template <>
__device__ __forceinline__ float rowdot_part<float, 4, 4>(const float *c, float v, float acc)
{
    asm volatile(
        "s_nop 4\n\t"
        "v_fmac_f32_dpp %0, %1, %2 row_newbcast:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %3 row_newbcast:5 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %4 row_newbcast:6 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %5 row_newbcast:7 row_mask:0xf bank_mask:0xf\n\t"
        : "+v"(acc)
        : "v"(v), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]));
    return acc;
}
template <>
__device__ __forceinline__ float rowdot_part<float, 8, 7>(const float *c, float v, float acc)
{
    asm volatile(
        "s_nop 4\n\t"
        "v_fmac_f32_dpp %0, %1, %2 row_newbcast:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %3 row_newbcast:9 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %4 row_newbcast:10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %5 row_newbcast:11 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %6 row_newbcast:12 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %7 row_newbcast:13 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %8 row_newbcast:14 row_mask:0xf bank_mask:0xf\n\t"
        : "+v"(acc)
        : "v"(v), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]), "v"(c[4]), "v"(c[5]), "v"(c[6]));
    return acc;
}

}  // namespace scp
