// scp_common.hpp -- layout constants and workgroup helpers shared by the solve kernels and
// the gradient kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "lander_model.hpp"

namespace scp {

constexpr int CST = 16;          // stride of one column (15 rows + pad)
// Block layout of one interval for NUC controls: the columns of [A^- | B^- | B^+], each
// stored with stride CST
template <int NUC>
struct Blk {
    static constexpr int COLS = NX + 2 * NUC;  // 23 with (T, s), 29 with the torque
    static constexpr int SIZE = COLS * CST;     // entries per interval
};
constexpr int COLS = Blk<NU>::COLS;  // thrust-and-dilation layout (the gradient kernels)
constexpr int BLK = Blk<NU>::SIZE;
constexpr int VST = 20;          // node stride of (x, u) vectors in LDS (15 + 4 + pad)
constexpr int DST = 16;          // interval stride of dual vectors

// Final boundary condition: r, v, (q2, q3) and the transverse rates (w2, w3) are imposed; m,
// the roll angle part (q0, q1), the roll rate w1 and y are free (roll is not controllable by
// thrust alone).
__device__ __forceinline__ bool final_fixed(int i)
{
    return i >= 1 && i <= 13 && i != 7 && i != 8 && i != 11;
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

}  // namespace scp
