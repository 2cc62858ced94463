// Device helpers shared by the libsem kernels: type conversion, per-point
// inverse multiplicity and deterministic workgroup reductions.
#pragma once
#include "sem_internal.h"

namespace semk {

template <typename T> struct TypeOf;
template <> struct TypeOf<double> { static constexpr int id = P64; };
template <> struct TypeOf<float> { static constexpr int id = P32; };
template <> struct TypeOf<__half> { static constexpr int id = P16; };
template <> struct TypeOf<__hip_bfloat16> { static constexpr int id = PBF; };

template <typename C, typename T> __device__ __forceinline__ C to(T v) { return (C)v; }
template <> __device__ __forceinline__ float to<float, __half>(__half v) { return __half2float(v); }
template <> __device__ __forceinline__ double to<double, __half>(__half v) { return (double)__half2float(v); }
template <> __device__ __forceinline__ float to<float, __hip_bfloat16>(__hip_bfloat16 v) { return __bfloat162float(v); }
template <> __device__ __forceinline__ double to<double, __hip_bfloat16>(__hip_bfloat16 v) { return (double)__bfloat162float(v); }
template <> __device__ __forceinline__ __half to<__half, float>(float v) { return __float2half_rn(v); }
// fp64 -> 16-bit with a single rounding: round to odd into fp32 (24-bit
// significand, at least two bits more than the target), then round to nearest
// even into the 16-bit format.
__device__ __forceinline__ float d2f_round_odd(double d)
{
    float f = (float)d;
    if ((double)f == d || !isfinite(f)) return f;
    if (fabs((double)f) > fabs(d)) f = nextafterf(f, 0.0f);
    unsigned u = __float_as_uint(f) | 1u;
    return __uint_as_float(u);
}
template <> __device__ __forceinline__ __half to<__half, double>(double v) { return __float2half_rn(d2f_round_odd(v)); }
template <> __device__ __forceinline__ __hip_bfloat16 to<__hip_bfloat16, float>(float v) { return __float2bfloat16(v); }
template <> __device__ __forceinline__ __hip_bfloat16 to<__hip_bfloat16, double>(double v) { return __float2bfloat16(d2f_round_odd(v)); }

// 1 / multiplicity of local point q (0 <= q < lx^3) of a conforming periodic
// box mesh: every coordinate on an element face doubles the number of copies.
__device__ __forceinline__ double inv_mult(int q, int lx)
{
    int i = q % lx, t = q / lx, j = t % lx, k = t / lx;
    int n = lx - 1;
    double r = 1.0;
    if (i == 0 || i == n) r *= 0.5;
    if (j == 0 || j == n) r *= 0.5;
    if (k == 0 || k == n) r *= 0.5;
    return r;
}

// wavefront sum (64 lanes), fixed butterfly order -> deterministic
template <typename A> __device__ __forceinline__ A wave_sum(A v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
template <typename A> __device__ __forceinline__ A wave_max(A v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) { A w = __shfl_xor(v, o, 64); v = v > w ? v : w; }
    return v;
}

// block sum of NV values per thread; result valid in thread 0 (fixed order).
// red must hold (blockDim.x/64) * NV values.
template <typename A, int NV> __device__ __forceinline__ void block_sum(A (&v)[NV], A* red)
{
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) red[wid * NV + q] = v[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            A s = 0;
            for (int w = 0; w < nw; ++w) s += red[w * NV + q];
            v[q] = s;
        }
    }
    __syncthreads();
}

__device__ __forceinline__ bool gate_ok(const ReqDesc* R, int gate)
{
    return gate < 0 || R->I[gate] != 0;
}

}  // namespace semk
