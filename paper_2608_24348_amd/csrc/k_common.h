// Device helpers shared by the libsem kernels: type conversion, per-point
// inverse multiplicity and deterministic workgroup reductions.
#pragma once
#include "sem_internal.h"

namespace semk {

// Field pointers are read from the request descriptor in device memory, so
// the compiler cannot infer their address space and would emit FLAT
// accesses (which also count against the LDS wait counter and so stall the
// LDS-heavy contractions on every outstanding HBM load).  Every kernel
// converts them to global-address-space pointers first.
#define SEM_GLOBAL __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ SEM_GLOBAL T* gp(T* p) { return (SEM_GLOBAL T*)p; }
template <typename T> __device__ __forceinline__ const SEM_GLOBAL T* gp(const T* p) { return (const SEM_GLOBAL T*)p; }
template <typename T> __device__ __forceinline__ const SEM_GLOBAL T* gfield(const ReqDesc* R, int id)
{
    return (const SEM_GLOBAL T*)R->f[id];
}
template <typename T> __device__ __forceinline__ SEM_GLOBAL T* gfieldw(const ReqDesc* R, int id)
{
    return (SEM_GLOBAL T*)R->f[id];
}

// Workgroup barrier for LDS producer/consumer hand-offs only: waits for this
// wave's LDS operations (lgkmcnt) but not for its outstanding global loads,
// so prefetched HBM data stays in flight across the barrier (__syncthreads()
// would also drain vmcnt).  Global data that other waves must see still goes
// through __syncthreads().
__device__ __forceinline__ void block_sync_lds()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Hand-off between per-element LDS layers.  WAVE: each element is exactly one
// wave, so its layers are private to that wave and a wave's LDS operations
// complete in order -- waiting for its own LDS traffic is enough and the waves
// of a workgroup never wait for each other.  Otherwise elements span waves and
// the workgroup barrier is needed.
template <bool WAVE> __device__ __forceinline__ void lds_handoff()
{
    if constexpr (WAVE) asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    else block_sync_lds();
}

// loads and stores through global pointers (16-bit types move as raw bits)
template <typename T> __device__ __forceinline__ T ldg(const SEM_GLOBAL T* p) { return *p; }
template <> __device__ __forceinline__ __half ldg<__half>(const SEM_GLOBAL __half* p)
{
    return __ushort_as_half(*(const SEM_GLOBAL unsigned short*)p);
}
template <> __device__ __forceinline__ __hip_bfloat16 ldg<__hip_bfloat16>(const SEM_GLOBAL __hip_bfloat16* p)
{
    return __ushort_as_bfloat16(*(const SEM_GLOBAL unsigned short*)p);
}
template <typename T> __device__ __forceinline__ void stg(SEM_GLOBAL T* p, T v) { *p = v; }
template <> __device__ __forceinline__ void stg<__half>(SEM_GLOBAL __half* p, __half v)
{
    *(SEM_GLOBAL unsigned short*)p = __half_as_ushort(v);
}
template <> __device__ __forceinline__ void stg<__hip_bfloat16>(SEM_GLOBAL __hip_bfloat16* p, __hip_bfloat16 v)
{
    *(SEM_GLOBAL unsigned short*)p = __bfloat16_as_ushort(v);
}

// Streaming loads for data each launch reads exactly once (geometric factors,
// metric terms): the nontemporal hint keeps them from evicting the solver
// vectors that the next kernel reads again from the caches.
template <typename T> __device__ __forceinline__ T ldg_stream(const SEM_GLOBAL T* p) { return __builtin_nontemporal_load(p); }
template <> __device__ __forceinline__ __half ldg_stream<__half>(const SEM_GLOBAL __half* p)
{
    return __ushort_as_half(__builtin_nontemporal_load((const SEM_GLOBAL unsigned short*)p));
}
template <> __device__ __forceinline__ __hip_bfloat16 ldg_stream<__hip_bfloat16>(const SEM_GLOBAL __hip_bfloat16* p)
{
    return __ushort_as_bfloat16(__builtin_nontemporal_load((const SEM_GLOBAL unsigned short*)p));
}

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

// Coordinates of local node (i,j,k) of element e: reference position in the
// box plus the optional smooth perturbation amp*h_c*prod_q sin(pi X_q/h_q + phi).
__device__ __forceinline__ void node_xyz(const MeshParams& mp, const double* xi, int e, int i, int j, int k, double out[3])
{
    const int ex = e % mp.nel[0];
    const int ey = (e / mp.nel[0]) % mp.nel[1];
    const int ez = e / (mp.nel[0] * mp.nel[1]);
    double X[3] = {(ex + 0.5 * (1.0 + xi[i])) * mp.h[0], (ey + 0.5 * (1.0 + xi[j])) * mp.h[1],
                   (ez + 0.5 * (1.0 + xi[k])) * mp.h[2]};
    const double pi = 3.14159265358979323846;
    for (int c = 0; c < 3; ++c) {
        double d = 0.0;
        if (mp.amp != 0.0) {
            d = mp.amp * mp.h[c];
            for (int q = 0; q < 3; ++q) d *= sin(pi * X[q] / mp.h[q] + mp.phase[3 * c + q]);
        }
        out[c] = mp.lo[c] + X[c] + d;
    }
}

__device__ __forceinline__ bool gate_ok(const ReqDesc* R, int gate)
{
    return gate < 0 || gp(R->I)[gate] != 0;
}

}  // namespace semk
