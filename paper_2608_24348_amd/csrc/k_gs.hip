// Direct stiffness summation (gather-scatter Q Q^T) without atomics.
//
// The shared nodes of a request are listed once, grouped by multiplicity:
// pairs (face interiors), quads (edge interiors), octets (vertices), each
// tuple holding the local indices of all copies of one unique node.  One
// thread owns one tuple: it adds the copies in list order and writes the sum
// back to every copy, so the result is deterministic and race free.  Nodes
// with a single copy are untouched.
#include "k_common.h"

namespace semk {

template <typename T, typename A, int M>
__device__ __forceinline__ void gs_tuple(SEM_GLOBAL T* u, const SEM_GLOBAL int* idx)
{
    int id[M];
#pragma unroll
    for (int q = 0; q < M; ++q) id[q] = idx[q];
    A s = (A)0;
#pragma unroll
    for (int q = 0; q < M; ++q) s += to<A>(ldg(u + id[q]));
    const T v = to<T>(s);
#pragma unroll
    for (int q = 0; q < M; ++q) stg(u + id[q], v);
}

template <typename T, typename A>
__global__ void __launch_bounds__(SEM_GS_CHUNK)
dssum_kernel(Batch bt, int field, int gate, void* raw)
{
    const int g = blockIdx.x;
    const int ri = find_req(bt.gs, bt.n, g);
    const ReqDesc* R = bt.r[ri];
    const int comp = blockIdx.y;
    if (!gate_ok(R, gate < 0 ? -1 : gate + comp)) return;
    SEM_GLOBAL T* u = field >= 0 ? gfieldw<T>(R, field + comp) : gp((T*)raw);
    int c = g - bt.gs[ri];
    const int t = threadIdx.x;
    if (c < R->c2) {
        int tup = c * SEM_GS_CHUNK + t;
        if (tup < R->n2) gs_tuple<T, A, 2>(u, gp(R->idx2) + 2LL * tup);
        return;
    }
    c -= R->c2;
    if (c < R->c4) {
        int tup = c * SEM_GS_CHUNK + t;
        if (tup < R->n4) gs_tuple<T, A, 4>(u, gp(R->idx4) + 4LL * tup);
        return;
    }
    c -= R->c4;
    int tup = c * SEM_GS_CHUNK + t;
    if (tup < R->n8) gs_tuple<T, A, 8>(u, gp(R->idx8) + 8LL * tup);
}

void launch_dssum(const Batch& b, int field, int ncomp, int tprec, int gate, void* raw, hipStream_t s)
{
    dim3 grid(b.gs[b.n], ncomp);
    if (grid.x == 0) return;
    switch (tprec) {
    case P64: hipLaunchKernelGGL((dssum_kernel<double, double>), grid, dim3(SEM_GS_CHUNK), 0, s, b, field, gate, raw); break;
    case P32: hipLaunchKernelGGL((dssum_kernel<float, float>), grid, dim3(SEM_GS_CHUNK), 0, s, b, field, gate, raw); break;
    case P16: hipLaunchKernelGGL((dssum_kernel<__half, float>), grid, dim3(SEM_GS_CHUNK), 0, s, b, field, gate, raw); break;
    case PBF: hipLaunchKernelGGL((dssum_kernel<__hip_bfloat16, float>), grid, dim3(SEM_GS_CHUNK), 0, s, b, field, gate, raw); break;
    default: break;
    }
}

}  // namespace semk
