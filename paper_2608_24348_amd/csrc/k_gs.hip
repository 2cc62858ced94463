// Direct stiffness summation (gather-scatter Q Q^T) without atomics.
//
// The shared nodes of a request are listed once, grouped by multiplicity:
// pairs (face interiors), quads (edge interiors), octets (vertices), each
// tuple holding the local indices of all copies of one unique node.  A thread
// owns TPT tuples (strided by the workgroup size, so a wave's accesses follow
// the list order): it loads all their indices, then for every component all
// copies, adds the copies in list order and writes the sum back to every
// copy -- deterministic and race free, with several gathers in flight per
// thread.  Nodes with a single copy are untouched.
#include "k_common.h"

namespace semk {

template <typename T, typename A, int M, int TPT, int NC>
__device__ __forceinline__ void gs_chunk(const ReqDesc* R, int field, int gate, void* raw,
                                         const SEM_GLOBAL int* idx, int ntup, int chunk)
{
    const int t = threadIdx.x;
    int id[TPT][M];
    bool own[TPT];
#pragma unroll
    for (int q = 0; q < TPT; ++q) {
        const int tup = (chunk * TPT + q) * SEM_GS_THREADS + t;
        own[q] = tup < ntup;
        // threads past the end repeat the last tuple and never store
        const long long base = (long long)M * (own[q] ? tup : ntup - 1);
#pragma unroll
        for (int m = 0; m < M; ++m) id[q][m] = idx[base + m];
    }
    // every component's gathers are issued before any scatter (a store may
    // alias a later component's loads in the compiler's view, which would
    // otherwise serialise the components)
    T v[NC][TPT][M];
    bool on[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        on[c] = gate_ok(R, gate < 0 ? -1 : gate + c);
        const SEM_GLOBAL T* u = field >= 0 ? gfield<T>(R, field + c) : gp((const T*)raw);
#pragma unroll
        for (int q = 0; q < TPT; ++q)
#pragma unroll
            for (int m = 0; m < M; ++m) v[c][q][m] = ldg(u + id[q][m]);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        if (!on[c]) continue;
        SEM_GLOBAL T* u = field >= 0 ? gfieldw<T>(R, field + c) : gp((T*)raw);
#pragma unroll
        for (int q = 0; q < TPT; ++q) {
            A s = (A)0;
#pragma unroll
            for (int m = 0; m < M; ++m) s += to<A>(v[c][q][m]);
            const T r = to<T>(s);
            if (own[q]) {
#pragma unroll
                for (int m = 0; m < M; ++m) stg(u + id[q][m], r);
            }
        }
    }
}

template <typename T, typename A, int NC>
__global__ void __launch_bounds__(SEM_GS_THREADS)
dssum_kernel(Batch bt, int field, int gate, void* raw)
{
    const int g = blockIdx.x;
    const int ri = find_req(bt.gs, bt.n, g);
    const ReqDesc* R = bt.r[ri];
    int c = g - bt.gs[ri];
    if (c < R->c2) {
        gs_chunk<T, A, 2, SEM_GS_TPT2, NC>(R, field, gate, raw, gp(R->idx2), R->n2, c);
        return;
    }
    c -= R->c2;
    if (c < R->c4) {
        gs_chunk<T, A, 4, SEM_GS_TPT4, NC>(R, field, gate, raw, gp(R->idx4), R->n4, c);
        return;
    }
    c -= R->c4;
    gs_chunk<T, A, 8, SEM_GS_TPT8, NC>(R, field, gate, raw, gp(R->idx8), R->n8, c);
}

template <typename T, typename A>
static void dssum_go(const Batch& b, int field, int ncomp, int gate, void* raw, hipStream_t s)
{
    dim3 grid(b.gs[b.n]);
    if (ncomp == 3)
        hipLaunchKernelGGL((dssum_kernel<T, A, 3>), grid, dim3(SEM_GS_THREADS), 0, s, b, field, gate, raw);
    else
        for (int c = 0; c < ncomp; ++c)
            hipLaunchKernelGGL((dssum_kernel<T, A, 1>), grid, dim3(SEM_GS_THREADS), 0, s, b,
                               field >= 0 ? field + c : field, gate < 0 ? gate : gate + c, raw);
}

void launch_dssum(const Batch& b, int field, int ncomp, int tprec, int gate, void* raw, hipStream_t s)
{
    if (b.gs[b.n] == 0) return;
    switch (tprec) {
    case P64: dssum_go<double, double>(b, field, ncomp, gate, raw, s); break;
    case P32: dssum_go<float, float>(b, field, ncomp, gate, raw, s); break;
    case P16: dssum_go<__half, float>(b, field, ncomp, gate, raw, s); break;
    case PBF: dssum_go<__hip_bfloat16, float>(b, field, ncomp, gate, raw, s); break;
    default: break;
    }
}

}  // namespace semk
