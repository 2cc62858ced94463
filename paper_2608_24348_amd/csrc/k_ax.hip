// Matrix-free Helmholtz operator  w = h1 sum_ab D_a^T (G_ab o D_b u) + h2 B o u
// on GLL hexahedra (sum factorisation), one element per lx*lx-thread slab.
//
// Thread (i,j) of an element owns the column u(i,j,:) in registers and walks
// k: the r- and s-derivatives come from the current k-layer staged in LDS,
// the t-derivative from the register column; the transposed t-contraction
// is accumulated into a register column, the r/s ones through two LDS
// layers.  Every global access is a contiguous lx*lx layer, so G, u and w
// stream coalesced.  Storage types (vectors TU, geometry TG) and compute
// type C are template parameters; 16-bit geometry carries a per-element scale.
#include "k_common.h"

namespace semk {

template <int LX> struct Epb {
    static constexpr int v = epb_of(LX);
};
template <int LX> struct Nthr {
    static constexpr int raw = LX * LX * Epb<LX>::v;
    static constexpr int v = (raw + 63) / 64 * 64;
};

template <typename TG, typename C> struct GeoLoad {
    // geometry value with optional element scale (16-bit storage)
    static __device__ __forceinline__ C ld(const TG* p, C scale) { return to<C>(*p) * scale; }
};
template <typename C> struct GeoLoad<double, C> {
    static __device__ __forceinline__ C ld(const double* p, C) { return (C)*p; }
};
template <typename C> struct GeoLoad<float, C> {
    static __device__ __forceinline__ C ld(const float* p, C) { return (C)*p; }
};

template <typename TG> __device__ __forceinline__ int gfield() { return F_G16; }
template <> __device__ __forceinline__ int gfield<double>() { return F_G64; }
template <> __device__ __forceinline__ int gfield<float>() { return F_G32; }
template <typename TG> __device__ __forceinline__ int bfield() { return F_B16; }
template <> __device__ __forceinline__ int bfield<double>() { return F_B64; }
template <> __device__ __forceinline__ int bfield<float>() { return F_B32; }

template <int LX, typename TU, typename TG, typename C>
__global__ void __launch_bounds__(Nthr<LX>::v)
ax_kernel(Batch bt, AxLaunch a)
{
    constexpr int EPB = Epb<LX>::v;
    constexpr int L2 = LX * LX;
    constexpr int L3 = LX * LX * LX;
    __shared__ C sD[L2];
    __shared__ C su[EPB][L2];
    __shared__ C sr[EPB][L2];
    __shared__ C ss[EPB][L2];
    __shared__ double red[Nthr<LX>::v / 64];

    const int g = blockIdx.x;
    const int ri = find_req(bt.eb, bt.n, g);
    const ReqDesc* R = bt.r[ri];
    const int blk = g - bt.eb[ri];
    const int comp = blockIdx.y;
    if (!gate_ok(R, a.gate < 0 ? -1 : a.gate + comp)) return;

    const int t = threadIdx.x;
    const int el = t / L2;
    const int ij = t - el * L2;
    const int i = ij % LX, j = ij / LX;
    const int e = blk * EPB + el;
    const bool live = el < EPB && e < R->E;

    for (int q = t; q < L2; q += blockDim.x) {
        if constexpr (sizeof(C) == 8) sD[q] = (C)R->D64[q];
        else sD[q] = (C)R->D32[q];
    }

    const TU* u = a.src_vj ? (const TU*)R->f[F_V] + (long long)R->I[I_GJ] * R->np
                           : a.src >= 0 ? (const TU*)R->f[a.src + comp] : (const TU*)a.u_raw;
    TU* w = a.dst >= 0 ? (TU*)R->f[a.dst + comp] : (TU*)a.w_raw;
    const TG* G = (const TG*)R->f[gfield<TG>()];
    const TG* Bm = (const TG*)R->f[bfield<TG>()];
    const double* pc64 = a.precond >= 0 && a.tpc == P64 ? (const double*)R->f[a.precond] : nullptr;
    const float* pc32 = a.precond >= 0 && a.tpc == P32 ? (const float*)R->f[a.precond] : nullptr;
    C h1, h2;
    if (a.hsel >= 0) { h1 = (C)R->S[a.hsel]; h2 = (C)R->S[a.hsel + 1]; }
    else { h1 = (C)a.h1; h2 = (C)a.h2; }
    C gsc = (C)1, bsc = (C)1;
    const int ee = live ? e : 0;
    if (sizeof(TG) == 2) {
        const float* sc = (const float*)R->f[F_GSC];
        gsc = (C)sc[ee];
        bsc = (C)sc[R->E + ee];
    }

    // The column's global loads are issued ahead of the k-walk: all of u and
    // B up front, and the six G_ab either all up front (when they fit in
    // registers) or one layer ahead, so the walk itself only waits on LDS.
#ifndef SEM_AX_GALL_BYTES
#define SEM_AX_GALL_BYTES 384
#endif
    constexpr bool GALL = 6 * LX * sizeof(C) <= SEM_AX_GALL_BYTES;
    constexpr int NG = GALL ? LX : 2;
    C ureg[LX], wacc[LX], bcol[LX], g6[6][NG];
    const long long ebase = (long long)ee * L3;
    const long long gbase = (long long)ee * 6 * L3;
    const bool helm = h2 != (C)0;
#pragma unroll
    for (int k = 0; k < LX; ++k) {
        const int p = k * L2 + ij;
        C v = (C)0;
        if (live) {
            v = to<C>(u[ebase + p]);
            if (pc64) v *= (C)pc64[ebase + p];
            else if (pc32) v *= (C)pc32[ebase + p];
        }
        ureg[k] = v;
        wacc[k] = (C)0;
        if (GALL) bcol[k] = (live && helm) ? GeoLoad<TG, C>::ld(Bm + ebase + p, bsc) : (C)0;
        if (GALL || k == 0) {
#pragma unroll
            for (int q = 0; q < 6; ++q) g6[q][GALL ? k : 0] = live ? GeoLoad<TG, C>::ld(G + gbase + q * L3 + p, gsc) : (C)0;
        }
    }
    __syncthreads();

#pragma unroll
    for (int k = 0; k < LX; ++k) {
        const int kc = GALL ? k : (k & 1);
        if (!GALL && k + 1 < LX) {
            const int pn = (k + 1) * L2 + ij;
#pragma unroll
            for (int q = 0; q < 6; ++q) g6[q][(k + 1) & 1] = live ? GeoLoad<TG, C>::ld(G + gbase + q * L3 + pn, gsc) : (C)0;
        }
        if (el < EPB) su[el][ij] = ureg[k];
        __syncthreads();
        C ur = 0, us = 0, ut = 0;
        if (el < EPB) {
#pragma unroll
            for (int l = 0; l < LX; ++l) {
                ur += sD[i * LX + l] * su[el][j * LX + l];
                us += sD[j * LX + l] * su[el][l * LX + i];
                ut += sD[k * LX + l] * ureg[l];
            }
        }
        const C wr = g6[0][kc] * ur + g6[1][kc] * us + g6[2][kc] * ut;
        const C ws = g6[1][kc] * ur + g6[3][kc] * us + g6[4][kc] * ut;
        const C wt = g6[2][kc] * ur + g6[4][kc] * us + g6[5][kc] * ut;
        if (el < EPB) { sr[el][ij] = wr; ss[el][ij] = ws; }
#pragma unroll
        for (int l = 0; l < LX; ++l) wacc[l] += sD[k * LX + l] * wt;
        __syncthreads();
        if (el < EPB) {
            C acc = 0;
#pragma unroll
            for (int l = 0; l < LX; ++l) {
                acc += sD[l * LX + i] * sr[el][j * LX + l];
                acc += sD[l * LX + j] * ss[el][l * LX + i];
            }
            wacc[k] += acc;
        }
    }

    double dot = 0.0;
    if (live) {
#pragma unroll
        for (int k = 0; k < LX; ++k) {
            const int p = k * L2 + ij;
            const C bk = GALL ? bcol[k] : (helm ? GeoLoad<TG, C>::ld(Bm + ebase + p, bsc) : (C)0);
            const C wv = h1 * wacc[k] + h2 * bk * ureg[k];
            const TU ws = to<TU>(wv);
            w[ebase + p] = ws;
            if (a.pdot >= 0) dot += (double)ureg[k] * (double)to<C>(ws);
        }
    }
    if (a.pdot >= 0) {
        double v[1] = {dot};
        block_sum<double, 1>(v, red);
        if (t == 0) {
            R->part[(long long)(a.pdot + comp) * R->pstride + blk] = v[0];
            if (blk == 0) R->I[I_PCNT + a.pdot + comp] = R->nb;
        }
    }
}

template <int LX, typename TU, typename TG, typename C>
static void ax_go(const Batch& b, const AxLaunch& a, hipStream_t s)
{
    dim3 grid(b.eb[b.n], a.ncomp);
    hipLaunchKernelGGL((ax_kernel<LX, TU, TG, C>), grid, dim3(Nthr<LX>::v), 0, s, b, a);
}

// supported (vector, geometry, arithmetic) instantiations; ax_supported()
// in the host runtime lists the same set
template <int LX>
static void ax_lx(const Batch& b, const AxLaunch& a, hipStream_t s)
{
    const int u = a.tu, g = a.tg, c = a.tc;
    if (u == P64 && g == P64 && c == P64) ax_go<LX, double, double, double>(b, a, s);
    else if (u == P64 && g == P32 && c == P64) ax_go<LX, double, float, double>(b, a, s);
    else if (u == P64 && g == P16 && c == P64) ax_go<LX, double, __half, double>(b, a, s);
    else if (u == P64 && g == PBF && c == P64) ax_go<LX, double, __hip_bfloat16, double>(b, a, s);
    else if (u == P64 && g == P32 && c == P32) ax_go<LX, double, float, float>(b, a, s);
    else if (u == P64 && g == P16 && c == P32) ax_go<LX, double, __half, float>(b, a, s);
    else if (u == P64 && g == PBF && c == P32) ax_go<LX, double, __hip_bfloat16, float>(b, a, s);
    else if (u == P32 && g == P32 && c == P32) ax_go<LX, float, float, float>(b, a, s);
    else if (u == P32 && g == P16 && c == P32) ax_go<LX, float, __half, float>(b, a, s);
    else if (u == P32 && g == PBF && c == P32) ax_go<LX, float, __hip_bfloat16, float>(b, a, s);
    else if (u == P16 && g == P16 && c == P32) ax_go<LX, __half, __half, float>(b, a, s);
    else if (u == PBF && g == PBF && c == P32) ax_go<LX, __hip_bfloat16, __hip_bfloat16, float>(b, a, s);
}

void launch_ax(const Batch& b, int lx, const AxLaunch& a, hipStream_t s)
{
    switch (lx) {
    case 3: ax_lx<3>(b, a, s); break;
    case 4: ax_lx<4>(b, a, s); break;
    case 5: ax_lx<5>(b, a, s); break;
    case 6: ax_lx<6>(b, a, s); break;
    case 7: ax_lx<7>(b, a, s); break;
    case 8: ax_lx<8>(b, a, s); break;
    case 9: ax_lx<9>(b, a, s); break;
    case 10: ax_lx<10>(b, a, s); break;
    case 11: ax_lx<11>(b, a, s); break;
    case 12: ax_lx<12>(b, a, s); break;
    default: break;
    }
}

}  // namespace semk
