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

    const TU* u = a.src >= 0 ? (const TU*)R->f[a.src + comp] : (const TU*)a.u_raw;
    TU* w = a.dst >= 0 ? (TU*)R->f[a.dst + comp] : (TU*)a.w_raw;
    const TG* G = (const TG*)R->f[gfield<TG>()];
    const TG* Bm = (const TG*)R->f[bfield<TG>()];
    const double* pc = a.precond >= 0 ? (const double*)R->f[a.precond] : nullptr;
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

    C ureg[LX], wacc[LX];
    const long long ebase = (long long)ee * L3;
#pragma unroll
    for (int k = 0; k < LX; ++k) {
        C v = (C)0;
        if (live) {
            v = to<C>(u[ebase + k * L2 + ij]);
            if (pc) v *= (C)pc[ebase + k * L2 + ij];
        }
        ureg[k] = v;
        wacc[k] = (C)0;
    }
    __syncthreads();

    const long long gbase = (long long)ee * 6 * L3;
#pragma unroll
    for (int k = 0; k < LX; ++k) {
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
        const int p = k * L2 + ij;
        C grr = 0, grs = 0, grt = 0, gss = 0, gst = 0, gtt = 0;
        if (live) {
            grr = GeoLoad<TG, C>::ld(G + gbase + 0 * L3 + p, gsc);
            grs = GeoLoad<TG, C>::ld(G + gbase + 1 * L3 + p, gsc);
            grt = GeoLoad<TG, C>::ld(G + gbase + 2 * L3 + p, gsc);
            gss = GeoLoad<TG, C>::ld(G + gbase + 3 * L3 + p, gsc);
            gst = GeoLoad<TG, C>::ld(G + gbase + 4 * L3 + p, gsc);
            gtt = GeoLoad<TG, C>::ld(G + gbase + 5 * L3 + p, gsc);
        }
        const C wr = grr * ur + grs * us + grt * ut;
        const C ws = grs * ur + gss * us + gst * ut;
        const C wt = grt * ur + gst * us + gtt * ut;
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
            C hb = (C)0;
            if (h2 != (C)0) hb = h2 * GeoLoad<TG, C>::ld(Bm + (long long)ee * L3 + p, bsc);
            C wv = h1 * wacc[k] + hb * ureg[k];
            TU ws = to<TU>(wv);
            w[ebase + p] = ws;
            if (a.pdot >= 0) dot += (double)ureg[k] * (double)to<C>(ws);
        }
    }
    if (a.pdot >= 0) {
        double v[1] = {dot};
        block_sum<double, 1>(v, red);
        if (t == 0) R->part[(long long)(a.pdot + comp) * R->nb + blk] = v[0];
    }
}

template <int LX, typename TU, typename TG, typename C>
static void ax_go(const Batch& b, const AxLaunch& a, hipStream_t s)
{
    dim3 grid(b.eb[b.n], a.ncomp);
    hipLaunchKernelGGL((ax_kernel<LX, TU, TG, C>), grid, dim3(Nthr<LX>::v), 0, s, b, a);
}

template <int LX>
static void ax_lx(const Batch& b, const AxLaunch& a, hipStream_t s)
{
    if (a.tu == P64 && a.tg == P64) ax_go<LX, double, double, double>(b, a, s);
    else if (a.tu == P32 && a.tg == P32) ax_go<LX, float, float, float>(b, a, s);
    else if (a.tu == P32 && a.tg == P16) ax_go<LX, float, __half, float>(b, a, s);
    else if (a.tu == P32 && a.tg == PBF) ax_go<LX, float, __hip_bfloat16, float>(b, a, s);
    else if (a.tu == P16 && a.tg == P16) ax_go<LX, __half, __half, float>(b, a, s);
    else if (a.tu == PBF && a.tg == PBF) ax_go<LX, __hip_bfloat16, __hip_bfloat16, float>(b, a, s);
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
