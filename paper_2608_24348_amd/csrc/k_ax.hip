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
// H16 (1 fp16, 2 bf16) selects 16-bit arithmetic with fp32 accumulation: the
// operands of every contraction are 16-bit values -- u scaled per element by
// the power of two s that puts max|u| in [0.5, 1), D, and the weighted
// derivatives entering the transposed contractions, each rounded to nearest
// even -- multiplied exactly and summed in fp32, with the stored normalised G
// in the point-wise stage and h1 gsc / s applied at the end (the matrix-core
// kernel computes the same).
#include "k_common.h"

#include <type_traits>

// register budget (bytes per thread) under which all six geometric factors of
// a column are loaded before the k-walk instead of one layer ahead: lx <= 8 in
// fp32.  At lx = 12 the whole column's G (72 VGPRs) held the fp32 operators
// at one five-wave workgroup per CU; loaded a layer ahead, two fit.
#ifndef SEM_AX_GALL_BYTES
#define SEM_AX_GALL_BYTES 192
#endif

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
    static __device__ __forceinline__ C ld(const SEM_GLOBAL TG* p, C scale) { return to<C>(ldg(p)) * scale; }
};
template <typename C> struct GeoLoad<double, C> {
    static __device__ __forceinline__ C ld(const SEM_GLOBAL double* p, C) { return (C)*p; }
};
template <typename C> struct GeoLoad<float, C> {
    static __device__ __forceinline__ C ld(const SEM_GLOBAL float* p, C) { return (C)*p; }
};

template <typename TG> __device__ __forceinline__ int gfield_id() { return F_G16; }
template <> __device__ __forceinline__ int gfield_id<double>() { return F_G64; }
template <> __device__ __forceinline__ int gfield_id<float>() { return F_G32; }
template <typename TG> __device__ __forceinline__ int bfield() { return F_B16; }
template <> __device__ __forceinline__ int bfield<double>() { return F_B64; }
template <> __device__ __forceinline__ int bfield<float>() { return F_B32; }

// a value rounded to the 16-bit format H16 names (1 fp16, 2 bf16) and back;
// H16 == 0 returns it unchanged in its own type (fp64 arithmetic stays fp64)
template <int H16, typename C> __device__ __forceinline__ C r16(C x)
{
    if constexpr (H16 == 1) return (C)(float)(_Float16)(float)x;
    else if constexpr (H16 == 2) return (C)(float)(__bf16)(float)x;
    else return x;
}

// one element per wave at lx = 8 (64 columns): the k-walk's layers are wave-private
template <int LX> struct AxWave {
    static constexpr bool v = LX * LX == 64 && Nthr<LX>::v == Epb<LX>::v * 64;
};

// PC: Jacobi scaling of the input on load (0 none, 1 fp64 diagonal, 2 fp32),
// a template parameter so the load stays unconditional
// SUB: residual form, w = r_L - (operator u) with r_L the local (unassembled)
// right-hand side a.sub; the caller assembles w afterwards, which equals
// dssum(r_L) - dssum(operator u) (QQ^T is linear)
template <int LX, typename TU, typename TG, typename C, int PC, typename TW, int SUB = 0, int H16 = 0, int SHG = 0>
__global__ void __launch_bounds__(Nthr<LX>::v)
ax_kernel(Batch bt, AxLaunch a)
{
    constexpr int EPB = Epb<LX>::v;
    constexpr int L2 = LX * LX;
    constexpr int L3 = LX * LX * LX;
    static_assert(H16 == 0 || (sizeof(C) == 4 && sizeof(TG) == 2 && SUB == 0), "16-bit arithmetic: fp32 sums, 16-bit G");
    __shared__ C sD[L2];
    __shared__ C su[EPB][L2];
    __shared__ C sr[EPB][L2];
    __shared__ C ss[EPB][L2];
    __shared__ double red[Nthr<LX>::v / 64];
    __shared__ float smax[H16 ? EPB : 1];

    // Components of one element block run as blocks x, x+8, x+16 of a 1-D
    // grid: workgroups go round-robin over the 8 XCDs, so those land on the
    // same XCD back to back and the geometric factors the components share
    // are read from HBM once and from that XCD's L2 after.
    const int bx = blockIdx.x;
    const int comp = (bx / 8) % a.ncomp;
    const int g = (bx / (8 * a.ncomp)) * 8 + (bx & 7);
    if (g >= bt.eb[bt.n]) return;
    const int ri = find_req(bt.eb, bt.n, g);
    const ReqDesc* R = bt.r[ri];
    const int blk = g - bt.eb[ri];
    if (!gate_ok(R, a.gate < 0 ? -1 : a.gate + comp)) return;

    const int t = threadIdx.x;
    const int el = t / L2;
    const int ij = t - el * L2;
    const int i = ij % LX, j = ij / LX;
    const int e = blk * EPB + el;
    const bool live = el < EPB && e < R->E;

    for (int q = t; q < L2; q += blockDim.x) {
        if constexpr (sizeof(C) == 8) sD[q] = (C)gp(R->D64)[q];
        else sD[q] = r16<H16>(gp(R->D32)[q]);
    }
    if constexpr (H16 != 0) {
        if (t < EPB) smax[t] = 0.0f;
        block_sync_lds();
    }

    const SEM_GLOBAL TU* u = a.src_vj ? gfield<TU>(R, F_V) + (long long)gp(R->I)[I_GJ] * R->np
                                      : a.src >= 0 ? gfield<TU>(R, a.src + comp) : gp((const TU*)a.u_raw);
    SEM_GLOBAL TW* w = a.dst >= 0 ? gfieldw<TW>(R, a.dst + comp) : gp((TW*)a.w_raw);
    const SEM_GLOBAL TG* G = gfield<TG>(R, gfield_id<TG>());
    const SEM_GLOBAL TG* Bm = gfield<TG>(R, bfield<TG>());
    using TPC = typename std::conditional<PC == 2, float, double>::type;
    const SEM_GLOBAL TPC* pcv = PC ? gfield<TPC>(R, a.precond) : nullptr;
    C h1, h2;
    if (a.hsel >= 0) { h1 = (C)gp(R->S)[a.hsel]; h2 = (C)gp(R->S)[a.hsel + 1]; }
    else { h1 = (C)a.h1; h2 = (C)a.h2; }
    // a stored GMRES basis vector is unnormalised: A (s_J V_J) = s_J A V_J
    if (a.src_vj) h1 *= (C)gp(R->S)[S_GVS + gp(R->I)[I_GJ]];
    C gsc = (C)1, bsc = (C)1;
    const int ee = live ? e : 0;
    const bool helm = h2 != (C)0;
    if (sizeof(TG) == 2) {
        const SEM_GLOBAL float* sc = gfield<float>(R, F_GSC);
        gsc = (C)sc[ee];
        bsc = (C)sc[R->E + ee];
    }
    // 16-bit arithmetic takes the stored normalised G; gsc goes to the end
    const C gmul = H16 ? (C)1 : gsc;

    // The column's global loads are issued ahead of the k-walk and kept in
    // their storage type (converted only where they are used): u first, then
    // the six G_ab one layer ahead (all up front for fp32 arithmetic on
    // short columns), B at the end.  The thread's D rows/columns live in
    // registers; only the k-uniform row D[k][.] is read from LDS (broadcast).
    constexpr bool GALL = sizeof(C) == 4 && 6 * LX * 4 <= SEM_AX_GALL_BYTES;
    constexpr int NG = GALL ? LX : 2;
    TU uraw[LX];
    TG graw[6][NG];
    TG braw[LX];
    TPC praw[PC ? LX : 1];
    TW rraw[SUB ? LX : 1];
    C ureg[LX], wacc[LX];
    const long long ebase = (long long)ee * L3;
    const long long gbase = (long long)ee * 6 * L3;
    // Loads are unconditional: threads without an element (block padding or
    // past the last element) address element 0 (ee == 0), which always
    // exists, and never store.  Guarding the loads would turn each into a
    // divergent branch whose join waits for it.
    // SHG: the geometric factors bypass L2 retention when one component reads
    // them; the components of a multi-component launch (SHG = 1) share them
    // through L2 (the three-component fp64 velocity residual at 32^3, N = 7:
    // 0.459 ms against 0.472 ms with the bypass).  A compile-time choice: a
    // run-time one cost the single-component forms 8%.
    auto gload = [](const SEM_GLOBAL TG* p) { if constexpr (SHG != 0) return ldg(p); else return ldg_stream(p); };
#pragma unroll
    for (int k = 0; k < LX; ++k) uraw[k] = ldg(u + ebase + k * L2 + ij);
    if constexpr (PC != 0) {
#pragma unroll
        for (int k = 0; k < LX; ++k) praw[k] = ldg(pcv + ebase + k * L2 + ij);
    }
    if (helm) {
#pragma unroll
        for (int k = 0; k < LX; ++k) braw[k] = ldg(Bm + ebase + k * L2 + ij);
    }
#pragma unroll
    for (int k = 0; k < NG; ++k) {
        if (GALL || k == 0) {
#pragma unroll
            for (int q = 0; q < 6; ++q)
                graw[q][k] = gload(G + gbase + q * L3 + k * L2 + ij);
        }
    }
    // uin: the operator's input as stored (Jacobi-scaled); ureg: what the
    // contractions read (uin, or its scaled 16-bit rounding)
    C uin[H16 ? LX : 1];
#pragma unroll
    for (int k = 0; k < LX; ++k) {
        C v = to<C>(uraw[k]);
        if constexpr (PC != 0) v *= (C)praw[k];
        ureg[k] = v;
        wacc[k] = (C)0;
    }
    if constexpr (H16 != 0) {
        float mx = 0.0f;
#pragma unroll
        for (int k = 0; k < LX; ++k) mx = fmaxf(mx, fabsf((float)ureg[k]));
        // the element's max over its columns (non-negative floats order as their bits)
        if (el < EPB) atomicMax((int*)&smax[el], __float_as_int(mx));
    }
    block_sync_lds();  // sD ready (and the element maxima)
    C Di[LX], Dj[LX], DTi[LX], DTj[LX];
#pragma unroll
    for (int l = 0; l < LX; ++l) {
        Di[l] = sD[i * LX + l];
        Dj[l] = sD[j * LX + l];
        DTi[l] = sD[l * LX + i];
        DTj[l] = sD[l * LX + j];
    }
    C hscale = (C)1;  // 1/s
    if constexpr (H16 != 0) {
        const float m = smax[el < EPB ? el : 0];
        float sc = 1.0f;
        if (m > 0.0f && m < INFINITY) {
            int ex;
            (void)frexpf(m, &ex);
            sc = ldexpf(1.0f, -ex);
        }
        hscale = (C)(1.0f / sc);
#pragma unroll
        for (int k = 0; k < LX; ++k) {
            uin[k] = ureg[k];
            ureg[k] = r16<H16>(ureg[k] * sc);
        }
    }

#pragma unroll
    for (int k = 0; k < LX; ++k) {
        const int kc = GALL ? k : (k & 1);
        if (!GALL && k + 1 < LX) {
            const int pn = (k + 1) * L2 + ij;
#pragma unroll
            for (int q = 0; q < 6; ++q)
                graw[q][(k + 1) & 1] = gload(G + gbase + q * L3 + pn);
        }
        if (el < EPB) su[el][ij] = ureg[k];
        lds_handoff<AxWave<LX>::v>();
        C ur = 0, us = 0, ut = 0;
        if (el < EPB) {
#pragma unroll
            for (int l = 0; l < LX; ++l) {
                ur += Di[l] * su[el][j * LX + l];
                us += Dj[l] * su[el][l * LX + i];
                ut += sD[k * LX + l] * ureg[l];
            }
        }
        C g6[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) g6[q] = to<C>(graw[q][kc]) * gmul;
        const C wr = r16<H16>(g6[0] * ur + g6[1] * us + g6[2] * ut);
        const C ws = r16<H16>(g6[1] * ur + g6[3] * us + g6[4] * ut);
        const C wt = r16<H16>(g6[2] * ur + g6[4] * us + g6[5] * ut);
        if (el < EPB) { sr[el][ij] = wr; ss[el][ij] = ws; }
#pragma unroll
        for (int l = 0; l < LX; ++l) wacc[l] += sD[k * LX + l] * wt;
        lds_handoff<AxWave<LX>::v>();
        if (el < EPB) {
            C acc = 0;
#pragma unroll
            for (int l = 0; l < LX; ++l) {
                acc += DTi[l] * sr[el][j * LX + l];
                acc += DTj[l] * ss[el][l * LX + i];
            }
            wacc[k] += acc;
        }
    }

    // the local rhs of the residual form is loaded only now: it is needed at
    // the store, and holding it through the k-walk would cost the registers
    // of a second wave per SIMD
    if constexpr (SUB != 0) {
        const SEM_GLOBAL TW* rl = gfield<TW>(R, a.sub + comp);
#pragma unroll
        for (int k = 0; k < LX; ++k) rraw[k] = ldg(rl + ebase + k * L2 + ij);
    }
    double dot = 0.0;
    if (live) {
        const C hs = H16 ? h1 * (gsc * hscale) : h1;
#pragma unroll
        for (int k = 0; k < LX; ++k) {
            const int p = k * L2 + ij;
            const C uk = H16 ? uin[H16 ? k : 0] : ureg[k];
            const C bk = helm ? to<C>(braw[k]) * bsc : (C)0;
            const C wv = hs * wacc[k] + h2 * bk * uk;
            const TW ws = SUB ? (TW)(rraw[k] - to<TW>(wv)) : to<TW>(wv);
            stg(w + ebase + p, ws);
            if (a.pdot >= 0) dot += (double)uk * (double)to<C>(ws);
        }
    }
    if (a.pdot >= 0) {
        double v[1] = {dot};
        block_sum<double, 1>(v, red);
        if (t == 0) {
            gp(R->part)[(long long)(a.pdot + comp) * R->pstride + blk] = v[0];
            if (blk == 0) gp(R->I)[I_PCNT + a.pdot + comp] = R->nb;
        }
    }
}

template <int LX, typename TU, typename TG, typename C, int H16 = 0>
static void ax_go(const Batch& b, const AxLaunch& a, hipStream_t s)
{
    // 1-D grid: groups of 8 element blocks, each group once per component
    dim3 grid(((b.eb[b.n] + 7) / 8) * 8 * a.ncomp);
    if constexpr (sizeof(TU) == 4) {
        // the Arnoldi operator of an fp32-stored GMRES basis: Jacobi scaling on
        // load and an fp64 output
        if (a.out64) {
            if (a.precond >= 0 && a.tpc == P64)
                hipLaunchKernelGGL((ax_kernel<LX, TU, TG, C, 1, double, 0, H16>), grid, dim3(Nthr<LX>::v), 0, s, b, a);
            else if (a.precond >= 0)
                hipLaunchKernelGGL((ax_kernel<LX, TU, TG, C, 2, double, 0, H16>), grid, dim3(Nthr<LX>::v), 0, s, b, a);
            else
                hipLaunchKernelGGL((ax_kernel<LX, TU, TG, C, 0, double, 0, H16>), grid, dim3(Nthr<LX>::v), 0, s, b, a);
            return;
        }
    }
    if constexpr (sizeof(TU) == 8) {
        // the Arnoldi operator of an fp64 GMRES basis (Jacobi scaling on load)
        if (a.precond >= 0 && a.tpc == P64) {
            hipLaunchKernelGGL((ax_kernel<LX, TU, TG, C, 1, TU, 0, H16>), grid, dim3(Nthr<LX>::v), 0, s, b, a);
            return;
        }
        if (a.precond >= 0) {
            hipLaunchKernelGGL((ax_kernel<LX, TU, TG, C, 2, TU, 0, H16>), grid, dim3(Nthr<LX>::v), 0, s, b, a);
            return;
        }
    }
    if constexpr (sizeof(TU) == 8 && sizeof(TG) == 8 && sizeof(C) == 8 && H16 == 0) {
        if (a.sub >= 0) {
            if (a.ncomp > 1) hipLaunchKernelGGL((ax_kernel<LX, TU, TG, C, 0, TU, 1, 0, 1>), grid, dim3(Nthr<LX>::v), 0, s, b, a);
            else hipLaunchKernelGGL((ax_kernel<LX, TU, TG, C, 0, TU, 1>), grid, dim3(Nthr<LX>::v), 0, s, b, a);
            return;
        }
    }
    if (a.ncomp > 1) hipLaunchKernelGGL((ax_kernel<LX, TU, TG, C, 0, TU, 0, H16, 1>), grid, dim3(Nthr<LX>::v), 0, s, b, a);
    else hipLaunchKernelGGL((ax_kernel<LX, TU, TG, C, 0, TU, 0, H16>), grid, dim3(Nthr<LX>::v), 0, s, b, a);
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
    else if (u == P32 && g == P32 && c == P64) ax_go<LX, float, float, double>(b, a, s);
    else if (u == P32 && g == P16 && c == P64) ax_go<LX, float, __half, double>(b, a, s);
    else if (u == P32 && g == PBF && c == P64) ax_go<LX, float, __hip_bfloat16, double>(b, a, s);
    else if (u == P32 && g == P32 && c == P32) ax_go<LX, float, float, float>(b, a, s);
    else if (u == P32 && g == P16 && c == P32) ax_go<LX, float, __half, float>(b, a, s);
    else if (u == P32 && g == PBF && c == P32) ax_go<LX, float, __hip_bfloat16, float>(b, a, s);
    else if (u == P16 && g == P16 && c == P32) ax_go<LX, __half, __half, float>(b, a, s);
    else if (u == PBF && g == PBF && c == P32) ax_go<LX, __hip_bfloat16, __hip_bfloat16, float>(b, a, s);
    // 16-bit arithmetic (fp32 sums)
    else if (u == P32 && g == P16 && c == P16) ax_go<LX, float, __half, float, 1>(b, a, s);
    else if (u == P16 && g == P16 && c == P16) ax_go<LX, __half, __half, float, 1>(b, a, s);
    else if (u == P32 && g == PBF && c == PBF) ax_go<LX, float, __hip_bfloat16, float, 2>(b, a, s);
    else if (u == PBF && g == PBF && c == PBF) ax_go<LX, __hip_bfloat16, __hip_bfloat16, float, 2>(b, a, s);
}

void launch_ax(const Batch& b, int lx, const AxLaunch& a0, hipStream_t s)
{
    AxLaunch a = a0;
    if (a.ncomp < 1) a.ncomp = 1;
    if (launch_ax_mfma(b, lx, a, s)) return;
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
