// Helmholtz/Poisson operator on matrix cores for 16-bit-stored geometry at
// lx = 8 (N = 7):  w = h1 sum_ab D_a^T (G_ab o D_b u) + h2 B o u, fp32
// arithmetic (16x16x4 fp32 MFMA), u and w in fp32, fp16 or bf16 storage.
//
// A wave owns a pair of elements.  Each one-dimensional contraction of the
// pair is a 16x16x16 product done as four 16x16x4 MFMA steps, the 1D matrix
// D (or D^T) one operand, held in registers, the element data the other,
// read from LDS.  The 16 x 16 output tile of tile t holds
//   rows (i, k = 2t + kk)  x  columns (j, e)          (layout "O1")
// for i, j = 0..7, kk, e = 0..1 (e: the element of the pair):
//  - the i-derivative: K runs over (l, kk'), A = delta(kk, kk') D[i][l],
//    B = u_e[2t + kk'][j][l];
//  - the j-derivative: K runs over (l, e'), A = u_e'[2t + kk][l][i],
//    B = delta(e, e') D[j][l];
// so both land in the same lanes and registers.  The k-derivative uses rows
// (k, i = 2t + ii) x columns (j, e) (K over (l, ii'), A = delta(ii, ii') D[k][l],
// B = u_e[l][j][2t + ii']) and goes through LDS once to layout O1, where the
// six G_ab multiply the three derivatives point by point.  The transposed
// contractions run the same way with D^T and accumulate into one tile.
//
// MFMA lane layout (16x16x4 fp32): lane (g = lane / 16, m = lane % 16)
// supplies A[row m][k g] and B[k g][column m] and holds output rows 4g + r,
// column m (r = 0..3).  In layout O1 a lane's four outputs are four
// consecutive i of one (k, j, e): one 8- or 16-byte global access each.
//
// 16-bit arithmetic (axmh_kernel): the operands of every contraction are
// 16-bit values (nearest-even rounding) and the products are summed in fp32;
// one 16x16x16 MFMA (f16 or bf16 inputs, fp32 accumulation) covers a whole
// contraction of a tile.  Its lane (g, m) supplies A[row m][k 4g..4g+3] and
// B[k 4g..4g+3][column m] and holds the same output rows as above.  Per
// element, u is scaled by the power of two s that puts max|u| in [0.5, 1)
// before rounding, D and D^T are rounded once, the stored (power-of-two
// normalised) 16-bit G multiplies in fp32 and the weighted derivatives are
// rounded before the transposed contractions; h1 gsc / s rescales at the end
// (exact), and the mass term is fp32 on the 16-bit B and the stored u.  The
// roundings are therefore relative to the element's own magnitude.
#include "k_common.h"

#include <type_traits>

namespace semk {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef unsigned int u2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f4v mfma16x16x4(float a, float b, f4v c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// LDS stride of an element (512 + 4: the two elements of a pair fall in
// different banks when a wave reads the same offset of both)
constexpr int AXM_ES = 516;
constexpr int AXM_WS = 2 * AXM_ES;  // floats of one buffer of one wave

// in-order LDS within a wave: wait for this wave's outstanding LDS operations
// (the buffers are private to the wave, so no workgroup barrier is needed)
__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// four consecutive values: 16 bytes of fp32 or 8 bytes of 16-bit storage
template <typename T> struct Q4;
template <> struct Q4<float> {
    static __device__ __forceinline__ void ld(const SEM_GLOBAL float* p, float (&o)[4])
    {
        const f4v v = *(const SEM_GLOBAL f4v*)p;
        o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
    }
    static __device__ __forceinline__ void st(SEM_GLOBAL float* p, const float (&o)[4])
    {
        f4v v;
        v.x = o[0]; v.y = o[1]; v.z = o[2]; v.w = o[3];
        *(SEM_GLOBAL f4v*)p = v;
    }
};
__device__ __forceinline__ float h2f(unsigned b) { return __half2float(__ushort_as_half((unsigned short)b)); }
__device__ __forceinline__ float bf2f(unsigned b) { return __uint_as_float(b << 16); }
template <> struct Q4<__half> {
    static __device__ __forceinline__ void unpack(u2v v, float (&o)[4])
    {
        o[0] = h2f(v.x & 0xffffu); o[1] = h2f(v.x >> 16); o[2] = h2f(v.y & 0xffffu); o[3] = h2f(v.y >> 16);
    }
    static __device__ __forceinline__ void ld(const SEM_GLOBAL __half* p, float (&o)[4])
    {
        unpack(*(const SEM_GLOBAL u2v*)p, o);
    }
    static __device__ __forceinline__ void ld_stream(const SEM_GLOBAL __half* p, float (&o)[4])
    {
        unpack(__builtin_nontemporal_load((const SEM_GLOBAL u2v*)p), o);
    }
    static __device__ __forceinline__ void st(SEM_GLOBAL __half* p, const float (&o)[4])
    {
        u2v v;
        v.x = (unsigned)__half_as_ushort(__float2half_rn(o[0])) | ((unsigned)__half_as_ushort(__float2half_rn(o[1])) << 16);
        v.y = (unsigned)__half_as_ushort(__float2half_rn(o[2])) | ((unsigned)__half_as_ushort(__float2half_rn(o[3])) << 16);
        *(SEM_GLOBAL u2v*)p = v;
    }
};
template <> struct Q4<__hip_bfloat16> {
    static __device__ __forceinline__ void unpack(u2v v, float (&o)[4])
    {
        o[0] = bf2f(v.x & 0xffffu); o[1] = bf2f(v.x >> 16); o[2] = bf2f(v.y & 0xffffu); o[3] = bf2f(v.y >> 16);
    }
    static __device__ __forceinline__ void ld(const SEM_GLOBAL __hip_bfloat16* p, float (&o)[4])
    {
        unpack(*(const SEM_GLOBAL u2v*)p, o);
    }
    static __device__ __forceinline__ void ld_stream(const SEM_GLOBAL __hip_bfloat16* p, float (&o)[4])
    {
        unpack(__builtin_nontemporal_load((const SEM_GLOBAL u2v*)p), o);
    }
    static __device__ __forceinline__ void st(SEM_GLOBAL __hip_bfloat16* p, const float (&o)[4])
    {
        u2v v;
        v.x = (unsigned)__bfloat16_as_ushort(__float2bfloat16(o[0])) |
              ((unsigned)__bfloat16_as_ushort(__float2bfloat16(o[1])) << 16);
        v.y = (unsigned)__bfloat16_as_ushort(__float2bfloat16(o[2])) |
              ((unsigned)__bfloat16_as_ushort(__float2bfloat16(o[3])) << 16);
        *(SEM_GLOBAL u2v*)p = v;
    }
};

// storage bits of four consecutive values (converted where they are used, so
// every global load of the kernel can be issued before the first MFMA)
template <typename T> struct Raw4 { typedef u2v type; };
template <> struct Raw4<float> { typedef f4v type; };
template <typename T> __device__ __forceinline__ typename Raw4<T>::type ld_raw(const SEM_GLOBAL T* p)
{
    return *(const SEM_GLOBAL typename Raw4<T>::type*)p;
}
template <typename T> __device__ __forceinline__ typename Raw4<T>::type ld_raw_stream(const SEM_GLOBAL T* p)
{
    return __builtin_nontemporal_load((const SEM_GLOBAL typename Raw4<T>::type*)p);
}
__device__ __forceinline__ void cvt4(f4v v, float (&o)[4]) { o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w; }
template <typename T> __device__ __forceinline__ void cvt4(u2v v, float (&o)[4]) { Q4<T>::unpack(v, o); }
template <typename T> __device__ __forceinline__ void cvt4t(typename Raw4<T>::type v, float (&o)[4])
{
    if constexpr (sizeof(T) == 4) cvt4(v, o);
    else cvt4<T>(v, o);
}

template <typename TU, typename TG, int SHG>
__global__ void __launch_bounds__(128, sizeof(TG) == 4 ? 2 : 3) axm_kernel(Batch bt, AxLaunch a)
{
    constexpr int LX = 8, L3 = 512;
    __shared__ float sbuf[2][3 * AXM_WS];
    __shared__ double red[2];

    // component blocks x, x+8, x+16 of the 1-D grid land on one XCD back to
    // back (the geometric factors they share come from that XCD's L2)
    const int bx = blockIdx.x;
    const int comp = (bx / 8) % a.ncomp;
    const int gi = (bx / (8 * a.ncomp)) * 8 + (bx & 7);
    if (gi >= bt.eb[bt.n]) return;
    const int ri = find_req(bt.eb, bt.n, gi);
    const ReqDesc* R = bt.r[ri];
    const int blk = gi - bt.eb[ri];
    if (!gate_ok(R, a.gate < 0 ? -1 : a.gate + comp)) return;

    const int t = threadIdx.x, w = t >> 6, lane = t & 63, g = lane >> 4, m = lane & 15;
    const int me = m >> 3, mj = m & 7, gh = g >> 1, gl = g & 1;
    float* sU = sbuf[w];
    float* sS = sU + AXM_WS;
    float* sT = sS + AXM_WS;
    // this lane's element: the block holds 4 elements, the wave a pair
    const int e = blk * 4 + 2 * w + me;
    const bool live = e < R->E;
    const int ee = live ? e : 0;  // padding lanes read element 0 (it exists) and never store

    const SEM_GLOBAL TU* u = a.src >= 0 ? gfield<TU>(R, a.src + comp) : gp((const TU*)a.u_raw);
    SEM_GLOBAL TU* wo = a.dst >= 0 ? gfieldw<TU>(R, a.dst + comp) : gp((TU*)a.w_raw);
    constexpr bool G32 = sizeof(TG) == 4;  // fp32 geometry: no element scale
    const SEM_GLOBAL TG* G = gfield<TG>(R, G32 ? F_G32 : F_G16);
    const SEM_GLOBAL TG* Bm = gfield<TG>(R, G32 ? F_B32 : F_B16);
    float h1, h2;
    if (a.hsel >= 0) { h1 = (float)gp(R->S)[a.hsel]; h2 = (float)gp(R->S)[a.hsel + 1]; }
    else { h1 = (float)a.h1; h2 = (float)a.h2; }
    float gsc = 1.0f, bsc = 1.0f;
    if constexpr (!G32) {
        const SEM_GLOBAL float* scl = gfield<float>(R, F_GSC);
        gsc = scl[ee];
        bsc = scl[R->E + ee];
    }

    // D (and D^T) operands of the four k-steps: step s covers l = 4(s%2) + g of
    // the half kk' (or e', ii') = s/2 of the K index; zero off the block
    float cD[4], cDT[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int l = 4 * (s & 1) + g;
        const bool on = me == (s >> 1);
        cD[s] = on ? gp(R->D32)[mj * LX + l] : 0.0f;
        cDT[s] = on ? gp(R->D32)[l * LX + mj] : 0.0f;
    }

    // the lane's points in layout O1: tile t, register r -> (i = 4 gl + r, k = 2t + gh, j = mj).
    // All global loads of the kernel are issued here, ahead of the matrix work.
    const long long eb = (long long)ee * L3;
    const long long gb = (long long)ee * 6 * L3;
    const bool helm = h2 != 0.0f;
    // SHG: the geometric factors bypass L2 retention when one component reads
    // them; the components of a multi-component launch (SHG = 1) share them
    // through L2 (three velocity components at 32^3, N = 7: 66.5 B/point of
    // traffic with the bypass against 52 B/point read once)
    constexpr bool shared_g = SHG != 0;
    typename Raw4<TU>::type uraw[4];
    typename Raw4<TG>::type graw[4][6], braw[4];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) uraw[tt] = ld_raw(u + eb + (2 * tt + gh) * 64 + mj * 8 + 4 * gl);
#pragma unroll
    for (int tt = 0; tt < 4; ++tt)
#pragma unroll
        for (int q = 0; q < 6; ++q)
            graw[tt][q] = shared_g ? ld_raw(G + gb + q * L3 + (2 * tt + gh) * 64 + mj * 8 + 4 * gl)
                                   : ld_raw_stream(G + gb + q * L3 + (2 * tt + gh) * 64 + mj * 8 + 4 * gl);
    if (helm) {
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) braw[tt] = ld_raw(Bm + eb + (2 * tt + gh) * 64 + mj * 8 + 4 * gl);
    }
    float ur[4][4];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        const int o = (2 * tt + gh) * 64 + mj * 8 + 4 * gl;
        cvt4t<TU>(uraw[tt], ur[tt]);
        *(f4v*)(sU + me * AXM_ES + o) = (f4v){ur[tt][0], ur[tt][1], ur[tt][2], ur[tt][3]};
    }
    wave_lds_sync();

    // ---- reference derivatives: i and j in layout O1 (registers), k in the
    // k-row layout, stored to sT in natural order
    f4v dR[4], dS[4];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        f4v aR = {0.f, 0.f, 0.f, 0.f}, aS = aR, aT = aR;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int l = 4 * (s & 1) + g, h = s >> 1;
            aR = mfma16x16x4(cD[s], sU[me * AXM_ES + (2 * tt + h) * 64 + mj * 8 + l], aR);
            aS = mfma16x16x4(sU[h * AXM_ES + (2 * tt + me) * 64 + l * 8 + mj], cD[s], aS);
            aT = mfma16x16x4(cD[s], sU[me * AXM_ES + l * 64 + mj * 8 + 2 * tt + h], aT);
        }
        dR[tt] = aR;
        dS[tt] = aS;
#pragma unroll
        for (int r = 0; r < 4; ++r) sT[me * AXM_ES + (4 * gl + r) * 64 + mj * 8 + 2 * tt + gh] = aT[r];
    }
    wave_lds_sync();

    // ---- point-wise metric terms in layout O1; the weighted derivatives go
    // back to LDS (sU, sS, sT) in natural order
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        const int o = (2 * tt + gh) * 64 + mj * 8 + 4 * gl;
        const f4v dt = *(const f4v*)(sT + me * AXM_ES + o);
        float gv[6][4];
#pragma unroll
        for (int q = 0; q < 6; ++q) cvt4t<TG>(graw[tt][q], gv[q]);
        float wr[4], ws[4], wt[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float x = dR[tt][r], y = dS[tt][r], z = dt[r];
            const float g0 = gv[0][r] * gsc, g1 = gv[1][r] * gsc, g2 = gv[2][r] * gsc;
            const float g3 = gv[3][r] * gsc, g4 = gv[4][r] * gsc, g5 = gv[5][r] * gsc;
            wr[r] = g0 * x + g1 * y + g2 * z;
            ws[r] = g1 * x + g3 * y + g4 * z;
            wt[r] = g2 * x + g4 * y + g5 * z;
        }
        *(f4v*)(sU + me * AXM_ES + o) = (f4v){wr[0], wr[1], wr[2], wr[3]};
        *(f4v*)(sS + me * AXM_ES + o) = (f4v){ws[0], ws[1], ws[2], ws[3]};
        *(f4v*)(sT + me * AXM_ES + o) = (f4v){wt[0], wt[1], wt[2], wt[3]};
    }
    wave_lds_sync();

    // ---- transposed contractions: k (k-row layout, through sT to O1), then
    // i and j accumulated together in O1
    f4v bT[4];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        f4v acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int l = 4 * (s & 1) + g, h = s >> 1;
            acc = mfma16x16x4(cDT[s], sT[me * AXM_ES + l * 64 + mj * 8 + 2 * tt + h], acc);
        }
        bT[tt] = acc;
    }
    wave_lds_sync();
#pragma unroll
    for (int tt = 0; tt < 4; ++tt)
#pragma unroll
        for (int r = 0; r < 4; ++r) sT[me * AXM_ES + (4 * gl + r) * 64 + mj * 8 + 2 * tt + gh] = bT[tt][r];
    f4v acc[4];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        f4v c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int l = 4 * (s & 1) + g, h = s >> 1;
            c = mfma16x16x4(cDT[s], sU[me * AXM_ES + (2 * tt + h) * 64 + mj * 8 + l], c);
            c = mfma16x16x4(sS[h * AXM_ES + (2 * tt + me) * 64 + l * 8 + mj], cDT[s], c);
        }
        acc[tt] = c;
    }
    wave_lds_sync();

    // ---- w = h1 (sum of the three) + h2 B u, stored in layout O1
    double dot = 0.0;
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        const int o = (2 * tt + gh) * 64 + mj * 8 + 4 * gl;
        const f4v kt = *(const f4v*)(sT + me * AXM_ES + o);
        float bv[4] = {0.f, 0.f, 0.f, 0.f};
        if (helm) cvt4t<TG>(braw[tt], bv);
        float wv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) wv[r] = h1 * (acc[tt][r] + kt[r]) + h2 * (bv[r] * bsc) * ur[tt][r];
        if (live) {
            Q4<TU>::st(wo + eb + o, wv);
            if (a.pdot >= 0) {
                // (u, w) with w as stored
#pragma unroll
                for (int r = 0; r < 4; ++r) dot += (double)ur[tt][r] * (double)to<float>(to<TU>(wv[r]));
            }
        }
    }
    if (a.pdot >= 0) {
        dot = wave_sum(dot);
        if (lane == 0) red[w] = dot;
        __syncthreads();
        if (t == 0) {
            gp(R->part)[(long long)(a.pdot + comp) * R->pstride + blk] = red[0] + red[1];
            if (blk == 0) gp(R->I)[I_PCNT + a.pdot + comp] = R->nb;
        }
    }
}


// ---------------------------------------------------------------------------
// 16-bit arithmetic on matrix cores
// ---------------------------------------------------------------------------
typedef _Float16 h4v __attribute__((ext_vector_type(4)));
typedef short s4v __attribute__((ext_vector_type(4)));

template <typename TH> __device__ __forceinline__ f4v mfma16x16x16(u2v a, u2v b, f4v c);
template <> __device__ __forceinline__ f4v mfma16x16x16<__half>(u2v a, u2v b, f4v c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(h4v, a), __builtin_bit_cast(h4v, b), c, 0, 0, 0);
}
template <> __device__ __forceinline__ f4v mfma16x16x16<__hip_bfloat16>(u2v a, u2v b, f4v c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4v, a), __builtin_bit_cast(s4v, b), c, 0, 0, 0);
}

// two fp32 values rounded (nearest even) to a packed pair of 16-bit values
typedef float f2v __attribute__((ext_vector_type(2)));
typedef _Float16 hf2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
template <typename TH> __device__ __forceinline__ unsigned pack2(float a, float b);
template <> __device__ __forceinline__ unsigned pack2<__half>(float a, float b)
{
    return __builtin_bit_cast(unsigned, __builtin_convertvector((f2v){a, b}, hf2v));
}
template <> __device__ __forceinline__ unsigned pack2<__hip_bfloat16>(float a, float b)
{
    return __builtin_bit_cast(unsigned, __builtin_convertvector((f2v){a, b}, bf2v));
}
template <typename TH> __device__ __forceinline__ u2v pack16(float a, float b, float c, float d)
{
    return (u2v){pack2<TH>(a, b), pack2<TH>(c, d)};
}
// four 16-bit values at stride st (in elements) from LDS, packed (the
// values are only moved, never computed on, so reading bf16 bits through
// the f16 type is exact)
__device__ __forceinline__ u2v lds4s(const unsigned short* p, int st)
{
    const _Float16* h = (const _Float16*)p;
    return __builtin_bit_cast(u2v, (h4v){h[0], h[st], h[2 * st], h[3 * st]});
}
__device__ __forceinline__ u2v lds4c(const unsigned short* p) { return *(const u2v*)p; }

// max over the 32 lanes of one element of the pair (lane bits 0-2 and 4-5)
__device__ __forceinline__ float pair_elem_max(float v)
{
    v = fmaxf(v, __shfl_xor(v, 1));
    v = fmaxf(v, __shfl_xor(v, 2));
    v = fmaxf(v, __shfl_xor(v, 4));
    v = fmaxf(v, __shfl_xor(v, 16));
    v = fmaxf(v, __shfl_xor(v, 32));
    return v;
}
// the power of two s with m s in [0.5, 1) (1 when m is 0 or not finite)
__device__ __forceinline__ float pow2_scale(float m)
{
    if (!(m > 0.0f) || !(m < INFINITY)) return 1.0f;
    int ex;
    (void)frexpf(m, &ex);
    return ldexpf(1.0f, -ex);
}

// 16-bit LDS stride of an element (512 + 8: the pair's copies start in
// different banks, and 4-value groups stay 8-byte aligned)
constexpr int AXH_ES = 520;
constexpr int AXH_WS = 2 * AXH_ES;

template <typename TU, typename TH, int SHG>
__global__ void __launch_bounds__(128, 3) axmh_kernel(Batch bt, AxLaunch a)
{
    constexpr int LX = 8, L3 = 512;
    __shared__ unsigned short hbuf[2][4 * AXH_WS];  // per wave: u, then w_r, w_s, w_t (16-bit)
    __shared__ float tbuf[2][AXM_WS];               // per wave: the k-contractions' layout change
    __shared__ double red[2];

    const int bx = blockIdx.x;
    const int comp = (bx / 8) % a.ncomp;
    const int gi = (bx / (8 * a.ncomp)) * 8 + (bx & 7);
    if (gi >= bt.eb[bt.n]) return;
    const int ri = find_req(bt.eb, bt.n, gi);
    const ReqDesc* R = bt.r[ri];
    const int blk = gi - bt.eb[ri];
    if (!gate_ok(R, a.gate < 0 ? -1 : a.gate + comp)) return;

    const int t = threadIdx.x, w = t >> 6, lane = t & 63, g = lane >> 4, m = lane & 15;
    const int me = m >> 3, mj = m & 7, gh = g >> 1, gl = g & 1;
    unsigned short* hU = hbuf[w];
    unsigned short* hR = hU + AXH_WS;
    unsigned short* hS = hR + AXH_WS;
    unsigned short* hT = hS + AXH_WS;
    float* sT = tbuf[w];
    const int e = blk * 4 + 2 * w + me;
    const bool live = e < R->E;
    const int ee = live ? e : 0;  // padding lanes read element 0 (it exists) and never store

    const SEM_GLOBAL TU* u = a.src >= 0 ? gfield<TU>(R, a.src + comp) : gp((const TU*)a.u_raw);
    SEM_GLOBAL TU* wo = a.dst >= 0 ? gfieldw<TU>(R, a.dst + comp) : gp((TU*)a.w_raw);
    const SEM_GLOBAL TH* G = gfield<TH>(R, F_G16);
    const SEM_GLOBAL TH* Bm = gfield<TH>(R, F_B16);
    float h1, h2;
    if (a.hsel >= 0) { h1 = (float)gp(R->S)[a.hsel]; h2 = (float)gp(R->S)[a.hsel + 1]; }
    else { h1 = (float)a.h1; h2 = (float)a.h2; }
    const SEM_GLOBAL float* scl = gfield<float>(R, F_GSC);
    const float gsc = scl[ee], bsc = scl[R->E + ee];

    // D and D^T in 16 bits, block-diagonal over the pair: lane (g, m) holds
    // K indices 4g..4g+3 = (block g/2, l = 4(g%2) + q) of row/column m = (block
    // m/8, index m%8); zero off the block
    const bool on = me == gh;
    const SEM_GLOBAL float* D = gp(R->D32);
    const u2v cD = on ? pack16<TH>(D[mj * LX + 4 * gl], D[mj * LX + 4 * gl + 1], D[mj * LX + 4 * gl + 2],
                                   D[mj * LX + 4 * gl + 3])
                      : (u2v){0u, 0u};
    const u2v cDT = on ? pack16<TH>(D[(4 * gl) * LX + mj], D[(4 * gl + 1) * LX + mj], D[(4 * gl + 2) * LX + mj],
                                    D[(4 * gl + 3) * LX + mj])
                       : (u2v){0u, 0u};

    // every global load first (layout O1: tile t, register r -> i = 4 gl + r, k = 2t + gh, j = mj)
    const long long eb = (long long)ee * L3;
    const long long gb = (long long)ee * 6 * L3;
    const bool helm = h2 != 0.0f;
    // SHG as in axm_kernel
    constexpr bool shared_g = SHG != 0;
    typename Raw4<TU>::type uraw[4];
    u2v graw[4][6], braw[4];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) uraw[tt] = ld_raw(u + eb + (2 * tt + gh) * 64 + mj * 8 + 4 * gl);
#pragma unroll
    for (int tt = 0; tt < 4; ++tt)
#pragma unroll
        for (int q = 0; q < 6; ++q)
            graw[tt][q] = shared_g ? ld_raw(G + gb + q * L3 + (2 * tt + gh) * 64 + mj * 8 + 4 * gl)
                                   : ld_raw_stream(G + gb + q * L3 + (2 * tt + gh) * 64 + mj * 8 + 4 * gl);
    if (helm) {
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) braw[tt] = ld_raw(Bm + eb + (2 * tt + gh) * 64 + mj * 8 + 4 * gl);
    }
    float ur[4][4];
    float mx = 0.0f;
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        cvt4t<TU>(uraw[tt], ur[tt]);
#pragma unroll
        for (int r = 0; r < 4; ++r) mx = fmaxf(mx, fabsf(ur[tt][r]));
    }
    const float su = pow2_scale(pair_elem_max(mx));
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        const int o = (2 * tt + gh) * 64 + mj * 8 + 4 * gl;
        *(u2v*)(hU + me * AXH_ES + o) =
            pack16<TH>(ur[tt][0] * su, ur[tt][1] * su, ur[tt][2] * su, ur[tt][3] * su);
    }
    wave_lds_sync();

    // ---- reference derivatives (one MFMA per tile and direction)
    f4v dR[4], dS[4];
    const f4v z4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        // r: B = u_e[2t + g/2][j][4(g%2) + q]
        dR[tt] = mfma16x16x16<TH>(cD, lds4c(hU + me * AXH_ES + (2 * tt + gh) * 64 + mj * 8 + 4 * gl), z4);
        // s: A = u_{g/2}[2t + kk][4(g%2) + q][i]
        dS[tt] = mfma16x16x16<TH>(lds4s(hU + gh * AXH_ES + (2 * tt + me) * 64 + (4 * gl) * 8 + mj, 8), cD, z4);
        // t (k-row layout): B = u_e[4(g%2) + q][j][2t + g/2]
        const f4v aT = mfma16x16x16<TH>(cD, lds4s(hU + me * AXH_ES + (4 * gl) * 64 + mj * 8 + 2 * tt + gh, 64), z4);
#pragma unroll
        for (int r = 0; r < 4; ++r) sT[me * AXM_ES + (4 * gl + r) * 64 + mj * 8 + 2 * tt + gh] = aT[r];
    }
    wave_lds_sync();

    // ---- point-wise metric terms (fp32 on the stored, normalised 16-bit G);
    // the weighted derivatives are rounded to 16 bits for the transposed
    // contractions
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        const int o = (2 * tt + gh) * 64 + mj * 8 + 4 * gl;
        const f4v dt = *(const f4v*)(sT + me * AXM_ES + o);
        float gv[6][4];
#pragma unroll
        for (int q = 0; q < 6; ++q) Q4<TH>::unpack(graw[tt][q], gv[q]);
        float wr[4], ws[4], wt[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float x = dR[tt][r], y = dS[tt][r], z = dt[r];
            wr[r] = gv[0][r] * x + gv[1][r] * y + gv[2][r] * z;
            ws[r] = gv[1][r] * x + gv[3][r] * y + gv[4][r] * z;
            wt[r] = gv[2][r] * x + gv[4][r] * y + gv[5][r] * z;
        }
        *(u2v*)(hR + me * AXH_ES + o) = pack16<TH>(wr[0], wr[1], wr[2], wr[3]);
        *(u2v*)(hS + me * AXH_ES + o) = pack16<TH>(ws[0], ws[1], ws[2], ws[3]);
        *(u2v*)(hT + me * AXH_ES + o) = pack16<TH>(wt[0], wt[1], wt[2], wt[3]);
    }
    wave_lds_sync();

    // ---- transposed contractions: k through the k-row layout, then r and s
    f4v bT[4];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt)
        bT[tt] = mfma16x16x16<TH>(cDT, lds4s(hT + me * AXH_ES + (4 * gl) * 64 + mj * 8 + 2 * tt + gh, 64), z4);
#pragma unroll
    for (int tt = 0; tt < 4; ++tt)
#pragma unroll
        for (int r = 0; r < 4; ++r) sT[me * AXM_ES + (4 * gl + r) * 64 + mj * 8 + 2 * tt + gh] = bT[tt][r];
    f4v acc[4];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        f4v c = mfma16x16x16<TH>(cDT, lds4c(hR + me * AXH_ES + (2 * tt + gh) * 64 + mj * 8 + 4 * gl), z4);
        acc[tt] = mfma16x16x16<TH>(lds4s(hS + gh * AXH_ES + (2 * tt + me) * 64 + (4 * gl) * 8 + mj, 8), cDT, c);
    }
    wave_lds_sync();

    // ---- w = h1 gsc / s (sum of the three) + h2 B u, stored in layout O1
    const float hs = h1 * (gsc / su);
    double dot = 0.0;
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        const int o = (2 * tt + gh) * 64 + mj * 8 + 4 * gl;
        const f4v kt = *(const f4v*)(sT + me * AXM_ES + o);
        float bv[4] = {0.f, 0.f, 0.f, 0.f};
        if (helm) Q4<TH>::unpack(braw[tt], bv);
        float wv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) wv[r] = hs * (acc[tt][r] + kt[r]) + h2 * (bv[r] * bsc) * ur[tt][r];
        if (live) {
            Q4<TU>::st(wo + eb + o, wv);
            if (a.pdot >= 0) {
#pragma unroll
                for (int r = 0; r < 4; ++r) dot += (double)ur[tt][r] * (double)to<float>(to<TU>(wv[r]));
            }
        }
    }
    if (a.pdot >= 0) {
        dot = wave_sum(dot);
        if (lane == 0) red[w] = dot;
        __syncthreads();
        if (t == 0) {
            gp(R->part)[(long long)(a.pdot + comp) * R->pstride + blk] = red[0] + red[1];
            if (blk == 0) gp(R->I)[I_PCNT + a.pdot + comp] = R->nb;
        }
    }
}

bool launch_ax_mfma(const Batch& b, int lx, const AxLaunch& a, hipStream_t s)
{
    if (lx != 8 || (a.tg != P16 && a.tg != PBF && a.tg != P32) || a.precond >= 0 || a.sub >= 0 || a.out64 || a.src_vj)
        return false;
    const int ncomp = a.ncomp < 1 ? 1 : a.ncomp;
    AxLaunch q = a;
    q.ncomp = ncomp;
    dim3 grid(((b.eb[b.n] + 7) / 8) * 8 * ncomp);
    static_assert(epb_of(8) == 4, "a workgroup of two waves covers one block of four elements");
    // components of one launch share the geometric factors through L2
#define AXM_GO(KER, TU_, TG_)                                                                \
    do {                                                                                     \
        if (ncomp > 1) hipLaunchKernelGGL((KER<TU_, TG_, 1>), grid, dim3(128), 0, s, b, q); \
        else hipLaunchKernelGGL((KER<TU_, TG_, 0>), grid, dim3(128), 0, s, b, q);           \
    } while (0)
    bool ok = true;
    if (a.tc == P16 && a.tg == P16) {
        if (a.tu == P32) AXM_GO(axmh_kernel, float, __half);
        else if (a.tu == P16) AXM_GO(axmh_kernel, __half, __half);
        else ok = false;
    } else if (a.tc == PBF && a.tg == PBF) {
        if (a.tu == P32) AXM_GO(axmh_kernel, float, __hip_bfloat16);
        else if (a.tu == PBF) AXM_GO(axmh_kernel, __hip_bfloat16, __hip_bfloat16);
        else ok = false;
    } else if (a.tc != P32) {
        ok = false;
    } else if (a.tg == P32) {
        if (a.tu == P32) AXM_GO(axm_kernel, float, float);
        else ok = false;
    } else if (a.tu == P32 && a.tg == P16) AXM_GO(axm_kernel, float, __half);
    else if (a.tu == P32 && a.tg == PBF) AXM_GO(axm_kernel, float, __hip_bfloat16);
    else if (a.tu == P16 && a.tg == P16) AXM_GO(axm_kernel, __half, __half);
    else if (a.tu == PBF && a.tg == PBF) AXM_GO(axm_kernel, __hip_bfloat16, __hip_bfloat16);
    else ok = false;
#undef AXM_GO
    return ok;
}

}  // namespace semk
