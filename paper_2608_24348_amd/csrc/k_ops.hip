// SEM operators on the element columns (same k-walk as the Helmholtz kernel):
//   convection   bn_i = -sum_c u_c sum_a M_ac D_a u_i   (= -B (u.grad) u_i)
//   opgrad       g_c  = sum_a M_ac D_a p               (= B grad p)
//   weak div     d    = sum_a D_a^T (sum_c M_ac v_c)   (= int grad(test) . v)
//   diagnostics  kinetic energy, enstrophy (element-local curl), max |div u|
// with M_ac = B dr_a/dx_c.  Inputs and outputs are fp64 fields; the metric
// terms M are read in the kernel's storage precision TM and the arithmetic
// runs in C.
#include "k_common.h"

namespace semk {

template <int LX> struct OEpb {
    static constexpr int v = epb_of(LX);
};
template <int LX> struct ONthr {
    static constexpr int v = (LX * LX * OEpb<LX>::v + 63) / 64 * 64;
};
// one element per wave at lx = 8: the k-loops' LDS layers are wave-private
template <int LX> struct OWave {
    static constexpr bool v = LX * LX == 64 && ONthr<LX>::v == OEpb<LX>::v * 64;
};

template <typename TM> __device__ __forceinline__ int mfield() { return F_M16; }
template <> __device__ __forceinline__ int mfield<double>() { return F_M64; }
template <> __device__ __forceinline__ int mfield<float>() { return F_M32; }

template <typename TM, typename C>
__device__ __forceinline__ C ldm(const SEM_GLOBAL TM* M, long long off, C sc)
{
    if constexpr (sizeof(TM) == 2) return to<C>(ldg_stream(M + off)) * sc;
    else return (C)ldg_stream(M + off);
}

template <typename TM, typename C>
__device__ __forceinline__ C melem_scale(const ReqDesc* R, int e)
{
    if constexpr (sizeof(TM) == 2) return (C)gfield<float>(R, F_MSC)[e];
    else return (C)1;
}

#define OPS_PROLOGUE(LX)                                  \
    constexpr int EPB = OEpb<LX>::v;                      \
    constexpr int L2 = LX * LX;                           \
    constexpr int L3 = LX * LX * LX;                      \
    const int g = blockIdx.x;                             \
    const int ri = find_req(bt.eb, bt.n, g);              \
    const ReqDesc* R = bt.r[ri];                          \
    if (!gate_ok(R, bt.gate)) return;                     \
    const int blk = g - bt.eb[ri];                        \
    const int t = threadIdx.x;                            \
    const int el = t / L2;                                \
    const int ij = t - el * L2;                           \
    const int i = ij % LX, j = ij / LX;                   \
    const int e = blk * EPB + el;                         \
    const bool live = el < EPB && e < R->E;               \
    const int ee = live ? e : 0;                          \
    const long long ebase = (long long)ee * L3;           \
    (void)j;

template <int LX, typename C>
__device__ __forceinline__ void load_D(const ReqDesc* R, C* sD)
{
    for (int q = threadIdx.x; q < LX * LX; q += blockDim.x) {
        if constexpr (sizeof(C) == 8) sD[q] = (C)gp(R->D64)[q];
        else sD[q] = (C)gp(R->D32)[q];
    }
}

template <int LX, typename TM, typename C>
__global__ void __launch_bounds__(ONthr<LX>::v) conv_kernel(Batch bt)
{
    OPS_PROLOGUE(LX)
    __shared__ C sD[L2];
    __shared__ C su[3][EPB][L2];
    load_D<LX, C>(R, sD);
    const SEM_GLOBAL TM* M = gfield<TM>(R, mfield<TM>());
    const C msc = melem_scale<TM, C>(R, ee);
    C col[3][LX];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const SEM_GLOBAL double* u = gfield<double>(R, F_U + c);
#pragma unroll
        for (int k = 0; k < LX; ++k) col[c][k] = (C)u[ebase + k * L2 + ij];
    }
    block_sync_lds();
#pragma unroll
    for (int k = 0; k < LX; ++k) {
        if (el < EPB) {
#pragma unroll
            for (int c = 0; c < 3; ++c) su[c][el][ij] = col[c][k];
        }
        lds_handoff<OWave<LX>::v>();
        if (live) {
            const int p = k * L2 + ij;
            C m[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) m[q] = ldm<TM, C>(M, ((long long)ee * 9 + q) * L3 + p, msc);
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                C dr = 0, ds = 0, dt = 0;
#pragma unroll
                for (int l = 0; l < LX; ++l) {
                    dr += sD[i * LX + l] * su[f][el][j * LX + l];
                    ds += sD[j * LX + l] * su[f][el][l * LX + i];
                    dt += sD[k * LX + l] * col[f][l];
                }
                C s = 0;
#pragma unroll
                for (int c = 0; c < 3; ++c) s += col[c][k] * (m[0 * 3 + c] * dr + m[1 * 3 + c] * ds + m[2 * 3 + c] * dt);
                gfieldw<double>(R, F_BN + f)[ebase + p] = -(double)s;
            }
        }
        lds_handoff<OWave<LX>::v>();
    }
}

// RHS: the step head's form.  Instead of storing grad p it forms the local
// velocity rhs of the BDF/EXT step point by point,
//   rhs_c = sum_q a_q BN_c^{n-q} + (B / dt) sum_q b_q u_c^{n-q} - (grad p)_c,
// so grad p is never written and read back (48 bytes per point)
template <int LX, typename TM, typename C, bool RHS = false>
__global__ void __launch_bounds__(ONthr<LX>::v) opgrad_kernel(Batch bt, int src, int dst)
{
    OPS_PROLOGUE(LX)
    __shared__ C sD[L2];
    __shared__ C su[EPB][L2];
    load_D<LX, C>(R, sD);
    const SEM_GLOBAL TM* M = gfield<TM>(R, mfield<TM>());
    const C msc = melem_scale<TM, C>(R, ee);
    const SEM_GLOBAL double* u = gfield<double>(R, src);
    double a1 = 0, a2 = 0, a3 = 0, b1 = 0, b2 = 0, b3 = 0, idt = 0;
    if constexpr (RHS) {
        const SEM_GLOBAL double* S = gp(R->S);
        a1 = S[S_EXT]; a2 = S[S_EXT + 1]; a3 = S[S_EXT + 2];
        b1 = S[S_BDF]; b2 = S[S_BDF + 1]; b3 = S[S_BDF + 2];
        idt = 1.0 / S[S_DT];
    }
    C col[LX];
#pragma unroll
    for (int k = 0; k < LX; ++k) col[k] = (C)u[ebase + k * L2 + ij];
    block_sync_lds();
#pragma unroll
    for (int k = 0; k < LX; ++k) {
        const int p = k * L2 + ij;
        // the rhs inputs of this layer are loaded ahead of the contraction
        double bv = 0, hv[3] = {0, 0, 0}, ev[3] = {0, 0, 0};
        if constexpr (RHS) {
            bv = gfield<double>(R, F_B64)[ebase + p];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                ev[c] = a1 * gfield<double>(R, F_BN + c)[ebase + p] + a2 * ldg_stream(gfield<double>(R, F_BNL1 + c) + ebase + p) +
                        a3 * ldg_stream(gfield<double>(R, F_BNL2 + c) + ebase + p);
                hv[c] = b1 * gfield<double>(R, F_U + c)[ebase + p] + b2 * ldg_stream(gfield<double>(R, F_UL1 + c) + ebase + p) +
                        b3 * ldg_stream(gfield<double>(R, F_UL2 + c) + ebase + p);
            }
        }
        if (el < EPB) su[el][ij] = col[k];
        lds_handoff<OWave<LX>::v>();
        if (live) {
            C dr = 0, ds = 0, dt = 0;
#pragma unroll
            for (int l = 0; l < LX; ++l) {
                dr += sD[i * LX + l] * su[el][j * LX + l];
                ds += sD[j * LX + l] * su[el][l * LX + i];
                dt += sD[k * LX + l] * col[l];
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                C gc = ldm<TM, C>(M, ((long long)ee * 9 + 0 * 3 + c) * L3 + p, msc) * dr
                     + ldm<TM, C>(M, ((long long)ee * 9 + 1 * 3 + c) * L3 + p, msc) * ds
                     + ldm<TM, C>(M, ((long long)ee * 9 + 2 * 3 + c) * L3 + p, msc) * dt;
                if constexpr (RHS) gfieldw<double>(R, F_RHS + c)[ebase + p] = ev[c] + (bv * idt) * hv[c] - (double)gc;
                else gfieldw<double>(R, dst + c)[ebase + p] = (double)gc;
            }
        }
        lds_handoff<OWave<LX>::v>();
    }
}

template <int LX, typename TM, typename C>
__global__ void __launch_bounds__(ONthr<LX>::v) wdiv_kernel(Batch bt, int src, int dst)
{
    OPS_PROLOGUE(LX)
    __shared__ C sD[L2];
    __shared__ C sr[EPB][L2];
    __shared__ C ss[EPB][L2];
    load_D<LX, C>(R, sD);
    const SEM_GLOBAL TM* M = gfield<TM>(R, mfield<TM>());
    const C msc = melem_scale<TM, C>(R, ee);
    C wacc[LX];
#pragma unroll
    for (int k = 0; k < LX; ++k) wacc[k] = 0;
    block_sync_lds();
#pragma unroll
    for (int k = 0; k < LX; ++k) {
        const int p = k * L2 + ij;
        C f[3] = {0, 0, 0};
        if (live) {
            C v[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) v[c] = (C)gfield<double>(R, src + c)[ebase + p];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) f[a] += ldm<TM, C>(M, ((long long)ee * 9 + a * 3 + c) * L3 + p, msc) * v[c];
        }
        if (el < EPB) { sr[el][ij] = f[0]; ss[el][ij] = f[1]; }
#pragma unroll
        for (int l = 0; l < LX; ++l) wacc[l] += sD[k * LX + l] * f[2];
        lds_handoff<OWave<LX>::v>();
        if (el < EPB) {
            C acc = 0;
#pragma unroll
            for (int l = 0; l < LX; ++l) {
                acc += sD[l * LX + i] * sr[el][j * LX + l];
                acc += sD[l * LX + j] * ss[el][l * LX + i];
            }
            wacc[k] += acc;
        }
        lds_handoff<OWave<LX>::v>();
    }
    if (live) {
        SEM_GLOBAL double* out = gfieldw<double>(R, dst);
#pragma unroll
        for (int k = 0; k < LX; ++k) out[ebase + k * L2 + ij] = (double)wacc[k];
    }
}

// (element kernels: the column loads are unconditional -- threads without an
// element read element 0 -- and the k-walk uses LDS-only barriers)

// kinetic energy and enstrophy integrands (B/2 |u|^2, B/2 |omega|^2) and the
// largest |div u|, element-local derivatives, fp64; partials R_X0, R_X1 (sum)
// and R_X2 (max)
template <int LX>
__global__ void __launch_bounds__(ONthr<LX>::v) diagnostics_kernel(Batch bt)
{
    OPS_PROLOGUE(LX)
    __shared__ double sD[L2];
    __shared__ double su[3][EPB][L2];
    __shared__ double red[ONthr<LX>::v / 64 * 2];
    load_D<LX, double>(R, sD);
    const SEM_GLOBAL double* M = gfield<double>(R, F_M64);
    const SEM_GLOBAL double* B = gfield<double>(R, F_B64);
    // 1 / (GLL spacing around each index): half the distance between the two
    // neighbours inside, the distance to the one neighbour at an end
    __shared__ double sidr[LX];
    if (t < LX) {
        const SEM_GLOBAL double* xi = gp(R->D64) + LX * LX + LX;
        const double d = t == 0 ? xi[1] - xi[0] : t == LX - 1 ? xi[LX - 1] - xi[LX - 2] : 0.5 * (xi[t + 1] - xi[t - 1]);
        sidr[t] = 1.0 / d;
    }
    double col[3][LX];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const SEM_GLOBAL double* u = gfield<double>(R, F_U + c);
#pragma unroll
        for (int k = 0; k < LX; ++k) col[c][k] = u[ebase + k * L2 + ij];
    }
    double ke = 0, en = 0, md = 0, cr = 0;
    block_sync_lds();
#pragma unroll
    for (int k = 0; k < LX; ++k) {
        if (el < EPB) {
#pragma unroll
            for (int c = 0; c < 3; ++c) su[c][el][ij] = col[c][k];
        }
        lds_handoff<OWave<LX>::v>();
        if (live) {
            const int p = k * L2 + ij;
            const double bm = B[ebase + p];
            double m[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) m[q] = ldg_stream(M + ((long long)ee * 9 + q) * L3 + p);
            double gr[3][3];  // gr[f][c] = d u_f / d x_c
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                double dr = 0, ds = 0, dt = 0;
#pragma unroll
                for (int l = 0; l < LX; ++l) {
                    dr += sD[i * LX + l] * su[f][el][j * LX + l];
                    ds += sD[j * LX + l] * su[f][el][l * LX + i];
                    dt += sD[k * LX + l] * col[f][l];
                }
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    gr[f][c] = (m[0 * 3 + c] * dr + m[1 * 3 + c] * ds + m[2 * 3 + c] * dt) / bm;
            }
            const double wx = gr[2][1] - gr[1][2];
            const double wy = gr[0][2] - gr[2][0];
            const double wz = gr[1][0] - gr[0][1];
            const double dv = gr[0][0] + gr[1][1] + gr[2][2];
            ke += bm * 0.5 * (col[0][k] * col[0][k] + col[1][k] * col[1][k] + col[2][k] * col[2][k]);
            en += bm * 0.5 * (wx * wx + wy * wy + wz * wz);
            md = fmax(md, fabs(dv));
            // advective CFL rate: sum_a |u . grad r_a| / dr_a, grad r_a = M_a. / B
            const int ia[3] = {i, j, k};
            double rate = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double ua = (col[0][k] * m[a * 3 + 0] + col[1][k] * m[a * 3 + 1] + col[2][k] * m[a * 3 + 2]) / bm;
                rate += fabs(ua) * sidr[ia[a]];
            }
            cr = fmax(cr, rate);
        }
        lds_handoff<OWave<LX>::v>();
    }
    double v[2] = {ke, en};
    block_sum<double, 2>(v, red);
    md = wave_max(md);
    cr = wave_max(cr);
    __shared__ double mred[ONthr<LX>::v / 64][2];
    if ((t & 63) == 0) { mred[t >> 6][0] = md; mred[t >> 6][1] = cr; }
    block_sync_lds();
    if (t == 0) {
        double m = 0, c = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { m = fmax(m, mred[w][0]); c = fmax(c, mred[w][1]); }
        SEM_GLOBAL double* part = gp(R->part);
        part[(long long)R_X0 * R->pstride + blk] = v[0];
        part[(long long)R_X1 * R->pstride + blk] = v[1];
        part[(long long)R_X2 * R->pstride + blk] = m;
        part[(long long)R_X4 * R->pstride + blk] = c;
        if (blk == 0) {
            gp(R->I)[I_PCNT + R_X0] = R->nb; gp(R->I)[I_PCNT + R_X1] = R->nb; gp(R->I)[I_PCNT + R_X2] = R->nb;
            gp(R->I)[I_PCNT + R_X4] = R->nb;
        }
    }
}

#define OPS_LX_SWITCH(lx, CALL) \
    switch (lx) { \
    case 3: CALL(3); break; case 4: CALL(4); break; case 5: CALL(5); break; case 6: CALL(6); break; \
    case 7: CALL(7); break; case 8: CALL(8); break; case 9: CALL(9); break; case 10: CALL(10); break; \
    case 11: CALL(11); break; case 12: CALL(12); break; default: break; }

// supported (metric storage, arithmetic) pairs: (fp64, fp64), (fp32, fp32),
// (fp16, fp32), (bf16, fp32) and (fp32, fp64)
#define OPS_DISPATCH(KERNEL, L, grid, blk, s, ...)                                                                  \
    if (tm == P64) hipLaunchKernelGGL((KERNEL<L, double, double>), grid, blk, 0, s, __VA_ARGS__);                 \
    else if (tm == P32 && tc == P64) hipLaunchKernelGGL((KERNEL<L, float, double>), grid, blk, 0, s, __VA_ARGS__);\
    else if (tm == P32) hipLaunchKernelGGL((KERNEL<L, float, float>), grid, blk, 0, s, __VA_ARGS__);              \
    else if (tm == P16) hipLaunchKernelGGL((KERNEL<L, __half, float>), grid, blk, 0, s, __VA_ARGS__);             \
    else hipLaunchKernelGGL((KERNEL<L, __hip_bfloat16, float>), grid, blk, 0, s, __VA_ARGS__);

void launch_conv(const Batch& b, int lx, int tm, int tc, hipStream_t s)
{
    dim3 grid(b.eb[b.n]);
#define GO(L) OPS_DISPATCH(conv_kernel, L, grid, dim3(ONthr<L>::v), s, b)
    OPS_LX_SWITCH(lx, GO)
#undef GO
}

void launch_opgrad(const Batch& b, int lx, int tm, int tc, int src, int dst, hipStream_t s)
{
    dim3 grid(b.eb[b.n]);
#define GO(L) OPS_DISPATCH(opgrad_kernel, L, grid, dim3(ONthr<L>::v), s, b, src, dst)
    OPS_LX_SWITCH(lx, GO)
#undef GO
}

void launch_opgrad_rhs(const Batch& b, int lx, int tm, int tc, int src, hipStream_t s)
{
    dim3 grid(b.eb[b.n]);
#define GO(L)                                                                                                          \
    if (tm == P64) hipLaunchKernelGGL((opgrad_kernel<L, double, double, true>), grid, dim3(ONthr<L>::v), 0, s, b, src, -1); \
    else if (tm == P32 && tc == P64)                                                                                   \
        hipLaunchKernelGGL((opgrad_kernel<L, float, double, true>), grid, dim3(ONthr<L>::v), 0, s, b, src, -1);       \
    else if (tm == P32) hipLaunchKernelGGL((opgrad_kernel<L, float, float, true>), grid, dim3(ONthr<L>::v), 0, s, b, src, -1); \
    else if (tm == P16) hipLaunchKernelGGL((opgrad_kernel<L, __half, float, true>), grid, dim3(ONthr<L>::v), 0, s, b, src, -1); \
    else hipLaunchKernelGGL((opgrad_kernel<L, __hip_bfloat16, float, true>), grid, dim3(ONthr<L>::v), 0, s, b, src, -1);
    OPS_LX_SWITCH(lx, GO)
#undef GO
}

void launch_wdiv(const Batch& b, int lx, int tm, int tc, int src, int dst, hipStream_t s)
{
    dim3 grid(b.eb[b.n]);
#define GO(L) OPS_DISPATCH(wdiv_kernel, L, grid, dim3(ONthr<L>::v), s, b, src, dst)
    OPS_LX_SWITCH(lx, GO)
#undef GO
}

void launch_diagnostics(const Batch& b, int lx, hipStream_t s)
{
    dim3 grid(b.eb[b.n]);
#define GO(L) hipLaunchKernelGGL(diagnostics_kernel<L>, grid, dim3(ONthr<L>::v), 0, s, b)
    OPS_LX_SWITCH(lx, GO)
#undef GO
}

}  // namespace semk
