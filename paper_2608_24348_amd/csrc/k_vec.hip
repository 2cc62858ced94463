// Point-wise Krylov and time-step kernels with fused partial reductions, and
// the one-workgroup-per-request "finalise" kernels that add the partials in a
// fixed order (fp64 global stage) and run the scalar logic of PCG, GMRES and
// the BDF/EXT step on the device.  Inner products of assembled vectors weight
// each local point by 1/multiplicity, i.e. they run over unique nodes.
#include "k_common.h"
#include "k_fin.h"

namespace semk {

struct PtRange {
    long long p0, p1, L3;
};

// points of point-wise block blk (vepb whole elements)
__device__ __forceinline__ PtRange pt_range(const ReqDesc* R, int blk)
{
    PtRange r;
    r.L3 = (long long)R->lx * R->lx * R->lx;
    r.p0 = (long long)blk * R->vepb * r.L3;
    long long e1 = (long long)(blk + 1) * R->vepb;
    if (e1 > R->E) e1 = R->E;
    r.p1 = e1 * r.L3;
    return r;
}

template <typename T> __device__ __forceinline__ const SEM_GLOBAL T* fld(const ReqDesc* R, int id) { return gfield<T>(R, id); }
template <typename T> __device__ __forceinline__ SEM_GLOBAL T* fldw(const ReqDesc* R, int id) { return gfieldw<T>(R, id); }

template <typename TV> __device__ __forceinline__ int idv_field() { return F_IDV32; }
template <> __device__ __forceinline__ int idv_field<double>() { return F_IDV64; }
template <typename TV> __device__ __forceinline__ int idp_field() { return F_IDP32; }
template <> __device__ __forceinline__ int idp_field<double>() { return F_IDP64; }

// 1/multiplicity of the points a thread visits in a point-wise loop
// (p = p0 + threadIdx.x, p += blockDim.x over whole elements): the local
// index q advances by blockDim.x mod lx^3 with one wrap, and the weight comes
// from the per-request table after D, weights and nodes.
struct MulWalk {
    const SEM_GLOBAL double* tab;
    int q, step, L3;
    __device__ __forceinline__ MulWalk(const ReqDesc* R, const PtRange& pr)
    {
        L3 = (int)pr.L3;
        tab = gp(R->D64) + R->lx * R->lx + 2 * R->lx;
        q = (int)threadIdx.x % L3;
        step = (int)blockDim.x % L3;
    }
    __device__ __forceinline__ double im() const { return tab[q]; }
    __device__ __forceinline__ void next()
    {
        q += step;
        if (q >= L3) q -= L3;
    }
};

// partial of point-wise block blk; block 0 also records how many partials the slot holds
__device__ __forceinline__ void put_partial(const ReqDesc* R, int slot, int blk, double v)
{
    gp(R->part)[(long long)slot * R->pstride + blk] = v;
    if (blk == 0) gp(R->I)[I_PCNT + slot] = R->nvb;
}

// ------------------------------------------------------------------ generic point-wise ops
// one instantiation per operation (OP == a.op): each kernel holds only its
// own loop, and profiles name the operation
template <typename TV, typename A, int OP>
__global__ void __launch_bounds__(SEM_VEC_THREADS) vec_kernel(Batch bt, VecArgs a)
{
    __shared__ double red[(SEM_VEC_THREADS / 64) * 2];
    const int g = blockIdx.x;
    const int ri = find_req(bt.vb, bt.n, g);
    const ReqDesc* R = bt.r[ri];
    const int blk = g - bt.vb[ri];
    const int c = blockIdx.y;
    if (!gate_ok(R, a.gate < 0 ? -1 : a.gate + (a.ncomp > 1 ? c : 0))) return;
    const PtRange pr = pt_range(R, blk);
    const SEM_GLOBAL double* S = gp(R->S);
    double acc[2] = {0.0, 0.0};

    switch (OP) {
    case V_PCG_INIT: {
        auto r64 = fld<double>(R, F_R64 + c);
        auto idv = fld<TV>(R, idv_field<TV>());
        auto x = fldw<TV>(R, F_PX + c);
        auto r = fldw<TV>(R, F_PR + c);
        auto z = fldw<TV>(R, F_PZ + c);
        auto pp = fldw<TV>(R, F_PP + c);
        A s = 0;
        MulWalk mw(R, pr);
        for (long long p = pr.p0 + threadIdx.x; p < pr.p1; p += blockDim.x, mw.next()) {
            const TV rv = (TV)r64[p];
            const TV zv = rv * idv[p];
            x[p] = (TV)0; r[p] = rv; z[p] = zv; pp[p] = zv;
            s += (A)(rv * zv) * (A)mw.im();
        }
        double v2[1] = {(double)s};
        block_sum<double, 1>(v2, red);
        if (threadIdx.x == 0) put_partial(R, R_B + c, blk, v2[0]);
        break;
    }
    case V_PCG_UPD: {
        const TV alpha = (TV)S[S_ALPHA + c];
        auto idv = fld<TV>(R, idv_field<TV>());
        auto x = fldw<TV>(R, F_PX + c);
        auto r = fldw<TV>(R, F_PR + c);
        auto z = fldw<TV>(R, F_PZ + c);
        auto pp = fld<TV>(R, F_PP + c);
        auto w = fld<TV>(R, F_PW + c);
        A rr = 0, rz = 0;
        MulWalk mw(R, pr);
        // four of the thread's points per pass, every load before the first
        // store (the stores could alias the loads in the compiler's view,
        // which would serialise the points); same per-thread order of the sums
        constexpr int U = 4;
        const long long st = blockDim.x;
        long long p = pr.p0 + threadIdx.x;
        for (; p + (U - 1) * st < pr.p1; p += U * st) {
            TV xv[U], pv[U], r0[U], wv[U], dv[U];
            A im[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const long long q = p + u * st;
                xv[u] = x[q]; pv[u] = pp[q]; r0[u] = r[q]; wv[u] = w[q]; dv[u] = idv[q];
                im[u] = (A)mw.im();
                mw.next();
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const long long q = p + u * st;
                x[q] = xv[u] + alpha * pv[u];
                const TV rv = r0[u] - alpha * wv[u];
                const TV zv = rv * dv[u];
                r[q] = rv; z[q] = zv;
                rr += (A)(rv * rv) * im[u];
                rz += (A)(rv * zv) * im[u];
            }
        }
        for (; p < pr.p1; p += st, mw.next()) {
            x[p] += alpha * pp[p];
            const TV rv = r[p] - alpha * w[p];
            const TV zv = rv * idv[p];
            r[p] = rv; z[p] = zv;
            const A im = (A)mw.im();
            rr += (A)(rv * rv) * im;
            rz += (A)(rv * zv) * im;
        }
        double v2[2] = {(double)rr, (double)rz};
        block_sum<double, 2>(v2, red);
        if (threadIdx.x == 0) { put_partial(R, R_B + c, blk, v2[0]); put_partial(R, R_C + c, blk, v2[1]); }
        break;
    }
    case V_PCG_P: {
        const TV beta = (TV)S[S_BETA + c];
        auto z = fld<TV>(R, F_PZ + c);
        auto pp = fldw<TV>(R, F_PP + c);
        for (long long p = pr.p0 + threadIdx.x; p < pr.p1; p += blockDim.x) pp[p] = z[p] + beta * pp[p];
        break;
    }
    case V_US_COPY: {
        auto u = fld<double>(R, F_U + c);
        auto us = fldw<double>(R, F_US + c);
        for (long long p = pr.p0 + threadIdx.x; p < pr.p1; p += blockDim.x) us[p] = u[p];
        break;
    }
    case V_US_ADD: {
        auto x = fld<TV>(R, F_PX + c);
        auto us = fldw<double>(R, F_US + c);
        // four of the thread's points per pass, every load before the first store
        constexpr int U = 4;
        const long long st = blockDim.x;
        const SEM_GLOBAL double* base = a.f0 == 1 ? fld<double>(R, F_U + c) : us;
        long long p = pr.p0 + threadIdx.x;
        for (; p + (U - 1) * st < pr.p1; p += U * st) {
            double bv[U];
            TV xv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) { bv[u] = base[p + u * st]; xv[u] = x[p + u * st]; }
#pragma unroll
            for (int u = 0; u < U; ++u) us[p + u * st] = bv[u] + (double)xv[u];
        }
        for (; p < pr.p1; p += st) us[p] = base[p] + (double)x[p];
        break;
    }
    case V_IDV: {
        const double h1 = S[S_H1], h2 = S[S_H2];
        auto da = fld<double>(R, F_DA64);
        auto ib = fld<double>(R, F_IBSUM64);
        auto idv = fldw<double>(R, F_IDV64);
        auto idv32 = fldw<float>(R, F_IDV32);
        for (long long p = pr.p0 + threadIdx.x; p < pr.p1; p += blockDim.x) {
            const double v = 1.0 / (h1 * da[p] + h2 / ib[p]);
            idv[p] = v;
            if (idv32) idv32[p] = (float)v;
        }
        break;
    }
    case V_SUM_UNIQUE:
    case V_SUM_MASS: {
        const SEM_GLOBAL double* f = a.f0 >= 0 ? fld<double>(R, a.f0) : nullptr;
        auto B = fld<double>(R, F_B64);
        MulWalk mw(R, pr);
        for (long long p = pr.p0 + threadIdx.x; p < pr.p1; p += blockDim.x, mw.next()) {
            const double fv = f ? f[p] : 1.0;
            if (OP == V_SUM_UNIQUE) acc[0] += fv * mw.im();
            else acc[0] += fv * B[p];
        }
        double v2[1] = {acc[0]};
        block_sum<double, 1>(v2, red);
        if (threadIdx.x == 0) put_partial(R, R_X3, blk, v2[0]);
        break;
    }
    case V_SUB_MEAN: {
        auto f = fldw<double>(R, a.f0);
        const double m = S[S_MEAN];
        const double sc = a.f1 >= 0 ? S[a.f1] : 1.0;
        for (long long p = pr.p0 + threadIdx.x; p < pr.p1; p += blockDim.x) f[p] = sc * (f[p] - m);
        break;
    }
    case V_COPY: {
        auto f = fld<double>(R, a.f0 + c);
        auto o = fldw<double>(R, a.f1 + c);
        for (long long p = pr.p0 + threadIdx.x; p < pr.p1; p += blockDim.x) o[p] = f[p];
        break;
    }
    case V_ZERO: {
        auto f = fldw<double>(R, a.f0 + c);
        for (long long p = pr.p0 + threadIdx.x; p < pr.p1; p += blockDim.x) f[p] = 0.0;
        break;
    }
    case V_GM_RESID: {
        // r = b - A x (fp64), stored as the next cycle's first basis vector
        // V_0 (unnormalised; FIN_GM_RESTART records 1/|r|)
        auto b = fld<double>(R, F_GB);
        auto w = fld<double>(R, F_GWD);
        const bool ax = gp(R->I)[I_GENDAX] != 0;  // iterate nonzero: GWD holds A x
        SEM_GLOBAL double* v64 = a.tb == P64 ? fldw<double>(R, F_V) : nullptr;
        SEM_GLOBAL float* v32 = a.tb == P64 ? nullptr : fldw<float>(R, F_V);
        MulWalk mw(R, pr);
        for (long long p = pr.p0 + threadIdx.x; p < pr.p1; p += blockDim.x, mw.next()) {
            const double v = ax ? b[p] - w[p] : b[p];
            if (v64) v64[p] = v;
            else v32[p] = (float)v;
            acc[0] += v * v * mw.im();
        }
        double v2[1] = {acc[0]};
        block_sum<double, 1>(v2, red);
        if (threadIdx.x == 0) put_partial(R, R_GN, blk, v2[0]);
        break;
    }
    case V_CORRECT: {
        // all three components per point, and p += phi
        const SEM_GLOBAL double *us[3], *gpr[3];
        SEM_GLOBAL double* un[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            us[q] = fld<double>(R, F_US + q);
            gpr[q] = fld<double>(R, F_GP + q);
            un[q] = fldw<double>(R, F_UL2 + q);
        }
        auto ib = fld<double>(R, F_IBSUM64);
        auto pres = fldw<double>(R, F_P);
        auto phi = fld<double>(R, F_GX);
        const double f = S[S_DT] / S[S_BETA0];
        // four of the thread's points per pass, every load before the first store
        constexpr int U = 4;
        const long long st = blockDim.x;
        long long p = pr.p0 + threadIdx.x;
        for (; p + (U - 1) * st < pr.p1; p += U * st) {
            double ibv[U], uv[U][3], gv[U][3], pv[U], fv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const long long x = p + u * st;
                ibv[u] = ib[x]; pv[u] = pres[x]; fv[u] = phi[x];
#pragma unroll
                for (int q = 0; q < 3; ++q) { uv[u][q] = us[q][x]; gv[u][q] = gpr[q][x]; }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const long long x = p + u * st;
#pragma unroll
                for (int q = 0; q < 3; ++q) un[q][x] = uv[u][q] - f * gv[u][q] * ibv[u];
                pres[x] = pv[u] + fv[u];
            }
        }
        for (; p < pr.p1; p += st) {
            const double ibp = ib[p];
#pragma unroll
            for (int q = 0; q < 3; ++q) un[q][p] = us[q][p] - f * gpr[q][p] * ibp;
            pres[p] += phi[p];
        }
        break;
    }
    case V_MASS_RAW: {
        const SEM_GLOBAL double* x = gp((const double*)a.x_raw);
        SEM_GLOBAL double* y = gp((double*)a.y_raw);
        auto B = fld<double>(R, F_B64);
        for (long long p = pr.p0 + threadIdx.x; p < pr.p1; p += blockDim.x) y[p] = B[p] * x[p];
        break;
    }
    case V_PR_V: {
        // the candidate direction: the correction the solver added to the
        // projected guess, or the whole solution when the space restarts
        auto gx = fld<double>(R, F_GX);
        auto xb = fld<double>(R, F_PRXB);
        auto v = fldw<double>(R, F_GW);
        if (gp(R->I)[I_PRFULL]) {
            for (long long p = pr.p0 + threadIdx.x; p < pr.p1; p += blockDim.x) v[p] = gx[p];
        } else {
            for (long long p = pr.p0 + threadIdx.x; p < pr.p1; p += blockDim.x) v[p] = gx[p] - xb[p];
        }
        break;
    }
    case V_AXPY_RAW: {
        const double* x = (const double*)a.x_raw;
        double* y = (double*)a.y_raw;
        for (long long p = pr.p0 + threadIdx.x; p < pr.p1; p += blockDim.x) y[p] += a.a * x[p];
        break;
    }
    default: break;
    }
}

// ------------------------------------------------------------------ GMRES orthogonalisation passes
// One pass over the points of a block touches every basis vector V_0..V_J
// once.  The body is instantiated for every basis size NJ = J+1 (J is read on
// the device and dispatched with a uniform switch), so each point issues its
// NJ independent loads back to back before any arithmetic consumes them.
// The periodic Poisson operator is singular with constant null vectors and a
// range orthogonal to them, so the first pass also sums the operator output
// over unique nodes and the second subtracts that mean: a no-op in exact
// arithmetic that keeps rounding (notably of fp32 operators) from feeding the
// null direction into the basis.
template <int NJ, int MODE, typename TB>
__device__ __forceinline__ void gm_body(const ReqDesc* R, const PtRange& pr, double (&acc)[SEM_MAXM + 1], double& accm)
{
    const SEM_GLOBAL TB* V = fld<TB>(R, F_V);
    const long long np = R->np;
    double h[NJ];
#pragma unroll
    for (int i = 0; i < NJ; ++i)
        h[i] = (MODE == 1 ? gp(R->S)[S_GHC + i] : MODE == 2 ? gp(R->S)[S_GH2 + i] : 0.0) * gp(R->S)[S_GVS + i];
    const double mean = MODE == 1 ? gp(R->S)[S_GMEAN] : 0.0;
    auto w = fld<double>(R, F_GW);
    auto wd = fldw<double>(R, F_GWD);
    // the last pass stores the orthogonalised vector as V_{J+1}, unnormalised
    SEM_GLOBAL TB* vn = fldw<TB>(R, F_V) + (long long)NJ * np;
    MulWalk mw(R, pr);
    // one point: every load of the point was issued before (vr, ws)
    auto point = [&](long long p, const double (&vr)[NJ], double ws, double im) {
        if (MODE == 0) {
            const double wv = ws * im;
            accm += wv;
#pragma unroll
            for (int i = 0; i < NJ; ++i) acc[i] += vr[i] * wv;
        } else if (MODE == 1) {
            double wv = ws - mean;
#pragma unroll
            for (int i = 0; i < NJ; ++i) wv -= h[i] * vr[i];
            wd[p] = wv;
            wv *= im;
#pragma unroll
            for (int i = 0; i < NJ; ++i) acc[i] += vr[i] * wv;
        } else {
            double wv = ws;
#pragma unroll
            for (int i = 0; i < NJ; ++i) wv -= h[i] * vr[i];
            vn[p] = (TB)wv;
            acc[0] += wv * wv * im;
        }
    };
    const SEM_GLOBAL double* win = MODE == 2 ? (const SEM_GLOBAL double*)wd : w;
    long long p = pr.p0 + threadIdx.x;
    const long long bd = blockDim.x;
#ifndef SEM_GM_PAIR_MAX
#define SEM_GM_PAIR_MAX 12
#endif
    if constexpr (NJ <= SEM_GM_PAIR_MAX) {
        // two points per iteration (p, p + blockDim): twice the loads in
        // flight; the accumulation order (p before p + blockDim) is unchanged
        for (; p + bd < pr.p1; p += 2 * bd) {
            double va[NJ], vb[NJ];
#pragma unroll
            for (int i = 0; i < NJ; ++i) { va[i] = (double)V[i * np + p]; vb[i] = (double)V[i * np + p + bd]; }
            const double wa = win[p], wb = win[p + bd];
            const double ia = mw.im();
            mw.next();
            const double ib = mw.im();
            mw.next();
            point(p, va, wa, ia);
            point(p + bd, vb, wb, ib);
        }
    }
    for (; p < pr.p1; p += bd, mw.next()) {
        double vr[NJ];
#pragma unroll
        for (int i = 0; i < NJ; ++i) vr[i] = (double)V[i * np + p];
        point(p, vr, win[p], mw.im());
    }
}

#define SEM_NJ_CASES(F)                                                                                 \
    F(1) F(2) F(3) F(4) F(5) F(6) F(7) F(8) F(9) F(10) F(11) F(12) F(13) F(14) F(15) F(16) F(17) F(18) \
    F(19) F(20) F(21) F(22) F(23) F(24) F(25) F(26) F(27) F(28) F(29) F(30) F(31)

template <int MODE, typename TB>
__global__ void __launch_bounds__(SEM_VEC_THREADS) gm_pass_kernel(Batch bt, int gate)
{
    constexpr int NV = SEM_MAXM + 1;
    __shared__ double red[(SEM_VEC_THREADS / 64) * NV];
    const int g = blockIdx.x;
    const int ri = find_req(bt.vb, bt.n, g);
    const ReqDesc* R = bt.r[ri];
    const int blk = g - bt.vb[ri];
    if (!gate_ok(R, gate)) return;
    const PtRange pr = pt_range(R, blk);
    const int J = gp(R->I)[I_GJ];
    double acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = 0.0;
    double accm = 0.0;
    switch (J + 1) {
#define GM_CASE(n) case n: gm_body<n, MODE, TB>(R, pr, acc, accm); break;
        SEM_NJ_CASES(GM_CASE)
#undef GM_CASE
    default: break;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int nv = MODE == 2 ? 1 : J + 1;
#pragma unroll
    for (int i = 0; i < NV; ++i)
        if (i < nv) acc[i] = wave_sum(acc[i]);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (i < nv) red[wid * NV + i] = acc[i];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nv; i += blockDim.x) {
        double s = 0;
        for (int w = 0; w < nw; ++w) s += red[w * NV + i];
        put_partial(R, MODE == 2 ? R_GN : R_GM + i, blk, s);
    }
    if (MODE == 0) {
        double v1[1] = {accm};
        block_sum<double, 1>(v1, red);
        if (threadIdx.x == 0) put_partial(R, R_GMEAN, blk, v1[0]);
    }
}

// ------------------------------------------------------------------ pressure projection passes
// The space holds l stored vectors X_i (unnormalised, scale s_i = 1/||X_i||_A
// kept in S_PRS), l read on the device; the body is instantiated per l.
//   MODE 0: partials (X_i, b)                      -> alpha_i = s_i (X_i, b)
//   MODE 1: GX = PRXB = sum alpha_i s_i X_i         (the projected guess)
//   MODE 2: partials (X_i, w), (v, w), w = A v      -> beta_i, ||v||_A^2
//   MODE 3: X_l = v - sum beta_i s_i X_i            (A-orthogonalised new vector)
template <int NJ, int MODE, typename TB>
__device__ __forceinline__ void pr_body(const ReqDesc* R, const PtRange& pr, double (&acc)[SEM_MAX_PROJ + 1])
{
    const SEM_GLOBAL TB* X = fld<TB>(R, F_PRX);
    const long long np = R->np;
    constexpr int NA = NJ > 0 ? NJ : 1;
    double cf[NA];
#pragma unroll
    for (int i = 0; i < NJ; ++i)
        cf[i] = MODE == 1 ? gp(R->S)[S_PRA + i] * gp(R->S)[S_PRS + i]
              : MODE == 3 ? gp(R->S)[S_PRB + i] * gp(R->S)[S_PRS + i] : 0.0;
    auto b = fld<double>(R, F_GB);
    auto w = fld<double>(R, F_GWD);
    auto v = fld<double>(R, F_GW);
    auto gx = fldw<double>(R, F_GX);
    auto xb = fldw<double>(R, F_PRXB);
    SEM_GLOBAL TB* xl = fldw<TB>(R, F_PRX) + (long long)NJ * np;
    MulWalk mw(R, pr);
    for (long long p = pr.p0 + threadIdx.x; p < pr.p1; p += blockDim.x, mw.next()) {
        double xr[NA];
#pragma unroll
        for (int i = 0; i < NJ; ++i) xr[i] = (double)X[i * np + p];
        if (MODE == 0) {
            const double bv = b[p] * mw.im();
#pragma unroll
            for (int i = 0; i < NJ; ++i) acc[i] += xr[i] * bv;
        } else if (MODE == 1) {
            double sum = 0.0;
#pragma unroll
            for (int i = 0; i < NJ; ++i) sum += cf[i] * xr[i];
            gx[p] = sum;
            xb[p] = sum;
        } else if (MODE == 2) {
            const double wv = w[p] * mw.im();
#pragma unroll
            for (int i = 0; i < NJ; ++i) acc[i] += xr[i] * wv;
            acc[NJ] += v[p] * wv;
        } else {
            double sum = v[p];
#pragma unroll
            for (int i = 0; i < NJ; ++i) sum -= cf[i] * xr[i];
            xl[p] = (TB)sum;
        }
    }
}

#define SEM_NP_CASES(F)                                                                                 \
    F(0) F(1) F(2) F(3) F(4) F(5) F(6) F(7) F(8) F(9) F(10) F(11) F(12) F(13) F(14) F(15) F(16) F(17)   \
    F(18) F(19) F(20)

template <int MODE, typename TB>
__global__ void __launch_bounds__(SEM_VEC_THREADS) pr_pass_kernel(Batch bt, int gate)
{
    constexpr int NV = SEM_MAX_PROJ + 1;
    __shared__ double red[(SEM_VEC_THREADS / 64) * NV];
    const int g = blockIdx.x;
    const int ri = find_req(bt.vb, bt.n, g);
    const ReqDesc* R = bt.r[ri];
    const int blk = g - bt.vb[ri];
    if (!gate_ok(R, gate)) return;
    const PtRange pr = pt_range(R, blk);
    const int l = gp(R->I)[I_PRL];
    double acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = 0.0;
    switch (l) {
#define PR_CASE(n) case n: pr_body<n, MODE, TB>(R, pr, acc); break;
        SEM_NP_CASES(PR_CASE)
#undef PR_CASE
    default: break;
    }
    if (MODE == 0 || MODE == 2) {
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
        const int nv = MODE == 0 ? l : l + 1;
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (i < nv) acc[i] = wave_sum(acc[i]);
        if (lane == 0) {
#pragma unroll
            for (int i = 0; i < NV; ++i)
                if (i < nv) red[wid * NV + i] = acc[i];
        }
        __syncthreads();
        for (int i = threadIdx.x; i < nv; i += blockDim.x) {
            double sum = 0;
            for (int q = 0; q < nw; ++q) sum += red[q * NV + i];
            put_partial(R, R_GM + i, blk, sum);
        }
    }
}

// x += IDP * sum_{i < jend} y_i V_i  (right preconditioning applied once per
// cycle, with the same stored diagonal the Arnoldi operator used)
// XZ = false: x += D^{-1} sum_i y_i s_i V_i (Jacobi);
// XZ = true:  x += sum_i y_i Z_i with Z_i = M^{-1} s_i V_i kept from the
// Arnoldi steps (HSMG; the same vector as M^{-1} V y for a linear M)
template <int NJ, typename TD, typename TB, bool XZ = false>
__device__ __forceinline__ void xupd_body(const ReqDesc* R, const PtRange& pr)
{
    const SEM_GLOBAL TB* V = fld<TB>(R, XZ ? F_HZS : F_V);
    auto idp = fld<TD>(R, sizeof(TD) == 8 ? F_IDP64 : F_IDP32);
    auto x = fldw<double>(R, F_GX);
    const long long np = R->np;
    double y[NJ];
#pragma unroll
    for (int i = 0; i < NJ; ++i) y[i] = gp(R->S)[S_GY + i] * (XZ ? 1.0 : gp(R->S)[S_GVS + i]);
    for (long long p = pr.p0 + threadIdx.x; p < pr.p1; p += blockDim.x) {
        double vr[NJ];
#pragma unroll
        for (int i = 0; i < NJ; ++i) vr[i] = (double)V[i * np + p];
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < NJ; ++i) s += y[i] * vr[i];
        if constexpr (XZ) x[p] += s;
        else x[p] += s * (double)idp[p];
    }
}

template <typename TD, typename TB, bool XZ = false>
__global__ void __launch_bounds__(SEM_VEC_THREADS) gm_xupd_kernel(Batch bt, int gate)
{
    const int g = blockIdx.x;
    const int ri = find_req(bt.vb, bt.n, g);
    const ReqDesc* R = bt.r[ri];
    const int blk = g - bt.vb[ri];
    if (!gate_ok(R, gate)) return;
    const PtRange pr = pt_range(R, blk);
    switch (gp(R->I)[I_GJEND]) {
#define XU_CASE(n) case n: xupd_body<n, TD, TB, XZ>(R, pr); break;
        SEM_NJ_CASES(XU_CASE)
#undef XU_CASE
    default: break;
    }
}

void launch_vec(const Batch& b, const VecArgs& a, hipStream_t s)
{
    dim3 grid(b.vb[b.n], a.ncomp > 0 ? a.ncomp : 1);
    dim3 blk(SEM_VEC_THREADS);
    if (grid.x == 0) return;
    switch (a.op) {
    case V_GM_DOTS:
        if (a.tb == P64) hipLaunchKernelGGL((gm_pass_kernel<0, double>), grid, blk, 0, s, b, a.gate);
        else hipLaunchKernelGGL((gm_pass_kernel<0, float>), grid, blk, 0, s, b, a.gate);
        return;
    case V_GM_UPD_DOTS:
        if (a.tb == P64) hipLaunchKernelGGL((gm_pass_kernel<1, double>), grid, blk, 0, s, b, a.gate);
        else hipLaunchKernelGGL((gm_pass_kernel<1, float>), grid, blk, 0, s, b, a.gate);
        return;
    case V_GM_UPD_NORM:
        if (a.tb == P64) hipLaunchKernelGGL((gm_pass_kernel<2, double>), grid, blk, 0, s, b, a.gate);
        else hipLaunchKernelGGL((gm_pass_kernel<2, float>), grid, blk, 0, s, b, a.gate);
        return;
    case V_PR_ADOTS:
    case V_PR_GUESS:
    case V_PR_BDOTS:
    case V_PR_ORTH: {
        const int mode = a.op == V_PR_ADOTS ? 0 : a.op == V_PR_GUESS ? 1 : a.op == V_PR_BDOTS ? 2 : 3;
#define PR_GO(M)                                                                                       \
    if (a.tb == P64) hipLaunchKernelGGL((pr_pass_kernel<M, double>), grid, blk, 0, s, b, a.gate);      \
    else hipLaunchKernelGGL((pr_pass_kernel<M, float>), grid, blk, 0, s, b, a.gate);
        if (mode == 0) { PR_GO(0) } else if (mode == 1) { PR_GO(1) } else if (mode == 2) { PR_GO(2) } else { PR_GO(3) }
#undef PR_GO
        return;
    }
    case V_GM_XZ:
        if (a.tb == P64) hipLaunchKernelGGL((gm_xupd_kernel<double, double, true>), grid, blk, 0, s, b, a.gate);
        else hipLaunchKernelGGL((gm_xupd_kernel<double, float, true>), grid, blk, 0, s, b, a.gate);
        return;
    case V_GM_XUPD:
        if (a.tv == P64 && a.tb == P64) hipLaunchKernelGGL((gm_xupd_kernel<double, double>), grid, blk, 0, s, b, a.gate);
        else if (a.tv == P64) hipLaunchKernelGGL((gm_xupd_kernel<double, float>), grid, blk, 0, s, b, a.gate);
        else if (a.tb == P64) hipLaunchKernelGGL((gm_xupd_kernel<float, double>), grid, blk, 0, s, b, a.gate);
        else hipLaunchKernelGGL((gm_xupd_kernel<float, float>), grid, blk, 0, s, b, a.gate);
        return;
    default: break;
    }
    // operations on the velocity solver vectors come in every storage /
    // accumulation pair; the others are fp64
#define VEC_T(OP)                                                                                        \
    case OP:                                                                                             \
        if (a.tv == P64) hipLaunchKernelGGL((vec_kernel<double, double, OP>), grid, blk, 0, s, b, a);   \
        else if (a.ta == P64) hipLaunchKernelGGL((vec_kernel<float, double, OP>), grid, blk, 0, s, b, a);\
        else hipLaunchKernelGGL((vec_kernel<float, float, OP>), grid, blk, 0, s, b, a);                 \
        return;
#define VEC_D(OP)                                                                                        \
    case OP: hipLaunchKernelGGL((vec_kernel<double, double, OP>), grid, blk, 0, s, b, a); return;
    switch (a.op) {
        VEC_T(V_PCG_INIT) VEC_T(V_PCG_UPD) VEC_T(V_PCG_P) VEC_T(V_US_ADD)
        VEC_D(V_US_COPY) VEC_D(V_IDV) VEC_D(V_SUM_UNIQUE) VEC_D(V_SUM_MASS)
        VEC_D(V_SUB_MEAN) VEC_D(V_COPY) VEC_D(V_ZERO) VEC_D(V_GM_RESID) VEC_D(V_CORRECT) VEC_D(V_MASS_RAW)
        VEC_D(V_PR_V) VEC_D(V_AXPY_RAW)
    default: break;
    }
#undef VEC_T
#undef VEC_D
}

// ------------------------------------------------------------------ finalise kernel
__global__ void __launch_bounds__(256) fin_kernel(Batch bt, FinArgs a)
{
    fin_body((ReqDesc*)bt.r[blockIdx.x], blockIdx.x, a);
}

void launch_fin(const Batch& b, const FinArgs& a, hipStream_t s)
{
    if (b.n == 0) return;
    hipLaunchKernelGGL(fin_kernel, dim3(b.n), dim3(256), 0, s, b, a);
}

}  // namespace semk
