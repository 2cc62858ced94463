// Finalisation of Krylov reductions and the scalar logic of PCG, GMRES and
// the BDF/EXT step, run by a one-workgroup-per-request kernel after the
// producer of the partials.  Partials of a slot are added in a fixed order
// (fp64), so a request's scalars do not depend on its batch.  (Letting the
// last workgroup of the producer finalise instead needs a device-scope
// release per workgroup, an L2 write-back on this chip that costs far more
// than the separate launch.)
#pragma once
#include "k_common.h"

namespace semk {

// ------------------------------------------------------------------ finalise kernels
// fixed-order sums of the partials of NS slots (valid in thread 0): for each
// slot, thread t adds partials t, t+bd, t+2bd, ... in that order, then the
// per-thread sums are added in a fixed tree.  The slots are read together,
// eight loads of each in flight, so a finaliser waits for one round of loads
// where it waited for NS.  red must hold (blockDim.x / 64) * NS values.
template <int NS>
static __device__ void slot_sums(const ReqDesc* R, const int (&slot)[NS], double (&out)[NS], double* red)
{
    constexpr int U = 8;
    const SEM_GLOBAL double* p[NS];
    int cnt[NS], most = 0;
    double s[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        p[k] = gp(R->part) + (long long)slot[k] * R->pstride;
        cnt[k] = gp(R->I)[I_PCNT + slot[k]];
        most = max(most, cnt[k]);
        s[k] = 0.0;
    }
    const int bd = blockDim.x;
    for (int q = threadIdx.x; q < most; q += U * bd) {
        double a[NS][U];
#pragma unroll
        for (int k = 0; k < NS; ++k)
#pragma unroll
            for (int u = 0; u < U; ++u) a[k][u] = q + u * bd < cnt[k] ? p[k][q + u * bd] : 0.0;
#pragma unroll
        for (int k = 0; k < NS; ++k)
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (q + u * bd < cnt[k]) s[k] += a[k][u];
    }
    block_sum<double, NS>(s, red);
#pragma unroll
    for (int k = 0; k < NS; ++k) out[k] = s[k];
}
static __device__ double slot_sum(const ReqDesc* R, int slot, double* red)
{
    const int sl[1] = {slot};
    double v[1];
    slot_sums<1>(R, sl, v, red);
    return v[0];
}
static __device__ double slot_max(const ReqDesc* R, int slot, double* red)
{
    double s = 0.0;
    const SEM_GLOBAL double* p = gp(R->part) + (long long)slot * R->pstride;
    const int cnt = gp(R->I)[I_PCNT + slot];
    for (int q = threadIdx.x; q < cnt; q += blockDim.x) s = fmax(s, p[q]);
    s = wave_max(s);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    double m = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, red[w]);
    __syncthreads();
    return m;
}

// fixed-order sums of nslots (<= 32) consecutive slots at once: 8 groups of
// 32 threads (the first 256 threads), thread (g, s) adds partials g, g+8, ...
// of slot s in that order (eight loads in flight); the 8 group sums are then
// added in group order.  out must hold nslots values.
static __device__ void multi_slot_sum(const ReqDesc* R, int slot0, int nslots, double* out, double* scratch)
{
    const int t = threadIdx.x, sl = t & 31, g = t >> 5;
    double acc = 0.0;
    if (t < 256 && sl < nslots) {
        const SEM_GLOBAL double* p = gp(R->part) + (long long)(slot0 + sl) * R->pstride;
        const int cnt = gp(R->I)[I_PCNT + slot0 + sl];
        int q = g;
        for (; q + 56 < cnt; q += 64) {
            double a[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) a[k] = p[q + 8 * k];
#pragma unroll
            for (int k = 0; k < 8; ++k) acc += a[k];
        }
        for (; q < cnt; q += 8) acc += p[q];
    }
    if (t < 256) scratch[t] = acc;
    __syncthreads();
    if (t < nslots) {
        double v = 0.0;
        for (int k = 0; k < 8; ++k) v += scratch[k * 32 + t];
        out[t] = v;
    }
    __syncthreads();
}

static __device__ __forceinline__ bool finite(double v) { return isfinite(v); }

// The scalar logic of one request, run by one workgroup of 256 threads (the
// slot sums use every thread and red holds 4 waves x 8 slots; the multi-slot
// sum uses the first 256).  ri is the request's position in its batch (host
// arrays).
static __device__ __noinline__ void fin_body(ReqDesc* R, int ri, const FinArgs a)
{
    __shared__ double red[32];
    __shared__ double sums[SEM_MAXM + 2];
    __shared__ double scratch[256];
    SEM_GLOBAL double* S = gp(R->S);
    SEM_GLOBAL int* I = gp(R->I);
    const int t = threadIdx.x;
    if (a.gate2 >= 0 && !I[a.gate2]) return;  // uniform per workgroup
    switch (a.op) {
    case FIN_VINIT: {
        const int sl[3] = {R_A, R_A + 1, R_A + 2};
        double v[3];
        slot_sums<3>(R, sl, v, red);
        for (int c = 0; c < 3; ++c) {
            const double s = v[c];
            if (t == 0) {
                double rn = sqrt(s);
                S[S_R0 + c] = rn;
                S[S_RN + c] = rn;
                bool act = rn > S[S_VTOL] && I[I_VREF + c] < I[I_VMAXREF];
                if (!finite(rn)) { I[I_NAN] = 1; act = false; }
                if (act) I[I_VREF + c] += 1;
                I[I_VACT + c] = act ? 1 : 0;
            }
        }
        break;
    }
    case FIN_PCG_RHO: {
        const int sl[3] = {R_B, R_B + 1, R_B + 2};
        double v[3];
        slot_sums<3>(R, sl, v, red);
        for (int c = 0; c < 3; ++c)
            if (t == 0 && I[I_VACT + c]) S[S_RHO + c] = v[c];
        break;
    }
    case FIN_PCG_ALPHA: {
        // (an idle component's slot is summed too; its result is not used)
        const int sl[3] = {R_A, R_A + 1, R_A + 2};
        double v[3];
        slot_sums<3>(R, sl, v, red);
        for (int c = 0; c < 3; ++c)
            if (t == 0 && I[I_VACT + c]) S[S_ALPHA + c] = S[S_RHO + c] / v[c];
        break;
    }
    case FIN_PCG_BETA: {
        const int sl[6] = {R_B, R_C, R_B + 1, R_C + 1, R_B + 2, R_C + 2};
        double v[6];
        slot_sums<6>(R, sl, v, red);
        for (int c = 0; c < 3; ++c) {
            if (!I[I_VACT + c]) continue;
            const double rr = v[2 * c], rz = v[2 * c + 1];
            if (t == 0) {
                double rn = sqrt(rr);
                S[S_RN + c] = rn;
                I[I_VIT + c] += 1;
                if (!finite(rn)) { I[I_NAN] = 1; I[I_VACT + c] = 0; }
                else if (rn <= S[S_VTOL] || I[I_VIT + c] >= I[I_VMAXIT]) I[I_VACT + c] = 0;
                else { S[S_BETA + c] = rz / S[S_RHO + c]; S[S_RHO + c] = rz; }
            }
        }
        break;
    }
    case FIN_MEAN_UNIQUE: {
        double s = slot_sum(R, R_X3, red);
        if (t == 0) S[S_MEAN] = s / (double)R->nglob;
        break;
    }
    case FIN_MEAN_MASS: {
        double s = slot_sum(R, R_X3, red);
        if (t == 0) S[S_MEAN] = s / S[S_VOL];
        break;
    }
    case FIN_GM_H1:
    case FIN_GM_H2: {
        if (!I[I_GARN]) break;
        const int J = I[I_GJ];
        multi_slot_sum(R, R_GM, J + 1, sums, scratch);
        // dots with the stored vectors, scaled to the normalised basis
        if (t <= J) S[(a.op == FIN_GM_H1 ? S_GHC : S_GH2) + t] = sums[t] * S[S_GVS + t];
        if (a.op == FIN_GM_H1) {
            double s = slot_sum(R, R_GMEAN, red);
            if (t == 0) S[S_GMEAN] = s / (double)R->nglob;
        }
        if (t == 0) I[I_GNORM] = 0;
        break;
    }
    case FIN_GM_COL: {
        if (!I[I_GARN]) break;
        double hn2 = slot_sum(R, R_GN, red);
        if (t == 0) {
            const int m = I[I_GM];
            const int J = I[I_GJ];
            SEM_GLOBAL double* H = S + S_GH;
            SEM_GLOBAL double* cs = S + S_GCS;
            SEM_GLOBAL double* sn = S + S_GSN;
            SEM_GLOBAL double* gg = S + S_GG;
            const double hn = sqrt(hn2);
            for (int i = 0; i <= J; ++i) H[i * m + J] = S[S_GHC + i] + S[S_GH2 + i];
            H[(J + 1) * m + J] = hn;
            for (int i = 0; i < J; ++i) {
                const double x = H[i * m + J], y = H[(i + 1) * m + J];
                H[i * m + J] = cs[i] * x + sn[i] * y;
                H[(i + 1) * m + J] = -sn[i] * x + cs[i] * y;
            }
            const double x = H[J * m + J], y = H[(J + 1) * m + J];
            const double den = sqrt(x * x + y * y);
            cs[J] = x / den;
            sn[J] = y / den;
            H[J * m + J] = den;
            H[(J + 1) * m + J] = 0.0;
            gg[J + 1] = -sn[J] * gg[J];
            gg[J] = cs[J] * gg[J];
            I[I_GIT] += 1;
            const bool bad = !finite(gg[J + 1]) || !finite(den);
            if (bad) I[I_NAN] = 1;
            if (bad || fabs(gg[J + 1]) <= S[S_PTOL] || hn == 0.0 || J + 1 == m || I[I_GIT] >= I[I_GMAXIT]) {
                const int jend = bad ? 0 : J + 1;
                SEM_GLOBAL double* yv = S + S_GY;
                for (int r = jend - 1; r >= 0; --r) {
                    double s = gg[r];
                    for (int k = r + 1; k < jend; ++k) s -= H[r * m + k] * yv[k];
                    yv[r] = s / H[r * m + r];
                }
                I[I_GJEND] = jend;
                I[I_GARN] = 0;
                I[I_GEND] = 1;
                I[I_GENDAX] = 1;
                I[I_GNORM] = 0;
            } else {
                I[I_GJ] = J + 1;
                S[S_GVS + J + 1] = 1.0 / hn;
                I[I_GNORM] = 1;
            }
        }
        break;
    }
    case FIN_GM_RESTART: {
        if (!I[I_GEND]) break;
        double s = slot_sum(R, R_GN, red);
        if (t == 0) {
            const double beta = sqrt(s);
            S[S_GBETA] = beta;
            I[I_GEND] = 0;
            I[I_GENDAX] = 0;
            if (!finite(beta)) I[I_NAN] = 1;
            if (!finite(beta) || beta <= S[S_PTOL] || I[I_GIT] >= I[I_GMAXIT]) {
                I[I_GACT] = 0; I[I_GARN] = 0; I[I_GNORM] = 0;
            } else {
                I[I_GJ] = 0;
                SEM_GLOBAL double* gg = S + S_GG;
                for (int i = 0; i <= SEM_MAXM; ++i) gg[i] = 0.0;
                gg[0] = beta;
                S[S_GVS] = 1.0 / beta;
                I[I_GARN] = 1; I[I_GNORM] = 1;
            }
        }
        break;
    }
    case FIN_GM_START: {
        // fresh solve: the first cycle end computes r = b, or r = b - A x0
        // when the iterate starts from a nonzero projected guess
        if (t == 0) {
            const int x0 = R->proj_L > 0 && I[I_PRL] > 0;
            I[I_GJ] = 0; I[I_GJEND] = 0; I[I_GIT] = 0;
            I[I_GACT] = 1; I[I_GARN] = 0; I[I_GEND] = 1; I[I_GENDAX] = x0; I[I_GNORM] = 0;
        }
        break;
    }
    case FIN_PR_ALPHA: {
        const int l = I[I_PRL];
        multi_slot_sum(R, R_GM, l, sums, scratch);
        if (t < l) S[S_PRA + t] = sums[t] * S[S_PRS + t];
        break;
    }
    case FIN_PR_POST: {
        if (t == 0) {
            const int full = I[I_PRL] >= R->proj_L;
            if (full) I[I_PRL] = 0;
            I[I_PRFULL] = full;
        }
        break;
    }
    case FIN_PR_BETA: {
        const int l = I[I_PRL];
        multi_slot_sum(R, R_GM, l + 1, sums, scratch);
        if (t == 0) {
            const double n2b = sums[l];
            double n2 = n2b;
            for (int i = 0; i < l; ++i) {
                const double bi = sums[i] * S[S_PRS + i];
                S[S_PRB + i] = bi;
                n2 -= bi * bi;
            }
            // a vector whose A-norm mostly lies in the space is dependent: dropped
            const int add = finite(n2b) && n2b > 0.0 && n2 > 1e-12 * n2b;
            I[I_PRADD] = add;
            if (add) S[S_PRS + l] = 1.0 / sqrt(n2);
        }
        break;
    }
    case FIN_PR_COMMIT: {
        if (t == 0 && I[I_PRADD]) I[I_PRL] += 1;
        break;
    }
    case FIN_COMMIT_CHECK: {
        // a captured step runs a fixed number of iterations: its correction,
        // lag rotation and projection update run only where every solve
        // stopped by itself within them (converged, hit its limit or met a
        // non-finite value); elsewhere the host re-runs the step
        if (t == 0) {
            const int done = !(I[I_VACT] | I[I_VACT + 1] | I[I_VACT + 2] | I[I_GACT]);
            I[I_COMMIT] = I[I_COMMIT + 1] = I[I_COMMIT + 2] = done;
            if (!done) I[I_PRADD] = 0;
        }
        break;
    }
    case FIN_DIAG: {
        const int sl[2] = {R_X0, R_X1};
        double v[2];
        slot_sums<2>(R, sl, v, red);
        const double ke = v[0], en = v[1];
        double md = slot_max(R, R_X2, red);
        double cr = slot_max(R, R_X4, red);
        if (t == 0) {
            S[S_KE] = ke / S[S_VOL];
            S[S_ENST] = en / S[S_VOL];
            S[S_MAXDIV] = md;
            S[S_CFLR] = cr;
            if (!finite(ke) || !finite(en)) I[I_NAN] = 1;
        }
        break;
    }
    case FIN_STEP_BEGIN: {
        if (t == 0) {
            const int torder = I[I_TORDER];
            const int k = I[I_STEP] + 1 < torder ? I[I_STEP] + 1 : torder;
            I[I_ORDER] = k;
            double b0, b1 = 0, b2 = 0, b3 = 0, a1 = 0, a2 = 0, a3 = 0;
            const double rate = S[S_CFLR];
            if (S[S_CFLT] > 0.0) {
                // adaptive step toward the target CFL, at most the configured dt,
                // and after the first step within [0.5, 1.1] of the previous one
                double dt = rate > 0.0 ? S[S_CFLT] / rate : S[S_DTMAX];
                if (I[I_STEP] > 0) {
                    const double prev = S[S_DTH];
                    if (dt > 1.1 * prev) dt = 1.1 * prev;
                    if (dt < 0.5 * prev) dt = 0.5 * prev;
                }
                if (dt > S[S_DTMAX]) dt = S[S_DTMAX];
                S[S_DTH + 2] = S[S_DTH + 1];
                S[S_DTH + 1] = S[S_DTH];
                S[S_DTH] = dt;
                S[S_DT] = dt;
                // BDF-k: derivative at t_{n+1} of the interpolant through the
                // last k+1 time levels; EXT-k: its value from the last k levels
                // (nodes measured back from t_{n+1}: 0, -h0, -h0-h1, -h0-h1-h2)
                double z[4];
                z[0] = 0.0;
                for (int q = 1; q < 4; ++q) z[q] = z[q - 1] - S[S_DTH + q - 1];
                double bb[4] = {0, 0, 0, 0}, aa[4] = {0, 0, 0, 0};
                double s0 = 0.0;
                for (int q = 1; q <= k; ++q) s0 += 1.0 / (z[0] - z[q]);
                bb[0] = dt * s0;
                for (int j = 1; j <= k; ++j) {
                    double nu_ = 1.0, de = 1.0, w = 1.0;
                    for (int q = 0; q <= k; ++q) {
                        if (q == j) continue;
                        de *= z[j] - z[q];
                        if (q != 0) {
                            nu_ *= z[0] - z[q];
                            w *= (z[0] - z[q]) / (z[j] - z[q]);
                        }
                    }
                    bb[j] = -dt * nu_ / de;
                    aa[j] = w;
                }
                b0 = bb[0]; b1 = bb[1]; b2 = bb[2]; b3 = bb[3];
                a1 = aa[1]; a2 = aa[2]; a3 = aa[3];
            } else if (k == 1) { b0 = 1.0; b1 = 1.0; a1 = 1.0; }
            else if (k == 2) { b0 = 1.5; b1 = 2.0; b2 = -0.5; a1 = 2.0; a2 = -1.0; }
            else { b0 = 11.0 / 6.0; b1 = 3.0; b2 = -1.5; b3 = 1.0 / 3.0; a1 = 3.0; a2 = -3.0; a3 = 1.0; }
            S[S_CFL] = S[S_DT] * rate;
            S[S_BETA0] = b0;
            S[S_BDF] = b1; S[S_BDF + 1] = b2; S[S_BDF + 2] = b3;
            S[S_EXT] = a1; S[S_EXT + 1] = a2; S[S_EXT + 2] = a3;
            S[S_H1] = S[S_NU];
            S[S_H2] = b0 / S[S_DT];
            const bool stale = I[I_STEP] == 0 || S[S_IDV_H1] != S[S_H1] || S[S_IDV_H2] != S[S_H2];
            I[I_IDVSTALE] = stale ? 1 : 0;
            S[S_IDV_H1] = S[S_H1];
            S[S_IDV_H2] = S[S_H2];
            S[S_MEAN + 0] = 0.0;
            for (int c = 0; c < 3; ++c) { I[I_VIT + c] = 0; I[I_VREF + c] = 0; I[I_VACT + c] = 0; }
        }
        break;
    }
    case FIN_STEP_END: {
        if (t == 0) {
            for (int c = 0; c < 3; ++c) {
                void* un = R->f[F_UL2 + c];          // holds u^{n+1}
                R->f[F_UL2 + c] = R->f[F_UL1 + c];
                R->f[F_UL1 + c] = R->f[F_U + c];
                R->f[F_U + c] = un;
                void* bs = R->f[F_BNL2 + c];
                R->f[F_BNL2 + c] = R->f[F_BNL1 + c];
                R->f[F_BNL1 + c] = R->f[F_BN + c];
                R->f[F_BN + c] = bs;
            }
            I[I_STEP] += 1;
            S[S_TIME] += S[S_DT];
        }
        break;
    }
    case FIN_POLL: {
        if (t == 0) {
            int v = 0;
            for (int c = 0; c < (a.ncomp > 1 ? a.ncomp : 1); ++c) v |= I[a.gate + c];
            a.host_flags[ri] = v;
        }
        break;
    }
    case FIN_SUM_RAW: {
        double s = slot_sum(R, a.f0, red);
        if (t == 0) S[S_RED + a.gate] = s;
        break;
    }
    case FIN_VOL: {
        double s = slot_sum(R, R_X3, red);
        if (t == 0) S[S_VOL] = s;
        break;
    }
    case FIN_STATS: {
        if (t == 0) {
            double* o = a.host_stats + (long long)ri * SEM_NSTAT;  // pinned host memory
            o[0] = S[S_TIME]; o[1] = S[S_KE]; o[2] = S[S_ENST]; o[3] = S[S_MAXDIV];
            for (int c = 0; c < 3; ++c) { o[4 + c] = I[I_VIT + c]; o[7 + c] = S[S_RN + c]; }
            o[10] = I[I_GIT]; o[11] = S[S_GBETA]; o[12] = I[I_NAN]; o[13] = I[I_STEP];
            o[14] = I[I_VREF] > I[I_VREF + 1] ? I[I_VREF] : I[I_VREF + 1];
            if (I[I_VREF + 2] > o[14]) o[14] = I[I_VREF + 2];
            o[15] = I[I_ORDER];
            o[16] = S[S_DT]; o[17] = S[S_CFL];
            o[18] = I[I_COMMIT];
        }
        break;
    }
    default: break;
    }
    (void)sums;
}


}  // namespace semk
