// Dealiased convection: the convective term integrated on LXD = ceil(3 LX / 2)
// Gauss-Legendre points per direction (the 3/2 rule) instead of by
// collocation on the GLL points:
//   BN_f(l) = - sum_q W_q phi_l(z_q) sum_c u_c(z_q) sum_a (dr_a/dx_c)(z_q) (du_f/dr_a)(z_q)
// with W = jac * (Gauss-Legendre weights).  The metric terms W dr_a/dx_c at
// the fine points are computed once per mesh (dealias_geom_kernel) from the
// interpolated coordinates.  Per element (one workgroup), the velocity and
// its reference derivatives are taken to the fine points by three staged
// one-dimensional contractions in LDS; the contravariant velocity
// V_a = sum_c u_c W dr_a/dx_c stays in registers (each thread owns fixed
// fine points), and the weighted integrand goes back to the GLL points by
// the transposed contractions.
#include "k_common.h"

namespace semk {

template <int LX> struct Dl {
    static constexpr int LXD = (3 * LX + 1) / 2;
    static constexpr int N3 = LX * LX * LX;
    static constexpr int ND3 = LXD * LXD * LXD;
    static constexpr int NT = ND3 <= 1728 ? 256 : 512;
    static constexpr int NQ = (ND3 + NT - 1) / NT;
    static constexpr int NA = LXD * LX * LX;
    static constexpr int NB = LXD * LXD * LX;
};

// tables after the GLL tables: fp64 [D lx^2][w lx][xi lx][1/mult lx^3][I][ID][wz],
// fp32 [D lx^2][w lx][xi lx][I][ID][wz]; I, ID are LXD x LX, wz has LXD entries
template <int LX> __device__ __forceinline__ int dl_off64() { return LX * LX + 2 * LX + LX * LX * LX; }
template <int LX> __device__ __forceinline__ int dl_off32() { return LX * LX + 2 * LX; }

// out[(k LXD + j) LXD + i] = sum_{a,b,c} A1[i][a] A2[j][b] A3[k][c] in[(c LX + b) LX + a]
template <int LX, typename C>
__device__ __forceinline__ void interp3(const C* A1, const C* A2, const C* A3, const C* in, C* tA, C* tB, C* out)
{
    constexpr int LXD = Dl<LX>::LXD, NT = Dl<LX>::NT;
    const int t = threadIdx.x;
    for (int idx = t; idx < LX * LX * LXD; idx += NT) {
        const int i = idx % LXD, kj = idx / LXD;
        C s = 0;
#pragma unroll
        for (int a = 0; a < LX; ++a) s += A1[i * LX + a] * in[kj * LX + a];
        tA[idx] = s;
    }
    __syncthreads();
    for (int idx = t; idx < LX * LXD * LXD; idx += NT) {
        const int i = idx % LXD, r = idx / LXD, j = r % LXD, k = r / LXD;
        C s = 0;
#pragma unroll
        for (int b = 0; b < LX; ++b) s += A2[j * LX + b] * tA[(k * LX + b) * LXD + i];
        tB[idx] = s;
    }
    __syncthreads();
    for (int idx = t; idx < LXD * LXD * LXD; idx += NT) {
        const int i = idx % LXD, r = idx / LXD, j = r % LXD, k = r / LXD;
        C s = 0;
#pragma unroll
        for (int c = 0; c < LX; ++c) s += A3[k * LX + c] * tB[(c * LXD + j) * LXD + i];
        out[idx] = s;
    }
    __syncthreads();
}

// transposed: out[(c LX + b) LX + a] = -sum_{k,j,i} A[i][a] A[j][b] A[k][c] in[(k LXD + j) LXD + i]
template <int LX, typename C>
__device__ __forceinline__ void back3_neg(const C* A, const C* in, C* tB, C* tA, SEM_GLOBAL double* out)
{
    constexpr int LXD = Dl<LX>::LXD, NT = Dl<LX>::NT;
    const int t = threadIdx.x;
    for (int idx = t; idx < LX * LXD * LXD; idx += NT) {
        const int i = idx % LXD, r = idx / LXD, j = r % LXD, c = r / LXD;
        C s = 0;
#pragma unroll
        for (int k = 0; k < LXD; ++k) s += A[k * LX + c] * in[(k * LXD + j) * LXD + i];
        tB[idx] = s;
    }
    __syncthreads();
    for (int idx = t; idx < LX * LX * LXD; idx += NT) {
        const int i = idx % LXD, r = idx / LXD, b = r % LX, c = r / LX;
        C s = 0;
#pragma unroll
        for (int j = 0; j < LXD; ++j) s += A[j * LX + b] * tB[(c * LXD + j) * LXD + i];
        tA[idx] = s;
    }
    __syncthreads();
    for (int idx = t; idx < LX * LX * LX; idx += NT) {
        const int a = idx % LX, r = idx / LX;
        C s = 0;
#pragma unroll
        for (int i = 0; i < LXD; ++i) s += A[i * LX + a] * tA[r * LXD + i];
        out[idx] = -(double)s;
    }
    __syncthreads();
}

// fine-grid metric terms MF[e][a*3+c][q] = W_q (dr_a/dx_c)(z_q), fp64, from
// the coordinates of the GLL nodes (the same mapping as the GLL geometry)
template <int LX>
__global__ void __launch_bounds__(Dl<LX>::NT) dealias_geom_kernel(Batch bt, MeshParams mp)
{
    constexpr int LXD = Dl<LX>::LXD, N3 = Dl<LX>::N3, ND3 = Dl<LX>::ND3, NT = Dl<LX>::NT, NQ = Dl<LX>::NQ;
    __shared__ double sI[LXD * LX], sID[LXD * LX], swz[LXD], sxi[LX];
    __shared__ double sx[3][N3];
    __shared__ double F[ND3];
    __shared__ double tA[Dl<LX>::NA], tB[Dl<LX>::NB];
    const int g = blockIdx.x;
    const int ri = find_req(bt.eb, bt.n, g);
    const ReqDesc* R = bt.r[ri];
    const int blk = g - bt.eb[ri];
    const int t = threadIdx.x;
    const SEM_GLOBAL double* tab = gp(R->D64);
    for (int q = t; q < LXD * LX; q += NT) {
        sI[q] = tab[dl_off64<LX>() + q];
        sID[q] = tab[dl_off64<LX>() + LXD * LX + q];
    }
    for (int q = t; q < LXD; q += NT) swz[q] = tab[dl_off64<LX>() + 2 * LXD * LX + q];
    for (int q = t; q < LX; q += NT) sxi[q] = tab[LX * LX + LX + q];
    __syncthreads();
    SEM_GLOBAL double* MF = gfieldw<double>(R, F_MFD64);
    for (int el = 0; el < R->epb; ++el) {
        const int e = blk * R->epb + el;
        if (e >= R->E) break;
        for (int p = t; p < N3; p += NT) {
            const int i = p % LX, j = (p / LX) % LX, k = p / (LX * LX);
            double xo[3];
            node_xyz(mp, sxi, e, i, j, k, xo);
            sx[0][p] = xo[0]; sx[1][p] = xo[1]; sx[2][p] = xo[2];
        }
        __syncthreads();
        SEM_GLOBAL double* me = MF + (long long)e * 9 * ND3;
        // J[c][a] = dx_c/dr_a at the fine points, parked in slot a*3+c
        for (int c = 0; c < 3; ++c)
            for (int a = 0; a < 3; ++a) {
                interp3<LX, double>(a == 0 ? sID : sI, a == 1 ? sID : sI, a == 2 ? sID : sI, sx[c], tA, tB, F);
                for (int r = 0; r < NQ; ++r) {
                    const int q = t + r * NT;
                    if (q < ND3) me[(a * 3 + c) * ND3 + q] = F[q];
                }
            }
        for (int r = 0; r < NQ; ++r) {
            const int q = t + r * NT;
            if (q >= ND3) break;
            double J[3][3];
            for (int c = 0; c < 3; ++c)
                for (int a = 0; a < 3; ++a) J[c][a] = me[(a * 3 + c) * ND3 + q];
            const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
                             - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
                             + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
            double inv[3][3];
            inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
            inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
            inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
            inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
            inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
            inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
            inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
            inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
            inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
            const int i = q % LXD, j = (q / LXD) % LXD, k = q / (LXD * LXD);
            const double W = det * swz[i] * swz[j] * swz[k];
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 3; ++c) me[(a * 3 + c) * ND3 + q] = W * inv[a][c];
        }
        __syncthreads();
    }
}

// fp32 and element-scaled 16-bit copies of the fine-grid metric terms, each
// rounded once from fp64 (power-of-two scales keep the 16-bit rounding single)
template <typename T16>
__global__ void __launch_bounds__(256) dealias_cast_kernel(Batch bt, int per_elem, int want32, int want16)
{
    __shared__ double red[4];
    const int g = blockIdx.x;
    const int ri = find_req(bt.eb, bt.n, g);
    const ReqDesc* R = bt.r[ri];
    const int blk = g - bt.eb[ri];
    const SEM_GLOBAL double* src = gfield<double>(R, F_MFD64);
    for (int el = 0; el < R->epb; ++el) {
        const int e = blk * R->epb + el;
        if (e >= R->E) break;
        const SEM_GLOBAL double* me = src + (long long)e * per_elem;
        if (want32) {
            SEM_GLOBAL float* dst = gfieldw<float>(R, F_MFD32) + (long long)e * per_elem;
            for (int p = threadIdx.x; p < per_elem; p += blockDim.x) dst[p] = (float)me[p];
        }
        if (want16) {
            double mx = 0.0;
            for (int p = threadIdx.x; p < per_elem; p += blockDim.x) mx = fmax(mx, fabs(me[p]));
            mx = wave_max(mx);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
            __syncthreads();
            mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
            __syncthreads();
            const double sc = mx > 0 ? exp2(ceil(log2(mx))) : 1.0;
            if (threadIdx.x == 0) gfieldw<float>(R, F_MFDSC)[e] = (float)sc;
            const int lx = R->lx;
            const int per16 = dl16_per_elem(lx);
            SEM_GLOBAL T16* dst = gfieldw<T16>(R, F_MFD16) + (long long)e * per16;
            if (dl16_lane(lx)) {
                // [tile][ac][g][m][r]: fine point (k' = 4g + r, n = 16 tile + m); zero outside
                const int nd = (3 * lx + 1) / 2, nn = nd * nd, ng = (nd + 3) / 4;
                for (int p = threadIdx.x; p < per16; p += blockDim.x) {
                    const int r = p & 3, m = (p >> 2) & 15, rest = p >> 6;
                    const int g = rest % ng, ac = (rest / ng) % 9, tile = rest / (ng * 9);
                    const int kk = 4 * g + r, n = 16 * tile + m;
                    const double v = (kk < nd && n < nn) ? me[(long long)ac * nd * nn + kk * nn + n] / sc : 0.0;
                    stg(dst + p, to<T16>(v));
                }
            } else {
                for (int p = threadIdx.x; p < per_elem; p += blockDim.x) stg(dst + p, to<T16>(me[p] / sc));
            }
        }
    }
}

template <typename TM> __device__ __forceinline__ int mfd_field() { return F_MFD16; }
template <> __device__ __forceinline__ int mfd_field<double>() { return F_MFD64; }
template <> __device__ __forceinline__ int mfd_field<float>() { return F_MFD32; }

// one fine-grid metric term in the arithmetic type (16-bit storage carries the element scale)
template <typename TM, typename C> __device__ __forceinline__ C mload(const SEM_GLOBAL TM* p, C sc)
{
    if constexpr (sizeof(TM) == 2) return to<C>(ldg(p)) * sc;
    else return (C)*p;
}
template <typename TM, typename C> __device__ __forceinline__ C mscale(const ReqDesc* R, int e)
{
    if constexpr (sizeof(TM) == 2) return (C)gfield<float>(R, F_MFDSC)[e];
    else return (C)1;
}

// BN = dealiased -B (u . grad) u of the velocity field (F_U), fp64 output
template <int LX, typename TM, typename C>
__global__ void __launch_bounds__(Dl<LX>::NT) conv_dealias_kernel(Batch bt)
{
    constexpr int LXD = Dl<LX>::LXD, N3 = Dl<LX>::N3, ND3 = Dl<LX>::ND3, NT = Dl<LX>::NT, NQ = Dl<LX>::NQ;
    __shared__ C sI[LXD * LX], sID[LXD * LX];
    __shared__ C su[3][N3];
    __shared__ C F[ND3];
    __shared__ C tA[Dl<LX>::NA], tB[Dl<LX>::NB];
    const int g = blockIdx.x;
    const int ri = find_req(bt.eb, bt.n, g);
    const ReqDesc* R = bt.r[ri];
    const int blk = g - bt.eb[ri];
    const int t = threadIdx.x;
    if constexpr (sizeof(C) == 8) {
        const SEM_GLOBAL double* tab = gp(R->D64);
        for (int q = t; q < LXD * LX; q += NT) {
            sI[q] = (C)tab[dl_off64<LX>() + q];
            sID[q] = (C)tab[dl_off64<LX>() + LXD * LX + q];
        }
    } else {
        const SEM_GLOBAL float* tab = gp(R->D32);
        for (int q = t; q < LXD * LX; q += NT) {
            sI[q] = (C)tab[dl_off32<LX>() + q];
            sID[q] = (C)tab[dl_off32<LX>() + LXD * LX + q];
        }
    }
    const SEM_GLOBAL TM* MF = gfield<TM>(R, mfd_field<TM>());
    const SEM_GLOBAL double* U[3];
    SEM_GLOBAL double* O[3];
    for (int c = 0; c < 3; ++c) { U[c] = gfield<double>(R, F_U + c); O[c] = gfieldw<double>(R, F_BN + c); }
    __syncthreads();
    for (int el = 0; el < R->epb; ++el) {
        const int e = blk * R->epb + el;
        if (e >= R->E) break;
        const long long eb = (long long)e * N3;
        for (int p = t; p < N3; p += NT) {
            su[0][p] = (C)U[0][eb + p];
            su[1][p] = (C)U[1][eb + p];
            su[2][p] = (C)U[2][eb + p];
        }
        __syncthreads();
        const SEM_GLOBAL TM* me = MF + (long long)e * 9 * ND3;
        const C msc = mscale<TM, C>(R, e);
        // contravariant velocity V_a = sum_c u_c W dr_a/dx_c at this thread's fine points
        C V[3][NQ];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int r = 0; r < NQ; ++r) V[a][r] = 0;
        for (int c = 0; c < 3; ++c) {
            interp3<LX, C>(sI, sI, sI, su[c], tA, tB, F);
#pragma unroll
            for (int r = 0; r < NQ; ++r) {
                const int q = t + r * NT;
                if (q < ND3) {
                    const C uf = F[q];
#pragma unroll
                    for (int a = 0; a < 3; ++a) V[a][r] += uf * mload<TM, C>(me + (a * 3 + c) * ND3 + q, msc);
                }
            }
            __syncthreads();
        }
        for (int f = 0; f < 3; ++f) {
            C T[NQ];
#pragma unroll
            for (int r = 0; r < NQ; ++r) T[r] = 0;
            for (int a = 0; a < 3; ++a) {
                interp3<LX, C>(a == 0 ? sID : sI, a == 1 ? sID : sI, a == 2 ? sID : sI, su[f], tA, tB, F);
#pragma unroll
                for (int r = 0; r < NQ; ++r) {
                    const int q = t + r * NT;
                    if (q < ND3) T[r] += V[a][r] * F[q];
                }
                __syncthreads();
            }
#pragma unroll
            for (int r = 0; r < NQ; ++r) {
                const int q = t + r * NT;
                if (q < ND3) F[q] = T[r];
            }
            __syncthreads();
            back3_neg<LX, C>(sI, F, tB, tA, O[f] + eb);
        }
    }
}

// ------------------------------------------------------------------
// Matrix-core form (LXD <= 16): every one-dimensional contraction is a small
// dense product with the 1D matrix (I, ID or I^T) as one operand, done with
// the 16x16x4 MFMA of the arithmetic type.  The matrix operands sit in
// registers for the whole kernel (for these shapes the lane layout of the
// A and B operands coincide: lane l holds row/column l % 16, k = l / 16), the
// tensor operand is read from LDS once per stage, and the fine-grid products
// stay in the accumulators, so LDS traffic drops from two reads per FMA to
// about one read and one write per staged value.  Four waves share an
// element; output tiles go round-robin over the waves.
template <typename C> struct Mma;
template <> struct Mma<float> {
    typedef float V4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ V4 mma(float a, float b, V4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    // accumulator entry r of a lane in row group g holds output row:
    static __device__ __forceinline__ int row(int g, int r) { return 4 * g + r; }
};
template <> struct Mma<double> {
    typedef double V4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ V4 mma(double a, double b, V4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    static __device__ __forceinline__ int row(int g, int r) { return g + 4 * r; }
};

template <int LX> struct Dm {
    static constexpr int LXD = (3 * LX + 1) / 2;
    static constexpr int NL = LX * LX, NN = LXD * LXD, N3 = LX * LX * LX, ND3 = LXD * LXD * LXD;
    static constexpr int KSX = (LX + 3) / 4, KSD = (LXD + 3) / 4;   // k-steps over coarse / fine indices
    static constexpr int NLT = (NL + 15) / 16, NNT = (NN + 15) / 16;  // tiles over lines / fine planes
    static constexpr int NW = 4, NT = 64 * NW;
    static constexpr int JW = (NNT + NW - 1) / NW;                  // fine-plane tiles per wave
    static constexpr int cmax(int a, int b) { return a > b ? a : b; }
    static constexpr int R1 = cmax(2 * NL * LXD, ND3);             // Y1 (P, Q) / T / Z2
    static constexpr int R2 = 3 * LX * NN;                          // Y2 (3 kinds) / Z1
};

template <int LX, typename TM, typename C>
__global__ void __launch_bounds__(Dm<LX>::NT) conv_dealias_mfma_kernel(Batch bt)
{
    using D = Dm<LX>;
    using M = Mma<C>;
    typedef typename M::V4 V4;
    constexpr int LXD = D::LXD, NL = D::NL, NN = D::NN, N3 = D::N3, ND3 = D::ND3;
    constexpr int KSX = D::KSX, KSD = D::KSD, NLT = D::NLT, NNT = D::NNT, JW = D::JW;
    static_assert(LXD <= 16, "one 16-row tile over the fine index");
    __shared__ C sU[3 * N3];
    __shared__ C R1[D::R1];
    __shared__ C R2[D::R2];
    const int gb = blockIdx.x;
    const int ri = find_req(bt.eb, bt.n, gb);
    const ReqDesc* R = bt.r[ri];
    const int blk = gb - bt.eb[ri];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, m = lane & 15, g = lane >> 4;
    // 1D matrices in registers: fI/fD[s] = I/ID[m][4s+g] (forward stages), bI[s] = I[4s+g][m] (transposed stages)
    C fI[KSX], fD[KSX], bI[KSD];
    {
        const int o = sizeof(C) == 8 ? dl_off64<LX>() : dl_off32<LX>();
#pragma unroll
        for (int s = 0; s < KSX; ++s) {
            const int k = 4 * s + g;
            const bool ok = m < LXD && k < LX;
            if constexpr (sizeof(C) == 8) {
                fI[s] = ok ? gp(R->D64)[o + m * LX + k] : 0.0;
                fD[s] = ok ? gp(R->D64)[o + LXD * LX + m * LX + k] : 0.0;
            } else {
                fI[s] = ok ? gp(R->D32)[o + m * LX + k] : 0.0f;
                fD[s] = ok ? gp(R->D32)[o + LXD * LX + m * LX + k] : 0.0f;
            }
        }
#pragma unroll
        for (int s = 0; s < KSD; ++s) {
            const int k = 4 * s + g;
            const bool ok = k < LXD && m < LX;
            if constexpr (sizeof(C) == 8) bI[s] = ok ? gp(R->D64)[o + k * LX + m] : 0.0;
            else bI[s] = ok ? gp(R->D32)[o + k * LX + m] : 0.0f;
        }
    }
    const SEM_GLOBAL TM* MF = gfield<TM>(R, mfd_field<TM>());
    const SEM_GLOBAL double* U[3];
    SEM_GLOBAL double* O[3];
    for (int c = 0; c < 3; ++c) { U[c] = gfield<double>(R, F_U + c); O[c] = gfieldw<double>(R, F_BN + c); }
    C* sY1 = R1;            // [2][NL][LXD]: P = I u, Q = ID u along the first index
    C* sT = R1;             // [LXD][NN]: weighted integrand at the fine points
    C* sZ2 = R1;            // [NL][LXD]
    C* sY2 = R2;            // [3][LX][NN]
    C* sZ1 = R2;            // [LX][NN]

    for (int el = 0; el < R->epb; ++el) {
        const int e = blk * R->epb + el;
        if (e >= R->E) break;
        const long long eb = (long long)e * N3;
        for (int p = t; p < 3 * N3; p += D::NT) {
            const int c = p / N3;
            sU[p] = (C)U[c][eb + (p - c * N3)];
        }
        block_sync_lds();
        const SEM_GLOBAL TM* me = MF + (long long)e * 9 * ND3;
        const C msc = mscale<TM, C>(R, e);

        // ---- contravariant velocity V_a = sum_c u_c (W dr_a/dx_c) at this wave's fine points
        V4 V[3][JW];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int j = 0; j < JW; ++j) V[a][j] = V4{0, 0, 0, 0};
        for (int c = 0; c < 3; ++c) {
            // first index: Y1[L][i'] = sum_a u[L][a] I[i'][a]
            for (int lt = w; lt < NLT; lt += 4) {
                V4 acc = {0, 0, 0, 0};
                const int L = 16 * lt + m;
#pragma unroll
                for (int s = 0; s < KSX; ++s) {
                    const int a = 4 * s + g;
                    const C av = (L < NL && a < LX) ? sU[c * N3 + L * LX + a] : (C)0;
                    acc = M::mma(av, fI[s], acc);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int Lo = 16 * lt + M::row(g, r);
                    if (Lo < NL && m < LXD) sY1[Lo * LXD + m] = acc[r];
                }
            }
            block_sync_lds();
            // second index, per third-index plane cc: Y2[cc][j'][i'] = sum_b I[j'][b] Y1[cc LX + b][i']
            for (int cc = w; cc < LX; cc += 4) {
                V4 acc = {0, 0, 0, 0};
#pragma unroll
                for (int s = 0; s < KSX; ++s) {
                    const int b = 4 * s + g;
                    const C bv = (b < LX && m < LXD) ? sY1[(cc * LX + b) * LXD + m] : (C)0;
                    acc = M::mma(fI[s], bv, acc);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int jo = M::row(g, r);
                    if (jo < LXD && m < LXD) sY2[cc * NN + jo * LXD + m] = acc[r];
                }
            }
            block_sync_lds();
            // third index: u_c(k', n) = sum_cc I[k'][cc] Y2[cc][n], straight into V
#pragma unroll
            for (int j = 0; j < JW; ++j) {
                const int tn = w + 4 * j;
                if (tn < NNT) {
                    const int n = 16 * tn + m;
                    V4 acc = {0, 0, 0, 0};
#pragma unroll
                    for (int s = 0; s < KSX; ++s) {
                        const int cc = 4 * s + g;
                        const C bv = (cc < LX && n < NN) ? sY2[cc * NN + n] : (C)0;
                        acc = M::mma(fI[s], bv, acc);
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int kk = M::row(g, r);
                        if (n < NN && kk < LXD) {
#pragma unroll
                            for (int a = 0; a < 3; ++a) V[a][j][r] += acc[r] * mload<TM, C>(me + (a * 3 + c) * ND3 + kk * NN + n, msc);
                        }
                    }
                }
            }
        }

        // ---- per component: T = sum_a V_a d_a u_f at the fine points, tested back on the GLL points
        for (int f = 0; f < 3; ++f) {
            block_sync_lds();
            // first index: P = I u_f, Q = ID u_f
            for (int job = w; job < 2 * NLT; job += 4) {
                const int which = job / NLT, lt = job - which * NLT;
                const int L = 16 * lt + m;
                V4 acc = {0, 0, 0, 0};
#pragma unroll
                for (int s = 0; s < KSX; ++s) {
                    const int a = 4 * s + g;
                    const C av = (L < NL && a < LX) ? sU[f * N3 + L * LX + a] : (C)0;
                    acc = M::mma(av, which ? fD[s] : fI[s], acc);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int Lo = 16 * lt + M::row(g, r);
                    if (Lo < NL && m < LXD) sY1[which * NL * LXD + Lo * LXD + m] = acc[r];
                }
            }
            block_sync_lds();
            // second index: kind 0: I P (for d/dt), 1: ID P (d/ds), 2: I Q (d/dr)
            for (int job = w; job < 3 * LX; job += 4) {
                const int kind = job / LX, cc = job - kind * LX;
                const C* src = sY1 + (kind == 2 ? NL * LXD : 0);
                V4 acc = {0, 0, 0, 0};
#pragma unroll
                for (int s = 0; s < KSX; ++s) {
                    const int b = 4 * s + g;
                    const C bv = (b < LX && m < LXD) ? src[(cc * LX + b) * LXD + m] : (C)0;
                    acc = M::mma(kind == 1 ? fD[s] : fI[s], bv, acc);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int jo = M::row(g, r);
                    if (jo < LXD && m < LXD) sY2[kind * LX * NN + cc * NN + jo * LXD + m] = acc[r];
                }
            }
            block_sync_lds();
            // third index: d/dt = ID (I P), d/ds = I (ID P), d/dr = I (I Q); T accumulated in registers
#pragma unroll
            for (int j = 0; j < JW; ++j) {
                const int tn = w + 4 * j;
                if (tn < NNT) {
                    const int n = 16 * tn + m;
                    V4 T = {0, 0, 0, 0};
#pragma unroll
                    for (int kind = 0; kind < 3; ++kind) {
                        V4 acc = {0, 0, 0, 0};
#pragma unroll
                        for (int s = 0; s < KSX; ++s) {
                            const int cc = 4 * s + g;
                            const C bv = (cc < LX && n < NN) ? sY2[kind * LX * NN + cc * NN + n] : (C)0;
                            acc = M::mma(kind == 0 ? fD[s] : fI[s], bv, acc);
                        }
                        const int a = 2 - kind;
#pragma unroll
                        for (int r = 0; r < 4; ++r) T[r] += V[a][j][r] * acc[r];
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int kk = M::row(g, r);
                        if (kk < LXD && n < NN) sT[kk * NN + n] = T[r];
                    }
                }
            }
            block_sync_lds();
            // transposed third index: Z1[c][n] = sum_k' I[k'][c] T[k'][n]
            for (int tn = w; tn < NNT; tn += 4) {
                const int n = 16 * tn + m;
                V4 acc = {0, 0, 0, 0};
#pragma unroll
                for (int s = 0; s < KSD; ++s) {
                    const int kk = 4 * s + g;
                    const C bv = (kk < LXD && n < NN) ? sT[kk * NN + n] : (C)0;
                    acc = M::mma(bI[s], bv, acc);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int c = M::row(g, r);
                    if (c < LX && n < NN) sZ1[c * NN + n] = acc[r];
                }
            }
            block_sync_lds();
            // transposed second index, per plane c: Z2[c][b][i'] = sum_j' I[j'][b] Z1[c][j'][i']
            for (int c = w; c < LX; c += 4) {
                V4 acc = {0, 0, 0, 0};
#pragma unroll
                for (int s = 0; s < KSD; ++s) {
                    const int jj = 4 * s + g;
                    const C bv = (jj < LXD && m < LXD) ? sZ1[c * NN + jj * LXD + m] : (C)0;
                    acc = M::mma(bI[s], bv, acc);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int b = M::row(g, r);
                    if (b < LX && m < LXD) sZ2[(c * LX + b) * LXD + m] = acc[r];
                }
            }
            block_sync_lds();
            // transposed first index: BN_f[L][a] = -sum_i' Z2[L][i'] I[i'][a]
            for (int lt = w; lt < NLT; lt += 4) {
                const int L = 16 * lt + m;
                V4 acc = {0, 0, 0, 0};
#pragma unroll
                for (int s = 0; s < KSD; ++s) {
                    const int ii = 4 * s + g;
                    const C av = (L < NL && ii < LXD) ? sZ2[L * LXD + ii] : (C)0;
                    acc = M::mma(av, bI[s], acc);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int Lo = 16 * lt + M::row(g, r);
                    if (Lo < NL && m < LX) O[f][eb + Lo * LX + m] = -(double)acc[r];
                }
            }
        }
    }
}

// Single-pass matrix-core form: the three components go through every
// stage together, so an element takes seven workgroup barriers.  About one
// wave per 16-point tile of a fine-grid plane keeps the heaviest stage
// (velocity, contravariant velocity and the three derivatives of each
// component on the fine points) nearly balanced; the smaller stages
// distribute their tiles round-robin.  Operand reads carry no bounds tests:
// every 1D-matrix register is zero outside its index range, and every LDS
// region is zero-filled at the start with a pad behind it, so out-of-range
// lanes read finite values that either meet a zero matrix entry or land in
// output rows/columns that are never stored.  Stores of partial tiles write
// their unused lanes to a scratch slot instead of branching.
template <int LX, typename C> struct Dv2 {
    using D = Dm<LX>;
    static constexpr int LXD = D::LXD, NL = D::NL, NN = D::NN, N3 = D::N3, ND3 = D::ND3;
    // waves: one per fine tile, rounded down to a multiple of four so that
    // two workgroups place evenly on the four SIMDs of a CU
    static constexpr int NW = D::NNT <= 4 ? D::NNT : (D::NNT / 4) * 4, NT = 64 * NW;
    static constexpr int PAD = 4 * NN + 64;
    static constexpr int cmax(int a, int b) { return a > b ? a : b; }
    // region X: u (3 N3) + Y1 (6 NL LXD) | T (3 LXD^3) | Z2 (3 NL LXD); region Y: Y2 (9 LX NN) | Z1 (3 LX NN)
    static constexpr int X = cmax(cmax(3 * N3 + 6 * NL * LXD, 3 * ND3), 3 * NL * LXD) + PAD;
    static constexpr int Y = 9 * LX * NN + PAD;
    static constexpr int DUMMY = X + Y;          // 64 scratch slots for unused lanes of partial tiles
    static constexpr int TOTAL = X + Y + 64;
    static constexpr bool fits = TOTAL * (int)sizeof(C) <= 160 * 1024 && LXD <= 16 && NW <= 16;
    // workgroups per CU that the LDS allows (at most 2), and the waves per SIMD
    // the register allocation must leave room for so that they are co-resident
    // (a workgroup's waves go round-robin over the four SIMDs, so a SIMD may
    // hold ceil(NW/4) waves of each)
    static constexpr int WG = TOTAL * (int)sizeof(C) * 2 <= 160 * 1024 ? 2 : 1;
    static constexpr int WPE = WG * ((NW + 3) / 4);
    static constexpr int NUP = (N3 + NT - 1) / NT;   // velocity points per thread
};

template <int LX, typename TM, typename C>
__global__ void __launch_bounds__((Dv2<LX, C>::NT), (Dv2<LX, C>::WPE)) conv_dealias_v2_kernel(Batch bt)
{
    using D = Dm<LX>;
    using Q = Dv2<LX, C>;
    using M = Mma<C>;
    typedef typename M::V4 V4;
    constexpr int LXD = D::LXD, NL = D::NL, NN = D::NN, N3 = D::N3, ND3 = D::ND3;
    constexpr int KSX = D::KSX, KSD = D::KSD, NLT = D::NLT, NNT = D::NNT, NW = Q::NW;
    static_assert(Q::fits, "LDS footprint");
    __shared__ C lds[Q::TOTAL];
    C* const sU = lds;                       // [3][N3]
    C* const sY1 = lds + 3 * N3;             // [3][2][NL][LXD]: P = I u, Q = ID u along the first index
    C* const sT = lds;                       // [3][LXD^3]
    C* const sZ2 = lds;                      // [3][NL][LXD]
    C* const sY2 = lds + Q::X;               // [3][3][LX][NN]: I P, ID P, I Q along the second index
    C* const sZ1 = lds + Q::X;               // [3][LX][NN]
    const int gb = blockIdx.x;
    const int ri = find_req(bt.eb, bt.n, gb);
    const ReqDesc* R = bt.r[ri];
    const int blk = gb - bt.eb[ri];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, m = lane & 15, g = lane >> 4;
    const int dummy = Q::DUMMY + lane;
    for (int p = t; p < Q::TOTAL; p += Q::NT) lds[p] = (C)0;
    C fI[KSX], fD[KSX], bI[KSD];
    {
        const int o = sizeof(C) == 8 ? dl_off64<LX>() : dl_off32<LX>();
#pragma unroll
        for (int s = 0; s < KSX; ++s) {
            const int k = 4 * s + g;
            const bool ok = m < LXD && k < LX;
            if constexpr (sizeof(C) == 8) {
                fI[s] = ok ? gp(R->D64)[o + m * LX + k] : 0.0;
                fD[s] = ok ? gp(R->D64)[o + LXD * LX + m * LX + k] : 0.0;
            } else {
                fI[s] = ok ? gp(R->D32)[o + m * LX + k] : 0.0f;
                fD[s] = ok ? gp(R->D32)[o + LXD * LX + m * LX + k] : 0.0f;
            }
        }
#pragma unroll
        for (int s = 0; s < KSD; ++s) {
            const int k = 4 * s + g;
            const bool ok = k < LXD && m < LX;
            if constexpr (sizeof(C) == 8) bI[s] = ok ? gp(R->D64)[o + k * LX + m] : 0.0;
            else bI[s] = ok ? gp(R->D32)[o + k * LX + m] : 0.0f;
        }
    }
    const SEM_GLOBAL TM* MF = gfield<TM>(R, mfd_field<TM>());
    const SEM_GLOBAL double* U0 = gfield<double>(R, F_U);
    const SEM_GLOBAL double* U1 = gfield<double>(R, F_U1);
    const SEM_GLOBAL double* U2 = gfield<double>(R, F_U2);
    SEM_GLOBAL double* O0 = gfieldw<double>(R, F_BN);
    SEM_GLOBAL double* O1 = gfieldw<double>(R, F_BNb);
    SEM_GLOBAL double* O2 = gfieldw<double>(R, F_BNc);

    // the velocity of the next element is loaded while the current one is processed
    constexpr int NUP = Q::NUP;
    double un[3][NUP];
    auto load_u = [&](int e) {
        const long long eb = (long long)e * N3;
#pragma unroll
        for (int q = 0; q < NUP; ++q) {
            const int p = t + q * Q::NT;
            const int pc = p < N3 ? p : N3 - 1;
            un[0][q] = U0[eb + pc];
            un[1][q] = U1[eb + pc];
            un[2][q] = U2[eb + pc];
        }
    };
    const int e0 = blk * R->epb;
    if (e0 < R->E) load_u(e0);
    for (int el = 0; el < R->epb; ++el) {
        const int e = blk * R->epb + el;
        if (e >= R->E) break;
        const long long eb = (long long)e * N3;
        block_sync_lds();  // the previous element's last stage has read region X
#pragma unroll
        for (int q = 0; q < NUP; ++q) {
            const int p = t + q * Q::NT;
            if (p < N3) {
                sU[p] = (C)un[0][q];
                sU[N3 + p] = (C)un[1][q];
                sU[2 * N3 + p] = (C)un[2][q];
            }
        }
        if (el + 1 < R->epb && e + 1 < R->E) load_u(e + 1);
        block_sync_lds();
        // S1, first index: Y1[c][mat][L][i'] = sum_a u_c[L][a] mat[i'][a]
        for (int job = w; job < 6 * NLT; job += NW) {
            const int cm = job / NLT, lt = job - cm * NLT;
            const int c = cm >> 1, mat = cm & 1;
            const C* src = sU + c * N3 + (16 * lt + m) * LX + g;
            V4 acc = {0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < KSX; ++s) acc = M::mma(src[4 * s], mat ? fD[s] : fI[s], acc);
            C* dst = sY1 + cm * NL * LXD;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int L = 16 * lt + M::row(g, r);
                lds[(L < NL && m < LXD) ? (int)(dst - lds) + L * LXD + m : dummy] = acc[r];
            }
        }
        block_sync_lds();
        // S2, second index per plane cc: kind 0 I P, 1 ID P, 2 I Q
        for (int job = w; job < 9 * LX; job += NW) {
            const int ck = job / LX, cc = job - ck * LX;
            const int c = ck / 3, kind = ck - 3 * c;
            const C* src = sY1 + (2 * c + (kind == 2)) * NL * LXD + (cc * LX + g) * LXD + m;
            V4 acc = {0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < KSX; ++s) acc = M::mma(kind == 1 ? fD[s] : fI[s], src[4 * s * LXD], acc);
            const int base = (int)(sY2 - lds) + ck * LX * NN + cc * NN;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int jo = M::row(g, r);
                lds[(jo < LXD && m < LXD) ? base + jo * LXD + m : dummy] = acc[r];
            }
        }
        block_sync_lds();
        // S3, third index, one fine tile per wave: u_c, V_a = sum_c u_c W dr_a/dx_c,
        // then T_f = V_r d_r u_f + V_s d_s u_f + V_t d_t u_f
        const SEM_GLOBAL TM* me = MF + (long long)e * 9 * ND3;
        const C msc = mscale<TM, C>(R, e);
        for (int tn = w; tn < NNT; tn += NW) {
            const int n = 16 * tn + m;
            int qoff[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int kk = M::row(g, r);
                qoff[r] = (kk < LXD ? kk : LXD - 1) * NN + (n < NN ? n : NN - 1);
            }
            C mf[9][4];
            if constexpr (sizeof(TM) == 2) {
                // lane-ordered 16-bit terms: four rows of one term in one 8-byte load
                static_assert(dl16_lane(LX), "lane-ordered 16-bit metric layout");
                constexpr int NG = (LXD + 3) / 4;
                const SEM_GLOBAL TM* m16 = MF + (long long)e * dl16_per_elem(LX) + (long long)tn * 9 * NG * 64;
                // row groups past the fine grid (g >= NG) read the last group
                // instead: unconditional loads, and those rows are never stored
                const int gg = g < NG ? g : NG - 1;
                unsigned long long raw[9];
#pragma unroll
                for (int ac = 0; ac < 9; ++ac)
                    raw[ac] = *(const SEM_GLOBAL unsigned long long*)(m16 + (ac * NG + gg) * 64 + m * 4);
#pragma unroll
                for (int ac = 0; ac < 9; ++ac)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const unsigned short hb = (unsigned short)((raw[ac] >> (16 * r)) & 0xffff);
                        TM hv;
                        __builtin_memcpy(&hv, &hb, 2);
                        mf[ac][r] = to<C>(hv) * msc;
                    }
            } else {
#pragma unroll
                for (int ac = 0; ac < 9; ++ac)
#pragma unroll
                    for (int r = 0; r < 4; ++r) mf[ac][r] = mload<TM, C>(me + ac * ND3 + qoff[r], msc);
            }
            const C* y2 = sY2 + g * NN + n;
            V4 V[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) V[a] = V4{0, 0, 0, 0};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                V4 uc = {0, 0, 0, 0};
#pragma unroll
                for (int s = 0; s < KSX; ++s) uc = M::mma(fI[s], y2[(3 * c) * LX * NN + 4 * s * NN], uc);
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int r = 0; r < 4; ++r) V[a][r] += uc[r] * mf[a * 3 + c][r];
            }
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                V4 dt = {0, 0, 0, 0}, ds = {0, 0, 0, 0}, dr = {0, 0, 0, 0};
#pragma unroll
                for (int s = 0; s < KSX; ++s) {
                    dt = M::mma(fD[s], y2[(3 * f + 0) * LX * NN + 4 * s * NN], dt);
                    ds = M::mma(fI[s], y2[(3 * f + 1) * LX * NN + 4 * s * NN], ds);
                    dr = M::mma(fI[s], y2[(3 * f + 2) * LX * NN + 4 * s * NN], dr);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int kk = M::row(g, r);
                    const C T = V[0][r] * dr[r] + V[1][r] * ds[r] + V[2][r] * dt[r];
                    lds[(kk < LXD && n < NN) ? (int)(sT - lds) + f * ND3 + kk * NN + n : dummy] = T;
                }
            }
        }
        block_sync_lds();
        // B1, transposed third index: Z1[f][c][n] = sum_k' I[k'][c] T_f[k'][n]
        for (int job = w; job < 3 * NNT; job += NW) {
            const int f = job / NNT, tn = job - f * NNT;
            const int n = 16 * tn + m;
            const C* src = sT + f * ND3 + g * NN + n;
            V4 acc = {0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < KSD; ++s) acc = M::mma(bI[s], src[4 * s * NN], acc);
            const int base = (int)(sZ1 - lds) + f * LX * NN;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c = M::row(g, r);
                lds[(c < LX && n < NN) ? base + c * NN + n : dummy] = acc[r];
            }
        }
        block_sync_lds();
        // B2, transposed second index per plane c: Z2[f][c LX + b][i'] = sum_j' I[j'][b] Z1[f][c][j'][i']
        for (int job = w; job < 3 * LX; job += NW) {
            const int f = job / LX, c = job - f * LX;
            const C* src = sZ1 + f * LX * NN + c * NN + g * LXD + m;
            V4 acc = {0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < KSD; ++s) acc = M::mma(bI[s], src[4 * s * LXD], acc);
            const int base = (int)(sZ2 - lds) + f * NL * LXD + c * LX * LXD;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int b = M::row(g, r);
                lds[(b < LX && m < LXD) ? base + b * LXD + m : dummy] = acc[r];
            }
        }
        block_sync_lds();
        // B3, transposed first index: BN_f[L][a] = -sum_i' Z2[f][L][i'] I[i'][a]
        for (int job = w; job < 3 * NLT; job += NW) {
            const int f = job / NLT, lt = job - f * NLT;
            const C* src = sZ2 + f * NL * LXD + (16 * lt + m) * LXD + g;
            V4 acc = {0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < KSD; ++s) acc = M::mma(src[4 * s], bI[s], acc);
            SEM_GLOBAL double* O = f == 0 ? O0 : f == 1 ? O1 : O2;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int L = 16 * lt + M::row(g, r);
                if (L < NL && m < LX) O[eb + L * LX + m] = -(double)acc[r];
            }
        }
    }
}

#define DL_LX_SWITCH(lx, CALL) \
    switch (lx) { \
    case 3: CALL(3); break; case 4: CALL(4); break; case 5: CALL(5); break; case 6: CALL(6); break; \
    case 7: CALL(7); break; case 8: CALL(8); break; case 9: CALL(9); break; case 10: CALL(10); break; \
    case 11: CALL(11); break; case 12: CALL(12); break; default: break; }

void launch_dealias_geom(const Batch& b, int lx, const MeshParams& mp, int want32, int want16, hipStream_t s)
{
    if (b.eb[b.n] == 0) return;
#define GO(L) hipLaunchKernelGGL(dealias_geom_kernel<L>, dim3(b.eb[b.n]), dim3(Dl<L>::NT), 0, s, b, mp)
    DL_LX_SWITCH(lx, GO)
#undef GO
    if (want32 || want16) {
        const int nd = (3 * lx + 1) / 2;
        const int per = 9 * nd * nd * nd;
        if (want16 == PBF)
            hipLaunchKernelGGL(dealias_cast_kernel<__hip_bfloat16>, dim3(b.eb[b.n]), dim3(256), 0, s, b, per, want32, 1);
        else
            hipLaunchKernelGGL(dealias_cast_kernel<__half>, dim3(b.eb[b.n]), dim3(256), 0, s, b, per, want32,
                               want16 == P16 ? 1 : 0);
    }
}

// metric storage tm and arithmetic tc (tables in the arithmetic precision):
// (fp64, fp64), (fp32, fp64), (fp32, fp32) or (fp16/bf16, fp32)
void launch_conv_dealias(const Batch& b, int lx, int tm, int tc, hipStream_t s)
{
    if (b.eb[b.n] == 0) return;
    // matrix-core form while the fine grid fits one 16-row tile (lx <= 10)
#define GO3(L, TM, C)                                                                                                  \
    do {                                                                                                               \
        if constexpr (Dv2<L, C>::fits)                                                                                 \
            hipLaunchKernelGGL((conv_dealias_v2_kernel<L, TM, C>), dim3(b.eb[b.n]), dim3((Dv2<L, C>::NT)), 0, s, b);  \
        else if constexpr ((3 * L + 1) / 2 <= 16)                                                                      \
            hipLaunchKernelGGL((conv_dealias_mfma_kernel<L, TM, C>), dim3(b.eb[b.n]), dim3(Dm<L>::NT), 0, s, b);      \
        else                                                                                                           \
            hipLaunchKernelGGL((conv_dealias_kernel<L, TM, C>), dim3(b.eb[b.n]), dim3(Dl<L>::NT), 0, s, b);           \
    } while (0)
    if (tm == P64) {
#define GO(L) GO3(L, double, double)
        DL_LX_SWITCH(lx, GO)
#undef GO
    } else if (tm == P16) {
#define GO(L) GO3(L, __half, float)
        DL_LX_SWITCH(lx, GO)
#undef GO
    } else if (tm == PBF) {
#define GO(L) GO3(L, __hip_bfloat16, float)
        DL_LX_SWITCH(lx, GO)
#undef GO
    } else if (tc == P64) {
#define GO(L) GO3(L, float, double)
        DL_LX_SWITCH(lx, GO)
#undef GO
    } else {
#define GO(L) GO3(L, float, float)
        DL_LX_SWITCH(lx, GO)
#undef GO
    }
#undef GO3
}

}  // namespace semk
