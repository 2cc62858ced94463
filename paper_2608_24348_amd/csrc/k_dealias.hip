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

// fp32 copy of the fine-grid metric terms
__global__ void __launch_bounds__(256) dealias_cast_kernel(Batch bt, long long per_elem)
{
    const int g = blockIdx.x;
    const int ri = find_req(bt.eb, bt.n, g);
    const ReqDesc* R = bt.r[ri];
    const int blk = g - bt.eb[ri];
    const long long e0 = (long long)blk * R->epb;
    long long e1 = e0 + R->epb;
    if (e1 > R->E) e1 = R->E;
    const SEM_GLOBAL double* src = gfield<double>(R, F_MFD64);
    SEM_GLOBAL float* dst = gfieldw<float>(R, F_MFD32);
    for (long long p = e0 * per_elem + threadIdx.x; p < e1 * per_elem; p += blockDim.x) dst[p] = (float)src[p];
}

template <typename TM> __device__ __forceinline__ int mfd_field() { return F_MFD32; }
template <> __device__ __forceinline__ int mfd_field<double>() { return F_MFD64; }

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
                    for (int a = 0; a < 3; ++a) V[a][r] += uf * (C)me[(a * 3 + c) * ND3 + q];
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

#define DL_LX_SWITCH(lx, CALL) \
    switch (lx) { \
    case 3: CALL(3); break; case 4: CALL(4); break; case 5: CALL(5); break; case 6: CALL(6); break; \
    case 7: CALL(7); break; case 8: CALL(8); break; case 9: CALL(9); break; case 10: CALL(10); break; \
    case 11: CALL(11); break; case 12: CALL(12); break; default: break; }

void launch_dealias_geom(const Batch& b, int lx, const MeshParams& mp, int want32, hipStream_t s)
{
    if (b.eb[b.n] == 0) return;
#define GO(L) hipLaunchKernelGGL(dealias_geom_kernel<L>, dim3(b.eb[b.n]), dim3(Dl<L>::NT), 0, s, b, mp)
    DL_LX_SWITCH(lx, GO)
#undef GO
    if (want32) {
        const long long per = 9LL * ((3 * lx + 1) / 2) * ((3 * lx + 1) / 2) * ((3 * lx + 1) / 2);
        hipLaunchKernelGGL(dealias_cast_kernel, dim3(b.eb[b.n]), dim3(256), 0, s, b, per);
    }
}

// metric storage tm and arithmetic tc (tables in the arithmetic precision):
// (fp64, fp64), (fp32, fp64) or (fp32, fp32)
void launch_conv_dealias(const Batch& b, int lx, int tm, int tc, hipStream_t s)
{
    if (b.eb[b.n] == 0) return;
#define GO3(L, TM, C) hipLaunchKernelGGL((conv_dealias_kernel<L, TM, C>), dim3(b.eb[b.n]), dim3(Dl<L>::NT), 0, s, b)
    if (tm == P64) {
#define GO(L) GO3(L, double, double)
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
