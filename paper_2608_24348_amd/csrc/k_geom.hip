// Setup kernels: node coordinates, geometric factors, Jacobi diagonal,
// reduced-precision geometry copies and the Taylor-Green initial fields.
// All of it runs once per request in FP64.
#include "k_common.h"

namespace semk {

// one element per workgroup; coordinates staged in LDS
template <int LX>
__global__ void __launch_bounds__(256) geometry_kernel(Batch bt, MeshParams mp)
{
    constexpr int L3 = LX * LX * LX;
    __shared__ double sx[3][L3];
    __shared__ double sD[LX * LX];
    __shared__ double sxi[LX];
    const int g = blockIdx.x;
    const int ri = find_req(bt.eb, bt.n, g);
    const ReqDesc* R = bt.r[ri];
    const int blk = g - bt.eb[ri];
    double* G = (double*)R->f[F_G64];
    double* B = (double*)R->f[F_B64];
    double* M = (double*)R->f[F_M64];
    for (int q = threadIdx.x; q < LX * LX; q += blockDim.x) sD[q] = R->D64[q];
    for (int q = threadIdx.x; q < LX; q += blockDim.x) sxi[q] = R->D64[LX * LX + LX + q];
    __syncthreads();
    for (int el = 0; el < R->epb; ++el) {
        const int e = blk * R->epb + el;
        if (e >= R->E) break;
        for (int q = threadIdx.x; q < L3; q += blockDim.x) {
            int i = q % LX, j = (q / LX) % LX, k = q / (LX * LX);
            double xo[3];
            node_xyz(mp, sxi, e, i, j, k, xo);
            sx[0][q] = xo[0]; sx[1][q] = xo[1]; sx[2][q] = xo[2];
        }
        __syncthreads();
        const double* wq = R->D64 + LX * LX;
        for (int q = threadIdx.x; q < L3; q += blockDim.x) {
            int i = q % LX, j = (q / LX) % LX, k = q / (LX * LX);
            double J[3][3];  // J[c][a] = dx_c/dr_a
            for (int c = 0; c < 3; ++c) {
                double a0 = 0, a1 = 0, a2 = 0;
                for (int l = 0; l < LX; ++l) {
                    a0 += sD[i * LX + l] * sx[c][l + LX * (j + LX * k)];
                    a1 += sD[j * LX + l] * sx[c][i + LX * (l + LX * k)];
                    a2 += sD[k * LX + l] * sx[c][i + LX * (j + LX * l)];
                }
                J[c][0] = a0; J[c][1] = a1; J[c][2] = a2;
            }
            const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
            const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
            const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
            const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
            const double id = 1.0 / det;
            double inv[3][3];  // inv[a][c] = dr_a/dx_c
            inv[0][0] = c00 * id;
            inv[1][0] = c01 * id;
            inv[2][0] = c02 * id;
            inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
            inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
            inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
            inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
            inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
            inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
            const double bm = det * wq[i] * wq[j] * wq[k];
            if (!(det > 0.0)) R->I[I_NAN] = 1;
            const long long p = (long long)e * L3 + q;
            B[p] = bm;
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 3; ++c) M[((long long)e * 9 + a * 3 + c) * L3 + q] = bm * inv[a][c];
            const int ga[6] = {0, 0, 0, 1, 1, 2}, gb[6] = {0, 1, 2, 1, 2, 2};
            for (int s = 0; s < 6; ++s) {
                double v = inv[ga[s]][0] * inv[gb[s]][0] + inv[ga[s]][1] * inv[gb[s]][1] + inv[ga[s]][2] * inv[gb[s]][2];
                G[((long long)e * 6 + s) * L3 + q] = bm * v;
            }
        }
        __syncthreads();
    }
}

// local diagonal of the stiffness operator A_L (h1 = 1, h2 = 0): the G_rr,
// G_ss, G_tt line sums plus the cross terms that survive where D has a
// non-zero diagonal (element end nodes); written to F_DA64 before assembly.
template <int LX>
__global__ void __launch_bounds__(256) diag_a_kernel(Batch bt)
{
    constexpr int L3 = LX * LX * LX;
    __shared__ double sD[LX * LX];
    const int g = blockIdx.x;
    const int ri = find_req(bt.eb, bt.n, g);
    const ReqDesc* R = bt.r[ri];
    const int blk = g - bt.eb[ri];
    const double* G = (const double*)R->f[F_G64];
    double* d = (double*)R->f[F_DA64];
    for (int q = threadIdx.x; q < LX * LX; q += blockDim.x) sD[q] = R->D64[q];
    __syncthreads();
    for (int el = 0; el < R->epb; ++el) {
        const int e = blk * R->epb + el;
        if (e >= R->E) break;
        const double* Ge = G + (long long)e * 6 * L3;
        for (int q = threadIdx.x; q < L3; q += blockDim.x) {
            int i = q % LX, j = (q / LX) % LX, k = q / (LX * LX);
            double s = 0;
            for (int l = 0; l < LX; ++l) {
                s += sD[l * LX + i] * sD[l * LX + i] * Ge[0 * L3 + l + LX * (j + LX * k)];
                s += sD[l * LX + j] * sD[l * LX + j] * Ge[3 * L3 + i + LX * (l + LX * k)];
                s += sD[l * LX + k] * sD[l * LX + k] * Ge[5 * L3 + i + LX * (j + LX * l)];
            }
            const double dii = sD[i * LX + i], djj = sD[j * LX + j], dkk = sD[k * LX + k];
            s += 2.0 * dii * djj * Ge[1 * L3 + q];
            s += 2.0 * dii * dkk * Ge[2 * L3 + q];
            s += 2.0 * djj * dkk * Ge[4 * L3 + q];
            d[(long long)e * L3 + q] = s;
        }
    }
}

// after assembly: 1/Bsum in place, pressure Jacobi 1/dA (and its fp32 copy)
__global__ void __launch_bounds__(256) geo_post_kernel(Batch bt)
{
    const int g = blockIdx.x;
    const int ri = find_req(bt.eb, bt.n, g);
    const ReqDesc* R = bt.r[ri];
    const int blk = g - bt.eb[ri];
    const long long L3 = (long long)R->lx * R->lx * R->lx;
    const long long p0 = (long long)blk * R->epb * L3;
    const long long p1 = min((long long)(blk + 1) * R->epb * L3, R->np);
    double* ib = (double*)R->f[F_IBSUM64];
    const double* da = (const double*)R->f[F_DA64];
    double* idp = (double*)R->f[F_IDP64];
    float* idp32 = (float*)R->f[F_IDP32];
    for (long long p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
        ib[p] = 1.0 / ib[p];
        const double v = da[p] > 0.0 ? 1.0 / da[p] : 0.0;
        idp[p] = v;
        if (idp32) idp32[p] = (float)v;
    }
}

// fp32 copies and element-scaled 16-bit copies of G, B, M (rounded once from fp64)
template <int LX, typename T16>
__global__ void __launch_bounds__(256) geo_cast_kernel(Batch bt, int want32, int want16)
{
    constexpr int L3 = LX * LX * LX;
    __shared__ double red[4 * 3];
    const int g = blockIdx.x;
    const int ri = find_req(bt.eb, bt.n, g);
    const ReqDesc* R = bt.r[ri];
    const int blk = g - bt.eb[ri];
    const double* G = (const double*)R->f[F_G64];
    const double* B = (const double*)R->f[F_B64];
    const double* M = (const double*)R->f[F_M64];
    for (int el = 0; el < R->epb; ++el) {
        const int e = blk * R->epb + el;
        if (e >= R->E) break;
        if (want32) {
            float* G32 = (float*)R->f[F_G32];
            float* B32 = (float*)R->f[F_B32];
            float* M32 = (float*)R->f[F_M32];
            for (int q = threadIdx.x; q < 6 * L3; q += blockDim.x) G32[(long long)e * 6 * L3 + q] = (float)G[(long long)e * 6 * L3 + q];
            for (int q = threadIdx.x; q < 9 * L3; q += blockDim.x) M32[(long long)e * 9 * L3 + q] = (float)M[(long long)e * 9 * L3 + q];
            for (int q = threadIdx.x; q < L3; q += blockDim.x) B32[(long long)e * L3 + q] = (float)B[(long long)e * L3 + q];
        }
        if (want16) {
            double mg = 0, mb = 0, mm = 0;
            for (int q = threadIdx.x; q < 6 * L3; q += blockDim.x) mg = fmax(mg, fabs(G[(long long)e * 6 * L3 + q]));
            for (int q = threadIdx.x; q < 9 * L3; q += blockDim.x) mm = fmax(mm, fabs(M[(long long)e * 9 * L3 + q]));
            for (int q = threadIdx.x; q < L3; q += blockDim.x) mb = fmax(mb, fabs(B[(long long)e * L3 + q]));
            mg = wave_max(mg); mb = wave_max(mb); mm = wave_max(mm);
            const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
            if (lane == 0) { red[wid * 3 + 0] = mg; red[wid * 3 + 1] = mb; red[wid * 3 + 2] = mm; }
            __syncthreads();
            mg = fmax(fmax(red[0], red[3]), fmax(red[6], red[9]));
            mb = fmax(fmax(red[1], red[4]), fmax(red[7], red[10]));
            mm = fmax(fmax(red[2], red[5]), fmax(red[8], red[11]));
            __syncthreads();
            // power-of-two scales keep the 16-bit rounding a single rounding from fp64
            const double sg = mg > 0 ? exp2(ceil(log2(mg))) : 1.0;
            const double sb = mb > 0 ? exp2(ceil(log2(mb))) : 1.0;
            const double sm = mm > 0 ? exp2(ceil(log2(mm))) : 1.0;
            T16* G16 = (T16*)R->f[F_G16];
            T16* B16 = (T16*)R->f[F_B16];
            T16* M16 = (T16*)R->f[F_M16];
            float* gsc = (float*)R->f[F_GSC];
            float* msc = (float*)R->f[F_MSC];
            if (threadIdx.x == 0) { gsc[e] = (float)sg; gsc[R->E + e] = (float)sb; msc[e] = (float)sm; }
            for (int q = threadIdx.x; q < 6 * L3; q += blockDim.x) G16[(long long)e * 6 * L3 + q] = to<T16>(G[(long long)e * 6 * L3 + q] / sg);
            for (int q = threadIdx.x; q < 9 * L3; q += blockDim.x) M16[(long long)e * 9 * L3 + q] = to<T16>(M[(long long)e * 9 * L3 + q] / sm);
            for (int q = threadIdx.x; q < L3; q += blockDim.x) B16[(long long)e * L3 + q] = to<T16>(B[(long long)e * L3 + q] / sb);
        }
    }
}

// initial condition: 1 = 3D Taylor-Green, 2 = 2D Taylor-Green extruded in z,
// 0 = zero; lags equal the initial state
template <int LX>
__global__ void __launch_bounds__(256) init_kernel(Batch bt, int init, MeshParams mp)
{
    constexpr int L3 = LX * LX * LX;
    __shared__ double sxi[LX];
    const int g = blockIdx.x;
    const int ri = find_req(bt.eb, bt.n, g);
    const ReqDesc* R = bt.r[ri];
    const int blk = g - bt.eb[ri];
    for (int q = threadIdx.x; q < LX; q += blockDim.x) sxi[q] = R->D64[LX * LX + LX + q];
    __syncthreads();
    for (int el = 0; el < R->epb; ++el) {
        const int e = blk * R->epb + el;
        if (e >= R->E) break;
        for (int q = threadIdx.x; q < L3; q += blockDim.x) {
            int i = q % LX, j = (q / LX) % LX, k = q / (LX * LX);
            double X[3];
            node_xyz(mp, sxi, e, i, j, k, X);
            double u = 0, v = 0, w = 0, p = 0;
            if (init == 1) {
                u = sin(X[0]) * cos(X[1]) * cos(X[2]);
                v = -cos(X[0]) * sin(X[1]) * cos(X[2]);
                p = (cos(2 * X[0]) + cos(2 * X[1])) * (cos(2 * X[2]) + 2.0) / 16.0;
            } else if (init == 2) {
                u = sin(X[0]) * cos(X[1]);
                v = -cos(X[0]) * sin(X[1]);
                p = (cos(2 * X[0]) + cos(2 * X[1])) / 4.0;
            }
            const long long pt = (long long)e * L3 + q;
            const double vals[3] = {u, v, w};
            for (int c = 0; c < 3; ++c) {
                ((double*)R->f[F_U + c])[pt] = vals[c];
                ((double*)R->f[F_UL1 + c])[pt] = vals[c];
                ((double*)R->f[F_UL2 + c])[pt] = vals[c];
            }
            ((double*)R->f[F_P])[pt] = p;
        }
    }
}

// node fields for inputs: what = 0,1,2 -> coordinate x_c; 3 -> amp sin x sin y sin z
template <int LX>
__global__ void __launch_bounds__(256) node_field_kernel(Batch bt, MeshParams mp, int what, double amp, double* out)
{
    constexpr int L3 = LX * LX * LX;
    __shared__ double sxi[LX];
    const int g = blockIdx.x;
    const int ri = find_req(bt.eb, bt.n, g);
    const ReqDesc* R = bt.r[ri];
    const int blk = g - bt.eb[ri];
    for (int q = threadIdx.x; q < LX; q += blockDim.x) sxi[q] = R->D64[LX * LX + LX + q];
    __syncthreads();
    for (int el = 0; el < R->epb; ++el) {
        const int e = blk * R->epb + el;
        if (e >= R->E) break;
        for (int q = threadIdx.x; q < L3; q += blockDim.x) {
            int i = q % LX, j = (q / LX) % LX, k = q / (LX * LX);
            double X[3];
            node_xyz(mp, sxi, e, i, j, k, X);
            out[(long long)e * L3 + q] = what < 3 ? X[what] : amp * sin(X[0]) * sin(X[1]) * sin(X[2]);
        }
    }
}

#define SEM_LX_SWITCH(lx, CALL) \
    switch (lx) { \
    case 3: CALL(3); break; case 4: CALL(4); break; case 5: CALL(5); break; case 6: CALL(6); break; \
    case 7: CALL(7); break; case 8: CALL(8); break; case 9: CALL(9); break; case 10: CALL(10); break; \
    case 11: CALL(11); break; case 12: CALL(12); break; default: break; }

void launch_geometry(const Batch& b, int lx, const MeshParams& mp, hipStream_t s)
{
#define GO(L) hipLaunchKernelGGL(geometry_kernel<L>, dim3(b.eb[b.n]), dim3(256), 0, s, b, mp)
    SEM_LX_SWITCH(lx, GO)
#undef GO
}
void launch_diag_a(const Batch& b, int lx, hipStream_t s)
{
#define GO(L) hipLaunchKernelGGL(diag_a_kernel<L>, dim3(b.eb[b.n]), dim3(256), 0, s, b)
    SEM_LX_SWITCH(lx, GO)
#undef GO
}
void launch_geo_post(const Batch& b, hipStream_t s)
{
    hipLaunchKernelGGL(geo_post_kernel, dim3(b.eb[b.n]), dim3(256), 0, s, b);
}
void launch_geo_cast(const Batch& b, int lx, int want32, int want16, hipStream_t s)
{
    if (want16 == PBF) {
#define GO(L) hipLaunchKernelGGL((geo_cast_kernel<L, __hip_bfloat16>), dim3(b.eb[b.n]), dim3(256), 0, s, b, want32, 1)
        SEM_LX_SWITCH(lx, GO)
#undef GO
    } else {
#define GO(L) hipLaunchKernelGGL((geo_cast_kernel<L, __half>), dim3(b.eb[b.n]), dim3(256), 0, s, b, want32, want16 == P16 ? 1 : 0)
        SEM_LX_SWITCH(lx, GO)
#undef GO
    }
}
void launch_node_field(const Batch& b, int lx, const MeshParams& mp, int what, double amp, double* out, hipStream_t s)
{
#define GO(L) hipLaunchKernelGGL(node_field_kernel<L>, dim3(b.eb[b.n]), dim3(256), 0, s, b, mp, what, amp, out)
    SEM_LX_SWITCH(lx, GO)
#undef GO
}
void launch_init_fields(const Batch& b, int lx, int init, const MeshParams& mp, hipStream_t s)
{
#define GO(L) hipLaunchKernelGGL(init_kernel<L>, dim3(b.eb[b.n]), dim3(256), 0, s, b, init, mp)
    SEM_LX_SWITCH(lx, GO)
#undef GO
}

}  // namespace semk
