// Three-level hybrid Schwarz multigrid (HSMG) preconditioner of the pressure
// Poisson operator (Sec. 3: the pressure GMRES is preconditioned by a
// three-level HSMG with a coarse-grid solve).  Periodic box of equal
// elements; levels of order N (fine), N/2 (middle) and 1 (coarse):
//
//   M^{-1} r = S_f r + P_fm ( S_m r_m + P_mc A_c^+ R_cm r_m ),  r_m = R_mf r
//
// S_l: additive Schwarz over element subdomains; the local problem is the
// element's separable stiffness, extended by one linear segment to a zero
// Dirichlet node on each side, solved by fast diagonalisation
// (u = S3 diag(1/(lx_i + ly_j + lz_k)) S3^T r); the local solutions of all
// copies of a node are summed and divided by their number.
// P: tensor-product Lagrange interpolation between the levels' GLL points;
// R = P^T in the unique-node inner product (R r = dssum(P_e^T (r / mult))).
// A_c^+: exact solve of the order-1 operator off the constant mode, by fast
// diagonalisation on the nx ny nz corner nodes.
//
// One apply = 8 launches, every one gated per request:
//   hs_down   (fine FDM solve -> F_HSF; fine->middle restriction -> F_HRM)
//   hs_mid    (sum copies of F_HRM; middle FDM -> F_HSM; middle->coarse -> F_HC8)
//   hs_cgath  (coarse rhs on unique corner nodes -> F_HCA)
//   hs_cxy, hs_cz, hs_cxy (coarse S^T along x and y, then z with the
//             eigenvalue scaling and S along z, then S along y and x)
//   hs_midup  (z_m = summed F_HSM / count + trilinear coarse correction -> F_HZM)
//   hs_up     (z = summed F_HSF / count + J3 z_m -> F_HZ and Z_J of F_HZS)
// It runs in the Arnoldi steps only: the cycle end forms x += sum_j y_j Z_j
// from the kept Z_j (M is linear, so this is x += M^{-1} V y).
// The copy sums use index arithmetic on the periodic box in an order shared
// by all copies of a node, so every copy receives the identical value.
#include "k_common.h"

namespace semk {

// the copies of 1D index i of element column ex (n elements, order N):
// (element, index) pairs, left element first
struct Cand {
    int e[2], i[2], n;
};
__device__ __forceinline__ Cand cand(int i, int ex, int n, int N)
{
    Cand c;
    if (i == 0) { c.e[0] = ex == 0 ? n - 1 : ex - 1; c.i[0] = N; c.e[1] = ex; c.i[1] = 0; c.n = 2; }
    else if (i == N) { c.e[0] = ex; c.i[0] = N; c.e[1] = ex + 1 == n ? 0 : ex + 1; c.i[1] = 0; c.n = 2; }
    else { c.e[0] = ex; c.i[0] = i; c.e[1] = ex; c.i[1] = i; c.n = 1; }
    return c;
}

// sum of the copies of node (i,j,k) of element (ex,ey,ez) in the [E][L^3]
// field f (AVG: divided by their number)
template <int L, bool AVG = false>
__device__ __forceinline__ double box_sum(const SEM_GLOBAL double* f, const int* nel, int ex, int ey, int ez,
                                          int i, int j, int k)
{
    constexpr int N = L - 1, L3 = L * L * L;
    const Cand cx = cand(i, ex, nel[0], N), cy = cand(j, ey, nel[1], N), cz = cand(k, ez, nel[2], N);
    double s = 0.0;
    // fixed trip counts keep the candidate arrays in registers
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        if (c >= cz.n) break;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            if (b >= cy.n) break;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                if (a >= cx.n) break;
                const long long e = cx.e[a] + (long long)nel[0] * (cy.e[b] + (long long)nel[1] * cz.e[c]);
                s += f[e * L3 + cx.i[a] + L * (cy.i[b] + L * cz.i[c])];
            }
        }
    }
    return AVG ? s / (double)(cx.n * cy.n * cz.n) : s;
}

__device__ __forceinline__ double inv_mult(int i, int j, int k, int N)
{
    const int m = (i == 0 || i == N ? 2 : 1) * (j == 0 || j == N ? 2 : 1) * (k == 0 || k == N ? 2 : 1);
    return 1.0 / (double)m;
}

// Fast-diagonalisation solve of one element at order L - 1.  Thread (i, j)
// of L*L holds column v[k] of the input and receives the column of the
// solution.  S[c][i*L+k] = component i of eigenvector k, lam[c][k].
// sA, sB: L^3 LDS scratch; one barrier before the first write.
template <int L>
__device__ __forceinline__ void fdm_solve(double (&v)[L], const double* sS, const double* sLam, double* sA,
                                          double* sB, int i, int j)
{
    constexpr int L2 = L * L;
    const double* Sx = sS;
    const double* Sy = sS + L2;
    const double* Sz = sS + 2 * L2;
    double w[L];
    // forward, x: w[k] = sum_a Sx[a][i] v(a, j, k)
    __syncthreads();
#pragma unroll
    for (int k = 0; k < L; ++k) sA[k * L2 + j * L + i] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < L; ++k) {
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < L; ++a) s += Sx[a * L + i] * sA[k * L2 + j * L + a];
        w[k] = s;
    }
    // forward, y
#pragma unroll
    for (int k = 0; k < L; ++k) sB[k * L2 + j * L + i] = w[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < L; ++k) {
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < L; ++b) s += Sy[b * L + j] * sB[k * L2 + b * L + i];
        v[k] = s;
    }
    // forward z, scaling, inverse z (in registers)
    const double lij = sLam[i] + sLam[L + j];
#pragma unroll
    for (int k = 0; k < L; ++k) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < L; ++c) s += Sz[c * L + k] * v[c];
        w[k] = s / (lij + sLam[2 * L + k]);
    }
#pragma unroll
    for (int k = 0; k < L; ++k) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < L; ++c) s += Sz[k * L + c] * w[c];
        v[k] = s;
    }
    // inverse y (sA was last read before the barrier above)
#pragma unroll
    for (int k = 0; k < L; ++k) sA[k * L2 + j * L + i] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < L; ++k) {
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < L; ++b) s += Sy[j * L + b] * sA[k * L2 + b * L + i];
        w[k] = s;
    }
    // inverse x
#pragma unroll
    for (int k = 0; k < L; ++k) sB[k * L2 + j * L + i] = w[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < L; ++k) {
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < L; ++a) s += Sx[i * L + a] * sB[k * L2 + j * L + a];
        v[k] = s;
    }
}

__device__ __forceinline__ void elem_xyz(int e, const int* nel, int& ex, int& ey, int& ez)
{
    ex = e % nel[0];
    const int r = e / nel[0];
    ey = r % nel[1];
    ez = r / nel[1];
}

// ---------------------------------------------------------------- fine level, down
// r = s_J V_J (basis storage TB)
template <int LX, typename TB>
__global__ void __launch_bounds__(LX * LX) hs_down_kernel(Batch bt, int gate)
{
    constexpr int LM = hs_lxm(LX), L2 = LX * LX, L3 = L2 * LX, N = LX - 1;
    __shared__ double sA[L3], sB[L3];
    __shared__ double sS[3 * L2], sLam[3 * LX], sJ[LX * LM];
    const int g = blockIdx.x;
    const int ri = find_req(bt.el, bt.n, g);
    const ReqDesc* R = bt.r[ri];
    const int e = g - bt.el[ri];
    if (!gate_ok(R, gate)) return;
    const int t = threadIdx.x, i = t % LX, j = t / LX;
    const HsOff o = hs_off(LX, R->nel);
    const SEM_GLOBAL double* tb = gfield<double>(R, F_HST);
    for (int q = t; q < 3 * L2; q += L2) sS[q] = tb[o.Sf + q];
    for (int q = t; q < 3 * LX; q += L2) sLam[q] = tb[o.Lf + q];
    for (int q = t; q < LX * LM; q += L2) sJ[q] = tb[o.J + q];

    const long long base = (long long)e * L3;
    double v[LX];
    {
        const int J = gp(R->I)[I_GJ];
        const double sc = gp(R->S)[S_GVS + J];
        const SEM_GLOBAL TB* V = gfield<TB>(R, F_V) + (long long)J * R->np;
#pragma unroll
        for (int k = 0; k < LX; ++k) v[k] = sc * (double)V[base + i + LX * (j + LX * k)];
    }

    // restriction to the middle level: t = J^T J^T J^T (r / mult)
    __syncthreads();
#pragma unroll
    for (int k = 0; k < LX; ++k) sA[k * L2 + j * LX + i] = v[k] * inv_mult(i, j, k, N);
    __syncthreads();
    if (i < LM) {
        // x: sB[k][j][a] = sum_q J[q][a] sA[k][j][q], a = i
#pragma unroll
        for (int k = 0; k < LX; ++k) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < LX; ++q) s += sJ[q * LM + i] * sA[k * L2 + j * LX + q];
            sB[k * L2 + j * LX + i] = s;
        }
    }
    __syncthreads();
    if (i < LM && j < LM) {
        // y then z for output column (a, b) = (i, j)
        double col[LX];
#pragma unroll
        for (int k = 0; k < LX; ++k) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < LX; ++q) s += sJ[q * LM + j] * sB[k * L2 + q * LX + i];
            col[k] = s;
        }
        SEM_GLOBAL double* out = gfieldw<double>(R, F_HRM) + (long long)e * LM * LM * LM;
#pragma unroll
        for (int c = 0; c < LM; ++c) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < LX; ++k) s += sJ[k * LM + c] * col[k];
            out[i + LM * (j + LM * c)] = s;
        }
    }
    // fine local solve
    fdm_solve<LX>(v, sS, sLam, sA, sB, i, j);
    SEM_GLOBAL double* u = gfieldw<double>(R, F_HSF);
#pragma unroll
    for (int k = 0; k < LX; ++k) u[base + i + LX * (j + LX * k)] = v[k];
}

// ---------------------------------------------------------------- middle level, down
// hs_mepb(LM) elements per workgroup (one request per workgroup)
template <int LM>
__global__ void __launch_bounds__(hs_mepb(LM) * LM * LM) hs_mid_kernel(Batch bt, int lx, int gate)
{
    constexpr int L2 = LM * LM, L3 = L2 * LM, N = LM - 1, EP = hs_mepb(LM);
    __shared__ double sA[EP * L3], sB[EP * L3];
    __shared__ double sS[3 * L2], sLam[3 * LM], sJc[2 * LM], sC[EP * 2 * L2];
    const int g = blockIdx.x;
    const int ri = find_req(bt.hm, bt.n, g);
    const ReqDesc* R = bt.r[ri];
    if (!gate_ok(R, gate)) return;
    const int t = threadIdx.x, el = t / L2, ij = t - el * L2, i = ij % LM, j = ij / LM;
    const int e = (g - bt.hm[ri]) * EP + el;
    const bool live = e < R->E;
    const int ee = live ? e : 0;        // lanes past the last element work on element 0 and store nothing
    const HsOff o = hs_off(lx, R->nel);
    const SEM_GLOBAL double* tb = gfield<double>(R, F_HST);
    for (int q = t; q < 3 * L2; q += EP * L2) sS[q] = tb[o.Sm + q];
    for (int q = t; q < 3 * LM; q += EP * L2) sLam[q] = tb[o.Lm + q];
    for (int q = t; q < 2 * LM; q += EP * L2) sJc[q] = tb[o.Jc + q];
    __syncthreads();
    int ex, ey, ez;
    elem_xyz(ee, R->nel, ex, ey, ez);
    const SEM_GLOBAL double* rm = gfield<double>(R, F_HRM);
    double v[LM];
    // the assembled middle residual: sum of the element contributions
#pragma unroll
    for (int k = 0; k < LM; ++k) v[k] = box_sum<LM>(rm, R->nel, ex, ey, ez, i, j, k);
    // coarse restriction of this element: c8 = Jc^T Jc^T Jc^T (r_m / mult)
    {
        double c0 = 0.0, c1 = 0.0;
#pragma unroll
        for (int k = 0; k < LM; ++k) {
            const double x = v[k] * inv_mult(i, j, k, N);
            c0 += sJc[k * 2 + 0] * x;
            c1 += sJc[k * 2 + 1] * x;
        }
        double* C = sC + el * 2 * L2;
        C[0 * L2 + j * LM + i] = c0;
        C[1 * L2 + j * LM + i] = c1;
        __syncthreads();
        if (ij < 8 && live) {
            const int ca = ij & 1, cb = (ij >> 1) & 1, cc = ij >> 2;
            double s = 0.0;
            for (int b = 0; b < LM; ++b)
                for (int a = 0; a < LM; ++a) s += sJc[a * 2 + ca] * sJc[b * 2 + cb] * C[cc * L2 + b * LM + a];
            gfieldw<double>(R, F_HC8)[(long long)e * 8 + ij] = s;
        }
    }
    fdm_solve<LM>(v, sS, sLam, sA + el * L3, sB + el * L3, i, j);
    if (live) {
        SEM_GLOBAL double* u = gfieldw<double>(R, F_HSM) + (long long)e * L3;
#pragma unroll
        for (int k = 0; k < LM; ++k) u[i + LM * (j + LM * k)] = v[k];
    }
}

// ---------------------------------------------------------------- coarse level
// unique corner node q = cx + nx (cy + ny cz) gathers the corner
// contributions of its 8 elements
__global__ void __launch_bounds__(256) hs_cgath_kernel(Batch bt, int gate)
{
    const int ri = blockIdx.y;
    const ReqDesc* R = bt.r[ri];
    if (!gate_ok(R, gate)) return;
    const int nx = R->nel[0], ny = R->nel[1], nz = R->nel[2];
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nx * ny * nz) return;
    const int cx = q % nx, cy = (q / nx) % ny, cz = q / (nx * ny);
    const SEM_GLOBAL double* c8 = gfield<double>(R, F_HC8);
    double s = 0.0;
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                const int ex = (cx - a + nx) % nx, ey = (cy - b + ny) % ny, ez = (cz - c + nz) % nz;
                s += c8[(long long)(ex + nx * (ey + ny * ez)) * 8 + a + 2 * (b + 2 * c)];
            }
    gfieldw<double>(R, F_HCA)[q] = s;
}

// coarse fast diagonalisation, x and y directions of one z-plane per
// workgroup (grid.x = z index): fwd: out = (S_y^T x S_x^T) in, else
// out = (S_y x S_x) in
__global__ void __launch_bounds__(256) hs_cxy_kernel(Batch bt, int lx, int fwd, int src, int dst, int gate)
{
    __shared__ double sP[HS_CPLANE], sQ[HS_CPLANE];
    const ReqDesc* R = bt.r[blockIdx.y];
    if (!gate_ok(R, gate)) return;
    const int nx = R->nel[0], ny = R->nel[1], nz = R->nel[2];
    const int cz = blockIdx.x;
    if (cz >= nz) return;
    const HsOff o = hs_off(lx, R->nel);
    const SEM_GLOBAL double* tb = gfield<double>(R, F_HST);
    const SEM_GLOBAL double* Sx = tb + o.Sc[0];
    const SEM_GLOBAL double* Sy = tb + o.Sc[1];
    const SEM_GLOBAL double* in = gfield<double>(R, src) + (long long)cz * nx * ny;
    const int np = nx * ny;
    for (int q = threadIdx.x; q < np; q += blockDim.x) sP[q] = in[q];
    __syncthreads();
    for (int q = threadIdx.x; q < np; q += blockDim.x) {
        const int x = q % nx, y = q / nx;
        double s = 0.0;
        for (int a = 0; a < nx; ++a) s += (fwd ? Sx[a * nx + x] : Sx[x * nx + a]) * sP[y * nx + a];
        sQ[q] = s;
    }
    __syncthreads();
    SEM_GLOBAL double* out = gfieldw<double>(R, dst) + (long long)cz * nx * ny;
    for (int q = threadIdx.x; q < np; q += blockDim.x) {
        const int x = q % nx, y = q / nx;
        double s = 0.0;
        for (int b = 0; b < ny; ++b) s += (fwd ? Sy[b * ny + y] : Sy[y * ny + b]) * sQ[b * nx + x];
        out[q] = s;
    }
}

// coarse fast diagonalisation, z direction of one y-row per workgroup
// (grid.x = y index): S_z^T, division by the eigenvalue sums (the constant
// mode is dropped), S_z
__global__ void __launch_bounds__(256) hs_cz_kernel(Batch bt, int lx, int src, int dst, int gate)
{
    __shared__ double sP[HS_CPLANE], sQ[HS_CPLANE];
    const ReqDesc* R = bt.r[blockIdx.y];
    if (!gate_ok(R, gate)) return;
    const int nx = R->nel[0], ny = R->nel[1], nz = R->nel[2];
    const int cy = blockIdx.x;
    if (cy >= ny) return;
    const HsOff o = hs_off(lx, R->nel);
    const SEM_GLOBAL double* tb = gfield<double>(R, F_HST);
    const SEM_GLOBAL double* Sz = tb + o.Sc[2];
    const SEM_GLOBAL double* in = gfield<double>(R, src);
    const int np = nx * nz;                 // (x, z) of row cy, x fastest
    for (int q = threadIdx.x; q < np; q += blockDim.x) {
        const int x = q % nx, z = q / nx;
        sP[q] = in[x + (long long)nx * (cy + (long long)ny * z)];
    }
    __syncthreads();
    const double ly = tb[o.Lc[1] + cy];
    for (int q = threadIdx.x; q < np; q += blockDim.x) {
        const int x = q % nx, z = q / nx;
        double s = 0.0;
        for (int c = 0; c < nz; ++c) s += Sz[c * nz + z] * sP[c * nx + x];
        if (x == R->hs_c0[0] && cy == R->hs_c0[1] && z == R->hs_c0[2]) s = 0.0;
        else s /= tb[o.Lc[0] + x] + ly + tb[o.Lc[2] + z];
        sQ[q] = s;
    }
    __syncthreads();
    SEM_GLOBAL double* out = gfieldw<double>(R, dst);
    for (int q = threadIdx.x; q < np; q += blockDim.x) {
        const int x = q % nx, z = q / nx;
        double s = 0.0;
        for (int c = 0; c < nz; ++c) s += Sz[z * nz + c] * sQ[c * nx + x];
        out[x + (long long)nx * (cy + (long long)ny * z)] = s;
    }
}

// ---------------------------------------------------------------- middle level, up
template <int LM>
__global__ void __launch_bounds__(hs_mepb(LM) * LM * LM) hs_midup_kernel(Batch bt, int lx, int gate)
{
    constexpr int L2 = LM * LM, L3 = L2 * LM, EP = hs_mepb(LM);
    __shared__ double sJc[2 * LM];
    __shared__ double sE[EP * 8];
    const int g = blockIdx.x;
    const int ri = find_req(bt.hm, bt.n, g);
    const ReqDesc* R = bt.r[ri];
    if (!gate_ok(R, gate)) return;
    const int t = threadIdx.x, el = t / L2, ij = t - el * L2, i = ij % LM, j = ij / LM;
    const int e = (g - bt.hm[ri]) * EP + el;
    const bool live = e < R->E;
    const int ee = live ? e : 0;
    const HsOff o = hs_off(lx, R->nel);
    const SEM_GLOBAL double* tb = gfield<double>(R, F_HST);
    for (int q = t; q < 2 * LM; q += EP * L2) sJc[q] = tb[o.Jc + q];
    int ex, ey, ez;
    elem_xyz(ee, R->nel, ex, ey, ez);
    const int nx = R->nel[0], ny = R->nel[1], nz = R->nel[2];
    if (ij < 8) {
        const int a = ij & 1, b = (ij >> 1) & 1, c = ij >> 2;
        const int cx = (ex + a) % nx, cy = (ey + b) % ny, cz = (ez + c) % nz;
        sE[el * 8 + ij] = gfield<double>(R, F_HCB)[cx + nx * (cy + ny * cz)];
    }
    __syncthreads();
    if (!live) return;
    const double* E8 = sE + el * 8;
    const SEM_GLOBAL double* sm = gfield<double>(R, F_HSM);
    SEM_GLOBAL double* zm = gfieldw<double>(R, F_HZM) + (long long)e * L3;
#pragma unroll
    for (int k = 0; k < LM; ++k) {
        double p = 0.0;
        for (int c = 0; c < 2; ++c)
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a)
                    p += E8[a + 2 * (b + 2 * c)] * sJc[i * 2 + a] * sJc[j * 2 + b] * sJc[k * 2 + c];
        zm[i + LM * (j + LM * k)] = box_sum<LM, true>(sm, R->nel, ex, ey, ez, i, j, k) + p;
    }
}

// ---------------------------------------------------------------- fine level, up
// z -> F_HZ (the operator's input) and Z_J of F_HZS (the cycle end's x update), type TZ
template <int LX, typename TZ>
__global__ void __launch_bounds__(LX * LX) hs_up_kernel(Batch bt, int gate)
{
    constexpr int LM = hs_lxm(LX), L2 = LX * LX, L3 = L2 * LX;
    __shared__ double sA[LM * LM * LM], sB[LM * LM * LX];
    __shared__ double sJ[LX * LM];
    const int g = blockIdx.x;
    const int ri = find_req(bt.el, bt.n, g);
    const ReqDesc* R = bt.r[ri];
    const int e = g - bt.el[ri];
    if (!gate_ok(R, gate)) return;
    const int t = threadIdx.x, i = t % LX, j = t / LX;
    const HsOff o = hs_off(LX, R->nel);
    const SEM_GLOBAL double* tb = gfield<double>(R, F_HST);
    for (int q = t; q < LX * LM; q += L2) sJ[q] = tb[o.J + q];
    const SEM_GLOBAL double* zm = gfield<double>(R, F_HZM) + (long long)e * LM * LM * LM;
    for (int q = t; q < LM * LM * LM; q += L2) sA[q] = zm[q];
    __syncthreads();
    // x: sB[c][b][i] = sum_a J[i][a] zm[c][b][a]
    if (j < LM) {
#pragma unroll
        for (int c = 0; c < LM; ++c) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a < LM; ++a) s += sJ[i * LM + a] * sA[c * LM * LM + j * LM + a];
            sB[c * LM * LX + j * LX + i] = s;
        }
    }
    __syncthreads();
    double col[LM];
#pragma unroll
    for (int c = 0; c < LM; ++c) {
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < LM; ++b) s += sJ[j * LM + b] * sB[c * LM * LX + b * LX + i];
        col[c] = s;
    }
    int ex, ey, ez;
    elem_xyz(e, R->nel, ex, ey, ez);
    const SEM_GLOBAL double* sf = gfield<double>(R, F_HSF);
    const long long base = (long long)e * L3 + i + LX * j;
    SEM_GLOBAL TZ* hz = gfieldw<TZ>(R, F_HZ) + base;
    SEM_GLOBAL TZ* zj = gfieldw<TZ>(R, F_HZS) + (long long)gp(R->I)[I_GJ] * R->np + base;
#pragma unroll
    for (int k = 0; k < LX; ++k) {
        double p = 0.0;
#pragma unroll
        for (int c = 0; c < LM; ++c) p += sJ[k * LM + c] * col[c];
        const TZ z = (TZ)(box_sum<LX, true>(sf, R->nel, ex, ey, ez, i, j, k) + p);
        hz[L2 * k] = z;
        zj[L2 * k] = z;
    }
}

template <int LX>
static void hsmg_go(const Batch& b, int tb, int gate, hipStream_t s)
{
    constexpr int LM = hs_lxm(LX);
    const int ne = b.el[b.n];
    if (ne == 0) return;
    if (tb == P64) hipLaunchKernelGGL((hs_down_kernel<LX, double>), dim3(ne), dim3(LX * LX), 0, s, b, gate);
    else hipLaunchKernelGGL((hs_down_kernel<LX, float>), dim3(ne), dim3(LX * LX), 0, s, b, gate);
    constexpr int EP = hs_mepb(LM);
    const int nmb = b.hm[b.n];
    hipLaunchKernelGGL((hs_mid_kernel<LM>), dim3(nmb), dim3(EP * LM * LM), 0, s, b, LX, gate);
    const dim3 cg((b.ncmax + 255) / 256, b.n);
    hipLaunchKernelGGL(hs_cgath_kernel, cg, dim3(256), 0, s, b, gate);
    // coarse fast diagonalisation: F_HCA -> (x, y fwd) F_HCB -> (z) F_HCA -> (x, y inv) F_HCB
    const dim3 cp(b.cnmax, b.n);
    hipLaunchKernelGGL(hs_cxy_kernel, cp, dim3(256), 0, s, b, LX, 1, (int)F_HCA, (int)F_HCB, gate);
    hipLaunchKernelGGL(hs_cz_kernel, cp, dim3(256), 0, s, b, LX, (int)F_HCB, (int)F_HCA, gate);
    hipLaunchKernelGGL(hs_cxy_kernel, cp, dim3(256), 0, s, b, LX, 0, (int)F_HCA, (int)F_HCB, gate);
    hipLaunchKernelGGL((hs_midup_kernel<LM>), dim3(nmb), dim3(EP * LM * LM), 0, s, b, LX, gate);
    if (tb == P64) hipLaunchKernelGGL((hs_up_kernel<LX, double>), dim3(ne), dim3(LX * LX), 0, s, b, gate);
    else hipLaunchKernelGGL((hs_up_kernel<LX, float>), dim3(ne), dim3(LX * LX), 0, s, b, gate);
}

void launch_hsmg(const Batch& b, int lx, int tb, int gate, hipStream_t s)
{
    switch (lx) {
    case 5: hsmg_go<5>(b, tb, gate, s); break;
    case 6: hsmg_go<6>(b, tb, gate, s); break;
    case 7: hsmg_go<7>(b, tb, gate, s); break;
    case 8: hsmg_go<8>(b, tb, gate, s); break;
    case 9: hsmg_go<9>(b, tb, gate, s); break;
    case 10: hsmg_go<10>(b, tb, gate, s); break;
    case 11: hsmg_go<11>(b, tb, gate, s); break;
    case 12: hsmg_go<12>(b, tb, gate, s); break;
    default: break;
    }
}

}  // namespace semk
