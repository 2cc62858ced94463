// Internal layout shared by the host runtime and the HIP kernels of libsem.
//
// A request (one sem_ctx) owns a device workspace carved from the caller's
// buffer.  Its descriptor ReqDesc lives at the start of that workspace and
// holds every field pointer by id, the per-request scalar area S (double),
// the integer state I, the reduction partials and the shared-node lists.
// Kernels receive a Batch by value: up to SEM_MAXB descriptors plus prefix
// tables over their element blocks and shared-node chunks, so one launch
// covers every request of a batch, and a batch of one is the plain case.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include "sem.h"

#define SEM_MAXB 48          // requests per batched launch
#define SEM_MAXM 30          // largest GMRES restart length
#define SEM_GS_THREADS 256   // threads of the gather-scatter kernel
#define SEM_VEC_THREADS 256  // threads of point-wise kernels
#define HS_NELMAX 64         // HSMG: elements per direction at most (a coarse plane fits in LDS)
#define HS_CPLANE (HS_NELMAX * HS_NELMAX)

namespace semk {

enum PrecId { P64 = 0, P32 = 1, P16 = 2, PBF = 3 };

// ---------------------------------------------------------------- fields
enum FieldId : int {
    // geometry, fp64 (always present)
    F_G64 = 0,      // [E][6][lx3]  G_rr G_rs G_rt G_ss G_st G_tt
    F_B64,          // [E][lx3]     mass B = jac w_i w_j w_k
    F_M64,          // [E][9][lx3]  M_ac = B dr_a/dx_c, index a*3+c
    F_IBSUM64,      // 1 / dssum(B)
    F_DA64,         // dssum(diag A_L)  (stiffness diagonal, assembled)
    F_IDP64,        // 1 / F_DA64 with the zero guard (pressure Jacobi)
    F_IDV64,        // 1 / (h1 dA + h2 dssum(B))  (velocity Jacobi, current h)
    // reduced-storage geometry copies
    F_G32, F_B32, F_M32, F_IDP32, F_IDV32,
    F_G16, F_B16, F_M16,       // 16-bit (fp16 or bf16, one kind per request), element-scaled
    F_GSC,                      // float[E]: scale of G16 (and of B16 in F_GSC + E)
    F_MSC,                      // float[E]: scale of M16
    // fluid state (fp64)
    F_U, F_U1, F_U2,            // u^n components
    F_UL1, F_UL1b, F_UL1c,      // u^{n-1}
    F_UL2, F_UL2b, F_UL2c,      // u^{n-2}
    F_BN, F_BNb, F_BNc,         // B N(u^n)
    F_BNL1, F_BNL1b, F_BNL1c,
    F_BNL2, F_BNL2b, F_BNL2c,
    F_P,                        // p^n
    F_RHS, F_RHSb, F_RHSc,      // assembled velocity rhs
    F_US, F_USb, F_USc,         // u*
    F_GP, F_GPb, F_GPc,         // gradient scratch (fp64)
    F_R64, F_R64b, F_R64c,      // fp64 residual scratch
    F_W64, F_W64b, F_W64c,      // fp64 operator output scratch
    F_RP,                       // pressure rhs
    F_PHI,                      // pressure increment
    // velocity PCG vectors (velocity storage precision), 3 components each
    F_PX, F_PXb, F_PXc,
    F_PR, F_PRb, F_PRc,
    F_PZ, F_PZb, F_PZc,
    F_PP, F_PPb, F_PPc,
    F_PW, F_PWb, F_PWc,
    // GMRES (fp64 basis and iterate; pressure-Ax precision for z and w)
    F_V,                        // (m+1) GMRES basis vectors, stride np, basis storage precision
    F_GW,                       // operator output of the Arnoldi step (fp64)
    F_GWD,                      // fp64 working vector of the Arnoldi step
    F_GB,                       // rhs (fp64)
    F_GX,                       // iterate (fp64)
    // pressure projection (fluid mode with proj_dim > 0)
    F_PRX,                      // proj_dim stored vectors, stride np, basis storage precision, unnormalised
    F_PRXB,                     // the projected guess of the current step (fp64)
    // dealiased convection (flow.dealias): metric terms at the LXD^3 Gauss-Legendre points
    F_MFD64,                    // [E][9][lxd3] W dr_a/dx_c, index a*3+c (W = jac * GL weights)
    F_MFD32,                    // fp32 copy (conv storage fp32)
    F_MFD16,                    // 16-bit copy (conv storage fp16/bf16), element-scaled
    F_MFDSC,                    // float[E]: scale of F_MFD16
    // HSMG pressure preconditioner (flow.hsmg): levels lx, hs_lxm(lx), 2
    F_HST,                      // double tables, layout HsOff
    F_HSF,                      // [E][lx3]   fine-level local Schwarz solutions (element copies, unsummed)
    F_HRM,                      // [E][lxm3]  restricted residual, element contributions (unsummed)
    F_HSM,                      // [E][lxm3]  middle-level local Schwarz solutions (unsummed)
    F_HZM,                      // [E][lxm3]  middle-level correction (continuous)
    F_HC8,                      // [E][8]     coarse-corner contributions of each element
    F_HCA, F_HCB,               // [nx ny nz] coarse vectors (unique corner nodes), ping-pong
    F_HZ,                       // [E][lx3]   M^{-1} V_J in the basis storage precision (Arnoldi operator input)
    F_HZS,                      // (m+1) x [E][lx3] Z_j = M^{-1} s_j V_j of every Arnoldi step, basis precision
    NFIELD
};

// ---------------------------------------------------------------- scalars (double S[])
enum ScalarId : int {
    S_H1 = 0, S_H2,             // velocity Helmholtz coefficients of the current step
    S_NU, S_DT, S_BETA0,
    S_BDF,                      // 3 values b_1..b_3
    S_EXT = S_BDF + 3,          // 3 values a_1..a_3
    S_TIME = S_EXT + 3,
    S_VTOL, S_PTOL,
    S_IDV_H1, S_IDV_H2,         // h of the stored velocity Jacobi diagonal
    S_RHO,                      // 3: PCG rho per component
    S_ALPHA = S_RHO + 3,
    S_BETA = S_ALPHA + 3,
    S_RN = S_BETA + 3,          // 3: current PCG residual norm
    S_R0 = S_RN + 3,            // 3: fp64 true residual norm
    S_GBETA = S_R0 + 3,         // GMRES true residual norm
    S_GH,                       // (m+1)*m Hessenberg, row-major H[i*m + j]
    S_GCS = S_GH + (SEM_MAXM + 1) * SEM_MAXM,
    S_GSN = S_GCS + SEM_MAXM,
    S_GG = S_GSN + SEM_MAXM,    // m+1 rotated rhs
    S_GY = S_GG + SEM_MAXM + 1, // m solution of the small system
    S_GHC = S_GY + SEM_MAXM,    // m+1 first-pass Gram-Schmidt coefficients
    S_GH2 = S_GHC + SEM_MAXM + 1,  // m+1 second-pass coefficients
    S_MEAN = S_GH2 + SEM_MAXM + 1, // scratch for mean removal
    S_KE, S_ENST, S_MAXDIV,
    S_VOL,                      // sum of B (domain volume)
    S_PRA,                      // SEM_MAX_PROJ: projection coefficients alpha_i of the guess
    S_PRB = S_PRA + SEM_MAX_PROJ,   // SEM_MAX_PROJ: A-orthogonalisation coefficients beta_i
    S_PRS = S_PRB + SEM_MAX_PROJ,   // SEM_MAX_PROJ: 1/||X_i||_A of the stored projection vectors
    S_GVS = S_PRS + SEM_MAX_PROJ,   // m+1: 1/norm of the stored (unnormalised) basis vectors V_i
    S_GMEAN = S_GVS + SEM_MAXM + 1,  // unique-node mean of the current Arnoldi operator output
    S_CFLT,                     // target CFL number (> 0: adaptive dt)
    S_DTMAX,                    // largest step (the configured dt)
    S_DTH,                      // 3: step sizes dt_n, dt_{n-1}, dt_{n-2}
    S_CFLR = S_DTH + 3,         // CFL rate of the current velocity (from the diagnostics kernel)
    S_CFL,                      // CFL number of the current step
    S_RED,                      // generic finalised reductions (SEM_NRED values)
    NSCALAR = S_RED + 64
};

// reduction slots (partials[slot][block])
enum RedSlot : int {
    R_A = 0,                    // 3 generic per-component slots
    R_B = 3,                    // 3
    R_C = 6,                    // 3
    R_GM = 9,                   // SEM_MAXM + 1 GMRES dot slots
    R_GN = R_GM + SEM_MAXM + 1, // GMRES norm
    R_GMEAN,                    // GMRES operator-output unique sum (null-space deflation)
    R_X0, R_X1, R_X2, R_X3,     // diagnostics and means
    R_X4,                       // CFL rate (max)
    NRED
};

// ---------------------------------------------------------------- integer state (int I[])
enum IntId : int {
    I_STEP = 0, I_ORDER, I_TORDER,
    I_VACT,                     // 3: PCG component active
    I_VIT = I_VACT + 3,         // 3: PCG iterations (cumulative over refinement cycles)
    I_VREF = I_VIT + 3,         // 3: refinement cycles
    I_VMAXIT = I_VREF + 3,
    I_GPHASE,                   // 0 Arnoldi, 1 cycle end pending, 2 done
    I_GJ,                       // current Arnoldi index j (vectors 0..j exist)
    I_GJEND,                    // size of the small system at cycle end
    I_GIT,                      // total Arnoldi steps
    I_GMAXIT, I_GM,
    I_GACT,                     // GMRES active (phase != done)
    I_NAN,                      // non-finite value seen
    I_ALWAYS,                   // constant 1 (gate for unconditional launches)
    I_VDONE,                    // velocity refinement finished for all components
    I_GARN,                     // GMRES: Arnoldi step pending (phase 0)
    I_GEND,                     // GMRES: cycle end pending (phase 1)
    I_GNORM,                    // GMRES: a new basis vector was stored (informational)
    I_VMAXREF,                  // velocity refinement cycle limit
    I_GENDAX,                   // GMRES: cycle end with a nonzero iterate (true residual needs A x)
    I_IDVSTALE,                 // velocity Jacobi diagonal must be rebuilt for new (h1,h2)
    I_PRL,                      // projection: vectors in the space
    I_PRFULL,                   // projection: the space was full and restarts from the whole solution
    I_PRADD,                    // projection: the new vector is independent and will be appended
    I_COMMIT,                   // 3 (equal): the step's solves finished, its results may be committed
    I_PCNT = I_COMMIT + 3,      // NRED: number of partials the last producer of each slot wrote
    NINT = I_PCNT + NRED + 8
};

struct ReqDesc {
    int E, lx, epb, nb;         // elements, points per direction, elements per block, blocks
    int vepb, nvb;              // elements per point-wise block, point-wise blocks
    int pstride;                // row stride of the partials: max(nb, nvb)
    int prec16;                 // 0 none, 2 fp16, 3 bf16
    int gm_m;                   // GMRES restart
    int proj_L;                 // pressure projection space dimension (0 = off)
    int nel[3];                 // elements per direction of the periodic box
    int hs;                     // HSMG pressure preconditioner on
    int hs_c0[3];               // index of the constant coarse mode per direction
    long long np, nglob;
    double* S;                  // scalars
    int* I;                     // integer state
    double* part;               // reduction partials [NRED][pstride]
    const double* D64;          // D[i*lx+l] (lx*lx), w[lx], xi[lx], 1/mult[lx^3], then the dealiasing
                                // tables I[lxd*lx], ID[lxd*lx] (= I D), wz[lxd]
    const float* D32;           // D, w, xi, I, ID, wz in fp32
    void* f[NFIELD];
};

// periodic box mesh, optional sinusoidal node perturbation
struct MeshParams {
    int nel[3];
    int N;
    double lo[3], h[3];
    double amp;
    double phase[9];
};

struct Batch {
    int n;                      // requests
    int lx;                     // points per direction, shared by every request of a batch
    int eb[SEM_MAXB + 1];       // prefix over element blocks
    int vb[SEM_MAXB + 1];       // prefix over point-wise blocks
    int el[SEM_MAXB + 1];       // prefix over elements (one-element-per-workgroup kernels)
    int hm[SEM_MAXB + 1];       // prefix over HSMG middle-level blocks (hs_mepb elements each)
    int gl[SEM_MAXB + 1];       // prefix over row-form gather-scatter workgroups (one per x-line of elements and k)
    int gq[SEM_MAXB + 1];       // prefix over plane-form gather-scatter workgroups (one per x-line and 4 planes k)
    int gate;                   // element operators (conv, opgrad, wdiv, diagnostics): I index that must
                                // be nonzero for a request's blocks to run, or -1
    int ncmax;                  // largest coarse HSMG grid (nx ny nz) of the batch
    int cnmax;                  // largest ny or nz of the batch (coarse-pass workgroups)
    const ReqDesc* r[SEM_MAXB];
};

// 16-bit fine-grid metric terms of the dealiased convection: lane-ordered for
// the matrix-core kernel (lx <= 10), per element [tile][ac][g][m][r] with
// r fastest (one 8-byte load per lane and term), else natural [ac][point]
__host__ __device__ constexpr int dl16_lane(int lx) { return lx <= 10 ? 1 : 0; }
__host__ __device__ constexpr int dl16_per_elem(int lx)
{
    return dl16_lane(lx) ? (((3 * lx + 1) / 2) * ((3 * lx + 1) / 2) + 15) / 16 * 9 * (((3 * lx + 1) / 2 + 3) / 4) * 64
                         : 9 * ((3 * lx + 1) / 2) * ((3 * lx + 1) / 2) * ((3 * lx + 1) / 2);
}

// HSMG middle level: order N/2; its kernels take hs_mepb elements per workgroup
__host__ __device__ constexpr int hs_lxm(int lx) { return (lx - 1) / 2 + 1; }
__host__ __device__ constexpr int hs_mepb(int lm) { return 64 / (lm * lm) > 0 ? 64 / (lm * lm) : 1; }

// offsets (doubles) of the HSMG tables in F_HST: fine S (3 lx^2, S[c][i*lx+k] =
// component i of eigenvector k), fine lambda (3 lx), middle S, middle lambda,
// J fine<-middle (lx*lxm, J[i*lxm+a]), J middle<-coarse (lxm*2), coarse S per
// direction (n_c^2 each), coarse lambda per direction (n_c each)
struct HsOff {
    int Sf, Lf, Sm, Lm, J, Jc, Sc[3], Lc[3], total;
};
__host__ __device__ inline HsOff hs_off(int lx, const int* nel)
{
    const int lm = hs_lxm(lx);
    HsOff o;
    o.Sf = 0;
    o.Lf = o.Sf + 3 * lx * lx;
    o.Sm = o.Lf + 3 * lx;
    o.Lm = o.Sm + 3 * lm * lm;
    o.J = o.Lm + 3 * lm;
    o.Jc = o.J + lx * lm;
    int q = o.Jc + 2 * lm;
    for (int c = 0; c < 3; ++c) { o.Sc[c] = q; q += nel[c] * nel[c]; }
    for (int c = 0; c < 3; ++c) { o.Lc[c] = q; q += nel[c]; }
    o.total = q;
    return o;
}

// gather-scatter: the plane form runs where an element's plane fits a wave
// with V nodes a lane (lx * lx / V <= 64), else the row form
__host__ __device__ constexpr bool gs_planes(int lx, int V) { return lx * (lx / V) <= 64; }
// most gather-scatter workgroups of one request, over both forms
__host__ __device__ constexpr int gs_blocks(int lx, int ny, int nz) { return ny * nz * (lx - 1); }

// elements per workgroup of the element kernels (shared by host and device)
__host__ __device__ constexpr int epb_of(int lx)
{
    return lx == 12 ? 2 : lx == 10 ? 5 : lx == 11 ? 2 : (256 / (lx * lx) > 0 ? 256 / (lx * lx) : 1);
}

// elements per point-wise block: about 1024 blocks per request, at most
// ~16K points per block (depends only on the request, so a request's
// reductions are identical alone and in a batch)
inline int vepb_of(int lx, int E)
{
    const int cap = 16384 / (lx * lx * lx) > 0 ? 16384 / (lx * lx * lx) : 1;
    int v = E / 1024;
    if (v < 1) v = 1;
    if (v > cap) v = cap;
    return v;
}

// locate the request of a flat block index in a prefix table
__device__ __forceinline__ int find_req(const int* prefix, int n, int g)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

}  // namespace semk

// ---------------------------------------------------------------- launch interface
namespace semk {

struct AxLaunch {
    int src, dst;               // field ids (components add blockIdx.y)
    int src_vj;                 // nonzero: input is GMRES basis vector V_J (J read on the device)
    int ncomp;                  // 1 or 3
    int hsel;                   // S index of (h1,h2) or -1 to use h1,h2 below
    double h1, h2;
    int precond;                // field id of the inverse diagonal applied to src on load, or -1
    int tpc;                    // PrecId of that diagonal (P64 or P32)
    int pdot;                   // reduction slot for sum(u*w) over local points, or -1
    int gate;                   // I index checked per component (nonzero = run), or -1
    int tu, tg, tc;             // PrecId of vectors, geometry and arithmetic
    int out64;                  // nonzero: the output is fp64 whatever tu is (Arnoldi operator output)
    int sub;                    // field id of a local rhs r_L: output r_L - (operator u) (fp64 only), or -1
    const void* u_raw;          // direct pointers (standalone sem_ax), used when src < 0
    void* w_raw;
};

void launch_ax(const Batch& b, int lx, const AxLaunch& a, hipStream_t s);
// the matrix-core operator (lx = 8, fp32 arithmetic, 16-bit geometry, no Jacobi
// scaling, residual form or fp64 output); false when it does not apply
bool launch_ax_mfma(const Batch& b, int lx, const AxLaunch& a, hipStream_t s);
// pslot >= 0: also the squared norm over unique nodes of each component c,
// as per-workgroup partials in slot pslot + c (see gs_blocks for their count)
void launch_dssum(const Batch& b, int field, int ncomp, int tprec, int gate, void* raw, hipStream_t s,
                  int pslot = -1);

// geometry and setup
void launch_geometry(const Batch& b, int lx, const MeshParams& mp, hipStream_t s);
void launch_diag_a(const Batch& b, int lx, hipStream_t s);
void launch_geo_post(const Batch& b, hipStream_t s);
void launch_geo_cast(const Batch& b, int lx, int want32, int want16, hipStream_t s);
void launch_init_fields(const Batch& b, int lx, int init, const MeshParams& mp, hipStream_t s);
void launch_node_field(const Batch& b, int lx, const MeshParams& mp, int what, double amp, double* out, hipStream_t s);

// SEM operators (output fp64)
void launch_conv(const Batch& b, int lx, int tm, int tc, hipStream_t s);
void launch_dealias_geom(const Batch& b, int lx, const MeshParams& mp, int want32, int want16, hipStream_t s);
void launch_conv_dealias(const Batch& b, int lx, int tm, int tc, hipStream_t s);
void launch_opgrad(const Batch& b, int lx, int tm, int tc, int src, int dst, hipStream_t s);
// grad p folded into the step's local velocity rhs (F_RHS), without storing grad p
void launch_opgrad_rhs(const Batch& b, int lx, int tm, int tc, int src, hipStream_t s);
void launch_wdiv(const Batch& b, int lx, int tm, int tc, int src, int dst, hipStream_t s);
void launch_diagnostics(const Batch& b, int lx, hipStream_t s);

// HSMG in the Arnoldi step: z = M^{-1} s_J V_J into F_HZ (the operator's
// input) and into Z_J of F_HZS (the cycle end's x update), both in the basis
// precision tb; gated per request
void launch_hsmg(const Batch& b, int lx, int tb, int gate, hipStream_t s);

// point-wise / reduction / scalar kernels
enum VecOp : int {
    V_PCG_INIT = 0,   // PX = 0, PR = R64, PZ = PR*IDV, PP = PZ, partial (r,z) -> R_B+c
    V_PCG_UPD,        // PX += a PP, PR -= a PW, PZ = PR*IDV, partials (r,r) -> R_B+c, (r,z) -> R_C+c
    V_PCG_P,          // PP = PZ + b PP
    V_US_COPY,        // US = U
    V_US_ADD,         // US += PX  (f0 == 1: US = U + PX)
    V_IDV,            // velocity Jacobi inverse diagonal for the current (h1,h2)
    V_SUM_UNIQUE,     // partial sum(f/mult) of field f0 -> R_X3
    V_SUM_MASS,       // partial sum(B f) of field f0 -> R_X3
    V_SUB_MEAN,       // f0 = scale*(f0 - S_MEAN)   (scale = S[f1] or 1 when f1 < 0)
    V_COPY,           // f1 = f0 (fp64)
    V_ZERO,           // f0 = 0 (fp64)
    V_GM_DOTS,        // partials (V_i, GW) -> R_GM+i, i <= J, and sum(GW/mult) -> R_GMEAN
    V_GM_UPD_DOTS,    // GWD = GW - S_GMEAN - sum GHC_i V_i ; partials (V_i, GWD) -> R_GM+i
    V_GM_UPD_NORM,    // V_{J+1} = GWD - sum GH2_i V_i (unnormalised); partial |V_{J+1}|^2 -> R_GN
    V_GM_XUPD,        // GX += IDP * sum_{i<jend} y_i V_i
    V_GM_RESID,       // V_0 = GB - GWD (GB alone when I_GENDAX == 0), partial |V_0|^2 -> R_GN
    V_CORRECT,        // U_new = US - dt/beta0 GP / Bsum  (into the u^{n-2} buffer); P += GX
    V_AXPY_RAW,       // raw y += a x (fp64), used by the standalone API
    V_MASS_RAW,       // raw y = B x (fp64)
    V_PR_ADOTS,       // partials (X_i, GB) -> R_GM+i, i < l
    V_PR_GUESS,       // GX = PRXB = sum_i alpha_i s_i X_i
    V_PR_V,           // GW = GX - PRXB (GX alone when the space restarts): the candidate direction
    V_PR_BDOTS,       // partials (X_i, GWD) -> R_GM+i, i < l, and (GW, GWD) -> R_GM+l
    V_PR_ORTH,        // X_l = GW - sum_i beta_i s_i X_i
    V_GM_XZ,          // GX += sum_{i<jend} y_i Z_i  (HSMG cycle end: Z_i = M^{-1} s_i V_i kept from the Arnoldi steps)
    NVECOP
};

struct VecArgs {
    int op, gate, ncomp;
    int tv;           // PrecId of the velocity/pressure solver vectors
    int ta;           // PrecId of the per-thread partial sums (fp64 or fp32)
    int tb;           // PrecId of the GMRES basis storage
    int f0, f1;
    double a;
    const void* x_raw;
    void* y_raw;
};

enum FinOp : int {
    FIN_VINIT = 0, FIN_PCG_RHO, FIN_PCG_ALPHA, FIN_PCG_BETA,
    FIN_MEAN_UNIQUE, FIN_MEAN_MASS,
    FIN_GM_H1, FIN_GM_H2, FIN_GM_COL, FIN_GM_RESTART, FIN_GM_START,
    FIN_DIAG, FIN_STEP_BEGIN, FIN_STEP_END,
    FIN_POLL,         // host flag[ri] = I[gate] (| I[gate+1] | I[gate+2] when ncomp = 3)
    FIN_SUM_RAW,      // S[S_RED + gate] = sum of slot f0 partials
    FIN_VOL,          // S_VOL = sum of slot R_X3 partials
    FIN_STATS,        // host_stats[ri*SEM_NSTAT ...] = step statistics
    FIN_PR_ALPHA,     // alpha_i = s_i (X_i, GB)
    FIN_PR_POST,      // a full space restarts (l = 0, I_PRFULL)
    FIN_PR_BETA,      // beta_i = s_i (X_i, A v); ||v_orth||_A^2 = (v, A v) - sum beta_i^2; I_PRADD, s_l
    FIN_PR_COMMIT,    // l += I_PRADD
    FIN_COMMIT_CHECK, // I_COMMIT = no velocity component and no GMRES solve still iterating
    NFINOP
};

#define SEM_NSTAT 19

struct FinArgs {
    int op, gate, ncomp, f0;
    int* host_flags;
    double* host_stats;
    int gate2;        // I index that must be nonzero for the op to run on a request, or -1
};

void launch_vec(const Batch& b, const VecArgs& a, hipStream_t s);
void launch_fin(const Batch& b, const FinArgs& a, hipStream_t s);

// Stand-alone Jacobi-GMRES Poisson solve of one bound context (any mode) on a
// caller-provided Krylov workspace ws (256-byte aligned, at least the bytes
// poisson_external_bytes reports; device is the context's HIP device).  Same
// arithmetic and launches as sem_poisson_solve; synchronises the stream.
int poisson_external_bytes(const sem_ctx* c, size_t* bytes, int* device);
int poisson_solve_external(sem_ctx* c, char* ws, size_t ws_bytes, const void* rhs, void* sol, sem_solve_stats* st);
// records msg as the library's last error and returns code
int set_error(int code, const char* msg);

}  // namespace semk
