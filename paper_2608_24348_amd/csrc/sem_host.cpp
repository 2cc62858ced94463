// Host runtime of libsem: descriptor validation, precision-policy resolution,
// GLL tables, shared-node lists, workspace layout, and the drivers of the
// batched Jacobi-PCG, GMRES and fluid step.  All arithmetic of the hot path
// runs in the HIP kernels; the host only sequences launches and polls small
// device-written convergence flags.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sem.h"
#include "sem_internal.h"

using namespace semk;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

// Stream capture in one host thread is invalidated by device-synchronising
// HIP calls in another (allocations and frees of device or pinned memory,
// copies on the legacy stream).  The library makes such calls only under this
// lock, which a capture holds throughout (with the graph cache), and exports
// it (sem_host_lock) to callers that make such calls from other threads.
std::recursive_mutex g_host_mu;

#define HIPCHK(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(SEM_EHIP, std::string(#call " failed: ") + hipGetErrorString(e_));     \
    } while (0)

// ------------------------------------------------------------------ GLL tables
// Nodes: -1, 1 and the zeros of q(x) = L_{N+1}(x) - L_{N-1}(x) (proportional
// to (1-x^2) L_N'(x)), found by Newton from Chebyshev-Gauss-Lobatto guesses.
// Weights 2 / (N (N+1) L_N(x)^2).  Derivative matrix from barycentric weights
// (off-diagonal (lam_j/lam_i)/(x_i-x_j), diagonal = minus the row sum).
void legendre_trio(int N, double x, double& lNm1, double& lN, double& lNp1, double& dNm1, double& dNp1)
{
    // values and derivatives of L_{N-1}, L_N, L_{N+1} by the Bonnet recurrence
    double p_prev = 1.0, p = x, d_prev = 0.0, d = 1.0;
    std::vector<double> P(N + 2), Dv(N + 2);
    P[0] = 1.0; Dv[0] = 0.0;
    P[1] = x; Dv[1] = 1.0;
    for (int n = 1; n <= N; ++n) {
        double pn = ((2 * n + 1) * x * p - n * p_prev) / (n + 1);
        double dn = d_prev + (2 * n + 1) * p;
        p_prev = p; p = pn; d_prev = d; d = dn;
        P[n + 1] = p; Dv[n + 1] = d;
    }
    lNm1 = P[N - 1]; lN = P[N]; lNp1 = P[N + 1];
    dNm1 = Dv[N - 1]; dNp1 = Dv[N + 1];
}

void gll_tables(int N, std::vector<double>& x, std::vector<double>& w, std::vector<double>& D)
{
    const int n = N + 1;
    x.assign(n, 0.0); w.assign(n, 0.0); D.assign(n * n, 0.0);
    const double pi = 3.14159265358979323846;
    for (int j = 0; j <= N; ++j) {
        double xj = -std::cos(pi * j / N);
        if (j > 0 && j < N) {
            for (int it = 0; it < 200; ++it) {
                double a, b, c, da, dc;
                legendre_trio(N, xj, a, b, c, da, dc);
                double q = c - a, dq = dc - da;
                double dx = q / dq;
                xj -= dx;
                if (std::fabs(dx) <= 1e-17) break;
            }
        }
        x[j] = xj;
    }
    x[0] = -1.0; x[N] = 1.0;
    for (int j = 1; j <= N / 2; ++j) {  // symmetric pairs
        double s = 0.5 * (x[N - j] - x[j]);
        x[j] = -s; x[N - j] = s;
    }
    if (N % 2 == 0) x[N / 2] = 0.0;
    for (int j = 0; j <= N; ++j) {
        double a, b, c, da, dc;
        legendre_trio(N, x[j], a, b, c, da, dc);
        w[j] = 2.0 / (N * (N + 1.0) * b * b);
    }
    std::vector<double> lam(n, 1.0);
    for (int j = 0; j < n; ++j) {
        double prod = 1.0;
        for (int k = 0; k < n; ++k)
            if (k != j) prod *= (x[j] - x[k]);
        lam[j] = 1.0 / prod;
    }
    for (int i = 0; i < n; ++i) {
        double rs = 0.0;
        for (int j = 0; j < n; ++j) {
            if (i == j) continue;
            double v = (lam[j] / lam[i]) / (x[i] - x[j]);
            D[i * n + j] = v;
            rs += v;
        }
        D[i * n + i] = -rs;
    }
}

// Symmetric eigenproblem a = V diag(lam) V^T (a: n x n row-major, destroyed;
// V[r*n + k] = component r of eigenvector k) by cyclic two-sided Jacobi
// rotations, each zeroing one off-diagonal pair (Rutishauser's formulas).
static void sym_eig_jacobi(int n, std::vector<double>& a, std::vector<double>& V, std::vector<double>& lam)
{
    V.assign((size_t)n * n, 0.0);
    for (int r = 0; r < n; ++r) V[(size_t)r * n + r] = 1.0;
    auto A = [&](int r, int q) -> double& { return a[(size_t)r * n + q]; };
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int r = 0; r < n; ++r)
            for (int q = 0; q < n; ++q) (r == q ? diag : off) += A(r, q) * A(r, q);
        if (off <= 1e-30 * (diag + off)) break;
        for (int p = 0; p + 1 < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A(p, q);
                if (apq == 0.0) continue;
                const double th = (A(q, q) - A(p, p)) / (2.0 * apq);
                const double t = (th >= 0.0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                A(p, p) -= t * apq;
                A(q, q) += t * apq;
                A(p, q) = A(q, p) = 0.0;
                for (int r = 0; r < n; ++r) {
                    if (r != p && r != q) {
                        const double arp = A(r, p), arq = A(r, q);
                        A(r, p) = A(p, r) = cs * arp - sn * arq;
                        A(r, q) = A(q, r) = sn * arp + cs * arq;
                    }
                    const double vp = V[(size_t)r * n + p], vq = V[(size_t)r * n + q];
                    V[(size_t)r * n + p] = cs * vp - sn * vq;
                    V[(size_t)r * n + q] = sn * vp + cs * vq;
                }
            }
    }
    lam.resize(n);
    for (int r = 0; r < n; ++r) lam[r] = A(r, r);
}

// A s = lambda B s with B = diag(bd) > 0: S = B^{-1/2} V, V the eigenvectors
// of B^{-1/2} A B^{-1/2}; then S^T B S = I and S^T A S = diag(lambda)
static void fdm_pair(int n, const std::vector<double>& A, const std::vector<double>& bd, double* S, double* lam)
{
    std::vector<double> C((size_t)n * n), V, l;
    for (int r = 0; r < n; ++r)
        for (int q = 0; q < n; ++q) C[(size_t)r * n + q] = A[(size_t)r * n + q] / std::sqrt(bd[r] * bd[q]);
    sym_eig_jacobi(n, C, V, l);
    for (int r = 0; r < n; ++r)
        for (int q = 0; q < n; ++q) S[(size_t)r * n + q] = V[(size_t)r * n + q] / std::sqrt(bd[r]);
    for (int q = 0; q < n; ++q) lam[q] = l[q];
}

// HSMG tables (layout HsOff) of a periodic box of equal elements, order N:
// per level (N and N/2) and direction the element's 1D stiffness
// (2/h) D^T W D and mass (h/2) W, each end extended by a linear segment of
// length delta = (h/2)(x_1 - x_0) to a zero Dirichlet node (stiffness
// 1/delta and lumped mass delta/2 added at that end), in fast-diagonalised
// form; the interpolation matrices between the levels; the coarse (order 1)
// periodic 1D stiffness (2/h on the diagonal, -1/h to each neighbour) and
// mass (h) per direction, fast-diagonalised.  c0: index of the zero
// (constant) coarse mode per direction.
static void hsmg_tables(int N, const int* nel, const double* h, std::vector<double>& T, int* c0)
{
    const int lx = N + 1, lm = hs_lxm(lx);
    const HsOff o = hs_off(lx, nel);
    T.assign(o.total, 0.0);
    auto level = [&](int Nl, int oS, int oL) {
        const int n = Nl + 1;
        std::vector<double> x, w, D;
        gll_tables(Nl, x, w, D);
        for (int c = 0; c < 3; ++c) {
            const double delta = 0.5 * h[c] * (x[1] - x[0]);
            std::vector<double> A((size_t)n * n, 0.0), bd(n);
            for (int r = 0; r < n; ++r)
                for (int q = 0; q < n; ++q) {
                    double sum = 0.0;
                    for (int m = 0; m < n; ++m) sum += D[(size_t)m * n + r] * w[m] * D[(size_t)m * n + q];
                    A[(size_t)r * n + q] = 2.0 / h[c] * sum;
                }
            for (int r = 0; r < n; ++r) bd[r] = 0.5 * h[c] * w[r];
            A[0] += 1.0 / delta;
            A[(size_t)Nl * n + Nl] += 1.0 / delta;
            bd[0] += 0.5 * delta;
            bd[Nl] += 0.5 * delta;
            fdm_pair(n, A, bd, &T[oS + c * n * n], &T[oL + c * n]);
        }
        return x;
    };
    const std::vector<double> xf = level(N, o.Sf, o.Lf);
    const std::vector<double> xm = level(lm - 1, o.Sm, o.Lm);
    for (int i = 0; i < lx; ++i)
        for (int a = 0; a < lm; ++a) {
            double v = 1.0;
            for (int q = 0; q < lm; ++q)
                if (q != a) v *= (xf[i] - xm[q]) / (xm[a] - xm[q]);
            T[o.J + i * lm + a] = v;
        }
    for (int a = 0; a < lm; ++a) {
        T[o.Jc + 2 * a + 0] = 0.5 * (1.0 - xm[a]);
        T[o.Jc + 2 * a + 1] = 0.5 * (1.0 + xm[a]);
    }
    for (int c = 0; c < 3; ++c) {
        const int n = nel[c];
        std::vector<double> A((size_t)n * n, 0.0), bd(n, 0.0);
        for (int k = 0; k < n; ++k) {      // element k joins nodes k and k+1 (periodic)
            const int p = k, q = (k + 1) % n;
            A[(size_t)p * n + p] += 1.0 / h[c];
            A[(size_t)q * n + q] += 1.0 / h[c];
            A[(size_t)p * n + q] -= 1.0 / h[c];
            A[(size_t)q * n + p] -= 1.0 / h[c];
            bd[p] += 0.5 * h[c];
            bd[q] += 0.5 * h[c];
        }
        fdm_pair(n, A, bd, &T[o.Sc[c]], &T[o.Lc[c]]);
        int i0 = 0;
        for (int q = 1; q < n; ++q)
            if (T[o.Lc[c] + q] < T[o.Lc[c] + i0]) i0 = q;
        c0[c] = i0;
    }
}

int prec_rank(int p)
{
    // FP64 > FP32 > FP16 = BF16
    switch (p) {
    case SEM_FP64: return 3;
    case SEM_FP32: return 2;
    case SEM_FP16: return 1;
    case SEM_BF16: return 1;
    default: return -1;
    }
}

const char* pname(int p)
{
    switch (p) {
    case SEM_FP64: return "fp64";
    case SEM_FP32: return "fp32";
    case SEM_FP16: return "fp16";
    case SEM_BF16: return "bf16";
    default: return "?";
    }
}

int to_pid(int p)
{
    switch (p) {
    case SEM_FP64: return P64;
    case SEM_FP32: return P32;
    case SEM_FP16: return P16;
    default: return PBF;
    }
}

size_t psize(int pid) { return pid == P64 ? 8 : pid == P32 ? 4 : 2; }

struct Resolved {
    int tv, tva;            // velocity vectors, velocity dot accumulation (PrecId)
    int axv_g, axv_c;       // velocity Ax geometry storage and arithmetic
    int tpd;                // pressure Jacobi diagonal storage
    int tb;                 // GMRES basis storage (orthogonalisation arithmetic is fp64)
    int axp_g, axp_c;       // pressure Ax geometry storage and arithmetic (vectors are the fp64 GMRES basis)
    int opg_m, opg_c, conv_m, conv_c, div_m, div_c;  // SEM operators: metric storage and arithmetic
    bool need32, need16;
    int kind16;             // P16 or PBF
};

// member-wise (the struct has padding, so a byte comparison is not meaningful)
bool same_policy(const Resolved& a, const Resolved& b)
{
    return a.tv == b.tv && a.tva == b.tva && a.axv_g == b.axv_g && a.axv_c == b.axv_c && a.tpd == b.tpd &&
           a.tb == b.tb && a.axp_g == b.axp_g && a.axp_c == b.axp_c && a.opg_m == b.opg_m && a.opg_c == b.opg_c &&
           a.conv_m == b.conv_m && a.conv_c == b.conv_c && a.div_m == b.div_m && a.div_c == b.div_c &&
           a.need32 == b.need32 && a.need16 == b.need16 && a.kind16 == b.kind16;
}

// (vector, geometry, arithmetic) instantiations of the Helmholtz kernel
bool ax_supported(int u, int g, int c)
{
    // 16-bit arithmetic: geometry of that format, fp32 or same-format vectors
    if (c == P16) return g == P16 && (u == P32 || u == P16);
    if (c == PBF) return g == PBF && (u == P32 || u == PBF);
    if (u == P64) return (c == P64) || (c == P32 && g != P64);
    if (u == P32) return g != P64;
    if (u == P16) return c == P32 && g == P16;
    if (u == PBF) return c == P32 && g == PBF;
    return false;
}

// (metric storage, arithmetic) instantiations of the SEM operator kernels
bool op_supported(int m, int c)
{
    return (m == P64 && c == P64) || (m != P64 && c == P32) || (m == P32 && c == P64);
}

}  // namespace

// Gauss-Legendre points of the dealiasing grid: the n zeros of P_n by Newton
// from cos(pi (4i+3)/(4n+2)), weights 2 / ((1 - z^2) P_n'(z)^2); the GLL
// Lagrange basis at those points, I[q][l] = prod_{m != l} (z_q - x_m)/(x_l - x_m),
// and ID = I D (the derivative polynomial D u is interpolated exactly).
static void dealias_tables(int lx, const std::vector<double>& x, const std::vector<double>& D, std::vector<double>& I,
                    std::vector<double>& ID, std::vector<double>& wz)
{
    const int n = (3 * lx + 1) / 2;
    const double pi = 3.14159265358979323846;
    std::vector<double> z(n);
    wz.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double t = -std::cos(pi * (4.0 * i + 3.0) / (4.0 * n + 2.0));
        double a, b, c, da, dc;
        for (int it = 0; it < 100; ++it) {
            legendre_trio(n - 1, t, a, b, c, da, dc);  // c = P_n(t), dc = P_n'(t)
            const double dt = c / dc;
            t -= dt;
            if (std::fabs(dt) <= 1e-16) break;
        }
        legendre_trio(n - 1, t, a, b, c, da, dc);
        z[i] = t;
        wz[i] = 2.0 / ((1.0 - t * t) * dc * dc);
    }
    for (int i = 0; i < n / 2; ++i) {  // exact symmetry of nodes and weights
        const double s = 0.5 * (z[n - 1 - i] - z[i]), w = 0.5 * (wz[i] + wz[n - 1 - i]);
        z[i] = -s; z[n - 1 - i] = s;
        wz[i] = w; wz[n - 1 - i] = w;
    }
    if (n % 2) z[n / 2] = 0.0;
    I.assign((size_t)n * lx, 0.0);
    ID.assign((size_t)n * lx, 0.0);
    for (int q = 0; q < n; ++q)
        for (int l = 0; l < lx; ++l) {
            double v = 1.0;
            for (int m = 0; m < lx; ++m)
                if (m != l) v *= (z[q] - x[m]) / (x[l] - x[m]);
            I[(size_t)q * lx + l] = v;
        }
    for (int q = 0; q < n; ++q)
        for (int l = 0; l < lx; ++l) {
            double s = 0.0;
            for (int m = 0; m < lx; ++m) s += I[(size_t)q * lx + m] * D[(size_t)m * lx + l];
            ID[(size_t)q * lx + l] = s;
        }
}

// ------------------------------------------------------------------ context
struct sem_ctx {
    sem_mesh_desc mesh;
    sem_flow_desc flow;
    sem_precision prec;
    Resolved rs;
    int N, lx, E, epb, nb, vepb, nvb, pstride;
    long long np, nglob;
    std::vector<double> D64tab;
    std::vector<float> D32tab;
    std::vector<double> hsT;    // HSMG tables (flow.hsmg)
    int hs_c0[3];
    double vol;
    // layout
    size_t off_desc, off_S, off_I, off_part, off_D64, off_D32;
    size_t foff[NFIELD];
    size_t fbytes[NFIELD];
    size_t bytes;
    // bound state
    bool bound = false;
    char* dev = nullptr;
    hipStream_t stream = nullptr;
    ReqDesc* ddesc = nullptr;
    ReqDesc hdesc;
    int* hflags = nullptr;  // pinned host flags for polls
    int device = 0;         // HIP device current at sem_bind
    MeshParams mp;
    // iteration counts of the previous step: where the host first reads the
    // convergence flags (launches past convergence are gated no-ops)
    int pred_v = 4, pred_p = 4;
    // the last steps' counts, for the iteration budgets of a captured step:
    // PCG iterations (largest component), refinement cycles, and the pressure
    // iterations of the last four steps (hist_n of them valid)
    int hist_v = 0, hist_c = 0, hist_p[4] = {0, 0, 0, 0}, hist_n = 0;
};

namespace {

// Precision policy (the paper's three-level model, Sec. 2 / Fig. 4, Table 2).
// rp caps the storage role of every block and kernel (the paper's Group B
// runs fp64 compute on fp32 storage under rp = fp32, so compute and
// accumulate may exceed rp).  Kernel overrides replace their block's roles.
int resolve_policy(const sem_precision* p, Resolved& r)
{
    if (!p || p->size != (int)sizeof(sem_precision)) return fail(SEM_EINVAL, "sem_precision: bad size field");
    if (p->rp != SEM_FP64 && p->rp != SEM_FP32) return fail(SEM_EINVAL, "rp must be SEM_FP64 or SEM_FP32");
    const int rp = prec_rank(p->rp);
    if (p->rp == SEM_FP32 && (p->fp64_exceptions & SEM_X_ALL) != SEM_X_ALL)
        return fail(SEM_EINVAL, "rp = fp32 requires the fp64 exceptions STATE|GMRES|RESID|REDUCE (state, GMRES "
                                "basis and orthogonalisation, residual checks and the global reduction stage stay fp64)");
    static const char* bname[SEM_NBLOCK] = {"sem", "velocity", "pressure"};
    sem_role blk[SEM_NBLOCK];
    for (int b = 0; b < SEM_NBLOCK; ++b) {
        blk[b] = p->block[b];
        const int v[3] = {blk[b].compute, blk[b].accumulate, blk[b].storage};
        for (int q = 0; q < 3; ++q)
            if (prec_rank(v[q]) < 0) return fail(SEM_EINVAL, std::string(bname[b]) + " block: unknown precision");
        if (prec_rank(blk[b].storage) > rp) return fail(SEM_EINVAL, std::string(bname[b]) + " block: storage above rp");
        if (prec_rank(blk[b].accumulate) < prec_rank(blk[b].compute))
            return fail(SEM_EINVAL, std::string(bname[b]) + " block: accumulate below compute");
    }
    static const int kblock[SEM_K_COUNT] = {SEM_BLOCK_VEL, SEM_BLOCK_PRES, SEM_BLOCK_SEM, SEM_BLOCK_SEM, SEM_BLOCK_SEM};
    static const char* kname[SEM_K_COUNT] = {"ax_vel", "ax_pres", "opgrad", "conv", "div"};
    sem_role kr[SEM_K_COUNT];
    for (int k = 0; k < SEM_K_COUNT; ++k) {
        const sem_role& o = p->kernel[k];
        const sem_role& d = blk[kblock[k]];
        kr[k].compute = o.compute == SEM_INHERIT ? d.compute : o.compute;
        kr[k].accumulate = o.accumulate == SEM_INHERIT ? d.accumulate : o.accumulate;
        kr[k].storage = o.storage == SEM_INHERIT ? d.storage : o.storage;
        const int v[3] = {kr[k].compute, kr[k].accumulate, kr[k].storage};
        for (int q = 0; q < 3; ++q)
            if (prec_rank(v[q]) < 0) return fail(SEM_EINVAL, std::string(kname[k]) + ": unknown precision");
        if (prec_rank(kr[k].storage) > rp) return fail(SEM_EINVAL, std::string(kname[k]) + ": storage above rp");
        if (kr[k].compute == SEM_FP16 || kr[k].compute == SEM_BF16) {
            // Table 2's fp16-compute overrides (B-6, B-7): 16-bit operands, fp32 sums
            if (k != SEM_K_AX_VEL && k != SEM_K_AX_PRES)
                return fail(SEM_EINVAL, std::string(kname[k]) + ": 16-bit arithmetic is available for ax_vel and "
                                        "ax_pres only (elsewhere 16-bit work is 16-bit storage)");
            if (kr[k].storage != kr[k].compute)
                return fail(SEM_EINVAL, std::string(kname[k]) + ": 16-bit arithmetic reads geometry stored in the "
                                        "same 16-bit format");
            if (kr[k].accumulate != SEM_FP32)
                return fail(SEM_EINVAL, std::string(kname[k]) + ": 16-bit arithmetic accumulates in fp32");
        } else if (kr[k].compute != SEM_FP64 && kr[k].compute != SEM_FP32) {
            return fail(SEM_EINVAL, std::string(kname[k]) + ": unknown arithmetic");
        }
        if (prec_rank(kr[k].accumulate) < prec_rank(kr[k].compute))
            return fail(SEM_EINVAL, std::string(kname[k]) + ": accumulate below compute");
    }
    const sem_role& vb = blk[SEM_BLOCK_VEL];
    const sem_role& pb = blk[SEM_BLOCK_PRES];
    if (vb.storage != SEM_FP64 && vb.storage != SEM_FP32)
        return fail(SEM_EINVAL, "velocity block storage must be fp64 or fp32 (16-bit storage is an ax_vel override)");
    if (vb.compute != vb.storage) return fail(SEM_EINVAL, "velocity block: compute must equal storage");
    if (pb.storage != SEM_FP64 && pb.storage != SEM_FP32)
        return fail(SEM_EINVAL, "pressure block storage must be fp64 or fp32 (16-bit storage is an ax_pres override)");
    r.tv = to_pid(vb.storage);
    r.tva = to_pid(vb.accumulate);
    r.tpd = to_pid(pb.storage);
    r.tb = r.tpd;
    r.axv_g = to_pid(kr[SEM_K_AX_VEL].storage);
    r.axv_c = to_pid(kr[SEM_K_AX_VEL].compute);
    if (!ax_supported(r.tv, r.axv_g, r.axv_c))
        return fail(SEM_EINVAL, std::string("ax_vel: no kernel for vectors ") + pname(vb.storage) + ", geometry " +
                                pname(kr[SEM_K_AX_VEL].storage) + ", arithmetic " + pname(kr[SEM_K_AX_VEL].compute));
    r.axp_g = to_pid(kr[SEM_K_AX_PRES].storage);
    r.axp_c = to_pid(kr[SEM_K_AX_PRES].compute);
    if (!ax_supported(r.tb, r.axp_g, r.axp_c))
        return fail(SEM_EINVAL, std::string("ax_pres: no kernel for geometry ") + pname(kr[SEM_K_AX_PRES].storage) +
                                ", arithmetic " + pname(kr[SEM_K_AX_PRES].compute));
    int* mm[3] = {&r.opg_m, &r.conv_m, &r.div_m};
    int* cc[3] = {&r.opg_c, &r.conv_c, &r.div_c};
    for (int q = 0; q < 3; ++q) {
        const int k = SEM_K_OPGRAD + q;
        *mm[q] = to_pid(kr[k].storage);
        *cc[q] = to_pid(kr[k].compute);
        if (!op_supported(*mm[q], *cc[q]))
            return fail(SEM_EINVAL, std::string(kname[k]) + ": no kernel for this storage/arithmetic pair");
    }
    const int all[5] = {r.axv_g, r.axp_g, r.opg_m, r.conv_m, r.div_m};
    r.need32 = r.tpd == P32;
    r.need16 = false;
    r.kind16 = 0;
    for (int v : all) {
        if (v == P32) r.need32 = true;
        if (v == P16 || v == PBF) {
            if (r.need16 && r.kind16 != v) return fail(SEM_EINVAL, "one context holds a single 16-bit format (fp16 or bf16)");
            r.need16 = true;
            r.kind16 = v;
        }
    }
    return 0;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

void build_layout(sem_ctx* c)
{
    const long long np = c->np;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    c->off_desc = take(sizeof(ReqDesc));
    c->off_S = take(sizeof(double) * NSCALAR);
    c->off_I = take(sizeof(int) * NINT);
    c->off_part = take(sizeof(double) * (size_t)NRED * c->pstride);
    c->off_D64 = take(sizeof(double) * c->D64tab.size());
    c->off_D32 = take(sizeof(float) * c->D32tab.size());
    for (int f = 0; f < NFIELD; ++f) { c->foff[f] = 0; c->fbytes[f] = 0; }
    auto field = [&](int f, size_t bytes) { c->fbytes[f] = bytes; c->foff[f] = take(bytes); };
    const size_t d = 8 * (size_t)np;
    field(F_G64, 6 * d);
    field(F_B64, d);
    field(F_M64, 9 * d);
    field(F_IBSUM64, d);
    field(F_DA64, d);
    field(F_IDP64, d);
    const Resolved& r = c->rs;
    if (r.need32) {
        field(F_G32, 6 * 4 * (size_t)np);
        field(F_B32, 4 * (size_t)np);
        field(F_M32, 9 * 4 * (size_t)np);
        field(F_IDP32, 4 * (size_t)np);
    }
    if (r.need16) {
        field(F_G16, 6 * 2 * (size_t)np);
        field(F_B16, 2 * (size_t)np);
        field(F_M16, 9 * 2 * (size_t)np);
        field(F_GSC, 2 * 4 * (size_t)c->E);
        field(F_MSC, 4 * (size_t)c->E);
    }
    const int mode = c->flow.mode;
    if (mode >= SEM_MODE_POISSON) {
        field(F_V, (size_t)(c->flow.gmres_restart + 1) * psize(r.tb) * (size_t)np);
        field(F_GW, d);
        field(F_GWD, d);
        field(F_GB, d);
        field(F_GX, d);
        if (c->flow.hsmg) {
            const int lm = hs_lxm(c->lx);
            const size_t dm = 8 * (size_t)c->E * lm * lm * lm;
            const size_t nc = (size_t)c->mesh.nel[0] * c->mesh.nel[1] * c->mesh.nel[2];
            field(F_HST, 8 * (size_t)hs_off(c->lx, c->mesh.nel).total);
            field(F_HSF, d);
            field(F_HRM, dm);
            field(F_HSM, dm);
            field(F_HZM, dm);
            field(F_HC8, 8 * 8 * (size_t)c->E);
            field(F_HCA, 8 * nc);
            field(F_HCB, 8 * nc);
            field(F_HZ, psize(r.tb) * (size_t)np);
            field(F_HZS, (size_t)(c->flow.gmres_restart + 1) * psize(r.tb) * (size_t)np);
        }
    }
    if (mode >= SEM_MODE_FLUID) {
        // the pressure solve's rhs is the pressure residual itself
        c->fbytes[F_GB] = 0;
        field(F_IDV64, d);
        if (r.tv == P32) field(F_IDV32, 4 * (size_t)np);
        for (int f = F_U; f <= F_PHI; ++f) field(f, d);
        const size_t tv = psize(r.tv);
        for (int f = F_PX; f <= F_PWc; ++f) field(f, tv * np);
        c->foff[F_GB] = c->foff[F_RP];
        c->fbytes[F_GB] = c->fbytes[F_RP];
        if (c->flow.proj_dim > 0) {
            field(F_PRX, (size_t)c->flow.proj_dim * psize(r.tb) * (size_t)np);
            field(F_PRXB, d);
        }
        if (c->flow.dealias) {
            const size_t lxd = (size_t)(3 * c->lx + 1) / 2;
            const size_t nf = 9 * (size_t)c->E * lxd * lxd * lxd;
            field(F_MFD64, 8 * nf);
            if (r.conv_m == P32) field(F_MFD32, 4 * nf);
            if (r.conv_m == P16 || r.conv_m == PBF) {
                field(F_MFD16, 2 * (size_t)c->E * dl16_per_elem(c->lx));
                field(F_MFDSC, 4 * (size_t)c->E);
            }
        }
    }
    c->bytes = off;
}

semk::Batch make_batch(sem_ctx* const* ctxs, int n)
{
    semk::Batch b;
    memset(&b, 0, sizeof(b));
    b.n = n;
    b.lx = n > 0 ? ctxs[0]->lx : 0;
    b.eb[0] = 0;
    b.vb[0] = 0;
    b.el[0] = 0;
    b.hm[0] = 0;
    b.gl[0] = 0;
    b.gq[0] = 0;
    b.gate = -1;
    b.ncmax = 0;
    b.cnmax = 0;
    for (int i = 0; i < n; ++i) {
        sem_ctx* c = ctxs[i];
        b.eb[i + 1] = b.eb[i] + c->nb;
        b.vb[i + 1] = b.vb[i] + c->nvb;
        b.el[i + 1] = b.el[i] + c->E;
        {
            const int mp = hs_mepb(hs_lxm(c->lx));
            b.hm[i + 1] = b.hm[i] + (c->E + mp - 1) / mp;
        }
        b.gl[i + 1] = b.gl[i] + c->mesh.nel[1] * c->mesh.nel[2] * (c->lx - 1);
        b.gq[i + 1] = b.gq[i] + c->mesh.nel[1] * c->mesh.nel[2] * ((c->lx - 1 + 3) / 4);
        b.ncmax = std::max(b.ncmax, c->mesh.nel[0] * c->mesh.nel[1] * c->mesh.nel[2]);
        b.cnmax = std::max(b.cnmax, std::max(c->mesh.nel[1], c->mesh.nel[2]));
        b.r[i] = c->ddesc;
    }
    return b;
}

int check_hip_last()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SEM_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return 0;
}

// Iterations launched between two reads of the device convergence flags:
// the first read comes after the batch's iteration count of the previous
// step (at most 8), later ones every SEM_POLL_K (default 2) iterations.
int poll_k()
{
    static int k = -1;
    if (k < 0) {
        const char* s = getenv("SEM_POLL_K");
        k = s ? std::max(1, atoi(s)) : 2;
    }
    return k;
}

// Largest iteration limit over a batch: the host loops run until every
// request has stopped by itself (each request's own limit is applied on the
// device), so a small limit of one request never truncates another's solve.
int batch_maxit(sem_ctx* const* ctxs, int n, bool pressure)
{
    int k = 0;
    for (int i = 0; i < n; ++i) k = std::max(k, pressure ? ctxs[i]->flow.pres_maxit : ctxs[i]->flow.vel_maxit);
    return k;
}

int first_chunk(sem_ctx* const* ctxs, int n, bool pressure)
{
    int k = 1;
    for (int i = 0; i < n; ++i) k = std::max(k, pressure ? ctxs[i]->pred_p : ctxs[i]->pred_v);
    return std::min(k, 8);
}

// ------------------------------------------------------------------ event profiler
struct Prof {
    int kclass = 0;
    std::vector<hipEvent_t> ev;  // pairs
    size_t used = 0;             // events used (2 per launch)
    std::vector<hipStream_t> st;
    // A captured step cannot hold event records, so while a step is captured
    // each mark of the armed class ends the current graph segment and starts
    // the next (split_hook): the profiled launches become segments of their
    // own, and a replay records an event pair around each of them (acc).
    void (*split_hook)(void*) = nullptr;
    void* split_arg = nullptr;
    double acc_ms = 0.0;
    int64_t acc_n = 0;
};
Prof g_prof;

void prof_mark(int kclass, hipStream_t s)
{
    if (g_prof.kclass != kclass) return;
    if (g_prof.split_hook) {
        g_prof.split_hook(g_prof.split_arg);
        return;
    }
    if (g_prof.used == g_prof.ev.size()) {
        for (int q = 0; q < 256; ++q) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return;
            g_prof.ev.push_back(e);
        }
    }
    (void)hipEventRecord(g_prof.ev[g_prof.used++], s);
}

struct ProfScope {
    int k;
    hipStream_t s;
    ProfScope(int kclass, hipStream_t st) : k(kclass), s(st) { prof_mark(k, s); }
    ~ProfScope() { prof_mark(k, s); }
};

// ------------------------------------------------------------------ launch helpers
// B N(u) of the current velocity into F_BN: dealiased (3/2 rule) or collocated
void convection(const Batch& b, const sem_ctx* c, hipStream_t s)
{
    ProfScope ps(SEM_PROF_CONV, s);
    if (c->flow.dealias) launch_conv_dealias(b, c->lx, c->rs.conv_m, c->rs.conv_c, s);
    else launch_conv(b, c->lx, c->rs.conv_m, c->rs.conv_c, s);
}

void ax(const Batch& b, int lx, int src, int dst, int ncomp, int hsel, double h1, double h2, int precond, int pdot,
        int gate, int tu, int tg, int tc, hipStream_t s)
{
    AxLaunch a;
    a.src = src; a.src_vj = 0; a.dst = dst; a.ncomp = ncomp; a.hsel = hsel; a.h1 = h1; a.h2 = h2;
    a.precond = precond; a.tpc = P64; a.pdot = pdot; a.gate = gate; a.tu = tu; a.tg = tg; a.tc = tc; a.out64 = 0;
    a.u_raw = nullptr; a.w_raw = nullptr; a.sub = -1;
    launch_ax(b, lx, a, s);
}

// fin: FinOp launched right after (the scalar step consuming the partials), or -1
// R64_L = RHS_L - (h1 A + h2 B) u for the three velocity components (fp64)
void resid_ax(const Batch& b, int lx, int src, hipStream_t s)
{
    AxLaunch a;
    a.src = src; a.src_vj = 0; a.dst = F_R64; a.ncomp = 3; a.hsel = S_H1; a.h1 = 0; a.h2 = 0;
    a.precond = -1; a.tpc = P64; a.pdot = -1; a.gate = -1; a.tu = P64; a.tg = P64; a.tc = P64; a.out64 = 0;
    a.u_raw = nullptr; a.w_raw = nullptr; a.sub = F_RHS;
    launch_ax(b, lx, a, s);
}

void vec(const Batch& b, int op, int ncomp, int tv, int gate, hipStream_t s, int f0 = -1, int f1 = -1, int ta = P64,
         int tb = P64, int fin_op = -1)
{
    VecArgs a;
    a.op = op; a.gate = gate; a.ncomp = ncomp; a.tv = tv; a.ta = ta; a.tb = tb; a.f0 = f0; a.f1 = f1; a.a = 0.0;
    a.x_raw = nullptr; a.y_raw = nullptr;
    launch_vec(b, a, s);
    if (fin_op >= 0) {
        FinArgs f;
        f.op = fin_op; f.gate = -1; f.ncomp = 1; f.f0 = 0; f.host_flags = nullptr; f.host_stats = nullptr;
        f.gate2 = -1;
        launch_fin(b, f, s);
    }
}

void fin(const Batch& b, int op, hipStream_t s, int gate = -1, int ncomp = 1, int* flags = nullptr, int f0 = 0,
         int gate2 = -1)
{
    FinArgs a;
    a.op = op; a.gate = gate; a.ncomp = ncomp; a.f0 = f0; a.host_flags = flags; a.host_stats = nullptr;
    a.gate2 = gate2;
    launch_fin(b, a, s);
}

// poll: returns number of requests whose flag (any component) is set, or <0 on error
int poll(const Batch& b, int gate, int ncomp, int* hflags, hipStream_t s)
{
    fin(b, FIN_POLL, s, gate, ncomp, hflags);
    int rc = check_hip_last();
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(SEM_EHIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
    int cnt = 0;
    for (int i = 0; i < b.n; ++i) cnt += hflags[i] != 0;
    return cnt;
}

// One Jacobi-PCG iteration of the three velocity components of every request
// (gated per component on I_VACT: converged components idle)
void pcg_iteration(const Batch& b, int lx, const Resolved& r, int tv, hipStream_t s)
{
    {
        ProfScope ps(SEM_PROF_AX_VEL, s);
        // alpha = rho / (p, w): the dot of a continuous p with dssum(w_L)
        // equals the plain local sum of p w_L, formed before the dssum
        ax(b, lx, F_PP, F_PW, 3, S_H1, 0, 0, -1, R_A, I_VACT, tv, r.axv_g, r.axv_c, s);
    }
    launch_dssum(b, F_PW, 3, tv, I_VACT, nullptr, s);
    fin(b, FIN_PCG_ALPHA, s);
    vec(b, V_PCG_UPD, 3, tv, I_VACT, s, -1, -1, r.tva, P64, FIN_PCG_BETA);
    vec(b, V_PCG_P, 3, tv, I_VACT, s);
}

// Jacobi-PCG on the assembled velocity Helmholtz operator for the three
// components of every request: solves H x_c = R64_c in the velocity storage
// precision; on return US_c += x_c.  With fp32 vectors the residual is
// recomputed in fp64 from US and further correction solves run until the
// fp64 residual meets the tolerance (or the refinement limit).
int velocity_solve(sem_ctx* const* ctxs, const Batch& b, hipStream_t s)
{
    sem_ctx* c0 = ctxs[0];
    const int lx = c0->lx;
    const Resolved& r = c0->rs;
    const int tv = r.tv;
    int* hf = c0->hflags;
    // fp64 residual of the current state: R64 = dssum(RHS_L - H_L U) (the
    // local rhs is not assembled on its own); the gather-scatter also forms
    // the norms over unique nodes, and the finaliser sets VACT
    {
        ProfScope ps(SEM_PROF_AX_RESID, s);
        resid_ax(b, lx, F_U, s);
    }
    launch_dssum(b, F_R64, 3, P64, -1, nullptr, s, R_A);
    fin(b, FIN_VINIT, s);
    const int vmax = batch_maxit(ctxs, b.n, false);
    int maxref = 0;
    for (int i = 0; i < b.n; ++i) maxref = std::max(maxref, ctxs[i]->flow.vel_max_refine);
    for (int cyc = 0; cyc < maxref; ++cyc) {
        if (cyc > 0) {
            // the first cycle runs without a read: if the initial residual
            // already meets the tolerance its launches are gated no-ops
            int act = poll(b, I_VACT, 3, hf, s);
            if (act < 0) return act;
            if (act == 0) break;
        }
        vec(b, V_PCG_INIT, 3, tv, -1, s, -1, -1, r.tva, P64, FIN_PCG_RHO);
        int K = first_chunk(ctxs, b.n, false);
        int guard = 0;
        for (;;) {
            for (int q = 0; q < K; ++q) pcg_iteration(b, lx, r, tv, s);
            guard += K;
            K = poll_k();
            int a2 = poll(b, I_VACT, 3, hf, s);
            if (a2 < 0) return a2;
            if (a2 == 0 || guard > vmax + K) break;
        }
        vec(b, V_US_ADD, 3, tv, -1, s, cyc == 0 ? 1 : 0);
        if (tv == P64) break;  // fp64 recurrence residual is the solver's stop criterion
        {
            ProfScope ps(SEM_PROF_AX_RESID, s);
            resid_ax(b, lx, F_US, s);
        }
        launch_dssum(b, F_R64, 3, P64, -1, nullptr, s, R_A);
        fin(b, FIN_VINIT, s);
    }
    return check_hip_last();
}

// Cycle end of GMRES(m), gated on requests whose cycle ended: x update, fp64
// true residual (no operator while x is still zero), then restart or finish.
void gmres_cycle_end(const Batch& b, int lx, const Resolved& r, bool hsmg, hipStream_t s)
{
    if (hsmg) {
        // x += M^{-1} V y = sum_j y_j Z_j with the Z_j = M^{-1} s_j V_j of the Arnoldi steps
        vec(b, V_GM_XZ, 1, P64, I_GEND, s, -1, -1, P64, r.tb);
    } else {
        vec(b, V_GM_XUPD, 1, r.tpd, I_GEND, s, -1, -1, P64, r.tb);
    }
    {
        ProfScope ps(SEM_PROF_AX_PRESID, s);
        ax(b, lx, F_GX, F_GWD, 1, -1, 1.0, 0.0, -1, -1, I_GENDAX, P64, P64, P64, s);
    }
    launch_dssum(b, F_GWD, 1, P64, I_GENDAX, nullptr, s);
    vec(b, V_GM_RESID, 1, P64, I_GEND, s, -1, -1, P64, r.tb, FIN_GM_RESTART);
}

// One Arnoldi step of GMRES(m); every kernel is gated so requests whose
// cycle ended (or that converged) idle until the next cycle end.
void gmres_arnoldi(const Batch& b, int lx, const Resolved& r, bool hsmg, hipStream_t s)
{
    if (hsmg) {
        // w = A M^{-1} V_J with z = M^{-1} V_J in HZ (basis storage precision)
        {
            ProfScope ps(SEM_PROF_HSMG, s);
            launch_hsmg(b, lx, r.tb, I_GARN, s);
        }
        ProfScope ps(SEM_PROF_AX_PRES, s);
        AxLaunch a;
        a.src = F_HZ; a.src_vj = 0; a.dst = F_GW; a.ncomp = 1; a.hsel = -1; a.h1 = 1.0; a.h2 = 0.0;
        a.precond = -1; a.tpc = P64; a.pdot = -1; a.gate = I_GARN;
        a.tu = r.tb; a.tg = r.axp_g; a.tc = r.axp_c; a.u_raw = nullptr; a.w_raw = nullptr;
        a.out64 = 1; a.sub = -1;
        launch_ax(b, lx, a, s);
    } else {
        // w = A M^{-1} V_J: the Jacobi scaling is applied while loading V_J
        ProfScope ps(SEM_PROF_AX_PRES, s);
        AxLaunch a;
        a.src = -1; a.src_vj = 1; a.dst = F_GW; a.ncomp = 1; a.hsel = -1; a.h1 = 1.0; a.h2 = 0.0;
        a.precond = r.tpd == P64 ? F_IDP64 : F_IDP32; a.tpc = r.tpd; a.pdot = -1; a.gate = I_GARN;
        a.tu = r.tb; a.tg = r.axp_g; a.tc = r.axp_c; a.u_raw = nullptr; a.w_raw = nullptr;
        a.out64 = 1; a.sub = -1;
        launch_ax(b, lx, a, s);
    }
    {
        ProfScope ps(SEM_PROF_DSSUM_PRES, s);
        launch_dssum(b, F_GW, 1, P64, I_GARN, nullptr, s);
    }
    {
        ProfScope ps(SEM_PROF_GM_DOTS, s);
        vec(b, V_GM_DOTS, 1, P64, I_GARN, s, -1, -1, P64, r.tb, FIN_GM_H1);
    }
    {
        ProfScope ps(SEM_PROF_GM_UPD_DOTS, s);
        vec(b, V_GM_UPD_DOTS, 1, P64, I_GARN, s, -1, -1, P64, r.tb, FIN_GM_H2);
    }
    {
        ProfScope ps(SEM_PROF_GM_UPD_NORM, s);
        vec(b, V_GM_UPD_NORM, 1, P64, I_GARN, s, -1, -1, P64, r.tb, FIN_GM_COL);
    }
}

// GMRES on F_GB -> F_GX in three pieces so a serving loop can change the
// batch between iteration chunks (all solver state is per request, on the
// device): start (GX zeroed by the caller), advance by up to max_iters Arnoldi
// steps, finish (mass-mean removal of GX).
// Start: the first cycle end runs at once (r = b, beta, V_0 = r / beta).
void gmres_start(const Batch& b, int lx, const Resolved& r, bool hsmg, hipStream_t s)
{
    fin(b, FIN_GM_START, s);
    gmres_cycle_end(b, lx, r, hsmg, s);
}

// Advance by up to max_iters Arnoldi steps; returns the number of requests
// still iterating, or a negative status.  lockstep: every request of the
// batch started its solve together, so all active ones reach J + 1 = m at
// the same step: the cycle-end kernels then run only where a restart is due
// and before each read of the convergence flags (a request whose cycle ended
// earlier idles, gated, until then).  Otherwise (requests that joined at
// different times) the cycle end follows every Arnoldi step.
int gmres_advance(sem_ctx* const* ctxs, const Batch& b, hipStream_t s, int max_iters, bool lockstep)
{
    sem_ctx* c0 = ctxs[0];
    const int m = c0->flow.gmres_restart;
    int K = first_chunk(ctxs, b.n, true);
    int done = 0, act = 0, since = 0;
    while (done < max_iters) {
        const int k = std::min(K, max_iters - done);
        for (int q = 0; q < k; ++q) {
            gmres_arnoldi(b, c0->lx, c0->rs, c0->flow.hsmg != 0, s);
            ++since;
            if (!lockstep || since == m || q == k - 1) {
                gmres_cycle_end(b, c0->lx, c0->rs, c0->flow.hsmg != 0, s);
                if (since == m) since = 0;
            }
        }
        done += k;
        K = poll_k();
        act = poll(b, I_GACT, 1, c0->hflags, s);
        if (act <= 0) return act;
    }
    return act;
}

void gmres_finish(const Batch& b, hipStream_t s)
{
    vec(b, V_SUM_MASS, 1, P64, -1, s, F_GX, -1, P64, P64, FIN_MEAN_MASS);
    vec(b, V_SUB_MEAN, 1, P64, -1, s, F_GX, -1);
}

// Projection of the pressure increment onto earlier ones (the pressure
// solver's projection space of Sec. 3): before the solve, the guess
// GX = sum_i (X_i, b) X_i over the A-orthonormal stored vectors, from which
// GMRES starts (its first cycle end forms b - A GX in fp64).
void projection_guess(const Batch& b, const Resolved& r, hipStream_t s)
{
    vec(b, V_PR_ADOTS, 1, P64, -1, s, -1, -1, P64, r.tb, FIN_PR_ALPHA);
    vec(b, V_PR_GUESS, 1, P64, -1, s, -1, -1, P64, r.tb);
}

// After the solve: the correction GX - guess (the whole GX when the space is
// full and restarts) is A-orthogonalised against the space with the fp64
// operator and appended unless dependent.  gate: I index that must be nonzero
// for a request to update its space (the commit flag of a captured step), or -1.
void projection_update(const Batch& b, int lx, const Resolved& r, hipStream_t s, int gate = -1)
{
    fin(b, FIN_PR_POST, s, -1, 1, nullptr, 0, gate);
    vec(b, V_PR_V, 1, P64, gate, s);
    {
        ProfScope ps(SEM_PROF_AX_PRESID, s);
        ax(b, lx, F_GW, F_GWD, 1, -1, 1.0, 0.0, -1, -1, gate, P64, P64, P64, s);
    }
    launch_dssum(b, F_GWD, 1, P64, gate, nullptr, s);
    vec(b, V_PR_BDOTS, 1, P64, gate, s, -1, -1, P64, r.tb);
    fin(b, FIN_PR_BETA, s, -1, 1, nullptr, 0, gate);
    // (FIN_COMMIT_CHECK cleared I_PRADD where the step is not committed)
    vec(b, V_PR_ORTH, 1, P64, I_PRADD, s, -1, -1, P64, r.tb);
    fin(b, FIN_PR_COMMIT, s, -1, 1, nullptr, 0, gate);
}

// use_proj: the fluid step's pressure solve updates the projection space of
// its contexts; stand-alone Poisson solves leave it alone
int pressure_solve(sem_ctx* const* ctxs, const Batch& b, hipStream_t s, bool use_proj)
{
    sem_ctx* c0 = ctxs[0];
    const int m = c0->flow.gmres_restart;
    const int pmax = batch_maxit(ctxs, b.n, true);
    const int limit = pmax + pmax / std::max(1, m) + 4;
    const bool proj = use_proj && c0->flow.mode == SEM_MODE_FLUID && c0->flow.proj_dim > 0;
    gmres_start(b, c0->lx, c0->rs, c0->flow.hsmg != 0, s);
    int rc = gmres_advance(ctxs, b, s, limit, true);
    if (rc < 0) return rc;
    if (proj) projection_update(b, c0->lx, c0->rs, s);
    gmres_finish(b, s);
    return check_hip_last();
}

void graph_forget(const sem_ctx* c);  // cached step graphs of c (defined with them below)

int bind_check(sem_ctx* c)
{
    if (!c) return fail(SEM_EINVAL, "null context");
    if (!c->bound) return fail(SEM_ESTATE, "context is not bound");
    return 0;
}

}  // namespace

// ------------------------------------------------------------------ C ABI
extern "C" {

const char* sem_strerror(int status)
{
    switch (status) {
    case SEM_OK: return "ok";
    case SEM_EINVAL: return "invalid argument";
    case SEM_ENOMEM: return "workspace too small";
    case SEM_EHIP: return "HIP runtime error";
    case SEM_ENAN: return "non-finite value in a solve";
    case SEM_ENOTCONV: return "solver did not converge";
    case SEM_ESTATE: return "invalid state";
    default: return "unknown status";
    }
}

const char* sem_last_error(void) { return g_err.c_str(); }

int sem_setup(const sem_mesh_desc* mesh, const sem_flow_desc* flow, const sem_precision* prec, sem_ctx** out)
{
    if (!mesh || !flow || !prec || !out) return fail(SEM_EINVAL, "null argument");
    *out = nullptr;
    if (mesh->size != (int)sizeof(sem_mesh_desc)) return fail(SEM_EINVAL, "sem_mesh_desc: bad size field");
    if (flow->size != (int)sizeof(sem_flow_desc)) return fail(SEM_EINVAL, "sem_flow_desc: bad size field");
    if (mesh->order < 2 || mesh->order > 11) return fail(SEM_EINVAL, "order must be in 2..11");
    long long E = 1;
    for (int d = 0; d < 3; ++d) {
        if (mesh->nel[d] < 1) return fail(SEM_EINVAL, "element counts must be >= 1");
        if (!(mesh->hi[d] > mesh->lo[d])) return fail(SEM_EINVAL, "hi must exceed lo");
        if (mesh->deform_amp != 0.0 && mesh->nel[d] % 2) return fail(SEM_EINVAL, "a perturbed mesh needs even element counts");
        E *= mesh->nel[d];
    }
    const long long lx = mesh->order + 1;
    if (E * lx * lx * lx >= (1LL << 31)) return fail(SEM_EINVAL, "more than 2^31 local points");
    // the gather-scatter addresses a line of elements along x with 32-bit byte offsets
    if (mesh->nel[0] * lx * lx * lx * 8 >= (1LL << 32))
        return fail(SEM_EINVAL, "more than 2^29 local points along one line of elements in x");
    if (!(std::fabs(mesh->deform_amp) < 0.25)) return fail(SEM_EINVAL, "deform_amp must be below 0.25 (positive Jacobian)");
    if (flow->mode < SEM_MODE_OPERATOR || flow->mode > SEM_MODE_FLUID) return fail(SEM_EINVAL, "bad mode");
    if (flow->mode >= SEM_MODE_POISSON) {
        if (flow->gmres_restart < 1 || flow->gmres_restart > SEM_MAXM) return fail(SEM_EINVAL, "gmres_restart must be 1..30");
        if (!(flow->pres_tol > 0) || flow->pres_maxit < 1) return fail(SEM_EINVAL, "bad pressure tolerance/limit");
    }
    if (flow->mode == SEM_MODE_FLUID) {
        if (!(flow->nu > 0) || !(flow->dt > 0)) return fail(SEM_EINVAL, "nu and dt must be positive");
        if (flow->torder < 1 || flow->torder > 3) return fail(SEM_EINVAL, "torder must be 1..3");
        if (!(flow->vel_tol > 0) || flow->vel_maxit < 1 || flow->vel_max_refine < 1)
            return fail(SEM_EINVAL, "bad velocity tolerance/limits");
        if (flow->init < SEM_INIT_ZERO || flow->init > SEM_INIT_TGV2D) return fail(SEM_EINVAL, "bad init");
        if (flow->proj_dim < 0 || flow->proj_dim > SEM_MAX_PROJ) return fail(SEM_EINVAL, "proj_dim must be 0..20");
        if (flow->dealias != 0 && flow->dealias != 1) return fail(SEM_EINVAL, "dealias must be 0 or 1");
        if (!(flow->cfl_target >= 0.0) || !std::isfinite(flow->cfl_target))
            return fail(SEM_EINVAL, "cfl_target must be finite and >= 0");
    } else if (flow->proj_dim != 0) {
        return fail(SEM_EINVAL, "proj_dim applies to the fluid mode only");
    } else if (flow->dealias != 0) {
        return fail(SEM_EINVAL, "dealias applies to the fluid mode only");
    } else if (flow->cfl_target != 0.0) {
        return fail(SEM_EINVAL, "cfl_target applies to the fluid mode only");
    }
    Resolved rs;
    int rc = resolve_policy(prec, rs);
    if (rc) return rc;
    if (flow->hsmg != 0 && flow->hsmg != 1) return fail(SEM_EINVAL, "hsmg must be 0 or 1");
    if (flow->hsmg) {
        if (flow->mode < SEM_MODE_POISSON) return fail(SEM_EINVAL, "hsmg applies to the Poisson and fluid modes");
        if (mesh->deform_amp != 0.0) return fail(SEM_EINVAL, "hsmg needs an unperturbed box mesh");
        if (mesh->order < 4) return fail(SEM_EINVAL, "hsmg needs order >= 4");
        for (int d = 0; d < 3; ++d)
            if (mesh->nel[d] < 2 || mesh->nel[d] > HS_NELMAX)
                return fail(SEM_EINVAL, "hsmg needs 2..64 elements per direction");
        if (rs.tb != P64 && rs.tb != P32) return fail(SEM_EINVAL, "hsmg needs an fp64 or fp32 pressure basis");
    }

    sem_ctx* c = new sem_ctx();
    c->mesh = *mesh;
    c->flow = *flow;
    c->prec = *prec;
    c->rs = rs;
    c->N = mesh->order;
    c->lx = (int)lx;
    c->E = (int)E;
    c->np = E * lx * lx * lx;
    c->nglob = E * (long long)mesh->order * mesh->order * mesh->order;
    c->epb = epb_of(c->lx);
    c->nb = (int)((E + c->epb - 1) / c->epb);
    c->vepb = vepb_of(c->lx, c->E);
    c->nvb = (c->E + c->vepb - 1) / c->vepb;
    // partials come from element blocks, point-wise blocks and gather-scatter workgroups
    c->pstride = std::max(std::max(c->nb, c->nvb), gs_blocks(c->lx, mesh->nel[1], mesh->nel[2]));
    if (c->nb > c->pstride || c->nvb > c->pstride || (long long)c->nb * c->epb < c->E ||
        (long long)c->nvb * c->vepb < c->E) {
        delete c;
        return fail(SEM_EINVAL, "internal block layout inconsistent");
    }
    std::vector<double> x, w, D;
    gll_tables(c->N, x, w, D);
    // fp64 table: D (lx*lx), GLL weights, GLL nodes, then 1/multiplicity of
    // every local point of a conforming box mesh (lx^3; a face coordinate
    // doubles the number of copies), then the dealiasing tables I, ID (lxd*lx
    // each) and the Gauss-Legendre weights (lxd); fp32 table: D, weights,
    // nodes, I, ID, Gauss-Legendre weights
    std::vector<double> dI, dID, dwz;
    dealias_tables((int)lx, x, D, dI, dID, dwz);
    std::vector<double> dl(dI);
    dl.insert(dl.end(), dID.begin(), dID.end());
    dl.insert(dl.end(), dwz.begin(), dwz.end());
    c->D64tab.resize(lx * lx + 2 * lx + lx * lx * lx);
    for (int q = 0; q < lx * lx; ++q) c->D64tab[q] = D[q];
    for (int q = 0; q < lx; ++q) { c->D64tab[lx * lx + q] = w[q]; c->D64tab[lx * lx + lx + q] = x[q]; }
    c->D32tab.resize(lx * lx + 2 * lx);
    for (size_t q = 0; q < c->D32tab.size(); ++q) c->D32tab[q] = (float)c->D64tab[q];
    for (int k = 0; k < lx; ++k)
        for (int j = 0; j < lx; ++j)
            for (int i = 0; i < lx; ++i) {
                double r = 1.0;
                if (i == 0 || i == lx - 1) r *= 0.5;
                if (j == 0 || j == lx - 1) r *= 0.5;
                if (k == 0 || k == lx - 1) r *= 0.5;
                c->D64tab[lx * lx + 2 * lx + i + lx * (j + lx * k)] = r;
            }
    c->D64tab.insert(c->D64tab.end(), dl.begin(), dl.end());
    for (double v : dl) c->D32tab.push_back((float)v);
    build_layout(c);
    MeshParams& mp = c->mp;
    for (int d = 0; d < 3; ++d) {
        mp.nel[d] = mesh->nel[d];
        mp.lo[d] = mesh->lo[d];
        mp.h[d] = (mesh->hi[d] - mesh->lo[d]) / mesh->nel[d];
    }
    mp.N = c->N;
    mp.amp = mesh->deform_amp;
    for (int q = 0; q < 9; ++q) mp.phase[q] = mesh->deform_phase[q];
    if (flow->hsmg) hsmg_tables(c->N, mesh->nel, mp.h, c->hsT, c->hs_c0);
    *out = c;
    return 0;
}

size_t sem_workspace_bytes(const sem_ctx* ctx) { return ctx ? ctx->bytes : 0; }

int sem_sizes(const sem_ctx* c, int64_t* np, int64_t* nglob, int* lx, int* nelem)
{
    if (!c) return fail(SEM_EINVAL, "null context");
    if (np) *np = c->np;
    if (nglob) *nglob = c->nglob;
    if (lx) *lx = c->lx;
    if (nelem) *nelem = c->E;
    return 0;
}

int sem_bind(sem_ctx* c, void* dev_buf, size_t bytes, void* hip_stream)
{
    std::lock_guard<std::recursive_mutex> lk(g_host_mu);
    if (!c || !dev_buf) return fail(SEM_EINVAL, "null argument");
    if (c->bound) return fail(SEM_ESTATE, "context already bound");
    if (bytes < c->bytes) return fail(SEM_ENOMEM, "workspace smaller than sem_workspace_bytes");
    if (((uintptr_t)dev_buf) & 255) return fail(SEM_EINVAL, "workspace must be 256-byte aligned");
    c->dev = (char*)dev_buf;
    c->stream = (hipStream_t)hip_stream;
    HIPCHK(hipGetDevice(&c->device));
    hipStream_t s = c->stream;
    ReqDesc& d = c->hdesc;
    memset(&d, 0, sizeof(d));
    d.E = c->E; d.lx = c->lx; d.epb = c->epb; d.nb = c->nb; d.vepb = c->vepb; d.nvb = c->nvb;
    d.pstride = c->pstride;
    if (c->nb > c->pstride || c->nvb > c->pstride || (long long)c->nb * c->epb < c->E || (long long)c->nvb * c->vepb < c->E)
        return fail(SEM_EINVAL, "internal block layout inconsistent");
    d.prec16 = c->rs.need16 ? c->rs.kind16 : 0;
    d.gm_m = c->flow.gmres_restart;
    d.proj_L = c->flow.mode == SEM_MODE_FLUID ? c->flow.proj_dim : 0;
    for (int q = 0; q < 3; ++q) d.nel[q] = c->mesh.nel[q];
    d.hs = c->flow.hsmg;
    for (int q = 0; q < 3; ++q) d.hs_c0[q] = c->flow.hsmg ? c->hs_c0[q] : 0;
    d.np = c->np; d.nglob = c->nglob;
    d.S = (double*)(c->dev + c->off_S);
    d.I = (int*)(c->dev + c->off_I);
    d.part = (double*)(c->dev + c->off_part);
    d.D64 = (const double*)(c->dev + c->off_D64);
    d.D32 = (const float*)(c->dev + c->off_D32);
    for (int f = 0; f < NFIELD; ++f) d.f[f] = c->fbytes[f] ? (void*)(c->dev + c->foff[f]) : nullptr;
    c->ddesc = (ReqDesc*)(c->dev + c->off_desc);

    // scalars and integer state
    std::vector<double> S(NSCALAR, 0.0);
    std::vector<int> I(NINT, 0);
    S[S_NU] = c->flow.nu;
    S[S_DT] = c->flow.dt;
    S[S_DTMAX] = c->flow.dt;
    S[S_CFLT] = c->flow.mode == SEM_MODE_FLUID ? c->flow.cfl_target : 0.0;
    S[S_VTOL] = c->flow.vel_tol;
    S[S_PTOL] = c->flow.pres_tol;
    S[S_H1] = 1.0;
    I[I_TORDER] = c->flow.torder;
    I[I_VMAXIT] = c->flow.vel_maxit;
    I[I_VMAXREF] = c->flow.vel_max_refine;
    I[I_PRL] = 0;
    I[I_GMAXIT] = c->flow.pres_maxit;
    I[I_GM] = c->flow.gmres_restart;
    I[I_ALWAYS] = 1;
    HIPCHK(hipHostMalloc((void**)&c->hflags, sizeof(int) * SEM_MAXB, hipHostMallocDefault));
    HIPCHK(hipMemcpyAsync(c->ddesc, &d, sizeof(d), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d.S, S.data(), sizeof(double) * NSCALAR, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d.I, I.data(), sizeof(int) * NINT, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync((void*)d.D64, c->D64tab.data(), sizeof(double) * c->D64tab.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync((void*)d.D32, c->D32tab.data(), sizeof(float) * c->D32tab.size(), hipMemcpyHostToDevice, s));
    if (c->flow.hsmg)
        HIPCHK(hipMemcpyAsync(d.f[F_HST], c->hsT.data(), sizeof(double) * c->hsT.size(), hipMemcpyHostToDevice, s));
    // the copies read pageable host memory: finish them before returning
    HIPCHK(hipStreamSynchronize(s));
    c->bound = true;

    sem_ctx* one[1] = {c};
    Batch b = make_batch(one, 1);
    launch_geometry(b, c->lx, c->mp, s);
    launch_diag_a(b, c->lx, s);
    launch_dssum(b, F_DA64, 1, P64, -1, nullptr, s);
    HIPCHK(hipMemcpyAsync(d.f[F_IBSUM64], d.f[F_B64], 8 * (size_t)c->np, hipMemcpyDeviceToDevice, s));
    launch_dssum(b, F_IBSUM64, 1, P64, -1, nullptr, s);
    launch_geo_post(b, s);
    if (c->rs.need32 || c->rs.need16) launch_geo_cast(b, c->lx, c->rs.need32 ? 1 : 0, c->rs.need16 ? c->rs.kind16 : 0, s);
    if (c->flow.mode == SEM_MODE_FLUID && c->flow.dealias)
        launch_dealias_geom(b, c->lx, c->mp, c->rs.conv_m == P32,
                            (c->rs.conv_m == P16 || c->rs.conv_m == PBF) ? c->rs.conv_m : 0, s);
    // domain volume (sum of B)
    vec(b, V_SUM_MASS, 1, P64, -1, s, -1, -1, P64, P64, FIN_VOL);
    int rc = check_hip_last();
    if (rc) return rc;
    if (c->flow.mode == SEM_MODE_FLUID) {
        launch_init_fields(b, c->lx, c->flow.init, c->mp, s);
        // history of the convective term starts at the initial field
        convection(b, c, s);
        vec(b, V_COPY, 3, P64, -1, s, F_BN, F_BNL1);
        vec(b, V_COPY, 3, P64, -1, s, F_BN, F_BNL2);
        // diagnostics of the initial field (also its CFL rate for the first step)
        launch_diagnostics(b, c->lx, s);
        fin(b, FIN_DIAG, s);
        rc = check_hip_last();
        if (rc) return rc;
    }
    HIPCHK(hipStreamSynchronize(s));
    int nanflag = 0;
    HIPCHK(hipMemcpyAsync(&nanflag, d.I + I_NAN, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (nanflag) return fail(SEM_EINVAL, "non-positive Jacobian in the mesh");
    return 0;
}

int sem_set_stream(sem_ctx* c, void* hip_stream)
{
    std::lock_guard<std::recursive_mutex> lk(g_host_mu);
    if (!c) return fail(SEM_EINVAL, "null argument");
    if (!c->bound) return fail(SEM_ESTATE, "context not bound");
    c->stream = (hipStream_t)hip_stream;
    return 0;
}

void sem_destroy(sem_ctx* c)
{
    if (!c) return;
    std::lock_guard<std::recursive_mutex> lk(g_host_mu);
    graph_forget(c);
    if (c->hflags) (void)hipHostFree(c->hflags);
    delete c;
}

}  // extern "C"

namespace {

int field_of(const sem_ctx* c, int which, int& fid)
{
    if (which >= SEM_F_U && which < SEM_F_U + 3) fid = F_U + (which - SEM_F_U);
    else if (which == SEM_F_P) fid = F_P;
    else if (which >= SEM_F_ULAG1 && which < SEM_F_ULAG1 + 3) fid = F_UL1 + (which - SEM_F_ULAG1);
    else if (which >= SEM_F_ULAG2 && which < SEM_F_ULAG2 + 3) fid = F_UL2 + (which - SEM_F_ULAG2);
    else if (which >= SEM_F_BNLAG1 && which < SEM_F_BNLAG1 + 3) fid = F_BNL1 + (which - SEM_F_BNLAG1);
    else if (which >= SEM_F_BNLAG2 && which < SEM_F_BNLAG2 + 3) fid = F_BNL2 + (which - SEM_F_BNLAG2);
    else if (which == SEM_F_MASS) fid = F_B64;
    else if (which == SEM_F_BSUM) fid = F_IBSUM64;
    else if (which >= SEM_F_G && which < SEM_F_G + 6) fid = F_G64;
    else if (which >= SEM_F_M && which < SEM_F_M + 9) fid = F_M64;
    else if (which == SEM_F_DIAG_A) fid = F_DA64;
    else return fail(SEM_EINVAL, "unknown field");
    if (!c->fbytes[fid]) return fail(SEM_EINVAL, "field not present in this context's mode");
    return 0;
}

// current device pointer of a field (state fields rotate on the device)
int current_ptr(sem_ctx* c, int fid, char** out)
{
    void* p = nullptr;
    HIPCHK(hipMemcpyAsync(&p, &c->ddesc->f[fid], sizeof(void*), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    *out = (char*)p;
    return 0;
}

}  // namespace

extern "C" {

int sem_ax(sem_ctx* c, const void* u, void* w, double h1, double h2, int buf_prec, int geom_prec, int flags)
{
    int rc = bind_check(c);
    if (rc) return rc;
    if (!u || !w) return fail(SEM_EINVAL, "null field pointer");
    if (buf_prec < SEM_FP64 || buf_prec > SEM_BF16) return fail(SEM_EINVAL, "bad buf_prec");
    int tg;
    if (geom_prec == SEM_INHERIT) tg = h2 == 0.0 ? c->rs.axp_g : c->rs.axv_g;
    else if (geom_prec >= SEM_FP64 && geom_prec <= SEM_BF16) tg = to_pid(geom_prec);
    else return fail(SEM_EINVAL, "bad geom_prec");
    const int tu = to_pid(buf_prec);
    bool held = tg == P64 || (tg == P32 && c->rs.need32) || ((tg == P16 || tg == PBF) && c->rs.need16 && c->rs.kind16 == tg);
    if (!held) return fail(SEM_EINVAL, "the requested geometry precision is not held by this context");
    int tc = (tu == P64 && !(flags & SEM_AX_FP32_COMPUTE)) ? P64 : P32;
    if (flags & SEM_AX_16BIT_COMPUTE) {
        if (tg != P16 && tg != PBF) return fail(SEM_EINVAL, "SEM_AX_16BIT_COMPUTE needs 16-bit geometry");
        tc = tg;
    }
    if (!ax_supported(tu, tg, tc)) return fail(SEM_EINVAL, "unsupported (vector, geometry, arithmetic) combination for Ax");
    sem_ctx* one[1] = {c};
    Batch b = make_batch(one, 1);
    AxLaunch a;
    a.src = -1; a.src_vj = 0; a.dst = -1; a.ncomp = 1; a.hsel = -1; a.h1 = h1; a.h2 = h2;
    a.precond = -1; a.tpc = P64; a.pdot = -1; a.gate = -1; a.tu = tu; a.tg = tg; a.tc = tc; a.out64 = 0;
    a.u_raw = u; a.w_raw = w; a.sub = -1;
    {
        ProfScope ps(SEM_PROF_AX_ANY, c->stream);
        launch_ax(b, c->lx, a, c->stream);
    }
    if (flags & SEM_ASSEMBLE) launch_dssum(b, -1, 1, tu, -1, w, c->stream);
    return check_hip_last();
}

int sem_dssum(sem_ctx* c, void* u, int buf_prec)
{
    int rc = bind_check(c);
    if (rc) return rc;
    if (!u) return fail(SEM_EINVAL, "null field pointer");
    if (buf_prec < SEM_FP64 || buf_prec > SEM_BF16) return fail(SEM_EINVAL, "bad buf_prec");
    sem_ctx* one[1] = {c};
    Batch b = make_batch(one, 1);
    launch_dssum(b, -1, 1, to_pid(buf_prec), -1, u, c->stream);
    return check_hip_last();
}

static int check_batch(sem_ctx* const* ctxs, int n, int min_mode)
{
    if (!ctxs || n < 1 || n > SEM_MAXB) return fail(SEM_EINVAL, "batch size must be 1..48");
    for (int i = 0; i < n; ++i) {
        int rc = bind_check(ctxs[i]);
        if (rc) return rc;
        if (ctxs[i]->flow.mode < min_mode) return fail(SEM_EINVAL, "context mode does not hold the needed workspaces");
        if (ctxs[i]->lx != ctxs[0]->lx) return fail(SEM_EINVAL, "batched contexts must share the order");
        if (!same_policy(ctxs[i]->rs, ctxs[0]->rs))
            return fail(SEM_EINVAL, "batched contexts must share the precision policy");
        if (ctxs[i]->stream != ctxs[0]->stream) return fail(SEM_EINVAL, "batched contexts must share the stream");
        if (ctxs[i]->flow.gmres_restart != ctxs[0]->flow.gmres_restart)
            return fail(SEM_EINVAL, "batched contexts must share the GMRES restart length");
        if (ctxs[i]->flow.proj_dim != ctxs[0]->flow.proj_dim)
            return fail(SEM_EINVAL, "batched contexts must share the projection dimension");
        if (ctxs[i]->flow.dealias != ctxs[0]->flow.dealias)
            return fail(SEM_EINVAL, "batched contexts must share the dealiasing setting");
        if ((ctxs[i]->flow.cfl_target > 0.0) != (ctxs[0]->flow.cfl_target > 0.0))
            return fail(SEM_EINVAL, "batched contexts must all use fixed or all adaptive dt");
        if (ctxs[i]->flow.hsmg != ctxs[0]->flow.hsmg)
            return fail(SEM_EINVAL, "batched contexts must use the same pressure preconditioner");
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return fail(SEM_EINVAL, "a context appears twice in a batch");
    }
    return 0;
}

}  // extern "C"

namespace {

// pinned host buffer the statistics kernel writes (one per host thread, so
// batches on different streams can step from different threads)
double* stats_buffer()
{
    thread_local double* buf = nullptr;
    if (!buf) {
        std::lock_guard<std::recursive_mutex> lk(g_host_mu);
        if (hipHostMalloc((void**)&buf, sizeof(double) * SEM_MAXB * SEM_NSTAT, hipHostMallocDefault) != hipSuccess)
            buf = nullptr;
    }
    return buf;
}

void launch_stats(const Batch& b, double* hs, hipStream_t s)
{
    FinArgs fa;
    fa.op = FIN_STATS; fa.gate = -1; fa.ncomp = 1; fa.f0 = 0; fa.host_flags = nullptr; fa.host_stats = hs;
    fa.gate2 = -1;
    launch_fin(b, fa, s);
}

// explicit terms of a step and the residual of its velocity solve (both paths)
void step_head(const Batch& b, const sem_ctx* c0, hipStream_t s)
{
    const int lx = c0->lx;
    const Resolved& r = c0->rs;
    fin(b, FIN_STEP_BEGIN, s);
    vec(b, V_IDV, 1, P64, I_IDVSTALE, s);
    // (i) explicit terms: convection, old pressure gradient, BDF/EXT history
    convection(b, c0, s);
    // local rhs (3 components) with the old pressure gradient folded in;
    // assembled together with the residual
    launch_opgrad_rhs(b, lx, r.opg_m, r.opg_c, F_P, s);
}

// (iii) pressure increment: A phi = (beta0/dt) dssum(wdiv(u*)), zero-mean rhs.
// This rhs is the initial residual of the pressure solve (phi = 0): it is
// formed in fp64 like every residual check, because the weak divergence of a
// nearly divergence-free u* is a small difference of large element terms
// whose fp32 rounding would dominate it.
void pressure_rhs(const Batch& b, const sem_ctx* c0, hipStream_t s)
{
    const int lx = c0->lx;
    launch_wdiv(b, lx, P64, P64, F_US, F_RP, s);
    launch_dssum(b, F_RP, 1, P64, -1, nullptr, s);
    vec(b, V_SUM_UNIQUE, 1, P64, -1, s, F_RP, -1, P64, P64, FIN_MEAN_UNIQUE);
    vec(b, V_SUB_MEAN, 1, P64, -1, s, F_RP, S_H2);  // F_GB aliases F_RP
    if (c0->flow.proj_dim > 0) projection_guess(b, c0->rs, s);
    else vec(b, V_ZERO, 1, P64, -1, s, F_GX);
}

// (iv) correction and pressure update, lag rotation, diagnostics; gate: the
// commit flag of a captured step, or -1
void step_tail(const Batch& b, const sem_ctx* c0, hipStream_t s, int gate)
{
    const int lx = c0->lx;
    const Resolved& r = c0->rs;
    Batch bg = b;
    bg.gate = gate;
    launch_opgrad(bg, lx, r.opg_m, r.opg_c, F_GX, F_GP, s);
    launch_dssum(b, F_GP, 3, P64, gate, nullptr, s);
    vec(b, V_CORRECT, 1, P64, gate, s);  // 3 components and p += phi
    fin(b, FIN_STEP_END, s, -1, 1, nullptr, 0, gate);
    launch_diagnostics(bg, lx, s);
    fin(b, FIN_DIAG, s, -1, 1, nullptr, 0, gate);
}

// One step of a batch driven from the host: the solver loops read the device
// convergence flags between iteration chunks.  Writes the statistics into hs.
int eager_step(sem_ctx* const* ctxs, const Batch& b, double* hs, hipStream_t s)
{
    sem_ctx* c0 = ctxs[0];
    step_head(b, c0, s);
    // (ii) velocity Helmholtz solves -> u*
    int rc = velocity_solve(ctxs, b, s);
    if (rc) return rc;
    pressure_rhs(b, c0, s);
    rc = pressure_solve(ctxs, b, s, true);
    if (rc) return rc;
    step_tail(b, c0, s, -1);
    launch_stats(b, hs, s);
    return check_hip_last();
}

// Iteration budgets of a captured step: PCG iterations per refinement cycle,
// refinement cycles, Arnoldi steps.
struct Budget {
    int kv, cyc, kp;
    bool operator<(const Budget& o) const { return std::tie(kv, cyc, kp) < std::tie(o.kv, o.cyc, o.kp); }
};

// One step with fixed iteration budgets and no host reads, in the order of
// eager_step.  Every solver kernel is gated on the device as in the host-driven
// path (a converged request idles), so a request whose solves stop by
// themselves within the budgets gets bitwise the results of eager_step; its
// commit flag is set.  Where a solve is still iterating at the end of its
// budget the flag stays clear and the correction, the lag rotation, the
// projection update and the diagnostics are gated off: the state is that of
// the step's start and the host runs the step again with eager_step.
void fixed_step(sem_ctx* const* ctxs, const Batch& b, const Budget& g, double* hs, hipStream_t s)
{
    sem_ctx* c0 = ctxs[0];
    const int lx = c0->lx;
    const Resolved& r = c0->rs;
    const int tv = r.tv;
    const bool hsmg = c0->flow.hsmg != 0;
    step_head(b, c0, s);
    {
        ProfScope ps(SEM_PROF_AX_RESID, s);
        resid_ax(b, lx, F_U, s);
    }
    launch_dssum(b, F_R64, 3, P64, -1, nullptr, s, R_A);
    fin(b, FIN_VINIT, s);
    const int ncyc = tv == P64 ? 1 : std::max(1, g.cyc);
    for (int cyc = 0; cyc < ncyc; ++cyc) {
        vec(b, V_PCG_INIT, 3, tv, -1, s, -1, -1, r.tva, P64, FIN_PCG_RHO);
        for (int q = 0; q < g.kv; ++q) pcg_iteration(b, lx, r, tv, s);
        vec(b, V_US_ADD, 3, tv, -1, s, cyc == 0 ? 1 : 0);
        if (tv == P64) break;
        {
            ProfScope ps(SEM_PROF_AX_RESID, s);
            resid_ax(b, lx, F_US, s);
        }
        launch_dssum(b, F_R64, 3, P64, -1, nullptr, s, R_A);
        fin(b, FIN_VINIT, s);
    }
    pressure_rhs(b, c0, s);
    gmres_start(b, lx, r, hsmg, s);
    const int m = c0->flow.gmres_restart;
    for (int q = 0; q < g.kp; ++q) {
        gmres_arnoldi(b, lx, r, hsmg, s);
        if ((q + 1) % m == 0 || q == g.kp - 1) gmres_cycle_end(b, lx, r, hsmg, s);
    }
    fin(b, FIN_COMMIT_CHECK, s);
    if (c0->flow.mode == SEM_MODE_FLUID && c0->flow.proj_dim > 0) projection_update(b, lx, r, s, I_COMMIT);
    gmres_finish(b, s);
    step_tail(b, c0, s, I_COMMIT);
    launch_stats(b, hs, s);
}

// A captured step of one batch and budget: the instantiated graph, its pinned
// statistics buffer and the profiling events recorded in it.
struct StepGraph {
    // the step as one graph, or, while a kernel class is profiled, as segments
    // split at that class's launches (timed[q]: segment q is one such launch)
    std::vector<hipGraph_t> graph;
    std::vector<hipGraphExec_t> exec;
    std::vector<char> timed;
    std::vector<hipEvent_t> ev;   // an event pair per timed segment
    double* hs = nullptr;
    uint64_t last_use = 0;
    // capture state
    hipStream_t cs = nullptr;
    bool in_timed = false;
    hipError_t err = hipSuccess;
    StepGraph() = default;
    StepGraph(const StepGraph&) = delete;
    StepGraph& operator=(const StepGraph&) = delete;
    ~StepGraph()
    {
        for (hipGraphExec_t x : exec) (void)hipGraphExecDestroy(x);
        for (hipGraph_t g : graph) (void)hipGraphDestroy(g);
        if (hs) (void)hipHostFree(hs);
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
    // close the segment being captured (kept if it holds any node)
    void close_segment()
    {
        hipGraph_t g = nullptr;
        const hipError_t le = hipGetLastError();
        const hipError_t e = hipStreamEndCapture(cs, &g);
        if (err == hipSuccess) err = le != hipSuccess ? le : e;
        if (e != hipSuccess || !g) return;
        size_t nn = 0;
        (void)hipGraphGetNodes(g, nullptr, &nn);
        if (nn == 0) { (void)hipGraphDestroy(g); return; }
        graph.push_back(g);
        timed.push_back(in_timed ? 1 : 0);
    }
    void open_segment()
    {
        const hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (err == hipSuccess) err = e;
    }
    static void split(void* self)
    {
        StepGraph* G = (StepGraph*)self;
        G->close_segment();
        G->in_timed = !G->in_timed;
        G->open_segment();
    }
};
struct GraphKey {
    std::vector<const sem_ctx*> ctxs;
    Budget g;
    int prof;
    bool operator<(const GraphKey& o) const { return std::tie(ctxs, g, prof) < std::tie(o.ctxs, o.g, o.prof); }
};
// shared ownership: a graph evicted or forgotten while another thread replays
// it lives until that replay's reference is dropped
std::map<GraphKey, std::shared_ptr<StepGraph>> g_graphs;
uint64_t g_graph_clock = 0;
// process-wide counts: graph replays, requests whose replayed step ran again
// eagerly, captures
std::atomic<int64_t> g_n_replay{0}, g_n_rerun{0}, g_n_capture{0};
#define SEM_GRAPH_CACHE 32

// drop every cached graph that launches work of context c
void graph_forget(const sem_ctx* c)
{
    std::lock_guard<std::recursive_mutex> lk(g_host_mu);
    for (auto it = g_graphs.begin(); it != g_graphs.end();) {
        if (std::find(it->first.ctxs.begin(), it->first.ctxs.end(), c) != it->first.ctxs.end()) {
            it = g_graphs.erase(it);
        } else {
            ++it;
        }
    }
}

// capture stream of the calling thread on the current device (default priority)
int capture_stream(int dev, hipStream_t* out)
{
    thread_local std::map<int, hipStream_t> streams;
    auto it = streams.find(dev);
    if (it != streams.end()) { *out = it->second; return 0; }
    hipStream_t st;
    HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    streams[dev] = st;
    *out = st;
    return 0;
}

// the cached graph of this batch and budget, captured on first use
int get_graph(sem_ctx* const* ctxs, int n, const Batch& b, const Budget& g, std::shared_ptr<StepGraph>* out)
{
    GraphKey key;
    key.ctxs.assign(ctxs, ctxs + n);
    key.g = g;
    key.prof = g_prof.kclass;
    std::lock_guard<std::recursive_mutex> lk(g_host_mu);
    auto it = g_graphs.find(key);
    if (it != g_graphs.end()) {
        it->second->last_use = ++g_graph_clock;
        *out = it->second;
        return 0;
    }
    if (g_graphs.size() >= SEM_GRAPH_CACHE) {
        auto lru = g_graphs.begin();
        for (auto jt = g_graphs.begin(); jt != g_graphs.end(); ++jt)
            if (jt->second->last_use < lru->second->last_use) lru = jt;
        g_graphs.erase(lru);
    }
    auto Gp = std::make_shared<StepGraph>();
    StepGraph& G = *Gp;
    HIPCHK(hipHostMalloc((void**)&G.hs, sizeof(double) * SEM_MAXB * SEM_NSTAT, hipHostMallocDefault));
    int rc = capture_stream(ctxs[0]->device, &G.cs);
    if (rc) return rc;
    G.open_segment();
    if (G.err != hipSuccess) return fail(SEM_EHIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(G.err));
    if (g_prof.kclass) {
        g_prof.split_hook = &StepGraph::split;
        g_prof.split_arg = &G;
    }
    fixed_step(ctxs, b, g, G.hs, G.cs);
    g_prof.split_hook = nullptr;
    g_prof.split_arg = nullptr;
    G.close_segment();
    if (G.err != hipSuccess) return fail(SEM_EHIP, std::string("step capture failed: ") + hipGetErrorString(G.err));
    for (size_t q = 0; q < G.graph.size(); ++q) {
        hipGraphExec_t x = nullptr;
        hipError_t e = hipGraphInstantiate(&x, G.graph[q], nullptr, nullptr, 0);
        if (e != hipSuccess) return fail(SEM_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        G.exec.push_back(x);
        if (G.timed[q]) {
            for (int k = 0; k < 2; ++k) {
                hipEvent_t ev;
                HIPCHK(hipEventCreate(&ev));
                G.ev.push_back(ev);
            }
        }
    }
    G.last_use = ++g_graph_clock;
    g_n_capture++;
    g_graphs.emplace(key, Gp);
    *out = Gp;
    return 0;
}

// statistics of request c from its row o of the statistics buffer
int take_stats(sem_ctx* c, const double* o, sem_step_stats* ss)
{
    int sti = SEM_OK;
    if (o[12] != 0.0) sti = SEM_ENAN;
    else if (o[11] > c->flow.pres_tol) sti = SEM_ENOTCONV;
    else
        for (int q = 0; q < 3; ++q)
            if (o[7 + q] > c->flow.vel_tol) sti = SEM_ENOTCONV;
    if (ss) {
        ss->t = o[0]; ss->ke = o[1]; ss->enst = o[2]; ss->maxdiv = o[3];
        for (int q = 0; q < 3; ++q) { ss->vel_iters[q] = (int)o[4 + q]; ss->vel_res[q] = o[7 + q]; }
        ss->pres_iters = (int)o[10];
        ss->pres_res = o[11];
        ss->status = sti;
        ss->vel_cycles = (int)o[14];
        ss->dt = o[16];
        ss->cfl = o[17];
    }
    const int vmax = (int)std::max(o[4], std::max(o[5], o[6]));
    c->pred_v = std::max(1, vmax);
    c->pred_p = std::max(1, (int)o[10]);
    c->hist_v = vmax;
    c->hist_c = (int)o[14];
    for (int q = 3; q > 0; --q) c->hist_p[q] = c->hist_p[q - 1];
    c->hist_p[0] = (int)o[10];
    c->hist_n = std::min(c->hist_n + 1, 4);
    return sti;
}

// budgets of a captured step from the batch's history (largest counts of the
// last step, and of the last four steps for the pressure); false while a
// request has no history yet
bool graph_budget(sem_ctx* const* ctxs, int n, Budget* g)
{
    Budget b{0, 1, 0};
    for (int i = 0; i < n; ++i) {
        const sem_ctx* c = ctxs[i];
        if (c->hist_n == 0) return false;
        b.kv = std::max(b.kv, c->hist_v);
        b.cyc = std::max(b.cyc, c->hist_c);
        for (int q = 0; q < c->hist_n; ++q) b.kp = std::max(b.kp, c->hist_p[q]);
    }
    b.kv = std::max(b.kv, 1);
    *g = b;
    return true;
}

int fluid_steps(sem_ctx* const* ctxs, int n, int nsteps, sem_step_stats* stats, bool graph)
{
    int rc = check_batch(ctxs, n, SEM_MODE_FLUID);
    if (rc) return rc;
    if (nsteps < 0) return fail(SEM_EINVAL, "nsteps must be >= 0");
    sem_ctx* c0 = ctxs[0];
    hipStream_t s = c0->stream;
    Batch b = make_batch(ctxs, n);
    double* hs = stats_buffer();
    if (!hs) return fail(SEM_EHIP, "pinned statistics buffer allocation failed");
    // adaptive dt changes the step's history at its start: such batches step eagerly
    if (c0->flow.cfl_target > 0.0) graph = false;
    if (c0->flow.cfl_target > 0.0 && nsteps > 0) {
        // the CFL rate of the current velocity (it may have been set since the last step)
        launch_diagnostics(b, c0->lx, s);
        fin(b, FIN_DIAG, s);
    }
    for (int st = 0; st < nsteps; ++st) {
        Budget g;
        std::shared_ptr<StepGraph> G;
        if (graph && graph_budget(ctxs, n, &g)) {
            rc = get_graph(ctxs, n, b, g, &G);
            if (rc) return rc;
        }
        if (!G) {
            if ((rc = eager_step(ctxs, b, hs, s))) return rc;
            HIPCHK(hipStreamSynchronize(s));
            for (int i = 0; i < n; ++i)
                take_stats(ctxs[i], hs + (size_t)i * SEM_NSTAT, stats ? &stats[(size_t)i * nsteps + st] : nullptr);
            continue;
        }
        size_t te = 0;
        for (size_t q = 0; q < G->exec.size(); ++q) {
            if (G->timed[q]) HIPCHK(hipEventRecord(G->ev[te], s));
            HIPCHK(hipGraphLaunch(G->exec[q], s));
            if (G->timed[q]) HIPCHK(hipEventRecord(G->ev[te + 1], s));
            if (G->timed[q]) te += 2;
        }
        HIPCHK(hipStreamSynchronize(s));
        g_n_replay++;
        for (size_t q = 0; q + 1 < te; q += 2) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, G->ev[q], G->ev[q + 1]) == hipSuccess) {
                g_prof.acc_ms += ms;
                g_prof.acc_n += 1;
            }
        }
        // requests whose solves did not finish within the budgets run the step again
        sem_ctx* redo[SEM_MAXB];
        int where[SEM_MAXB];
        int nr = 0;
        for (int i = 0; i < n; ++i) {
            const double* o = G->hs + (size_t)i * SEM_NSTAT;
            if (o[18] == 0.0) { redo[nr] = ctxs[i]; where[nr++] = i; continue; }
            take_stats(ctxs[i], o, stats ? &stats[(size_t)i * nsteps + st] : nullptr);
        }
        if (nr) {
            g_n_rerun += nr;
            Batch br = make_batch(redo, nr);
            if ((rc = eager_step(redo, br, hs, s))) return rc;
            HIPCHK(hipStreamSynchronize(s));
            for (int q = 0; q < nr; ++q)
                take_stats(redo[q], hs + (size_t)q * SEM_NSTAT,
                           stats ? &stats[(size_t)where[q] * nsteps + st] : nullptr);
        }
    }
    return 0;
}

}  // namespace

extern "C" {

int sem_fluid_step(sem_ctx* const* ctxs, int n, int nsteps, sem_step_stats* stats)
{
    return fluid_steps(ctxs, n, nsteps, stats, false);
}

int sem_fluid_step_graph(sem_ctx* const* ctxs, int n, int nsteps, sem_step_stats* stats)
{
    return fluid_steps(ctxs, n, nsteps, stats, true);
}

int sem_host_lock(int acquire)
{
    if (acquire) g_host_mu.lock();
    else g_host_mu.unlock();
    return 0;
}

int sem_graph_counters(int64_t* replays, int64_t* reruns, int64_t* captures)
{
    if (replays) *replays = g_n_replay.load();
    if (reruns) *reruns = g_n_rerun.load();
    if (captures) *captures = g_n_capture.load();
    return 0;
}

int sem_poisson_solve(sem_ctx* const* ctxs, int n, const void* const* rhs, void* const* sol, sem_solve_stats* stats)
{
    int rc = check_batch(ctxs, n, SEM_MODE_POISSON);
    if (rc) return rc;
    if (!rhs || !sol) return fail(SEM_EINVAL, "null rhs/sol");
    sem_ctx* c0 = ctxs[0];
    hipStream_t s = c0->stream;
    for (int i = 0; i < n; ++i) {
        if (!rhs[i] || !sol[i]) return fail(SEM_EINVAL, "null rhs/sol entry");
        HIPCHK(hipMemcpyAsync(ctxs[i]->hdesc.f[F_GB], rhs[i], 8 * (size_t)ctxs[i]->np, hipMemcpyDeviceToDevice, s));
    }
    Batch b = make_batch(ctxs, n);
    vec(b, V_SUM_UNIQUE, 1, P64, -1, s, F_GB, -1, P64, P64, FIN_MEAN_UNIQUE);
    vec(b, V_SUB_MEAN, 1, P64, -1, s, F_GB, -1);
    vec(b, V_ZERO, 1, P64, -1, s, F_GX);
    rc = pressure_solve(ctxs, b, s, false);
    if (rc) return rc;
    for (int i = 0; i < n; ++i)
        HIPCHK(hipMemcpyAsync(sol[i], ctxs[i]->hdesc.f[F_GX], 8 * (size_t)ctxs[i]->np, hipMemcpyDeviceToDevice, s));
    if (stats) {
        for (int i = 0; i < n; ++i) {
            int it = 0, nan = 0;
            double res = 0;
            HIPCHK(hipMemcpyAsync(&it, ctxs[i]->hdesc.I + I_GIT, sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(&nan, ctxs[i]->hdesc.I + I_NAN, sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(&res, ctxs[i]->hdesc.S + S_GBETA, sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            stats[i].iters = it;
            stats[i].res = res;
            stats[i].status = nan ? SEM_ENAN : (res > ctxs[i]->flow.pres_tol ? SEM_ENOTCONV : SEM_OK);
        }
    }
    return check_hip_last();
}

int sem_poisson_begin(sem_ctx* const* ctxs, int n, const void* const* rhs)
{
    int rc = check_batch(ctxs, n, SEM_MODE_POISSON);
    if (rc) return rc;
    if (!rhs) return fail(SEM_EINVAL, "null rhs");
    sem_ctx* c0 = ctxs[0];
    hipStream_t s = c0->stream;
    for (int i = 0; i < n; ++i) {
        if (!rhs[i]) return fail(SEM_EINVAL, "null rhs entry");
        HIPCHK(hipMemcpyAsync(ctxs[i]->hdesc.f[F_GB], rhs[i], 8 * (size_t)ctxs[i]->np, hipMemcpyDeviceToDevice, s));
    }
    Batch b = make_batch(ctxs, n);
    vec(b, V_SUM_UNIQUE, 1, P64, -1, s, F_GB, -1, P64, P64, FIN_MEAN_UNIQUE);
    vec(b, V_SUB_MEAN, 1, P64, -1, s, F_GB, -1);
    vec(b, V_ZERO, 1, P64, -1, s, F_GX);
    gmres_start(b, c0->lx, c0->rs, c0->flow.hsmg != 0, s);
    return check_hip_last();
}

int sem_poisson_advance(sem_ctx* const* ctxs, int n, int max_iters, int* active)
{
    int rc = check_batch(ctxs, n, SEM_MODE_POISSON);
    if (rc) return rc;
    if (max_iters < 1) return fail(SEM_EINVAL, "max_iters must be >= 1");
    Batch b = make_batch(ctxs, n);
    rc = gmres_advance(ctxs, b, ctxs[0]->stream, max_iters, false);
    if (rc < 0) return rc;
    if (active)
        for (int i = 0; i < n; ++i) active[i] = ctxs[0]->hflags[i] != 0;
    return 0;
}

int sem_poisson_finish(sem_ctx* c, void* sol, sem_solve_stats* st)
{
    int rc = bind_check(c);
    if (rc) return rc;
    if (c->flow.mode < SEM_MODE_POISSON) return fail(SEM_EINVAL, "context mode has no solver workspace");
    sem_ctx* one[1] = {c};
    Batch b = make_batch(one, 1);
    hipStream_t s = c->stream;
    gmres_finish(b, s);
    if (sol) HIPCHK(hipMemcpyAsync(sol, c->hdesc.f[F_GX], 8 * (size_t)c->np, hipMemcpyDeviceToDevice, s));
    int it = 0, nan = 0;
    double res = 0;
    HIPCHK(hipMemcpyAsync(&it, c->hdesc.I + I_GIT, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&nan, c->hdesc.I + I_NAN, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&res, c->hdesc.S + S_GBETA, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (st) {
        st->iters = it;
        st->res = res;
        st->status = nan ? SEM_ENAN : (res > c->flow.pres_tol ? SEM_ENOTCONV : SEM_OK);
    }
    return check_hip_last();
}

int sem_prof_start(int kclass)
{
    if (kclass < SEM_PROF_AX_VEL || kclass > SEM_PROF_HSMG) return fail(SEM_EINVAL, "unknown profiling class");
    g_prof.kclass = kclass;
    g_prof.used = 0;
    g_prof.acc_ms = 0.0;
    g_prof.acc_n = 0;
    return 0;
}

int sem_prof_stop(double* total_ms, int64_t* launches)
{
    double tot = 0.0;
    const size_t n = g_prof.used / 2;
    for (size_t i = 0; i < n; ++i) {
        HIPCHK(hipEventSynchronize(g_prof.ev[2 * i + 1]));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, g_prof.ev[2 * i], g_prof.ev[2 * i + 1]));
        tot += ms;
    }
    // plus the launches recorded inside replayed step graphs
    tot += g_prof.acc_ms;
    const int64_t ng = g_prof.acc_n;
    g_prof.kclass = 0;
    g_prof.used = 0;
    g_prof.acc_ms = 0.0;
    g_prof.acc_n = 0;
    if (total_ms) *total_ms = tot;
    if (launches) *launches = (int64_t)n + ng;
    return 0;
}

int sem_get_field(sem_ctx* c, int which, void* dst, int is_host)
{
    int rc = bind_check(c);
    if (rc) return rc;
    if (!dst) return fail(SEM_EINVAL, "null destination");
    int fid;
    if ((rc = field_of(c, which, fid))) return rc;
    char* p;
    if ((rc = current_ptr(c, fid, &p))) return rc;
    size_t off = 0;
    if (which >= SEM_F_G && which < SEM_F_G + 6) off = (size_t)(which - SEM_F_G);
    if (which >= SEM_F_M && which < SEM_F_M + 9) off = (size_t)(which - SEM_F_M);
    const long long L3 = (long long)c->lx * c->lx * c->lx;
    if (fid == F_G64 || fid == F_M64) {
        // [E][ncomp][lx3] -> component-major copy, one element at a time (host-side gather)
        const int nc = fid == F_G64 ? 6 : 9;
        std::vector<double> tmp((size_t)c->np * nc);
        HIPCHK(hipStreamSynchronize(c->stream));
        HIPCHK(hipMemcpyAsync(tmp.data(), p, 8 * tmp.size(), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        std::vector<double> out((size_t)c->np);
        for (long long e = 0; e < c->E; ++e)
            memcpy(out.data() + e * L3, tmp.data() + (e * nc + (long long)off) * L3, 8 * L3);
        if (is_host) memcpy(dst, out.data(), 8 * out.size());
        else {
            HIPCHK(hipMemcpyAsync(dst, out.data(), 8 * out.size(), hipMemcpyHostToDevice, c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
        }
        return 0;
    }
    if (fid == F_IBSUM64) {
        // stored as 1/Bsum
        std::vector<double> out((size_t)c->np);
        HIPCHK(hipStreamSynchronize(c->stream));
        HIPCHK(hipMemcpyAsync(out.data(), p, 8 * out.size(), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        for (auto& v : out) v = 1.0 / v;
        if (is_host) memcpy(dst, out.data(), 8 * out.size());
        else {
            HIPCHK(hipMemcpyAsync(dst, out.data(), 8 * out.size(), hipMemcpyHostToDevice, c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
        }
        return 0;
    }
    if (is_host) {
        HIPCHK(hipMemcpyAsync(dst, p, 8 * (size_t)c->np, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    } else {
        HIPCHK(hipMemcpyAsync(dst, p, 8 * (size_t)c->np, hipMemcpyDeviceToDevice, c->stream));
    }
    return 0;
}

int sem_set_field(sem_ctx* c, int which, const void* src, int is_host)
{
    int rc = bind_check(c);
    if (rc) return rc;
    if (!src) return fail(SEM_EINVAL, "null source");
    if (which >= SEM_F_MASS) return fail(SEM_EINVAL, "geometry fields are read-only");
    int fid;
    if ((rc = field_of(c, which, fid))) return rc;
    char* p;
    if ((rc = current_ptr(c, fid, &p))) return rc;
    HIPCHK(hipMemcpyAsync(p, src, 8 * (size_t)c->np, is_host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, c->stream));
    if (is_host) HIPCHK(hipStreamSynchronize(c->stream));
    return 0;
}

int sem_mass(sem_ctx* c, const double* f, double* out, int flags)
{
    int rc = bind_check(c);
    if (rc) return rc;
    if (!f || !out) return fail(SEM_EINVAL, "null field pointer");
    sem_ctx* one[1] = {c};
    Batch b = make_batch(one, 1);
    VecArgs a;
    memset(&a, 0, sizeof(a));
    a.op = V_MASS_RAW; a.gate = -1; a.ncomp = 1; a.tv = P64; a.ta = P64; a.tb = P64; a.f0 = -1; a.f1 = -1;
    a.x_raw = f; a.y_raw = out;
    launch_vec(b, a, c->stream);
    if (flags & SEM_ASSEMBLE) launch_dssum(b, -1, 1, P64, -1, out, c->stream);
    return check_hip_last();
}

int sem_node_field(sem_ctx* c, int what, double amp, double* out)
{
    int rc = bind_check(c);
    if (rc) return rc;
    if (!out || what < 0 || what > 3) return fail(SEM_EINVAL, "bad node field request");
    sem_ctx* one[1] = {c};
    Batch b = make_batch(one, 1);
    launch_node_field(b, c->lx, c->mp, what, amp, out, c->stream);
    return check_hip_last();
}

// The time/step level of the precision model (Fig. 4): a run may change
// tiers between steps by carrying its state into a context of another tier.
// Every state field is fp64 in every tier, so the copy is exact.
int sem_copy_state(sem_ctx* dst, sem_ctx* src)
{
    int rc = bind_check(dst);
    if (rc) return rc;
    if ((rc = bind_check(src))) return rc;
    if (dst == src) return fail(SEM_EINVAL, "source and destination are the same context");
    if (dst->flow.mode != SEM_MODE_FLUID || src->flow.mode != SEM_MODE_FLUID)
        return fail(SEM_EINVAL, "sem_copy_state needs two fluid-mode contexts");
    const sem_mesh_desc& a = dst->mesh;
    const sem_mesh_desc& b = src->mesh;
    bool same = a.order == b.order && a.deform_amp == b.deform_amp;
    for (int d = 0; d < 3; ++d) same = same && a.nel[d] == b.nel[d] && a.lo[d] == b.lo[d] && a.hi[d] == b.hi[d];
    for (int q = 0; q < 9; ++q) same = same && a.deform_phase[q] == b.deform_phase[q];
    if (!same) return fail(SEM_EINVAL, "sem_copy_state needs the same mesh");
    if (dst->flow.dt != src->flow.dt || dst->flow.torder != src->flow.torder)
        return fail(SEM_EINVAL, "sem_copy_state needs the same time step and BDF/EXT order (the history is at dt spacing)");
    static const int fids[] = {F_U, F_U + 1, F_U + 2, F_UL1, F_UL1 + 1, F_UL1 + 2, F_UL2, F_UL2 + 1, F_UL2 + 2,
                               F_BNL1, F_BNL1 + 1, F_BNL1 + 2, F_BNL2, F_BNL2 + 1, F_BNL2 + 2, F_P};
    HIPCHK(hipStreamSynchronize(src->stream));
    HIPCHK(hipStreamSynchronize(dst->stream));
    for (int fid : fids) {
        char *ps, *pd;
        if ((rc = current_ptr(src, fid, &ps))) return rc;
        if ((rc = current_ptr(dst, fid, &pd))) return rc;
        HIPCHK(hipMemcpyAsync(pd, ps, 8 * (size_t)dst->np, hipMemcpyDeviceToDevice, dst->stream));
    }
    // clock and step (the BDF/EXT order ramp follows the step count); the
    // projection space starts empty in the new tier
    HIPCHK(hipMemcpyAsync(dst->hdesc.S + S_TIME, src->hdesc.S + S_TIME, sizeof(double), hipMemcpyDeviceToDevice,
                          dst->stream));
    // step-size history (variable-step BDF/EXT under adaptive dt)
    HIPCHK(hipMemcpyAsync(dst->hdesc.S + S_DTH, src->hdesc.S + S_DTH, 3 * sizeof(double), hipMemcpyDeviceToDevice,
                          dst->stream));
    HIPCHK(hipMemcpyAsync(dst->hdesc.I + I_STEP, src->hdesc.I + I_STEP, sizeof(int), hipMemcpyDeviceToDevice,
                          dst->stream));
    const int zero = 0;
    HIPCHK(hipMemcpyAsync(dst->hdesc.I + I_PRL, &zero, sizeof(int), hipMemcpyHostToDevice, dst->stream));
    HIPCHK(hipStreamSynchronize(dst->stream));
    dst->pred_v = src->pred_v;
    dst->pred_p = src->pred_p;
    return 0;
}

int sem_set_clock(sem_ctx* c, double t, int step)
{
    int rc = bind_check(c);
    if (rc) return rc;
    if (step < 0) return fail(SEM_EINVAL, "negative step");
    HIPCHK(hipMemcpyAsync(c->hdesc.S + S_TIME, &t, sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->hdesc.I + I_STEP, &step, sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return 0;
}

int sem_diagnostics(sem_ctx* c, sem_diag* out)
{
    int rc = bind_check(c);
    if (rc) return rc;
    if (!out) return fail(SEM_EINVAL, "null output");
    if (c->flow.mode != SEM_MODE_FLUID) return fail(SEM_EINVAL, "diagnostics need a fluid-mode context");
    sem_ctx* one[1] = {c};
    Batch b = make_batch(one, 1);
    launch_diagnostics(b, c->lx, c->stream);
    fin(b, FIN_DIAG, c->stream);
    if ((rc = check_hip_last())) return rc;
    double v[3];
    int st = 0;
    double t = 0;
    HIPCHK(hipMemcpyAsync(v, c->hdesc.S + S_KE, sizeof(v), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(&t, c->hdesc.S + S_TIME, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(&st, c->hdesc.I + I_STEP, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    out->ke = v[0]; out->enst = v[1]; out->maxdiv = v[2]; out->t = t; out->step = st;
    return 0;
}

// element-local operators on caller arrays: staged through the context's
// own fields (fluid-mode workspace), then copied out
int sem_conv(sem_ctx* c, const double* const* u3, double* const* out3)
{
    int rc = bind_check(c);
    if (rc) return rc;
    if (c->flow.mode != SEM_MODE_FLUID) return fail(SEM_EINVAL, "needs a fluid-mode context");
    const size_t nb = 8 * (size_t)c->np;
    char* sv[3];
    char* bnp[3];
    for (int q = 0; q < 3; ++q) {
        if ((rc = current_ptr(c, F_U + q, &sv[q]))) return rc;
        if ((rc = current_ptr(c, F_BN + q, &bnp[q]))) return rc;
    }
    // save state, run, restore
    for (int q = 0; q < 3; ++q) {
        HIPCHK(hipMemcpyAsync(c->hdesc.f[F_W64 + q], sv[q], nb, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(sv[q], u3[q], nb, hipMemcpyDeviceToDevice, c->stream));
    }
    sem_ctx* one[1] = {c};
    Batch b = make_batch(one, 1);
    convection(b, c, c->stream);
    for (int q = 0; q < 3; ++q) {
        HIPCHK(hipMemcpyAsync(out3[q], bnp[q], nb, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(sv[q], c->hdesc.f[F_W64 + q], nb, hipMemcpyDeviceToDevice, c->stream));
    }
    return check_hip_last();
}

int sem_opgrad(sem_ctx* c, const double* p, double* const* out3)
{
    int rc = bind_check(c);
    if (rc) return rc;
    if (c->flow.mode != SEM_MODE_FLUID) return fail(SEM_EINVAL, "needs a fluid-mode context");
    const size_t nb = 8 * (size_t)c->np;
    HIPCHK(hipMemcpyAsync(c->hdesc.f[F_PHI], p, nb, hipMemcpyDeviceToDevice, c->stream));
    sem_ctx* one[1] = {c};
    Batch b = make_batch(one, 1);
    launch_opgrad(b, c->lx, c->rs.opg_m, c->rs.opg_c, F_PHI, F_R64, c->stream);
    for (int q = 0; q < 3; ++q)
        HIPCHK(hipMemcpyAsync(out3[q], c->hdesc.f[F_R64 + q], nb, hipMemcpyDeviceToDevice, c->stream));
    return check_hip_last();
}

int sem_wdiv(sem_ctx* c, const double* const* v3, double* out)
{
    int rc = bind_check(c);
    if (rc) return rc;
    if (c->flow.mode != SEM_MODE_FLUID) return fail(SEM_EINVAL, "needs a fluid-mode context");
    const size_t nb = 8 * (size_t)c->np;
    for (int q = 0; q < 3; ++q)
        HIPCHK(hipMemcpyAsync(c->hdesc.f[F_R64 + q], v3[q], nb, hipMemcpyDeviceToDevice, c->stream));
    sem_ctx* one[1] = {c};
    Batch b = make_batch(one, 1);
    launch_wdiv(b, c->lx, c->rs.div_m, c->rs.div_c, F_R64, F_PHI, c->stream);
    HIPCHK(hipMemcpyAsync(out, c->hdesc.f[F_PHI], nb, hipMemcpyDeviceToDevice, c->stream));
    return check_hip_last();
}

}  // extern "C"


// ------------------------------------------------------------------ Poisson solve on an external workspace
// The Krylov vectors of a stand-alone Jacobi-GMRES solve (the basis V_0..V_m
// in the basis storage precision; the operator output, the working vector,
// the rhs and the iterate in fp64) taken from memory the caller provides
// instead of the context's bound workspace, so that a context bound in any
// mode can solve.  The kernels reach their fields through the device copy of
// the request descriptor: for the duration of the solve it points the Krylov
// fields into ws, and it is restored afterwards.  Both descriptor writes are
// kernels that take the descriptor as an argument (no host staging buffer,
// no memset), on the context's stream.

namespace {

__global__ void desc_store_kernel(ReqDesc* dst, ReqDesc src)
{
    const unsigned long long* a = (const unsigned long long*)&src;
    unsigned long long* b = (unsigned long long*)dst;
    for (unsigned i = threadIdx.x; i < sizeof(ReqDesc) / 8; i += blockDim.x) b[i] = a[i];
}
static_assert(sizeof(ReqDesc) % 8 == 0, "descriptor copied in 8-byte words");

int desc_store(ReqDesc* dst, const ReqDesc& src, hipStream_t s)
{
    hipLaunchKernelGGL(desc_store_kernel, dim3(1), dim3(64), 0, s, dst, src);
    return check_hip_last();
}

}  // namespace

namespace semk {

int poisson_external_bytes(const sem_ctx* c, size_t* bytes, int* device)
{
    int rc = bind_check(const_cast<sem_ctx*>(c));
    if (rc) return rc;
    const size_t np = (size_t)c->np;
    *bytes = align256((size_t)(c->flow.gmres_restart + 1) * psize(c->rs.tb) * np) + 4 * align256(8 * np);
    *device = c->device;
    return 0;
}

int poisson_solve_external(sem_ctx* c, char* ws, size_t ws_bytes, const void* rhs, void* sol, sem_solve_stats* st)
{
    size_t need = 0;
    int dev = 0;
    int rc = poisson_external_bytes(c, &need, &dev);
    if (rc) return rc;
    if (!ws || ws_bytes < need || (((uintptr_t)ws) & 255)) return fail(SEM_EINVAL, "external Krylov workspace too small or misaligned");
    if (!rhs || !sol) return fail(SEM_EINVAL, "null rhs/sol");
    if (c->flow.hsmg) return fail(SEM_EINVAL, "a solve on an external workspace runs the Jacobi preconditioner (flow.hsmg must be 0)");
    const size_t np = (size_t)c->np;
    const size_t vbytes = align256((size_t)(c->flow.gmres_restart + 1) * psize(c->rs.tb) * np);
    const size_t dbytes = align256(8 * np);
    hipStream_t s = c->stream;
    ReqDesc d = c->hdesc;
    d.f[F_V] = ws;
    d.f[F_GW] = ws + vbytes;
    d.f[F_GWD] = ws + vbytes + dbytes;
    d.f[F_GB] = ws + vbytes + 2 * dbytes;
    d.f[F_GX] = ws + vbytes + 3 * dbytes;
    if ((rc = desc_store(c->ddesc, d, s))) return rc;
    // event profiling would create events: it is paused for this solve
    const int prof_saved = g_prof.kclass;
    g_prof.kclass = 0;
    sem_ctx* one[1] = {c};
    Batch b = make_batch(one, 1);
    hipError_t e = hipMemcpyAsync(d.f[F_GB], rhs, 8 * np, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) rc = fail(SEM_EHIP, std::string("hipMemcpyAsync(rhs): ") + hipGetErrorString(e));
    if (!rc) {
        vec(b, V_SUM_UNIQUE, 1, P64, -1, s, F_GB, -1, P64, P64, FIN_MEAN_UNIQUE);
        vec(b, V_SUB_MEAN, 1, P64, -1, s, F_GB, -1);
        vec(b, V_ZERO, 1, P64, -1, s, F_GX);  // ws may hold an earlier solve's values
        rc = pressure_solve(one, b, s, false);
    }
    g_prof.kclass = prof_saved;
    if (!rc) {
        e = hipMemcpyAsync(sol, d.f[F_GX], 8 * np, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) rc = fail(SEM_EHIP, std::string("hipMemcpyAsync(sol): ") + hipGetErrorString(e));
    }
    // the bound descriptor comes back also after a failed solve
    const int rc2 = desc_store(c->ddesc, c->hdesc, s);
    if (rc) return rc;
    if (rc2) return rc2;
    int it = 0, nan = 0;
    double res = 0;
    HIPCHK(hipMemcpyAsync(&it, c->hdesc.I + I_GIT, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&nan, c->hdesc.I + I_NAN, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&res, c->hdesc.S + S_GBETA, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (st) {
        st->iters = it;
        st->res = res;
        st->status = nan ? SEM_ENAN : (res > c->flow.pres_tol ? SEM_ENOTCONV : SEM_OK);
    }
    return check_hip_last();
}

int set_error(int code, const char* msg) { return fail(code, msg); }

}  // namespace semk
