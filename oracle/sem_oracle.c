/*
 * sem_oracle.c -- plain FP64 CPU oracle of the SEM incompressible
 * Navier-Stokes step on the Taylor-Green vortex.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * GPU library is checked against.  It shares no code, header, table or helper
 * with the HIP path; only tests, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.
 *
 * Everything is double precision, written as plain loops in the order the
 * mathematics is stated, with OpenMP only over independent elements.  Sums
 * over the whole mesh are formed as per-element partial sums that are then
 * added serially in element order, so the result does not depend on the
 * number of threads.
 *
 * Sources (the paper is "Mixed-Precision SEM-Based CFD Simulations on GPUs:
 * A Taylor-Green Vortex case"):
 *   - matrix-free SEM on hexahedra with Gauss-Lobatto-Legendre points, the
 *     P_N-P_N fluid step and its Fig. 3 ordering (explicit RHS, velocity
 *     solve, u*, pressure residual, pressure solve, correction): Sec. 2,
 *     Fig. 3, Fig. 5 discussion;
 *   - CG+Jacobi for velocity, GMRES for pressure, third-order time
 *     integration: Sec. 1.1 and Sec. 3 (solver settings paragraph);
 *   - the Taylor-Green initial condition and Re = v0 L / nu: Sec. 3 eqs.;
 *   - GLL nodes/weights/derivative matrix, geometric factors and the
 *     sum-factorised operators are textbook SEM (Deville, Fischer & Mund,
 *     "High-Order Methods for Incompressible Fluid Flow", 2002, ch. 2-4).
 *   - GMRES(m): Saad & Schultz (1986), right preconditioned, Givens rotations,
 *     classical Gram-Schmidt applied twice.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXLX 16

/* ------------------------------------------------------------------ */
/* Legendre polynomial L_N(x) and its derivative by the three-term     */
/* recurrence (textbook).                                               */
/* ------------------------------------------------------------------ */
static void legendre(int N, double x, double* L, double* dL)
{
    double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
    if (N == 0) { *L = 1.0; *dL = 0.0; return; }
    for (int k = 1; k < N; ++k) {
        double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        double d2 = d0 + (2.0 * k + 1.0) * p1;   /* L'_{k+1} = L'_{k-1} + (2k+1) L_k */
        p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    }
    *L = p1; *dL = d1;
}

/* GLL nodes (endpoints and roots of L'_N) and weights
 * w_i = 2 / (N (N+1) L_N(xi_i)^2).  Newton on L'_N uses the Legendre ODE for
 * L''_N.  Returns 0 on success. */
int orc_gll(int N, double* xi, double* w)
{
    if (N < 1 || N + 1 > ORC_MAXLX) return -1;
    const double pi = 3.14159265358979323846;
    xi[0] = -1.0; xi[N] = 1.0;
    for (int i = 1; i < N; ++i) {
        double x = -cos(pi * i / N);     /* Chebyshev-Gauss-Lobatto start */
        for (int it = 0; it < 100; ++it) {
            double L, dL;
            legendre(N, x, &L, &dL);
            double d2L = (2.0 * x * dL - N * (N + 1.0) * L) / (1.0 - x * x);
            double dx = dL / d2L;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        xi[i] = x;
    }
    /* enforce the exact symmetry of the node set */
    for (int i = 0; i <= N / 2; ++i) {
        double s = 0.5 * (xi[N - i] - xi[i]);
        xi[i] = -s; xi[N - i] = s;
    }
    if (N % 2 == 0) xi[N / 2] = 0.0;
    for (int i = 0; i <= N; ++i) {
        double L, dL;
        legendre(N, xi[i], &L, &dL);
        w[i] = 2.0 / (N * (N + 1.0) * L * L);
    }
    return 0;
}

/* Derivative matrix of the Lagrange interpolant on the GLL nodes,
 * D[i*lx+j] = l_j'(xi_i):
 *   L_N(xi_i) / (L_N(xi_j) (xi_i - xi_j))   for i != j,
 *   -N(N+1)/4 at (0,0),  +N(N+1)/4 at (N,N),  0 on the rest of the diagonal. */
void orc_deriv(int N, const double* xi, double* D)
{
    int lx = N + 1;
    double Lv[ORC_MAXLX];
    for (int i = 0; i < lx; ++i) { double dL; legendre(N, xi[i], &Lv[i], &dL); }
    for (int i = 0; i < lx; ++i)
        for (int j = 0; j < lx; ++j) {
            double v = 0.0;
            if (i != j) v = Lv[i] / (Lv[j] * (xi[i] - xi[j]));
            else if (i == 0) v = -N * (N + 1.0) / 4.0;
            else if (i == N) v = N * (N + 1.0) / 4.0;
            D[i * lx + j] = v;
        }
}

/* ------------------------------------------------------------------ */
/* Mesh: nx*ny*nz hexahedra on the box [lo,hi], periodic in all three  */
/* directions, optional smooth sinusoidal node perturbation.           */
/* Field layout: element-major, u[e][k][j][i], i fastest,              */
/* e = ex + nx (ey + ny ez).                                            */
/* ------------------------------------------------------------------ */
typedef struct {
    int nel[3], N, lx, E;
    long np;                    /* E * lx^3 local points */
    long nglob;                 /* unique periodic nodes */
    double lo[3], hi[3], h[3];
    double amp, phase[9];
    double xi[ORC_MAXLX], w[ORC_MAXLX], D[ORC_MAXLX * ORC_MAXLX];
    double *xyz;                /* 3*np coordinates */
    double *jac, *B;            /* np */
    double *drdx;               /* 9*np: (a*3+c) -> d r_a / d x_c */
    double *G;                  /* 6*np: rr rs rt ss st tt */
    double *M;                  /* 9*np: M_ac = B d r_a / d x_c */
    long *gid;                  /* np */
    int *mult;                  /* np */
    double *Bsum;               /* dssum(B) */
    double vol;                 /* sum of B */
} orc_mesh;

#define PT(m, e, i, j, k) ((long)(e) * (m)->lx * (m)->lx * (m)->lx + (i) + (m)->lx * ((j) + (m)->lx * (k)))

static double* dalloc(long n) { return (double*)calloc((size_t)n, sizeof(double)); }

void orc_dssum(const orc_mesh* m, double* u);
void orc_remove_mean_unique(const orc_mesh* m, double* r);

/* Perturbed coordinate of the reference position (X,Y,Z) measured from lo:
 * each coordinate c gets amp*h_c*sin(pi X/hx + ph[3c]) sin(pi Y/hy + ph[3c+1])
 * sin(pi Z/hz + ph[3c+2]).  A function of global position only, so the mesh
 * stays conforming; periodic when every element count is even. */
static void perturb(const orc_mesh* m, const double X[3], double out[3])
{
    const double pi = 3.14159265358979323846;
    for (int c = 0; c < 3; ++c) {
        double d = 0.0;
        if (m->amp != 0.0) {
            d = m->amp * m->h[c];
            for (int q = 0; q < 3; ++q) d *= sin(pi * X[q] / m->h[q] + m->phase[3 * c + q]);
        }
        out[c] = m->lo[c] + X[c] + d;
    }
}

/* Geometric factors of every element of m from its coordinates (m->xyz):
 * dx_c/dr_a = D_a x_c, jac = det, dr/dx = inverse, B = jac w_i w_j w_k,
 * G_ab = B sum_c dr_a/dx_c dr_b/dx_c, M_ac = B dr_a/dx_c.  Returns nonzero
 * if some Jacobian is not positive. */
static int mesh_geometry(orc_mesh* m)
{
    const int lx = m->lx;
    const long np = m->np;
    const double* D = m->D;
    int bad = 0;
    #pragma omp parallel for reduction(|:bad)
    for (int e = 0; e < m->E; ++e)
        for (int k = 0; k < lx; ++k)
        for (int j = 0; j < lx; ++j)
        for (int i = 0; i < lx; ++i) {
            long p = PT(m, e, i, j, k);
            double J[3][3];              /* J[c][a] = d x_c / d r_a */
            for (int c = 0; c < 3; ++c) {
                const double* X = m->xyz + (long)c * np;
                double dr = 0, ds = 0, dt = 0;
                for (int l = 0; l < lx; ++l) {
                    dr += D[i * lx + l] * X[PT(m, e, l, j, k)];
                    ds += D[j * lx + l] * X[PT(m, e, i, l, k)];
                    dt += D[k * lx + l] * X[PT(m, e, i, j, l)];
                }
                J[c][0] = dr; J[c][1] = ds; J[c][2] = dt;
            }
            double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
                       - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
                       + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
            if (!(det > 0.0)) bad = 1;
            /* inverse: (dr/dx)[a][c] = cofactor(J)[c][a] / det */
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
            double Bp = det * m->w[i] * m->w[j] * m->w[k];
            m->jac[p] = det;
            m->B[p] = Bp;
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 3; ++c) {
                    m->drdx[(long)(a * 3 + c) * np + p] = inv[a][c];
                    m->M[(long)(a * 3 + c) * np + p] = Bp * inv[a][c];
                }
            static const int ga[6] = {0, 0, 0, 1, 1, 2}, gb[6] = {0, 1, 2, 1, 2, 2};
            for (int q = 0; q < 6; ++q) {
                double s = 0;
                for (int c = 0; c < 3; ++c) s += inv[ga[q]][c] * inv[gb[q]][c];
                m->G[(long)q * np + p] = Bp * s;
            }
        }
    return bad;
}

orc_mesh* orc_mesh_new(int nx, int ny, int nz, int N, const double* lo, const double* hi,
                       double amp, const double* phase)
{
    if (nx < 1 || ny < 1 || nz < 1 || N < 1 || N + 1 > ORC_MAXLX) return NULL;
    if (amp != 0.0 && (nx % 2 || ny % 2 || nz % 2)) return NULL;
    orc_mesh* m = (orc_mesh*)calloc(1, sizeof(orc_mesh));
    m->nel[0] = nx; m->nel[1] = ny; m->nel[2] = nz;
    m->N = N; m->lx = N + 1; m->E = nx * ny * nz;
    int lx = m->lx;
    m->np = (long)m->E * lx * lx * lx;
    for (int c = 0; c < 3; ++c) {
        m->lo[c] = lo[c]; m->hi[c] = hi[c];
        m->h[c] = (hi[c] - lo[c]) / m->nel[c];
    }
    m->amp = amp;
    for (int q = 0; q < 9; ++q) m->phase[q] = phase ? phase[q] : 0.0;
    orc_gll(N, m->xi, m->w);
    orc_deriv(N, m->xi, m->D);

    long np = m->np;
    m->xyz = dalloc(3 * np);
    m->jac = dalloc(np); m->B = dalloc(np);
    m->drdx = dalloc(9 * np); m->G = dalloc(6 * np); m->M = dalloc(9 * np);
    m->gid = (long*)calloc((size_t)np, sizeof(long));
    m->mult = (int*)calloc((size_t)np, sizeof(int));
    m->Bsum = dalloc(np);

    /* coordinates and periodic global numbering */
    long ngx = (long)nx * N, ngy = (long)ny * N, ngz = (long)nz * N;
    m->nglob = ngx * ngy * ngz;
    for (int ez = 0; ez < nz; ++ez)
    for (int ey = 0; ey < ny; ++ey)
    for (int ex = 0; ex < nx; ++ex) {
        int e = ex + nx * (ey + ny * ez);
        for (int k = 0; k < lx; ++k)
        for (int j = 0; j < lx; ++j)
        for (int i = 0; i < lx; ++i) {
            long p = PT(m, e, i, j, k);
            double X[3] = { (ex + 0.5 * (1.0 + m->xi[i])) * m->h[0],
                            (ey + 0.5 * (1.0 + m->xi[j])) * m->h[1],
                            (ez + 0.5 * (1.0 + m->xi[k])) * m->h[2] };
            double xo[3];
            perturb(m, X, xo);
            m->xyz[p] = xo[0]; m->xyz[np + p] = xo[1]; m->xyz[2 * np + p] = xo[2];
            long gx = ((long)ex * N + i) % ngx;
            long gy = ((long)ey * N + j) % ngy;
            long gz = ((long)ez * N + k) % ngz;
            m->gid[p] = gx + ngx * (gy + ngy * gz);
        }
    }
    int* cnt = (int*)calloc((size_t)m->nglob, sizeof(int));
    for (long p = 0; p < np; ++p) cnt[m->gid[p]]++;
    for (long p = 0; p < np; ++p) m->mult[p] = cnt[m->gid[p]];
    free(cnt);

    if (mesh_geometry(m)) {
        /* non-positive Jacobian: the mesh is invalid */
        free(m->xyz); free(m->jac); free(m->B); free(m->drdx); free(m->G); free(m->M);
        free(m->gid); free(m->mult); free(m->Bsum); free(m);
        return NULL;
    }
    memcpy(m->Bsum, m->B, (size_t)np * sizeof(double));
    orc_dssum(m, m->Bsum);
    double vol = 0;
    for (long p = 0; p < np; ++p) vol += m->B[p];
    m->vol = vol;
    return m;
}

/* A mesh holding only the listed elements of the nx x ny x nz box (with the
 * same optional perturbation): coordinates and geometric factors of each
 * listed element are those it has in the full mesh, so every element-local
 * operator (Ax, Jacobi diagonal, convection, gradient, weak divergence) of
 * the subset equals the full mesh's on those elements.  No assembly: every
 * point is its own unique node (mult 1).  Checks large meshes element by
 * element. */
orc_mesh* orc_mesh_subset_new(int nx, int ny, int nz, int N, const double* lo, const double* hi,
                              double amp, const double* phase, const int* elems, int ne)
{
    if (nx < 1 || ny < 1 || nz < 1 || N < 1 || N + 1 > ORC_MAXLX || ne < 1) return NULL;
    if (amp != 0.0 && (nx % 2 || ny % 2 || nz % 2)) return NULL;
    for (int q = 0; q < ne; ++q)
        if (elems[q] < 0 || (long)elems[q] >= (long)nx * ny * nz) return NULL;
    orc_mesh* m = (orc_mesh*)calloc(1, sizeof(orc_mesh));
    m->nel[0] = nx; m->nel[1] = ny; m->nel[2] = nz;
    m->N = N; m->lx = N + 1; m->E = ne;
    int lx = m->lx;
    m->np = (long)ne * lx * lx * lx;
    for (int c = 0; c < 3; ++c) {
        m->lo[c] = lo[c]; m->hi[c] = hi[c];
        m->h[c] = (hi[c] - lo[c]) / m->nel[c];
    }
    m->amp = amp;
    for (int q = 0; q < 9; ++q) m->phase[q] = phase ? phase[q] : 0.0;
    orc_gll(N, m->xi, m->w);
    orc_deriv(N, m->xi, m->D);
    long np = m->np;
    m->xyz = dalloc(3 * np);
    m->jac = dalloc(np); m->B = dalloc(np);
    m->drdx = dalloc(9 * np); m->G = dalloc(6 * np); m->M = dalloc(9 * np);
    m->gid = (long*)calloc((size_t)np, sizeof(long));
    m->mult = (int*)calloc((size_t)np, sizeof(int));
    m->Bsum = dalloc(np);
    m->nglob = np;
    for (int q = 0; q < ne; ++q) {
        const int ef = elems[q];
        const int ex = ef % nx, ey = (ef / nx) % ny, ez = ef / (nx * ny);
        for (int k = 0; k < lx; ++k)
        for (int j = 0; j < lx; ++j)
        for (int i = 0; i < lx; ++i) {
            long p = PT(m, q, i, j, k);
            double X[3] = { (ex + 0.5 * (1.0 + m->xi[i])) * m->h[0],
                            (ey + 0.5 * (1.0 + m->xi[j])) * m->h[1],
                            (ez + 0.5 * (1.0 + m->xi[k])) * m->h[2] };
            double xo[3];
            perturb(m, X, xo);
            m->xyz[p] = xo[0]; m->xyz[np + p] = xo[1]; m->xyz[2 * np + p] = xo[2];
            m->gid[p] = p;
            m->mult[p] = 1;
        }
    }
    if (mesh_geometry(m)) {
        free(m->xyz); free(m->jac); free(m->B); free(m->drdx); free(m->G); free(m->M);
        free(m->gid); free(m->mult); free(m->Bsum); free(m);
        return NULL;
    }
    memcpy(m->Bsum, m->B, (size_t)np * sizeof(double));
    double vol = 0;
    for (long p = 0; p < np; ++p) vol += m->B[p];
    m->vol = vol;
    return m;
}

void orc_mesh_free(orc_mesh* m)
{
    if (!m) return;
    free(m->xyz); free(m->jac); free(m->B); free(m->drdx); free(m->G); free(m->M);
    free(m->gid); free(m->mult); free(m->Bsum); free(m);
}

/* accessors (copy-out into caller arrays) */
long orc_mesh_np(const orc_mesh* m) { return m->np; }
long orc_mesh_nglob(const orc_mesh* m) { return m->nglob; }
int orc_mesh_lx(const orc_mesh* m) { return m->lx; }
int orc_mesh_E(const orc_mesh* m) { return m->E; }
double orc_mesh_vol(const orc_mesh* m) { return m->vol; }
/* which: 0 xyz(3np) 1 jac 2 B 3 drdx(9np) 4 G(6np) 5 M(9np) 6 Bsum 7 mult 8 gid */
int orc_mesh_get(const orc_mesh* m, int which, double* out)
{
    long np = m->np;
    switch (which) {
    case 0: memcpy(out, m->xyz, 3 * np * sizeof(double)); break;
    case 1: memcpy(out, m->jac, np * sizeof(double)); break;
    case 2: memcpy(out, m->B, np * sizeof(double)); break;
    case 3: memcpy(out, m->drdx, 9 * np * sizeof(double)); break;
    case 4: memcpy(out, m->G, 6 * np * sizeof(double)); break;
    case 5: memcpy(out, m->M, 9 * np * sizeof(double)); break;
    case 6: memcpy(out, m->Bsum, np * sizeof(double)); break;
    case 7: for (long p = 0; p < np; ++p) out[p] = m->mult[p]; break;
    case 8: for (long p = 0; p < np; ++p) out[p] = (double)m->gid[p]; break;
    default: return -1;
    }
    return 0;
}
void orc_mesh_tables(const orc_mesh* m, double* xi, double* w, double* D)
{
    int lx = m->lx;
    memcpy(xi, m->xi, lx * sizeof(double));
    memcpy(w, m->w, lx * sizeof(double));
    memcpy(D, m->D, lx * lx * sizeof(double));
}

/* Expand a field given on the periodic lattice of unique nodes
 * (index gx + ngx (gy + ngy gz)) to the element-local layout. */
void orc_from_lattice(const orc_mesh* m, const double* lat, double* u)
{
    for (long p = 0; p < m->np; ++p) u[p] = lat[m->gid[p]];
}

/* ------------------------------------------------------------------ */
/* Direct stiffness summation Q Q^T: every local copy of a unique node */
/* receives the sum of all its copies.                                  */
/* ------------------------------------------------------------------ */
void orc_dssum(const orc_mesh* m, double* u)
{
    double* g = dalloc(m->nglob);
    for (long p = 0; p < m->np; ++p) g[m->gid[p]] += u[p];
    for (long p = 0; p < m->np; ++p) u[p] = g[m->gid[p]];
    free(g);
}

/* Inner product of two assembled (continuous) vectors over unique nodes:
 * (a,b) = sum_local a b / mult. */
double orc_glsc(const orc_mesh* m, const double* a, const double* b)
{
    int E = m->E;
    long n3 = (long)m->lx * m->lx * m->lx;
    double* part = dalloc(E);
    #pragma omp parallel for
    for (int e = 0; e < E; ++e) {
        double s = 0;
        for (long q = 0; q < n3; ++q) { long p = e * n3 + q; s += a[p] * b[p] / m->mult[p]; }
        part[e] = s;
    }
    double s = 0;
    for (int e = 0; e < E; ++e) s += part[e];
    free(part);
    return s;
}

/* Sum of all local values (no multiplicity weighting). */
double orc_sum(const orc_mesh* m, const double* a)
{
    int E = m->E;
    long n3 = (long)m->lx * m->lx * m->lx;
    double* part = dalloc(E);
    #pragma omp parallel for
    for (int e = 0; e < E; ++e) {
        double s = 0;
        for (long q = 0; q < n3; ++q) s += a[e * n3 + q];
        part[e] = s;
    }
    double s = 0;
    for (int e = 0; e < E; ++e) s += part[e];
    free(part);
    return s;
}

/* ------------------------------------------------------------------ */
/* Element-local operators (sum factorisation).                         */
/* ------------------------------------------------------------------ */

/* reference derivatives of one element field: ur = D_r u, us = D_s u, ut = D_t u */
static void ref_grad(const orc_mesh* m, int e, const double* u, double* ur, double* us, double* ut)
{
    int lx = m->lx;
    const double* D = m->D;
    for (int k = 0; k < lx; ++k)
    for (int j = 0; j < lx; ++j)
    for (int i = 0; i < lx; ++i) {
        double a = 0, b = 0, c = 0;
        for (int l = 0; l < lx; ++l) {
            a += D[i * lx + l] * u[PT(m, e, l, j, k)];
            b += D[j * lx + l] * u[PT(m, e, i, l, k)];
            c += D[k * lx + l] * u[PT(m, e, i, j, l)];
        }
        int q = i + lx * (j + lx * k);
        ur[q] = a; us[q] = b; ut[q] = c;
    }
}

/* transposed reference derivatives: out = D_r^T fr + D_s^T fs + D_t^T ft */
static void ref_div_t(const orc_mesh* m, const double* fr, const double* fs, const double* ft, double* out)
{
    int lx = m->lx;
    const double* D = m->D;
    for (int k = 0; k < lx; ++k)
    for (int j = 0; j < lx; ++j)
    for (int i = 0; i < lx; ++i) {
        double s = 0;
        for (int l = 0; l < lx; ++l) {
            s += D[l * lx + i] * fr[l + lx * (j + lx * k)];
            s += D[l * lx + j] * fs[i + lx * (l + lx * k)];
            s += D[l * lx + k] * ft[i + lx * (j + lx * l)];
        }
        out[i + lx * (j + lx * k)] = s;
    }
}

/* Local Helmholtz operator w = h1 sum_ab D_a^T (G_ab o D_b u) + h2 B o u
 * (no assembly; apply orc_dssum for the assembled operator). */
void orc_ax(const orc_mesh* m, const double* u, double* w, double h1, double h2)
{
    int lx = m->lx;
    long n3 = (long)lx * lx * lx, np = m->np;
    #pragma omp parallel
    {
        double ur[ORC_MAXLX * ORC_MAXLX * ORC_MAXLX], us[ORC_MAXLX * ORC_MAXLX * ORC_MAXLX],
               ut[ORC_MAXLX * ORC_MAXLX * ORC_MAXLX], o[ORC_MAXLX * ORC_MAXLX * ORC_MAXLX];
        #pragma omp for
        for (int e = 0; e < m->E; ++e) {
            ref_grad(m, e, u, ur, us, ut);
            for (long q = 0; q < n3; ++q) {
                long p = e * n3 + q;
                double grr = m->G[p], grs = m->G[np + p], grt = m->G[2 * np + p];
                double gss = m->G[3 * np + p], gst = m->G[4 * np + p], gtt = m->G[5 * np + p];
                double a = ur[q], b = us[q], c = ut[q];
                ur[q] = grr * a + grs * b + grt * c;
                us[q] = grs * a + gss * b + gst * c;
                ut[q] = grt * a + gst * b + gtt * c;
            }
            ref_div_t(m, ur, us, ut, o);
            for (long q = 0; q < n3; ++q) {
                long p = e * n3 + q;
                w[p] = h1 * o[q] + h2 * m->B[p] * u[p];
            }
        }
    }
}

/* Exact diagonal of the local Helmholtz operator, including the G cross
 * terms that survive at element-boundary nodes (D has a non-zero diagonal
 * only at the two end nodes). */
void orc_diag(const orc_mesh* m, double h1, double h2, double* d)
{
    int lx = m->lx;
    long np = m->np;
    const double* D = m->D;
    #pragma omp parallel for
    for (int e = 0; e < m->E; ++e)
        for (int k = 0; k < lx; ++k)
        for (int j = 0; j < lx; ++j)
        for (int i = 0; i < lx; ++i) {
            long p = PT(m, e, i, j, k);
            double s = 0;
            for (int l = 0; l < lx; ++l) {
                s += D[l * lx + i] * D[l * lx + i] * m->G[0 * np + PT(m, e, l, j, k)];
                s += D[l * lx + j] * D[l * lx + j] * m->G[3 * np + PT(m, e, i, l, k)];
                s += D[l * lx + k] * D[l * lx + k] * m->G[5 * np + PT(m, e, i, j, l)];
            }
            double dii = D[i * lx + i], djj = D[j * lx + j], dkk = D[k * lx + k];
            s += 2.0 * dii * djj * m->G[1 * np + p];
            s += 2.0 * dii * dkk * m->G[2 * np + p];
            s += 2.0 * djj * dkk * m->G[4 * np + p];
            d[p] = h1 * s + h2 * m->B[p];
        }
}

/* Physical gradient of a scalar: g_c = sum_a (dr_a/dx_c) D_a u. */
void orc_grad(const orc_mesh* m, const double* u, double* gx, double* gy, double* gz)
{
    int lx = m->lx;
    long n3 = (long)lx * lx * lx, np = m->np;
    #pragma omp parallel
    {
        double ur[ORC_MAXLX * ORC_MAXLX * ORC_MAXLX], us[ORC_MAXLX * ORC_MAXLX * ORC_MAXLX],
               ut[ORC_MAXLX * ORC_MAXLX * ORC_MAXLX];
        #pragma omp for
        for (int e = 0; e < m->E; ++e) {
            ref_grad(m, e, u, ur, us, ut);
            for (long q = 0; q < n3; ++q) {
                long p = e * n3 + q;
                double g[3];
                for (int c = 0; c < 3; ++c)
                    g[c] = m->drdx[(long)(0 * 3 + c) * np + p] * ur[q]
                         + m->drdx[(long)(1 * 3 + c) * np + p] * us[q]
                         + m->drdx[(long)(2 * 3 + c) * np + p] * ut[q];
                gx[p] = g[0]; gy[p] = g[1]; gz[p] = g[2];
            }
        }
    }
}

/* Mass-weighted gradient (B grad p)_c = sum_a M_ac D_a p. */
void orc_opgrad(const orc_mesh* m, const double* p_, double* ox, double* oy, double* oz)
{
    int lx = m->lx;
    long n3 = (long)lx * lx * lx, np = m->np;
    #pragma omp parallel
    {
        double ur[ORC_MAXLX * ORC_MAXLX * ORC_MAXLX], us[ORC_MAXLX * ORC_MAXLX * ORC_MAXLX],
               ut[ORC_MAXLX * ORC_MAXLX * ORC_MAXLX];
        #pragma omp for
        for (int e = 0; e < m->E; ++e) {
            ref_grad(m, e, p_, ur, us, ut);
            for (long q = 0; q < n3; ++q) {
                long p = e * n3 + q;
                double g[3];
                for (int c = 0; c < 3; ++c)
                    g[c] = m->M[(long)(0 * 3 + c) * np + p] * ur[q]
                         + m->M[(long)(1 * 3 + c) * np + p] * us[q]
                         + m->M[(long)(2 * 3 + c) * np + p] * ut[q];
                ox[p] = g[0]; oy[p] = g[1]; oz[p] = g[2];
            }
        }
    }
}

/* Weak divergence of a vector field: out = sum_a D_a^T (sum_c M_ac v_c),
 * i.e. the integral of grad(test) . v for every test basis function. */
void orc_wdiv(const orc_mesh* m, const double* vx, const double* vy, const double* vz, double* out)
{
    int lx = m->lx;
    long n3 = (long)lx * lx * lx, np = m->np;
    #pragma omp parallel
    {
        double fr[ORC_MAXLX * ORC_MAXLX * ORC_MAXLX], fs[ORC_MAXLX * ORC_MAXLX * ORC_MAXLX],
               ft[ORC_MAXLX * ORC_MAXLX * ORC_MAXLX], o[ORC_MAXLX * ORC_MAXLX * ORC_MAXLX];
        #pragma omp for
        for (int e = 0; e < m->E; ++e) {
            for (long q = 0; q < n3; ++q) {
                long p = e * n3 + q;
                double v[3] = { vx[p], vy[p], vz[p] };
                double f[3];
                for (int a = 0; a < 3; ++a) {
                    f[a] = 0;
                    for (int c = 0; c < 3; ++c) f[a] += m->M[(long)(a * 3 + c) * np + p] * v[c];
                }
                fr[q] = f[0]; fs[q] = f[1]; ft[q] = f[2];
            }
            ref_div_t(m, fr, fs, ft, o);
            for (long q = 0; q < n3; ++q) out[e * n3 + q] = o[q];
        }
    }
}

/* Convective term in collocation form, mass weighted:
 * bn_i = -sum_c u_c sum_a M_ac D_a u_i  (= -B (u . grad) u_i). */
void orc_conv(const orc_mesh* m, const double* ux, const double* uy, const double* uz,
              double* bx, double* by, double* bz)
{
    int lx = m->lx;
    long n3 = (long)lx * lx * lx, np = m->np;
    const double* U[3] = { ux, uy, uz };
    double* O[3] = { bx, by, bz };
    #pragma omp parallel
    {
        double ur[ORC_MAXLX * ORC_MAXLX * ORC_MAXLX], us[ORC_MAXLX * ORC_MAXLX * ORC_MAXLX],
               ut[ORC_MAXLX * ORC_MAXLX * ORC_MAXLX];
        #pragma omp for
        for (int e = 0; e < m->E; ++e) {
            for (int f = 0; f < 3; ++f) {
                ref_grad(m, e, U[f], ur, us, ut);
                for (long q = 0; q < n3; ++q) {
                    long p = e * n3 + q;
                    double s = 0;
                    for (int c = 0; c < 3; ++c) {
                        double bg = m->M[(long)(0 * 3 + c) * np + p] * ur[q]
                                  + m->M[(long)(1 * 3 + c) * np + p] * us[q]
                                  + m->M[(long)(2 * 3 + c) * np + p] * ut[q];
                        s += U[c][p] * bg;
                    }
                    O[f][p] = -s;
                }
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* Dealiased convection (3/2 rule): the convective term is integrated   */
/* on lxd = ceil(3 lx / 2) Gauss-Legendre points per direction instead  */
/* of by collocation on the GLL points (the paper runs with dealiasing, */
/* Sec. 3).  Velocity and its reference derivatives are interpolated to */
/* the fine points, the geometry there comes from the interpolated      */
/* coordinates, and the weighted integrand is tested against every GLL  */
/* basis function (transposed interpolation):                            */
/*   BN_f(l) = - sum_q w_q jac_q phi_l(z_q) sum_c u_c(z_q) du_f/dx_c(z_q) */
/* ------------------------------------------------------------------ */
#define ORC_MAXLXD 24

int orc_lxd(int lx) { return (3 * lx + 1) / 2; }

/* Gauss-Legendre nodes (roots of P_n) and weights 2 / ((1 - z^2) P_n'(z)^2). */
int orc_gl(int n, double* z, double* w)
{
    if (n < 1 || n > ORC_MAXLXD) return -1;
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        double x = -cos(pi * (i + 0.75) / (n + 0.5));   /* Chebyshev-like start */
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(n, x, &P, &dP);
            double dx = P / dP;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        double P, dP;
        legendre(n, x, &P, &dP);
        z[i] = x;
        w[i] = 2.0 / ((1.0 - x * x) * dP * dP);
    }
    /* symmetric node set */
    for (int i = 0; i < n / 2; ++i) {
        double a = 0.5 * (z[n - 1 - i] - z[i]);
        z[i] = -a; z[n - 1 - i] = a;
        double b = 0.5 * (w[i] + w[n - 1 - i]);
        w[i] = b; w[n - 1 - i] = b;
    }
    if (n % 2) z[n / 2] = 0.0;
    return 0;
}

/* Lagrange basis of the GLL nodes xi (lx of them) at the points z (nz):
 * I[q * lx + l] = prod_{m != l} (z_q - xi_m) / (xi_l - xi_m). */
void orc_interp(int lx, const double* xi, int nz, const double* z, double* I)
{
    for (int q = 0; q < nz; ++q)
        for (int l = 0; l < lx; ++l) {
            double v = 1.0;
            for (int mm = 0; mm < lx; ++mm)
                if (mm != l) v *= (z[q] - xi[mm]) / (xi[l] - xi[mm]);
            I[q * lx + l] = v;
        }
}

/* out[c3][c2][c1] = sum A1[c1][a] A2[c2][b] A3[c3][c] in[c][b][a] with
 * A_d of size (nout_d x nin): the tensor-product map of three 1D matrices
 * (index order k slowest, i fastest on both sides). */
static void tensor3(int nin, int n1, int n2, int n3, const double* A1, const double* A2, const double* A3,
                    const double* in, double* out)
{
    double t1[ORC_MAXLXD * ORC_MAXLXD * ORC_MAXLXD], t2[ORC_MAXLXD * ORC_MAXLXD * ORC_MAXLXD];
    /* along i */
    for (int c = 0; c < nin; ++c)
        for (int b = 0; b < nin; ++b)
            for (int i = 0; i < n1; ++i) {
                double s = 0;
                for (int a = 0; a < nin; ++a) s += A1[i * nin + a] * in[a + nin * (b + nin * c)];
                t1[i + n1 * (b + nin * c)] = s;
            }
    /* along j */
    for (int c = 0; c < nin; ++c)
        for (int j = 0; j < n2; ++j)
            for (int i = 0; i < n1; ++i) {
                double s = 0;
                for (int b = 0; b < nin; ++b) s += A2[j * nin + b] * t1[i + n1 * (b + nin * c)];
                t2[i + n1 * (j + n2 * c)] = s;
            }
    /* along k */
    for (int k = 0; k < n3; ++k)
        for (int j = 0; j < n2; ++j)
            for (int i = 0; i < n1; ++i) {
                double s = 0;
                for (int c = 0; c < nin; ++c) s += A3[k * nin + c] * t2[i + n1 * (j + n2 * c)];
                out[i + n1 * (j + n2 * k)] = s;
            }
}

/* transposed map: out[c][b][a] = sum_{k,j,i} A1[i][a] A2[j][b] A3[k][c] in[k][j][i] */
static void tensor3_t(int nout, int n1, int n2, int n3, const double* A1, const double* A2, const double* A3,
                      const double* in, double* out)
{
    double t1[ORC_MAXLXD * ORC_MAXLXD * ORC_MAXLXD], t2[ORC_MAXLXD * ORC_MAXLXD * ORC_MAXLXD];
    for (int k = 0; k < n3; ++k)
        for (int j = 0; j < n2; ++j)
            for (int a = 0; a < nout; ++a) {
                double s = 0;
                for (int i = 0; i < n1; ++i) s += A1[i * nout + a] * in[i + n1 * (j + n2 * k)];
                t1[a + nout * (j + n2 * k)] = s;
            }
    for (int k = 0; k < n3; ++k)
        for (int b = 0; b < nout; ++b)
            for (int a = 0; a < nout; ++a) {
                double s = 0;
                for (int j = 0; j < n2; ++j) s += A2[j * nout + b] * t1[a + nout * (j + n2 * k)];
                t2[a + nout * (b + nout * k)] = s;
            }
    for (int c = 0; c < nout; ++c)
        for (int b = 0; b < nout; ++b)
            for (int a = 0; a < nout; ++a) {
                double s = 0;
                for (int k = 0; k < n3; ++k) s += A3[k * nout + c] * t2[a + nout * (b + nout * k)];
                out[a + nout * (b + nout * c)] = s;
            }
}

void orc_conv_dealias(const orc_mesh* m, const double* ux, const double* uy, const double* uz,
                      double* bx, double* by, double* bz)
{
    const int lx = m->lx, nd = orc_lxd(lx);
    const long n3 = (long)lx * lx * lx, np = m->np;
    const long nd3 = (long)nd * nd * nd;
    double z[ORC_MAXLXD], wz[ORC_MAXLXD], I[ORC_MAXLXD * ORC_MAXLX], ID[ORC_MAXLXD * ORC_MAXLX];
    orc_gl(nd, z, wz);
    orc_interp(lx, m->xi, nd, z, I);
    /* derivative values at the fine points: ID = I D (D u holds the nodal
     * values of the derivative polynomial, which I interpolates exactly) */
    for (int q = 0; q < nd; ++q)
        for (int l = 0; l < lx; ++l) {
            double s = 0;
            for (int mm = 0; mm < lx; ++mm) s += I[q * lx + mm] * m->D[mm * lx + l];
            ID[q * lx + l] = s;
        }
    const double* U[3] = { ux, uy, uz };
    double* O[3] = { bx, by, bz };
    #pragma omp parallel
    {
        double* xr = dalloc(9 * nd3);     /* xr[(c*3+a)] = d x_c / d r_a at fine points */
        double* rx = dalloc(9 * nd3);     /* rx[(a*3+c)] = d r_a / d x_c times the fine weight W */
        double* uf = dalloc(3 * nd3);     /* velocity at fine points */
        double* g = dalloc(3 * nd3);      /* reference derivatives of one component */
        double* t = dalloc(nd3);
        double ue[ORC_MAXLX * ORC_MAXLX * ORC_MAXLX], o[ORC_MAXLX * ORC_MAXLX * ORC_MAXLX];
        #pragma omp for
        for (int e = 0; e < m->E; ++e) {
            /* geometry at the fine points from the interpolated coordinates */
            for (int c = 0; c < 3; ++c) {
                for (long q = 0; q < n3; ++q) ue[q] = m->xyz[(long)c * np + e * n3 + q];
                tensor3(lx, nd, nd, nd, ID, I, I, ue, xr + (long)(c * 3 + 0) * nd3);
                tensor3(lx, nd, nd, nd, I, ID, I, ue, xr + (long)(c * 3 + 1) * nd3);
                tensor3(lx, nd, nd, nd, I, I, ID, ue, xr + (long)(c * 3 + 2) * nd3);
            }
            for (int k = 0; k < nd; ++k)
            for (int j = 0; j < nd; ++j)
            for (int i = 0; i < nd; ++i) {
                long q = i + nd * (j + (long)nd * k);
                double J[3][3];
                for (int c = 0; c < 3; ++c)
                    for (int a = 0; a < 3; ++a) J[c][a] = xr[(long)(c * 3 + a) * nd3 + q];
                double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
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
                double W = det * wz[i] * wz[j] * wz[k];
                for (int a = 0; a < 3; ++a)
                    for (int c = 0; c < 3; ++c) rx[(long)(a * 3 + c) * nd3 + q] = W * inv[a][c];
            }
            for (int c = 0; c < 3; ++c) {
                for (long q = 0; q < n3; ++q) ue[q] = U[c][e * n3 + q];
                tensor3(lx, nd, nd, nd, I, I, I, ue, uf + (long)c * nd3);
            }
            for (int f = 0; f < 3; ++f) {
                for (long q = 0; q < n3; ++q) ue[q] = U[f][e * n3 + q];
                tensor3(lx, nd, nd, nd, ID, I, I, ue, g);
                tensor3(lx, nd, nd, nd, I, ID, I, ue, g + nd3);
                tensor3(lx, nd, nd, nd, I, I, ID, ue, g + 2 * nd3);
                for (long q = 0; q < nd3; ++q) {
                    double s = 0;
                    for (int c = 0; c < 3; ++c) {
                        double dx = 0;
                        for (int a = 0; a < 3; ++a) dx += rx[(long)(a * 3 + c) * nd3 + q] * g[(long)a * nd3 + q];
                        s += uf[(long)c * nd3 + q] * dx;
                    }
                    t[q] = s;
                }
                tensor3_t(lx, nd, nd, nd, I, I, I, t, o);
                for (long q = 0; q < n3; ++q) O[f][e * n3 + q] = -o[q];
            }
        }
        free(xr); free(rx); free(uf); free(g); free(t);
    }
}

/* Element-local vorticity and divergence (no inter-element averaging). */
void orc_curl_div(const orc_mesh* m, const double* ux, const double* uy, const double* uz,
                  double* wx, double* wy, double* wz, double* dv)
{
    long np = m->np;
    double* g = dalloc(9 * np);      /* g[(f*3+c)] = d u_f / d x_c */
    orc_grad(m, ux, g, g + np, g + 2 * np);
    orc_grad(m, uy, g + 3 * np, g + 4 * np, g + 5 * np);
    orc_grad(m, uz, g + 6 * np, g + 7 * np, g + 8 * np);
    #pragma omp parallel for
    for (long p = 0; p < np; ++p) {
        double dudy = g[1 * np + p], dudz = g[2 * np + p];
        double dvdx = g[3 * np + p], dvdz = g[5 * np + p];
        double dwdx = g[6 * np + p], dwdy = g[7 * np + p];
        wx[p] = dwdy - dvdz;
        wy[p] = dudz - dwdx;
        wz[p] = dvdx - dudy;
        dv[p] = g[0 * np + p] + g[4 * np + p] + g[8 * np + p];
    }
    free(g);
}

/* Volume-averaged kinetic energy (1/|V|) int 1/2 |u|^2, enstrophy
 * (1/|V|) int 1/2 |omega|^2 and the largest pointwise |div u|. */
void orc_diagnostics(const orc_mesh* m, const double* ux, const double* uy, const double* uz,
                     double* ke, double* enst, double* maxdiv)
{
    long np = m->np;
    double* wx = dalloc(np); double* wy = dalloc(np); double* wz = dalloc(np); double* dv = dalloc(np);
    double* a = dalloc(np); double* b = dalloc(np);
    orc_curl_div(m, ux, uy, uz, wx, wy, wz, dv);
    double md = 0;
    for (long p = 0; p < np; ++p) {
        a[p] = m->B[p] * 0.5 * (ux[p] * ux[p] + uy[p] * uy[p] + uz[p] * uz[p]);
        b[p] = m->B[p] * 0.5 * (wx[p] * wx[p] + wy[p] * wy[p] + wz[p] * wz[p]);
        if (fabs(dv[p]) > md) md = fabs(dv[p]);
    }
    *ke = orc_sum(m, a) / m->vol;
    *enst = orc_sum(m, b) / m->vol;
    *maxdiv = md;
    free(wx); free(wy); free(wz); free(dv); free(a); free(b);
}

/* ------------------------------------------------------------------ */
/* Krylov solvers on the assembled operator  x -> dssum(A_L x).          */
/* ------------------------------------------------------------------ */
static void apply_assembled(const orc_mesh* m, const double* x, double* y, double h1, double h2)
{
    orc_ax(m, x, y, h1, h2);
    orc_dssum(m, y);
}

/* Jacobi-preconditioned CG for (h1 A + h2 B) x = b, assembled.  x holds the
 * initial guess on entry.  Stops when sqrt((r,r)) <= tol or after maxit
 * iterations.  Returns the iteration count; *res gets the final residual
 * norm (recurrence).  Optional hist[maxit+1] receives the residual history. */
int orc_pcg(const orc_mesh* m, double h1, double h2, const double* b, double* x,
            double tol, int maxit, double* res, double* hist)
{
    long np = m->np;
    double* r = dalloc(np); double* z = dalloc(np); double* p = dalloc(np);
    double* w = dalloc(np); double* d = dalloc(np);
    orc_diag(m, h1, h2, d);
    orc_dssum(m, d);
    apply_assembled(m, x, w, h1, h2);
    for (long i = 0; i < np; ++i) r[i] = b[i] - w[i];
    double rn = sqrt(orc_glsc(m, r, r));
    if (hist) hist[0] = rn;
    int it = 0;
    if (rn > tol) {
        for (long i = 0; i < np; ++i) { z[i] = r[i] / d[i]; p[i] = z[i]; }
        double rho = orc_glsc(m, r, z);
        while (it < maxit) {
            apply_assembled(m, p, w, h1, h2);
            double alpha = rho / orc_glsc(m, p, w);
            for (long i = 0; i < np; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * w[i]; }
            ++it;
            rn = sqrt(orc_glsc(m, r, r));
            if (hist) hist[it] = rn;
            if (rn <= tol) break;
            for (long i = 0; i < np; ++i) z[i] = r[i] / d[i];
            double rho1 = orc_glsc(m, r, z);
            double beta = rho1 / rho;
            rho = rho1;
            for (long i = 0; i < np; ++i) p[i] = z[i] + beta * p[i];
        }
    }
    if (res) *res = rn;
    free(r); free(z); free(p); free(w); free(d);
    return it;
}

/* Right-Jacobi-preconditioned restarted GMRES(mrst) for the assembled
 * Helmholtz operator (h1 A + h2 B) x = b.  Arnoldi with classical
 * Gram-Schmidt applied twice, Givens rotations on the Hessenberg matrix,
 * absolute stop on the rotated residual |g_{j+1}| <= tol, and the true
 * residual recomputed at every restart.  x holds the initial guess.
 * With deflate != 0 (the singular periodic Poisson operator, whose range is
 * orthogonal to constants) each operator output has its unique-node mean
 * removed before orthogonalisation: a no-op in exact arithmetic that keeps
 * rounding errors from feeding the constant null direction into the basis.
 * Returns the number of Arnoldi steps; *res = final true residual norm. */
typedef struct orc_hsmg orc_hsmg;
void orc_hsmg_apply(const orc_hsmg* H, const double* r, double* z);

/* GMRES right-preconditioned by Jacobi (pc == NULL) or by the HSMG
 * preconditioner pc (defined further down): z_j = M^{-1} v_j and, at each
 * cycle end, x += M^{-1} (V y); M^{-1} is linear in both cases. */
static int gmres_pc(const orc_mesh* m, double h1, double h2, const double* b, double* x,
                    double tol, int maxit, int mrst, int deflate, const orc_hsmg* pc, double* res, double* hist);

int orc_gmres_ex(const orc_mesh* m, double h1, double h2, const double* b, double* x,
                 double tol, int maxit, int mrst, int deflate, double* res, double* hist)
{
    return gmres_pc(m, h1, h2, b, x, tol, maxit, mrst, deflate, NULL, res, hist);
}

static int gmres_pc(const orc_mesh* m, double h1, double h2, const double* b, double* x,
                    double tol, int maxit, int mrst, int deflate, const orc_hsmg* pc, double* res, double* hist)
{
    long np = m->np;
    int mm = mrst;
    double* V = dalloc((long)(mm + 1) * np);
    double* w = dalloc(np); double* z = dalloc(np); double* d = dalloc(np); double* r = dalloc(np);
    double* H = dalloc((long)(mm + 1) * mm);    /* H[i*mm + j] */
    double* cs = dalloc(mm); double* sn = dalloc(mm); double* g = dalloc(mm + 1);
    double* y = dalloc(mm); double* hc = dalloc(mm + 1); double* h2v = dalloc(mm + 1);
    orc_diag(m, h1, h2, d);
    orc_dssum(m, d);
    int it = 0;
    double beta = 0;
    int hpos = 0;
    for (;;) {
        apply_assembled(m, x, w, h1, h2);
        for (long i = 0; i < np; ++i) r[i] = b[i] - w[i];
        beta = sqrt(orc_glsc(m, r, r));
        if (hist) hist[hpos++] = beta;
        if (beta <= tol || it >= maxit) break;
        for (long i = 0; i < np; ++i) V[i] = r[i] / beta;
        for (int i = 0; i <= mm; ++i) g[i] = 0;
        g[0] = beta;
        int jend = 0;
        for (int j = 0; j < mm && it < maxit; ++j) {
            double* vj = V + (long)j * np;
            if (pc) orc_hsmg_apply(pc, vj, z);
            else for (long i = 0; i < np; ++i) z[i] = vj[i] / d[i];
            apply_assembled(m, z, w, h1, h2);
            if (deflate) orc_remove_mean_unique(m, w);
            /* classical Gram-Schmidt, twice */
            for (int i = 0; i <= j; ++i) hc[i] = 0;
            for (int pass = 0; pass < 2; ++pass) {
                for (int i = 0; i <= j; ++i) h2v[i] = orc_glsc(m, V + (long)i * np, w);
                for (int i = 0; i <= j; ++i) {
                    const double* vi = V + (long)i * np;
                    double hi = h2v[i];
                    for (long q = 0; q < np; ++q) w[q] -= hi * vi[q];
                    hc[i] += hi;
                }
            }
            double hn = sqrt(orc_glsc(m, w, w));
            for (int i = 0; i <= j; ++i) H[i * mm + j] = hc[i];
            H[(j + 1) * mm + j] = hn;
            double* vn = V + (long)(j + 1) * np;
            if (hn != 0.0) for (long q = 0; q < np; ++q) vn[q] = w[q] / hn;
            /* apply previous rotations to column j, then form the new one */
            for (int i = 0; i < j; ++i) {
                double a = H[i * mm + j], c = H[(i + 1) * mm + j];
                H[i * mm + j] = cs[i] * a + sn[i] * c;
                H[(i + 1) * mm + j] = -sn[i] * a + cs[i] * c;
            }
            double a = H[j * mm + j], c = H[(j + 1) * mm + j];
            double den = sqrt(a * a + c * c);
            cs[j] = a / den; sn[j] = c / den;
            H[j * mm + j] = den;
            H[(j + 1) * mm + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++it;
            jend = j + 1;
            if (hist) hist[hpos++] = fabs(g[j + 1]);
            if (fabs(g[j + 1]) <= tol || hn == 0.0) break;
        }
        /* back substitution H(0:jend,0:jend) y = g */
        for (int i = jend - 1; i >= 0; --i) {
            double s = g[i];
            for (int k = i + 1; k < jend; ++k) s -= H[i * mm + k] * y[k];
            y[i] = s / H[i * mm + i];
        }
        /* x += M^{-1} V y */
        for (long q = 0; q < np; ++q) {
            double s = 0;
            for (int i = 0; i < jend; ++i) s += V[(long)i * np + q] * y[i];
            z[q] = s;
        }
        if (pc) {
            orc_hsmg_apply(pc, z, w);
            for (long q = 0; q < np; ++q) x[q] += w[q];
        } else {
            for (long q = 0; q < np; ++q) x[q] += z[q] / d[q];
        }
    }
    if (res) *res = beta;
    free(V); free(w); free(z); free(d); free(r); free(H); free(cs); free(sn); free(g);
    free(y); free(hc); free(h2v);
    return it;
}

int orc_gmres(const orc_mesh* m, double h1, double h2, const double* b, double* x,
              double tol, int maxit, int mrst, double* res, double* hist)
{
    return orc_gmres_ex(m, h1, h2, b, x, tol, maxit, mrst, 0, res, hist);
}

/* Remove the arithmetic mean over unique nodes from an assembled vector. */
void orc_remove_mean_unique(const orc_mesh* m, double* r)
{
    long np = m->np;
    double* one = dalloc(np);
    for (long i = 0; i < np; ++i) one[i] = 1.0;
    double s = orc_glsc(m, r, one) / (double)m->nglob;
    for (long i = 0; i < np; ++i) r[i] -= s;
    free(one);
}

/* Remove the volume (mass-weighted) mean: x -= int x / |V|. */
void orc_remove_mean_mass(const orc_mesh* m, double* x)
{
    long np = m->np;
    double* a = dalloc(np);
    for (long i = 0; i < np; ++i) a[i] = m->B[i] * x[i];
    double s = orc_sum(m, a) / m->vol;
    for (long i = 0; i < np; ++i) x[i] -= s;
    free(a);
}

/* ------------------------------------------------------------------ */
/* Three-level hybrid Schwarz multigrid (HSMG) preconditioner of the   */
/* pressure Poisson operator.  Sec. 3 names GMRES preconditioned by a  */
/* three-level HSMG with a coarse-grid solve; it fixes no more than     */
/* that, so the operator is defined here (after Lottes & Fischer 2005, */
/* "Hybrid multigrid/Schwarz algorithms for the spectral element       */
/* method", with the additive form across levels):                     */
/*                                                                      */
/*   levels f (order N), m (order N_m = N/2), c (order 1), all on the   */
/*   same periodic box of equal elements;                               */
/*   M^{-1} r = S_f r + P_fm ( S_m r_m + P_mc A_c^+ R_cm r_m ),          */
/*   r_m = R_mf r.                                                       */
/*                                                                      */
/* S_l (levels f, m): additive Schwarz on element subdomains: for each   */
/* element the local problem L_e u = r_e (r_e = the element's copy of    */
/* the assembled residual) with the separable operator                  */
/*   L = B_z x B_y x A_x + B_z x A_y x B_x + A_z x B_y x B_x,            */
/* whose 1D matrices are the element's GLL stiffness and mass, extended  */
/* by one linear segment of length delta = (h/2)(xi_1 - xi_0) (the gap  */
/* to the next node inside the neighbour) ending at a zero Dirichlet    */
/* node on each side:                                                    */
/*   A = (2/h) D^T W D + (E_00 + E_NN) / delta,                          */
/*   B = (h/2) W       + (E_00 + E_NN) delta / 2;                        */
/* solved by fast diagonalisation (A S = B S Lambda, S^T B S = I); the   */
/* local solutions are summed over element copies (dssum) and weighted  */
/* by 1/multiplicity.                                                   */
/* P_fm, P_mc: tensor-product Lagrange interpolation from the coarser    */
/* level's GLL points to the finer level's, element by element.         */
/* R = P^T in the unique-node inner product: R r = dssum(P_e^T (r/mult)).*/
/* A_c^+: exact solve with the assembled order-1 SEM Poisson operator on */
/* the unique corner nodes, on the complement of the constant vector     */
/* (periodic: the operator is singular); separable on the box, so it is */
/* also solved by fast diagonalisation.                                  */
/* The symmetric eigenproblems use cyclic Jacobi rotations (Golub & Van */
/* Loan, Sec. 8.5).                                                     */
/* ------------------------------------------------------------------ */

/* Eigen-decomposition of the symmetric n x n matrix a (destroyed):
 * a = Q diag(lam) Q^T, Q[i*n + k] = component i of eigenvector k. */
static void jacobi_eig(int n, double* a, double* Q, double* lam)
{
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) Q[i * n + k] = i == k ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) {
                tot += a[i * n + k] * a[i * n + k];
                if (i != k) off += a[i * n + k] * a[i * n + k];
            }
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = a[p * n + q];
                if (apq == 0.0) continue;
                double theta = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < n; ++k) {        /* rows/cols p, q of a */
                    double akp = a[k * n + p], akq = a[k * n + q];
                    a[k * n + p] = c * akp - sn * akq;
                    a[k * n + q] = sn * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    double apk = a[p * n + k], aqk = a[q * n + k];
                    a[p * n + k] = c * apk - sn * aqk;
                    a[q * n + k] = sn * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    double qkp = Q[k * n + p], qkq = Q[k * n + q];
                    Q[k * n + p] = c * qkp - sn * qkq;
                    Q[k * n + q] = sn * qkp + c * qkq;
                }
            }
    }
    for (int i = 0; i < n; ++i) lam[i] = a[i * n + i];
}

/* Generalised problem A s = lambda B s with B diagonal positive (bd):
 * S = B^{-1/2} Q with Q the eigenvectors of B^{-1/2} A B^{-1/2}. */
static void gen_eig_diag(int n, const double* A, const double* bd, double* S, double* lam)
{
    double* C = dalloc((long)n * n);
    double* Q = dalloc((long)n * n);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) C[i * n + k] = A[i * n + k] / sqrt(bd[i] * bd[k]);
    jacobi_eig(n, C, Q, lam);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) S[i * n + k] = Q[i * n + k] / sqrt(bd[i]);
    free(C); free(Q);
}

typedef struct {
    int N, lx;
    double xi[ORC_MAXLX], w[ORC_MAXLX], D[ORC_MAXLX * ORC_MAXLX];
    double A[3][ORC_MAXLX * ORC_MAXLX], Bd[3][ORC_MAXLX];   /* local 1D matrices (B diagonal) */
    double S[3][ORC_MAXLX * ORC_MAXLX], lam[3][ORC_MAXLX];  /* their fast diagonalisation */
} hs_level;

struct orc_hsmg {
    const orc_mesh* m;
    int nel[3], E;
    hs_level lv[2];                 /* 0 = fine, 1 = middle */
    double* Jfm;                    /* lx_f x lx_m: fine GLL points from middle Lagrange basis */
    double* Jmc;                    /* lx_m x 2 */
    double* Sc[3]; double* lamc[3]; /* coarse 1D periodic fast diagonalisation, n_c x n_c */
    int c0[3];                      /* index of the constant (zero-eigenvalue) mode per direction */
    long nm;                        /* middle-level local points E * lx_m^3 */
    long* gid_m; int* mult_m; long nglob_m;
    long nc;                        /* unique coarse nodes */
};

static void hs_level_init(hs_level* L, int N, const double h[3])
{
    L->N = N; L->lx = N + 1;
    int lx = L->lx;
    orc_gll(N, L->xi, L->w);
    orc_deriv(N, L->xi, L->D);
    for (int c = 0; c < 3; ++c) {
        double delta = 0.5 * h[c] * (L->xi[1] - L->xi[0]);
        for (int i = 0; i < lx; ++i)
            for (int j = 0; j < lx; ++j) {
                double s = 0.0;     /* (D^T W D)_ij */
                for (int q = 0; q < lx; ++q) s += L->D[q * lx + i] * L->w[q] * L->D[q * lx + j];
                L->A[c][i * lx + j] = 2.0 / h[c] * s;
            }
        for (int i = 0; i < lx; ++i) L->Bd[c][i] = 0.5 * h[c] * L->w[i];
        L->A[c][0] += 1.0 / delta; L->A[c][N * lx + N] += 1.0 / delta;
        L->Bd[c][0] += 0.5 * delta; L->Bd[c][N] += 0.5 * delta;
        gen_eig_diag(lx, L->A[c], L->Bd[c], L->S[c], L->lam[c]);
    }
}

orc_hsmg* orc_hsmg_new(const orc_mesh* m)
{
    if (m->amp != 0.0 || m->N < 4) return NULL;
    orc_hsmg* H = (orc_hsmg*)calloc(1, sizeof(orc_hsmg));
    H->m = m; H->E = m->E;
    for (int c = 0; c < 3; ++c) H->nel[c] = m->nel[c];
    hs_level_init(&H->lv[0], m->N, m->h);
    hs_level_init(&H->lv[1], m->N / 2, m->h);
    const int lxf = H->lv[0].lx, lxm = H->lv[1].lx;
    H->Jfm = dalloc((long)lxf * lxm);
    orc_interp(lxm, H->lv[1].xi, lxf, H->lv[0].xi, H->Jfm);
    double xc[2] = {-1.0, 1.0};
    H->Jmc = dalloc((long)lxm * 2);
    orc_interp(2, xc, lxm, H->lv[1].xi, H->Jmc);
    /* middle-level periodic numbering */
    const int Nm = H->lv[1].N;
    H->nm = (long)m->E * lxm * lxm * lxm;
    long ngx = (long)m->nel[0] * Nm, ngy = (long)m->nel[1] * Nm, ngz = (long)m->nel[2] * Nm;
    H->nglob_m = ngx * ngy * ngz;
    H->gid_m = (long*)calloc((size_t)H->nm, sizeof(long));
    H->mult_m = (int*)calloc((size_t)H->nm, sizeof(int));
    for (int ez = 0; ez < m->nel[2]; ++ez)
    for (int ey = 0; ey < m->nel[1]; ++ey)
    for (int ex = 0; ex < m->nel[0]; ++ex) {
        int e = ex + m->nel[0] * (ey + m->nel[1] * ez);
        for (int k = 0; k < lxm; ++k)
        for (int j = 0; j < lxm; ++j)
        for (int i = 0; i < lxm; ++i) {
            long p = (long)e * lxm * lxm * lxm + i + lxm * (j + lxm * k);
            long gx = ((long)ex * Nm + i) % ngx, gy = ((long)ey * Nm + j) % ngy, gz = ((long)ez * Nm + k) % ngz;
            H->gid_m[p] = gx + ngx * (gy + ngy * gz);
        }
    }
    int* cnt = (int*)calloc((size_t)H->nglob_m, sizeof(int));
    for (long p = 0; p < H->nm; ++p) cnt[H->gid_m[p]]++;
    for (long p = 0; p < H->nm; ++p) H->mult_m[p] = cnt[H->gid_m[p]];
    free(cnt);
    /* coarse 1D periodic operators: element k joins nodes k and k+1 (mod n) */
    H->nc = (long)m->nel[0] * m->nel[1] * m->nel[2];
    for (int c = 0; c < 3; ++c) {
        int n = m->nel[c];
        double h = m->h[c];
        double* A = dalloc((long)n * n);
        double* bd = dalloc(n);
        for (int k = 0; k < n; ++k) {
            int a = k, b = (k + 1) % n;
            A[a * n + a] += 1.0 / h; A[b * n + b] += 1.0 / h;
            A[a * n + b] -= 1.0 / h; A[b * n + a] -= 1.0 / h;
            bd[a] += 0.5 * h; bd[b] += 0.5 * h;
        }
        H->Sc[c] = dalloc((long)n * n); H->lamc[c] = dalloc(n);
        gen_eig_diag(n, A, bd, H->Sc[c], H->lamc[c]);
        int i0 = 0;
        for (int i = 1; i < n; ++i) if (H->lamc[c][i] < H->lamc[c][i0]) i0 = i;
        H->c0[c] = i0;
        free(A); free(bd);
    }
    return H;
}

void orc_hsmg_free(orc_hsmg* H)
{
    if (!H) return;
    free(H->Jfm); free(H->Jmc); free(H->gid_m); free(H->mult_m);
    for (int c = 0; c < 3; ++c) { free(H->Sc[c]); free(H->lamc[c]); }
    free(H);
}

/* 1D tables of one level (0 fine, 1 middle), direction c: A (lx*lx), the
 * diagonal of B (lx), S (lx*lx), lambda (lx).  Returns lx. */
int orc_hsmg_level(const orc_hsmg* H, int level, int c, double* A, double* Bd, double* S, double* lam)
{
    const hs_level* L = &H->lv[level];
    int lx = L->lx;
    if (A) memcpy(A, L->A[c], sizeof(double) * lx * lx);
    if (Bd) memcpy(Bd, L->Bd[c], sizeof(double) * lx);
    if (S) memcpy(S, L->S[c], sizeof(double) * lx * lx);
    if (lam) memcpy(lam, L->lam[c], sizeof(double) * lx);
    return lx;
}

/* Local solve u = L^{-1} r of one element at level L (lx^3 values):
 * u = (S_z x S_y x S_x) diag(1 / (lam_x + lam_y + lam_z)) (S_z x S_y x S_x)^T r. */
static void hs_local_solve(const hs_level* L, const double* r, double* u)
{
    int lx = L->lx;
    long n3 = (long)lx * lx * lx;
    double St[3][ORC_MAXLX * ORC_MAXLX];
    for (int c = 0; c < 3; ++c)
        for (int i = 0; i < lx; ++i)
            for (int k = 0; k < lx; ++k) St[c][k * lx + i] = L->S[c][i * lx + k];
    double* t = dalloc(n3);
    tensor3(lx, lx, lx, lx, St[0], St[1], St[2], r, t);
    for (int k = 0; k < lx; ++k)
        for (int j = 0; j < lx; ++j)
            for (int i = 0; i < lx; ++i)
                t[i + lx * (j + lx * k)] /= L->lam[0][i] + L->lam[1][j] + L->lam[2][k];
    tensor3(lx, lx, lx, lx, L->S[0], L->S[1], L->S[2], t, u);
    free(t);
}

void orc_hsmg_local_solve(const orc_hsmg* H, int level, const double* r, double* u)
{
    hs_local_solve(&H->lv[level], r, u);
}

/* Exact coarse solve: rc, ec on the unique corner nodes (cx + nx (cy + ny cz));
 * the constant mode is dropped. */
void orc_hsmg_coarse_solve(const orc_hsmg* H, const double* rc, double* ec)
{
    const int nx = H->nel[0], ny = H->nel[1], nz = H->nel[2];
    double* St[3];
    for (int c = 0; c < 3; ++c) {
        int n = H->nel[c];
        St[c] = dalloc((long)n * n);
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) St[c][k * n + i] = H->Sc[c][i * n + k];
    }
    double* t = dalloc(H->nc);
    /* tensor3 takes equal input extents; apply the three directions one by one */
    double* u = dalloc(H->nc);
    memcpy(u, rc, sizeof(double) * H->nc);
    for (int pass = 0; pass < 2; ++pass) {
        for (int dir = 0; dir < 3; ++dir) {
            const double* Mt = pass == 0 ? St[dir] : H->Sc[dir];
            int n = H->nel[dir];
            for (int cz = 0; cz < nz; ++cz)
            for (int cy = 0; cy < ny; ++cy)
            for (int cx = 0; cx < nx; ++cx) {
                int o[3] = {cx, cy, cz};
                double s = 0.0;
                for (int a = 0; a < n; ++a) {
                    int q[3] = {cx, cy, cz};
                    q[dir] = a;
                    s += Mt[o[dir] * n + a] * u[q[0] + (long)nx * (q[1] + (long)ny * q[2])];
                }
                t[cx + (long)nx * (cy + (long)ny * cz)] = s;
            }
            memcpy(u, t, sizeof(double) * H->nc);
        }
        if (pass == 0)
            for (int cz = 0; cz < nz; ++cz)
            for (int cy = 0; cy < ny; ++cy)
            for (int cx = 0; cx < nx; ++cx) {
                long q = cx + (long)nx * (cy + (long)ny * cz);
                if (cx == H->c0[0] && cy == H->c0[1] && cz == H->c0[2]) u[q] = 0.0;
                else u[q] /= H->lamc[0][cx] + H->lamc[1][cy] + H->lamc[2][cz];
            }
    }
    memcpy(ec, u, sizeof(double) * H->nc);
    free(t); free(u);
    for (int c = 0; c < 3; ++c) free(St[c]);
}

/* element e's middle-level local block of a middle-level vector */
#define HSM(H, e) ((long)(e) * (H)->lv[1].lx * (H)->lv[1].lx * (H)->lv[1].lx)

static void dssum_m(const orc_hsmg* H, double* u)
{
    double* g = dalloc(H->nglob_m);
    for (long p = 0; p < H->nm; ++p) g[H->gid_m[p]] += u[p];
    for (long p = 0; p < H->nm; ++p) u[p] = g[H->gid_m[p]];
    free(g);
}

/* prolongation fine <- middle of a continuous middle vector (element by element) */
void orc_hsmg_prolong_fm(const orc_hsmg* H, const double* zm, double* zf)
{
    const int lxf = H->lv[0].lx, lxm = H->lv[1].lx;
    long nf3 = (long)lxf * lxf * lxf;
    for (int e = 0; e < H->E; ++e) tensor3(lxm, lxf, lxf, lxf, H->Jfm, H->Jfm, H->Jfm, zm + HSM(H, e), zf + e * nf3);
}

/* restriction middle <- fine of an assembled fine vector: dssum_m(J^T (r / mult)) */
void orc_hsmg_restrict_mf(const orc_hsmg* H, const double* rf, double* rm)
{
    const orc_mesh* m = H->m;
    const int lxf = H->lv[0].lx, lxm = H->lv[1].lx;
    long nf3 = (long)lxf * lxf * lxf;
    double* Jt = dalloc((long)lxm * lxf);
    for (int i = 0; i < lxf; ++i)
        for (int a = 0; a < lxm; ++a) Jt[a * lxf + i] = H->Jfm[i * lxm + a];
    double* t = dalloc(nf3);
    for (int e = 0; e < H->E; ++e) {
        for (long q = 0; q < nf3; ++q) t[q] = rf[e * nf3 + q] / m->mult[e * nf3 + q];
        tensor3(lxf, lxm, lxm, lxm, Jt, Jt, Jt, t, rm + HSM(H, e));
    }
    dssum_m(H, rm);
    free(Jt); free(t);
}

/* coarse corner node of element e, corner (a, b, c) in {0,1}^3 */
static long hs_corner(const orc_hsmg* H, int e, int a, int b, int c)
{
    const int nx = H->nel[0], ny = H->nel[1], nz = H->nel[2];
    int ex = e % nx, ey = (e / nx) % ny, ez = e / (nx * ny);
    return (ex + a) % nx + (long)nx * ((ey + b) % ny + (long)ny * ((ez + c) % nz));
}

/* restriction coarse <- middle: rc (unique corner nodes) = sum over elements of J^T (rm / mult_m) */
void orc_hsmg_restrict_cm(const orc_hsmg* H, const double* rm, double* rc)
{
    const int lxm = H->lv[1].lx;
    long nm3 = (long)lxm * lxm * lxm;
    double Jt[2 * ORC_MAXLX];
    for (int i = 0; i < lxm; ++i)
        for (int a = 0; a < 2; ++a) Jt[a * lxm + i] = H->Jmc[i * 2 + a];
    double* t = dalloc(nm3);
    double c8[8];
    for (long q = 0; q < H->nc; ++q) rc[q] = 0.0;
    for (int e = 0; e < H->E; ++e) {
        for (long q = 0; q < nm3; ++q) t[q] = rm[HSM(H, e) + q] / H->mult_m[HSM(H, e) + q];
        tensor3(lxm, 2, 2, 2, Jt, Jt, Jt, t, c8);
        for (int c = 0; c < 2; ++c)
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a) rc[hs_corner(H, e, a, b, c)] += c8[a + 2 * (b + 2 * c)];
    }
    free(t);
}

/* prolongation middle <- coarse: trilinear interpolation of the corner values */
void orc_hsmg_prolong_mc(const orc_hsmg* H, const double* ec, double* zm)
{
    for (int e = 0; e < H->E; ++e) {
        double c8[8];
        for (int c = 0; c < 2; ++c)
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a) c8[a + 2 * (b + 2 * c)] = ec[hs_corner(H, e, a, b, c)];
        tensor3(2, H->lv[1].lx, H->lv[1].lx, H->lv[1].lx, H->Jmc, H->Jmc, H->Jmc, c8, zm + HSM(H, e));
    }
}

/* Schwarz smoother of one level: W (dssum (local solves of the element copies of r)) */
static void hs_smooth(const orc_hsmg* H, int level, const double* r, double* z)
{
    const hs_level* L = &H->lv[level];
    long n3 = (long)L->lx * L->lx * L->lx;
    #pragma omp parallel for
    for (int e = 0; e < H->E; ++e) hs_local_solve(L, r + e * n3, z + e * n3);
    if (level == 0) {
        orc_dssum(H->m, z);
        for (long p = 0; p < H->m->np; ++p) z[p] /= H->m->mult[p];
    } else {
        dssum_m(H, z);
        for (long p = 0; p < H->nm; ++p) z[p] /= H->mult_m[p];
    }
}

void orc_hsmg_smooth(const orc_hsmg* H, int level, const double* r, double* z) { hs_smooth(H, level, r, z); }

/* z = M^{-1} r (r assembled, z continuous) */
void orc_hsmg_apply(const orc_hsmg* H, const double* r, double* z)
{
    const long np = H->m->np, nm = H->nm;
    double* rm = dalloc(nm); double* zm = dalloc(nm); double* em = dalloc(nm);
    double* rc = dalloc(H->nc); double* ec = dalloc(H->nc);
    double* zf = dalloc(np);
    orc_hsmg_restrict_mf(H, r, rm);
    orc_hsmg_restrict_cm(H, rm, rc);
    orc_hsmg_coarse_solve(H, rc, ec);
    hs_smooth(H, 1, rm, zm);
    orc_hsmg_prolong_mc(H, ec, em);
    for (long p = 0; p < nm; ++p) zm[p] += em[p];
    hs_smooth(H, 0, r, z);
    orc_hsmg_prolong_fm(H, zm, zf);
    for (long p = 0; p < np; ++p) z[p] += zf[p];
    free(rm); free(zm); free(em); free(rc); free(ec); free(zf);
}

long orc_hsmg_nm(const orc_hsmg* H) { return H->nm; }
long orc_hsmg_nc(const orc_hsmg* H) { return H->nc; }
int orc_hsmg_lxm(const orc_hsmg* H) { return H->lv[1].lx; }

/* Periodic Poisson solve A p = rhs (rhs assembled): unique-node mean of the
 * rhs removed, GMRES from zero, mass-weighted mean of p removed. */
int orc_poisson_pc(const orc_mesh* m, const orc_hsmg* H, const double* rhs, double* p, double tol, int maxit,
                   int mrst, double* res)
{
    long np = m->np;
    double* b = dalloc(np);
    memcpy(b, rhs, np * sizeof(double));
    orc_remove_mean_unique(m, b);
    for (long i = 0; i < np; ++i) p[i] = 0.0;
    int it = gmres_pc(m, 1.0, 0.0, b, p, tol, maxit, mrst, 1, H, res, NULL);
    orc_remove_mean_mass(m, p);
    free(b);
    return it;
}

int orc_poisson(const orc_mesh* m, const double* rhs, double* p, double tol, int maxit, int mrst, double* res)
{
    return orc_poisson_pc(m, NULL, rhs, p, tol, maxit, mrst, res);
}

/* ------------------------------------------------------------------ */
/* Projection of the pressure solve onto earlier solutions (the solver  */
/* settings of Sec. 3 give the pressure a projection space of dimension */
/* 20).  Written from the successive-right-hand-side method of Fischer  */
/* (1998): keep X = [x_1..x_l], orthonormal in the A inner product       */
/* (x_i^T A x_j = delta_ij, inner products over unique nodes).  For a new*/
/* rhs b the best approximation of A^-1 b in span X in the A-norm is     */
/* xbar = sum_i (x_i, b) x_i; the solver starts from xbar.  Afterwards   */
/* the correction v = x - xbar (or, when the space is full, the whole    */
/* solution x with the space emptied first) is A-orthogonalised against  */
/* X, normalised with ||v||_A^2 = (v, A v) - sum_i beta_i^2 (exact for an */
/* A-orthonormal X), and appended unless it is numerically dependent.    */
/* ------------------------------------------------------------------ */
typedef struct {
    const orc_mesh* m;
    int L, l;
    double* X;          /* L * np */
} orc_proj;

orc_proj* orc_proj_new(const orc_mesh* m, int L)
{
    if (L < 1 || L > 64) return NULL;
    orc_proj* P = (orc_proj*)calloc(1, sizeof(orc_proj));
    P->m = m; P->L = L; P->l = 0;
    P->X = dalloc((long)L * m->np);
    return P;
}

void orc_proj_free(orc_proj* P)
{
    if (!P) return;
    free(P->X); free(P);
}

int orc_proj_size(const orc_proj* P) { return P->l; }

int orc_proj_get(const orc_proj* P, int i, double* out)
{
    if (i < 0 || i >= P->l) return -1;
    memcpy(out, P->X + (long)i * P->m->np, P->m->np * sizeof(double));
    return 0;
}

/* xbar = sum_i (x_i, b) x_i */
void orc_proj_guess(const orc_proj* P, const double* b, double* xbar)
{
    long np = P->m->np;
    for (long q = 0; q < np; ++q) xbar[q] = 0.0;
    for (int i = 0; i < P->l; ++i) {
        const double* xi = P->X + (long)i * np;
        double a = orc_glsc(P->m, xi, b);
        for (long q = 0; q < np; ++q) xbar[q] += a * xi[q];
    }
}

/* add the new direction after a solve that started from xbar and ended at
 * x (the periodic Poisson operator, h1 = 1, h2 = 0).  Returns 1 if added. */
int orc_proj_update(orc_proj* P, const double* x, const double* xbar)
{
    const orc_mesh* m = P->m;
    long np = m->np;
    if (P->l == P->L) P->l = 0;                 /* full: restart from x */
    const int whole = P->l == 0;
    double* v = dalloc(np); double* w = dalloc(np);
    double beta[64];
    for (long q = 0; q < np; ++q) v[q] = whole ? x[q] : x[q] - xbar[q];
    apply_assembled(m, v, w, 1.0, 0.0);
    double n2 = orc_glsc(m, v, w);
    const double n2b = n2;
    for (int i = 0; i < P->l; ++i) beta[i] = orc_glsc(m, P->X + (long)i * np, w);
    for (int i = 0; i < P->l; ++i) {
        const double* xi = P->X + (long)i * np;
        for (long q = 0; q < np; ++q) v[q] -= beta[i] * xi[q];
        n2 -= beta[i] * beta[i];
    }
    int added = 0;
    if (n2b > 0.0 && n2 > 1e-12 * n2b) {
        double s = 1.0 / sqrt(n2);
        double* xl = P->X + (long)P->l * np;
        for (long q = 0; q < np; ++q) xl[q] = v[q] * s;
        P->l += 1;
        added = 1;
    }
    free(v); free(w);
    return added;
}

/* Periodic Poisson solve with projection: unique-node mean of the rhs
 * removed, GMRES from the projected guess, space updated, mass-weighted
 * mean of p removed. */
static int poisson_proj(const orc_mesh* m, orc_proj* P, const orc_hsmg* H, const double* rhs, double* p,
                        double tol, int maxit, int mrst, double* res)
{
    long np = m->np;
    double* b = dalloc(np); double* xbar = dalloc(np);
    memcpy(b, rhs, np * sizeof(double));
    orc_remove_mean_unique(m, b);
    orc_proj_guess(P, b, xbar);
    memcpy(p, xbar, np * sizeof(double));
    int it = gmres_pc(m, 1.0, 0.0, b, p, tol, maxit, mrst, 1, H, res, NULL);
    orc_proj_update(P, p, xbar);
    orc_remove_mean_mass(m, p);
    free(b); free(xbar);
    return it;
}

int orc_poisson_proj(const orc_mesh* m, orc_proj* P, const double* rhs, double* p, double tol, int maxit,
                     int mrst, double* res)
{
    return poisson_proj(m, P, NULL, rhs, p, tol, maxit, mrst, res);
}

/* ------------------------------------------------------------------ */
/* Fluid step: BDF-k / EXT-k (k ramps 1,2,3) velocity-first incremental */
/* pressure correction, in the order of the paper's Fig. 3 workflow.     */
/* ------------------------------------------------------------------ */
typedef struct {
    const orc_mesh* m;
    double nu, dt, vtol, ptol;
    int torder, vmaxit, pmaxit, mrst;
    double t;
    int step;
    double *u[3], *ul1[3], *ul2[3];     /* u^n, u^{n-1}, u^{n-2} */
    double *bn1[3], *bn2[3];            /* B N(u^{n-1}), B N(u^{n-2}) */
    double *p;
    /* last step statistics */
    int vit[3], pit;
    double vres[3], pres;
    orc_proj* proj;                     /* pressure projection space, or NULL */
    int dealias;                        /* convection on the 3/2 Gauss-Legendre grid */
    double cfl_target;                  /* > 0: adaptive dt (Sec. 3: target CFL 0.4); dt is then the maximum */
    double dth[3];                      /* steps dt_n, dt_{n-1}, dt_{n-2} of the latest steps */
    double last_cfl;                    /* CFL number of the last step */
    orc_hsmg* hsmg;                     /* pressure preconditioner: HSMG, or NULL for Jacobi */
} orc_fluid;

typedef struct {
    double t, ke, enst, maxdiv;
    int vit[3], pit;
    double vres[3], pres;
    double dt, cfl;                     /* step size and CFL number of the step */
} orc_step_stats;

/* init: 0 = 3D Taylor-Green, 1 = 2D Taylor-Green extruded in z, 2 = zero */
orc_fluid* orc_fluid_new(const orc_mesh* m, double nu, double dt, int torder,
                         double vtol, double ptol, int vmaxit, int pmaxit, int mrst, int init)
{
    if (torder < 1 || torder > 3) return NULL;
    orc_fluid* f = (orc_fluid*)calloc(1, sizeof(orc_fluid));
    long np = m->np;
    f->m = m; f->nu = nu; f->dt = dt; f->torder = torder;
    f->vtol = vtol; f->ptol = ptol; f->vmaxit = vmaxit; f->pmaxit = pmaxit; f->mrst = mrst;
    for (int c = 0; c < 3; ++c) {
        f->u[c] = dalloc(np); f->ul1[c] = dalloc(np); f->ul2[c] = dalloc(np);
        f->bn1[c] = dalloc(np); f->bn2[c] = dalloc(np);
    }
    f->p = dalloc(np);
    const double* X = m->xyz;
    const double* Y = m->xyz + np;
    const double* Z = m->xyz + 2 * np;
    for (long q = 0; q < np; ++q) {
        double x = X[q], y = Y[q], z = Z[q];
        if (init == 0) {
            f->u[0][q] = sin(x) * cos(y) * cos(z);
            f->u[1][q] = -cos(x) * sin(y) * cos(z);
            f->u[2][q] = 0.0;
            f->p[q] = (cos(2 * x) + cos(2 * y)) * (cos(2 * z) + 2.0) / 16.0;
        } else if (init == 1) {
            f->u[0][q] = sin(x) * cos(y);
            f->u[1][q] = -cos(x) * sin(y);
            f->u[2][q] = 0.0;
            f->p[q] = (cos(2 * x) + cos(2 * y)) / 4.0;
        }
    }
    /* history starts at the initial condition */
    for (int c = 0; c < 3; ++c) {
        memcpy(f->ul1[c], f->u[c], np * sizeof(double));
        memcpy(f->ul2[c], f->u[c], np * sizeof(double));
    }
    orc_conv(m, f->u[0], f->u[1], f->u[2], f->bn1[0], f->bn1[1], f->bn1[2]);
    for (int c = 0; c < 3; ++c) memcpy(f->bn2[c], f->bn1[c], np * sizeof(double));
    return f;
}

/* pressure projection space of dimension L (0 switches it off) */
int orc_fluid_set_proj(orc_fluid* f, int L)
{
    if (L < 0 || L > 64) return -1;
    orc_proj_free(f->proj);
    f->proj = L > 0 ? orc_proj_new(f->m, L) : NULL;
    return 0;
}

int orc_fluid_proj_size(const orc_fluid* f) { return f->proj ? f->proj->l : 0; }

/* pressure preconditioner: 1 = HSMG (needs an unperturbed box and N >= 4), 0 = Jacobi */
int orc_fluid_set_hsmg(orc_fluid* f, int on)
{
    orc_hsmg_free(f->hsmg);
    f->hsmg = NULL;
    if (!on) return 0;
    f->hsmg = orc_hsmg_new(f->m);
    return f->hsmg ? 0 : -1;
}

static void fluid_conv(const orc_fluid* f, const double* ux, const double* uy, const double* uz,
                       double* bx, double* by, double* bz)
{
    if (f->dealias) orc_conv_dealias(f->m, ux, uy, uz, bx, by, bz);
    else orc_conv(f->m, ux, uy, uz, bx, by, bz);
}

/* dealiased (1) or collocated (0) convection; the history of a fresh run
 * (lags = initial condition) is recomputed with the chosen form */
int orc_fluid_set_dealias(orc_fluid* f, int on)
{
    f->dealias = on ? 1 : 0;
    if (f->step == 0) {
        long np = f->m->np;
        fluid_conv(f, f->u[0], f->u[1], f->u[2], f->bn1[0], f->bn1[1], f->bn1[2]);
        for (int c = 0; c < 3; ++c) memcpy(f->bn2[c], f->bn1[c], np * sizeof(double));
    }
    return 0;
}

void orc_fluid_free(orc_fluid* f)
{
    if (!f) return;
    orc_proj_free(f->proj);
    orc_hsmg_free(f->hsmg);
    for (int c = 0; c < 3; ++c) { free(f->u[c]); free(f->ul1[c]); free(f->ul2[c]); free(f->bn1[c]); free(f->bn2[c]); }
    free(f->p); free(f);
}

/* field ids: 0..2 u, 3 p, 4..6 u lag1, 7..9 u lag2, 10..12 BN lag1, 13..15 BN lag2 */
static double* fluid_field(orc_fluid* f, int which)
{
    if (which >= 0 && which < 3) return f->u[which];
    if (which == 3) return f->p;
    if (which >= 4 && which < 7) return f->ul1[which - 4];
    if (which >= 7 && which < 10) return f->ul2[which - 7];
    if (which >= 10 && which < 13) return f->bn1[which - 10];
    if (which >= 13 && which < 16) return f->bn2[which - 13];
    return NULL;
}
int orc_fluid_get(orc_fluid* f, int which, double* out)
{
    double* s = fluid_field(f, which);
    if (!s) return -1;
    memcpy(out, s, f->m->np * sizeof(double));
    return 0;
}
int orc_fluid_set(orc_fluid* f, int which, const double* in)
{
    double* s = fluid_field(f, which);
    if (!s) return -1;
    memcpy(s, in, f->m->np * sizeof(double));
    return 0;
}
void orc_fluid_set_clock(orc_fluid* f, double t, int step) { f->t = t; f->step = step; }
double orc_fluid_time(const orc_fluid* f) { return f->t; }
int orc_fluid_stepno(const orc_fluid* f) { return f->step; }

/* BDF-k / EXT-k coefficients for the step sizes h[0] = t_{n+1} - t_n,
 * h[1] = t_n - t_{n-1}, h[2] = t_{n-1} - t_{n-2}.  With the time nodes
 * tau_0 = t_{n+1}, tau_j = t_{n+1-j}:
 *   du/dt(t_{n+1}) ~ (beta0 u^{n+1} - sum_j b_j u^{n+1-j}) / h[0],
 *   beta0 = h[0] l_0'(tau_0), b_j = -h[0] l_j'(tau_0)   (Lagrange basis over tau_0..tau_k)
 *   N(t_{n+1}) ~ sum_j a_j N^{n+1-j},  a_j = L_j(tau_0)  (Lagrange basis over tau_1..tau_k). */
void orc_bdf_ext_var(int k, const double h[3], double* beta0, double b[3], double a[3])
{
    double tau[4];
    tau[0] = 0.0;
    for (int j = 1; j <= 3; ++j) tau[j] = tau[j - 1] - h[j - 1];
    b[0] = b[1] = b[2] = a[0] = a[1] = a[2] = 0.0;
    /* derivative of the Lagrange basis over tau_0..tau_k at tau_0 */
    double d0 = 0.0;
    for (int m = 1; m <= k; ++m) d0 += 1.0 / (tau[0] - tau[m]);
    *beta0 = h[0] * d0;
    for (int j = 1; j <= k; ++j) {
        double num = 1.0, den = 1.0;
        for (int m = 0; m <= k; ++m) {
            if (m == j) continue;
            den *= tau[j] - tau[m];
            if (m != 0) num *= tau[0] - tau[m];
        }
        b[j - 1] = -h[0] * num / den;
    }
    /* extrapolation weights over tau_1..tau_k at tau_0 */
    for (int j = 1; j <= k; ++j) {
        double v = 1.0;
        for (int m = 1; m <= k; ++m)
            if (m != j) v *= (tau[0] - tau[m]) / (tau[j] - tau[m]);
        a[j - 1] = v;
    }
}

/* Advective CFL rate of a velocity field: the largest, over all local points,
 * of sum_a |u . grad r_a| / dr_a, with dr_a the spacing of the GLL nodes
 * around the point's index along direction a (half the distance between its
 * two neighbours inside, the distance to the one neighbour at an end).  The
 * CFL number of a step is dt times this rate. */
double orc_cfl_rate(const orc_mesh* m, const double* ux, const double* uy, const double* uz)
{
    const int lx = m->lx;
    const long np = m->np, n3 = (long)lx * lx * lx;
    double dr[ORC_MAXLX];
    for (int i = 0; i < lx; ++i) {
        if (i == 0) dr[i] = m->xi[1] - m->xi[0];
        else if (i == lx - 1) dr[i] = m->xi[lx - 1] - m->xi[lx - 2];
        else dr[i] = 0.5 * (m->xi[i + 1] - m->xi[i - 1]);
    }
    const double* U[3] = { ux, uy, uz };
    double best = 0.0;
    for (long p = 0; p < np; ++p) {
        const long q = p % n3;
        const int idx[3] = { (int)(q % lx), (int)((q / lx) % lx), (int)(q / ((long)lx * lx)) };
        double rate = 0.0;
        for (int a = 0; a < 3; ++a) {
            double v = 0.0;
            for (int c = 0; c < 3; ++c) v += U[c][p] * m->drdx[(long)(a * 3 + c) * np + p];
            rate += fabs(v) / dr[idx[a]];
        }
        if (rate > best) best = rate;
    }
    return best;
}

/* Adaptive time stepping toward a target CFL number (Sec. 3 runs with a
 * target of 0.4): dt_n = target / rate(u^n), at most the configured dt, and
 * after the first step within [0.5, 1.1] times the previous step. */
int orc_fluid_set_cfl(orc_fluid* f, double target)
{
    if (!(target >= 0.0)) return -1;
    f->cfl_target = target;
    return 0;
}

/* BDF-k and EXT-k coefficients for constant dt. */
static void bdf_ext(int k, double* beta0, double b[3], double a[3])
{
    b[0] = b[1] = b[2] = a[0] = a[1] = a[2] = 0.0;
    if (k == 1) { *beta0 = 1.0; b[0] = 1.0; a[0] = 1.0; }
    else if (k == 2) { *beta0 = 1.5; b[0] = 2.0; b[1] = -0.5; a[0] = 2.0; a[1] = -1.0; }
    else { *beta0 = 11.0 / 6.0; b[0] = 3.0; b[1] = -1.5; b[2] = 1.0 / 3.0; a[0] = 3.0; a[1] = -3.0; a[2] = 1.0; }
}

int orc_fluid_step(orc_fluid* f, orc_step_stats* st)
{
    const orc_mesh* m = f->m;
    long np = m->np;
    int k = f->step + 1 < f->torder ? f->step + 1 : f->torder;
    double beta0, b[3], a[3];
    double dt = f->dt, nu = f->nu;
    const double rate = orc_cfl_rate(m, f->u[0], f->u[1], f->u[2]);
    if (f->cfl_target > 0.0) {
        /* the step that meets the target CFL with the current velocity */
        double want = rate > 0.0 ? f->cfl_target / rate : f->dt;
        if (f->step > 0) {
            if (want > 1.1 * f->dth[0]) want = 1.1 * f->dth[0];
            if (want < 0.5 * f->dth[0]) want = 0.5 * f->dth[0];
        }
        dt = want < f->dt ? want : f->dt;
        f->dth[2] = f->dth[1]; f->dth[1] = f->dth[0]; f->dth[0] = dt;
        orc_bdf_ext_var(k, f->dth, &beta0, b, a);
    } else {
        bdf_ext(k, &beta0, b, a);
    }
    const double cfl = dt * rate;
    f->last_cfl = cfl;
    double h1 = nu, h2 = beta0 / dt;

    double *bn[3], *rhs[3], *gp[3], *us[3];
    for (int c = 0; c < 3; ++c) { bn[c] = dalloc(np); rhs[c] = dalloc(np); gp[c] = dalloc(np); us[c] = dalloc(np); }
    double* r = dalloc(np); double* du = dalloc(np); double* w = dalloc(np);
    double* rp = dalloc(np); double* phi = dalloc(np);

    /* (i) explicit RHS: extrapolated convection, BDF history, old pressure gradient */
    fluid_conv(f, f->u[0], f->u[1], f->u[2], bn[0], bn[1], bn[2]);
    orc_opgrad(m, f->p, gp[0], gp[1], gp[2]);
    for (int c = 0; c < 3; ++c) {
        const double* BN[3] = { bn[c], f->bn1[c], f->bn2[c] };
        const double* UL[3] = { f->u[c], f->ul1[c], f->ul2[c] };
        for (long q = 0; q < np; ++q) {
            double s = 0, hsum = 0;
            for (int j = 0; j < 3; ++j) { s += a[j] * BN[j][q]; hsum += b[j] * UL[j][q]; }
            rhs[c][q] = s + m->B[q] / dt * hsum - gp[c][q];
        }
        orc_dssum(m, rhs[c]);
    }
    /* (ii) velocity: H du = rhs - H u^n, u* = u^n + du */
    for (int c = 0; c < 3; ++c) {
        apply_assembled(m, f->u[c], w, h1, h2);
        for (long q = 0; q < np; ++q) { r[q] = rhs[c][q] - w[q]; du[q] = 0.0; }
        f->vit[c] = orc_pcg(m, h1, h2, r, du, f->vtol, f->vmaxit, &f->vres[c], NULL);
        for (long q = 0; q < np; ++q) us[c][q] = f->u[c][q] + du[q];
    }
    /* (iii) pressure increment: A phi = (beta0/dt) dssum(wdiv(u*)) */
    orc_wdiv(m, us[0], us[1], us[2], rp);
    orc_dssum(m, rp);
    for (long q = 0; q < np; ++q) rp[q] *= beta0 / dt;
    if (f->proj) f->pit = poisson_proj(m, f->proj, f->hsmg, rp, phi, f->ptol, f->pmaxit, f->mrst, &f->pres);
    else f->pit = orc_poisson_pc(m, f->hsmg, rp, phi, f->ptol, f->pmaxit, f->mrst, &f->pres);
    /* (iv) correction u^{n+1} = u* - (dt/beta0) dssum(B grad phi) / Bsum, p += phi */
    orc_opgrad(m, phi, gp[0], gp[1], gp[2]);
    for (int c = 0; c < 3; ++c) orc_dssum(m, gp[c]);
    for (int c = 0; c < 3; ++c) {
        double* t2 = f->ul2[c];          /* recycle the oldest lag as the new state */
        for (long q = 0; q < np; ++q) t2[q] = us[c][q] - dt / beta0 * gp[c][q] / m->Bsum[q];
        f->ul2[c] = f->ul1[c];
        f->ul1[c] = f->u[c];
        f->u[c] = t2;
        double* tb = f->bn2[c];
        f->bn2[c] = f->bn1[c];
        f->bn1[c] = tb;
        memcpy(f->bn1[c], bn[c], np * sizeof(double));
    }
    for (long q = 0; q < np; ++q) f->p[q] += phi[q];
    f->t += dt;
    f->step += 1;

    if (st) {
        st->t = f->t;
        st->dt = dt;
        st->cfl = cfl;
        orc_diagnostics(m, f->u[0], f->u[1], f->u[2], &st->ke, &st->enst, &st->maxdiv);
        for (int c = 0; c < 3; ++c) { st->vit[c] = f->vit[c]; st->vres[c] = f->vres[c]; }
        st->pit = f->pit; st->pres = f->pres;
    }
    for (int c = 0; c < 3; ++c) { free(bn[c]); free(rhs[c]); free(gp[c]); free(us[c]); }
    free(r); free(du); free(w); free(rp); free(phi);
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
