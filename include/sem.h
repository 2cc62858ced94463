/*
 * sem.h -- C ABI of libsem, the MI355X (gfx950) hot path of a matrix-free
 * spectral-element (SEM) incompressible Navier-Stokes step on the
 * Taylor-Green vortex with per-component precision control.
 *
 * Method: "Mixed-Precision SEM-Based CFD Simulations on GPUs: A Taylor-Green
 * Vortex case".  The step follows the workflow of the paper's Fig. 3
 * (explicit RHS, velocity CG+Jacobi solve, intermediate velocity u*,
 * pressure residual, pressure GMRES solve, projection/correction), with the
 * third-order time integration and solver settings of Sec. 3, the Taylor-
 * Green initial condition of Sec. 3 (eqs. for u, v, w and Re = v0 L / nu),
 * and the three-level precision model of Sec. 2 / Fig. 4: a global cap rp,
 * block-level (SEM, velocity, pressure) compute/accumulate/storage
 * precisions, and kernel-level overrides of hotspot kernels (Table 2).
 *
 * Conventions
 *  - Every field is element-major, E*lx^3 values, u[e][k][j][i] with i
 *    fastest, e = ex + nx*(ey + ny*ez), lx = order + 1.  Assembled fields
 *    hold equal values in every local copy of a shared node.
 *  - Device pointers are plain device addresses on the device current when
 *    sem_bind was called.  The caller owns all device memory (the workspace
 *    passed to sem_bind and every field buffer) and the stream.
 *  - Calls that take device pointers are stream-ordered and asynchronous on
 *    the bound stream unless stated otherwise.
 *  - Return values: 0 (SEM_OK) or a negative sem_status.  No C++ exception
 *    crosses this interface.  sem_strerror gives a message.
 *  - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef SEM_H
#define SEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SEM_ABI_VERSION 1

typedef enum {
    SEM_OK = 0,
    SEM_EINVAL = -1,     /* invalid argument or unsupported precision combination */
    SEM_ENOMEM = -2,     /* workspace passed to sem_bind is too small */
    SEM_EHIP = -3,       /* a HIP runtime call failed (see sem_strerror / sem_last_error) */
    SEM_ENAN = -4,       /* a non-finite value appeared in a solve */
    SEM_ENOTCONV = -5,   /* a Krylov solve hit its iteration limit */
    SEM_ESTATE = -6      /* call not valid in the context's current state (e.g. not bound) */
} sem_status;

/* Floating-point formats.  SEM_INHERIT in a kernel override means "use the
 * block default".  Ordering for the cap: FP64 > FP32 > FP16 = BF16. */
typedef enum { SEM_FP64 = 0, SEM_FP32 = 1, SEM_FP16 = 2, SEM_BF16 = 3, SEM_INHERIT = -1 } sem_prec;

/* Compute, accumulate and storage precision of a block or kernel (Fig. 4). */
typedef struct { int compute, accumulate, storage; } sem_role;

enum { SEM_BLOCK_SEM = 0, SEM_BLOCK_VEL = 1, SEM_BLOCK_PRES = 2, SEM_NBLOCK = 3 };

/* Hotspot kernels that may override their block (Table 2 rows B-5..B-7 and
 * the SEM operators of the step). */
enum {
    SEM_K_AX_VEL = 0,    /* velocity Helmholtz operator (block VEL) */
    SEM_K_AX_PRES = 1,   /* pressure Poisson operator (block PRES) */
    SEM_K_OPGRAD = 2,    /* mass-weighted gradient (block SEM) */
    SEM_K_CONV = 3,      /* convective term (block SEM) */
    SEM_K_DIV = 4,       /* weak divergence (block SEM; sem_wdiv).  Inside sem_fluid_step the
                            weak divergence of u* is the pressure solve's initial residual and
                            is always formed in fp64 (SEM_X_RESID). */
    SEM_K_COUNT = 5
};

/* Quantities that stay in FP64 even when rp = FP32 (Sec. 2: reductions may
 * use a higher precision capped at fp64; Sec. 4 design: accumulation kept in
 * fp64).  This implementation requires all four whenever rp = FP32. */
enum {
    SEM_X_STATE = 1u << 0,   /* BDF/EXT velocity state, history and pressure */
    SEM_X_GMRES = 1u << 1,   /* GMRES basis, Hessenberg, orthogonalisation dots */
    SEM_X_RESID = 1u << 2,   /* true-residual checks */
    SEM_X_REDUCE = 1u << 3,  /* global stage of every reduction */
    SEM_X_ALL = 0xF
};

typedef struct {
    int size;                        /* sizeof(sem_precision) */
    int rp;                          /* global cap: SEM_FP64 or SEM_FP32 */
    sem_role block[SEM_NBLOCK];
    sem_role kernel[SEM_K_COUNT];    /* SEM_INHERIT fields take the block value.  Compute
                                        SEM_FP16/SEM_BF16 (Table 2's fp16-compute overrides)
                                        is accepted for AX_VEL and AX_PRES only, with storage
                                        of the same format and accumulate SEM_FP32 (see
                                        SEM_AX_16BIT_COMPUTE at sem_ax); SEM_EINVAL otherwise. */
    unsigned fp64_exceptions;        /* SEM_X_* bits */
} sem_precision;

/* Periodic box [lo,hi] of nel[0]*nel[1]*nel[2] hexahedra of polynomial
 * order `order` (2..11), optionally perturbed by the smooth map
 *   x_c += amp*h_c*prod_q sin(pi (x_q - lo_q)/h_q + phase[3c+q])
 * (conforming; periodic because every nel must then be even). */
typedef struct {
    int size;                        /* sizeof(sem_mesh_desc) */
    int nel[3];
    int order;
    double lo[3], hi[3];
    double deform_amp;
    double deform_phase[9];
} sem_mesh_desc;

enum { SEM_INIT_ZERO = 0, SEM_INIT_TGV3D = 1, SEM_INIT_TGV2D = 2 };
enum { SEM_MODE_OPERATOR = 0, SEM_MODE_POISSON = 1, SEM_MODE_FLUID = 2 };

typedef struct {
    int size;                        /* sizeof(sem_flow_desc) */
    int mode;                        /* SEM_MODE_*: which workspaces sem_bind carves */
    double nu, dt;                   /* viscosity (1/Re for v0 = L = 1), time step */
    int torder;                      /* BDF/EXT order 1..3 (ramped 1,2,3 at start) */
    double vel_tol, pres_tol;        /* absolute tolerances on the unique-node l2 norm */
    int vel_maxit, pres_maxit;       /* Krylov iteration limits per solve */
    int gmres_restart;               /* 1..30 */
    int vel_max_refine;              /* FP64 true-residual refinement cycles (>= 1) */
    int init;                        /* SEM_INIT_* */
    int proj_dim;                    /* pressure projection space 0..SEM_MAX_PROJ (0 = off; fluid mode):
                                        GMRES starts from the A-norm best approximation of the new
                                        pressure increment in the span of earlier ones (Sec. 3 uses 20) */
    int dealias;                     /* 1: the convective term is integrated on ceil(3 lx / 2) Gauss-Legendre
                                        points per direction (the 3/2 rule; Sec. 3 runs with dealiasing)
                                        instead of by collocation on the GLL points; fluid mode only.
                                        Adds 9 E ceil(3 lx/2)^3 fp64 metric terms, plus a copy in the conv
                                        storage precision when that is fp32 or 16-bit (element-scaled). */
    double cfl_target;               /* > 0: adaptive time stepping toward this CFL number (Sec. 3 uses
                                        0.4; fluid mode): each step takes dt_n = cfl_target / rate(u^n),
                                        at most dt, and after the first step within [0.5, 1.1] dt_{n-1};
                                        rate(u) = max over local points of sum_a |u . grad r_a| / dr_a
                                        (dr: local GLL spacing); BDF/EXT use the variable-step
                                        coefficients.  0: fixed dt. */
    int hsmg;                        /* pressure GMRES preconditioner (Poisson and fluid modes):
                                        0 = Jacobi (the assembled diagonal);
                                        1 = three-level hybrid Schwarz multigrid (Sec. 3 names HSMG
                                        for the pressure): levels of order N, N/2 and 1; additive
                                        Schwarz on element subdomains (fast diagonalisation of the
                                        separable element stiffness extended by one segment to a
                                        zero Dirichlet node) on the two upper levels, Lagrange
                                        interpolation between levels and its unique-node transpose,
                                        an exact order-1 coarse solve off the constant mode, the
                                        levels added (a linear preconditioner).  fp64 arithmetic in
                                        every tier.  Needs an unperturbed mesh, order 4..11, 2..64
                                        elements per direction and an fp64 or fp32 pressure
                                        basis.  GMRES keeps Z_j = M^{-1} V_j of each Arnoldi step
                                        (flexible-GMRES storage), so a cycle end adds sum_j y_j Z_j
                                        instead of applying M once more.  Adds E lx^3 doubles,
                                        (restart + 2) E lx^3 values in the pressure basis precision
                                        and 3 E (N/2 + 1)^3 doubles. */
} sem_flow_desc;

#define SEM_MAX_PROJ 20

typedef struct sem_ctx sem_ctx;

/* Per-step statistics of one context (filled after the stream is synced by
 * sem_fluid_step, which synchronises before returning). */
typedef struct {
    double t, ke, enst, maxdiv;      /* after the step */
    int vel_iters[3], pres_iters;
    double vel_res[3], pres_res;     /* final residual norms */
    int status;                      /* SEM_OK, SEM_ENAN or SEM_ENOTCONV */
    int vel_cycles;                  /* velocity solve cycles (fp64 residual checks after the first) */
    double dt, cfl;                  /* step size and CFL number (dt * rate(u^n)) of the step */
} sem_step_stats;

typedef struct {
    int iters;
    double res;
    int status;
} sem_solve_stats;

typedef struct {
    double t, ke, enst, maxdiv;
    int step;
} sem_diag;

/* Validates the descriptors and builds the host tables (GLL nodes and
 * weights, derivative matrix, shared-node lists).  Host only: no device
 * allocation and no HIP call.  Errors: SEM_EINVAL (invalid mesh, order,
 * flow parameters, 2^31 or more local points, 2^29 or more local points along
 * one line of elements in x, a precision above rp outside the SEM_X
 * exceptions, or a combination the library has no kernel for). */
int sem_setup(const sem_mesh_desc* mesh, const sem_flow_desc* flow, const sem_precision* prec, sem_ctx** out);

/* Exact device bytes sem_bind needs for this context (geometry in every
 * precision its policy uses, plus the workspaces of its mode). */
size_t sem_workspace_bytes(const sem_ctx* ctx);

/* Binds a caller-owned device buffer (>= sem_workspace_bytes, 256-byte
 * aligned) and stream (a hipStream_t, 0 = null stream) to the context, then
 * computes the geometric factors, Jacobi diagonals and, in fluid mode, the
 * initial condition on that stream.  Errors: SEM_ENOMEM, SEM_EHIP,
 * SEM_ESTATE (already bound). */
int sem_bind(sem_ctx* ctx, void* dev_buf, size_t bytes, void* hip_stream);

/* Moves a bound context to another stream (a hipStream_t, 0 = null stream):
 * its later calls, and batches whose first context it is, run there.  Work
 * already queued on the old stream is not waited for: the caller orders the
 * two streams (for instance by synchronising the old one first).  Lets a
 * server bind requests on a stream of their own and then hand them to the
 * stream that runs their batches.  Host only.  Errors: SEM_EINVAL (null
 * context), SEM_ESTATE (not bound). */
int sem_set_stream(sem_ctx* ctx, void* hip_stream);

/* Helmholtz operator w = h1 * sum_ab D_a^T G_ab D_b u + h2 * B u on every
 * element (the paper's ax_helm), u and w device arrays of E*lx^3 values in
 * buf_prec (FP64, FP32, FP16 or BF16 storage), geometry in geom_prec (must
 * be one the context holds; SEM_INHERIT = the AX_PRES policy when h2 == 0,
 * else AX_VEL).  Arithmetic is fp64 for fp64 vectors (fp32 with
 * SEM_AX_FP32_COMPUTE) and fp32 otherwise; SEM_AX_16BIT_COMPUTE selects the
 * 16-bit arithmetic of Table 2's fp16-compute overrides (B-6, B-7) in the
 * geometry's format: per element, u scaled by the power of two s that puts
 * max|u| in [0.5, 1), D, and the metric-weighted derivatives are rounded to
 * 16 bits (nearest even), products summed in fp32, h1 gsc / s and the mass
 * term applied in fp32 (needs 16-bit geometry and fp32 or same-format
 * vectors).  flags & SEM_ASSEMBLE additionally applies dssum to w. */
#define SEM_ASSEMBLE 1
#define SEM_AX_FP32_COMPUTE 2   /* fp64 vectors, fp32 arithmetic (needs fp32 or 16-bit geometry) */
#define SEM_AX_16BIT_COMPUTE 4  /* 16-bit operands, fp32 sums (needs 16-bit geometry) */
int sem_ax(sem_ctx* ctx, const void* u, void* w, double h1, double h2, int buf_prec, int geom_prec, int flags);

/* Direct stiffness summation in place: every local copy of a shared node
 * receives the sum of all copies (Q Q^T; the paper's gather/scatter). */
int sem_dssum(sem_ctx* ctx, void* u, int buf_prec);

/* Advances each of n fluid-mode contexts by nsteps time steps in one batch
 * (same order and precision policy required, n <= 48).  stats has
 * n*nsteps entries (ctx-major).  Synchronises the stream of ctxs[0], which
 * all contexts of the batch must share.  A request whose solve fails is
 * reported in its stats and keeps no influence on the others. */
int sem_fluid_step(sem_ctx* const* ctxs, int n, int nsteps, sem_step_stats* stats);

/* The same steps with each step replayed as a HIP graph (the step of Fig. 3
 * captured once per batch and iteration budget, then launched with one call
 * and one synchronisation).  The budgets (PCG iterations per refinement cycle,
 * refinement cycles, Arnoldi steps) are the largest counts of the batch's
 * previous step (pressure: of its last four steps); every solver kernel is
 * gated on the device as in sem_fluid_step, so a request whose solves stop
 * within the budgets gets bitwise the results of sem_fluid_step.  A request
 * still iterating at the end of a budget has its correction, lag rotation and
 * diagnostics gated off on the device and its step run again by
 * sem_fluid_step's host-driven path, so results never depend on the budgets.
 * A request's first step, and batches with adaptive dt (whose step history
 * changes at the step's start), always take the host-driven path.  Graphs are
 * cached per batch (up to 32) and dropped by sem_destroy of any member. */
int sem_fluid_step_graph(sem_ctx* const* ctxs, int n, int nsteps, sem_step_stats* stats);

/* Process-wide counts since load: graph replays, requests whose replayed step
 * ran again on the host-driven path, graph captures (all nullable). */
int sem_graph_counters(int64_t* replays, int64_t* reruns, int64_t* captures);

/* The library's host lock (recursive; acquire = 1 locks, 0 unlocks, on the
 * calling thread).  A step capture in one thread fails if another thread makes
 * a device-synchronising HIP call meanwhile (allocating or freeing device or
 * pinned memory, a copy on the legacy stream).  sem_fluid_step_graph captures
 * under this lock, and sem_bind, sem_destroy and the library's own pinned
 * allocations take it; a caller that makes such calls itself from another
 * thread while graph steps run takes it around them. */
int sem_host_lock(int acquire);

/* Periodic Poisson solves A p = rhs for n POISSON- or FLUID-mode contexts of
 * the same order and policy: rhs[i] (device, fp64, assembled) has its
 * unique-node mean removed, GMRES runs from zero, and sol[i] (device, fp64)
 * receives p with its mass-weighted mean removed. */
int sem_poisson_solve(sem_ctx* const* ctxs, int n, const void* const* rhs, void* const* sol, sem_solve_stats* stats);

/* The same solve in steps, for serving loops that change the batch between
 * iteration chunks (continuous batching): sem_poisson_begin starts the solves
 * of n contexts (copies and mean-centres rhs[i], zero initial guess);
 * sem_poisson_advance runs up to max_iters Arnoldi steps on any batch of
 * begun contexts (same order/policy/stream; finished ones idle) and sets
 * active[i] (nullable) to whether context i still iterates (synchronises);
 * sem_poisson_finish removes the mass-weighted mean, copies the solution to
 * sol (device fp64, nullable) and fills st (nullable). */
int sem_poisson_begin(sem_ctx* const* ctxs, int n, const void* const* rhs);
int sem_poisson_advance(sem_ctx* const* ctxs, int n, int max_iters, int* active);
int sem_poisson_finish(sem_ctx* ctx, void* sol, sem_solve_stats* st);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as sem_poisson_solve for one context, bound in any mode, with the
 * Jacobi preconditioner (flow.hsmg must be 0).  The GMRES workspace (the
 * m + 1 basis vectors in the context's basis storage precision and four fp64
 * vectors of E*lx^3 values, each rounded up to 256 bytes) is taken from a
 * static device array of sem_noalloc_max_bytes() bytes that the library
 * holds on every device it runs on until the process ends; nothing is
 * allocated and no memset is recorded.  rhs and sol: device fp64 arrays of
 * E*lx^3 values (rhs assembled; sol receives p with its mass-weighted mean
 * removed).  Synchronises the context's stream.  Every call on a device
 * shares that device's array: calls that overlap on one device (on any
 * stream, from any thread) race and must be serialised by the caller; the
 * context's own projection space is not touched.  Errors: SEM_ENOMEM when
 * the workspace exceeds the array (no kernel runs), SEM_EINVAL, SEM_ESTATE,
 * SEM_EHIP; solver status in stats as for sem_poisson_solve. */
size_t sem_noalloc_max_bytes(void);
int sem_poisson_solve_noalloc(sem_ctx* ctx, const void* rhs, void* sol, sem_solve_stats* stats);

/* Field access for checkpoints and tests.  which: SEM_F_*; component fields
 * use which + c.  src/dst are fp64 arrays of E*lx^3 values, on the host when
 * is_host != 0 (the call then synchronises), else device pointers. */
enum {
    SEM_F_U = 0,          /* +0..2 velocity u^n */
    SEM_F_P = 3,
    SEM_F_ULAG1 = 4,      /* +0..2 */
    SEM_F_ULAG2 = 7,      /* +0..2 */
    SEM_F_BNLAG1 = 10,    /* +0..2  B N(u^{n-1}) */
    SEM_F_BNLAG2 = 13,    /* +0..2 */
    SEM_F_MASS = 16,      /* read-only geometry */
    SEM_F_BSUM = 17,
    SEM_F_G = 18,         /* +0..5 */
    SEM_F_M = 24,         /* +0..8  M_ac, index a*3+c */
    SEM_F_DIAG_A = 33,    /* assembled stiffness diagonal */
    SEM_F_COUNT = 34
};
int sem_get_field(sem_ctx* ctx, int which, void* dst, int is_host);
int sem_set_field(sem_ctx* ctx, int which, const void* src, int is_host);
/* Mass matrix: out = B o f (element-local), plus dssum when flags &
 * SEM_ASSEMBLE (out then is the assembled load vector of f).  Device fp64
 * arrays of E*lx^3 values; asynchronous. */
int sem_mass(sem_ctx* ctx, const double* f, double* out, int flags);

/* Node fields for synthetic inputs: what = 0, 1, 2 writes the x, y or z
 * coordinate of every local node; what = 3 writes amp sin x sin y sin z (the
 * manufactured Poisson solution family).  out: device fp64, E*lx^3. */
int sem_node_field(sem_ctx* ctx, int what, double amp, double* out);

/* time and step counter (for checkpoint/restart) */
int sem_set_clock(sem_ctx* ctx, double t, int step);

/* Step-level precision (the time/step level of Fig. 4): copy the fluid state
 * of src (velocity and its two lags, the two convection lags, pressure, time
 * and step count) into dst, a bound fluid context on the same device with
 * the same mesh, dt and BDF/EXT order and any precision tier; dst then
 * continues the run in its tier.  Exact (the state is fp64 in every tier);
 * dst's projection space starts empty.  Synchronises both streams.  Returns
 * SEM_EINVAL when the contexts do not match, SEM_ESTATE when one is not bound. */
int sem_copy_state(sem_ctx* dst, sem_ctx* src);

/* Kinetic energy, enstrophy and max |div u| of the current velocity
 * (computes them; synchronises). */
int sem_diagnostics(sem_ctx* ctx, sem_diag* out);

/* Element-local SEM operators on caller arrays (fp64, E*lx^3 each, not
 * assembled): conv -> 3 outputs, opgrad(p) -> 3 outputs, wdiv(3 inputs) ->
 * 1 output; the SEM-block precision policy of the context applies.  conv is
 * -B (u . grad) u (Sec. 2), dealiased when the context's flow has dealias set;
 * it needs a fluid-mode context. */
int sem_conv(sem_ctx* ctx, const double* const* u3, double* const* out3);
int sem_opgrad(sem_ctx* ctx, const double* p, double* const* out3);
int sem_wdiv(sem_ctx* ctx, const double* const* v3, double* out);

/* Optional HIP-event timing of one kernel class on the stream it is launched
 * on (for roofline measurements).  sem_prof_start arms recording of every
 * launch of that class made by any context on this process; sem_prof_stop
 * synchronises the recorded events and returns the summed kernel time and
 * the number of launches (inactive, gated launches included).  Not
 * thread-safe; recording adds one event pair per launch. */
enum {
    SEM_PROF_AX_VEL = 1,      /* velocity Helmholtz operator inside PCG */
    SEM_PROF_AX_PRES = 2,     /* pressure operator inside the Arnoldi step */
    SEM_PROF_GM_DOTS = 3,     /* GMRES first Gram-Schmidt pass */
    SEM_PROF_GM_UPD_DOTS = 4, /* GMRES update + second-pass dots */
    SEM_PROF_GM_UPD_NORM = 5, /* GMRES second update + norm */
    SEM_PROF_DSSUM_PRES = 6,  /* dssum of the Arnoldi operator output */
    SEM_PROF_AX_ANY = 7,      /* every standalone sem_ax call */
    SEM_PROF_AX_RESID = 8,    /* fp64 velocity residual operator, RHS_L - H_L u (3 components) */
    SEM_PROF_AX_PRESID = 9,   /* fp64 Poisson operator of the GMRES cycle-end residuals and the
                                 projection update */
    SEM_PROF_CONV = 10,       /* convective term of the fluid step (collocated or dealiased) */
    SEM_PROF_HSMG = 11        /* HSMG preconditioner applications of the Arnoldi steps */
};
int sem_prof_start(int kclass);
int sem_prof_stop(double* total_ms, int64_t* launches);

/* Sizes of a bound or unbound context. */
int sem_sizes(const sem_ctx* ctx, int64_t* np, int64_t* nglob, int* lx, int* nelem);

/* Frees the context's host state: its tables, its pinned status words and the step
 * graphs cached for any batch it belongs to.  NULL is a no-op.  It neither waits for
 * nor frees device memory: the workspace belongs to the caller, and kernels of this
 * context still queued on its stream may use it, so synchronise that stream before
 * the workspace is reused or freed.  Takes the library's host lock. */
void sem_destroy(sem_ctx* ctx);
/* Static text naming a status code (SEM_OK, SEM_E*); never NULL, unknown codes
 * included.  The caller does not free it. */
const char* sem_strerror(int status);
/* Text of the last error recorded by any call on this thread. */
const char* sem_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SEM_H */
