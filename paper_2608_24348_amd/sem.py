"""Python binding of libsem (argument marshalling only).

Every step of the hot path runs in the HIP kernels of ``libsem.so``; this
module builds the C descriptor structs, hands torch-owned device memory and
the current torch stream to the library, and converts status codes into
exceptions.  It never falls back to any other implementation: a missing or
unloadable library raises.
"""
import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libsem.so")

FP64, FP32, FP16, BF16, INHERIT = 0, 1, 2, 3, -1
BLOCK_SEM, BLOCK_VEL, BLOCK_PRES = 0, 1, 2
K_AX_VEL, K_AX_PRES, K_OPGRAD, K_CONV, K_DIV, K_COUNT = 0, 1, 2, 3, 4, 5
X_ALL = 0xF
INIT_ZERO, INIT_TGV3D, INIT_TGV2D = 0, 1, 2
MODE_OPERATOR, MODE_POISSON, MODE_FLUID = 0, 1, 2
ASSEMBLE = 1
AX_FP32_COMPUTE = 2
AX_16BIT_COMPUTE = 4
F_U, F_P, F_ULAG1, F_ULAG2, F_BNLAG1, F_BNLAG2 = 0, 3, 4, 7, 10, 13
F_MASS, F_BSUM, F_G, F_M, F_DIAG_A = 16, 17, 18, 24, 33

STATUS = {0: "SEM_OK", -1: "SEM_EINVAL", -2: "SEM_ENOMEM", -3: "SEM_EHIP", -4: "SEM_ENAN",
          -5: "SEM_ENOTCONV", -6: "SEM_ESTATE"}


class SemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code


class Role(C.Structure):
    _fields_ = [("compute", C.c_int), ("accumulate", C.c_int), ("storage", C.c_int)]


class Precision(C.Structure):
    _fields_ = [("size", C.c_int), ("rp", C.c_int), ("block", Role * 3), ("kernel", Role * K_COUNT),
                ("fp64_exceptions", C.c_uint)]


class MeshDesc(C.Structure):
    _fields_ = [("size", C.c_int), ("nel", C.c_int * 3), ("order", C.c_int), ("lo", C.c_double * 3),
                ("hi", C.c_double * 3), ("deform_amp", C.c_double), ("deform_phase", C.c_double * 9)]


class FlowDesc(C.Structure):
    _fields_ = [("size", C.c_int), ("mode", C.c_int), ("nu", C.c_double), ("dt", C.c_double),
                ("torder", C.c_int), ("vel_tol", C.c_double), ("pres_tol", C.c_double),
                ("vel_maxit", C.c_int), ("pres_maxit", C.c_int), ("gmres_restart", C.c_int),
                ("vel_max_refine", C.c_int), ("init", C.c_int), ("proj_dim", C.c_int),
                ("dealias", C.c_int), ("cfl_target", C.c_double), ("hsmg", C.c_int)]


class StepStats(C.Structure):
    _fields_ = [("t", C.c_double), ("ke", C.c_double), ("enst", C.c_double), ("maxdiv", C.c_double),
                ("vel_iters", C.c_int * 3), ("pres_iters", C.c_int), ("vel_res", C.c_double * 3),
                ("pres_res", C.c_double), ("status", C.c_int), ("vel_cycles", C.c_int), ("dt", C.c_double),
                ("cfl", C.c_double)]


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("res", C.c_double), ("status", C.c_int)]


class Diag(C.Structure):
    _fields_ = [("t", C.c_double), ("ke", C.c_double), ("enst", C.c_double), ("maxdiv", C.c_double),
                ("step", C.c_int)]


EXPORTS = ["sem_setup", "sem_workspace_bytes", "sem_bind", "sem_ax", "sem_dssum", "sem_fluid_step",
           "sem_poisson_solve", "sem_get_field", "sem_set_field", "sem_set_clock", "sem_diagnostics",
           "sem_conv", "sem_opgrad", "sem_wdiv", "sem_sizes", "sem_destroy", "sem_strerror", "sem_last_error",
           "sem_prof_start", "sem_prof_stop", "sem_poisson_begin", "sem_poisson_advance", "sem_poisson_finish",
           "sem_mass", "sem_node_field", "sem_copy_state", "sem_fluid_step_graph", "sem_graph_counters", "sem_host_lock",
           "sem_noalloc_max_bytes", "sem_poisson_solve_noalloc", "sem_set_stream"]
PROF_AX_VEL, PROF_AX_PRES, PROF_GM_DOTS, PROF_GM_UPD_DOTS, PROF_GM_UPD_NORM, PROF_DSSUM_PRES, PROF_AX_ANY, PROF_AX_RESID, \
    PROF_AX_PRESID, PROF_CONV, PROF_HSMG = range(1, 12)

_lib = None


def load():
    """Load libsem.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise RuntimeError("libsem.so is not built (run __graft_entry__.build() or paper_2608_24348_amd/build.py)")
    # torch provides device memory and streams: its HIP runtime must be the
    # process's only one, so it is loaded before libsem (whose HIP dependency
    # then resolves to the same library instead of a second runtime)
    import torch  # noqa: F401
    L = C.CDLL(LIBPATH)
    vp = C.c_void_p
    L.sem_setup.argtypes = [C.POINTER(MeshDesc), C.POINTER(FlowDesc), C.POINTER(Precision), C.POINTER(vp)]
    L.sem_workspace_bytes.restype = C.c_size_t
    L.sem_workspace_bytes.argtypes = [vp]
    L.sem_bind.argtypes = [vp, vp, C.c_size_t, vp]
    L.sem_set_stream.argtypes = [vp, vp]
    L.sem_ax.argtypes = [vp, vp, vp, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int]
    L.sem_dssum.argtypes = [vp, vp, C.c_int]
    L.sem_fluid_step.argtypes = [C.POINTER(vp), C.c_int, C.c_int, C.POINTER(StepStats)]
    L.sem_fluid_step_graph.argtypes = [C.POINTER(vp), C.c_int, C.c_int, C.POINTER(StepStats)]
    L.sem_graph_counters.argtypes = [C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.sem_host_lock.argtypes = [C.c_int]
    L.sem_poisson_solve.argtypes = [C.POINTER(vp), C.c_int, C.POINTER(vp), C.POINTER(vp), C.POINTER(SolveStats)]
    L.sem_get_field.argtypes = [vp, C.c_int, vp, C.c_int]
    L.sem_set_field.argtypes = [vp, C.c_int, vp, C.c_int]
    L.sem_set_clock.argtypes = [vp, C.c_double, C.c_int]
    L.sem_diagnostics.argtypes = [vp, C.POINTER(Diag)]
    L.sem_conv.argtypes = [vp, C.POINTER(vp), C.POINTER(vp)]
    L.sem_opgrad.argtypes = [vp, vp, C.POINTER(vp)]
    L.sem_wdiv.argtypes = [vp, C.POINTER(vp), vp]
    L.sem_sizes.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.sem_destroy.argtypes = [vp]
    L.sem_strerror.restype = C.c_char_p
    L.sem_strerror.argtypes = [C.c_int]
    L.sem_last_error.restype = C.c_char_p
    L.sem_poisson_begin.argtypes = [C.POINTER(vp), C.c_int, C.POINTER(vp)]
    L.sem_poisson_advance.argtypes = [C.POINTER(vp), C.c_int, C.c_int, C.POINTER(C.c_int)]
    L.sem_poisson_finish.argtypes = [vp, vp, C.POINTER(SolveStats)]
    L.sem_mass.argtypes = [vp, vp, vp, C.c_int]
    L.sem_node_field.argtypes = [vp, C.c_int, C.c_double, vp]
    L.sem_copy_state.argtypes = [vp, vp]
    L.sem_prof_start.argtypes = [C.c_int]
    L.sem_prof_stop.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    L.sem_noalloc_max_bytes.restype = C.c_size_t
    L.sem_noalloc_max_bytes.argtypes = []
    L.sem_poisson_solve_noalloc.argtypes = [vp, vp, vp, C.POINTER(SolveStats)]
    _lib = L
    return L


def _check(rc):
    if rc != 0:
        raise SemError(rc, load().sem_last_error().decode())


# ---------------------------------------------------------------- precision policies
def precision(rp=FP64, blocks=None, kernels=None, exceptions=None):
    """Build a sem_precision: blocks maps block id -> (compute, accumulate,
    storage); kernels maps kernel id -> (compute, accumulate, storage) with
    INHERIT allowed."""
    p = Precision()
    p.size = C.sizeof(Precision)
    p.rp = rp
    for b in range(3):
        v = (blocks or {}).get(b, (rp, rp, rp))
        p.block[b] = Role(*v)
    for k in range(K_COUNT):
        v = (kernels or {}).get(k, (INHERIT, INHERIT, INHERIT))
        p.kernel[k] = Role(*v)
    p.fp64_exceptions = (X_ALL if rp == FP32 else 0) if exceptions is None else exceptions
    return p


TIERS = ("fp64", "fp32b", "fp32b-p32", "fp32b+fp16", "fp32b+bf16", "fp32b+fp16p", "fp32b+fp16a", "fp32b+bf16a",
         "fp32b+fp16all", "fp32b+bf16all")


def tier(name):
    """Named precision presets (the paper's Table 2 configurations on this path).

    fp64          global fp64 (A-0)
    fp32b         rp = fp32 storage; SEM operators and velocity solver fp32;
                  pressure operator fp64 arithmetic on fp32-stored geometry and
                  Jacobi diagonal (B-4 "pressure-only fp64 compute"); BDF/EXT
                  state, GMRES basis/orthogonalisation, residual checks and the
                  global reduction stage fp64
    fp32b-p32     fp32b with fp32 arithmetic in the pressure operator too (B-0
                  with fp64 accumulation); with Jacobi preconditioning its GMRES
                  cannot meet an absolute 1e-8 on large meshes
    fp32b+fp16    fp32b with fp16-stored geometry for the velocity Helmholtz
                  operator and opgrad (B-6 style)
    fp32b+bf16    same with bf16
    fp32b+fp16p   fp32b with fp16-stored geometry for the pressure operator (B-7)
    fp32b+fp16a   fp32b with fp16-stored metric terms for the convective term,
                  collocated or dealiased (B-5, adv_dealias); fp32b+bf16a with bf16
    fp32b+fp16all / fp32b+bf16all  16-bit geometry for both operators and
                  opgrad (operator microbenchmarks)
    fp32b+fp16c   B-6 as Table 2 states it: the velocity Helmholtz operator in
                  16-bit arithmetic (16-bit operands, fp32 sums) on fp16
                  geometry; fp32b+bf16c with bf16
    fp32b+fp16pc  B-7 likewise: the pressure operator in 16-bit arithmetic
    """
    if name == "fp64":
        return precision(FP64)
    h = {"fp32b": None, "fp32b-p32": None, "fp32b+fp16": FP16, "fp32b+bf16": BF16, "fp32b+fp16p": FP16,
         "fp32b+fp16a": FP16, "fp32b+bf16a": BF16, "fp32b+fp16all": FP16, "fp32b+bf16all": BF16,
         "fp32b+fp16c": FP16, "fp32b+bf16c": BF16, "fp32b+fp16pc": FP16}
    if name not in h:
        raise ValueError("unknown tier %r" % name)
    blocks = {BLOCK_SEM: (FP32, FP32, FP32), BLOCK_VEL: (FP32, FP32, FP32), BLOCK_PRES: (FP64, FP64, FP32)}
    if name == "fp32b-p32":
        blocks[BLOCK_PRES] = (FP32, FP32, FP32)
    ks = {}
    if name in ("fp32b+fp16", "fp32b+bf16", "fp32b+fp16all", "fp32b+bf16all"):
        ks[K_AX_VEL] = (FP32, FP32, h[name])
        ks[K_OPGRAD] = (FP32, FP32, h[name])
    if name in ("fp32b+fp16p", "fp32b+fp16all", "fp32b+bf16all"):
        ks[K_AX_PRES] = (FP64, FP64, h[name])
    if name in ("fp32b+fp16a", "fp32b+bf16a"):
        ks[K_CONV] = (FP32, FP32, h[name])
    if name in ("fp32b+fp16c", "fp32b+bf16c"):
        ks[K_AX_VEL] = (h[name], FP32, h[name])
    if name == "fp32b+fp16pc":
        ks[K_AX_PRES] = (h[name], FP32, h[name])
    return precision(FP32, blocks=blocks, kernels=ks)


def mesh_desc(nel, order, lo=(-math.pi,) * 3, hi=(math.pi,) * 3, amp=0.0, phase=None):
    m = MeshDesc()
    m.size = C.sizeof(MeshDesc)
    for d in range(3):
        m.nel[d] = int(nel[d])
        m.lo[d] = float(lo[d])
        m.hi[d] = float(hi[d])
    m.order = int(order)
    m.deform_amp = float(amp)
    ph = np.zeros(9) if phase is None else np.asarray(phase, dtype=np.float64)
    for q in range(9):
        m.deform_phase[q] = float(ph[q])
    return m


def flow_desc(mode=MODE_FLUID, nu=1.0 / 1600, dt=1e-3, torder=3, vel_tol=1e-8, pres_tol=1e-8, vel_maxit=500,
              pres_maxit=1000, restart=30, max_refine=8, init=INIT_TGV3D, proj=0, dealias=0, cfl=0.0, hsmg=0):
    f = FlowDesc()
    f.size = C.sizeof(FlowDesc)
    f.mode = mode
    f.nu = nu
    f.dt = dt
    f.torder = torder
    f.vel_tol = vel_tol
    f.pres_tol = pres_tol
    f.vel_maxit = vel_maxit
    f.pres_maxit = pres_maxit
    f.gmres_restart = restart
    f.vel_max_refine = max_refine
    f.init = init
    f.proj_dim = proj
    f.dealias = int(dealias)
    f.cfl_target = float(cfl)
    f.hsmg = int(hsmg)
    return f


_TORCH_DT = None


def _torch():
    import torch
    return torch


def dtype_of(prec):
    torch = _torch()
    return {FP64: torch.float64, FP32: torch.float32, FP16: torch.float16, BF16: torch.bfloat16}[prec]


def prec_of(t):
    torch = _torch()
    return {torch.float64: FP64, torch.float32: FP32, torch.float16: FP16, torch.bfloat16: BF16}[t.dtype]


class Context:
    """One request: mesh + flow + precision policy, bound to a torch-owned
    device workspace and the current torch stream of ``device``."""

    def __init__(self, mesh, flow, prec, device="cuda:0", bind=True):
        L = load()
        self.L = L
        self.mesh = mesh
        self.flow = flow
        self.prec = prec
        h = C.c_void_p()
        _check(L.sem_setup(C.byref(mesh), C.byref(flow), C.byref(prec), C.byref(h)))
        self.h = h
        np_, ng = C.c_int64(), C.c_int64()
        lx, ne = C.c_int(), C.c_int()
        _check(L.sem_sizes(h, C.byref(np_), C.byref(ng), C.byref(lx), C.byref(ne)))
        self.np, self.nglob, self.lx, self.E = np_.value, ng.value, lx.value, ne.value
        self.bytes = L.sem_workspace_bytes(h)
        self.ws = None
        self.device = device
        if bind:
            self.bind(device)

    def bind(self, device="cuda:0", stream=None, workspace=None):
        """workspace: a uint8 device tensor of at least ``bytes`` bytes, 256-byte
        aligned (for instance a slice of a server's arena); else one is allocated."""
        torch = _torch()
        if workspace is None:
            self.ws = torch.empty(self.bytes + 256, dtype=torch.uint8, device=device)
            base = self.ws.data_ptr()
            aligned = (base + 255) // 256 * 256
        else:
            if workspace.dtype != torch.uint8:
                raise ValueError("workspace must be a uint8 tensor, got %s" % workspace.dtype)
            if workspace.numel() < self.bytes:
                raise ValueError("workspace holds %d bytes, the context needs %d" % (workspace.numel(), self.bytes))
            if workspace.data_ptr() % 256:
                raise ValueError("workspace must start on a 256-byte boundary")
            if not workspace.is_cuda or not workspace.is_contiguous():
                raise ValueError("workspace must be a contiguous device tensor")
            self.ws = workspace
            aligned = workspace.data_ptr()
        s = stream if stream is not None else torch.cuda.current_stream(device)
        self.stream = s
        _check(self.L.sem_bind(self.h, C.c_void_p(aligned), C.c_size_t(self.bytes), C.c_void_p(s.cuda_stream)))

    def set_stream(self, stream):
        """later calls (and batches led by this context) run on ``stream``; the
        caller orders it after the old stream's work"""
        _check(self.L.sem_set_stream(self.h, C.c_void_p(stream.cuda_stream)))
        self.stream = stream

    def close(self):
        if getattr(self, "h", None):
            self.L.sem_destroy(self.h)
            self.h = None
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- operators on torch device tensors
    def ax(self, u, w, h1=1.0, h2=0.0, geom=INHERIT, assemble=False, fp32_compute=False, half_compute=False):
        assert u.is_cuda and w.is_cuda and u.numel() == self.np and w.numel() == self.np and u.dtype == w.dtype
        assert u.is_contiguous() and w.is_contiguous()
        flags = ((ASSEMBLE if assemble else 0) | (AX_FP32_COMPUTE if fp32_compute else 0) |
                 (AX_16BIT_COMPUTE if half_compute else 0))
        _check(self.L.sem_ax(self.h, C.c_void_p(u.data_ptr()), C.c_void_p(w.data_ptr()), float(h1), float(h2),
                             prec_of(u), int(geom), flags))
        return w

    def dssum(self, u):
        assert u.is_cuda and u.numel() == self.np and u.is_contiguous()
        _check(self.L.sem_dssum(self.h, C.c_void_p(u.data_ptr()), prec_of(u)))
        return u

    def get(self, which):
        out = np.zeros(self.np)
        _check(self.L.sem_get_field(self.h, int(which), out.ctypes.data_as(C.c_void_p), 1))
        return out

    def set(self, which, arr):
        a = np.ascontiguousarray(arr, dtype=np.float64)
        assert a.size == self.np
        _check(self.L.sem_set_field(self.h, int(which), a.ctypes.data_as(C.c_void_p), 1))

    def set_clock(self, t, step):
        _check(self.L.sem_set_clock(self.h, float(t), int(step)))

    def velocity(self):
        return np.stack([self.get(F_U + c) for c in range(3)])

    def pressure(self):
        return self.get(F_P)

    def diagnostics(self):
        d = Diag()
        _check(self.L.sem_diagnostics(self.h, C.byref(d)))
        return {"t": d.t, "ke": d.ke, "enst": d.enst, "maxdiv": d.maxdiv, "step": d.step}

    def mass(self, f, out=None, assemble=True):
        """out = B o f (assembled when assemble); fp64 device tensors."""
        torch = _torch()
        out = torch.empty_like(f) if out is None else out
        _check(self.L.sem_mass(self.h, C.c_void_p(f.data_ptr()), C.c_void_p(out.data_ptr()), ASSEMBLE if assemble else 0))
        return out

    def node_field(self, what, amp=1.0):
        """Device fp64 tensor of node coordinates (what 0..2) or amp sin x sin y sin z (what 3)."""
        torch = _torch()
        out = torch.empty(self.np, dtype=torch.float64, device=self.device)
        _check(self.L.sem_node_field(self.h, int(what), float(amp), C.c_void_p(out.data_ptr())))
        return out

    def conv(self, u3):
        torch = _torch()
        outs = [torch.empty_like(u3[0]) for _ in range(3)]
        ins = (C.c_void_p * 3)(*[C.c_void_p(t.data_ptr()) for t in u3])
        os_ = (C.c_void_p * 3)(*[C.c_void_p(t.data_ptr()) for t in outs])
        _check(self.L.sem_conv(self.h, ins, os_))
        return outs

    def opgrad(self, p):
        torch = _torch()
        outs = [torch.empty_like(p) for _ in range(3)]
        os_ = (C.c_void_p * 3)(*[C.c_void_p(t.data_ptr()) for t in outs])
        _check(self.L.sem_opgrad(self.h, C.c_void_p(p.data_ptr()), os_))
        return outs

    def wdiv(self, v3):
        torch = _torch()
        out = torch.empty_like(v3[0])
        ins = (C.c_void_p * 3)(*[C.c_void_p(t.data_ptr()) for t in v3])
        _check(self.L.sem_wdiv(self.h, ins, C.c_void_p(out.data_ptr())))
        return out


def _stats_dict(s):
    return {"t": s.t, "ke": s.ke, "enst": s.enst, "maxdiv": s.maxdiv, "vit": list(s.vel_iters),
            "pit": s.pres_iters, "vres": list(s.vel_res), "pres": s.pres_res, "status": s.status,
            "vcyc": s.vel_cycles, "dt": s.dt, "cfl": s.cfl}


def fluid_step(ctxs, nsteps=1, graph=False):
    """Advance a batch of fluid contexts by nsteps (graph: each step replayed as
    a HIP graph, sem_fluid_step_graph); returns per-context lists of step stats."""
    if isinstance(ctxs, Context):
        ctxs = [ctxs]
    n = len(ctxs)
    arr = (C.c_void_p * n)(*[c.h for c in ctxs])
    st = (StepStats * (n * max(nsteps, 1)))()
    fn = load().sem_fluid_step_graph if graph else load().sem_fluid_step
    _check(fn(arr, n, int(nsteps), st))
    return [[_stats_dict(st[i * nsteps + k]) for k in range(nsteps)] for i in range(n)]


class host_lock:
    """Context manager holding the library's host lock (sem_host_lock): wrap
    device allocations, frees and legacy-stream work made from one thread while
    another may be running graph steps."""

    def __enter__(self):
        _check(load().sem_host_lock(1))
        return self

    def __exit__(self, *exc):
        load().sem_host_lock(0)
        return False


def graph_counters():
    """(graph replays, requests re-run on the host-driven path, captures) since load."""
    a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
    _check(load().sem_graph_counters(C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def prof_start(kclass):
    """Arm HIP-event timing of one kernel class (see sem.h SEM_PROF_*)."""
    _check(load().sem_prof_start(int(kclass)))


def prof_stop():
    """Return (total kernel milliseconds, number of launches) since prof_start."""
    ms, n = C.c_double(), C.c_int64()
    _check(load().sem_prof_stop(C.byref(ms), C.byref(n)))
    return ms.value, n.value


def poisson_begin(ctxs, rhs):
    """Start batched Poisson solves (rhs: fp64 device tensors, assembled)."""
    n = len(ctxs)
    arr = (C.c_void_p * n)(*[c.h for c in ctxs])
    r = (C.c_void_p * n)(*[C.c_void_p(t.data_ptr()) for t in rhs])
    _check(load().sem_poisson_begin(arr, n, r))


def poisson_advance(ctxs, max_iters):
    """Run up to max_iters Arnoldi steps on a batch of begun solves; returns the still-active flags."""
    n = len(ctxs)
    arr = (C.c_void_p * n)(*[c.h for c in ctxs])
    act = (C.c_int * n)()
    _check(load().sem_poisson_advance(arr, n, int(max_iters), act))
    return [bool(a) for a in act]


def poisson_finish(ctx, sol=None):
    """Finish one solve: mean removal, copy to sol (fp64 device tensor or None); returns its stats."""
    st = SolveStats()
    _check(load().sem_poisson_finish(ctx.h, C.c_void_p(sol.data_ptr()) if sol is not None else None, C.byref(st)))
    return {"iters": st.iters, "res": st.res, "status": st.status}


def poisson_solve(ctxs, rhs, sol):
    """Batched periodic Poisson solves; rhs/sol are lists of fp64 device tensors."""
    n = len(ctxs)
    arr = (C.c_void_p * n)(*[c.h for c in ctxs])
    r = (C.c_void_p * n)(*[C.c_void_p(t.data_ptr()) for t in rhs])
    s = (C.c_void_p * n)(*[C.c_void_p(t.data_ptr()) for t in sol])
    st = (SolveStats * n)()
    _check(load().sem_poisson_solve(arr, n, r, s, st))
    return [{"iters": st[i].iters, "res": st[i].res, "status": st[i].status} for i in range(n)]


def poisson_solve_noalloc(ctx, rhs, sol):
    """Poisson solve of one context (any mode, Jacobi preconditioner) whose
    Krylov workspace is the library's static device array (no allocation);
    rhs/sol are fp64 device tensors.  Returns the solve stats."""
    st = SolveStats()
    _check(load().sem_poisson_solve_noalloc(ctx.h, C.c_void_p(rhs.data_ptr()), C.c_void_p(sol.data_ptr()),
                                            C.byref(st)))
    return {"iters": st.iters, "res": st.res, "status": st.status}


def noalloc_max_bytes():
    """Size of the static device array of the allocation-free entry points."""
    return load().sem_noalloc_max_bytes()


def copy_state(dst, src):
    """Carry the fluid state of context src into dst (same mesh and dt, any tier)."""
    _check(load().sem_copy_state(dst.h, src.h))


def run_schedule(mesh, flow, schedule, device="cuda:0"):
    """Run a step-level precision schedule, e.g. [("fp64", 100), ("fp32b", 100)]:
    each phase runs its steps in a context of its tier, starting from the
    state the previous phase ended with.  Returns the per-step statistics."""
    stats = []
    prev = None
    for name, nsteps in schedule:
        ctx = Context(mesh, flow, tier(name), device=device)
        if prev is not None:
            copy_state(ctx, prev)
            prev.close()
        stats += fluid_step([ctx], nsteps)[0]
        prev = ctx
    return stats, prev
