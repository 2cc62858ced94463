"""ctypes wrapper of the FP64 CPU oracle (sem_oracle.c).

TEST INFRASTRUCTURE ONLY -- see the package docstring.  Builds
``liboracle.so`` with gcc/OpenMP on demand (``build_oracle``).
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sem_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


class _StepStats(C.Structure):
    _fields_ = [("t", C.c_double), ("ke", C.c_double), ("enst", C.c_double), ("maxdiv", C.c_double),
                ("vit", C.c_int * 3), ("pit", C.c_int), ("vres", C.c_double * 3), ("pres", C.c_double),
                ("dt", C.c_double), ("cfl", C.c_double)]


def build_oracle(force=False):
    """Compile liboracle.so (gcc -O2 -fopenmp).  Always recompiles when force."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build_oracle()
    L = C.CDLL(_LIB)
    vp = C.c_void_p
    L.orc_gll.argtypes = [C.c_int, _dp, _dp]
    L.orc_deriv.argtypes = [C.c_int, _dp, _dp]
    L.orc_mesh_new.restype = vp
    L.orc_mesh_new.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _dp, _dp, C.c_double, _dp]
    L.orc_mesh_subset_new.restype = vp
    L.orc_mesh_subset_new.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _dp, _dp, C.c_double, _dp,
                                      C.POINTER(C.c_int), C.c_int]
    L.orc_mesh_free.argtypes = [vp]
    for f in ("orc_mesh_np", "orc_mesh_nglob"):
        getattr(L, f).restype = C.c_long
        getattr(L, f).argtypes = [vp]
    for f in ("orc_mesh_lx", "orc_mesh_E"):
        getattr(L, f).restype = C.c_int
        getattr(L, f).argtypes = [vp]
    L.orc_mesh_vol.restype = C.c_double
    L.orc_mesh_vol.argtypes = [vp]
    L.orc_mesh_get.argtypes = [vp, C.c_int, _dp]
    L.orc_mesh_tables.argtypes = [vp, _dp, _dp, _dp]
    L.orc_from_lattice.argtypes = [vp, _dp, _dp]
    L.orc_dssum.argtypes = [vp, _dp]
    L.orc_glsc.restype = C.c_double
    L.orc_glsc.argtypes = [vp, _dp, _dp]
    L.orc_sum.restype = C.c_double
    L.orc_sum.argtypes = [vp, _dp]
    L.orc_ax.argtypes = [vp, _dp, _dp, C.c_double, C.c_double]
    L.orc_diag.argtypes = [vp, C.c_double, C.c_double, _dp]
    L.orc_grad.argtypes = [vp, _dp, _dp, _dp, _dp]
    L.orc_opgrad.argtypes = [vp, _dp, _dp, _dp, _dp]
    L.orc_wdiv.argtypes = [vp, _dp, _dp, _dp, _dp]
    L.orc_conv.argtypes = [vp, _dp, _dp, _dp, _dp, _dp, _dp]
    L.orc_conv_dealias.argtypes = [vp, _dp, _dp, _dp, _dp, _dp, _dp]
    L.orc_gl.restype = C.c_int
    L.orc_gl.argtypes = [C.c_int, _dp, _dp]
    L.orc_lxd.restype = C.c_int
    L.orc_lxd.argtypes = [C.c_int]
    L.orc_interp.argtypes = [C.c_int, _dp, C.c_int, _dp, _dp]
    L.orc_fluid_set_dealias.restype = C.c_int
    L.orc_fluid_set_dealias.argtypes = [vp, C.c_int]
    L.orc_fluid_set_cfl.restype = C.c_int
    L.orc_fluid_set_cfl.argtypes = [vp, C.c_double]
    L.orc_bdf_ext_var.argtypes = [C.c_int, _dp, C.POINTER(C.c_double), _dp, _dp]
    L.orc_cfl_rate.restype = C.c_double
    L.orc_cfl_rate.argtypes = [vp, _dp, _dp, _dp]
    L.orc_curl_div.argtypes = [vp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    L.orc_diagnostics.argtypes = [vp, _dp, _dp, _dp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                  C.POINTER(C.c_double)]
    L.orc_pcg.restype = C.c_int
    L.orc_pcg.argtypes = [vp, C.c_double, C.c_double, _dp, _dp, C.c_double, C.c_int,
                          C.POINTER(C.c_double), vp]
    L.orc_gmres.restype = C.c_int
    L.orc_gmres.argtypes = [vp, C.c_double, C.c_double, _dp, _dp, C.c_double, C.c_int, C.c_int,
                            C.POINTER(C.c_double), vp]
    L.orc_gmres_ex.restype = C.c_int
    L.orc_gmres_ex.argtypes = [vp, C.c_double, C.c_double, _dp, _dp, C.c_double, C.c_int, C.c_int, C.c_int,
                               C.POINTER(C.c_double), vp]
    L.orc_remove_mean_unique.argtypes = [vp, _dp]
    L.orc_remove_mean_mass.argtypes = [vp, _dp]
    L.orc_poisson.restype = C.c_int
    L.orc_poisson.argtypes = [vp, _dp, _dp, C.c_double, C.c_int, C.c_int, C.POINTER(C.c_double)]
    L.orc_fluid_new.restype = vp
    L.orc_fluid_new.argtypes = [vp, C.c_double, C.c_double, C.c_int, C.c_double, C.c_double,
                                C.c_int, C.c_int, C.c_int, C.c_int]
    L.orc_fluid_free.argtypes = [vp]
    L.orc_fluid_get.argtypes = [vp, C.c_int, _dp]
    L.orc_fluid_set.argtypes = [vp, C.c_int, _dp]
    L.orc_fluid_set_clock.argtypes = [vp, C.c_double, C.c_int]
    L.orc_fluid_time.restype = C.c_double
    L.orc_fluid_time.argtypes = [vp]
    L.orc_fluid_stepno.restype = C.c_int
    L.orc_fluid_stepno.argtypes = [vp]
    L.orc_fluid_step.argtypes = [vp, C.POINTER(_StepStats)]
    L.orc_fluid_set_proj.restype = C.c_int
    L.orc_fluid_set_proj.argtypes = [vp, C.c_int]
    L.orc_fluid_proj_size.restype = C.c_int
    L.orc_fluid_proj_size.argtypes = [vp]
    L.orc_proj_new.restype = vp
    L.orc_proj_new.argtypes = [vp, C.c_int]
    L.orc_proj_free.argtypes = [vp]
    L.orc_proj_size.restype = C.c_int
    L.orc_proj_size.argtypes = [vp]
    L.orc_proj_guess.argtypes = [vp, _dp, _dp]
    L.orc_proj_get.restype = C.c_int
    L.orc_proj_get.argtypes = [vp, C.c_int, _dp]
    L.orc_proj_update.restype = C.c_int
    L.orc_proj_update.argtypes = [vp, _dp, _dp]
    L.orc_poisson_proj.restype = C.c_int
    L.orc_poisson_proj.argtypes = [vp, vp, _dp, _dp, C.c_double, C.c_int, C.c_int, C.POINTER(C.c_double)]
    L.orc_num_threads.restype = C.c_int
    L.orc_hsmg_new.restype = vp
    L.orc_hsmg_new.argtypes = [vp]
    L.orc_hsmg_free.argtypes = [vp]
    L.orc_hsmg_level.restype = C.c_int
    L.orc_hsmg_level.argtypes = [vp, C.c_int, C.c_int, _dp, _dp, _dp, _dp]
    for f in ("orc_hsmg_local_solve", "orc_hsmg_smooth"):
        getattr(L, f).argtypes = [vp, C.c_int, _dp, _dp]
    for f in ("orc_hsmg_coarse_solve", "orc_hsmg_prolong_fm", "orc_hsmg_restrict_mf", "orc_hsmg_restrict_cm",
              "orc_hsmg_prolong_mc", "orc_hsmg_apply"):
        getattr(L, f).argtypes = [vp, _dp, _dp]
    for f in ("orc_hsmg_nm", "orc_hsmg_nc"):
        getattr(L, f).restype = C.c_long
        getattr(L, f).argtypes = [vp]
    L.orc_hsmg_lxm.restype = C.c_int
    L.orc_hsmg_lxm.argtypes = [vp]
    L.orc_poisson_pc.restype = C.c_int
    L.orc_poisson_pc.argtypes = [vp, vp, _dp, _dp, C.c_double, C.c_int, C.c_int, C.POINTER(C.c_double)]
    L.orc_fluid_set_hsmg.restype = C.c_int
    L.orc_fluid_set_hsmg.argtypes = [vp, C.c_int]
    _lib = L
    return L


def num_threads():
    return _load().orc_num_threads()


def gl(n):
    """Gauss-Legendre nodes and weights (n points)."""
    L = _load()
    z = np.zeros(n)
    w = np.zeros(n)
    if L.orc_gl(n, z, w) != 0:
        raise ValueError("unsupported point count %d" % n)
    return z, w


def bdf_ext_var(k, h):
    """BDF-k / EXT-k coefficients for step sizes h = (t_{n+1}-t_n, t_n-t_{n-1},
    t_{n-1}-t_{n-2}): (beta0, b[3], a[3])."""
    hh = np.ascontiguousarray(np.array(list(h) + [0.0] * (3 - len(h)), dtype=np.float64))
    b0 = C.c_double(0.0)
    b = np.zeros(3)
    a = np.zeros(3)
    _load().orc_bdf_ext_var(int(k), hh, C.byref(b0), b, a)
    return b0.value, b, a


def lxd(lx):
    """Points per direction of the 3/2-rule dealiasing grid."""
    return _load().orc_lxd(int(lx))


def interp_matrix(xi, z):
    """Lagrange basis of the nodes xi evaluated at the points z: I[q, l]."""
    I = np.zeros(len(z) * len(xi))
    _load().orc_interp(len(xi), _c(xi), len(z), _c(z), I)
    return I.reshape(len(z), len(xi))


def gll(N):
    """GLL nodes and weights of order N."""
    L = _load()
    xi = np.zeros(N + 1)
    w = np.zeros(N + 1)
    if L.orc_gll(N, xi, w) != 0:
        raise ValueError("unsupported order %d" % N)
    return xi, w


def deriv_matrix(N):
    """GLL derivative matrix D[i, j] = l_j'(xi_i)."""
    L = _load()
    xi, _ = gll(N)
    D = np.zeros((N + 1) * (N + 1))
    L.orc_deriv(N, xi, D)
    return D.reshape(N + 1, N + 1)


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleMesh:
    """Periodic box mesh of nel[0]*nel[1]*nel[2] hexahedra of order N with
    its geometric factors; fields are flat arrays of E*lx^3 local values."""

    def __init__(self, nel, N, lo=(-np.pi,) * 3, hi=(np.pi,) * 3, amp=0.0, phase=None, elements=None):
        """elements: optional list of element indices of the full box; the mesh
        then holds only those elements (element-local operators only, no
        assembly), for element-by-element checks of large meshes."""
        self.L = _load()
        ph = np.zeros(9) if phase is None else _c(phase)
        if elements is None:
            self.h = self.L.orc_mesh_new(int(nel[0]), int(nel[1]), int(nel[2]), int(N),
                                         _c(lo), _c(hi), float(amp), ph)
        else:
            el = np.ascontiguousarray(elements, dtype=np.int32)
            self.h = self.L.orc_mesh_subset_new(int(nel[0]), int(nel[1]), int(nel[2]), int(N), _c(lo), _c(hi),
                                                float(amp), ph, el.ctypes.data_as(C.POINTER(C.c_int)), len(el))
        if not self.h:
            raise ValueError("invalid mesh (element count, order or non-positive Jacobian)")
        self.nel = tuple(int(v) for v in nel)
        self.N = int(N)
        self.lx = self.N + 1
        self.E = self.L.orc_mesh_E(self.h)
        self.np = self.L.orc_mesh_np(self.h)
        self.nglob = self.L.orc_mesh_nglob(self.h)
        self.vol = self.L.orc_mesh_vol(self.h)

    def __del__(self):
        if getattr(self, "h", None):
            self.L.orc_mesh_free(self.h)
            self.h = None

    def _get(self, which, n):
        out = np.zeros(n * self.np)
        self.L.orc_mesh_get(self.h, which, out)
        return out.reshape(n, self.np) if n > 1 else out

    def coords(self):
        return self._get(0, 3)

    def jac(self):
        return self._get(1, 1)

    def mass(self):
        return self._get(2, 1)

    def drdx(self):
        return self._get(3, 9)

    def G(self):
        return self._get(4, 6)

    def M(self):
        return self._get(5, 9)

    def bsum(self):
        return self._get(6, 1)

    def mult(self):
        return self._get(7, 1)

    def gid(self):
        return self._get(8, 1).astype(np.int64)

    def tables(self):
        xi = np.zeros(self.lx)
        w = np.zeros(self.lx)
        D = np.zeros(self.lx * self.lx)
        self.L.orc_mesh_tables(self.h, xi, w, D)
        return xi, w, D.reshape(self.lx, self.lx)

    def from_lattice(self, lat):
        out = np.zeros(self.np)
        self.L.orc_from_lattice(self.h, _c(lat).ravel(), out)
        return out

    def dssum(self, u):
        u = _c(u).copy()
        self.L.orc_dssum(self.h, u)
        return u

    def glsc(self, a, b):
        return self.L.orc_glsc(self.h, _c(a), _c(b))

    def sum(self, a):
        return self.L.orc_sum(self.h, _c(a))

    def ax(self, u, h1=1.0, h2=0.0):
        w = np.zeros(self.np)
        self.L.orc_ax(self.h, _c(u), w, float(h1), float(h2))
        return w

    def diag(self, h1=1.0, h2=0.0):
        d = np.zeros(self.np)
        self.L.orc_diag(self.h, float(h1), float(h2), d)
        return d

    def grad(self, u):
        g = [np.zeros(self.np) for _ in range(3)]
        self.L.orc_grad(self.h, _c(u), *g)
        return np.stack(g)

    def opgrad(self, p):
        g = [np.zeros(self.np) for _ in range(3)]
        self.L.orc_opgrad(self.h, _c(p), *g)
        return np.stack(g)

    def wdiv(self, v):
        out = np.zeros(self.np)
        self.L.orc_wdiv(self.h, _c(v[0]), _c(v[1]), _c(v[2]), out)
        return out

    def conv(self, u):
        o = [np.zeros(self.np) for _ in range(3)]
        self.L.orc_conv(self.h, _c(u[0]), _c(u[1]), _c(u[2]), *o)
        return np.stack(o)

    def cfl_rate(self, u):
        """Advective CFL rate max_points sum_a |u . grad r_a| / dr_a (CFL = dt * rate)."""
        return self.L.orc_cfl_rate(self.h, _c(u[0]), _c(u[1]), _c(u[2]))

    def conv_dealias(self, u):
        """-B (u . grad) u integrated on the 3/2-rule Gauss-Legendre grid."""
        o = [np.zeros(self.np) for _ in range(3)]
        self.L.orc_conv_dealias(self.h, _c(u[0]), _c(u[1]), _c(u[2]), *o)
        return np.stack(o)

    def curl_div(self, u):
        o = [np.zeros(self.np) for _ in range(4)]
        self.L.orc_curl_div(self.h, _c(u[0]), _c(u[1]), _c(u[2]), *o)
        return np.stack(o[:3]), o[3]

    def diagnostics(self, u):
        ke, en, md = C.c_double(), C.c_double(), C.c_double()
        self.L.orc_diagnostics(self.h, _c(u[0]), _c(u[1]), _c(u[2]), C.byref(ke), C.byref(en), C.byref(md))
        return ke.value, en.value, md.value

    def pcg(self, b, h1=1.0, h2=0.0, x0=None, tol=1e-8, maxit=500, history=False):
        x = np.zeros(self.np) if x0 is None else _c(x0).copy()
        res = C.c_double()
        hist = np.zeros(maxit + 2) if history else None
        it = self.L.orc_pcg(self.h, float(h1), float(h2), _c(b), x, float(tol), int(maxit), C.byref(res),
                            hist.ctypes.data if history else None)
        if history:
            return x, it, res.value, hist[:it + 1].copy()
        return x, it, res.value

    def gmres(self, b, h1=1.0, h2=0.0, x0=None, tol=1e-8, maxit=1000, restart=30, history=False, deflate=False):
        x = np.zeros(self.np) if x0 is None else _c(x0).copy()
        res = C.c_double()
        hist = np.zeros(2 * maxit + 4) if history else None
        it = self.L.orc_gmres_ex(self.h, float(h1), float(h2), _c(b), x, float(tol), int(maxit), int(restart),
                                 int(bool(deflate)), C.byref(res), hist.ctypes.data if history else None)
        if history:
            return x, it, res.value, hist
        return x, it, res.value

    def remove_mean_unique(self, r):
        r = _c(r).copy()
        self.L.orc_remove_mean_unique(self.h, r)
        return r

    def remove_mean_mass(self, x):
        x = _c(x).copy()
        self.L.orc_remove_mean_mass(self.h, x)
        return x

    def poisson(self, rhs, tol=1e-8, maxit=1000, restart=30):
        p = np.zeros(self.np)
        res = C.c_double()
        it = self.L.orc_poisson(self.h, _c(rhs), p, float(tol), int(maxit), int(restart), C.byref(res))
        return p, it, res.value


class OracleProjection:
    """Pressure projection space (A-orthonormal earlier solutions) on an OracleMesh."""

    def __init__(self, mesh, dim=20):
        self.mesh = mesh
        self.L = mesh.L
        self.h = self.L.orc_proj_new(mesh.h, int(dim))
        if not self.h:
            raise ValueError("projection dimension must be >= 1")

    def __del__(self):
        if getattr(self, "h", None):
            self.L.orc_proj_free(self.h)
            self.h = None

    @property
    def size(self):
        return self.L.orc_proj_size(self.h)

    def vector(self, i):
        out = np.zeros(self.mesh.np)
        if self.L.orc_proj_get(self.h, int(i), out) != 0:
            raise IndexError(i)
        return out

    def guess(self, b):
        x = np.zeros(self.mesh.np)
        self.L.orc_proj_guess(self.h, _c(b), x)
        return x

    def update(self, x, xbar):
        return bool(self.L.orc_proj_update(self.h, _c(x), _c(xbar)))

    def poisson(self, rhs, tol=1e-8, maxit=1000, restart=30):
        p = np.zeros(self.mesh.np)
        res = C.c_double()
        it = self.L.orc_poisson_proj(self.mesh.h, self.h, _c(rhs), p, float(tol), int(maxit), int(restart),
                                     C.byref(res))
        return p, it, res.value


class OracleHSMG:
    """Three-level hybrid Schwarz multigrid preconditioner of the pressure
    Poisson operator on an unperturbed periodic OracleMesh with N >= 4
    (levels N, N/2, 1; Schwarz smoothing by fast diagonalisation on the two
    upper levels, exact coarse solve).  Vectors: fine level as the mesh's
    local layout, middle level [E][lxm^3], coarse level on the unique corner
    nodes cx + nx (cy + ny cz)."""

    def __init__(self, mesh):
        self.mesh = mesh
        self.L = mesh.L
        self.h = self.L.orc_hsmg_new(mesh.h)
        if not self.h:
            raise ValueError("HSMG needs an unperturbed box mesh with N >= 4")
        self.lxm = self.L.orc_hsmg_lxm(self.h)
        self.nm = self.L.orc_hsmg_nm(self.h)
        self.nc = self.L.orc_hsmg_nc(self.h)

    def __del__(self):
        if getattr(self, "h", None):
            self.L.orc_hsmg_free(self.h)
            self.h = None

    def level(self, level, c):
        """1D tables of level 0 (fine) or 1 (middle), direction c: A, diag(B), S, lambda."""
        lx = self.mesh.lx if level == 0 else self.lxm
        A = np.zeros(lx * lx); Bd = np.zeros(lx); S = np.zeros(lx * lx); lam = np.zeros(lx)
        self.L.orc_hsmg_level(self.h, int(level), int(c), A, Bd, S, lam)
        return A.reshape(lx, lx), Bd, S.reshape(lx, lx), lam

    def local_solve(self, level, r):
        out = np.zeros(len(r))
        self.L.orc_hsmg_local_solve(self.h, int(level), _c(r), out)
        return out

    def smooth(self, level, r):
        out = np.zeros(len(r))
        self.L.orc_hsmg_smooth(self.h, int(level), _c(r), out)
        return out

    def _map(self, fn, x, n):
        out = np.zeros(n)
        getattr(self.L, fn)(self.h, _c(x), out)
        return out

    def coarse_solve(self, rc):
        return self._map("orc_hsmg_coarse_solve", rc, self.nc)

    def prolong_fm(self, zm):
        return self._map("orc_hsmg_prolong_fm", zm, self.mesh.np)

    def restrict_mf(self, rf):
        return self._map("orc_hsmg_restrict_mf", rf, self.nm)

    def restrict_cm(self, rm):
        return self._map("orc_hsmg_restrict_cm", rm, self.nc)

    def prolong_mc(self, ec):
        return self._map("orc_hsmg_prolong_mc", ec, self.nm)

    def apply(self, r):
        return self._map("orc_hsmg_apply", r, self.mesh.np)

    def poisson(self, rhs, tol=1e-8, maxit=1000, restart=30):
        """HSMG-preconditioned GMRES for A p = rhs, as OracleMesh.poisson."""
        p = np.zeros(self.mesh.np)
        res = C.c_double()
        it = self.L.orc_poisson_pc(self.mesh.h, self.h, _c(rhs), p, float(tol), int(maxit), int(restart),
                                   C.byref(res))
        return p, it, res.value


INIT_TGV3D, INIT_TGV2D, INIT_ZERO = 0, 1, 2
FIELD_U, FIELD_P, FIELD_ULAG1, FIELD_ULAG2, FIELD_BNLAG1, FIELD_BNLAG2 = 0, 3, 4, 7, 10, 13


class OracleFluid:
    """FP64 TGV stepper on an OracleMesh (keeps a reference to the mesh)."""

    def __init__(self, mesh, nu, dt, torder=3, vtol=1e-8, ptol=1e-8, vmaxit=500, pmaxit=1000,
                 restart=30, init=INIT_TGV3D, proj=0, dealias=False, cfl=0.0, hsmg=False):
        self.mesh = mesh
        self.L = mesh.L
        self.h = self.L.orc_fluid_new(mesh.h, float(nu), float(dt), int(torder), float(vtol), float(ptol),
                                      int(vmaxit), int(pmaxit), int(restart), int(init))
        if not self.h:
            raise ValueError("invalid fluid parameters")
        if self.L.orc_fluid_set_proj(self.h, int(proj)) != 0:
            raise ValueError("invalid projection dimension")
        self.L.orc_fluid_set_dealias(self.h, 1 if dealias else 0)
        if self.L.orc_fluid_set_cfl(self.h, float(cfl)) != 0:
            raise ValueError("invalid CFL target")
        if self.L.orc_fluid_set_hsmg(self.h, 1 if hsmg else 0) != 0:
            raise ValueError("HSMG needs an unperturbed box mesh with N >= 4")

    @property
    def proj_size(self):
        return self.L.orc_fluid_proj_size(self.h)

    def __del__(self):
        if getattr(self, "h", None):
            self.L.orc_fluid_free(self.h)
            self.h = None

    def get(self, which):
        out = np.zeros(self.mesh.np)
        if self.L.orc_fluid_get(self.h, int(which), out) != 0:
            raise ValueError(which)
        return out

    def set(self, which, arr):
        if self.L.orc_fluid_set(self.h, int(which), _c(arr)) != 0:
            raise ValueError(which)

    def velocity(self):
        return np.stack([self.get(c) for c in range(3)])

    def pressure(self):
        return self.get(FIELD_P)

    @property
    def time(self):
        return self.L.orc_fluid_time(self.h)

    @property
    def stepno(self):
        return self.L.orc_fluid_stepno(self.h)

    def set_clock(self, t, step):
        self.L.orc_fluid_set_clock(self.h, float(t), int(step))

    def step(self):
        st = _StepStats()
        self.L.orc_fluid_step(self.h, C.byref(st))
        return {"t": st.t, "ke": st.ke, "enst": st.enst, "maxdiv": st.maxdiv,
                "vit": list(st.vit), "pit": st.pit, "vres": list(st.vres), "pres": st.pres,
                "dt": st.dt, "cfl": st.cfl}
