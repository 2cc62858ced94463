"""GPU parity of libsem (called through the C ABI) against the FP64 CPU oracle.

Bars: FP64 operators within 1e-12 relative (max-norm, scaled by the output's
max-norm); reduced-storage operators within a rounding-error bound derived
from the arithmetic (Higham-style gamma_k for the contraction length plus the
storage roundings); solver iteration counts equal to the oracle's; kinetic
energy after 10 C1 steps within 1e-9 relative.
"""
import math

import numpy as np
import pytest

from oracle import OracleMesh, OracleFluid, gl, lxd, interp_matrix
from oracle.oracle import INIT_TGV3D, INIT_TGV2D
from paper_2608_24348_amd import inputs
import opbounds

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sem():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_24348_amd import sem as s
    s.load()
    return s


def _ctx(sem, nel, N, tier="fp64", mode=None, amp=0.0, **kw):
    mode = sem.MODE_FLUID if mode is None else mode
    ph = inputs.deform_phases() if amp else None
    return sem.Context(sem.mesh_desc(nel, N, amp=amp, phase=ph), sem.flow_desc(mode=mode, **kw), sem.tier(tier))


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    return t if dtype is None else t.to(dtype)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


# the last two have a single element along a direction: there both periodic
# copies of a face node (all 8 copies of the corner node on 1 x 1 x 1) sit in
# the same element
CASES = [((4, 4, 4), 5, 0.1), ((3, 2, 4), 4, 0.0), ((8, 8, 8), 7, 0.0), ((4, 4, 4), 7, 0.1), ((2, 2, 2), 11, 0.1),
         ((2, 4, 2), 9, 0.0), ((2, 2, 2), 2, 0.0), ((1, 2, 3), 5, 0.0), ((1, 1, 1), 4, 0.0)]


@pytest.mark.parametrize("nel,N,amp", CASES)
def test_geometry_matches_oracle(sem, nel, N, amp):
    c = _ctx(sem, nel, N, mode=sem.MODE_OPERATOR, amp=amp)
    m = OracleMesh(nel, N, amp=amp, phase=inputs.deform_phases() if amp else None)
    assert _rel(c.get(sem.F_MASS), m.mass()) < 1e-13
    assert _rel(c.get(sem.F_BSUM), m.bsum()) < 1e-13
    G = m.G()
    for q in range(6):
        assert np.abs(c.get(sem.F_G + q) - G[q]).max() < 1e-13 * np.abs(G).max()
    M = m.M()
    for q in range(9):
        assert np.abs(c.get(sem.F_M + q) - M[q]).max() < 1e-13 * np.abs(M).max()
    assert _rel(c.get(sem.F_DIAG_A), m.dssum(m.diag(1.0, 0.0))) < 1e-12


@pytest.mark.parametrize("nel,N,amp", CASES)
@pytest.mark.parametrize("h1,h2", [(1.0, 0.0), (1 / 1600, 11 / 6 / 5e-4)])
def test_ax_fp64_matches_oracle(sem, nel, N, amp, h1, h2):
    c = _ctx(sem, nel, N, mode=sem.MODE_OPERATOR, amp=amp)
    m = OracleMesh(nel, N, amp=amp, phase=inputs.deform_phases() if amp else None)
    u = inputs.local_normal(nel, N, seed=0)
    ref = m.ax(u, h1, h2)
    w = torch.empty(c.np, dtype=torch.float64, device="cuda:0")
    c.ax(_dev(u), w, h1, h2)
    got = w.cpu().numpy()
    assert _rel(got, ref) < 1e-12
    # assembled
    c.ax(_dev(u), w, h1, h2, assemble=True)
    assert _rel(w.cpu().numpy(), m.dssum(ref)) < 1e-12


@pytest.mark.parametrize("nel,N,amp", CASES)
def test_dssum_matches_oracle(sem, nel, N, amp):
    c = _ctx(sem, nel, N, mode=sem.MODE_OPERATOR, amp=amp)
    m = OracleMesh(nel, N, amp=amp, phase=None)
    u = inputs.local_normal(nel, N, seed=1)
    t = _dev(u)
    c.dssum(t)
    ref = m.dssum(u)
    assert np.abs(t.cpu().numpy() - ref).max() <= 4e-16 * np.abs(ref).max() * 8
    # fp32 storage: sums of at most 8 fp32 values
    t32 = _dev(u, torch.float32)
    c.dssum(t32)
    ref32 = m.dssum(u.astype(np.float32).astype(np.float64))
    assert np.abs(t32.cpu().numpy() - ref32).max() <= 8 * 2 ** -23 * np.abs(ref32).max()
    _copies_equal(m.gid(), t.cpu().numpy())
    _copies_equal(m.gid(), t32.cpu().numpy())
    # 16-bit storage: the copies are summed in fp32 and the sum rounded once;
    # per point |err| <= u_16 |sum| + 7 * 2^-24 sum|copies| (+ half the fp16
    # subnormal spacing)
    for dt, u16, tiny in ((torch.float16, 2 ** -11, 2 ** -25), (torch.bfloat16, 2 ** -8, 0.0)):
        th = _dev(u, dt)
        uh = th.double().cpu().numpy()
        c.dssum(th)
        got = th.double().cpu().numpy()
        refh = m.dssum(uh)
        bound = u16 * np.abs(refh) + 7 * 2 ** -24 * m.dssum(np.abs(uh)) + tiny
        assert (np.abs(got - refh) <= bound).all()
        _copies_equal(m.gid(), got)


def _copies_equal(gid, v):
    """every copy of a global node holds the same value"""
    o = np.argsort(gid, kind="stable")
    g, x = gid[o], v[o]
    same = g[1:] == g[:-1]
    assert (x[1:][same] == x[:-1][same]).all()


@pytest.mark.parametrize("tier,buf,eps_geo,eps_vec", [
    ("fp32b", "float32", 2 ** -24, 2 ** -24),
    ("fp32b", "float64", 2 ** -24, 0.0),
    ("fp32b+fp16all", "float64", 2 ** -11, 0.0),
    ("fp32b+fp16all", "float32", 2 ** -11, 2 ** -24),
    ("fp32b+bf16all", "float32", 2 ** -8, 2 ** -24),
    ("fp32b+fp16all", "float16", 2 ** -11, 2 ** -11),
    ("fp32b+bf16all", "bfloat16", 2 ** -8, 2 ** -8),
])
# (3, 1, 3): nine elements, so the last block of four holds a single element
# (undeformed: the deformation map needs even element counts)
@pytest.mark.parametrize("nel,N,amp", [((4, 4, 4), 7, 0.1), ((3, 1, 3), 7, 0.0), ((2, 2, 2), 11, 0.1)])
@pytest.mark.parametrize("h1,h2", [(1.0, 0.0), (1 / 1600, 11 / 6 / 5e-4)])
def test_ax_reduced_precision_within_rounding_bound(sem, tier, buf, eps_geo, eps_vec, nel, N, amp, h1, h2):
    """Per point: |w_gpu - w| <= (gamma_k(u_arith) + 2 eps_geo + eps_out) (|A| |u|)_i,
    with |A| |u| the operator chain on |D|, |G|, |B|, |u| (tests/opbounds.py)
    and the oracle's w of the stored input.  Normwise, the error is a small
    multiple of the storage unit roundoff times ||(|A||u|)|| / ||w||."""
    c = _ctx(sem, nel, N, tier=tier, mode=sem.MODE_OPERATOR, amp=amp)
    m = OracleMesh(nel, N, amp=amp, phase=inputs.deform_phases() if amp else None)
    u = inputs.local_normal(nel, N, seed=0)
    dt = getattr(torch, buf)
    ut = _dev(u, dt)
    u_rounded = ut.double().cpu().numpy()  # the input is what it is in storage precision
    ref = m.ax(u_rounded, h1, h2)
    w = torch.empty(c.np, dtype=dt, device="cuda:0")
    geom = sem.FP32 if tier == "fp32b" else (sem.FP16 if "fp16" in tier else sem.BF16)
    c.ax(ut, w, h1, h2, geom=geom)
    got = w.double().cpu().numpy()
    u_arith = 2 ** -24 if buf != "float64" else 2 ** -53  # fp64 vectors run fp64 arithmetic
    bound = opbounds.ax_bound(m, u_rounded, h1, h2, u_arith, eps_geo, eps_vec, opbounds.TINY[buf])
    err = np.abs(got - ref)
    assert np.all(err <= bound), (err / bound).max()
    # normwise: rounding errors of independent terms do not align, so the
    # error norm stays within the storage unit roundoff (arithmetic: its
    # square-root growth over the chain) times the |A||u| / |Au| norm ratio
    ratio = np.linalg.norm(opbounds.abs_ax(m, u_rounded, h1, h2)) / np.linalg.norm(ref)
    unit = max(eps_geo, eps_vec, u_arith * math.sqrt(2 * (N + 1) + 8))
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(tier, buf, nel, N, (h1, h2), "max err/bound %.3f" % (err / bound).max(),
          "normwise %.3e = %.3f unit x ratio %.2f" % (rel, rel / unit / ratio, ratio))
    assert rel <= 2 * unit * ratio


@pytest.mark.parametrize("tier,buf,eps16,tiny16", [
    ("fp32b+fp16all", "float32", 2 ** -11, 2 ** -25),
    ("fp32b+fp16all", "float16", 2 ** -11, 2 ** -25),
    ("fp32b+bf16all", "float32", 2 ** -8, 2 ** -134),
    ("fp32b+bf16all", "bfloat16", 2 ** -8, 2 ** -134),
])
# N = 7 runs the matrix-core kernel (the undeformed (3, 1, 3) mesh leaves the
# last block of four with one element); N = 5 and N = 11 the vector kernel's
# 16-bit mode
@pytest.mark.parametrize("nel,N,amp", [((4, 4, 4), 7, 0.1), ((3, 1, 3), 7, 0.0), ((4, 2, 2), 5, 0.1),
                                       ((2, 2, 2), 11, 0.1)])
@pytest.mark.parametrize("h1,h2", [(1.0, 0.0), (1 / 1600, 11 / 6 / 5e-4)])
def test_ax_16bit_arithmetic_within_rounding_bound(sem, tier, buf, eps16, tiny16, nel, N, amp, h1, h2):
    """Table 2's fp16-compute overrides (16-bit operands, fp32 sums): per point
    within ax_bound's fp32 terms plus gamma_4(eps16) (|A||u|) for the four
    16-bit operand roundings (tests/opbounds.py ax16_bound).  The rounding
    must really happen: in Poisson form the result differs from the
    fp32-arithmetic one by at least a hundredth of the 16-bit unit roundoff,
    normwise (in Helmholtz form the fp32 mass term dominates the norm)."""
    c = _ctx(sem, nel, N, tier=tier, mode=sem.MODE_OPERATOR, amp=amp)
    m = OracleMesh(nel, N, amp=amp, phase=inputs.deform_phases() if amp else None)
    u = inputs.local_normal(nel, N, seed=0)
    dt = getattr(torch, buf)
    ut = _dev(u, dt)
    u_rounded = ut.double().cpu().numpy()
    ref = m.ax(u_rounded, h1, h2)
    geom = sem.FP16 if "fp16" in tier else sem.BF16
    w = torch.empty(c.np, dtype=dt, device="cuda:0")
    c.ax(ut, w, h1, h2, geom=geom, half_compute=True)
    got = w.double().cpu().numpy()
    eps_out = 2 ** -24 if buf == "float32" else eps16
    bound = opbounds.ax16_bound(m, u_rounded, h1, h2, eps16, tiny16, eps16, eps_out, opbounds.TINY[buf])
    err = np.abs(got - ref)
    w32 = torch.empty_like(w)
    c.ax(ut, w32, h1, h2, geom=geom)
    d32 = np.linalg.norm(got - w32.double().cpu().numpy()) / np.linalg.norm(ref)
    print(tier, buf, nel, N, (h1, h2), "max err/bound %.3f" % (err / bound).max(),
          "normwise err %.2e, vs fp32 arithmetic %.2e" % (np.linalg.norm(got - ref) / np.linalg.norm(ref), d32))
    assert np.all(err <= bound), (err / bound).max()
    if h2 == 0.0:
        assert d32 >= 0.01 * eps16


@pytest.mark.parametrize("geom,tier", [("FP16", "fp32b+fp16all"), ("BF16", "fp32b+bf16all")])
@pytest.mark.parametrize("N", [7, 5])
def test_ax_16bit_arithmetic_is_scale_invariant(sem, geom, tier, N):
    """The per-element power-of-two scale makes the 16-bit roundings relative
    to each element's own magnitude: with fp32 vectors, w(2^-20 u) equals
    2^-20 w(u) bit for bit (a PCG correction of size 1e-6 loses nothing to
    the 16-bit format's subnormal range)."""
    nel = (4, 2, 2)
    c = _ctx(sem, nel, N, tier=tier, mode=sem.MODE_OPERATOR, amp=0.1)
    u = inputs.local_normal(nel, N, seed=3)
    g = getattr(sem, geom)
    for h1, h2 in [(1.0, 0.0), (1 / 1600, 11 / 6 / 5e-4)]:
        ut = _dev(u, torch.float32)
        w1 = torch.empty_like(ut)
        w2 = torch.empty_like(ut)
        c.ax(ut, w1, h1, h2, geom=g, half_compute=True)
        c.ax(ut * 2.0 ** -20, w2, h1, h2, geom=g, half_compute=True)
        assert torch.equal(w2, w1 * 2.0 ** -20)


def test_poisson_solve_matches_oracle(sem):
    nel, N = (4, 4, 4), 7
    c = _ctx(sem, nel, N, mode=sem.MODE_POISSON, pres_tol=1e-10, pres_maxit=2000)
    m = OracleMesh(nel, N)
    X = m.coords()
    f = 3 * np.sin(X[0]) * np.sin(X[1]) * np.sin(X[2]) + 1e-3 * m.from_lattice(inputs.lattice_normal(nel, N, 7))
    rhs = m.dssum(m.mass() * f)
    pref, itref, resref = m.poisson(rhs, tol=1e-10, maxit=2000)
    sol = torch.empty(c.np, dtype=torch.float64, device="cuda:0")
    st = sem.poisson_solve([c], [_dev(rhs)], [sol])[0]
    assert st["status"] == 0
    assert st["iters"] == itref
    assert _rel(sol.cpu().numpy(), pref) < 1e-9


@pytest.mark.parametrize("proj", [0, 20])
def test_fluid_c1_ten_steps_match_oracle(sem, proj):
    """C1 (8^3, N=7, 10 steps, tolerances 1e-8): per-step iteration counts
    equal, KE and enstrophy within 1e-9, without and with the pressure
    projection space of Sec. 3 (dimension 20)."""
    nel, N = (8, 8, 8), 7
    nu, dt = 1 / 1600, 1e-3
    c = _ctx(sem, nel, N, nu=nu, dt=dt, proj=proj)
    m = OracleMesh(nel, N)
    f = OracleFluid(m, nu, dt, init=INIT_TGV3D, proj=proj)
    d0 = c.diagnostics()
    ke0, en0, _ = m.diagnostics(f.velocity())
    assert abs(d0["ke"] - ke0) < 1e-12 * ke0 and abs(d0["enst"] - en0) < 1e-12 * en0
    L = opbounds.div_lipschitz(m)
    for k in range(10):
        g = sem.fluid_step([c], 1)[0][0]
        o = f.step()
        print("step", k + 1, "gpu its", g["vit"], g["pit"], "oracle its", o["vit"], o["pit"])
        assert g["status"] == 0
        assert g["vit"] == o["vit"]
        # with projection the guess carries the rounding of earlier solves,
        # so a solve may stop one iteration apart at the tolerance edge
        assert abs(g["pit"] - o["pit"]) <= (1 if proj else 0)
        assert abs(g["ke"] - o["ke"]) <= 1e-9 * o["ke"]
        assert abs(g["enst"] - o["enst"]) <= 1e-9 * o["enst"]
        opbounds.check_maxdiv(m, L, g["maxdiv"], o["maxdiv"], c.velocity(), f.velocity(), k + 1)
    assert _rel(c.velocity(), f.velocity()) < 1e-8
    assert np.abs(c.pressure() - f.pressure()).max() < 1e-8 * np.abs(f.pressure()).max()
    if proj:
        assert f.proj_size > 0


def test_fluid_tgv2d_ragged_mesh_matches_oracle(sem):
    nel, N = (4, 2, 2), 5
    nu, dt = 0.05, 1e-3
    c = _ctx(sem, nel, N, nu=nu, dt=dt, init=sem.INIT_TGV2D)
    m = OracleMesh(nel, N)
    f = OracleFluid(m, nu, dt, init=INIT_TGV2D)
    gst = sem.fluid_step([c], 5)[0]
    for k in range(5):
        o = f.step()
        assert gst[k]["vit"] == o["vit"] and gst[k]["pit"] == o["pit"]
        assert abs(gst[k]["ke"] - o["ke"]) <= 1e-10 * o["ke"]
    assert _rel(c.velocity(), f.velocity()) < 1e-9


@pytest.mark.parametrize("nel", [(1, 2, 2), (2, 1, 1)])
def test_fluid_single_element_direction_matches_oracle(sem, nel):
    """One element along a direction (the element meets its own periodic
    image): 5 TGV steps, N = 6, tolerances 1e-8, Jacobi pressure
    preconditioner: counts equal, KE and enstrophy within 1e-9."""
    N, nu, dt = 6, 1 / 100, 1e-3
    c = _ctx(sem, nel, N, nu=nu, dt=dt)
    m = OracleMesh(nel, N)
    f = OracleFluid(m, nu, dt, init=INIT_TGV3D)
    gst = sem.fluid_step([c], 5)[0]
    for k in range(5):
        o = f.step()
        g = gst[k]
        print(nel, "step", k + 1, "gpu its", g["vit"], g["pit"], "oracle its", o["vit"], o["pit"])
        assert g["status"] == 0
        assert g["vit"] == o["vit"] and g["pit"] == o["pit"]
        assert abs(g["ke"] - o["ke"]) <= 1e-9 * o["ke"]
        assert abs(g["enst"] - o["enst"]) <= 1e-9 * o["enst"]
    assert _rel(c.velocity(), f.velocity()) < 1e-8


@pytest.mark.parametrize("nel,N,amp", [((4, 4, 4), 5, 0.1), ((2, 2, 2), 11, 0.0)])
def test_sem_operators_match_oracle(sem, nel, N, amp):
    c = _ctx(sem, nel, N, amp=amp)
    m = OracleMesh(nel, N, amp=amp, phase=inputs.deform_phases() if amp else None)
    u = np.stack([inputs.local_normal(nel, N, seed=s) for s in (0, 1, 2)])
    ref = m.conv(u)
    got = c.conv([_dev(u[q]) for q in range(3)])
    for q in range(3):
        assert _rel(got[q].cpu().numpy(), ref[q]) < 1e-12
    refg = m.opgrad(u[0])
    gotg = c.opgrad(_dev(u[0]))
    for q in range(3):
        assert _rel(gotg[q].cpu().numpy(), refg[q]) < 1e-12
    refd = m.wdiv(u)
    gotd = c.wdiv([_dev(u[q]) for q in range(3)])
    assert _rel(gotd.cpu().numpy(), refd) < 1e-12


DEALIAS_CASES = [((4, 4, 4), 5, 0.1), ((2, 2, 2), 11, 0.1), ((2, 4, 2), 7, 0.0), ((2, 2, 2), 2, 0.1),
                 ((4, 2, 2), 9, 0.1), ((2, 2, 2), 6, 0.0)]


@pytest.mark.parametrize("nel,N,amp", DEALIAS_CASES)
def test_dealiased_convection_fp64_matches_oracle(sem, nel, N, amp):
    """Convection on the 3/2-rule Gauss-Legendre grid (Sec. 3 runs dealiased),
    fp64 tier: within 1e-12 of the oracle on curved and affine elements, with
    lxd^3 from 125 (N = 2) to 5832 (N = 11) fine points per element."""
    c = _ctx(sem, nel, N, amp=amp, dealias=1)
    m = OracleMesh(nel, N, amp=amp, phase=inputs.deform_phases() if amp else None)
    u = np.stack([inputs.local_normal(nel, N, seed=s) for s in (3, 4, 5)])
    ref = m.conv_dealias(u)
    got = c.conv([_dev(u[q]) for q in range(3)])
    for q in range(3):
        assert _rel(got[q].cpu().numpy(), ref[q]) < 1e-12


def _dealias_abs_bound(m, u, floor=0.0):
    """Magnitude of every term of the dealiased convection, element by element:
    the same contractions as the method with every factor replaced by its
    absolute value (the Higham-style bound multiplies it by gamma_K).  With
    floor > 0 every metric term is raised by floor * (the element's largest
    metric term), which covers absolute (subnormal) rounding of scaled 16-bit
    storage."""
    xi, _, D = m.tables()
    lx = m.lx
    nd = lxd(lx)
    z, wz = gl(nd)
    I = interp_matrix(xi, z)
    ID = I @ D
    aI, aID = np.abs(I), np.abs(ID)
    E = m.np // lx ** 3
    X = m.coords().reshape(3, E, lx, lx, lx)           # [c][e][k][j][i]
    U = np.abs(np.asarray(u)).reshape(3, E, lx, lx, lx)

    def t3(A1, A2, A3, v):                              # v[..., k, j, i]
        return np.einsum("ia,jb,kc,...cba->...kji", A1, A2, A3, v, optimize=True)

    J = np.stack([np.stack([t3(ID, I, I, X[c]), t3(I, ID, I, X[c]), t3(I, I, ID, X[c])], 1) for c in range(3)], 1)
    J = np.moveaxis(J, (1, 2), (-2, -1))                # [e][k][j][i][c][a] = dx_c/dr_a
    det = np.linalg.det(J)
    W = det * np.einsum("k,j,i->kji", wz, wz, wz)
    rx = np.abs(np.linalg.inv(J) * W[..., None, None])  # [..][a][c] = |W dr_a/dx_c|
    if floor:
        rx = rx + floor * rx.reshape(E, -1).max(axis=1)[:, None, None, None, None, None]
    uf = np.stack([t3(aI, aI, aI, U[c]) for c in range(3)], -1)     # [e][k][j][i][c]
    V = np.abs(np.einsum("ekjiac,ekjic->ekjia", np.abs(rx), uf))
    out = np.zeros((3, E, lx, lx, lx))
    for f in range(3):
        g = np.stack([t3(aID, aI, aI, U[f]), t3(aI, aID, aI, U[f]), t3(aI, aI, aID, U[f])], -1)
        T = (V * g).sum(-1)
        out[f] = np.einsum("ia,jb,kc,ekji->ecba", aI, aI, aI, T, optimize=True)
    return out.reshape(3, m.np)


@pytest.mark.parametrize("tier,eps16", [("fp32b+fp16a", 2.0 ** -11), ("fp32b+bf16a", 2.0 ** -8)])
@pytest.mark.parametrize("nel,N,amp", [((4, 4, 4), 5, 0.1), ((2, 2, 2), 11, 0.1), ((2, 4, 2), 7, 0.1)])
def test_dealiased_convection_16bit_metric_within_rounding_bound(sem, nel, N, amp, tier, eps16):
    """B-5 (Table 2: fp16 in adv_dealias): the fine-grid metric terms stored in
    16 bits with a power-of-two scale per element, fp32 arithmetic.  Bound:
    gamma_K |terms| (fp32 arithmetic as in the fp32 case) + eps16 |terms|
    (one rounding of each metric term; the floor covers fp16 subnormals)."""
    c = _ctx(sem, nel, N, tier=tier, amp=amp, dealias=1)
    m = OracleMesh(nel, N, amp=amp, phase=inputs.deform_phases() if amp else None)
    u = np.stack([inputs.local_normal(nel, N, seed=s) for s in (9, 10, 11)])
    ref = m.conv_dealias(u)
    got = np.stack([g.cpu().numpy() for g in c.conv([_dev(u[q]) for q in range(3)])])
    lx = N + 1
    K = 6 * lx + 3 * lxd(lx) + 6 + 12
    gam = K * 2.0 ** -24 / (1 - K * 2.0 ** -24)
    bound = gam * _dealias_abs_bound(m, u) + eps16 * _dealias_abs_bound(m, u, floor=2.0 ** -13)
    err = np.abs(got - ref)
    assert np.all(err <= bound), float((err / bound).max())
    # the 16-bit storage is in effect: errors well above fp32 rounding
    assert _rel(got, ref) > 10 * gam


@pytest.mark.parametrize("nel,N,amp", [((4, 4, 4), 5, 0.1), ((2, 2, 2), 11, 0.1), ((2, 4, 2), 7, 0.0)])
def test_dealiased_convection_fp32_within_rounding_bound(sem, nel, N, amp):
    """fp32 metric terms and arithmetic (tier fp32b): |err| <= gamma_K |terms|
    point by point, K = 3 lx (velocity to the fine grid) + 3 lx (derivatives)
    + 3 lxd (back to the GLL points) + 6 (the two 3-term sums) + 12 storage
    roundings (input, metric terms, I and ID entries, the fp32 tables)."""
    c = _ctx(sem, nel, N, tier="fp32b", amp=amp, dealias=1)
    m = OracleMesh(nel, N, amp=amp, phase=inputs.deform_phases() if amp else None)
    u = np.stack([inputs.local_normal(nel, N, seed=s) for s in (6, 7, 8)])
    ref = m.conv_dealias(u)
    got = np.stack([g.cpu().numpy() for g in c.conv([_dev(u[q]) for q in range(3)])])
    lx = N + 1
    K = 6 * lx + 3 * lxd(lx) + 6 + 12
    gam = K * 2.0 ** -24 / (1 - K * 2.0 ** -24)
    bound = gam * _dealias_abs_bound(m, u)
    err = np.abs(got - ref)
    assert np.all(err <= bound), float((err / bound).max())
    # fp32 arithmetic really ran (fp64 throughout would agree to ~1e-15)
    assert _rel(got, ref) > 1e-9


def test_fluid_dealiased_c1_matches_oracle(sem):
    """C1 (8^3, N = 7, 10 steps) with dealiased convection, fp64 tier: the
    iteration counts equal the oracle's and KE / enstrophy agree to 1e-9."""
    nel, N = (8, 8, 8), 7
    nu, dt = 1 / 1600, 1e-3
    c = _ctx(sem, nel, N, nu=nu, dt=dt, dealias=1)
    m = OracleMesh(nel, N)
    f = OracleFluid(m, nu, dt, init=INIT_TGV3D, dealias=True)
    gst = sem.fluid_step([c], 10)[0]
    for k in range(10):
        o = f.step()
        g = gst[k]
        assert g["status"] == 0
        assert g["vit"] == o["vit"] and g["pit"] == o["pit"], (k, g, o)
        assert abs(g["ke"] - o["ke"]) <= 1e-9 * o["ke"]
        assert abs(g["enst"] - o["enst"]) <= 1e-9 * o["enst"]
    assert _rel(c.velocity(), f.velocity()) < 1e-8


def test_fluid_adaptive_cfl_c1_matches_oracle(sem):
    """Adaptive time stepping toward CFL 0.4 (Sec. 3) on C1 (8^3, N = 7, 10
    steps, tolerances 1e-8): every step size agrees with the oracle's to 1e-9
    relative (a step is the target over a maximum of velocity terms, so it
    carries the velocity's own parity, ~1e-11; the first step ~1e-14), each
    CFL number is the target, iteration counts are equal, KE and enstrophy
    agree to 1e-9, and the clock is the sum of the steps."""
    nel, N = (8, 8, 8), 7
    nu, dtmax, target = 1 / 1600, 0.05, 0.4
    c = _ctx(sem, nel, N, nu=nu, dt=dtmax, cfl=target)
    m = OracleMesh(nel, N)
    f = OracleFluid(m, nu, dtmax, init=INIT_TGV3D, cfl=target)
    gst = sem.fluid_step([c], 10)[0]
    for k in range(10):
        o = f.step()
        g = gst[k]
        print("step", k + 1, "dt", g["dt"], o["dt"], "cfl", g["cfl"], "its", g["vit"], g["pit"], o["vit"], o["pit"])
        assert g["status"] == 0
        assert abs(g["dt"] - o["dt"]) <= (1e-12 if k == 0 else 1e-9) * o["dt"]
        assert abs(g["cfl"] - o["cfl"]) <= 1e-12
        assert g["vit"] == o["vit"] and g["pit"] == o["pit"]
        assert abs(g["ke"] - o["ke"]) <= 1e-9 * o["ke"]
        assert abs(g["enst"] - o["enst"]) <= 1e-9 * o["enst"]
    assert abs(gst[-1]["t"] - sum(s["dt"] for s in gst)) < 1e-13
    assert gst[0]["dt"] < dtmax and abs(gst[0]["cfl"] - target) < 1e-12
    assert _rel(c.velocity(), f.velocity()) < 1e-8


def test_paper_solver_settings_match_oracle(sem):
    """The solver settings of Sec. 3 together: dealiased convection, adaptive dt
    toward CFL 0.4, pressure projection space of dimension 20 (4^3 elements,
    N = 7, 8 steps, tolerances 1e-8).  Velocity iteration counts equal,
    pressure counts within 1 (the projected guess carries earlier rounding),
    step sizes within 1e-9, KE and enstrophy within 1e-9."""
    nel, N = (4, 4, 4), 7
    nu, dtmax, target = 1 / 1600, 0.05, 0.4
    c = _ctx(sem, nel, N, nu=nu, dt=dtmax, cfl=target, dealias=1, proj=20)
    m = OracleMesh(nel, N)
    f = OracleFluid(m, nu, dtmax, init=INIT_TGV3D, cfl=target, dealias=True, proj=20)
    gst = sem.fluid_step([c], 8)[0]
    for k in range(8):
        o = f.step()
        g = gst[k]
        assert g["status"] == 0
        assert g["vit"] == o["vit"] and abs(g["pit"] - o["pit"]) <= 1, (k, g, o)
        assert abs(g["dt"] - o["dt"]) <= 1e-9 * o["dt"]
        assert abs(g["ke"] - o["ke"]) <= 1e-9 * o["ke"]
        assert abs(g["enst"] - o["enst"]) <= 1e-9 * o["enst"]
    assert f.proj_size > 0
    assert _rel(c.velocity(), f.velocity()) < 1e-8


def test_batched_adaptive_dt_is_bitwise_equal_to_alone(sem):
    """Each request of a batch keeps its own step size under adaptive dt."""
    specs = [((4, 4, 4), 7, 1 / 400), ((2, 2, 4), 7, 1 / 100)]
    alone = []
    for nel, N, nu in specs:
        c = _ctx(sem, nel, N, nu=nu, dt=0.05, cfl=0.4)
        st = sem.fluid_step([c], 4)[0]
        alone.append((st, c.velocity()))
    ctxs = [_ctx(sem, nel, N, nu=nu, dt=0.05, cfl=0.4) for nel, N, nu in specs]
    mix = sem.fluid_step(ctxs, 4)
    for i, c in enumerate(ctxs):
        st, u = alone[i]
        assert [s["dt"] for s in mix[i]] == [s["dt"] for s in st]
        assert np.array_equal(c.velocity(), u)
    assert mix[0][0]["dt"] != mix[1][0]["dt"]


@pytest.mark.parametrize("proj,dealias,tier", [(0, 0, "fp64"), (3, 0, "fp64"), (0, 1, "fp64"), (0, 0, "fp32b+fp16"),
                                               (0, 0, "fp32b+fp16c")])
def test_batched_step_is_bitwise_equal_to_alone(sem, proj, dealias, tier):
    # with a 3-vector projection space, 5 steps include a full-space restart;
    # the 16-bit-geometry tier runs element counts that leave the last block
    # of four elements part empty (9 and 18 elements)
    specs = [((4, 4, 4), 7, 1 / 400), ((6, 4, 4), 7, 1 / 1000), ((2, 2, 4), 7, 1 / 100)]
    if tier != "fp64":
        specs = [((4, 4, 4), 7, 1 / 400), ((3, 1, 3), 7, 1 / 1000), ((3, 2, 3), 7, 1 / 100)]
    nst = 5 if proj else 3
    alone = []
    for nel, N, nu in specs:
        c = _ctx(sem, nel, N, nu=nu, dt=1e-3, proj=proj, dealias=dealias, tier=tier)
        st = sem.fluid_step([c], nst)[0]
        alone.append((st, c.velocity(), c.pressure()))
    ctxs = [_ctx(sem, nel, N, nu=nu, dt=1e-3, proj=proj, dealias=dealias, tier=tier) for nel, N, nu in specs]
    mix = sem.fluid_step(ctxs, nst)
    for i, c in enumerate(ctxs):
        st, u, p = alone[i]
        assert [s["pit"] for s in mix[i]] == [s["pit"] for s in st]
        assert np.array_equal(c.velocity(), u)
        assert np.array_equal(c.pressure(), p)


@pytest.mark.parametrize("tier,proj,dealias", [("fp32b", 0, 0), ("fp32b+fp16", 0, 0), ("fp32b+bf16", 0, 0),
                                               ("fp32b", 20, 0), ("fp32b", 0, 1), ("fp32b+fp16a", 0, 1),
                                               ("fp32b+fp16c", 0, 0), ("fp32b+bf16c", 0, 0), ("fp32b+fp16pc", 0, 0)])
def test_mixed_tier_c1_energy_and_enstrophy_error(sem, tier, proj, dealias):
    """Mixed tiers against the FP64 oracle on C1 (8^3, N=7, 10 steps): the error
    metrics of the paper (Sec. 4.2 equations) stay inside the stated bounds:
    fp32b e_E,max <= 1e-4 %, e_Omega,max <= 1e-3 %; 16-bit geometry tiers
    e_E,max <= 1e-2 %, e_Omega,max <= 1e-1 %."""
    from oracle import e_max
    nel, N, nu, dt = (8, 8, 8), 7, 1 / 1600, 1e-3
    c = _ctx(sem, nel, N, tier=tier, nu=nu, dt=dt, proj=proj, dealias=dealias)
    m = OracleMesh(nel, N)
    f = OracleFluid(m, nu, dt, init=INIT_TGV3D, proj=proj, dealias=bool(dealias))
    gst = sem.fluid_step([c], 10)[0]
    ost = [f.step() for _ in range(10)]
    assert all(s["status"] == 0 for s in gst)
    eE = e_max([s["ke"] for s in gst], [s["ke"] for s in ost])
    eO = e_max([s["enst"] for s in gst], [s["enst"] for s in ost])
    print(tier, "e_E,max %.3e %%  e_Omega,max %.3e %%" % (eE, eO), "pit", [s["pit"] for s in gst])
    lim = (1e-4, 1e-3) if tier == "fp32b" else (1e-2, 1e-1)
    assert eE <= lim[0] and eO <= lim[1]


def test_copy_state_continues_the_run_bitwise(sem):
    """Carrying the state to a fresh context (same tier) continues the run
    exactly: the step-level precision control hands over an exact state."""
    nel, N, nu, dt = (4, 4, 4), 7, 1 / 800, 1e-3
    a = _ctx(sem, nel, N, nu=nu, dt=dt)
    sem.fluid_step([a], 5)
    b = _ctx(sem, nel, N, nu=nu, dt=dt)
    sem.copy_state(b, a)
    sa = sem.fluid_step([a], 3)[0]
    sb = sem.fluid_step([b], 3)[0]
    assert [s["pit"] for s in sa] == [s["pit"] for s in sb]
    assert [s["t"] for s in sa] == [s["t"] for s in sb]
    assert np.array_equal(a.velocity(), b.velocity()) and np.array_equal(a.pressure(), b.pressure())
    # mismatched meshes are refused
    c = _ctx(sem, (4, 4, 2), N, nu=nu, dt=dt)
    with pytest.raises(sem.SemError):
        sem.copy_state(c, a)


def test_precision_schedule_fp64_then_fp32b_c1(sem):
    """Time/step-level precision (Fig. 4): fp64 for the first 5 steps of C1,
    fp32b for the next 5; the fp64 phase is bitwise the fp64 run, the whole
    series stays within the fp32b error bounds against the oracle."""
    from oracle import e_max
    nel, N, nu, dt = (8, 8, 8), 7, 1 / 1600, 1e-3
    mesh = sem.mesh_desc(nel, N)
    flow = sem.flow_desc(nu=nu, dt=dt)
    sched, last = sem.run_schedule(mesh, flow, [("fp64", 5), ("fp32b", 5)])
    ref = _ctx(sem, nel, N, nu=nu, dt=dt)
    r64 = sem.fluid_step([ref], 5)[0]
    assert [s["ke"] for s in sched[:5]] == [s["ke"] for s in r64]
    m = OracleMesh(nel, N)
    f = OracleFluid(m, nu, dt, init=INIT_TGV3D)
    ost = [f.step() for _ in range(10)]
    assert all(s["status"] == 0 for s in sched)
    assert abs(sched[-1]["t"] - 10 * dt) < 1e-12
    eE = e_max([s["ke"] for s in sched], [s["ke"] for s in ost])
    eO = e_max([s["enst"] for s in sched], [s["enst"] for s in ost])
    print("schedule fp64 x5 + fp32b x5: e_E,max %.3e %%  e_Omega,max %.3e %%" % (eE, eO))
    assert eE <= 1e-4 and eO <= 1e-3
