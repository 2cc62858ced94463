"""Pins of the oracle's three-level hybrid Schwarz multigrid (HSMG) pressure
preconditioner against independent constructions.

Each check builds its reference another way than the oracle:
- numpy polynomial integration for the 1D stiffness and mass;
- dense Kronecker matrices for the local operator;
- the oracle's geometric-factor Poisson operator on an order-1 mesh for the coarse solve;
- closed-form interpolants;
- unique-node inner products for the transposes;
- an unpreconditioned reference solve.
So a wrong sign, a dropped extension term, a transposed interpolation or a
missing weight fails one of them.
"""
import numpy as np
import pytest

from oracle import OracleMesh, OracleFluid, OracleHSMG, gll
from oracle.oracle import INIT_TGV3D

LO, HI = -np.pi, np.pi


def _mesh(nel=(4, 3, 2), N=7):
    return OracleMesh(nel, N)


def _mult(nel, lx):
    """multiplicity of every local point of a periodic box, from index arithmetic"""
    n = lx - 1
    face = np.array([2 if (i == 0 or i == n) else 1 for i in range(lx)])
    m3 = (face[None, None, :] * face[None, :, None] * face[:, None, None]).ravel()
    return np.tile(m3, nel[0] * nel[1] * nel[2]).astype(float)


def test_hsmg_rejects_unsupported_meshes():
    with pytest.raises(ValueError):
        OracleHSMG(OracleMesh((2, 2, 2), 3))
    with pytest.raises(ValueError):
        OracleHSMG(OracleMesh((2, 2, 2), 6, amp=0.05))


@pytest.mark.parametrize("level", [0, 1])
def test_local_1d_matrices_by_polynomial_integration(level):
    """v^T A v = int_e (v')^2 + (v_0^2 + v_N^2) / delta and
    B = (h/2) w + delta/2 at the two end nodes, for v of degree <= N (exact
    GLL quadrature of (v')^2), with delta = (h/2)(xi_1 - xi_0)."""
    nel = (4, 3, 2)
    m = _mesh(nel)
    H = OracleHSMG(m)
    N = 7 if level == 0 else 3
    xi, w = gll(N)
    rng = np.random.default_rng(level)
    for c in range(3):
        A, Bd, S, lam = H.level(level, c)
        h = (HI - LO) / nel[c]
        delta = 0.5 * h * (xi[1] - xi[0])
        for _ in range(3):
            coef = rng.standard_normal(N + 1)
            # v(x) on the element [0, h] as a power series in x
            P = np.polynomial.Polynomial(coef)
            x = 0.5 * h * (1 + xi)
            v = P(x)
            dP = P.deriv()
            energy = (dP * dP).integ()(h) - (dP * dP).integ()(0.0)
            want = energy + (v[0] ** 2 + v[-1] ** 2) / delta
            assert abs(v @ A @ v - want) <= 1e-11 * abs(want)
        Bw = 0.5 * h * w
        Bw[0] += 0.5 * delta
        Bw[-1] += 0.5 * delta
        assert np.allclose(Bd, Bw, rtol=1e-14, atol=0)
        # fast diagonalisation: S^T B S = I, S^T A S = diag(lam)
        assert np.allclose(S.T @ np.diag(Bd) @ S, np.eye(N + 1), atol=1e-12)
        assert np.allclose(S.T @ A @ S, np.diag(lam), atol=1e-9 * lam.max())
        assert lam.min() > 0


@pytest.mark.parametrize("level", [0, 1])
def test_local_solve_inverts_the_kronecker_operator(level):
    m = _mesh()
    H = OracleHSMG(m)
    mats = [H.level(level, c) for c in range(3)]
    A = [q[0] for q in mats]
    B = [np.diag(q[1]) for q in mats]
    L = (np.kron(B[2], np.kron(B[1], A[0])) + np.kron(B[2], np.kron(A[1], B[0]))
         + np.kron(A[2], np.kron(B[1], B[0])))
    r = np.random.default_rng(3).standard_normal(L.shape[0])
    u = H.local_solve(level, r)
    assert np.abs(L @ u - r).max() <= 1e-12 * np.abs(r).max()
    # a sign error in one direction (A_x -> -A_x) would not invert L
    assert np.abs(np.linalg.solve(L, r) - u).max() <= 1e-10 * np.abs(u).max()


def _to_local_corners(nel, ec):
    nx, ny, nz = nel
    out = np.zeros(nx * ny * nz * 8)
    for e in range(nx * ny * nz):
        ex, ey, ez = e % nx, (e // nx) % ny, e // (nx * ny)
        for c in range(2):
            for b in range(2):
                for a in range(2):
                    out[e * 8 + a + 2 * (b + 2 * c)] = ec[(ex + a) % nx + nx * ((ey + b) % ny + ny * ((ez + c) % nz))]
    return out


def test_coarse_solve_inverts_the_order1_sem_operator():
    """A_c e = r - mean(r) with A_c the oracle's geometric-factor Poisson
    operator on the order-1 mesh of the same box (assembled); e has zero mean."""
    nel = (4, 3, 2)
    m = _mesh(nel)
    H = OracleHSMG(m)
    mc = OracleMesh(nel, 1)
    rng = np.random.default_rng(5)
    rc = rng.standard_normal(H.nc)
    ec = H.coarse_solve(rc)
    el = _to_local_corners(nel, ec)
    w = mc.dssum(mc.ax(el, 1.0, 0.0))
    want = _to_local_corners(nel, rc - rc.mean())
    assert np.abs(w - want).max() <= 1e-12 * np.abs(rc).max()
    assert abs(ec.sum()) <= 1e-12 * np.abs(ec).max() * H.nc


def test_prolongations_reproduce_polynomials():
    """P_fm is exact for element-wise polynomials of degree <= N_m; P_mc is
    trilinear interpolation of the corner values."""
    nel = (2, 2, 2)
    m = _mesh(nel)
    H = OracleHSMG(m)
    xf, _ = gll(7)
    xm, _ = gll(3)
    E = 8
    rng = np.random.default_rng(7)
    cf = rng.standard_normal((E, 4, 3))     # per element, a cubic per direction (product form)

    def field(nodes, coef):
        lx = len(nodes)
        out = np.zeros((E, lx, lx, lx))
        for e in range(E):
            px = np.polyval(coef[e, :, 0], nodes)
            py = np.polyval(coef[e, :, 1], nodes)
            pz = np.polyval(coef[e, :, 2], nodes)
            out[e] = pz[:, None, None] * py[None, :, None] * px[None, None, :]
        return out.ravel()

    zf = H.prolong_fm(field(xm, cf))
    assert np.abs(zf - field(xf, cf)).max() <= 1e-12 * np.abs(zf).max()

    ec = rng.standard_normal(H.nc)
    zm = H.prolong_mc(ec).reshape(E, 4, 4, 4)
    corners = _to_local_corners(nel, ec).reshape(E, 2, 2, 2)   # [e][c][b][a]
    lo_, hi_ = (1 - xm) / 2, (1 + xm) / 2
    for e in range(E):
        want = np.zeros((4, 4, 4))
        for c in range(2):
            for b in range(2):
                for a in range(2):
                    want += (corners[e, c, b, a] * (lo_, hi_)[c][:, None, None]
                             * (lo_, hi_)[b][None, :, None] * (lo_, hi_)[a][None, None, :])
        assert np.abs(zm[e] - want).max() <= 1e-14 * max(1.0, np.abs(want).max())


def test_restrictions_are_transposes_of_prolongations():
    """<P z, r>_fine = <z, R r>_coarser in the unique-node inner products
    (sum over local points divided by the multiplicity)."""
    nel = (3, 2, 2)
    m = _mesh(nel)
    H = OracleHSMG(m)
    rng = np.random.default_rng(11)
    mult_f = _mult(nel, 8)
    mult_m = _mult(nel, 4)
    assert np.array_equal(mult_f, np.asarray(m.mult(), dtype=float))
    # continuous middle vector: assembled random / mult
    zm = H.restrict_mf(m.dssum(rng.standard_normal(m.np))) / mult_m   # any continuous middle vector
    r = m.dssum(rng.standard_normal(m.np))
    lhs = np.sum(H.prolong_fm(zm) * r / mult_f)
    rhs = np.sum(zm * H.restrict_mf(r) / mult_m)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)
    # middle <-> coarse
    ec = rng.standard_normal(H.nc)
    rm = H.restrict_mf(r)
    lhs = np.sum(H.prolong_mc(ec) * rm / mult_m)
    rhs = np.sum(ec * H.restrict_cm(rm))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)


@pytest.mark.parametrize("level", [0, 1])
def test_smoother_weights_one_element_solution(level):
    """A residual that lives on the interior nodes of one element reaches only
    that element's local solve: the smoother returns that solution divided by
    the multiplicity (1/mult weighting of the summed copies)."""
    nel = (3, 3, 3)
    m = _mesh(nel)
    H = OracleHSMG(m)
    lx = 8 if level == 0 else 4
    n3 = lx ** 3
    E = 27
    e0 = 13                                  # the centre element
    r = np.zeros(E * n3)
    blk = np.zeros((lx, lx, lx))
    blk[1:-1, 1:-1, 1:-1] = np.random.default_rng(2).standard_normal((lx - 2,) * 3)
    r[e0 * n3:(e0 + 1) * n3] = blk.ravel()
    z = H.smooth(level, r)
    u = H.local_solve(level, blk.ravel())
    mult = _mult(nel, lx)[:n3]
    assert np.abs(z[e0 * n3:(e0 + 1) * n3] - u / mult).max() <= 1e-15 * np.abs(u).max()
    # every element that does not touch e0 holds zero
    ex0, ey0, ez0 = 1, 1, 1
    for e in range(E):
        ex, ey, ez = e % 3, (e // 3) % 3, e // 9
        if max(abs(ex - ex0), abs(ey - ey0), abs(ez - ez0)) > 1:
            assert not z[e * n3:(e + 1) * n3].any()


def test_apply_is_linear_and_continuous():
    """GMRES applies M^{-1} to V y at the cycle end, which needs a linear M;
    the output is a continuous field (equal values on all copies of a node)."""
    m = _mesh()
    H = OracleHSMG(m)
    rng = np.random.default_rng(13)
    r1 = m.dssum(rng.standard_normal(m.np))
    r2 = m.dssum(rng.standard_normal(m.np))
    a, b = 0.7, -1.9
    z = H.apply(a * r1 + b * r2)
    assert np.abs(z - (a * H.apply(r1) + b * H.apply(r2))).max() <= 1e-12 * np.abs(z).max()
    mult = np.asarray(m.mult(), dtype=float)
    assert np.abs(m.dssum(z) / mult - z).max() <= 1e-13 * np.abs(z).max()


@pytest.mark.parametrize("nel,N", [((4, 4, 4), 7), ((3, 4, 2), 5), ((2, 2, 2), 11)])
def test_hsmg_gmres_solves_the_same_poisson_problem_in_fewer_steps(nel, N):
    """Same solution as Jacobi-preconditioned GMRES (within the tolerance)
    and several times fewer Arnoldi steps."""
    m = OracleMesh(nel, N)
    H = OracleHSMG(m)
    rng = np.random.default_rng(17)
    b = m.remove_mean_unique(m.dssum(rng.standard_normal(m.np)))
    tol = 1e-9 * np.sqrt(m.glsc(b, b))
    pj, itj, rj = m.poisson(b, tol=tol, maxit=5000)
    ph, ith, rh = H.poisson(b, tol=tol, maxit=5000)
    assert rj <= tol and rh <= tol
    assert np.abs(ph - pj).max() <= 1e-6 * np.abs(pj).max()
    assert ith * 4 <= itj, (ith, itj)


def test_fluid_with_hsmg_matches_jacobi_fluid():
    """Three TGV steps: same kinetic energy and enstrophy as the Jacobi run
    (pressure tolerance 1e-10), fewer pressure iterations."""
    m = OracleMesh((4, 4, 4), 5)
    fj = OracleFluid(m, 1 / 1600, 2e-3, vtol=1e-10, ptol=1e-10, init=INIT_TGV3D)
    fh = OracleFluid(m, 1 / 1600, 2e-3, vtol=1e-10, ptol=1e-10, init=INIT_TGV3D, hsmg=True)
    for _ in range(3):
        sj = fj.step()
        sh = fh.step()
        assert abs(sj["ke"] - sh["ke"]) <= 1e-10 * sj["ke"]
        assert abs(sj["enst"] - sh["enst"]) <= 1e-8 * sj["enst"]
        assert sh["pit"] < sj["pit"]
    assert np.abs(fj.velocity() - fh.velocity()).max() <= 1e-8
