"""Pins of the FP64 CPU oracle against facts fixed by mathematics and the paper.

None of these re-types an oracle formula: each check uses an independent
construction (numpy's Legendre/polynomial routines, coordinate-based node
identification, dense linear algebra, closed-form solutions derived by hand)
so that a dropped term, sign, index or transposed operand in the oracle fails
at least one of them.
"""
import math

import numpy as np
import pytest

from oracle import OracleMesh, OracleFluid, OracleProjection, gll, gl, lxd, interp_matrix, deriv_matrix, e_max, e_peak, e_series
from oracle.oracle import INIT_TGV2D, INIT_TGV3D
from paper_2608_24348_amd import inputs

PI = math.pi


# ---------------------------------------------------------------- GLL tables
@pytest.mark.parametrize("N,xi_ref,w_ref", [
    (2, [-1.0, 0.0, 1.0], [1 / 3, 4 / 3, 1 / 3]),
    (3, [-1.0, -1 / math.sqrt(5), 1 / math.sqrt(5), 1.0], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    (4, [-1.0, -math.sqrt(3 / 7), 0.0, math.sqrt(3 / 7), 1.0], [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
])
def test_gll_closed_forms(N, xi_ref, w_ref):
    xi, w = gll(N)
    assert np.allclose(xi, xi_ref, atol=1e-15, rtol=0)
    assert np.allclose(w, w_ref, atol=1e-15, rtol=0)


@pytest.mark.parametrize("N", range(1, 16))
def test_gll_nodes_are_legendre_derivative_roots(N):
    xi, w = gll(N)
    assert abs(w.sum() - 2.0) < 1e-14
    if N >= 2:
        roots = np.sort(np.polynomial.legendre.Legendre.basis(N).deriv().roots().real)
        assert np.allclose(xi[1:-1], roots, atol=1e-13, rtol=0)
    assert xi[0] == -1.0 and xi[-1] == 1.0


@pytest.mark.parametrize("N", range(1, 16))
def test_gll_quadrature_exact_to_degree_2N_minus_1(N):
    xi, w = gll(N)
    for k in range(0, 2 * N):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, xi ** k) - exact) < 1e-14 * max(1.0, 2 ** (k / 8))


@pytest.mark.parametrize("N", range(1, 16))
def test_derivative_matrix_exact_on_polynomials(N):
    xi, _ = gll(N)
    D = deriv_matrix(N)
    nrm = np.abs(D).max()
    assert np.abs(D.sum(axis=1)).max() < 1e-13 * nrm
    for k in range(1, N + 1):
        assert np.abs(D @ xi ** k - k * xi ** (k - 1)).max() < 1e-13 * nrm * k


def _lagrange_deriv_numpy(x):
    """Independent D from numpy polynomial algebra: D[i, j] = l_j'(x_i)."""
    n = len(x)
    P = np.polynomial.polynomial
    D = np.zeros((n, n))
    for j in range(n):
        others = np.delete(x, j)
        c = P.polyfromroots(others) / np.prod(x[j] - others)
        D[:, j] = P.polyval(x, P.polyder(c))
    return D


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7])
def test_derivative_matrix_vs_numpy_lagrange(N):
    xi, _ = gll(N)
    assert np.allclose(deriv_matrix(N), _lagrange_deriv_numpy(xi), atol=1e-11, rtol=0)


# ---------------------------------------------------------------- mesh / dssum
def _unique_ids_from_coords(X, L=2 * PI):
    """Identify periodic unique nodes from coordinates (independent of any gid formula)."""
    keys = []
    for c in range(3):
        xm = np.mod(X[c] + PI, L)
        xm[np.abs(xm - L) < 1e-8] = 0.0
        keys.append(np.round(xm * 1e6).astype(np.int64))
    k = np.stack(keys, axis=1)
    _, inv = np.unique(k, axis=0, return_inverse=True)
    return inv.ravel()


@pytest.mark.parametrize("nel,N", [((2, 2, 2), 3), ((3, 2, 4), 2), ((2, 2, 2), 5), ((1, 2, 2), 3)])
def test_dssum_is_dense_QQt(nel, N):
    m = OracleMesh(nel, N)
    uid = _unique_ids_from_coords(m.coords())
    nu = uid.max() + 1
    assert nu == m.nglob == nel[0] * nel[1] * nel[2] * N ** 3
    Q = np.zeros((m.np, nu))
    Q[np.arange(m.np), uid] = 1.0
    u = np.random.default_rng(3).standard_normal(m.np)
    assert np.allclose(m.dssum(u), Q @ (Q.T @ u), atol=1e-13, rtol=0)
    mult = m.dssum(np.ones(m.np))
    assert set(np.unique(mult)) <= {1.0, 2.0, 4.0, 8.0}
    assert np.array_equal(mult, m.mult())
    E = nel[0] * nel[1] * nel[2]
    assert np.count_nonzero(mult == 1.0) == E * (N - 1) ** 3


def test_affine_geometry_closed_form():
    n, N = 4, 5
    m = OracleMesh((n, n, n), N)
    h = 2 * PI / n
    _, w, _ = m.tables()
    w3 = np.einsum("k,j,i->kji", w, w, w).ravel()
    jac = m.jac()
    # D applied to coordinates of size pi loses about |D| pi eps relative to h/2
    assert np.allclose(jac, (h / 2) ** 3, rtol=1e-13, atol=0)
    B = m.mass().reshape(-1, (N + 1) ** 3)
    assert np.allclose(B, (h / 2) ** 3 * w3[None, :], rtol=1e-13, atol=0)
    G = m.G().reshape(6, -1, (N + 1) ** 3)
    for q, diag in enumerate([True, False, False, True, False, True]):
        ref = (h / 2) ** 3 * (2 / h) ** 2 * w3 if diag else 0.0 * w3
        assert np.allclose(G[q], ref[None, :], rtol=1e-13, atol=1e-15)
    assert abs(m.vol - (2 * PI) ** 3) < 1e-13 * (2 * PI) ** 3


@pytest.mark.parametrize("amp", [0.0, 0.1])
def test_gradient_of_coordinates_is_identity(amp):
    ph = inputs.deform_phases()
    m = OracleMesh((4, 4, 4), 5, amp=amp, phase=ph)
    X = m.coords()
    B = m.mass()
    assert np.all(m.jac() > 0)
    for c in range(3):
        g = m.grad(X[c])
        og = m.opgrad(X[c])
        for d in range(3):
            ref = 1.0 if c == d else 0.0
            assert np.abs(g[d] - ref).max() < 1e-12
            assert np.abs(og[d] - ref * B).max() < 1e-12 * B.max()


def test_deformed_mesh_is_perturbed_and_periodic():
    ph = inputs.deform_phases()
    m = OracleMesh((4, 4, 4), 5, amp=0.1, phase=ph)
    m0 = OracleMesh((4, 4, 4), 5)
    d = np.abs(m.coords() - m0.coords()).max()
    h = 2 * PI / 4
    assert 0.02 * h < d <= 0.1 * h + 1e-12
    # the perturbed mesh still has the periodic unique-node structure
    uid = _unique_ids_from_coords(m.coords())
    assert uid.max() + 1 == m.nglob
    assert abs(m.vol - (2 * PI) ** 3) < 1e-3 * (2 * PI) ** 3


# ---------------------------------------------------------------- Ax
def _dense_element_stiffness(N, h):
    """(h/2)^3 (2/h)^2 [K1 x W x W + W x K1 x W + W x W x K1] via numpy Lagrange algebra."""
    x = np.sort(np.concatenate([[-1.0, 1.0], np.polynomial.legendre.Legendre.basis(N).deriv().roots().real]))
    D = _lagrange_deriv_numpy(x)
    # GLL weights by exactness on monomials (Vandermonde solve), independent of the L_N formula
    V = np.vander(x, increasing=True).T
    mom = np.array([0.0 if k % 2 else 2.0 / (k + 1) for k in range(N + 1)])
    w = np.linalg.solve(V, mom)
    W = np.diag(w)
    K1 = D.T @ W @ D
    s = (h / 2) ** 3 * (2 / h) ** 2
    # point index i + lx (j + lx k): k slowest
    return s * (np.kron(W, np.kron(W, K1)) + np.kron(W, np.kron(K1, W)) + np.kron(K1, np.kron(W, W)))


@pytest.mark.parametrize("N", [2, 3, 4])
def test_ax_affine_equals_dense_kronecker_assembly(N):
    n = 2
    m = OracleMesh((n, n, n), N)
    uid = _unique_ids_from_coords(m.coords())
    Ke = _dense_element_stiffness(N, 2 * PI / n)
    n3 = (N + 1) ** 3
    Aglob = np.zeros((m.nglob, m.nglob))
    for e in range(m.E):
        ids = uid[e * n3:(e + 1) * n3]
        Aglob[np.ix_(ids, ids)] += Ke
    y = np.random.default_rng(5).standard_normal(m.nglob)
    u = y[uid]
    w = m.dssum(m.ax(u))
    assert np.allclose(w, (Aglob @ y)[uid], atol=1e-13 * np.abs(Aglob).max() * np.abs(y).max() * n3, rtol=0)
    # local (unassembled) operator is the block diagonal
    ul = np.random.default_rng(6).standard_normal(m.np)
    wl = m.ax(ul)
    for e in range(m.E):
        assert np.allclose(wl[e * n3:(e + 1) * n3], Ke @ ul[e * n3:(e + 1) * n3], atol=1e-12, rtol=0)


@pytest.mark.parametrize("amp", [0.0, 0.1])
def test_ax_symmetry_nullspace_psd(amp):
    m = OracleMesh((4, 4, 4), 6, amp=amp, phase=inputs.deform_phases())
    rng = np.random.default_rng(11)
    u = rng.standard_normal(m.np)
    v = rng.standard_normal(m.np)
    Au, Av = m.ax(u), m.ax(v)
    anorm = np.abs(Au).max() / np.abs(u).max()
    assert abs(v @ Au - u @ Av) <= 1e-13 * np.linalg.norm(u) * np.linalg.norm(v) * anorm * 10
    assert u @ Au >= 0 and v @ Av >= 0
    assert np.abs(m.ax(np.ones(m.np))).max() < 1e-12 * anorm
    # Helmholtz: h2 B part is exactly the mass matrix
    B = m.mass()
    assert np.allclose(m.ax(u, 0.0, 2.5), 2.5 * B * u, rtol=1e-15, atol=0)


def test_ax_energy_of_sine_is_spectral():
    m = OracleMesh((8, 8, 8), 7)
    X = m.coords()
    u = np.sin(X[0])
    # int |grad sin x|^2 over the periodic box = (2 pi)^2 * pi = 4 pi^3
    assert abs(u @ m.ax(u) - 4 * PI ** 3) < 1e-9 * 4 * PI ** 3


def test_jacobi_diagonal_is_operator_diagonal():
    m = OracleMesh((2, 2, 2), 3, amp=0.1, phase=inputs.deform_phases())
    d = m.diag(0.7, 3.0)
    n3 = 4 ** 3
    # brute force: local operator applied to unit vectors of element 0 and 5
    for e in (0, 5):
        for q in range(n3):
            ev = np.zeros(m.np)
            ev[e * n3 + q] = 1.0
            assert abs(m.ax(ev, 0.7, 3.0)[e * n3 + q] - d[e * n3 + q]) < 1e-13 * abs(d[e * n3 + q])


# ---------------------------------------------------------------- SEM operators
def test_wdiv_is_adjoint_of_opgrad():
    m = OracleMesh((4, 4, 4), 5, amp=0.1, phase=inputs.deform_phases())
    rng = np.random.default_rng(12)
    p = rng.standard_normal(m.np)
    v = rng.standard_normal((3, m.np))
    lhs = p @ m.wdiv(v)
    rhs = np.sum(m.opgrad(p) * v)
    assert abs(lhs - rhs) < 1e-12 * np.abs(lhs)
    assert abs(m.wdiv(v).sum()) < 1e-11 * np.abs(m.wdiv(v)).sum()


def _tgv3d(X):
    x, y, z = X
    return np.stack([np.sin(x) * np.cos(y) * np.cos(z), -np.cos(x) * np.sin(y) * np.cos(z), 0 * x])


def test_convection_of_tgv_closed_form():
    m = OracleMesh((8, 8, 8), 7)
    X = m.coords()
    u = _tgv3d(X)
    B = m.mass()
    bn = m.conv(u)
    x, y, z = X
    # (u . grad) u for the TGV initial field, derived by hand
    ref = np.stack([0.5 * np.sin(2 * x) * np.cos(z) ** 2, 0.5 * np.sin(2 * y) * np.cos(z) ** 2, 0 * x])
    assert np.abs(bn / B + ref).max() < 1e-6


def test_tgv3d_initial_invariants():
    m = OracleMesh((8, 8, 8), 7)
    X = m.coords()
    u = _tgv3d(X)
    ke, en, md = m.diagnostics(u)
    assert abs(ke - 1 / 8) < 1e-12
    assert abs(en - 3 / 8) < 1e-9
    assert md < 1e-6
    w, dv = m.curl_div(u)
    x, y, z = X
    wref = np.stack([-np.cos(x) * np.sin(y) * np.sin(z), -np.sin(x) * np.cos(y) * np.sin(z),
                     2 * np.sin(x) * np.sin(y) * np.cos(z)])
    assert np.abs(w - wref).max() < 1e-6


def test_tgv3d_initial_pressure_solves_pressure_poisson():
    # -lap p = div((u.grad)u)  <=>  A p = wdiv(N(u)) with N = -(u.grad)u
    m = OracleMesh((8, 8, 8), 7)
    X = m.coords()
    u = _tgv3d(X)
    nvec = m.conv(u) / m.mass()
    rhs = m.dssum(m.wdiv(nvec))
    p, it, res = m.poisson(rhs, tol=1e-10, maxit=3000)
    x, y, z = X
    pex = (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2) / 16
    assert abs(m.sum(m.mass() * pex)) < 1e-12
    assert np.abs(p - pex).max() < 1e-6


# ---------------------------------------------------------------- Krylov
def _assembled_dense(m, h1, h2):
    uid = _unique_ids_from_coords(m.coords())
    A = np.zeros((m.nglob, m.nglob))
    for g in range(m.nglob):
        y = np.zeros(m.nglob)
        y[g] = 1.0
        w = m.ax(y[uid], h1, h2)
        col = np.zeros(m.nglob)
        np.add.at(col, uid, w)
        A[:, g] = col
    return A, uid


def test_pcg_matches_dense_solve():
    m = OracleMesh((2, 2, 2), 3, amp=0.1, phase=inputs.deform_phases())
    A, uid = _assembled_dense(m, 0.3, 40.0)
    assert np.allclose(A, A.T, atol=1e-12 * np.abs(A).max())
    y = np.random.default_rng(7).standard_normal(m.nglob)
    x, it, res = m.pcg(y[uid], 0.3, 40.0, tol=1e-13, maxit=500)
    ref = np.linalg.solve(A, y)
    assert res <= 1e-13 and it > 0
    assert np.abs(x - ref[uid]).max() < 1e-10 * np.abs(ref).max()


def test_gmres_matches_dense_solve_nonsingular_and_singular():
    m = OracleMesh((2, 2, 2), 3, amp=0.1, phase=inputs.deform_phases())
    A, uid = _assembled_dense(m, 0.3, 40.0)
    y = np.random.default_rng(8).standard_normal(m.nglob)
    x, it, res = m.gmres(y[uid], 0.3, 40.0, tol=1e-12, maxit=2000, restart=10)
    assert res <= 1e-12
    assert np.abs(x - np.linalg.solve(A, y)[uid]).max() < 1e-10
    # singular periodic Poisson: consistent rhs, compare the unique-mean-free parts
    A0, _ = _assembled_dense(m, 1.0, 0.0)
    y0 = y - y.mean()
    ref, *_ = np.linalg.lstsq(A0, y0, rcond=None)
    ref -= ref.mean()
    x0, it0, res0 = m.gmres(y0[uid], 1.0, 0.0, tol=1e-12, maxit=3000, restart=30)
    got = x0 - m.glsc(x0, np.ones(m.np)) / m.nglob
    assert np.abs(got - ref[uid]).max() < 1e-9 * np.abs(ref).max()


def test_element_subset_mesh_reproduces_full_mesh_elements():
    nel, N = (4, 4, 4), 5
    ph = inputs.deform_phases()
    full = OracleMesh(nel, N, amp=0.1, phase=ph)
    els = [0, 5, 17, 63, 40]
    sub = OracleMesh(nel, N, amp=0.1, phase=ph, elements=els)
    n3 = (N + 1) ** 3
    pick = np.concatenate([np.arange(e * n3, (e + 1) * n3) for e in els])
    assert np.array_equal(sub.coords(), full.coords()[:, pick])
    assert np.array_equal(sub.G(), full.G()[:, pick]) and np.array_equal(sub.mass(), full.mass()[pick])
    u = np.random.default_rng(9).standard_normal(full.np)
    assert np.array_equal(sub.ax(u[pick], 0.3, 7.0), full.ax(u, 0.3, 7.0)[pick])
    v = np.random.default_rng(10).standard_normal((3, full.np))
    assert np.array_equal(sub.conv(v[:, pick]), full.conv(v)[:, pick])


# ---------------------------------------------------------------- dealiased convection
@pytest.mark.parametrize("n", list(range(1, 25)))
def test_gauss_legendre_matches_numpy(n):
    z, w = gl(n)
    zr, wr = np.polynomial.legendre.leggauss(n)
    assert np.allclose(z, zr, atol=1e-14, rtol=0) and np.allclose(w, wr, atol=1e-14, rtol=0)


def test_dealias_grid_and_interpolation_matrix():
    assert [lxd(lx) for lx in (4, 6, 8, 10, 12)] == [6, 9, 12, 15, 18]
    for N in (3, 5, 7):
        xi, _ = gll(N)
        z, _ = gl(lxd(N + 1))
        I = interp_matrix(xi, z)
        P = np.polynomial.polynomial
        for l in range(N + 1):
            others = np.delete(xi, l)
            c = P.polyfromroots(others) / np.prod(xi[l] - others)
            assert np.allclose(I[:, l], P.polyval(z, c), atol=1e-13, rtol=0)
        # interpolation reproduces polynomials of degree <= N
        for k in range(N + 1):
            assert np.allclose(I @ xi ** k, z ** k, atol=1e-13, rtol=0)


def _lagrange_polys(xi):
    P = np.polynomial.polynomial
    out = []
    for l in range(len(xi)):
        others = np.delete(xi, l)
        out.append(P.polyfromroots(others) / np.prod(xi[l] - others))
    return out


def _brute_dealias(m, u, nq):
    """-sum_q W_q phi(z_q) u.grad u on an nq^3 Gauss-Legendre rule per element, by
    numpy polynomial evaluation of the nodal fields and of the coordinates."""
    P = np.polynomial.polynomial
    xi, _, _ = m.tables()
    lx = m.lx
    z, wq = np.polynomial.legendre.leggauss(nq)
    polys = _lagrange_polys(xi)
    V = np.stack([P.polyval(z, c) for c in polys], axis=1)               # (nq, lx)
    dV = np.stack([P.polyval(z, P.polyder(c)) for c in polys], axis=1)   # (nq, lx)
    X = m.coords()
    n3 = lx ** 3
    out = np.zeros((3, m.np))
    for e in range(m.E):
        sl = slice(e * n3, (e + 1) * n3)
        xe = X[:, sl].reshape(3, lx, lx, lx)      # [c][k][j][i]
        ue = u[:, sl].reshape(3, lx, lx, lx)

        def ev(f, A, B, Cm):  # A along i, B along j, Cm along k
            return np.einsum("ai,bj,ck,kji->cba", A, B, Cm, f)
        J = np.zeros((nq, nq, nq, 3, 3))
        for c in range(3):
            J[..., c, 0] = ev(xe[c], dV, V, V)
            J[..., c, 1] = ev(xe[c], V, dV, V)
            J[..., c, 2] = ev(xe[c], V, V, dV)
        jac = np.linalg.det(J)
        rx = np.linalg.inv(J)                       # [.., a, c] = d r_a / d x_c
        W = jac * np.einsum("k,j,i->kji", wq, wq, wq)
        uf = np.stack([ev(ue[c], V, V, V) for c in range(3)])
        for f in range(3):
            g = np.stack([ev(ue[f], dV, V, V), ev(ue[f], V, dV, V), ev(ue[f], V, V, dV)], axis=-1)
            dx = np.einsum("...ac,...a->...c", rx, g)
            T = W * np.einsum("c...,...c->...", uf, dx)
            # test against every GLL basis function: sum_q phi_l(z_q) T_q
            o = np.einsum("ai,bj,ck,cba->kji", V, V, V, T)
            out[f, sl] = -o.ravel()
    return out


def test_dealiased_convection_is_exact_galerkin_on_affine_elements():
    # affine, non-cubic elements: the integrand has degree 3N-1 per direction,
    # integrated exactly by the 3/2 rule and by any finer rule
    N = 4
    m = OracleMesh((2, 2, 2), N, lo=(-1.0, -2.0, 0.5), hi=(2.0, 1.0, 3.0))
    u = np.random.default_rng(21).standard_normal((3, m.np))
    got = m.conv_dealias(u)
    ref = _brute_dealias(m, u, 2 * (N + 1) + 2)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


def test_dealiased_convection_matches_same_rule_brute_force_on_curved_elements():
    N = 3
    m = OracleMesh((2, 2, 2), N, amp=0.1, phase=inputs.deform_phases())
    u = np.random.default_rng(22).standard_normal((3, m.np))
    got = m.conv_dealias(u)
    ref = _brute_dealias(m, u, lxd(N + 1))
    assert np.abs(got - ref).max() < 1e-11 * np.abs(ref).max()


def test_dealiased_and_collocated_convection_agree_on_smooth_fields():
    # both converge to the continuous B u.grad u for the smooth TGV field
    diffs = []
    for N in (5, 7, 9):
        m = OracleMesh((4, 4, 4), N)
        X = m.coords()
        u = np.stack([np.sin(X[0]) * np.cos(X[1]) * np.cos(X[2]), -np.cos(X[0]) * np.sin(X[1]) * np.cos(X[2]),
                      0 * X[0]])
        a, b = m.conv_dealias(u), m.conv(u)
        diffs.append(np.abs(a - b).max() / np.abs(b).max())
    assert diffs[1] < diffs[0] / 10 and diffs[2] < diffs[1] / 10


# ---------------------------------------------------------------- pressure projection
def _unique(loc, uid, n):
    u = np.zeros(n)
    u[uid] = loc
    return u


def test_projection_space_is_A_orthonormal_and_guess_is_A_optimal():
    m = OracleMesh((2, 2, 2), 3, amp=0.1, phase=inputs.deform_phases())
    A, uid = _assembled_dense(m, 1.0, 0.0)
    P = OracleProjection(m, dim=3)
    rng = np.random.default_rng(11)
    sizes = []
    for _ in range(5):
        y = rng.standard_normal(m.nglob)
        y -= y.mean()
        p, it, res = P.poisson(y[uid], tol=1e-12, maxit=3000)
        assert res <= 1e-12
        # the solution is that of the dense singular system (zero-mean parts)
        ref, *_ = np.linalg.lstsq(A, y, rcond=None)
        got = _unique(p, uid, m.nglob)
        assert np.abs((got - got.mean()) - (ref - ref.mean())).max() < 1e-9 * np.abs(ref).max()
        sizes.append(P.size)
    # one direction per solve; a full space restarts from the latest solution
    assert sizes == [1, 2, 3, 1, 2]
    X = np.stack([_unique(P.vector(i), uid, m.nglob) for i in range(P.size)])
    assert np.abs(X @ A @ X.T - np.eye(P.size)).max() < 1e-9
    # the guess is the A-norm best approximation in span X: its residual is
    # orthogonal to the space (Galerkin condition), checked with the dense A
    y = rng.standard_normal(m.nglob)
    y -= y.mean()
    xbar = _unique(P.guess(y[uid]), uid, m.nglob)
    r = y - A @ xbar
    assert np.abs(X @ r).max() < 1e-10 * np.abs(y).max()
    # a rhs inside the space is reproduced exactly by the guess
    b_in = A @ (0.7 * X[0] - 1.3 * X[1])
    xg = _unique(P.guess(b_in[uid]), uid, m.nglob)
    assert np.abs(A @ xg - b_in).max() < 1e-9 * np.abs(b_in).max()


def test_projection_repeated_rhs_needs_no_iterations():
    m = OracleMesh((4, 4, 4), 5)
    X = m.coords()
    s = np.sin(X[0]) * np.sin(X[1]) * np.sin(X[2])
    b = m.dssum(m.mass() * 3 * s)
    P = OracleProjection(m, dim=20)
    p1, it1, res1 = P.poisson(b, tol=1e-10, maxit=5000)
    p2, it2, res2 = P.poisson(b, tol=1e-10, maxit=5000)
    assert it1 > 0 and it2 == 0 and res2 <= 1e-10
    assert np.abs(p2 - p1).max() < 1e-9
    # without projection the plain solver gives the same answer
    p0, it0, _ = m.poisson(b, tol=1e-10, maxit=5000)
    assert it0 == it1 and np.abs(p0 - p1).max() < 1e-9


def test_fluid_with_projection_matches_plain_solver():
    nu, dt = 1 / 1600, 1e-3
    m = OracleMesh((4, 4, 4), 5)
    f0 = OracleFluid(m, nu, dt, init=INIT_TGV3D)
    f1 = OracleFluid(m, nu, dt, init=INIT_TGV3D, proj=20)
    it0 = it1 = 0
    for _ in range(8):
        a, b = f0.step(), f1.step()
        it0 += a["pit"]
        it1 += b["pit"]
        assert b["pres"] <= 1e-8
        assert abs(a["ke"] - b["ke"]) <= 1e-10 * a["ke"]
        assert abs(a["enst"] - b["enst"]) <= 1e-8 * a["enst"]
    assert f1.proj_size > 0
    # projection onto earlier increments cuts the pressure iterations
    assert it1 < it0


def test_poisson_spectral_convergence():
    errs = []
    for N in (3, 5, 7, 9):
        m = OracleMesh((4, 4, 4), N)
        X = m.coords()
        s = np.sin(X[0]) * np.sin(X[1]) * np.sin(X[2])
        p, it, res = m.poisson(m.dssum(m.mass() * 3 * s), tol=1e-11, maxit=5000)
        errs.append(np.abs(p - s).max())
    # at least 10x per +2 in order until the solver floor
    for a, b in zip(errs[:-1], errs[1:]):
        assert b < a / 10 or b < 1e-10
    assert errs[-1] < 1e-10


# ---------------------------------------------------------------- fluid step
def test_tgv2d_extruded_decays_exactly():
    nu, dt, nsteps = 0.05, 1e-3, 100
    m = OracleMesh((4, 4, 2), 7)
    f = OracleFluid(m, nu, dt, init=INIT_TGV2D)
    for _ in range(nsteps):
        st = f.step()
    X = m.coords()
    t = f.time
    assert abs(t - nsteps * dt) < 1e-12
    u = f.velocity()
    decay = math.exp(-2 * nu * t)
    ue = np.stack([np.sin(X[0]) * np.cos(X[1]) * decay, -np.cos(X[0]) * np.sin(X[1]) * decay])
    assert np.abs(u[:2] - ue).max() < 1e-6
    assert np.abs(u[2]).max() < 1e-10
    pe = (np.cos(2 * X[0]) + np.cos(2 * X[1])) / 4 * math.exp(-4 * nu * t)
    assert np.abs(f.pressure() - pe).max() < 1e-5
    # KE0 = 1/4 decaying as exp(-2 nu t) squared
    assert abs(st["ke"] - 0.25 * decay ** 2) < 1e-8


def test_tgv2d_extruded_decays_exactly_with_dealiased_convection():
    nu, dt, nsteps = 0.05, 1e-3, 50
    m = OracleMesh((4, 4, 2), 7)
    f = OracleFluid(m, nu, dt, init=INIT_TGV2D, dealias=True)
    for _ in range(nsteps):
        st = f.step()
    X = m.coords()
    decay = math.exp(-2 * nu * f.time)
    ue = np.stack([np.sin(X[0]) * np.cos(X[1]) * decay, -np.cos(X[0]) * np.sin(X[1]) * decay])
    u = f.velocity()
    assert np.abs(u[:2] - ue).max() < 1e-6 and np.abs(u[2]).max() < 1e-10
    assert abs(st["ke"] - 0.25 * decay ** 2) < 1e-8


def test_tgv3d_energy_budget():
    nu, dt = 1 / 1600, 1e-3
    m = OracleMesh((8, 8, 8), 7)
    f = OracleFluid(m, nu, dt, init=INIT_TGV3D)
    ke = [m.diagnostics(f.velocity())[0]]
    en = [m.diagnostics(f.velocity())[1]]
    for _ in range(6):
        st = f.step()
        ke.append(st["ke"])
        en.append(st["enst"])
        assert max(st["vit"]) < 50 and st["pres"] <= 1e-8 and max(st["vres"]) <= 1e-8
    ke, en = np.array(ke), np.array(en)
    # dE/dt = -2 nu Omega for periodic incompressible flow (central differences)
    for n in range(2, 6):
        dedt = (ke[n + 1] - ke[n - 1]) / (2 * dt)
        assert abs(dedt + 2 * nu * en[n]) < 0.01 * 2 * nu * en[n]


# ---------------------------------------------------------------- metrics
def test_error_metrics_hand_example():
    ref = np.array([1.0, 2.0, 4.0, 3.0])
    mxp = np.array([1.0, 2.2, 3.6, 3.0])
    assert np.allclose(e_series(mxp, ref), [0.0, 5.0, 10.0, 0.0])
    assert abs(e_max(mxp, ref) - 10.0) < 1e-12
    # peak: |3.6 - 4.0| / 4 * 100
    assert abs(e_peak(mxp, ref) - 10.0) < 1e-12
    assert e_max(ref, ref) == 0.0 and e_peak(ref, ref) == 0.0


def test_poisson_manufactured_on_deformed_mesh():
    # exercises every cross term G_ab of the curved geometry
    errs = []
    for N in (5, 7):
        m = OracleMesh((4, 4, 4), N, amp=0.1, phase=inputs.deform_phases())
        X = m.coords()
        s = np.sin(X[0]) * np.sin(X[1]) * np.sin(X[2])
        p, it, res = m.poisson(m.dssum(m.mass() * 3 * s), tol=1e-11, maxit=5000)
        # the manufactured solution has zero mean only up to quadrature error on a curved mesh
        errs.append(np.abs(p - m.remove_mean_mass(s)).max())
    # curved elements: GLL quadrature of the mapped integrands converges spectrally too
    assert errs[1] < errs[0] / 10 and errs[1] < 2e-4


# ---------------------------------------------------------------- adaptive time stepping (Sec. 3: target CFL 0.4)
def test_variable_step_bdf_ext_reduce_to_the_constant_step_schemes():
    from oracle import bdf_ext_var
    want = {1: (1.0, [1, 0, 0], [1, 0, 0]), 2: (1.5, [2, -0.5, 0], [2, -1, 0]),
            3: (11 / 6, [3, -1.5, 1 / 3], [3, -3, 1])}
    for k, (b0, b, a) in want.items():
        for h in (1e-3, 0.25):
            g0, gb, ga = bdf_ext_var(k, (h, h, h))
            assert abs(g0 - b0) < 1e-14 and np.allclose(gb, b, atol=1e-14) and np.allclose(ga, a, atol=1e-14)


def test_variable_step_bdf_ext_are_exact_on_polynomials():
    """BDF-k differentiates polynomials of degree <= k exactly at t_{n+1} and
    EXT-k extrapolates degree <= k-1 exactly, for any step sizes; one degree
    more is not exact (the order is k, not higher)."""
    from oracle import bdf_ext_var
    rng = np.random.default_rng(31)
    for _ in range(20):
        h = rng.uniform(0.5, 1.5, 3) * 0.01
        T = rng.uniform(-1, 1)
        tau = [T, T - h[0], T - h[0] - h[1], T - h[0] - h[1] - h[2]]
        for k in (1, 2, 3):
            b0, b, a = bdf_ext_var(k, h)
            for d in range(k + 2):
                p = lambda t: (t - 0.3) ** d
                dp = d * (T - 0.3) ** (d - 1) if d else 0.0
                approx = (b0 * p(tau[0]) - sum(b[j] * p(tau[j + 1]) for j in range(k))) / h[0]
                ext = sum(a[j] * p(tau[j + 1]) for j in range(k))
                if d <= k:
                    assert abs(approx - dp) < 1e-8 * (1 + abs(dp)), (k, d)
                else:
                    assert abs(approx - dp) > 1e-12
                if d <= k - 1:
                    assert abs(ext - p(T)) < 1e-10 * (1 + abs(p(T))), (k, d)


def test_cfl_rate_matches_the_affine_closed_form():
    """On affine elements dr_a/dx_c = 2/h_a delta_ac, so the rate at a node is
    sum_a |u_a| (2/h_a) / dr(i_a) with the GLL spacing dr."""
    N = 5
    m = OracleMesh((2, 3, 2), N, lo=(-1.0, 0.0, 0.5), hi=(2.0, 1.5, 2.5))
    X = m.coords()
    u = np.stack([np.sin(X[0]) * np.cos(X[1]), -np.cos(X[0]) * np.sin(X[1]) + 0.3, np.sin(X[2])])
    xi, _ = gll(N)
    dr = np.array([xi[1] - xi[0]] + [0.5 * (xi[i + 1] - xi[i - 1]) for i in range(1, N)] + [xi[N] - xi[N - 1]])
    hs = np.array([3.0 / 2, 1.5 / 3, 2.0 / 2])
    lx = N + 1
    idx = np.arange(m.np) % lx ** 3
    ii = [idx % lx, (idx // lx) % lx, idx // lx ** 2]
    rate = sum(np.abs(u[a]) * (2 / hs[a]) / dr[ii[a]] for a in range(3))
    assert abs(m.cfl_rate(u) - rate.max()) < 1e-12 * rate.max()


def test_adaptive_dt_follows_the_controller_and_keeps_the_2d_tgv_exact_decay():
    nu, dtmax, target = 0.05, 0.1, 0.4
    m = OracleMesh((4, 4, 2), 7)
    f = OracleFluid(m, nu, dtmax, init=INIT_TGV2D, cfl=target)
    rate0 = m.cfl_rate(f.velocity())
    sts = [f.step() for _ in range(25)]
    dts = [s["dt"] for s in sts]
    assert abs(dts[0] - min(dtmax, target / rate0)) < 1e-15 * dts[0]
    for p, q in zip(dts, dts[1:]):
        assert 0.5 * p * (1 - 1e-15) <= q <= 1.1 * p * (1 + 1e-15) and q <= dtmax
    assert all(s["cfl"] <= target * (1 + 1e-12) for s in sts)
    # the decaying field's CFL rate falls, so the step grows toward the target
    assert dts[-1] > dts[0] and abs(sts[-1]["cfl"] - target) < 1e-12
    assert abs(sts[-1]["t"] - sum(dts)) < 1e-13
    X = m.coords()
    decay = math.exp(-2 * nu * f.time)
    ue = np.stack([np.sin(X[0]) * np.cos(X[1]) * decay, -np.cos(X[0]) * np.sin(X[1]) * decay])
    u = f.velocity()
    assert np.abs(u[:2] - ue).max() < 5e-5 and np.abs(u[2]).max() < 1e-8


# ---------------------------------------------------------------- collocated convection on curved elements
def _gll_numpy(N):
    """GLL nodes from numpy's Legendre roots and weights from their closed form
    w_i = 2 / (N (N + 1) L_N(x_i)^2) (independent of the oracle's tables)."""
    Leg = np.polynomial.legendre.Legendre
    x = np.concatenate([[-1.0], np.sort(Leg.basis(N).deriv().roots().real), [1.0]])
    w = 2.0 / (N * (N + 1) * Leg.basis(N)(x) ** 2)
    return x, w


def _brute_force_conv(X, U, N):
    """-B (u . grad) u per local point from first principles: numpy Lagrange
    differentiation of the element-local coordinates and fields along each
    reference direction, the Jacobian matrix inverted point by point with
    numpy.linalg, and B = det(J) w_i w_j w_k."""
    lx = N + 1
    x, w = _gll_numpy(N)
    D = _lagrange_deriv_numpy(x)
    E = X.shape[1] // lx ** 3
    Xe = X.reshape(3, E, lx, lx, lx)          # [c][e][k][j][i]
    Ue = U.reshape(3, E, lx, lx, lx)

    def dref(f):
        # derivatives along r (i axis), s (j axis), t (k axis)
        return np.stack([np.einsum("il,...kjl->...kji", D, f), np.einsum("jl,...kli->...kji", D, f),
                         np.einsum("kl,...lji->...kji", D, f)])

    dX = dref(Xe)                             # [a][c][e][k][j][i] = dx_c / dr_a
    J = np.moveaxis(dX, (0, 1), (-1, -2))     # [e][k][j][i][c][a]
    Jinv = np.linalg.inv(J)                   # [..][a][c] = dr_a / dx_c
    jac = np.linalg.det(J)
    W = np.einsum("k,j,i->kji", w, w, w)
    B = jac * W[None]
    dU = dref(Ue)                             # [a][f][e][k][j][i]
    out = np.zeros_like(Ue)
    for f in range(3):
        for c in range(3):
            gfc = sum(dU[a, f] * Jinv[..., a, c] for a in range(3))   # du_f / dx_c
            out[f] -= Ue[c] * gfc
    return (B[None] * out).reshape(3, -1)


def test_collocated_convection_of_linear_field_on_curved_elements():
    """On isoparametric elements a field linear in x is represented exactly,
    its gradient is the constant matrix A, so -B (u . grad) u = -B (A u) at
    every node to rounding, whatever the metric terms look like.  M is full
    on the deformed mesh, so an index or transposition slip in the metric
    contraction fails this."""
    N = 6
    m = OracleMesh((4, 4, 4), N, amp=0.1, phase=inputs.deform_phases())
    X = m.coords()
    B = m.mass()
    rng = np.random.default_rng(41)
    for trial in range(4):
        A = rng.standard_normal((3, 3))
        b = rng.standard_normal(3)
        u = np.einsum("ic,cp->ip", A, X) + b[:, None]
        ref = -B[None] * np.einsum("ic,cp->ip", A, u)
        got = np.stack(m.conv(u))
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), (trial, np.abs(got - ref).max())


def test_collocated_convection_matches_numpy_brute_force_on_curved_elements():
    """A quadratic field on the deformed mesh (not exact in the element basis):
    the oracle's collocated convective term equals a from-scratch numpy
    evaluation with the Jacobian inverted point by point."""
    N = 5
    m = OracleMesh((2, 2, 2), N, amp=0.1, phase=inputs.deform_phases())
    X = m.coords()
    rng = np.random.default_rng(42)
    Q = rng.standard_normal((3, 3, 3))
    A = rng.standard_normal((3, 3))
    u = np.einsum("ijk,jp,kp->ip", Q, X, X) + np.einsum("ic,cp->ip", A, X)
    got = np.stack(m.conv(u))
    ref = _brute_force_conv(X, u, N)
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()
