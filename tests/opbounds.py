"""Per-point rounding-error bounds for the reduced-precision operator tests.

The element operator w = h1 sum_ab D_a^T (G_ab o D_b u) + h2 B o u is a chain
of sums; its computed value in unit roundoff u_a differs from the exact one
by at most gamma_k (|A| |u|)_i per point (Higham, Accuracy and Stability of
Numerical Algorithms, Sec. 3.1), where |A| |u| is the same chain evaluated
with |D|, |G|, |B| and |u|.  Rounding the geometry to storage adds its unit
roundoff times the same quantity; rounding the output adds the output's.
"""
import numpy as np

# G_ab storage order: rr rs rt ss st tt
_GI = {(0, 0): 0, (0, 1): 1, (0, 2): 2, (1, 1): 3, (1, 2): 4, (2, 2): 5}


def element_chain(D, G, B, u, h1, h2, lx):
    """h1 sum_ab D_a^T (G_ab o D_b u) + h2 B o u on element-major arrays
    (u[e][k][j][i], i along r); with absolute values as inputs it is |A| |u|."""
    E = u.size // lx ** 3
    ue = u.reshape(E, lx, lx, lx)
    Ge = G.reshape(6, E, lx, lx, lx)
    d = [np.einsum("il,ekjl->ekji", D, ue), np.einsum("jl,ekli->ekji", D, ue), np.einsum("kl,elji->ekji", D, ue)]
    s = [sum(Ge[_GI[tuple(sorted((a, b)))]] * d[b] for b in range(3)) for a in range(3)]
    out = (np.einsum("li,ekjl->ekji", D, s[0]) + np.einsum("lj,ekli->ekji", D, s[1])
           + np.einsum("lk,elji->ekji", D, s[2]))
    return h1 * out.ravel() + h2 * B * u


def abs_ax(m, u, h1, h2):
    """(|A| |u|)_i at every local point of the oracle mesh m."""
    _, _, D = m.tables()
    return element_chain(np.abs(D), np.abs(m.G()), np.abs(m.mass()), np.abs(u), h1, h2, m.lx)


def gamma(k, unit):
    return k * unit / (1 - k * unit)


# half the spacing of the subnormal numbers of each storage format: a result
# rounded into the subnormal range carries this absolute error instead of a
# relative one (gradual underflow; the relative model holds for normal results)
TINY = {"float64": 2.0 ** -1075, "float32": 2.0 ** -150, "float16": 2.0 ** -25, "bfloat16": 2.0 ** -134}


def ax_bound(m, u, h1, h2, unit_arith, eps_geo, eps_out, tiny_out=0.0):
    """Per-point bound on |w_computed - w_exact| for the operator on the
    stored (already rounded) input u: chain length k = 2 lx + 8 (two
    lx-term contractions, the three-term metric sum, the sum over a, the
    Helmholtz term), geometry rounded once to storage (twice its unit
    roundoff: the per-element power-of-two scale is exact but the scaled
    value is rounded from fp64 through the kernel's load), output rounded
    once to storage (relative eps_out, or the absolute tiny_out where the
    output is subnormal in its format)."""
    k = 2 * m.lx + 8
    return (gamma(k, unit_arith) + 2 * eps_geo + eps_out) * abs_ax(m, u, h1, h2) + tiny_out


def ax16_bound(m, u, h1, h2, eps_op, tiny_op, eps_geo, eps_out, tiny_out=0.0):
    """Per-point bound for 16-bit arithmetic with fp32 sums (Table 2's
    fp16-compute overrides as the kernels define them): on top of ax_bound's
    fp32 terms, four operand roundings in the 16-bit format -- the input
    (after the element's power-of-two scale s with max|u_e| s in [0.5, 1)),
    D, the metric-weighted derivatives, D^T -- each relative eps_op, so
    gamma_4(eps_op) (|A| |u|).  Operands that fall below the 16-bit normal
    range carry an absolute error tiny_op in scaled units instead: 2^E_e
    tiny_op on an input of element e (1/s = 2^E_e) propagates through |A|,
    and on a weighted derivative (scaled by gsc_e/s, gsc_e < 2 max|G_e|)
    through h1 |D^T| in each of the three directions."""
    lx = m.lx
    E = u.size // lx ** 3
    ue = np.abs(u).reshape(E, -1).max(axis=1)
    c = np.where(ue > 0, 2.0 ** (np.floor(np.log2(np.where(ue > 0, ue, 1.0))) + 1), 1.0)
    _, _, D = m.tables()
    gmax = np.abs(m.G()).reshape(6, E, -1).max(axis=(0, 2))
    ones = np.repeat(c, lx ** 3)
    t_in = abs_ax(m, ones, h1, 0.0)
    t_mid = np.repeat(abs(h1) * 3 * np.abs(D).sum(axis=0).max() * 2 * gmax * c, lx ** 3)
    return (ax_bound(m, u, h1, h2, 2.0 ** -24, eps_geo, eps_out, tiny_out) + gamma(4, eps_op) * abs_ax(m, u, h1, h2)
            + tiny_op * (t_in + t_mid))


def div_lipschitz(m):
    """L with |div u - div v| <= L max|u - v| at every node: the strong
    divergence sum_c sum_a (dr_a/dx_c) D_a u_c is linear in u with row sums
    at most max_p sum_ac |dr_a/dx_c| times the largest row sum of |D|."""
    _, _, D = m.tables()
    return float(np.abs(m.drdx()).sum(axis=0).max() * np.abs(D).sum(axis=1).max())


def check_maxdiv(m, L, div_gpu, div_oracle, ug, uo, step):
    """max|div u| after a step: (1) the GPU's value equals the oracle's
    diagnostics of the GPU's own velocity to rounding (the divergence at a
    node sums 9 lx terms of size at most L max|u| / 9), and (2) it differs
    from the oracle run's value by at most L max|u_gpu - u_oracle| (the
    divergence is linear in u with that Lipschitz constant)."""
    own = m.diagnostics(ug)[2]
    du = float(np.abs(ug - uo).max())
    scale = L * float(np.abs(ug).max())
    print("step %d max|div| gpu %.6e oracle %.6e (of gpu field %.6e); L max|du| %.2e"
          % (step, div_gpu, div_oracle, own, L * du))
    assert abs(div_gpu - own) <= 1e-13 * scale
    assert abs(div_gpu - div_oracle) <= L * du + 1e-13 * scale

