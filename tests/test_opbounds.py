"""The rounding-bound helper of the GPU operator tests evaluates the same
chain as the operator: with signed inputs it reproduces the oracle's Ax, and
its absolute form dominates |Ax| pointwise."""
import numpy as np
import pytest

from oracle import OracleMesh
from paper_2608_24348_amd import inputs
from opbounds import element_chain, abs_ax


@pytest.mark.parametrize("nel,N,amp", [((2, 2, 2), 5, 0.1), ((3, 2, 2), 7, 0.0)])
def test_chain_reproduces_oracle_operator(nel, N, amp):
    m = OracleMesh(nel, N, amp=amp, phase=inputs.deform_phases() if amp else None)
    u = inputs.local_normal(nel, N, seed=0)
    _, _, D = m.tables()
    for h1, h2 in [(1.0, 0.0), (1 / 1600, 11 / 6 / 5e-4)]:
        ref = m.ax(u, h1, h2)
        got = element_chain(D, m.G(), m.mass(), u, h1, h2, m.lx)
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
        assert np.all(abs_ax(m, u, h1, h2) >= np.abs(ref) * (1 - 1e-12))
