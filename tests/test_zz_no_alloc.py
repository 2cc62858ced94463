"""The allocation-free Poisson entry point (sem_poisson_solve_noalloc),
through the C ABI, against sem_poisson_solve on a context with its own
solver workspace: the same launches on the same data, so solutions and
iteration counts are bitwise equal.  Two calls in a row, the second on a
smaller mesh and another tier (the static array then holds the first call's
values, which the solve must not read); a solve that would not fit the array
is rejected before any kernel runs; the context stays usable afterwards."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sem():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_24348_amd import sem as s
    s.load()
    return s


def _rhs(c, seed):
    # assembled load vector of a smooth field plus seeded noise
    g = torch.Generator(device="cuda:0")
    g.manual_seed(seed)
    f = c.node_field(3, 3.0) + 1e-3 * torch.randn(c.np, dtype=torch.float64, device="cuda:0", generator=g)
    return c.mass(f, assemble=True)


def _pair(sem, nel, N, tier):
    kw = dict(pres_tol=1e-9, pres_maxit=3000)
    op = sem.Context(sem.mesh_desc(nel, N), sem.flow_desc(mode=sem.MODE_OPERATOR, **kw), sem.tier(tier))
    ref = sem.Context(sem.mesh_desc(nel, N), sem.flow_desc(mode=sem.MODE_POISSON, **kw), sem.tier(tier))
    return op, ref


def test_noalloc_poisson_equals_poisson_solve_two_calls(sem):
    for call, (nel, N, tier) in enumerate([((4, 4, 4), 7, "fp64"), ((2, 3, 2), 5, "fp32b")]):
        op, ref = _pair(sem, nel, N, tier)
        rhs = _rhs(ref, 7 + call)
        sol_ref = torch.empty_like(rhs)
        st_ref = sem.poisson_solve([ref], [rhs], [sol_ref])[0]
        sol = torch.full_like(rhs, float("nan"))
        print("call", call + 1, nel, N, tier, flush=True)
        st = sem.poisson_solve_noalloc(op, rhs, sol)
        print("  iters", st["iters"], "ref", st_ref["iters"], "res", st["res"], flush=True)
        assert st == st_ref
        assert st["status"] == 0 and st["iters"] > 0
        assert torch.equal(sol, sol_ref)
        # the operator context still works with its own workspace afterwards
        w1 = torch.empty_like(rhs)
        w2 = torch.empty_like(rhs)
        op.ax(sol, w1, 1.0, 0.0, assemble=True)
        ref.ax(sol, w2, 1.0, 0.0, assemble=True)
        torch.cuda.synchronize()
        assert torch.equal(w1, w2)
        # and a Poisson-mode context gives the same answer through both entry points
        sol2 = torch.empty_like(rhs)
        assert sem.poisson_solve_noalloc(ref, rhs, sol2) == st_ref
        assert torch.equal(sol2, sol_ref)
        op.close()
        ref.close()


def test_noalloc_rejects_a_workspace_beyond_the_static_array(sem):
    nel, N = (16, 16, 16), 7
    c = sem.Context(sem.mesh_desc(nel, N), sem.flow_desc(mode=sem.MODE_OPERATOR), sem.tier("fp64"))
    need = (31 * 8 + 4 * 8) * c.np
    assert need > sem.noalloc_max_bytes()
    rhs = torch.zeros(c.np, dtype=torch.float64, device="cuda:0")
    sol = torch.zeros_like(rhs)
    with pytest.raises(sem.SemError) as ei:
        sem.poisson_solve_noalloc(c, rhs, sol)
    assert ei.value.code == -2 and "static array" in str(ei.value)
    assert torch.count_nonzero(sol) == 0
    c.close()
