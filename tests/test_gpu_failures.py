"""Failure isolation and checkpoint/restart of the batched fluid step,
through the C ABI.

A request whose state turns non-finite, or whose solver hits its iteration
limit, reports SEM_ENAN / SEM_ENOTCONV in its own step statistics; the other
requests of the batch keep results bitwise equal to their runs alone (every
reduction and convergence flag is per request).  A checkpoint of the fluid
state through sem_get_field, restored into a fresh context with
sem_set_field and sem_set_clock, continues the run bitwise.  The faults are
planted from the host into the request's data (a NaN value, an iteration
limit of 1); every kernel still runs its normal, bounded course.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SEM_ENAN, SEM_ENOTCONV = -4, -5


@pytest.fixture(scope="module")
def sem():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_24348_amd import sem as s
    s.load()
    return s


SPECS = [((4, 4, 4), 1 / 400), ((6, 4, 2), 1 / 1000), ((2, 2, 4), 1 / 100)]


def _ctx(sem, nel, nu, tier="fp64", **kw):
    return sem.Context(sem.mesh_desc(nel, 7), sem.flow_desc(nu=nu, dt=1e-3, **kw), sem.tier(tier))


def _alone(sem, tier, hsmg, nsteps=3):
    out = []
    for nel, nu in SPECS:
        c = _ctx(sem, nel, nu, tier, hsmg=hsmg)
        st = sem.fluid_step([c], nsteps)[0]
        out.append((st, c.velocity(), c.pressure()))
        c.close()
    return out


def _same(a, b):
    st, u, p = a
    st2, u2, p2 = b
    assert [s["pit"] for s in st] == [s["pit"] for s in st2]
    assert [s["vit"] for s in st] == [s["vit"] for s in st2]
    assert [s["ke"] for s in st] == [s["ke"] for s in st2]
    assert np.array_equal(u, u2) and np.array_equal(p, p2)


@pytest.mark.parametrize("tier,hsmg", [("fp64", 0), ("fp32b", 1)])
def test_nan_in_one_request_leaves_batch_mates_bitwise(sem, tier, hsmg):
    alone = _alone(sem, tier, hsmg)
    ctxs = [_ctx(sem, nel, nu, tier, hsmg=hsmg) for nel, nu in SPECS]
    u = ctxs[1].get(sem.F_U)
    u[12345 % u.size] = np.nan
    ctxs[1].set(sem.F_U, u)
    mix = sem.fluid_step(ctxs, 3)
    print("statuses", [[s["status"] for s in m] for m in mix])
    assert all(s["status"] == SEM_ENAN for s in mix[1])
    for i in (0, 2):
        assert all(s["status"] == 0 for s in mix[i])
        _same(alone[i], (mix[i], ctxs[i].velocity(), ctxs[i].pressure()))


@pytest.mark.parametrize("tier,hsmg", [("fp64", 0), ("fp32b", 1)])
def test_iteration_limit_in_one_request_leaves_batch_mates_bitwise(sem, tier, hsmg):
    alone = _alone(sem, tier, hsmg)
    ctxs = []
    for i, (nel, nu) in enumerate(SPECS):
        # one PCG iteration per refinement cycle and a single cycle (with
        # fp32 vectors further fp64-residual cycles would restart the solve)
        kw = dict(vel_maxit=1, max_refine=1) if i == 0 else {}
        if i == 2:
            kw = dict(pres_maxit=1)
        ctxs.append(_ctx(sem, nel, nu, tier, hsmg=hsmg, **kw))
    mix = sem.fluid_step(ctxs, 3)
    print("statuses", [[s["status"] for s in m] for m in mix], "pit", [[s["pit"] for s in m] for m in mix])
    # request 0: one PCG iteration per solve cannot reach 1e-8
    assert all(s["status"] == SEM_ENOTCONV for s in mix[0])
    assert all(max(s["vres"]) > 1e-8 for s in mix[0])
    # request 2: one Arnoldi step; the first steps of the ramp may need none
    assert any(s["status"] == SEM_ENOTCONV for s in mix[2])
    assert all(s["pit"] <= 1 for s in mix[2])
    assert all(s["status"] == 0 for s in mix[1])
    _same(alone[1], (mix[1], ctxs[1].velocity(), ctxs[1].pressure()))


FIELDS = ["F_U", "F_ULAG1", "F_ULAG2", "F_BNLAG1", "F_BNLAG2"]


@pytest.mark.parametrize("tier,hsmg", [("fp64", 0), ("fp32b", 1), ("fp32b", 0)])
def test_checkpoint_restore_into_fresh_context_continues_bitwise(sem, tier, hsmg):
    nel, nu = (4, 4, 4), 1 / 400
    a = _ctx(sem, nel, nu, tier, hsmg=hsmg)
    sem.fluid_step([a], 4)
    # checkpoint: every state field to host memory, plus the clock
    ck = {}
    for name in FIELDS:
        base = getattr(sem, name)
        for c in range(3):
            ck[base + c] = a.get(base + c)
    ck[sem.F_P] = a.get(sem.F_P)
    d = a.diagnostics()
    b = _ctx(sem, nel, nu, tier, hsmg=hsmg)
    for which, arr in ck.items():
        b.set(which, arr)
    b.set_clock(d["t"], d["step"])
    sa = sem.fluid_step([a], 3)[0]
    sb = sem.fluid_step([b], 3)[0]
    print("after restore", [s["pit"] for s in sa], [s["pit"] for s in sb])
    _same((sa, a.velocity(), a.pressure()), (sb, b.velocity(), b.pressure()))
    assert [s["t"] for s in sa] == [s["t"] for s in sb]
