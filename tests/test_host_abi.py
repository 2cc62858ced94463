"""Host-side checks of libsem that need no GPU: the library loads, exports
every symbol include/sem.h declares, and sem_setup validates descriptors and
precision policies and sizes workspaces without touching the device."""
import ctypes as C
import os
import re

import pytest

from paper_2608_24348_amd import sem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    txt = open(os.path.join(ROOT, "include", "sem.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|size_t|void|const char\*)\s+(sem_[a-z_0-9]+)\s*\(", txt, re.M)))


def test_library_exports_every_declared_symbol():
    L = sem.load()
    names = _declared_symbols()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), n
    assert set(names) <= set(sem.EXPORTS)


def test_strerror_and_status_codes():
    L = sem.load()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.sem_strerror(code).decode()


@pytest.mark.parametrize("nel,N", [((1, 1, 1), 2), ((2, 3, 4), 3), ((8, 8, 8), 7), ((4, 4, 4), 11), ((3, 5, 7), 9),
                                   ((32, 32, 32), 7), ((16, 16, 16), 11), ((24, 24, 24), 5), ((1, 1, 64), 4)])
@pytest.mark.parametrize("tier", ["fp64", "fp32b", "fp32b+fp16"])
def test_setup_sizes_and_layout(nel, N, tier):
    c = sem.Context(sem.mesh_desc(nel, N), sem.flow_desc(), sem.tier(tier), bind=False)
    E = nel[0] * nel[1] * nel[2]
    assert c.E == E and c.lx == N + 1
    assert c.np == E * (N + 1) ** 3
    assert c.nglob == E * N ** 3
    # fluid workspace holds at least ~40 fp64 fields per point
    assert c.bytes >= 40 * 8 * c.np
    op = sem.Context(sem.mesh_desc(nel, N), sem.flow_desc(mode=sem.MODE_OPERATOR), sem.tier(tier), bind=False)
    assert op.bytes < c.bytes


@pytest.mark.parametrize("bad", [
    dict(order=1), dict(order=12), dict(nel=(0, 2, 2)),
    dict(amp=0.1, nel=(3, 2, 2)), dict(amp=0.3),
    # 2^29 local points along one line of elements in x (4 GiB of fp64)
    dict(nel=(1 << 20, 1, 1), order=7),
])
def test_setup_rejects_bad_meshes(bad):
    nel = bad.get("nel", (2, 2, 2))
    with pytest.raises(sem.SemError) as e:
        sem.Context(sem.mesh_desc(nel, bad.get("order", 4), amp=bad.get("amp", 0.0)), sem.flow_desc(), sem.tier("fp64"),
                    bind=False)
    assert e.value.code == -1


def test_policy_rules():
    md, fd = sem.mesh_desc((2, 2, 2), 4), sem.flow_desc()
    # rp = fp32 without the fp64 exceptions is rejected
    with pytest.raises(sem.SemError):
        sem.Context(md, fd, sem.precision(sem.FP32, exceptions=0), bind=False)
    # storage above rp is rejected
    with pytest.raises(sem.SemError):
        sem.Context(md, fd, sem.precision(sem.FP32, blocks={sem.BLOCK_VEL: (sem.FP64, sem.FP64, sem.FP64)}), bind=False)
    # fp64 compute on fp32 storage is the paper's Group B pattern and is accepted for the pressure block
    sem.Context(md, fd, sem.precision(sem.FP32, blocks={sem.BLOCK_PRES: (sem.FP64, sem.FP64, sem.FP32)}), bind=False)
    # 16-bit storage with fp32 arithmetic, and Table 2's 16-bit arithmetic (fp32
    # sums) on the Helmholtz/Poisson operators, are accepted
    sem.Context(md, fd, sem.precision(sem.FP32, kernels={sem.K_AX_VEL: (sem.FP32, sem.FP32, sem.FP16)}), bind=False)
    for k in (sem.K_AX_VEL, sem.K_AX_PRES):
        for h in (sem.FP16, sem.BF16):
            sem.Context(md, fd, sem.precision(sem.FP32, kernels={k: (h, sem.FP32, h)}), bind=False)
    for t in ("fp32b+fp16c", "fp32b+bf16c", "fp32b+fp16pc"):
        sem.Context(md, fd, sem.tier(t), bind=False)
    # ... but not elsewhere, not on geometry of another format, and not with
    # 16-bit or fp64 sums
    bad16 = [{sem.K_OPGRAD: (sem.FP16, sem.FP32, sem.FP16)}, {sem.K_CONV: (sem.BF16, sem.FP32, sem.BF16)},
             {sem.K_AX_VEL: (sem.FP16, sem.FP32, sem.FP32)}, {sem.K_AX_VEL: (sem.FP16, sem.FP32, sem.BF16)},
             {sem.K_AX_VEL: (sem.FP16, sem.FP16, sem.FP16)}, {sem.K_AX_PRES: (sem.BF16, sem.FP64, sem.BF16)}]
    for ks in bad16:
        with pytest.raises(sem.SemError):
            sem.Context(md, fd, sem.precision(sem.FP32, kernels=ks), bind=False)
    # fp64 velocity vectors have no 16-bit-arithmetic kernel
    with pytest.raises(sem.SemError):
        sem.Context(md, fd, sem.precision(sem.FP64, kernels={sem.K_AX_VEL: (sem.FP16, sem.FP32, sem.FP16)}), bind=False)
    # two 16-bit formats in one context are rejected
    with pytest.raises(sem.SemError):
        sem.Context(md, fd, sem.precision(sem.FP32, kernels={sem.K_AX_VEL: (sem.FP32, sem.FP32, sem.FP16),
                                                             sem.K_OPGRAD: (sem.FP32, sem.FP32, sem.BF16)}), bind=False)
    # velocity vectors below fp32 are rejected
    with pytest.raises(sem.SemError):
        sem.Context(md, fd, sem.precision(sem.FP32, blocks={sem.BLOCK_VEL: (sem.FP32, sem.FP32, sem.FP16)}), bind=False)
    for t in sem.TIERS:
        sem.Context(md, fd, sem.tier(t), bind=False)


def test_flow_validation():
    md = sem.mesh_desc((2, 2, 2), 4)
    for kw in (dict(nu=0.0), dict(dt=-1.0), dict(torder=4), dict(restart=31), dict(vel_tol=0.0), dict(max_refine=0),
               dict(proj=-1), dict(proj=21), dict(mode=sem.MODE_POISSON, proj=5), dict(cfl=-0.1),
               dict(cfl=float("inf")), dict(cfl=float("nan")), dict(mode=sem.MODE_POISSON, cfl=0.4)):
        with pytest.raises(sem.SemError):
            sem.Context(md, sem.flow_desc(**kw), sem.tier("fp64"), bind=False)


def test_dealias_validation_and_workspace():
    md = sem.mesh_desc((2, 2, 2), 4)
    for kw in (dict(dealias=2), dict(dealias=-1), dict(mode=sem.MODE_POISSON, dealias=1),
               dict(mode=sem.MODE_OPERATOR, dealias=1)):
        with pytest.raises(sem.SemError):
            sem.Context(md, sem.flow_desc(**kw), sem.tier("fp64"), bind=False)
    # 16-bit conv storage needs fp32 arithmetic (as for every 16-bit kernel)
    with pytest.raises(sem.SemError):
        sem.Context(md, sem.flow_desc(dealias=1), sem.precision(sem.FP32, kernels={sem.K_CONV: (sem.FP64, sem.FP64, sem.FP16)}),
                    bind=False)
    # workspace grows by the 9 metric terms per fine point: fp64, plus the copy in
    # the conv storage precision (fp32, or 16-bit with one float scale per element)
    E, nd = 8, (3 * 5 + 1) // 2
    for t, per, extra in (("fp64", 8, 0), ("fp32b", 12, 0), ("fp32b+fp16a", 10, 4 * E), ("fp32b+bf16a", 10, 4 * E)):
        a = sem.Context(md, sem.flow_desc(), sem.tier(t), bind=False)
        b = sem.Context(md, sem.flow_desc(dealias=1), sem.tier(t), bind=False)
        assert 0 <= (b.bytes - a.bytes) - 9 * E * nd ** 3 * per - extra < 768, t


def test_hsmg_validation_and_workspace():
    fd = sem.flow_desc(hsmg=1)
    for md, fdd in ((sem.mesh_desc((2, 2, 2), 3), fd),                       # order below 4
                    (sem.mesh_desc((2, 2, 2), 6, amp=0.05), fd),             # perturbed mesh
                    (sem.mesh_desc((1, 2, 2), 6), fd),                       # one element in x
                    (sem.mesh_desc((2, 65, 2), 4), fd),                      # coarse plane beyond 64 x 64
                    (sem.mesh_desc((2, 2, 2), 6), sem.flow_desc(mode=sem.MODE_OPERATOR, hsmg=1)),
                    (sem.mesh_desc((2, 2, 2), 6), sem.flow_desc(hsmg=2))):
        with pytest.raises(sem.SemError):
            sem.Context(md, fdd, sem.tier("fp64"), bind=False)
    # 16-bit pressure basis storage is refused (the preconditioner output is stored in it)
    md = sem.mesh_desc((3, 2, 2), 7)
    with pytest.raises(sem.SemError):
        sem.Context(md, fd, sem.precision(sem.FP32, blocks={sem.BLOCK_PRES: (sem.FP32, sem.FP32, sem.FP16)}), bind=False)
    # workspace: tables, the fine local solutions (fp64), M^{-1} V_J and the
    # kept Z_0..Z_m (basis precision), 3 middle vectors, 8 corner values per
    # element, 2 coarse vectors
    E, lx, lm, nc, m = 12, 8, 4, 12, 30
    for t, pb in (("fp64", 8), ("fp32b", 4)):
        a = sem.Context(md, sem.flow_desc(), sem.tier(t), bind=False)
        b = sem.Context(md, fd, sem.tier(t), bind=False)
        tables = 8 * (3 * lx * lx + 3 * lx + 3 * lm * lm + 3 * lm + lx * lm + 2 * lm + 9 + 2 * 4 + 3 + 2 * 2)
        want = tables + E * lx ** 3 * (8 + (m + 2) * pb) + 3 * 8 * E * lm ** 3 + 64 * E + 2 * 8 * nc
        assert 0 <= (b.bytes - a.bytes) - want < 11 * 256, t
    for t in ("fp64", "fp32b", "fp32b+fp16", "fp32b+fp16a"):
        sem.Context(md, fd, sem.tier(t), bind=False)
    sem.Context(md, sem.flow_desc(mode=sem.MODE_POISSON, hsmg=1), sem.tier("fp64"), bind=False)


def test_unbound_context_calls_fail_cleanly():
    c = sem.Context(sem.mesh_desc((2, 2, 2), 3), sem.flow_desc(), sem.tier("fp64"), bind=False)
    L = sem.load()
    assert L.sem_dssum(c.h, C.c_void_p(1), 0) == -6
    assert L.sem_ax(c.h, C.c_void_p(1), C.c_void_p(1), 1.0, 0.0, 0, -1, 0) == -6
    d = sem.Context(sem.mesh_desc((2, 2, 2), 3), sem.flow_desc(), sem.tier("fp32b"), bind=False)
    assert L.sem_copy_state(d.h, c.h) == -6
    # moving an unbound context to a stream, or a null context
    assert L.sem_set_stream(c.h, None) == -6
    assert L.sem_set_stream(None, None) == -1


def test_bind_rejects_unfit_workspaces():
    """A caller-provided workspace is checked before anything reaches the
    device: element type, size, 256-byte alignment, device residence."""
    import torch
    c = sem.Context(sem.mesh_desc((2, 2, 2), 3), sem.flow_desc(), sem.tier("fp64"), bind=False)
    raw = torch.empty(c.bytes + 512, dtype=torch.uint8)
    off = (-raw.data_ptr()) % 256
    fit = raw[off:off + c.bytes]
    with pytest.raises(ValueError, match="uint8"):
        c.bind("cpu", workspace=torch.empty(c.bytes, dtype=torch.float32))
    with pytest.raises(ValueError, match="needs"):
        c.bind("cpu", workspace=fit[:c.bytes - 256])
    with pytest.raises(ValueError, match="256-byte"):
        c.bind("cpu", workspace=raw[off + 1:off + 1 + c.bytes])
    with pytest.raises(ValueError, match="device tensor"):
        c.bind("cpu", workspace=fit)
    assert c.ws is None
