#!/usr/bin/env python3
"""Benchmark of the SEM Taylor-Green fluid step on one MI355X.

Workload (default): Taylor-Green vortex, Re = 1600, periodic box [-pi, pi]^3,
32^3 hexahedra of order N = 7 (16.8 M local points), dt = 5e-4, BDF3/EXT3,
Jacobi-PCG velocity (absolute 1e-6) and GMRES(30) pressure (absolute 1e-4),
the solver tolerances of the paper's TGV runs; 200 timed steps (t = 0.1)
after a few untimed ones.  One "step" is one full fluid time step
(convection, RHS, three velocity solves with fp64 residual refinement,
pressure residual, pressure solve, correction, diagnostics).  The reported
value is steps/s of the fp32-bounded tier; the plain fp64 tier runs the same
steps on the same GPU for the speedup and for the kinetic-energy / enstrophy
error series.

Also reported: Ax GDOF/s of the Helmholtz operator on the same mesh, a
roofline record for the dominant kernel (HIP-event kernel times measured in
the timed region, algorithmic bytes per launch), and the FP64 CPU oracle
timed on the host cores on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "TGV steps/s & Ax GDOF/s, mixed vs fp64 at stated enstrophy error; p99 latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def gmres_j_sequence(iters, m):
    """Arnoldi indices J of every step of a GMRES(m) solve with `iters` steps."""
    out = []
    for it in range(iters):
        out.append(it % m)
    return out


def run_tier(sem, torch, tier, nel, N, nu, dt, warmup, steps, prof_class=None, vtol=1e-6, ptol=1e-4, proj=0,
             dealias=0, cfl=0.0, hsmg=0, graph=0):
    ctx = sem.Context(sem.mesh_desc(nel, N), sem.flow_desc(nu=nu, dt=dt, restart=30, vel_tol=vtol, pres_tol=ptol,
                                                           proj=proj, dealias=dealias, cfl=cfl, hsmg=hsmg),
                      sem.tier(tier))
    torch.cuda.synchronize()
    series = []
    d0 = ctx.diagnostics()
    series.append((0.0, d0["ke"], d0["enst"], d0["maxdiv"]))
    if warmup:
        for s in sem.fluid_step([ctx], warmup, graph=bool(graph))[0]:
            series.append((s["t"], s["ke"], s["enst"], s["maxdiv"]))
            log("  %s warmup step t=%.4f its v=%s p=%d" % (tier, s["t"], s["vit"], s["pit"]))
    torch.cuda.synchronize()
    if prof_class:
        sem.prof_start(prof_class)
    g0 = sem.graph_counters()
    t0 = time.perf_counter()
    st = sem.fluid_step([ctx], steps, graph=bool(graph))[0]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g1 = sem.graph_counters()
    ctx.graph_counts = {"replays": g1[0] - g0[0], "reruns": g1[1] - g0[1], "captures": g1[2] - g0[2]}
    prof = sem.prof_stop() if prof_class else None
    for s in st:
        series.append((s["t"], s["ke"], s["enst"], s["maxdiv"]))
        log("  %s step t=%.4f its v=%s p=%d ke=%.12f" % (tier, s["t"], s["vit"], s["pit"], s["ke"]))
        if s["status"] != 0:
            raise RuntimeError("%s step failed with status %d" % (tier, s["status"]))
    return ctx, (t1 - t0), st, series, prof


def ax_rate(sem, torch, ctx, dtype, geom, reps=20, nvec=2, h1=1.0, h2=0.0, half=False):
    """Operator GDOF/s (HIP events, current stream).  The launches cycle
    through nvec distinct input/output pairs so that no launch finds its
    vectors in the last-level cache left by the previous one.  half: 16-bit
    arithmetic (Table 2's fp16-compute overrides)."""
    g = torch.Generator(device="cuda:0")
    g.manual_seed(0)
    us = [torch.randn(ctx.np, dtype=torch.float64, device="cuda:0", generator=g).to(dtype) for _ in range(nvec)]
    ws = [torch.empty_like(us[0]) for _ in range(nvec)]
    for q in range(nvec):
        ctx.ax(us[q], ws[q], h1, h2, geom=geom, half_compute=half)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for r in range(reps):
        ctx.ax(us[r % nvec], ws[r % nvec], h1, h2, geom=geom, half_compute=half)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del us, ws
    return ctx.np / (ms * 1e-3) / 1e9, ms


def dssum_rate(sem, torch, ctx, dtype, reps=20, nvec=2):
    """Gather-scatter (dssum) time per launch, HIP events, nvec distinct vectors."""
    g = torch.Generator(device="cuda:0")
    g.manual_seed(1)
    us = [torch.randn(ctx.np, dtype=torch.float64, device="cuda:0", generator=g).to(dtype) for _ in range(nvec)]
    for q in range(nvec):
        ctx.dssum(us[q])
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for r in range(reps):
        ctx.dssum(us[r % nvec])
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del us
    return ms


def ax_leg(sem, torch, inputs, nel=64, N=7):
    """The Ax microbenchmark workload: 64^3 elements N=7 (134 M points),
    sinusoidally deformed (amplitude 0.1 h, seeded phases), u ~ N(0,1)
    seeded; the operator in Poisson form in every storage tier and in
    Helmholtz form (h1 = 1/1600, h2 = 11/6 / 5e-4) in fp64 and fp32 (bytes per
    point: vectors in and out + 6 geometric factors, + B for Helmholtz), then
    dssum of a vector in fp64, fp32 and fp16 (bytes per point: the shared
    fraction of points read and written once; also the line floor, every point
    read and written once).  Legs named
    *_c16 run 16-bit arithmetic (16-bit operands, fp32 sums)."""
    out = {"workload": "%d^3 elements N=%d (%d points), deformed amp 0.1 h, u ~ N(0,1); HIP events over 20 launches "
                       "cycling through 2 vector pairs" % (nel, N, nel ** 3 * (N + 1) ** 3)}
    for tier16, legs in (("fp32b+fp16all", (("fp64", torch.float64, sem.FP64, 64, 0),
                                             ("fp32", torch.float32, sem.FP32, 32, 0),
                                             ("fp32_fp16geom", torch.float32, sem.FP16, 20, 0),
                                             ("fp16", torch.float16, sem.FP16, 16, 0),
                                             ("fp32_fp16geom_c16", torch.float32, sem.FP16, 20, 2),
                                             ("fp16_c16", torch.float16, sem.FP16, 16, 2),
                                             ("fp32_fp16geom_c16_helmholtz", torch.float32, sem.FP16, 22, 3),
                                             ("fp64_helmholtz", torch.float64, sem.FP64, 72, 1),
                                             ("fp32_helmholtz", torch.float32, sem.FP32, 36, 1))),
                         ("fp32b+bf16all", (("bf16", torch.bfloat16, sem.BF16, 16, 0),
                                            ("fp32_bf16geom", torch.float32, sem.BF16, 20, 0),
                                            ("bf16_c16", torch.bfloat16, sem.BF16, 16, 2),
                                            ("fp32_bf16geom_c16", torch.float32, sem.BF16, 20, 2)))):
        ctx = sem.Context(sem.mesh_desc((nel,) * 3, N, amp=0.1, phase=inputs.deform_phases()),
                          sem.flow_desc(mode=sem.MODE_OPERATOR), sem.tier(tier16))
        for name, dt, geom, bpp, kind in legs:
            # kind: 0 Poisson, 1 Helmholtz, 2 Poisson in 16-bit arithmetic, 3 Helmholtz in 16-bit arithmetic
            h1, h2 = (1.0 / 1600, 11.0 / 6.0 / 5e-4) if kind in (1, 3) else (1.0, 0.0)
            gd, ms = ax_rate(sem, torch, ctx, dt, geom, h1=h1, h2=h2, half=kind >= 2)
            out[name] = {"gdof_per_s": gd, "ms": ms, "bytes_per_point": bpp, "hbm_GBps": gd * bpp,
                         "frac": gd * bpp / HBM_PEAK_GBS}
        if tier16 == "fp32b+fp16all":
            lx = N + 1
            shared = 1.0 - ((lx - 2) / lx) ** 3
            for name, dt, b in (("dssum_fp64", torch.float64, 8), ("dssum_fp32", torch.float32, 4),
                                ("dssum_fp16", torch.float16, 2)):
                ms = dssum_rate(sem, torch, ctx, dt)
                alg = ctx.np * shared * 2 * b
                # every row of lx nodes holds a shared node (i = 0 and N), so every
                # line is read and written: one read and one write of the vector
                line = ctx.np * 2 * b
                out[name] = {"ms": ms, "alg_bytes": alg, "hbm_GBps": alg / (ms * 1e-3) / 1e9,
                             "frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "line_floor_bytes": line,
                             "line_GBps": line / (ms * 1e-3) / 1e9}
        del ctx
        torch.cuda.empty_cache()
    return out


def c4_leg(sem, torch, steps, tiers=("fp64", "fp32b-p32", "fp32b", "fp32b+fp16", "fp32b+fp16c"), graph=0):
    """The higher-order workload: 16^3 elements, N = 11 (7.1 M points), Re 1600,
    dt 2.5e-4, tolerances 1e-6 / 1e-4, HSMG; steps/s per tier, and each tier's
    error metrics and max|div| against the oracle's stored series."""
    nel, N, dt = 16, 11, 2.5e-4
    ref = oracle_series(nel, N, dt, 1600.0, 1e-6, 1e-4, 1, 0, 0.0, 0)
    out = {"workload": "TGV Re=1600, 16^3 elements, N=11 (7077888 local pts), dt=2.5e-4, HSMG, %d steps" % steps}
    for t in tiers:
        c, secs, st, ser, _ = run_tier(sem, torch, t, (nel,) * 3, N, 1.0 / 1600, dt, 0, steps, None, 1e-6, 1e-4,
                                       0, 0, 0.0, 1, graph)
        out[t] = {"steps_per_s": steps / secs, "max_div": max(r[3] for r in ser),
                  "vel_iters_mean": sum(max(x["vit"]) for x in st) / len(st),
                  "vel_cycles_mean": sum(x["vcyc"] for x in st) / len(st),
                  "pres_iters_mean": sum(x["pit"] for x in st) / len(st)}
        if ref is not None:
            out[t]["error_vs_oracle"] = error_vs_oracle(ser, ref)
        del c
        torch.cuda.synchronize()
    out["speedup_vs_fp64"] = {t: out[t]["steps_per_s"] / out["fp64"]["steps_per_s"] for t in tiers if t != "fp64"}
    return out


# algorithmic bytes per local point of one active (component) launch, by tier
def _bytes_per_point(kind, tier):
    mixed = tier != "fp64"
    g16 = "fp16" in tier or "bf16" in tier
    if kind == "ax_vel":
        # u, w (velocity vectors) + 6 G + B (geometry of the velocity operator)
        vec = 4 if mixed else 8
        geo = 2 if (mixed and g16) else vec
        return 2 * vec + 7 * geo
    if kind == "ax_pres":
        # V_J (basis) + Jacobi diagonal + 6 G + w (fp64)
        geo = 8 if not mixed else (2 if tier.endswith("16p") else 4)
        bv = 4 if mixed else 8
        dg = 4 if mixed else 8
        return bv + dg + 6 * geo + 8
    raise ValueError(kind)


def _basis_bytes(tier):
    return 8 if tier in ("fp64",) else 4


# the roofline kernel classes: kernel name as rocprofv3 reports it, and the
# algorithmic bytes of one launch as a function of the Arnoldi index J
PROF_KERNELS = {
    "gm_upd_dots": ("gm_pass_kernel<1, %s>", "GMRES CGS2 pass 1: w' = w - mean - sum h_i V_i, dots (V_i, w')",
                    lambda npts, J, bv: npts * (16 + (J + 1) * bv)),
    "gm_upd_norm": ("gm_pass_kernel<2, %s>", "GMRES CGS2 pass 2: V_{J+1} = w' - sum h2_i V_i, |V_{J+1}|^2",
                    lambda npts, J, bv: npts * (8 + (J + 2) * bv)),
}


KERNEL_SOURCES = {"ax_resid": ("k_ax.hip", "k_common.h", "sem_internal.h"),
                  "ax_presid": ("k_ax.hip", "k_common.h", "sem_internal.h"),
                  "ax_vel": ("k_ax.hip", "k_common.h", "sem_internal.h"),
                  "ax_pres": ("k_ax.hip", "k_common.h", "sem_internal.h")}


def kernel_sources_sha(kind="gm_upd_dots"):
    """Hash of the sources that make a kernel class (a stored PMC traffic
    figure is valid only for the exact kernel it was taken on)."""
    import hashlib
    h = hashlib.sha256()
    base = os.path.join(ROOT, "paper_2608_24348_amd", "csrc")
    for f in KERNEL_SOURCES.get(kind, ("k_vec.hip", "k_common.h", "k_fin.h", "sem_internal.h")):
        with open(os.path.join(base, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic(kind, tier, workload):
    """HBM bytes per launch from the committed rocprofv3 PMC summary of this
    kernel class and workload, if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "pmc_%s_%s.json" % (kind, tier))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("sources_sha256") != kernel_sources_sha(kind) or d.get("workload") != workload:
        return None
    return d["hbm_bytes_per_launch"]


def conv_units(N, dealias, tier):
    """Algorithmic HBM bytes and flops of the convective term per element:
    u (3 fp64 fields) in, B N(u) (3 fp64 fields) out, 9 metric terms per
    point of the grid it integrates on (GLL points, or the lxd^3 Gauss-Legendre
    points when dealiased) in the conv storage precision.  Flops of the
    dealiased form: 12 interpolations to the fine grid (u and its three
    reference derivatives per component, 2 lx flops per output point of each
    of the three one-dimensional stages), 3 transposed ones back, and the
    point-wise contravariant products."""
    lx = N + 1
    tm = 8 if tier == "fp64" else 4
    if not dealias:
        byt = lx ** 3 * (3 * 8 + 9 * tm + 3 * 8)
        fl = lx ** 3 * 3 * (3 * 2 * lx + 3 * 6 + 2)
        return byt, fl
    nd = (3 * lx + 1) // 2
    byt = lx ** 3 * 6 * 8 + 9 * tm * nd ** 3
    interp = 2 * lx * (lx * lx * nd + lx * nd * nd + nd ** 3)
    back = 2 * nd * (lx * nd * nd + lx * lx * nd + lx ** 3)
    point = nd ** 3 * (3 * 3 * 2 + 3 * 3 * 2)
    return byt, 12 * interp + 3 * back + point


def roofline(kind, tier, prof, steps, npts, workload, N=7, dealias=0):
    """Achieved HBM bandwidth of one kernel class over the timed region:
    algorithmic bytes of its launches / summed HIP-event kernel time of all
    its launches (gated no-op launches after convergence included)."""
    tot_ms, nlaunch = prof
    bv = _basis_bytes(tier)
    if kind == "ax_resid":
        # fp64 velocity residual operator R_L = RHS_L - H_L u for the three
        # components in one launch: the least the launch must move is u, RHS_L
        # and w of each component plus the 6 G and B the components share,
        # 16 values = 128 B/point (three separate applications would be
        # 3 x 80); per step one check before the solve and, with fp32
        # vectors, one after every cycle
        alg = 0.0
        active = 0
        for s in steps:
            nv = 1 + (s["vcyc"] if tier != "fp64" else 0)
            alg += nv * npts * 128
            active += nv
        name = "ax_kernel<%d, double, double, double, 0, double, 1, 0, 1> -- fp64 velocity residual RHS_L - H_L u" % (N + 1)
    elif kind == "ax_presid":
        # fp64 Poisson residual operator at the end of every GMRES cycle that
        # started from a nonzero iterate (u, w, 6 G = 64 B/point); the other
        # launches are gated no-ops of converged requests
        alg = 0.0
        active = 0
        for s in steps:
            ncyc = (s["pit"] + 29) // 30 if s["pit"] > 0 else 0
            alg += ncyc * npts * 64
            active += ncyc
        name = "ax_kernel<%d, double, double, double, 0, double, 0, 0, 0> -- fp64 GMRES cycle-end residual" % (N + 1)
    elif kind in PROF_KERNELS:
        kname, what, fbytes = PROF_KERNELS[kind]
        alg = 0.0
        active = 0
        for s in steps:
            for J in gmres_j_sequence(s["pit"], 30):
                alg += fbytes(npts, J, bv)
                active += 1
        name = (kname % ("float" if bv == 4 else "double")) + " -- " + what
    elif kind == "conv":
        lx = N + 1
        E = npts // lx ** 3
        byt, fl = conv_units(N, dealias, tier)
        tot_ms, nlaunch = prof
        alg = nlaunch * E * byt
        achieved = alg / (tot_ms * 1e-3) / 1e9 if tot_ms > 0 else 0.0
        flops = nlaunch * E * fl / (tot_ms * 1e-3) / 1e12 if tot_ms > 0 else 0.0
        peak_fl = 78.6 if tier == "fp64" else 157.3
        name = ("conv_dealias_v2_kernel<%d, %s>" % (lx, "double, double" if tier == "fp64" else "float, float")
                if dealias else "conv_kernel<%d, ...>" % lx) + " -- convective term B N(u)"
        return {"kernel": name, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None, "launches": nlaunch, "active_units": nlaunch,
                "kernel_ms_total": tot_ms, "avg_launch_ms": tot_ms / max(nlaunch, 1),
                "alg_bytes_per_launch": E * byt, "alg_bytes_total": alg,
                "vector_tflops": flops, "vector_peak_tflops": peak_fl, "vector_frac": flops / peak_fl}
    elif kind == "ax_vel":
        active = sum(sum(s["vit"]) for s in steps)  # component launches that did work
        alg = active * npts * _bytes_per_point(kind, tier)
        name = "ax_kernel<%d,...> velocity Helmholtz operator (PCG)" % (N + 1)
    else:
        active = sum(s["pit"] for s in steps)
        alg = active * npts * _bytes_per_point(kind, tier)
        name = "ax_kernel<%d,...> pressure operator (Arnoldi step)" % (N + 1)
    achieved = alg / (tot_ms * 1e-3) / 1e9 if tot_ms > 0 else 0.0
    traffic = stored_traffic(kind, tier, workload)
    return {"kernel": name, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "launches": nlaunch, "active_units": active,
            "kernel_ms_total": tot_ms, "avg_launch_ms": tot_ms / max(nlaunch, 1),
            "alg_bytes_per_launch": alg / max(nlaunch, 1), "alg_bytes_total": alg}


GOLDEN = os.path.join(ROOT, "tests", "golden")

# which operators of a step compute in which precision, by tier (the config string)
TIER_NOTE = {
    "fp64": "everything fp64",
    "fp32b": "fp32: SEM operators (convection, opgrad), velocity operator and PCG vectors, GMRES basis and "
             "projection storage; fp64: pressure-operator arithmetic (fp32-stored geometry), HSMG, weak divergence "
             "of u*, GMRES orthogonalisation/dots/H, BDF/EXT state, residual checks, global reductions",
    "fp32b-p32": "fp32: SEM operators, velocity operator and PCG vectors, pressure operator (arithmetic and "
                 "storage), GMRES basis storage; fp64: HSMG, weak divergence of u*, GMRES orthogonalisation/dots/H, "
                 "BDF/EXT state, residual checks, global reductions",
    "fp32b+fp16": "fp32b with fp16-stored geometry in the velocity operator and opgrad (fp32 arithmetic)",
    "fp32b+fp16c": "fp32b with the velocity operator in 16-bit arithmetic (fp16 operands, fp32 sums) on fp16 "
                   "geometry",
    "fp32b+fp16pc": "fp32b with the pressure operator in 16-bit arithmetic (fp16 operands, fp32 sums) on fp16 "
                    "geometry",
}


def oracle_series(nel, N, dt, re, vtol, ptol, hsmg, dealias, cfl, proj):
    """The FP64 oracle's stored series of the same workload (written by
    tests/golden/make_tgv_series.py, which runs only the CPU oracle), or None
    when no stored series matches the workload."""
    if dealias or cfl > 0 or proj or not hsmg:
        return None
    for name in ("tgv32_n7", "tgv16_n11"):
        path = os.path.join(GOLDEN, "oracle_series_%s.json" % name)
        if not os.path.exists(path):
            continue
        with open(path) as fh:
            d = json.load(fh)
        if (d["nel"], d["N"], d["dt"], d["re"], d["vel_tol"], d["pres_tol"]) == (nel, N, dt, re, vtol, ptol):
            return d
    return None


def error_vs_oracle(series, ref):
    """Sec. 4.2 error metrics of a GPU series (t, KE, enstrophy, max|div|) against
    the oracle's series over the steps both hold (the denominators are the
    maxima of the oracle series over those steps)."""
    from oracle.metrics import e_max, e_peak
    rows = ref["series"]
    n = min(len(series), len(rows))
    assert all(abs(series[k][0] - rows[k]["t"]) <= 1e-12 for k in range(n)), "time levels differ"
    ke, ke_o = [series[k][1] for k in range(n)], [rows[k]["ke"] for k in range(n)]
    en, en_o = [series[k][2] for k in range(n)], [rows[k]["enst"] for k in range(n)]
    return {"e_E_max_pct": e_max(ke, ke_o), "e_Omega_max_pct": e_max(en, en_o),
            "e_Omega_peak_pct": e_peak(en, en_o),
            "max_div_diff": max(abs(series[k][3] - rows[k]["maxdiv"]) for k in range(n)),
            "max_div_oracle": max(rows[k]["maxdiv"] for k in range(n)), "steps_compared": n - 1}


def cpu_baseline(nel, N, nu, dt, pres_iters_per_step, restart=30, hsmg=0):
    """FP64 oracle on the host cores, on a bounded sample of the same workload.

    Sample: (a) the oracle's first fluid step from the initial condition (all
    operators, three velocity solves and its pressure solve, with p0
    iterations), and (b) when the timed GPU steps average p > p0 pressure
    iterations, one full GMRES(restart) cycle of the oracle's pressure solver
    (same preconditioner) on the same mesh.  A steady step is (a) plus
    (p - p0)/restart cycles of (b) (the oracle's counts equal the GPU's by the
    parity tests); steps/s = 1 / that time.  With p <= p0 the first step alone
    is the (pessimistic) estimate.
    """
    import numpy as np
    from oracle import OracleMesh, OracleFluid, OracleHSMG, num_threads
    m = OracleMesh(nel, N)
    f = OracleFluid(m, nu, dt, hsmg=bool(hsmg))
    t0 = time.perf_counter()
    o = f.step()
    t_step = time.perf_counter() - t0
    its, t_cycle = restart, 0.0
    if pres_iters_per_step > o["pit"]:
        # the steady step needs more pressure iterations than the first: time a cycle
        rhs = m.remove_mean_unique(m.dssum(m.mass() * np.random.default_rng(0).standard_normal(m.np)))
        t0 = time.perf_counter()
        if hsmg:
            _, its, _ = OracleHSMG(m).poisson(rhs, tol=1e-30, maxit=restart, restart=restart)
        else:
            _, its, _ = m.gmres(rhs, 1.0, 0.0, tol=1e-30, maxit=restart, restart=restart)
        t_cycle = time.perf_counter() - t0
    t_est = t_step + max(pres_iters_per_step - o["pit"], 0.0) / its * t_cycle
    return {"value": 1.0 / t_est, "unit": "steps/s", "cores": num_threads(), "kind": "oracle",
            "sample": ("oracle first step of the same workload (%.2f s, %d pressure its, %s preconditioner)"
                       % (t_step, o["pit"], "HSMG" if hsmg else "Jacobi"))
                      + ("; + one %d-iteration GMRES cycle on the same mesh (%.2f s); steady step = first step + "
                         "(%.1f - %d)/%d cycles" % (its, t_cycle, pres_iters_per_step, o["pit"], its)
                         if t_cycle > 0 else
                         "; the timed GPU steps average %.1f pressure its, no more than the first step's, so the "
                         "first step is the estimate" % pres_iters_per_step)}


def calib_copies(torch):
    """Plain device copies of known size: what the PMC byte counters read for
    exactly 1 GiB read + 1 GiB written per dispatch."""
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    b_ = torch.empty_like(a)
    for _ in range(3):
        b_.copy_(a)
    torch.cuda.synchronize()
    del a, b_


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--vtol", type=float, default=1e-6)
    ap.add_argument("--ptol", type=float, default=1e-4)
    ap.add_argument("--proj", type=int, default=0, help="pressure projection space (0 = off; the paper uses 20)")
    ap.add_argument("--cfl", type=float, default=0.0,
                    help="> 0: adaptive dt toward this CFL number, --dt the largest step (the paper uses 0.4)")
    ap.add_argument("--hsmg", type=int, default=1, choices=[0, 1],
                    help="pressure preconditioner: 1 HSMG (the paper's runs use HSMG; default), 0 Jacobi")
    ap.add_argument("--other-pc", type=int, default=1, choices=[0, 1],
                    help="also run the workload with the other pressure preconditioner in both tiers "
                         "(the jacobi_leg or hsmg_leg record)")
    ap.add_argument("--dealias", type=int, default=0, choices=[0, 1],
                    help="1: convection on the 3/2-rule Gauss-Legendre grid (the paper's runs are dealiased)")
    ap.add_argument("--prof", default="ax_resid",
                    choices=["ax_resid", "ax_presid", "ax_vel", "ax_pres", "gm_upd_dots", "gm_upd_norm", "conv",
                             "hsmg", "none"],
                    help="kernel class timed with HIP events for the roofline record (default: the dominant kernel)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="finish with plain 1 GiB device copies (calibration of the PMC byte counters)")
    ap.add_argument("--graph", type=int, default=0, choices=[0, 1],
                    help="1: every step replayed as a HIP graph (sem_fluid_step_graph), in every tier")
    ap.add_argument("--tier", default="fp32b-p32",
                    help="headline tier (default: the fp32-bounded tier as the 32^3 workload defines it)")
    ap.add_argument("--nel", type=int, default=32)
    ap.add_argument("--order", type=int, default=7)
    ap.add_argument("--dt", type=float, default=5e-4)
    ap.add_argument("--re", type=float, default=1600.0)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ax", action="store_true")
    ap.add_argument("--ax-only", action="store_true",
                    help="run only the operator/dssum leg on the 64^3 deformed mesh (for kernel profiling)")
    ap.add_argument("--serve", type=int, default=256,
                    help="requests of the serving leg (seeded TGV/Poisson stream; 0 = skip)")
    ap.add_argument("--serve-loads", default="0.4,0.7,1.0", help="serving: fractions of the saturated rate")
    ap.add_argument("--serve-streams", type=int, default=4, help="serving: worker streams (host threads), 1..4")
    ap.add_argument("--serve-graph", type=int, default=1, choices=[0, 1],
                    help="serving: TGV steps replayed as HIP graphs")
    ap.add_argument("--alt-tier", default="fp32b",
                    help="another tier run on the headline workload beside --tier ('' = skip)")
    ap.add_argument("--c4-steps", type=int, default=400,
                    help="steps of the 16^3, N = 11 leg in fp64, fp32b-p32, fp32b, fp32b+fp16 and fp32b+fp16c (0 = skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (a request's elements would be "
              "sharded by slabs of the box, with face exchanges around each dssum); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2608_24348_amd import sem
    from oracle.metrics import e_max, e_peak
    sem.load()
    if args.ax_only:
        from paper_2608_24348_amd import inputs
        res = {"ax_gdofs": ax_leg(sem, torch, inputs)}
        if args.calib_copy:
            calib_copies(torch)
        print(json.dumps(res), flush=True)
        return
    nel = (args.nel,) * 3
    N = args.order
    nu = 1.0 / args.re
    dt = args.dt
    npts = args.nel ** 3 * (N + 1) ** 3

    log("bench: %s  %d^3 elements N=%d (%d pts)  dt=%g  Re=%g" % (args.tier, args.nel, N, npts, dt, args.re))
    prof_class = {"ax_resid": sem.PROF_AX_RESID, "ax_presid": sem.PROF_AX_PRESID, "ax_vel": sem.PROF_AX_VEL,
                  "ax_pres": sem.PROF_AX_PRES,
                  "gm_upd_dots": sem.PROF_GM_UPD_DOTS,
                  "gm_upd_norm": sem.PROF_GM_UPD_NORM, "conv": sem.PROF_CONV, "hsmg": sem.PROF_HSMG,
                  "none": None}[args.prof]
    ctx, t_mx, st_mx, ser_mx, prof = run_tier(sem, torch, args.tier, nel, N, nu, dt, args.warmup, args.steps, prof_class,
                                              args.vtol, args.ptol, args.proj, args.dealias, args.cfl, args.hsmg,
                                              args.graph)
    steps_s = args.steps / t_mx
    out = {"metric": METRIC, "value": steps_s, "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * t_mx / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64" if args.tier != "fp64" else "f64",
           "data": "synthetic",
           "config": {"workload": "TGV Re=%g, %d^3 elements, N=%d (%d local pts), dt=%g, tier %s (%s)%s"
                                  % (args.re, args.nel, N, npts, dt, args.tier,
                                     TIER_NOTE.get(args.tier, "see sem.tier"),
                                                                                     (", dealiased convection"
                                                                                      if args.dealias else "")
                                                                                     + (", adaptive dt CFL %g" % args.cfl
                                                                                        if args.cfl > 0 else "")
                                                                                     + (", HSMG pressure preconditioner"
                                                                                        if args.hsmg else
                                                                                        ", Jacobi pressure preconditioner")),
                      "global_batch": 1, "seq_len": npts, "parallelism": "single-gpu"}}
    out["iters"] = {"vel": [s["vit"] for s in st_mx], "pres": [s["pit"] for s in st_mx]}
    out["step_launch"] = "hip graph per step (sem_fluid_step_graph)" if args.graph else "host-driven (sem_fluid_step)"
    if args.graph:
        out["graph_counts"] = ctx.graph_counts
    if args.cfl > 0:
        dts = [s["dt"] for s in st_mx]
        out["adaptive_dt"] = {"cfl_target": args.cfl, "dt_min": min(dts), "dt_max": max(dts),
                              "simulated_time": sum(dts), "simulated_time_per_s": sum(dts) / t_mx}

    if prof is not None and args.prof == "hsmg":
        # one record per preconditioner application of an Arnoldi step (11 launches)
        out["hsmg"] = {"applies": prof[1], "ms_per_apply": prof[0] / max(prof[1], 1)}
    elif prof is not None and not (args.proj and args.prof == "ax_presid"):
        # (the launch accounting of ax_presid covers the solver without projection)
        out["roofline"] = roofline(args.prof, args.tier, prof, st_mx, npts, out["config"]["workload"], N,
                                   args.dealias)

    if not args.no_fp64:
        ctx64, t64, st64, ser64, _ = run_tier(sem, torch, "fp64", nel, N, nu, dt, args.warmup, args.steps, None,
                                              args.vtol, args.ptol, args.proj, args.dealias, args.cfl, args.hsmg,
                                              args.graph)
        out["fp64_steps_per_s"] = args.steps / t64
        out["speedup_vs_fp64"] = steps_s / (args.steps / t64)
        ke_mx = [r[1] for r in ser_mx]
        ke64 = [r[1] for r in ser64]
        en_mx = [r[2] for r in ser_mx]
        en64 = [r[2] for r in ser64]
        out["error_vs_fp64_gpu"] = {"e_E_max_pct": e_max(ke_mx, ke64), "e_Omega_max_pct": e_max(en_mx, en64),
                                    "e_Omega_peak_pct": e_peak(en_mx, en64),
                                    "max_div_mx": max(r[3] for r in ser_mx), "max_div_fp64": max(r[3] for r in ser64),
                                    "steps_compared": len(ke64)}
        out["iters_fp64"] = {"vel": [s["vit"] for s in st64], "pres": [s["pit"] for s in st64]}
        del ctx64
    ref = oracle_series(args.nel, N, dt, args.re, args.vtol, args.ptol, args.hsmg, args.dealias, args.cfl, args.proj)
    if args.alt_tier and args.alt_tier != args.tier and not args.no_fp64:
        # the other fp32-bounded tier on the same workload (fp32b: fp64 arithmetic
        # in the pressure operator, Table 2's B-4 pattern)
        c32, t32, st32, ser32, _ = run_tier(sem, torch, args.alt_tier, nel, N, nu, dt, args.warmup, args.steps, None,
                                            args.vtol, args.ptol, args.proj, args.dealias, args.cfl, args.hsmg,
                                            args.graph)
        leg = {"tier": args.alt_tier, "note": TIER_NOTE.get(args.alt_tier, "see sem.tier"),
               "steps_per_s": args.steps / t32, "speedup_vs_fp64": (args.steps / t32) / out["fp64_steps_per_s"],
               "pres_iters_mean": sum(s["pit"] for s in st32) / len(st32)}
        if ref is not None:
            leg["error_vs_oracle"] = error_vs_oracle(ser32, ref)
        out["alt_tier_leg"] = leg
        del c32
    if ref is not None:
        ev = {"reference": "FP64 CPU oracle series, tests/golden/oracle_series_%s.json" % ref["workload"],
              args.tier: error_vs_oracle(ser_mx, ref)}
        if not args.no_fp64:
            ev["fp64"] = error_vs_oracle(ser64, ref)
        out["error_vs_oracle"] = ev
    del ctx
    torch.cuda.synchronize()
    if not args.no_fp64 and args.other_pc:
        # the same workload with the other pressure preconditioner (both tiers)
        other = 0 if args.hsmg else 1
        name = "hsmg_leg" if other else "jacobi_leg"
        # at least 200 steps: with Jacobi the pressure iteration counts swing
        # from step to step (1 to 40 at the loose absolute tolerance), so short
        # windows compare the tiers on a few counts (over the first 20 steps
        # fp32b averages 14.0 against fp64's 6.25; over 200, 10.3 against 9.8)
        nsteps = max(args.steps, 200)
        log("%s: the same workload, %s pressure preconditioner, %d steps"
            % (name, "HSMG" if other else "Jacobi", nsteps))
        leg = {}
        sers = {}
        for t in (args.tier, "fp64"):
            c_h, t_h, st_h, ser_h, _ = run_tier(sem, torch, t, nel, N, nu, dt, args.warmup, nsteps, None,
                                                args.vtol, args.ptol, args.proj, args.dealias, args.cfl, other,
                                                args.graph)
            leg[t] = {"steps_per_s": nsteps / t_h, "steps": nsteps,
                      "pres_iters_mean": sum(s["pit"] for s in st_h) / len(st_h)}
            sers[t] = ser_h
            del c_h
        hm, h64 = sers[args.tier], sers["fp64"]
        out[name] = {"tier": leg[args.tier], "fp64": leg["fp64"],
                     "speedup_vs_fp64": leg[args.tier]["steps_per_s"] / leg["fp64"]["steps_per_s"],
                     "headline_pres_iters_mean": sum(s["pit"] for s in st_mx) / len(st_mx),
                     "e_E_max_pct": e_max([r[1] for r in hm], [r[1] for r in h64]),
                     "e_Omega_max_pct": e_max([r[2] for r in hm], [r[2] for r in h64])}
        torch.cuda.synchronize()
    if not args.no_ax:
        from paper_2608_24348_amd import inputs
        torch.cuda.empty_cache()
        log("ax: 64^3 deformed mesh, every storage tier")
        out["ax_gdofs"] = ax_leg(sem, torch, inputs)
    if args.c4_steps > 0:
        log("c4: 16^3 elements N=11, %d steps per tier" % args.c4_steps)
        out["c4"] = c4_leg(sem, torch, args.c4_steps, graph=args.graph)
    if args.serve > 0:
        from paper_2608_24348_amd import serve
        loads = tuple(float(x) for x in args.serve_loads.split(","))
        log("serving: %d requests, burst then Poisson arrivals at %s x the burst rate" % (args.serve, loads))
        sv = serve.measure(args.serve, loads=loads, log=log, streams=args.serve_streams, graph=bool(args.serve_graph))
        sat = sv["saturated"]
        out["serving"] = {"requests": args.serve, "stream_seed": sv["seed"],
                          "workload": "TGV (20 steps) and Poisson (tol 1e-8) requests, n 4-24, N 5/7/9, "
                                      "Re 100-1600, tiers fp64/fp32b, HSMG where the order allows (>= 4), "
                                      "batched by (order, tier, kind, preconditioner)",
                          "streams": args.serve_streams, "graph_steps": bool(args.serve_graph),
                          "saturated_requests_per_s": sat["requests_per_s"], "saturated_gdof_per_s": sat["gdof_per_s"],
                          "saturated_ok": sat["ok"]}
        for f in loads:
            r = sv["load_%.1f" % f]
            out["serving"]["load_%.1f" % f] = {"qps": r["qps"], "p50_s": r.get("p50_s"), "p99_s": r.get("p99_s"),
                                               "requests_per_s": r["requests_per_s"], "gdof_per_s": r["gdof_per_s"],
                                               "ok": r["ok"]}
    if not args.no_cpu:
        log("cpu baseline: oracle sample of the same workload")
        pbar = sum(s["pit"] for s in st_mx) / len(st_mx)
        out["cpu_baseline"] = cpu_baseline(nel, N, nu, dt, pbar, hsmg=args.hsmg)
    if args.calib_copy:
        calib_copies(torch)
    out["time_breakdown_note"] = ("value = %d timed steps / wall time of %s (HIP event profiling of one kernel class on)"
                                  % (args.steps, "sem_fluid_step_graph" if args.graph else "sem_fluid_step"))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
