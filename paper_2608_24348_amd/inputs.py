"""Seeded synthetic inputs shared by the GPU path, its tests and the oracle.

This module only draws random numbers and lays them out; it contains none of
the method's arithmetic.  Random values that the method consumes are drawn
here and handed to both sides as inputs.

Recipe (all numpy PCG64 ``default_rng``):
  * deformation phases of the sinusoidal mesh perturbation: 9 values
    uniform in [0, 2 pi) from seed 2608;
  * continuous random fields: one N(0,1) value per unique periodic node,
    array shape (nz*N, ny*N, nx*N) indexed [gz, gy, gx]; seed 0 for "u",
    seed 1 for "v";
  * element-local random vectors (discontinuous across elements):
    N(0,1) per local point, shape (E*lx^3,);
  * request streams: see ``request_stream``.
"""
import math

import numpy as np

DEFORM_SEED = 2608
STREAM_SEED = 24348


def deform_phases(seed=DEFORM_SEED):
    """Nine phases in [0, 2 pi) for the sinusoidal node perturbation."""
    return np.random.default_rng(seed).uniform(0.0, 2.0 * math.pi, 9)


def lattice_normal(nel, N, seed):
    """N(0,1) per unique node of the periodic lattice, shape (nz N, ny N, nx N)."""
    nx, ny, nz = nel
    return np.random.default_rng(seed).standard_normal((nz * N, ny * N, nx * N))


def local_normal(nel, N, seed):
    """N(0,1) per element-local point, flat array of E*(N+1)^3 values."""
    nx, ny, nz = nel
    return np.random.default_rng(seed).standard_normal(nx * ny * nz * (N + 1) ** 3)


def request_stream(n_requests=256, qps=10.0, seed=STREAM_SEED, nmin=4, nmax=24, orders=(5, 7, 9),
                   re_range=(100.0, 1600.0), tiers=("fp64", "fp32b"), tgv_steps=20, dt=1e-3,
                   noise=1e-3):
    """A seeded stream of TGV and Poisson requests with Poisson arrivals.

    Each request: arrival time (exponential gaps at rate ``qps``), kind
    ('tgv' or 'poisson', probability 1/2 each), elements per direction
    n ~ U{nmin..nmax}, order N ~ U(orders), Re log-uniform on ``re_range``,
    tier ~ U(tiers), and a per-request noise seed for the Poisson rhs.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / qps)
        kind = "tgv" if rng.random() < 0.5 else "poisson"
        n = int(rng.integers(nmin, nmax + 1))
        N = int(orders[int(rng.integers(0, len(orders)))])
        re = float(math.exp(rng.uniform(math.log(re_range[0]), math.log(re_range[1]))))
        tier = tiers[int(rng.integers(0, len(tiers)))]
        out.append({"id": i, "arrival": t, "kind": kind, "nel": (n, n, n), "N": N, "Re": re,
                    "tier": tier, "steps": tgv_steps, "dt": dt, "noise": noise,
                    "noise_seed": int(rng.integers(0, 2 ** 31 - 1))})
    return out
