"""Seeded synthetic workloads.  Shapes, sizes and parameter draws only; no
arithmetic of the method lives here, so the oracle side and the GPU side can
both take their inputs from this module.

The paper validates on a differentially heated cube of air (Pr = 0.71) at
Ra = 1e3..1e5 (Sec. 3); no dataset is involved.  The workloads below use that
setup at the sizes the benchmarks name.
"""
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class CavityCase:
    name: str
    n: int
    Ra: float
    Pr: float = 0.71
    u0: float = 0.05
    thermal_q: int = 7
    steps: int = 0


# The five workloads: small parity case, 64^3 steady case, 512^3 precision
# and throughput case, the 64-cavity batch and the warm-start set.
SMALL_PARITY = CavityCase("cavity16_ra1e3_2000", 16, 1e3, steps=2000)
STEADY_64 = CavityCase("cavity64_ra1e4_steady", 64, 1e4)
LARGE_512 = CavityCase("cavity512_ra1e6_d3q7", 512, 1e6, steps=10000)
LARGE_512_REF128 = CavityCase("cavity128_ra1e6_d3q7", 128, 1e6, steps=2500)


def perturbation(shape, q, seed, scale):
    """Seeded Gaussian perturbation field [q][*shape] (float64)."""
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal((q, *shape))


def smooth_field(shape, seed, amplitude, modes=3):
    """Seeded smooth random field on a [nz][ny][nx] grid: a sum of a few
    low sine modes with random amplitudes and phases."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    z, y, x = np.meshgrid((np.arange(nz) + 0.5) / nz, (np.arange(ny) + 0.5) / ny,
                          (np.arange(nx) + 0.5) / nx, indexing="ij")
    out = np.zeros(shape)
    for _ in range(modes):
        kx, ky, kz = rng.integers(1, 4, size=3)
        ph = rng.uniform(0, 2 * np.pi, size=3)
        out += rng.standard_normal() * (np.sin(np.pi * kx * x + ph[0]) *
                                        np.sin(np.pi * ky * y + ph[1]) *
                                        np.sin(np.pi * kz * z + ph[2]))
    return amplitude * out / max(1e-30, np.max(np.abs(out)))


def sample_cells(shape, n, seed, include_edges=True):
    """Seeded sample of cell coordinates [n][3] (x, y, z) of a [nz][ny][nx]
    grid; the first cells are the 8 corners, edge and face centres so that
    every wall case is covered."""
    nz, ny, nx = shape
    pts = []
    if include_edges:
        for z in (0, nz // 2, nz - 1):
            for y in (0, ny // 2, ny - 1):
                for x in (0, nx // 2, nx - 1):
                    pts.append((x, y, z))
    rng = np.random.default_rng(seed)
    while len(pts) < n:
        pts.append((int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))))
    return np.array(pts[:n], dtype=np.int32)


# Rate set of the uneven batch and the warm-start runs, which reach
# relaxation rates up to 1.98 (small boxes at Ra = 1e6): bulk rate 1, the
# Maxwellian fourth-order flow equilibrium, and the D3Q7 scalar lattice with
# c_sphi^2 = 1/4 (rest weight 1/4).  With c_sphi^2 = 1/3 the D3Q7 lattice
# has no rest population and 64^3 cavities at Ra >= 1e5 diverge.
STABLE_RATES = {"omega_bulk": 1.0, "fourth_maxwell": 1, "cs2_T": 0.25}


# Steady-state rule: max |T_n - T_(n-1000)| < 1e-8, or, when the residual
# has stalled for 10 checks below 1e-6 (16 units in the last place of
# T = 0.5 in FP32), the precision's floor.  A residual that has reached no
# new minimum for 30 checks while staying above 1e-6 ends the run as
# "stalled": the state came near a steady state and left it (measured on
# 64^3 and 128^3 cavities: runs that converge reach a new minimum at least
# every 15 checks).
STEADY_RULE = {"tol": 1e-8, "check_every": 1000, "plateau_checks": 10, "plateau_floor": 1e-6,
               "stall_checks": 30}


def batched_cavities(count=64, seed=1710, sizes=(32, 48, 64, 80, 96), log_ra=(3.0, 6.0)):
    """The uneven batch: edge lengths uniform over `sizes`, Ra log-uniform."""
    rng = np.random.default_rng(seed)
    n = rng.choice(np.array(sizes), size=count)
    ra = 10.0 ** rng.uniform(log_ra[0], log_ra[1], size=count)
    return [(int(a), float(b)) for a, b in zip(n, ra)]


def warm_start_rayleigh(count, seed, log_ra=(3.0, 6.0)):
    """Rayleigh numbers for the learned warm start (log-uniform)."""
    rng = np.random.default_rng(seed)
    return 10.0 ** rng.uniform(log_ra[0], log_ra[1], size=count)
