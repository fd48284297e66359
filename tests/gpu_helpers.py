"""Shared helpers of the GPU parity tests (comparison metrics and the
neighbourhood gather used for sampled one-step parity at full size)."""
import sys

import numpy as np


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def field_errors(gpu, ref):
    """Normalised max errors of rho, u and T.

    gpu: dict of arrays (rho, ux, uy, uz, T); ref: array [5][...] from the
    oracle.  rho is normalised by max |rho| (~1), the velocity components by
    the largest speed component of the reference, T by max |T|.
    """
    g = [np.asarray(gpu[k], dtype=np.float64) for k in ("rho", "ux", "uy", "uz", "T")]
    umax = max(np.max(np.abs(ref[k])) for k in (1, 2, 3))
    out = {
        "rho": np.max(np.abs(g[0] - ref[0])) / np.max(np.abs(ref[0])),
        "u": max(np.max(np.abs(g[k] - ref[k])) for k in (1, 2, 3)) / umax,
        "T": np.max(np.abs(g[4] - ref[4])) / np.max(np.abs(ref[4])),
        "rho_minus_1": np.max(np.abs(g[0] - ref[0])) / max(1e-300, np.max(np.abs(ref[0] - 1))),
    }
    return out


def to_np(t):
    return t.detach().cpu().numpy()


def neighbourhood_indices(pos, shape):
    """Linear indices [n][27] of the 3x3x3 neighbourhoods of cells pos [n][3]
    (x, y, z) on a [nz][ny][nx] grid, clamped into the grid, and a mask of
    the entries that are really inside."""
    nz, ny, nx = shape
    d = np.array([(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)])
    p = pos[:, None, :].astype(np.int64) + d[None, :, :]
    inside = ((p[..., 0] >= 0) & (p[..., 0] < nx) & (p[..., 1] >= 0) & (p[..., 1] < ny) &
              (p[..., 2] >= 0) & (p[..., 2] < nz))
    pc = np.stack([np.clip(p[..., 0], 0, nx - 1), np.clip(p[..., 1], 0, ny - 1),
                   np.clip(p[..., 2], 0, nz - 1)], axis=-1)
    idx = (pc[..., 2] * ny + pc[..., 1]) * nx + pc[..., 0]
    return idx, inside


def gather_neighbourhoods(cav, pos):
    """[n][27][15+q] FP64 populations of the neighbourhoods of pos (entries
    outside the grid are NaN; the oracle never reads them)."""
    idx, inside = neighbourhood_indices(pos, cav.shape)
    F, G = cav.gather_cells(idx.reshape(-1))
    F = to_np(F).reshape(len(pos), 27, 15)
    G = to_np(G).reshape(len(pos), 27, -1)
    nb = np.concatenate([F, G], axis=2)
    nb[~inside] = np.nan
    return nb


def cell_index(pos, shape):
    nz, ny, nx = shape
    return (pos[:, 2].astype(np.int64) * ny + pos[:, 1]) * nx + pos[:, 0]
