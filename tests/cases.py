"""Shared set-up of GPU-vs-oracle comparisons: the same seeded inputs go to
the HIP library (through the C ABI) and to the FP64 oracle."""
from __future__ import annotations

import numpy as np

from paper_2503_18616_amd import workloads as W

# parity gate: max per-particle position error of 1e-4 of the mesh extent
EXTENT = max(W.SLAB_EXTENT)
POS_TOL = 1e-4 * EXTENT


def f32(v):
    return float(np.float32(v))


def oracle_params(oracle, wl: W.Workload):
    return oracle.OracleParams(f32(wl.dt), wl.substeps, wl.iterations,
                               tuple(f32(g) for g in wl.gravity), wl.num_tools,
                               tuple(f32(r) for r in wl.tool_radius))


def lib_params(xp, wl: W.Workload, flags=0, block_size=0):
    return xp.make_params(wl.dt, wl.substeps, wl.iterations, wl.gravity, wl.num_tools,
                          wl.tool_radius, flags, block_size)


def lib_meshes(wl: W.Workload):
    return [(m.rest_pos, m.inv_mass, m.tets) for m in wl.meshes]


def oracle_meshes(oracle, wl: W.Workload):
    return [oracle.prepare_mesh(m.rest_pos, m.inv_mass, m.tets) for m in wl.meshes]


def env_block(arr, offsets, e):
    return arr[offsets[e]:offsets[e + 1]]


def max_position_error(gpu_x, oracle_x):
    return float(np.max(np.linalg.norm(np.asarray(gpu_x, np.float64) - oracle_x, axis=1)))


def contact_band(x, centre, radius, rel=1e-5):
    """Particles whose squared distance to the centre is within rel of (2r)^2:
    float32 and FP64 trajectories may classify them differently."""
    d2 = np.sum((np.asarray(x, np.float64) - np.asarray(centre, np.float64)) ** 2, axis=1)
    reach2 = (2.0 * radius) ** 2
    return np.nonzero(np.abs(d2 - reach2) <= rel * reach2)[0]
