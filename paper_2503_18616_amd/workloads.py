"""Seeded synthetic inputs for the batched XPBD substep.

This module only *generates inputs*: grid vertex positions and tetrahedron
connectivity of a hexahedral tissue slab, per-vertex inverse masses (with the
bottom face pinned), per-environment compliances and per-environment tool
paths.  It contains none of the solver's arithmetic: rest lengths, rest
volumes, tetrahedron orientation, edge extraction and constraint colouring
are computed independently by the library and by the oracle from these raw
arrays.

The paper's scene is a tissue-retraction slab of about a thousand tetrahedra
fixed along one side (Sec. IV, Table II); no mesh file is published, so the
slab below stands in for it.  All units are SI (metres, kilograms, seconds).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# Slab extent shared by every workload: 10 x 6 x 3 cm.
SLAB_EXTENT = (0.10, 0.06, 0.03)
PARTICLE_MASS = 1.0e-3          # kg per particle
TOOL_RADIUS = 0.005             # m, kinematic sphere
GRAVITY = (0.0, 0.0, -9.81)     # m/s^2, z up
DT = 1.0 / 60.0                 # s per step
SUBSTEPS = 10

_STREAM_TOOL = 1
_STREAM_COMPLIANCE = 2
_STREAM_GRID = 3


@dataclass
class SlabMesh:
    """Raw slab: vertices, tetrahedra in generation order, inverse masses."""
    nx: int
    ny: int
    nz: int
    rest_pos: np.ndarray      # [V,3] float32
    tets: np.ndarray          # [T,4] int32, generation order (orientation NOT fixed)
    inv_mass: np.ndarray      # [V] float32, 0 on the z = 0 face
    extent: tuple = field(default=SLAB_EXTENT)

    @property
    def num_vertices(self) -> int:
        return int(self.rest_pos.shape[0])

    @property
    def num_tets(self) -> int:
        return int(self.tets.shape[0])


def vertex_id(i: int, j: int, k: int, nx: int, ny: int) -> int:
    """Vertex numbering of the grid: x fastest, then y, then z."""
    return (k * (ny + 1) + j) * (nx + 1) + i


def slab_mesh(nx: int, ny: int, nz: int, extent=SLAB_EXTENT,
              mass: float = PARTICLE_MASS, pin_bottom: bool = True) -> SlabMesh:
    """Hexahedral slab split into 5 tetrahedra per hexahedron.

    Each hex (i, j, k) contributes a central tetrahedron on its four corners
    of even global parity (i+j+k+dx+dy+dz even) and one corner tetrahedron
    per odd-parity corner together with that corner's three edge neighbours.
    Because the parity is global, the face diagonals of neighbouring hexes
    coincide and the mesh is conforming.  Vertex order inside a tetrahedron
    is the generation order; about half come out negatively oriented, which
    consumers must fix.
    """
    if min(nx, ny, nz) < 1:
        raise ValueError("grid resolution must be >= 1 in every axis")
    lx, ly, lz = extent
    ii, jj, kk = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1),
                             indexing="ij")
    # flatten with x fastest: order by (k, j, i)
    order = np.lexsort((ii.ravel(), jj.ravel(), kk.ravel()))
    gi, gj, gk = ii.ravel()[order], jj.ravel()[order], kk.ravel()[order]
    pos = np.stack([gi * (lx / nx), gj * (ly / ny), gk * (lz / nz)], axis=1)
    rest = pos.astype(np.float32)

    tets = []
    corners = [(dx, dy, dz) for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)]
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                vid = {c: vertex_id(i + c[0], j + c[1], k + c[2], nx, ny) for c in corners}
                even = [c for c in corners if (i + j + k + sum(c)) % 2 == 0]
                odd = [c for c in corners if (i + j + k + sum(c)) % 2 == 1]
                tets.append([vid[c] for c in even])
                for c in odd:
                    nbrs = [(1 - c[0], c[1], c[2]), (c[0], 1 - c[1], c[2]), (c[0], c[1], 1 - c[2])]
                    tets.append([vid[c]] + [vid[n] for n in nbrs])
    tets = np.asarray(tets, dtype=np.int32)

    inv_mass = np.full(rest.shape[0], 1.0 / mass, dtype=np.float32)
    if pin_bottom:
        inv_mass[gk == 0] = 0.0
    return SlabMesh(nx, ny, nz, rest, tets, inv_mass, tuple(extent))


def _env_rng(seed: int, stream: int, env: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(stream), int(env)]))


def log_uniform_compliance(num_envs: int, lo: float, hi: float, seed: int,
                           env_ids=None) -> np.ndarray:
    """Per-environment (edge, tet) compliances, each log-uniform in [lo, hi].

    Environment ``e`` always draws from its own stream, so a subset of
    environments reproduces exactly the values of the full batch.
    """
    env_ids = np.arange(num_envs) if env_ids is None else np.asarray(env_ids)
    out = np.empty((len(env_ids), 2), dtype=np.float32)
    for n, e in enumerate(env_ids):
        u = _env_rng(seed, _STREAM_COMPLIANCE, e).uniform(0.0, 1.0, size=2)
        out[n] = np.exp(np.log(lo) + u * (np.log(hi) - np.log(lo)))
    return out


def constant_compliance(num_envs: int, alpha_edge: float, alpha_tet: float) -> np.ndarray:
    out = np.empty((num_envs, 2), dtype=np.float32)
    out[:, 0] = alpha_edge
    out[:, 1] = alpha_tet
    return out


def tool_path(num_steps: int, num_envs: int, seed: int, extent=SLAB_EXTENT,
              radius: float = TOOL_RADIUS, num_tools: int = 1, env_ids=None,
              step_len: float = 1.0e-3, start_depth: float = 2.0e-3) -> np.ndarray:
    """Seeded random-walk sphere centres, float32 [num_steps][envs][tools][3].

    Start: slab centre in x, y, sphere pressed ``start_depth`` into the top
    face.  Each step moves by ``step_len * u`` with u ~ U[-1, 1]^3, clamped to
    x in [0.2, 0.8] Lx, y in [0.2, 0.8] Ly, z in [Lz - 8 mm, Lz + 10 mm].
    A second tool (if any) starts mirrored in x.  Environment ``e`` draws from
    its own stream.
    """
    lx, ly, lz = extent
    env_ids = np.arange(num_envs) if env_ids is None else np.asarray(env_ids)
    lo = np.array([0.2 * lx, 0.2 * ly, lz - 8.0e-3])
    hi = np.array([0.8 * lx, 0.8 * ly, lz + 10.0e-3])
    u = np.stack([_env_rng(seed, _STREAM_TOOL, e).uniform(-1.0, 1.0, size=(num_steps, num_tools, 3))
                  for e in env_ids], axis=1) if len(env_ids) else np.zeros((num_steps, 0, num_tools, 3))
    c = np.empty((len(env_ids), num_tools, 3))
    for t in range(num_tools):
        fx = 0.5 if num_tools == 1 else (0.35 if t == 0 else 0.65)
        c[:, t] = [fx * lx, 0.5 * ly, lz + radius - start_depth]
    out = np.empty((num_steps, len(env_ids), num_tools, 3), dtype=np.float32)
    for s in range(num_steps):
        c = np.clip(c + step_len * u[s], lo, hi)
        out[s] = c
    return out


def capsule_path(num_steps: int, num_envs: int, seed: int, length: float = 0.02,
                 radius: float = TOOL_RADIUS, start_depth: float = 6.0e-3,
                 env_ids=None) -> np.ndarray:
    """Capsule tools: the sphere walk of ``tool_path`` as the centre of a
    horizontal axis of ``length`` along x; float32 [num_steps][envs][1][6]
    (axis ends p0, p1)."""
    c = tool_path(num_steps, num_envs, seed, radius=radius, start_depth=start_depth,
                  env_ids=env_ids)[:, :, 0]
    half = np.array([length / 2, 0.0, 0.0], np.float32)
    return np.concatenate([c - half, c + half], axis=-1)[:, :, None, :].astype(np.float32)


def uneven_grids(num_envs: int, seed: int, nx=(6, 20), ny=(4, 12), nz=(2, 6)) -> np.ndarray:
    """Per-environment slab resolutions drawn uniformly from inclusive ranges."""
    out = np.empty((num_envs, 3), dtype=np.int32)
    for e in range(num_envs):
        r = _env_rng(seed, _STREAM_GRID, e)
        out[e] = [r.integers(nx[0], nx[1] + 1), r.integers(ny[0], ny[1] + 1),
                  r.integers(nz[0], nz[1] + 1)]
    return out


@dataclass
class Workload:
    """One named workload: mesh(es), per-env mesh id, compliances, solver settings."""
    name: str
    meshes: list
    env_mesh: np.ndarray      # [N] int32
    compliance: np.ndarray    # [N,2] float32
    iterations: int
    num_steps: int
    seed: int
    dt: float = DT
    substeps: int = SUBSTEPS
    gravity: tuple = GRAVITY
    num_tools: int = 1
    tool_radius: tuple = (TOOL_RADIUS, TOOL_RADIUS)

    @property
    def num_envs(self) -> int:
        return int(self.env_mesh.shape[0])

    def tools(self, num_steps=None, env_ids=None) -> np.ndarray:
        n = self.num_steps if num_steps is None else num_steps
        return tool_path(n, self.num_envs, self.seed, radius=self.tool_radius[0],
                         num_tools=self.num_tools, env_ids=env_ids)


def single_env_workload(seed: int = 0) -> Workload:
    """One environment, 8x5x3 slab (216 particles, 600 tets), compliances
    1e-6 (edge) / 1e-7 (tet), 4 iterations, 100 steps."""
    mesh = slab_mesh(8, 5, 3)
    return Workload("single-env-8x5x3", [mesh], np.zeros(1, np.int32),
                    constant_compliance(1, 1e-6, 1e-7), iterations=4, num_steps=100, seed=seed)


def batch_workload(num_envs: int = 1024, seed: int = 0, num_steps: int = 1000) -> Workload:
    """Identical 16x10x4 slabs (935 particles, 3200 tets), per-env compliances
    log-uniform in [1e-7, 1e-5], 8 iterations, 1000 steps."""
    mesh = slab_mesh(16, 10, 4)
    return Workload(f"batch-{num_envs}x16x10x4", [mesh], np.zeros(num_envs, np.int32),
                    log_uniform_compliance(num_envs, 1e-7, 1e-5, seed),
                    iterations=8, num_steps=num_steps, seed=seed)


def uneven_workload(num_envs: int = 4096, seed: int = 0, num_steps: int = 1000) -> Workload:
    """Slabs of per-environment resolutions nx in [6, 20], ny in [4, 12],
    nz in [2, 6] (105 to 1911 particles), one mesh per distinct resolution,
    per-env compliances log-uniform in [1e-7, 1e-5], 8 iterations."""
    grids = uneven_grids(num_envs, seed)
    keys = sorted({tuple(int(v) for v in g) for g in grids})
    index = {k: i for i, k in enumerate(keys)}
    meshes = [slab_mesh(*k) for k in keys]
    env_mesh = np.array([index[tuple(int(v) for v in g)] for g in grids], np.int32)
    return Workload(f"uneven-{num_envs}", meshes, env_mesh,
                    log_uniform_compliance(num_envs, 1e-7, 1e-5, seed),
                    iterations=8, num_steps=num_steps, seed=seed)



# ---------------------------------------------------------------- RL-style step
_STREAM_RL = 4

# Settings of the RL-style step: grasp reach r_l (the paper gives no value),
# dragging point at the bottom of the grasping sphere, tool speed at full
# action, observation scale (about +-1.5 across the slab) and origin (centre
# of the top face, ``rl_origin``) and the tools' workspace (``rl_box``).
RL_GRASP_RADIUS = 0.01
RL_GRASP_OFFSET = (0.0, 0.0, -TOOL_RADIUS)
RL_MAX_SPEED = 0.05
RL_OBS_SCALE = 30.0
RL_TRACKED = 18


def rl_origin(extent=SLAB_EXTENT):
    """Origin of the observed points: the centre of the slab's top face."""
    lx, ly, lz = extent
    return (0.5 * lx, 0.5 * ly, lz)


def rl_box(extent=SLAB_EXTENT):
    """Workspace of the tool centres: 5 % .. 95 % of the slab in x and y,
    8 mm below to 30 mm above its top face."""
    lx, ly, lz = extent
    return (0.05 * lx, 0.05 * ly, lz - 8.0e-3), (0.95 * lx, 0.95 * ly, lz + 30.0e-3)


def rl_workload(num_envs: int = 8192, seed: int = 0, num_steps: int = 100) -> Workload:
    """Identical 12x8x3 slabs (468 particles, 1440 tets), two sphere tools
    (grasp, probe), per-env compliances log-uniform in [1e-7, 1e-5],
    8 iterations, 10 substeps per 1/60 s step."""
    mesh = slab_mesh(12, 8, 3)
    return Workload(f"rl-{num_envs}x12x8x3", [mesh], np.zeros(num_envs, np.int32),
                    log_uniform_compliance(num_envs, 1e-7, 1e-5, seed),
                    iterations=8, num_steps=num_steps, seed=seed, num_tools=2)


def rl_tracked(mesh: SlabMesh, count: int = RL_TRACKED) -> np.ndarray:
    """Observed particles: a 6 x 3 lattice of top-face vertices spread evenly
    over the slab (int32 [18], vertex ids of ``vertex_id``)."""
    cols, rows = 6, count // 6
    ii = np.round(np.linspace(1, mesh.nx - 1, cols)).astype(int)
    jj = np.round(np.linspace(1, mesh.ny - 1, rows + 2)[1:-1]).astype(int)
    return np.array([vertex_id(int(i), int(j), mesh.nz, mesh.nx, mesh.ny)
                     for j in jj for i in ii], np.int32)


def rl_start(num_envs: int, seed: int, extent=SLAB_EXTENT, radius: float = TOOL_RADIUS,
             env_ids=None):
    """Per-environment start of the RL-style step: tool centres float32
    [envs][2][3] (grasper in the left half, probe in the right half, both
    pressed 2 mm into the top face) and target points float32 [envs][3]
    (5 to 20 mm above the top face).  Environment ``e`` draws from its own
    stream."""
    lx, ly, lz = extent
    env_ids = np.arange(num_envs) if env_ids is None else np.asarray(env_ids)
    tools = np.empty((len(env_ids), 2, 3), np.float32)
    target = np.empty((len(env_ids), 3), np.float32)
    for n, e in enumerate(env_ids):
        r = _env_rng(seed, _STREAM_RL, int(e))
        u = r.uniform(0.0, 1.0, size=7)
        z = lz + radius - 2.0e-3
        tools[n, 0] = [(0.25 + 0.2 * u[0]) * lx, (0.3 + 0.4 * u[1]) * ly, z]
        tools[n, 1] = [(0.55 + 0.2 * u[2]) * lx, (0.3 + 0.4 * u[3]) * ly, z]
        target[n] = [(0.2 + 0.6 * u[4]) * lx, (0.2 + 0.6 * u[5]) * ly, lz + 5.0e-3 + 15.0e-3 * u[6]]
    return tools, target


def rl_policy_params(seed: int, obs: int = 64, hidden: int = 256, actions: int = 7) -> np.ndarray:
    """Random-init policy, flat float32: W1 [256][64], b1, W2 [256][256], b2,
    W3 [7][256], b3; He-uniform weights, zero biases.  The rows of W2 and W3
    are shifted to zero mean: the inputs of those layers are non-negative, so
    rows with a common offset would give every environment the same sign of
    an action, and the grasp command would never differ between them."""
    r = np.random.default_rng([seed, _STREAM_RL])
    w2 = r.uniform(-1, 1, (hidden, hidden)) * np.sqrt(6.0 / hidden)
    w3 = r.uniform(-1, 1, (actions, hidden)) * np.sqrt(6.0 / hidden)
    w1 = r.uniform(-1, 1, hidden * obs) * np.sqrt(6.0 / obs)
    parts = [w1, np.zeros(hidden), (w2 - w2.mean(axis=1, keepdims=True)).ravel(), np.zeros(hidden),
             (w3 - w3.mean(axis=1, keepdims=True)).ravel(), np.zeros(actions)]
    return np.concatenate(parts).astype(np.float32)
