"""FP64 reference of the RL-style step (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module; the GPU library never calls it.

The paper couples its simulator to an RL library through a thin layer that,
once per simulation step, extracts the observations, applies the actions and
steps the simulation (Sec. III-B); its grasper holds tissue through a dragging
constraint (Sec. III-A.2).  This module writes that step out for one
environment with two sphere tools (tool 0 grasps, tool 1 probes) and a
randomly initialised policy network standing in for the RL agent.  One step:

1. Observation (64 values) of the start-of-step state; points are taken
   relative to ``obs_origin`` and every length is in metres times
   ``obs_scale``:
     o[0:3]   tool 0 centre          o[3:6]  tool 1 centre
     o[6:9]   the environment's target point
     o[9]     1 while the grasper holds a particle, else 0
     o[10+3j : 13+3j], j = 0..17, x_p - X_p of tracked particle p = tracked[j]
             (displacement from its rest position X_p).
2. Policy: a0 = bf16(o); a1 = bf16(relu(W1 a0 + b1)); a2 = bf16(relu(W2 a1 + b2));
   a = W3 a2 + b3 (64 -> 256 -> 256 -> 7, weights [out][in] rounded to
   bfloat16, biases float32, sums exact here).  bf16() rounds to the nearest
   bfloat16, ties to even, through float32 (the GPU holds float32 values
   before it rounds).
3. Tool motion: tool t moves by clamp(a[3t:3t+3], -1, 1) * max_speed * dt and
   its centre is then clamped into the box [box_lo, box_hi].
4. Grasp (reading R12 of the C oracle): a[6] > 0 closes the grasper.  Closed
   with nothing held: the free particle closest to the dragging point (tool 0
   centre + grasp_offset) strictly within grasp_radius, on the start-of-step
   positions, is taken (``oracle_grasp_select``); open: released; closed and
   holding: kept.
5. The simulation step (Alg. 1) with both spheres at their moved centres:
   contact candidates on the start-of-step positions (R6), then per substep
   the prediction, the Gauss-Seidel iterations (edges, tetrahedra, tool
   contacts: ``oracle_iterate``) each followed by the dragging constraint of
   the held particle (``oracle_project_drag``), and the velocity update.
   With ``learned`` (``RlLearned``) each substep follows the learned warm
   start of ``oracle.run_env_learned`` instead: the corrector's correction
   added to the prediction, the minimum sweeps, the residual check with the
   stall rule, the fallback sweeps (every sweep followed by the drag).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import OracleMesh, OracleParams, _dp, _f64, _i32, _ip, _load
from .warmstart import bf16

OBS = 64
HIDDEN = 256
ACTIONS = 7
TRACKED = 18
TOOLS = 2

# flat float32 parameter order: W1 [256][64], b1, W2 [256][256], b2, W3 [7][256], b3
_SHAPES = [(HIDDEN, OBS), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,), (ACTIONS, HIDDEN), (ACTIONS,)]
NUM_PARAMS = int(sum(np.prod(s) for s in _SHAPES))


@dataclass
class RlParams:
    grasp_radius: float          # r_l (m)
    grasp_offset: tuple          # dragging point relative to the tool 0 centre (m)
    max_speed: float             # m/s per axis at |action| >= 1
    obs_scale: float             # observation lengths are metres times this
    obs_origin: tuple            # observed points are relative to this point (m)
    box_lo: tuple                # tool centres are clamped into [box_lo, box_hi]
    box_hi: tuple
    tracked: np.ndarray          # int32 [18] observed particles


@dataclass
class PolicyNet:
    """Policy weights as the step uses them: bfloat16-rounded weights (as
    float64), float32 biases (as float64)."""
    w1: np.ndarray
    b1: np.ndarray
    w2: np.ndarray
    b2: np.ndarray
    w3: np.ndarray
    b3: np.ndarray


def unpack_policy(flat) -> PolicyNet:
    flat = np.asarray(flat, np.float32).ravel()
    if flat.size != NUM_PARAMS:
        raise ValueError(f"policy has {NUM_PARAMS} parameters, got {flat.size}")
    parts, at = [], 0
    for s in _SHAPES:
        n = int(np.prod(s))
        parts.append(flat[at:at + n].reshape(s).astype(np.float64))
        at += n
    w1, b1, w2, b2, w3, b3 = parts
    return PolicyNet(bf16(w1), b1, bf16(w2), b2, bf16(w3), b3)


def observe(x, rest, tools, target, grasped, tracked, obs_scale, obs_origin):
    """The 64 observations of one environment (float64)."""
    x = np.asarray(x, np.float64).reshape(-1, 3)
    rest = np.asarray(rest, np.float64).reshape(-1, 3)
    tools = np.asarray(tools, np.float64).reshape(TOOLS, 3)
    o = np.empty(OBS)
    origin = np.asarray(obs_origin, np.float64)
    o[0:3] = (tools[0] - origin) * obs_scale
    o[3:6] = (tools[1] - origin) * obs_scale
    o[6:9] = (np.asarray(target, np.float64) - origin) * obs_scale
    o[9] = 1.0 if grasped >= 0 else 0.0
    tr = np.asarray(tracked, np.int64)
    o[10:] = ((x[tr] - rest[tr]) * obs_scale).ravel()
    return o


def policy(net: PolicyNet, obs):
    """Actions [..., 7] of observations [..., 64]."""
    a0 = bf16(obs)
    a1 = bf16(np.maximum(a0 @ net.w1.T + net.b1, 0.0))
    a2 = bf16(np.maximum(a1 @ net.w2.T + net.b2, 0.0))
    return a2 @ net.w3.T + net.b3


def move_tools(tools, actions, rl: RlParams, dt):
    """Tool centres after one step's motion: [2][3]."""
    tools = np.asarray(tools, np.float64).reshape(TOOLS, 3)
    a = np.asarray(actions, np.float64)
    out = np.empty_like(tools)
    for t in range(TOOLS):
        v = np.clip(a[3 * t:3 * t + 3], -1.0, 1.0) * rl.max_speed
        out[t] = np.clip(tools[t] + v * dt, rl.box_lo, rl.box_hi)
    return out


@dataclass
class RlLearned:
    """The learned warm start's settings (see ``oracle.run_env_learned``)."""
    corrector: object            # (x_prev, v_start, x_hat, nbr) -> [V, 3], or None
    min_iterations: int
    max_iterations: int
    threshold: float
    stall_ratio: float = 0.0


@dataclass
class RlResult:
    x: np.ndarray                # [V][3] after the last step
    v: np.ndarray
    tools: np.ndarray            # [steps][2][3] tool centres each step ran with
    grasped: np.ndarray          # [steps] particle held during each step, -1 for none
    obs: np.ndarray              # [steps][64]
    actions: np.ndarray          # [steps][7]
    select_margin: np.ndarray    # [steps] relative gap of the grasp choice (inf: no choice made)
    iterations: np.ndarray = None  # [steps][substeps] sweeps (learned runs)


def _select_margin(x, w, point, radius):
    """Relative gap between the squared distance of the best free particle
    and both the runner-up and r_l^2 (how far the choice is from a tie)."""
    d2 = np.sum((np.asarray(x).reshape(-1, 3) - point) ** 2, axis=1)
    d2 = d2[np.asarray(w) > 0]
    r2 = radius * radius
    order = np.sort(d2)
    gaps = [abs(order[0] - r2)]
    if order.size > 1:
        gaps.append(order[1] - order[0])
    return min(gaps) / r2


def run_env_rl(mesh: OracleMesh, compliance, params: OracleParams, rl: RlParams, net: PolicyNet,
               tools0, target, num_steps, x0=None, v0=None, grasped0=-1,
               learned: RlLearned = None) -> RlResult:
    """Advance one environment by ``num_steps`` RL steps (module docstring)."""
    from . import warmstart as ws
    lib = _load()
    if params.num_tools != TOOLS:
        raise ValueError("the RL step has two tools")
    V, E, T = mesh.num_vertices, mesh.num_edges, mesh.num_tets
    x = _f64(mesh.rest if x0 is None else x0).reshape(V, 3).copy()
    v = np.zeros((V, 3)) if v0 is None else _f64(v0).reshape(V, 3).copy()
    tools = _f64(tools0).reshape(TOOLS, 3).copy()
    radius = _f64(np.asarray(params.tool_radius[:TOOLS]))
    grav = _f64(params.gravity)
    eptr, eorder, tptr, torder = (_i32(mesh.edge_ptr), _i32(mesh.edge_order),
                                  _i32(mesh.tet_ptr), _i32(mesh.tet_order))
    edges = _i32(mesh.edges if E else np.zeros((1, 2), np.int32))
    tets = _i32(mesh.tets if T else np.zeros((1, 4), np.int32))
    rlen = _f64(mesh.rest_length if E else np.ones(1))
    rv = _f64(mesh.rest_volume if T else np.ones(1))
    h = float(params.dt) / params.substeps
    atd, atv = float(compliance[0]) / (h * h), float(compliance[1]) / (h * h)
    lam = np.zeros(max(E + T, 1))
    cand = np.zeros((TOOLS, V), np.int32)
    ncand = (ctypes.c_int * TOOLS)()
    x_prev = np.zeros((V, 3))
    offset = _f64(rl.grasp_offset)
    g = int(grasped0)
    out_tools = np.zeros((num_steps, TOOLS, 3))
    out_g = np.zeros(num_steps, np.int32)
    out_obs = np.zeros((num_steps, OBS))
    out_act = np.zeros((num_steps, ACTIONS))
    margin = np.full(num_steps, np.inf)
    its = np.zeros((num_steps, params.substeps), np.int32)
    nbr = ws.axis_neighbours(mesh.rest) if learned is not None and learned.corrector else None
    r2 = np.zeros(2)

    def sweep(centres, g, point):
        lib.oracle_iterate(_dp(x), _dp(mesh.w), E, _ip(edges), _dp(rlen), _dp(rv),
                           _ip(tets), len(eptr) - 1, _ip(eptr),
                           _ip(eorder if eorder.size else np.zeros(1, np.int32)),
                           len(tptr) - 1, _ip(tptr),
                           _ip(torder if torder.size else np.zeros(1, np.int32)),
                           atd, atv, _dp(lam), V, TOOLS, _dp(centres), _dp(radius),
                           _ip(cand), ncand)
        if g >= 0:
            lib.oracle_project_drag(_dp(x), _dp(mesh.w), g, _dp(point))

    def residual():
        lib.oracle_residual(_dp(x), E, _ip(edges), _dp(rlen), T, _ip(tets), _dp(rv), atd, atv,
                            _dp(lam), _dp(r2))
        return float(r2[0])

    for step in range(num_steps):
        o = observe(x, mesh.rest, tools, target, g, rl.tracked, rl.obs_scale, rl.obs_origin)
        a = policy(net, o)
        tools = move_tools(tools, a, rl, float(params.dt))
        point = np.ascontiguousarray(tools[0] + offset)
        if not a[6] > 0.0:
            g = -1
        elif g < 0:
            g = int(lib.oracle_grasp_select(V, _dp(mesh.w), _dp(x), _dp(point),
                                            float(rl.grasp_radius), None))
            margin[step] = _select_margin(x, mesh.w, point, float(rl.grasp_radius))
        out_obs[step], out_act[step], out_tools[step], out_g[step] = o, a, tools, g
        centres = np.ascontiguousarray(tools)
        for t in range(TOOLS):
            row = np.ascontiguousarray(cand[t])
            ncand[t] = lib.oracle_candidates(V, _dp(mesh.w), _dp(x),
                                             _dp(np.ascontiguousarray(centres[t])),
                                             float(radius[t]), _ip(row))
            cand[t] = row
        for sub in range(params.substeps):
            v_start = v.copy()
            lib.oracle_predict(V, _dp(mesh.w), h, _dp(grav), _dp(x), _dp(v), _dp(x_prev))
            lam[:] = 0.0
            if learned is None:
                for _ in range(params.iterations):
                    sweep(centres, g, point)
                its[step, sub] = params.iterations
            else:
                if learned.corrector is not None:
                    x += learned.corrector(x_prev, v_start, x, nbr)
                n_it = 0
                lo, hi = learned.min_iterations, learned.max_iterations
                stall_check = learned.stall_ratio > 0.0 and lo >= 1 and hi > lo
                before = np.nan
                for _ in range(lo):
                    if stall_check and n_it == lo - 1:
                        before = residual()
                    sweep(centres, g, point)
                    n_it += 1
                if hi > lo:
                    rms = residual()
                    go_on = rms > learned.threshold
                    if go_on and stall_check:
                        go_on = rms <= learned.stall_ratio * before
                    while go_on and n_it < hi:
                        sweep(centres, g, point)
                        n_it += 1
                its[step, sub] = n_it
            lib.oracle_velocity(V, h, _dp(x), _dp(x_prev), _dp(v))
    return RlResult(x, v, out_tools, out_g, out_obs, out_act, margin, its)
