"""Pins of the oracle's RL-style step: the grasp selection and the dragging
constraint (Sec. III-A.2), the observations, the policy network and the tool
motion, and the step driver (Sec. III-B).  Values fixed by closed forms,
reductions to the plain stepping oracle and invariants."""
import ctypes

import numpy as np
import pytest

import oracle
import oracle.rl as R
from paper_2503_18616_amd import workloads as W

D = ctypes.POINTER(ctypes.c_double)


def dp(a):
    return a.ctypes.data_as(D)


def select(x, w, point, radius):
    lib = oracle._load()
    x = np.ascontiguousarray(x, np.float64)
    w = np.ascontiguousarray(w, np.float64)
    point = np.ascontiguousarray(point, np.float64)
    d2 = np.zeros(1)
    i = lib.oracle_grasp_select(len(w), dp(w), dp(x), dp(point), float(radius), dp(d2))
    return i, d2[0]


def drag(x, w, i, point):
    lib = oracle._load()
    x = np.ascontiguousarray(x, np.float64).copy()
    lib.oracle_project_drag(dp(x), dp(np.ascontiguousarray(w, np.float64)), int(i),
                            dp(np.ascontiguousarray(point, np.float64)))
    return x


# ------------------------------------------------------------ grasp selection
def test_grasp_select_closest_within_reach():
    x = np.array([[0.5, 0, 0], [0, 0.25, 0], [0, 0, -0.375], [0.125, 0, 0]], float)
    w = np.array([1.0, 1.0, 1.0, 0.0])            # particle 3 is pinned (closest, not eligible)
    assert select(x, w, [0, 0, 0], 0.3) == (1, 0.0625)
    assert select(x, w, [0, 0, 0], 0.25)[0] == -1   # reach is strict: |x - p| = r_l is out
    assert select(x, w, [0, 0, 0], 0.2)[0] == -1
    assert select(x, w, [0, 0, -0.25], 0.2) == (2, 0.015625)
    w[3] = 1.0
    assert select(x, w, [0, 0, 0], 0.3) == (3, 0.015625)


def test_grasp_select_tie_takes_lowest_id():
    x = np.array([[1.0, 0, 0], [0, 0.5, 0], [0, -0.5, 0], [0.5, 0, 0]], float)
    assert select(x, np.ones(4), [0, 0, 0], 1.0) == (1, 0.25)


def test_grasp_select_brute_force_cloud():
    rng = np.random.default_rng(5)
    for _ in range(50):
        n = int(rng.integers(1, 40))
        x = rng.uniform(-1, 1, (n, 3))
        w = (rng.uniform(size=n) < 0.7).astype(float)
        p = rng.uniform(-1, 1, 3)
        r = rng.uniform(0.1, 1.5)
        d2 = np.sum((x - p) ** 2, axis=1)
        ok = [i for i in range(n) if w[i] > 0 and d2[i] < r * r]
        want = min(ok, key=lambda i: (d2[i], i)) if ok else -1
        assert select(x, w, p, r)[0] == want


# ------------------------------------------------------------ drag constraint
def test_drag_moves_the_particle_onto_the_point():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(5, 3))
    w = np.array([1.0, 2.0, 0.5, 0.0, 1.0])
    p = np.array([0.3, -0.2, 0.7])
    for i in (0, 1, 2):
        y = drag(x, w, i, p)
        np.testing.assert_allclose(y[i], p, atol=1e-15)       # k_s = 1: the full correction
        others = [j for j in range(5) if j != i]
        assert np.array_equal(y[others], x[others])
    assert np.array_equal(drag(x, w, 3, p), x)                 # a pinned particle stays
    x[4] = p
    assert np.array_equal(drag(x, w, 4, p), x)                 # already on the point


def test_drag_is_the_distance_constraint_with_a_kinematic_end():
    """Eq. 1 with rest length 0, no compliance and a second end of inverse
    mass 0 (the dragging point) gives the same update."""
    lib = oracle._load()
    rng = np.random.default_rng(8)
    for _ in range(20):
        a, p = rng.normal(size=(2, 3))
        wa = rng.uniform(0.1, 3.0)
        x = np.ascontiguousarray(np.stack([a, p]))
        w = np.array([wa, 0.0])
        lam = np.zeros(1)
        lib.oracle_project_distance(dp(x), dp(w), 0, 1, 0.0, 0.0, dp(lam))
        y = drag(np.stack([a, p]), w, 0, p)
        np.testing.assert_allclose(y[0], x[0], atol=1e-15)
        assert np.array_equal(x[1], p)


# ------------------------------------------------------------ observations, policy, motion
def test_observation_layout():
    rest = np.arange(60, dtype=float).reshape(20, 3) * 1e-3
    tracked = np.array([19, 0, 5] + list(range(1, 5)) + list(range(6, 17)), np.int32)
    x = rest.copy()
    for j, p in enumerate(tracked):
        x[p] += [(j + 1) * 1e-4, -(j + 1) * 2e-4, (j + 1) * 3e-4]
    origin = (0.05, 0.03, 0.03)
    tools = np.array([[0.06, 0.03, 0.04], [0.05, 0.02, 0.03]])
    target = np.array([0.05, 0.05, 0.035])
    o = R.observe(x, rest, tools, target, 7, tracked, 20.0, origin)
    np.testing.assert_allclose(o[0:3], [0.2, 0.0, 0.2], atol=1e-15)
    np.testing.assert_allclose(o[3:6], [0.0, -0.2, 0.0], atol=1e-15)
    np.testing.assert_allclose(o[6:9], [0.0, 0.4, 0.1], atol=1e-15)
    assert o[9] == 1.0
    for j in range(18):
        np.testing.assert_allclose(o[10 + 3 * j:13 + 3 * j],
                                   [(j + 1) * 2e-3, -(j + 1) * 4e-3, (j + 1) * 6e-3], atol=1e-15)
    assert R.observe(x, rest, tools, target, -1, tracked, 20.0, origin)[9] == 0.0


def one_hot_net(path, gain=2.0, b1=0.0):
    """W1[u, k] = 1, W2[v, u] = 1, W3[o, v] = gain, everything else 0."""
    k, u, v, o = path
    flat = np.zeros(R.NUM_PARAMS, np.float32)
    H, F, A = R.HIDDEN, R.OBS, R.ACTIONS
    flat[u * F + k] = 1.0
    flat[H * F + u] = b1
    off2 = H * F + H
    flat[off2 + v * H + u] = 1.0
    off3 = off2 + H * H + H
    flat[off3 + o * H + v] = gain
    return R.unpack_policy(flat)


def test_policy_follows_one_path_through_the_layers():
    net = one_hot_net((12, 5, 7, 2), gain=2.0)
    o = np.zeros(64)
    o[12] = 0.75
    a = R.policy(net, o)
    want = np.zeros(7)
    want[2] = 1.5
    assert np.array_equal(a, want)
    o[12] = -0.75                         # relu of the first layer blocks it
    assert np.array_equal(R.policy(net, o), np.zeros(7))
    o[12] = 0.0
    o[13] = 1.0                           # a transposed W1 would read another input
    assert np.array_equal(R.policy(net, o), np.zeros(7))
    net = one_hot_net((12, 5, 7, 2), gain=2.0, b1=0.5)
    o[:] = 0.0
    o[12] = 0.25
    assert R.policy(net, o)[2] == 1.5     # bias of the first layer


def test_policy_rounds_inputs_and_hidden_values_to_bfloat16():
    net = one_hot_net((3, 0, 0, 6), gain=1.0)
    o = np.zeros(64)
    o[3] = 1.0 + 2.0 ** -8                # a tie: to even (1.0)
    assert R.policy(net, o)[6] == 1.0
    o[3] = 1.0 + 2.0 ** -8 + 2.0 ** -10   # above the tie: up
    assert R.policy(net, o)[6] == 1.0 + 2.0 ** -7
    # a product that is not a bfloat16 is rounded before the next layer
    flat = np.zeros(R.NUM_PARAMS, np.float32)
    flat[0 * 64 + 3] = 1.0 + 2.0 ** -7
    off2 = 256 * 64 + 256
    flat[off2 + 0] = 1.0
    flat[off2 + 256 * 256 + 256 + 6 * 256 + 0] = 1.0
    net = R.unpack_policy(flat)
    o[3] = 1.0 + 2.0 ** -7
    assert R.policy(net, o)[6] == 1.0 + 2.0 ** -6       # (1 + 2^-6 + 2^-14) rounded


def test_tool_motion_closed_form():
    rl = R.RlParams(0.01, (0, 0, 0), 0.05, 1.0, (0, 0, 0), (0.0, 0.0, 0.0), (0.1, 0.1, 0.1),
                    np.zeros(18, np.int32))
    tools = np.array([[0.05, 0.05, 0.05], [0.0999, 0.05, 0.0001]])
    a = np.array([2.0, -0.5, 0.0, 0.7, 0.0, -3.0, 0.0])
    dt = 0.1
    out = R.move_tools(tools, a, rl, dt)
    np.testing.assert_allclose(out[0], [0.05 + 0.005, 0.05 - 0.0025, 0.05], atol=1e-16)
    np.testing.assert_allclose(out[1], [0.1, 0.05, 0.0], atol=1e-16)   # clamped into the box


# ------------------------------------------------------------ the step driver
@pytest.fixture(scope="module")
def scene():
    m = W.slab_mesh(6, 4, 2)
    om = oracle.prepare_mesh(m.rest_pos, m.inv_mass, m.tets)
    lx, ly, lz = m.extent
    rl = R.RlParams(0.01, (0.0, 0.0, -W.TOOL_RADIUS), 0.05, 30.0, W.rl_origin(), *W.rl_box(),
                    W.rl_tracked(m))
    params = oracle.OracleParams(W.DT, 4, 3, W.GRAVITY, 2, (W.TOOL_RADIUS, W.TOOL_RADIUS))
    tools0 = np.array([[0.4 * lx, 0.5 * ly, lz + W.TOOL_RADIUS - 2e-3],
                       [0.7 * lx, 0.5 * ly, lz + W.TOOL_RADIUS - 2e-3]])
    target = np.array([0.5 * lx, 0.5 * ly, lz + 0.01])
    return m, om, rl, params, tools0, target


def constant_net(actions):
    """Zero weights, b3 = actions: every step takes the same actions."""
    flat = np.zeros(R.NUM_PARAMS, np.float32)
    flat[-R.ACTIONS:] = actions
    return R.unpack_policy(flat)


def test_open_grasper_reduces_to_the_plain_step(scene):
    m, om, rl, params, tools0, target = scene
    acts = np.array([0.5, -0.25, 2.0, -1.0, 0.5, -0.125, -1.0], np.float32)
    steps = 6
    res = R.run_env_rl(om, (1e-6, 1e-7), params, rl, constant_net(acts), tools0, target, steps)
    assert np.all(res.grasped == -1)
    path = np.empty((steps, 2, 3))
    t = tools0.copy()
    a64 = acts.astype(np.float64)
    for s in range(steps):
        for k in range(2):
            t[k] = np.clip(t[k] + np.clip(a64[3 * k:3 * k + 3], -1, 1) * rl.max_speed * params.dt,
                           rl.box_lo, rl.box_hi)
        path[s] = t
    np.testing.assert_allclose(res.tools, path, rtol=0, atol=1e-15)
    plain = oracle.run_env(om, (1e-6, 1e-7), params, path, steps)
    np.testing.assert_allclose(res.x, plain.x, atol=1e-13)
    np.testing.assert_allclose(res.v, plain.v, atol=1e-10)
    assert np.all(res.actions == acts.astype(np.float64))


def test_released_particle_is_not_dragged(scene):
    m, om, rl, params, tools0, target = scene
    acts = np.array([0, 0, 0.5, 0, 0, 0, -0.5], np.float32)
    held = int(rl.tracked[3])
    res = R.run_env_rl(om, (1e-6, 1e-7), params, rl, constant_net(acts), tools0, target, 3,
                       grasped0=held)
    assert np.all(res.grasped == -1)
    assert res.obs[0, 9] == 1.0 and np.all(res.obs[1:, 9] == 0.0)
    plain = oracle.run_env(om, (1e-6, 1e-7), params, res.tools, 3)
    np.testing.assert_allclose(res.x, plain.x, atol=1e-13)


def test_closed_grasper_lifts_the_closest_particle(scene):
    m, om, rl, params, tools0, target = scene
    acts = np.array([0, 0, 1.0, 0, 0, 0, 1.0], np.float32)      # grasper up at full speed
    steps = 5
    res = R.run_env_rl(om, (1e-6, 1e-7), params, rl, constant_net(acts), tools0, target, steps)
    point0 = res.tools[0, 0] + rl.grasp_offset
    d2 = np.sum((om.rest - point0) ** 2, axis=1)
    d2[om.w == 0] = np.inf
    want = int(np.argmin(d2))
    assert d2[want] < rl.grasp_radius ** 2
    assert np.all(res.grasped == want)
    assert np.all(res.obs[1:, 9] == 1.0) and res.obs[0, 9] == 0.0
    # the held particle ends every step on the dragging point
    np.testing.assert_allclose(res.x[want], res.tools[-1, 0] + rl.grasp_offset, atol=1e-15)
    lift = steps * rl.max_speed * params.dt
    assert res.x[want, 2] - om.rest[want, 2] > 0.5 * lift
    # neighbours follow upwards
    up = res.x[:, 2] - om.rest[:, 2]
    assert np.sum(up > 1e-4) > 3


def test_closed_grasper_keeps_what_it_holds(scene):
    m, om, rl, params, tools0, target = scene
    acts = np.array([0, 0, 0, 0, 0, 0, 1.0], np.float32)
    far = int(np.argmax(np.sum((om.rest - tools0[0]) ** 2, axis=1) * (om.w > 0)))
    res = R.run_env_rl(om, (1e-6, 1e-7), params, rl, constant_net(acts), tools0, target, 2,
                       grasped0=far)
    assert np.all(res.grasped == far)      # no new selection while holding
    np.testing.assert_allclose(res.x[far], tools0[0] + rl.grasp_offset, atol=1e-15)


def test_rl_generators():
    m = W.slab_mesh(12, 8, 3)
    tr = W.rl_tracked(m)
    assert tr.shape == (18,) and len(set(tr.tolist())) == 18
    assert np.all(m.rest_pos[tr, 2] == np.float32(m.extent[2])) and np.all(m.inv_mass[tr] > 0)
    tools, target = W.rl_start(50, 3)
    lo, hi = W.rl_box()
    assert np.all(tools >= np.float32(lo) - 1e-7) and np.all(tools <= np.float32(hi) + 1e-7)
    assert np.all(target[:, 2] > m.extent[2])
    again, _ = W.rl_start(5, 3, env_ids=[10, 11, 12, 13, 14])
    assert np.array_equal(again, tools[10:15])
    assert W.rl_policy_params(0).size == R.NUM_PARAMS


# ------------------------------------------------------------ learned warm start inside the step
def grasping_net():
    """Grasper up at half speed and closed; probe still."""
    return constant_net(np.array([0, 0, 0.5, 0, 0, 0, 1.0], np.float32))


@pytest.mark.parametrize("lo,hi,threshold,expect", [(3, 3, np.inf, 3), (2, 6, np.inf, 2),
                                                    (2, 6, -1.0, 6)])
def test_learned_driver_without_corrector_is_the_plain_step(scene, lo, hi, threshold, expect):
    m, om, rl, params, tools0, target = scene
    net = grasping_net()
    learned = R.RlLearned(None, lo, hi, threshold)
    got = R.run_env_rl(om, (1e-6, 1e-7), params, rl, net, tools0, target, 4, learned=learned)
    p = oracle.OracleParams(params.dt, params.substeps, expect, params.gravity, 2,
                            params.tool_radius)
    plain = R.run_env_rl(om, (1e-6, 1e-7), p, rl, net, tools0, target, 4)
    assert np.all(got.iterations == expect)
    assert np.array_equal(got.x, plain.x) and np.array_equal(got.v, plain.v)
    assert np.array_equal(got.grasped, plain.grasped) and np.all(got.grasped >= 0)


def test_learned_driver_stall_rule_and_corrector(scene):
    m, om, rl, params, tools0, target = scene
    net = grasping_net()
    # a corrector that moves nothing changes nothing
    zero = R.RlLearned(lambda xp, vs, xh, nbr: np.zeros_like(xh), 2, 6, -1.0, stall_ratio=0.9)
    none = R.RlLearned(None, 2, 6, -1.0, stall_ratio=0.9)
    a = R.run_env_rl(om, (1e-6, 1e-7), params, rl, net, tools0, target, 4, learned=zero)
    b = R.run_env_rl(om, (1e-6, 1e-7), params, rl, net, tools0, target, 4, learned=none)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.iterations, b.iterations)
    assert set(np.unique(b.iterations)) <= {2, 6}
    # a stall ratio near 0 stops every substep at the minimum (no sweep lowers
    # the residual a trillionfold); with ratio 1 only the sweeps that raised
    # the residual stop, and the grasper's drag makes some do
    least = R.run_env_rl(om, (1e-6, 1e-7), params, rl, net, tools0, target, 2,
                         learned=R.RlLearned(None, 2, 6, -1.0, stall_ratio=1e-12))
    one = R.run_env_rl(om, (1e-6, 1e-7), params, rl, net, tools0, target, 2,
                       learned=R.RlLearned(None, 2, 6, -1.0, stall_ratio=1.0))
    assert np.all(least.iterations == 2)
    assert set(np.unique(one.iterations)) == {2, 6}
    # the held particle still ends every step on the dragging point
    g = int(b.grasped[-1])
    np.testing.assert_allclose(b.x[g], b.tools[-1, 0] + rl.grasp_offset, atol=1e-15)


def path_net(w1=1.0, w2=1.0, w3=1.0, b2=0.0, k=3, u=0, v=0, o=6):
    """One path input k -> unit u -> unit v -> output o with the given weights."""
    H, F = R.HIDDEN, R.OBS
    flat = np.zeros(R.NUM_PARAMS, np.float32)
    flat[u * F + k] = w1
    off2 = H * F + H
    flat[off2 + v * H + u] = w2
    flat[off2 + H * H + v] = b2
    off3 = off2 + H * H + H
    flat[off3 + o * H + v] = w3
    return R.unpack_policy(flat)


def test_policy_relu_and_rounding_of_every_layer():
    o = np.zeros(64)
    # relu after layer 2: a negative second-layer value is blocked
    o[3] = 0.75
    assert R.policy(path_net(w2=-1.0), o)[6] == 0.0
    # the input is rounded: 1 + 2^-8 ties to 1, so 3 x input is 3, not 3.0117 -> 3.015625
    o[3] = 1.0 + 2.0 ** -8
    assert R.policy(path_net(w1=3.0), o)[6] == 3.0
    # the first hidden layer is rounded: (1 + 2^-7)^2 = 1 + 2^-6 + 2^-14 becomes 1 + 2^-6,
    # and with b2 = 2^-8 - 2^-6 the second layer lands exactly on the tie 1 + 2^-8,
    # which rounds to even (1); the unrounded value would sit above the tie (1 + 2^-7)
    o[3] = 1.0 + 2.0 ** -7
    net = path_net(w1=1.0 + 2.0 ** -7, b2=2.0 ** -8 - 2.0 ** -6)
    assert R.policy(net, o)[6] == 1.0


def test_learned_driver_adds_the_correction_to_the_prediction(scene):
    """Without sweeps a substep is the prediction plus the correction: with a
    constant correction c on free particles and zero start velocity, after K
    substeps v = K (h g + c / h) and x = x0 + h (h g + c / h) K (K + 1) / 2."""
    m, om, rl, params, tools0, target = scene
    c = np.array([1e-5, -2e-5, 3e-6])
    free = om.w > 0

    def corr(x_prev, v_start, x_hat, nbr):
        out = np.zeros_like(x_hat)
        out[free] = c
        return out
    net = constant_net(np.array([0, 0, 0, 0, 0, 0, -1.0], np.float32))
    res = R.run_env_rl(om, (1e-6, 1e-7), params, rl, net, tools0, target, 1,
                       learned=R.RlLearned(corr, 0, 0, np.inf))
    assert np.all(res.iterations == 0)
    K = params.substeps
    h = params.dt / K
    step = h * np.asarray(params.gravity) + c / h
    np.testing.assert_allclose(res.v[free], np.broadcast_to(K * step, res.v[free].shape), atol=1e-9)
    np.testing.assert_allclose(res.x[free], om.rest[free] + h * step * K * (K + 1) / 2, atol=1e-12)
    assert np.array_equal(res.x[~free], om.rest[~free])
