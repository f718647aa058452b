"""Pins of the oracle's learned warm start (no GPU).

The network, its loss gradient and Adam are checked against closed forms,
finite differences and homogeneity; bfloat16 rounding against torch's CPU
conversion; the features against the slab's grid structure; the learned
substep driver against the monolithic oracle run it must reduce to.
"""
import numpy as np
import pytest

import oracle
from oracle import warmstart as ws
from paper_2503_18616_amd import workloads as W
from tests import cases as K


def test_bf16_rounding_ties_to_even_and_matches_torch():
    import torch
    one = 1.0
    assert ws.bf16(one) == 1.0
    assert ws.bf16(1.0 + 2.0 ** -8) == 1.0                      # tie -> even (down)
    assert ws.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6      # tie -> even (up)
    assert ws.bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(20000) * 10.0 ** rng.uniform(-8, 4, 20000)).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ws.bf16(x), ref)


def test_axis_neighbours_follow_the_grid():
    nx, ny, nz = 4, 3, 2
    m = W.slab_mesh(nx, ny, nz)
    nbr = ws.axis_neighbours(m.rest_pos)

    def vid(i, j, k):
        return (k * (ny + 1) + j) * (nx + 1) + i
    for k in range(nz + 1):
        for j in range(ny + 1):
            for i in range(nx + 1):
                want = [vid(i - 1, j, k) if i > 0 else -1, vid(i + 1, j, k) if i < nx else -1,
                        vid(i, j - 1, k) if j > 0 else -1, vid(i, j + 1, k) if j < ny else -1,
                        vid(i, j, k - 1) if k > 0 else -1, vid(i, j, k + 1) if k < nz else -1]
                assert nbr[vid(i, j, k)].tolist() == want


def test_features_of_translations_and_a_hand_example():
    m = W.slab_mesh(3, 2, 1)
    rest = m.rest_pos.astype(np.float64)
    nbr = ws.axis_neighbours(rest)
    V = rest.shape[0]
    d = np.array([1e-3, -2e-3, 5e-4])
    v = np.tile([0.1, 0.0, -0.2], (V, 1))
    f = ws.features(rest, v, rest + d, rest, nbr)
    assert np.allclose(f[:, 0:3], d) and np.allclose(f[:, 3:6], v) and np.allclose(f[:, 6:9], d)
    assert np.all(f[:, 9:] == 0.0)          # a translation strains no axis pair
    # stretch along x by s: the +x neighbour offset grows by s * spacing, -x by -s * spacing
    s = 0.01
    x = rest.copy()
    x[:, 0] *= 1.0 + s
    f = ws.features(rest, np.zeros((V, 3)), x, rest, nbr)
    dx = np.diff(np.unique(rest[:, 0]))[0]
    for i in range(V):
        if nbr[i, 1] >= 0:
            assert np.allclose(f[i, 12:15], [s * dx, 0, 0])
        else:
            assert np.all(f[i, 12:15] == 0.0)
        if nbr[i, 0] >= 0:
            assert np.allclose(f[i, 9:12], [-s * dx, 0, 0])
        assert np.allclose(f[i, 15:27], 0.0)


def test_network_zero_weights_gives_bias_and_hand_example():
    net = ws.init_net(0)
    for p in (net.W1, net.W2, net.W3, net.b1, net.b2):
        p[...] = 0.0
    net.b3[:] = [0.5, -1.0, 2.0]
    y, _ = ws.forward(net, np.ones((4, ws.FEATURES)))
    assert np.array_equal(y, np.tile(net.b3, (4, 1)))
    # one active path: f0 -> unit 0 -> unit 0 -> output 1
    net.b3[:] = 0.0
    net.W1[0, 0] = 2.0
    net.W2[0, 0] = 3.0
    net.W3[1, 0] = -0.5
    f = np.zeros((2, ws.FEATURES))
    f[0, 0], f[1, 0] = 1.5, -1.5
    y, _ = ws.forward(net, f, emulate_bf16=False)
    assert np.allclose(y, [[0.0, -4.5, 0.0], [0.0, 0.0, 0.0]])


def test_correction_clamps_the_output_and_skips_pinned_particles():
    net = ws.init_net(0, out_scale=np.array([1e-3, 2e-3, 3e-3]))
    for p in (net.W1, net.W2, net.W3, net.b1, net.b2):
        p[...] = 0.0
    net.b3[:] = [20.0, -3.0, -9.0]
    c = ws.correction(net, np.zeros((3, ws.FEATURES)), np.array([True, False, True]))
    assert np.allclose(c, [[8e-3, -6e-3, -24e-3], [0.0, 0.0, 0.0], [8e-3, -6e-3, -24e-3]])


def test_network_is_positively_homogeneous_without_biases():
    net = ws.init_net(1)
    rng = np.random.default_rng(2)
    f = rng.standard_normal((16, ws.FEATURES))
    y1, _ = ws.forward(net, f, emulate_bf16=False)
    y2, _ = ws.forward(net, 3.0 * f, emulate_bf16=False)
    assert np.allclose(y2, 3.0 * y1, rtol=1e-12, atol=1e-12)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(3)
    net = ws.init_net(4)
    for b in (net.b1, net.b2, net.b3):
        b[:] = rng.standard_normal(b.shape) * 0.1
    f = rng.standard_normal((12, ws.FEATURES))
    t = rng.standard_normal((12, 3))
    mask = rng.random(12) > 0.25
    loss, grads = ws.loss_and_grads(net, f, t, mask, emulate_bf16=False)
    eps = 1e-6
    for p, g in zip(net.params(), grads):
        flat = p.reshape(-1)
        for idx in rng.choice(flat.size, size=min(12, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp, _ = ws.loss_and_grads(net, f, t, mask, emulate_bf16=False)
            flat[idx] = old - eps
            lm, _ = ws.loss_and_grads(net, f, t, mask, emulate_bf16=False)
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - g.reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(fd)), (p.shape, idx)


def test_masked_particles_do_not_contribute():
    rng = np.random.default_rng(5)
    net = ws.init_net(6)
    f = rng.standard_normal((8, ws.FEATURES))
    t = rng.standard_normal((8, 3))
    mask = np.array([1, 1, 0, 1, 0, 1, 1, 0], bool)
    l1, g1 = ws.loss_and_grads(net, f, t, mask)
    l2, g2 = ws.loss_and_grads(net, f[mask], t[mask], np.ones(mask.sum(), bool))
    assert np.isclose(l1, l2)
    for a, b in zip(g1, g2):
        assert np.allclose(a, b, rtol=1e-12, atol=1e-15)


def test_adam_first_step_moves_by_lr_against_the_gradient_sign():
    p = [np.array([1.0, -2.0, 3.0])]
    g = [np.array([0.5, -4.0, 1e-3])]
    opt = ws.Adam(lr=0.01, eps=1e-12)
    opt.step(p, g)
    assert np.allclose(p[0], [1.0 - 0.01, -2.0 + 0.01, 3.0 - 0.01], rtol=0, atol=1e-9)


def test_adam_constant_gradient_has_unbiased_moments():
    """With the same gradient g every step, the bias-corrected moments are g
    and g^2 exactly (Kingma and Ba 2015, Sec. 3), so every step moves by
    lr g / (|g| + eps), for any beta1 and beta2."""
    g = np.array([0.5, -4.0, 2e-3, 0.0])
    for beta1, beta2 in ((0.9, 0.999), (0.5, 0.9)):
        p = [np.array([1.0, -2.0, 3.0, 0.25])]
        opt = ws.Adam(lr=0.01, beta1=beta1, beta2=beta2, eps=1e-6)
        for t in range(1, 6):
            before = p[0].copy()
            opt.step(p, [g.copy()])
            assert np.allclose(p[0], before - 0.01 * g / (np.abs(g) + 1e-6), rtol=0, atol=1e-14)


def test_adam_moments_are_the_bias_corrected_exponential_averages():
    """Five steps of varying gradients against the non-recursive form of
    Adam's moments: m_t = (1 - b1) sum_k b1^(t-k) g_k and v_t = (1 - b2)
    sum_k b2^(t-k) g_k^2, divided by 1 - b1^t and 1 - b2^t (Kingma and Ba
    2015, Alg. 1 and Sec. 3).  A missing accumulation of either moment, a
    wrong decay or a missing bias correction changes the second step on."""
    rng = np.random.default_rng(9)
    grads = [rng.normal(size=6) * rng.uniform(0.01, 3.0, size=6) for _ in range(5)]
    lr, b1, b2, eps = 0.01, 0.9, 0.999, 1e-8
    p = [np.linspace(-1.0, 1.0, 6)]
    want = p[0].copy()
    opt = ws.Adam(lr=lr, beta1=b1, beta2=b2, eps=eps)
    for t in range(1, 6):
        opt.step(p, [grads[t - 1].copy()])
        m = sum((1 - b1) * b1 ** (t - k) * grads[k - 1] for k in range(1, t + 1))
        v = sum((1 - b2) * b2 ** (t - k) * grads[k - 1] ** 2 for k in range(1, t + 1))
        want = want - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
        np.testing.assert_allclose(p[0], want, rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(opt.m[0], m, rtol=1e-13, atol=1e-16)
        np.testing.assert_allclose(opt.v[0], v, rtol=1e-13, atol=1e-18)


@pytest.fixture(scope="module")
def small():
    wl = W.single_env_workload(seed=0)
    om = K.oracle_meshes(oracle, wl)[0]
    return wl, om, K.oracle_params(oracle, wl), W.tool_path(12, 1, 0, start_depth=6e-3)


def test_learned_driver_without_corrector_is_the_plain_run(small):
    wl, om, P, tools = small
    ref = oracle.run_env(om, wl.compliance[0], P, tools[:, 0], 12, want_residual=True)
    r = oracle.run_env_learned(om, wl.compliance[0], P, tools[:, 0], 12, None,
                               wl.iterations, wl.iterations, np.inf)
    assert np.array_equal(r.x, ref.x) and np.array_equal(r.v, ref.v)
    assert np.array_equal(r.residual, ref.residual)
    assert np.all(r.iterations == wl.iterations)
    # a threshold below every residual always falls back to the full count
    r = oracle.run_env_learned(om, wl.compliance[0], P, tools[:, 0], 12, None, 1,
                               wl.iterations, -1.0)
    assert np.array_equal(r.x, ref.x) and np.all(r.iterations == wl.iterations)


def test_exact_corrector_needs_no_fallback(small):
    """A corrector that returns the converged correction of every substep leaves a
    residual below that of the plain solver after fewer sweeps."""
    wl, om, P, tools = small
    steps = 6
    tools = tools[:steps]
    ref = oracle.run_env(om, wl.compliance[0], P, tools[:, 0], steps, want_residual=True)
    plain = oracle.run_env_learned(om, wl.compliance[0], P, tools[:, 0], steps, None, 1,
                                   wl.iterations, -1.0)

    # the corrector replays a 40-sweep solve of the same substep from the same state
    def corrector(x_prev, v_start, x_hat, nbr):
        sub = oracle.run_env_learned(om, wl.compliance[0],
                                     oracle.OracleParams(P.dt / P.substeps, 1, 40, P.gravity,
                                                         0, P.tool_radius),
                                     None, 1, None, 40, 40, np.inf, x0=x_prev, v0=v_start)
        c = sub.x - x_hat
        return np.where(om.w[:, None] > 0, c, 0.0)
    thr = float(np.median(ref.residual[:, :, 0]))
    lr = oracle.run_env_learned(om, wl.compliance[0], P, tools[:, 0], steps, corrector, 1,
                                wl.iterations, thr)
    assert lr.iterations.mean() < plain.iterations.mean()
    assert np.all(lr.residual[:, :, 0][lr.iterations == 1] <= thr)


def test_stall_rule_limits(small):
    """The stall rule's two limits are plain runs: a ratio no sweep can exceed
    never stops the further sweeps (the extra evaluation leaves the state
    untouched), and a tiny ratio always does, which is a run with the minimum
    number of sweeps."""
    wl, om, P, tools = small
    full = oracle.run_env_learned(om, wl.compliance[0], P, tools[:, 0], 12, None, 2,
                                  wl.iterations, -1.0)
    never = oracle.run_env_learned(om, wl.compliance[0], P, tools[:, 0], 12, None, 2,
                                   wl.iterations, -1.0, stall_ratio=1e300)
    assert np.array_equal(never.x, full.x) and np.all(never.iterations == wl.iterations)
    always = oracle.run_env_learned(om, wl.compliance[0], P, tools[:, 0], 12, None, 2,
                                    wl.iterations, -1.0, stall_ratio=1e-300)
    two = oracle.run_env_learned(om, wl.compliance[0], P, tools[:, 0], 12, None, 2, 2, np.inf)
    assert np.all(always.iterations == 2)
    assert np.array_equal(always.x, two.x) and np.array_equal(always.v, two.v)


def test_stall_rule_decisions_follow_the_recorded_residuals(small):
    """The further sweeps ran exactly where the residual after the minimum was
    above the threshold and the last of the minimum sweeps had lowered it to at
    most stall_ratio times the value before it."""
    wl, om, P, tools = small
    stall, thr = 0.9, 2e-4
    r = oracle.run_env_learned(om, wl.compliance[0], P, tools[:, 0], 12, None, 2,
                               wl.iterations, thr, stall_ratio=stall)
    c = r.checks
    go_on = (c[:, :, 2] > thr) & (c[:, :, 2] <= stall * c[:, :, 1])
    assert np.array_equal(r.iterations, np.where(go_on, wl.iterations, 2))
    assert 0 < go_on.sum() < go_on.size
