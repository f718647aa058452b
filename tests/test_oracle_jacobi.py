"""Pins of the oracle's Jacobi iteration, the paper's own parallel solver
(Sec. III-A.1, Alg. 1): every constraint projected from the same positions,
the corrections summed per particle and divided by its number of
constraints n.  Values fixed by hand or by closed forms, not by the
implementation."""
import numpy as np
import pytest

import oracle
from paper_2503_18616_amd import workloads as W

H = 1.0 / 600.0


def params(**kw):
    base = dict(dt=1 / 60, substeps=10, iterations=1, gravity=(0.0, 0.0, -9.81), num_tools=0,
                tool_radius=(0.005, 0.005))
    base.update(kw)
    return oracle.OracleParams(base["dt"], base["substeps"], base["iterations"],
                               tuple(base["gravity"]), base["num_tools"],
                               tuple(base["tool_radius"]))


def test_chain_hand_example():
    """Three free particles on the x axis, edges of rest lengths 1 and 0.8:
    from the same positions edge ab moves a by +0.1 and b by -0.1, edge bc
    moves b by +0.2 and c by -0.2; b, in two constraints, takes the mean."""
    x = np.array([[0.0, 0, 0], [1.2, 0, 0], [2.4, 0, 0]])
    x, lam = oracle.iterate_jacobi(x, np.ones(3), [[0, 1], [1, 2]], [1.0, 0.8], [], [])
    np.testing.assert_allclose(x[:, 0], [0.1, 1.25, 2.2], rtol=0, atol=1e-15)
    np.testing.assert_allclose(lam[:2], [-0.1, -0.2], rtol=0, atol=1e-15)
    assert np.all(x[:, 1:] == 0.0)


def test_star_moves_by_the_mean_correction():
    """A free particle tied to three pinned anchors along the axes, each edge
    stretched by 0.1: each edge alone would move it 0.1 towards its anchor;
    together it moves by their mean, 0.1/3 along every axis."""
    x = np.array([[0.0, 0, 0], [1.1, 0, 0], [0, 1.1, 0], [0, 0, 1.1]])
    w = np.array([1.0, 0, 0, 0])
    x, _ = oracle.iterate_jacobi(x, w, [[0, 1], [0, 2], [0, 3]], [1.0] * 3, [], [])
    np.testing.assert_allclose(x[0], [0.1 / 3] * 3, rtol=0, atol=1e-15)
    np.testing.assert_array_equal(x[1:], [[1.1, 0, 0], [0, 1.1, 0], [0, 0, 1.1]])


def test_single_tetrahedron_newton_step():
    """A regular tetrahedron scaled by sigma with only its volume constraint
    (n = 1 for every vertex): one iteration rescales it to the Newton iterate
    of sigma^3 = 1, sigma - (sigma^3 - 1) / (3 sigma^2)."""
    reg = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float) / np.sqrt(8.0)
    v0 = abs(np.linalg.det(np.stack([reg[1] - reg[0], reg[2] - reg[0], reg[3] - reg[0]]))) / 6
    q = [0, 1, 2, 3]
    if np.linalg.det(np.stack([reg[1] - reg[0], reg[2] - reg[0], reg[3] - reg[0]])) < 0:
        q = [0, 2, 1, 3]
    for sigma in (0.9, 1.1):
        x, _ = oracle.iterate_jacobi(sigma * reg, np.ones(4), [], [], [q], [v0])
        want = sigma - (sigma ** 3 - 1) / (3 * sigma ** 2)
        np.testing.assert_allclose(x, want * reg, rtol=0, atol=1e-14)


def test_free_fall_closed_form():
    m = W.slab_mesh(3, 2, 2, pin_bottom=False)
    om = oracle.prepare_mesh(m.rest_pos, m.inv_mass, m.tets)
    p = params(iterations=2)
    steps = 10
    r = oracle.run_env(om, (1e-6, 1e-7), p, None, steps, jacobi=True)
    h = p.dt / p.substeps
    n = steps * p.substeps
    expect = om.rest + np.array([0, 0, p.gravity[2]]) * h * h * n * (n + 1) / 2
    np.testing.assert_allclose(r.x, expect, rtol=0, atol=1e-12)


def test_rigid_motion_invariance():
    m = W.slab_mesh(4, 3, 2)
    rng = np.random.default_rng(11)
    qm, rr = np.linalg.qr(rng.normal(size=(3, 3)))
    R = qm * np.sign(np.diag(rr))
    if np.linalg.det(R) < 0:
        R[:, 0] = -R[:, 0]
    t = rng.normal(scale=0.1, size=3)
    p = params(iterations=3)
    tools = W.tool_path(12, 1, 11, start_depth=6e-3)[:, 0]
    p1 = params(iterations=3, num_tools=1)
    om = oracle.prepare_mesh(m.rest_pos, m.inv_mass, m.tets)
    base = oracle.run_env(om, (1e-6, 1e-7), p1, tools, 12, jacobi=True, want_contacts=True)
    assert base.contact_count.sum() > 0
    om2 = oracle.prepare_mesh(om.rest @ R.T + t, m.inv_mass, m.tets)
    p2 = oracle.OracleParams(p.dt, p.substeps, p.iterations, tuple(R @ np.array(p.gravity)), 1,
                             p.tool_radius)
    moved = oracle.run_env(om2, (1e-6, 1e-7), p2, tools.astype(np.float64) @ R.T + t, 12,
                           jacobi=True, want_contacts=True)
    assert np.array_equal(moved.contact_count, base.contact_count)
    np.testing.assert_allclose(moved.x, base.x @ R.T + t, rtol=0, atol=1e-12)


@pytest.mark.parametrize("grid", [(1, 1, 1), (2, 1, 1)])
def test_zero_compliance_converges(grid):
    """Jacobi with averaging is a damped fixed-point iteration: from a small
    perturbation, many iterations satisfy every constraint."""
    m = W.slab_mesh(*grid)
    om = oracle.prepare_mesh(m.rest_pos, m.inv_mass, m.tets)
    rng = np.random.default_rng(12)
    x0 = om.rest + rng.normal(scale=1e-3, size=om.rest.shape) * (om.w[:, None] > 0)
    p = params(iterations=20000, gravity=(0, 0, 0), substeps=1, dt=H)
    r = oracle.run_env(om, (0.0, 0.0), p, None, 1, x0=x0, jacobi=True, want_residual=True)
    L = np.linalg.norm(r.x[om.edges[:, 0]] - r.x[om.edges[:, 1]], axis=1)
    assert np.max(np.abs(L - om.rest_length) / om.rest_length) < 1e-9
    assert r.residual[0, 0, 1] < 1e-9


def test_differs_from_gauss_seidel():
    """Jacobi and Gauss-Seidel agree on a rest mesh under gravity alone but not
    once constraints act."""
    m = W.slab_mesh(4, 3, 2)
    om = oracle.prepare_mesh(m.rest_pos, m.inv_mass, m.tets)
    p = params(iterations=2)
    gs = oracle.run_env(om, (1e-6, 1e-7), p, None, 5)
    jc = oracle.run_env(om, (1e-6, 1e-7), p, None, 5, jacobi=True)
    assert np.max(np.abs(gs.x - jc.x)) > 1e-7
