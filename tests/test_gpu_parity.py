"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

Gate: max per-particle position error <= 1e-4 of the mesh extent after 100
steps; the constraint colouring and the contact-candidate lists bit-exact
(candidates are decided in float32 on both sides from the GPU's own
start-of-step positions; against the FP64 trajectory they may differ only for
particles whose distance to the sphere is within the trajectories' position
error of the reach 2r).
"""
import ctypes

import numpy as np
import pytest

from paper_2503_18616_amd import workloads as W
from tests import cases as K

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def xp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2503_18616_amd import xpbd
    return xpbd


VARIANTS = [1, 2]   # multipliers in registers, multipliers in LDS
VARIANT_IDS = ["registers", "lds"]


def make_batch(xp, wl, flags=0, block_size=0, variant=0, colouring=0):
    p = K.lib_params(xp, wl, flags, block_size)
    p.solver_variant = variant
    p.colouring = colouring
    return xp.Batch(K.lib_meshes(wl), wl.env_mesh, wl.compliance, p)


def check_contacts_step(xp, oracle_lib, batch, wl, start_x, tools_step, oracle_lists=None,
                        envs=None, pos_err=0.0):
    """Bit-exact candidate lists against the float32 rule on the GPU's start-of-step
    positions; against the oracle's FP64 lists up to the ambiguous band."""
    offs = batch.env_offsets
    counts = batch.read(xp.FIELD_CONTACT_COUNTS).reshape(wl.num_envs, wl.num_tools)
    lists = batch.read(xp.FIELD_CONTACTS).reshape(wl.num_tools, -1)
    envs = range(wl.num_envs) if envs is None else envs
    for n, e in enumerate(envs):
        m = wl.meshes[int(wl.env_mesh[e])]
        x0 = K.env_block(start_x, offs, e)
        for t in range(wl.num_tools):
            got = K.env_block(lists[t], offs, e)
            c = int(counts[e, t])
            assert (got[c:] == -1).all()
            got = got[:c]
            expect = oracle_lib.contact_candidates_f32(x0, m.inv_mass, tools_step[e, t],
                                                       wl.tool_radius[t])
            assert np.array_equal(got, expect), f"env {e} tool {t}"
            if oracle_lists is not None:
                ol = oracle_lists[n][t]
                diff = np.setxor1d(got, ol)
                if diff.size:
                    d = np.linalg.norm(x0[diff].astype(np.float64) - tools_step[e, t], axis=1)
                    assert np.all(np.abs(d - 2 * wl.tool_radius[t]) <= 10 * pos_err + 1e-7), \
                        f"env {e} tool {t}: candidates {diff} differ outside the band"


# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("variant", VARIANTS, ids=VARIANT_IDS)
@pytest.mark.parametrize("start_depth", [2e-3, 6e-3])
def test_single_env_parity_per_step(xp, oracle_lib, start_depth, variant):
    """One environment, 8x5x3 slab, 4 iterations, 100 steps launched one step at a time."""
    wl = W.single_env_workload(seed=0)
    steps = 100
    tools = W.tool_path(steps, 1, wl.seed, start_depth=start_depth)
    om = K.oracle_meshes(oracle_lib, wl)[0]
    ref = oracle_lib.run_env(om, wl.compliance[0], K.oracle_params(oracle_lib, wl), tools[:, 0],
                             steps, want_lambda=True, want_contacts=True, want_residual=True)
    with make_batch(xp, wl, flags=xp.F_RESIDUAL | xp.F_LAMBDA, variant=variant) as b:
        x_hist = []
        for s in range(steps):
            x0 = b.positions()
            x_hist.append(x0)
            b.step(1, tools[s:s + 1])
            check_contacts_step(xp, oracle_lib, b, wl, x0, tools[s],
                                [[ref.contacts[s, t, :ref.contact_count[s, t]]
                                  for t in range(wl.num_tools)]],
                                pos_err=1e-6)
        x, v = b.positions(), b.velocities()
        lam = b.read(xp.FIELD_LAMBDA)
        res = b.read(xp.FIELD_RESIDUAL)
    err = K.max_position_error(x, ref.x)
    assert err <= K.POS_TOL, f"max position error {err:.3e} m > {K.POS_TOL:.1e}"
    h = wl.dt / wl.substeps
    assert np.max(np.abs(v - ref.v)) <= 2 * K.POS_TOL / h
    # multipliers and residual of the final substep
    lam_scale = np.max(np.abs(ref.lam))
    assert np.max(np.abs(lam - ref.lam)) <= 1e-2 * lam_scale
    r_ref = ref.residual[-1, -1]
    assert abs(res[0] - r_ref[0]) <= 0.05 * r_ref[0] + 1e-6
    assert abs(res[1] - r_ref[1]) <= 0.05 * r_ref[1] + 1e-6


@pytest.mark.parametrize("variant", VARIANTS, ids=VARIANT_IDS)
def test_single_launch_equals_step_by_step(xp, variant):
    wl = W.single_env_workload(seed=1)
    tools = wl.tools(100)
    with make_batch(xp, wl, variant=variant) as a, make_batch(xp, wl, variant=variant) as b:
        a.step(100, tools)
        for s in range(100):
            b.step(1, tools[s:s + 1])
        assert np.array_equal(a.positions(), b.positions())
        assert np.array_equal(a.velocities(), b.velocities())


def test_uneven_single_launch_equals_step_by_step(xp):
    """A batch of several size classes (classes on forked streams, one launch
    per class per call) stepped 12 steps in one call equals 12 calls of one
    step, bit for bit, contacts included."""
    meshes = [W.slab_mesh(6, 4, 2), W.slab_mesh(12, 8, 3), W.slab_mesh(20, 12, 6)]
    wl = W.Workload("classes", meshes, np.array([0, 2, 1, 0, 1, 2, 0], np.int32),
                    W.log_uniform_compliance(7, 1e-7, 1e-5, 29), iterations=4, num_steps=12,
                    seed=29)
    tools = wl.tools(12)
    with make_batch(xp, wl) as a, make_batch(xp, wl) as b:
        assert a.info()["size_classes"] >= 2
        a.step(12, tools)
        for s in range(12):
            b.step(1, tools[s:s + 1])
        assert np.array_equal(a.positions(), b.positions())
        assert np.array_equal(a.velocities(), b.velocities())
        assert np.array_equal(a.read(xp.FIELD_CONTACTS), b.read(xp.FIELD_CONTACTS))


@pytest.mark.parametrize("variant", VARIANTS, ids=VARIANT_IDS)
def test_batch_parity_sampled_envs(xp, oracle_lib, variant):
    """1024 environments of the 16x10x4 slab, 8 iterations, per-env compliances and
    tool paths, launched one step at a time; 16 sampled environments against the oracle."""
    steps = 100
    wl = W.batch_workload(1024, seed=0, num_steps=steps)
    sample = list(range(0, 1024, 64))
    tools = wl.tools(steps)
    om = K.oracle_meshes(oracle_lib, wl)
    refs = oracle_lib.run_batch(om, wl.env_mesh, wl.compliance, K.oracle_params(oracle_lib, wl),
                                tools[:, sample], steps, env_ids=sample, threads=8,
                                want_contacts=True)
    with make_batch(xp, wl, flags=xp.F_RESIDUAL, variant=variant) as b:
        offs = b.env_offsets
        for s in range(steps):
            check = s % 10 == 0 or s == steps - 1
            x0 = b.positions() if check else None
            b.step(1, tools[s:s + 1])
            if check:
                lists = [[r.contacts[s, t, :r.contact_count[s, t]] for t in range(1)] for r in refs]
                check_contacts_step(xp, oracle_lib, b, wl, x0, tools[s], lists, envs=sample,
                                    pos_err=1e-5)
        x = b.positions()
        res = b.read(xp.FIELD_RESIDUAL).reshape(-1, 2)
    assert np.all(np.isfinite(res)) and np.all(res[:, 0] > 0) and np.all(res[:, 1] >= res[:, 0])
    worst = 0.0
    for n, e in enumerate(sample):
        err = K.max_position_error(K.env_block(x, offs, e), refs[n].x)
        worst = max(worst, err)
    assert worst <= K.POS_TOL, f"max position error {worst:.3e} m"


@pytest.mark.parametrize("colouring", [1, 3], ids=["largest-first", "capped-256"])
def test_batch_parity_other_colourings(xp, oracle_lib, colouring):
    """The batch workload (1024 environments of the 16x10x4 slab, 8 iterations)
    under the largest-first colourings, plain and capped at 256 members (a
    different Gauss-Seidel order, taken by both sides from the same rules):
    colours read back bit-exact, 16 sampled environments against the oracle
    after 100 steps (one launch per step, as the benchmark runs it)."""
    steps = 100
    wl = W.batch_workload(1024, seed=2, num_steps=steps)
    sample = list(range(5, 1024, 64))
    tools = wl.tools(steps)
    m = wl.meshes[0]
    om = oracle_lib.prepare_mesh(m.rest_pos, m.inv_mass, m.tets, colouring=colouring)
    refs = oracle_lib.run_batch([om], wl.env_mesh, wl.compliance, K.oracle_params(oracle_lib, wl),
                                tools[:, sample], steps, env_ids=sample, threads=8)
    p = K.lib_params(xp, wl)
    p.colouring = colouring
    with xp.Batch(K.lib_meshes(wl), wl.env_mesh, wl.compliance, p) as b:
        col = b.read(xp.FIELD_COLOURS)
        assert np.array_equal(col, np.concatenate([om.edge_colour, om.tet_colour]))
        assert b.info()["solver_variant"] == xp.VARIANT_REGISTERS
        for s in range(steps):
            b.step(1, tools[s:s + 1])
        x = b.positions()
        offs = b.env_offsets
    worst = max(K.max_position_error(K.env_block(x, offs, e), refs[n].x)
                for n, e in enumerate(sample))
    assert worst <= K.POS_TOL, f"max position error {worst:.3e} m"


def test_step_checks_the_pose_byte_count(xp):
    """The C ABI's step calls take the byte count of the tool poses: a count
    that differs from what the steps read (either way, host or device poses)
    is XPBD_E_ARG and changes nothing; the exact count runs."""
    import torch
    wl = W.batch_workload(4, seed=0, num_steps=3)
    tools = np.ascontiguousarray(wl.tools(3), dtype=np.float32)
    dev = torch.from_numpy(tools).cuda()
    lp = xp.XpbdLearnedParams(0, wl.iterations, wl.iterations, 0.0, -1, None, None, None, 0.0,
                              None)
    p = K.lib_params(xp, wl)
    p.envs_per_group = 1   # what the learned step needs
    with xp.Batch(K.lib_meshes(wl), wl.env_mesh, wl.compliance, p) as b:
        x0 = b.positions()
        for ptr in (tools.ctypes.data, dev.data_ptr()):
            for nbytes in (tools.nbytes - 4, tools.nbytes + 4, 0):
                assert xp._lib.xpbd_step(b.handle, 3, ptr, nbytes) == xp.XPBD_E_ARG
                assert "bytes" in xp.xpbd_last_error()
                assert xp._lib.xpbd_step_learned(b.handle, None, 3, ptr, nbytes,
                                                 ctypes.byref(lp)) == xp.XPBD_E_ARG
        assert xp._lib.xpbd_step(b.handle, 3, None, tools.nbytes) == xp.XPBD_E_ARG
        assert np.array_equal(b.positions(), x0)
        assert xp._lib.xpbd_step(b.handle, 3, dev.data_ptr(), tools.nbytes) == xp.XPBD_OK
        assert not np.array_equal(b.positions(), x0)


def test_colours_read_back(xp, oracle_lib):
    wl = W.batch_workload(4, seed=0, num_steps=1)
    om = K.oracle_meshes(oracle_lib, wl)[0]
    with make_batch(xp, wl) as b:
        col = b.read(xp.FIELD_COLOURS)
    assert np.array_equal(col, np.concatenate([om.edge_colour, om.tet_colour]))


def test_rest_mesh_stays_at_rest(xp):
    wl = W.single_env_workload()
    wl.gravity = (0.0, 0.0, 0.0)
    wl.num_tools = 0
    with make_batch(xp, wl) as b:
        b.step(100, None)
        x = b.positions()
    drift = np.max(np.abs(x - wl.meshes[0].rest_pos))
    assert drift < 1e-6 * K.EXTENT


def test_free_fall_closed_form(xp):
    m = W.slab_mesh(3, 2, 2, pin_bottom=False)
    wl = W.Workload("free", [m], np.zeros(2, np.int32), W.constant_compliance(2, 1e-6, 1e-7),
                    iterations=4, num_steps=10, seed=0, num_tools=0)
    with make_batch(xp, wl) as b:
        b.step(10, None)
        x = b.positions().astype(np.float64)
    h = K.f32(wl.dt) / wl.substeps
    n = 10 * wl.substeps
    expect = np.tile(m.rest_pos.astype(np.float64), (2, 1)) + \
        np.array([0, 0, K.f32(-9.81)]) * h * h * n * (n + 1) / 2
    assert np.max(np.abs(x - expect)) < K.POS_TOL


@pytest.mark.parametrize("variant", VARIANTS, ids=VARIANT_IDS)
@pytest.mark.parametrize("block", [64, 128, 256, 512])
def test_block_size_does_not_change_results(xp, block, variant):
    """Which lane projects which constraint of a colour cannot matter: bitwise equal."""
    wl = W.single_env_workload(seed=3)
    tools = W.tool_path(30, 1, 3, start_depth=6e-3)
    with make_batch(xp, wl, variant=variant) as ref, \
            make_batch(xp, wl, block_size=block, variant=variant) as b:
        ref.step(30, tools)
        b.step(30, tools)
        assert np.array_equal(ref.positions(), b.positions())


def uneven_workload(seed=0):
    grids = [(6, 4, 2), (8, 5, 3), (10, 6, 3)]
    meshes = [W.slab_mesh(*g) for g in grids]
    env_mesh = np.array([0, 1, 2, 2, 1, 0], np.int32)
    return W.Workload("uneven", meshes, env_mesh,
                      W.log_uniform_compliance(6, 1e-7, 1e-5, seed), iterations=8,
                      num_steps=100, seed=seed)


@pytest.mark.parametrize("variant", VARIANTS, ids=VARIANT_IDS)
def test_uneven_meshes_parity(xp, oracle_lib, variant):
    wl = uneven_workload()
    steps = 100
    tools = W.tool_path(steps, wl.num_envs, wl.seed, start_depth=5e-3)
    om = K.oracle_meshes(oracle_lib, wl)
    refs = oracle_lib.run_batch(om, wl.env_mesh, wl.compliance, K.oracle_params(oracle_lib, wl),
                                tools, steps, threads=6)
    with make_batch(xp, wl, variant=variant) as b:
        b.step(steps, tools)
        x = b.positions()
        for e in range(wl.num_envs):
            err = K.max_position_error(K.env_block(x, b.env_offsets, e), refs[e].x)
            assert err <= K.POS_TOL, f"env {e}: {err:.3e}"


@pytest.mark.parametrize("variant", VARIANTS, ids=VARIANT_IDS)
def test_two_tools_parity(xp, oracle_lib, variant):
    wl = W.single_env_workload(seed=4)
    wl.num_tools = 2
    steps = 60
    tools = W.tool_path(steps, 1, 4, num_tools=2, start_depth=6e-3)
    om = K.oracle_meshes(oracle_lib, wl)[0]
    ref = oracle_lib.run_env(om, wl.compliance[0], K.oracle_params(oracle_lib, wl), tools[:, 0],
                             steps, want_contacts=True)
    assert ref.contact_count.sum() > 0
    with make_batch(xp, wl, variant=variant) as b:
        for s in range(steps):
            x0 = b.positions()
            b.step(1, tools[s:s + 1])
            check_contacts_step(xp, oracle_lib, b, wl, x0, tools[s],
                                [[ref.contacts[s, t, :ref.contact_count[s, t]] for t in range(2)]],
                                pos_err=1e-6)
        err = K.max_position_error(b.positions(), ref.x)
    assert err <= K.POS_TOL


@pytest.mark.parametrize("variant", VARIANTS, ids=VARIANT_IDS)
def test_largest_mesh_parity(xp, oracle_lib, variant):
    """The 20x12x6 slab (1911 particles), the largest of the uneven range: its
    constraint lists do not fit LDS next to the particles and are read from
    global memory."""
    m = W.slab_mesh(20, 12, 6)
    wl = W.Workload("large", [m], np.zeros(3, np.int32),
                    W.log_uniform_compliance(3, 1e-7, 1e-5, 9), iterations=8, num_steps=100, seed=9)
    steps = 100
    tools = W.tool_path(steps, 3, 9, start_depth=5e-3)
    om = K.oracle_meshes(oracle_lib, wl)
    refs = oracle_lib.run_batch(om, wl.env_mesh, wl.compliance, K.oracle_params(oracle_lib, wl),
                                tools, steps, threads=3)
    with make_batch(xp, wl, variant=variant) as b:
        b.step(steps, tools)
        x = b.positions()
        for e in range(3):
            err = K.max_position_error(K.env_block(x, b.env_offsets, e), refs[e].x)
            assert err <= K.POS_TOL, f"env {e}: {err:.3e}"


@pytest.mark.parametrize("variant", VARIANTS, ids=VARIANT_IDS)
def test_resume_is_bitwise(xp, variant):
    wl = W.batch_workload(8, seed=2, num_steps=40)
    tools = wl.tools(40)
    with make_batch(xp, wl, variant=variant) as full, make_batch(xp, wl, variant=variant) as half:
        full.step(40, tools)
        half.step(20, tools[:20])
        x, v = half.positions(), half.velocities()
        with make_batch(xp, wl, variant=variant) as resumed:
            resumed.write(xp.FIELD_POS, x)
            resumed.write(xp.FIELD_VEL, v)
            resumed.step(20, tools[20:])
            assert np.array_equal(resumed.positions(), full.positions())
            assert np.array_equal(resumed.velocities(), full.velocities())


@pytest.mark.parametrize("variant", VARIANTS, ids=VARIANT_IDS)
def test_runs_are_deterministic(xp, variant):
    wl = W.batch_workload(32, seed=3, num_steps=20)
    tools = wl.tools(20)
    with make_batch(xp, wl, flags=xp.F_LAMBDA, variant=variant) as a, \
            make_batch(xp, wl, flags=xp.F_LAMBDA, variant=variant) as b:
        a.step(20, tools)
        b.step(20, tools)
        assert np.array_equal(a.positions(), b.positions())
        assert np.array_equal(a.read(xp.FIELD_LAMBDA), b.read(xp.FIELD_LAMBDA))


def test_device_tool_poses_match_host(xp):
    import torch
    wl = W.batch_workload(16, seed=4, num_steps=10)
    tools = wl.tools(10)
    with make_batch(xp, wl) as a, make_batch(xp, wl) as b:
        a.step(10, tools)
        dev = torch.from_numpy(tools).cuda()
        b.step(10, dev)
        out = torch.empty(int(b.env_offsets[-1]) * 3, dtype=torch.float32, device="cuda")
        b.read(xp.FIELD_POS, out)
        assert np.array_equal(a.positions().ravel(), out.cpu().numpy())


def test_nonfinite_state_is_reported(xp):
    wl = W.batch_workload(3, seed=5, num_steps=1)
    with make_batch(xp, wl) as b:
        x = b.positions()
        x[b.env_offsets[1] + 500] = np.nan
        b.write(xp.FIELD_POS, x)
        b.step(1, wl.tools(1))
        with pytest.raises(xp.XpbdError) as e:
            b.positions()
        assert e.value.status == xp.XPBD_E_NONFINITE
        flags = b.read(xp.FIELD_NONFINITE, raise_nonfinite=False)
        assert flags.tolist() == [0, 1, 0]
        b.write(xp.FIELD_POS, np.tile(wl.meshes[0].rest_pos, (3, 1)))
        assert b.read(xp.FIELD_NONFINITE).tolist() == [0, 0, 0]


def test_extreme_compliances_follow_the_oracle(xp, oracle_lib):
    """Compliances at the ends of the range: zero (the stiff PBD limit of
    the compliance form) for both kinds, for one kind only, and 1e-3 (a soft
    solid), with the tool pressing: every environment follows the oracle over
    50 steps."""
    steps = 50
    m = W.slab_mesh(8, 5, 3)
    comp = np.array([[0.0, 0.0], [1e-8, 0.0], [1e-3, 1e-3], [0.0, 1e-4]], np.float32)
    wl = W.Workload("compliance-ends", [m], np.zeros(4, np.int32), comp, iterations=4,
                    num_steps=steps, seed=17)
    tools = W.tool_path(steps, wl.num_envs, wl.seed, start_depth=5e-3)
    om = K.oracle_meshes(oracle_lib, wl)
    refs = oracle_lib.run_batch(om, wl.env_mesh, wl.compliance, K.oracle_params(oracle_lib, wl),
                                tools, steps, threads=4)
    with make_batch(xp, wl) as b:
        b.step(steps, tools)
        x = b.positions()
        offs = b.env_offsets
    for e in range(wl.num_envs):
        err = K.max_position_error(K.env_block(x, offs, e), refs[e].x)
        assert err <= K.POS_TOL, f"env {e} (compliance {comp[e].tolist()}): {err:.3e}"


def test_irregular_meshes_follow_the_oracle(xp, oracle_lib):
    """Meshes off the regular grid: rest positions perturbed by 0.5 mm,
    tetrahedra shuffled (so some are given inside out and are reoriented),
    inverse masses scaled per particle by 0.5..2; two such meshes, three
    environments, the tool pressing: every environment follows the oracle
    over 30 steps."""
    import dataclasses
    rng = np.random.default_rng(23)
    meshes = []
    for grid in ((6, 4, 2), (9, 5, 3)):
        m = W.slab_mesh(*grid)
        rest = (m.rest_pos + rng.normal(scale=5e-4, size=m.rest_pos.shape)).astype(np.float32)
        perm = rng.permutation(m.num_tets)
        tets = m.tets[perm].copy()
        flip = rng.random(len(tets)) < 0.5
        tets[flip] = tets[flip][:, [1, 0, 2, 3]]
        w = (m.inv_mass * rng.uniform(0.5, 2.0, size=m.num_vertices)).astype(np.float32)
        meshes.append(dataclasses.replace(m, rest_pos=rest, tets=tets, inv_mass=w))
    steps = 30
    wl = W.Workload("irregular", meshes, np.array([1, 0, 1], np.int32),
                    W.log_uniform_compliance(3, 1e-7, 1e-5, 23), iterations=4, num_steps=steps,
                    seed=23)
    tools = W.tool_path(steps, wl.num_envs, wl.seed, start_depth=5e-3)
    om = K.oracle_meshes(oracle_lib, wl)
    refs = oracle_lib.run_batch(om, wl.env_mesh, wl.compliance, K.oracle_params(oracle_lib, wl),
                                tools, steps, threads=3)
    with make_batch(xp, wl) as b:
        col = b.read(xp.FIELD_COLOURS)
        assert np.array_equal(col, np.concatenate([np.concatenate([o.edge_colour, o.tet_colour])
                                                   for o in om]))
        b.step(steps, tools)
        x = b.positions()
        offs = b.env_offsets
    for e in range(wl.num_envs):
        err = K.max_position_error(K.env_block(x, offs, e), refs[e].x)
        assert err <= K.POS_TOL, f"env {e}: {err:.3e}"


def test_degenerate_meshes_beside_a_slab(xp, oracle_lib):
    """Degenerate meshes in one batch with an ordinary slab, the tool pressing
    each: a slab whose every particle is pinned (no constraint is kept: no
    rounds at all) stays exactly at rest with zero velocity; a single
    tetrahedron with one free corner (three edges and one volume) and the
    8x5x3 slab follow the oracle after 20 steps."""
    import dataclasses
    slab = W.slab_mesh(8, 5, 3)
    pinned = W.slab_mesh(2, 1, 1)
    pinned = dataclasses.replace(pinned, inv_mass=np.zeros_like(pinned.inv_mass))
    tet_pos = np.array([[0.0, 0.0, 0.0], [0.02, 0.0, 0.0], [0.0, 0.02, 0.0],
                        [0.005, 0.005, 0.02]], np.float32)
    one_tet = dataclasses.replace(slab, nx=1, ny=1, nz=1, rest_pos=tet_pos,
                                  tets=np.array([[0, 1, 2, 3]], np.int32),
                                  inv_mass=np.array([0.0, 0.0, 0.0, 1000.0], np.float32))
    meshes = [pinned, one_tet, slab]
    wl = W.Workload("degenerate", meshes, np.array([0, 1, 2, 2], np.int32),
                    W.log_uniform_compliance(4, 1e-7, 1e-5, 3), iterations=4, num_steps=20, seed=3)
    steps = 20
    tools = W.tool_path(steps, wl.num_envs, wl.seed, start_depth=4e-3)
    om = K.oracle_meshes(oracle_lib, wl)
    assert len(om[0].edges) == 0 and len(om[0].tets) == 0
    assert len(om[1].edges) == 3 and len(om[1].tets) == 1
    refs = oracle_lib.run_batch(om, wl.env_mesh, wl.compliance, K.oracle_params(oracle_lib, wl),
                                tools, steps, threads=4)
    with make_batch(xp, wl) as b:
        assert b.info()["solver_variant"] == xp.VARIANT_REGISTERS
        b.step(steps, tools)
        x, v = b.positions(), b.velocities()
        offs = b.env_offsets
    assert np.array_equal(K.env_block(x, offs, 0), pinned.rest_pos)
    assert not K.env_block(v, offs, 0).any()
    for e in (1, 2, 3):
        err = K.max_position_error(K.env_block(x, offs, e), refs[e].x)
        assert err <= K.POS_TOL, f"env {e}: {err:.3e}"
    assert not np.array_equal(K.env_block(x, offs, 1)[3], tet_pos[3])   # the free corner moved


def test_zero_steps_and_zero_iterations(xp):
    wl = W.single_env_workload()
    with make_batch(xp, wl) as b:
        b.step(0, None)
        assert np.array_equal(b.positions(), wl.meshes[0].rest_pos)
    wl.iterations = 0
    wl.num_tools = 0
    with make_batch(xp, wl) as b:
        b.step(3, None)
        x = b.positions().astype(np.float64)
    m = wl.meshes[0]
    h = K.f32(wl.dt) / wl.substeps
    n = 3 * wl.substeps
    expect = m.rest_pos.astype(np.float64).copy()
    free = m.inv_mass > 0
    expect[free, 2] += K.f32(-9.81) * h * h * n * (n + 1) / 2
    assert np.max(np.abs(x - expect)) < 1e-6


def test_tool_centred_on_a_particle(xp, oracle_lib):
    """Degenerate push-out direction: a particle exactly at the sphere centre moves
    to centre + (0, 0, r)."""
    wl = W.single_env_workload()
    m = wl.meshes[0]
    i = int(np.nonzero(m.inv_mass > 0)[0][-1])
    tools = np.tile(m.rest_pos[i], (1, 1, 1, 1)).astype(np.float32)
    wl.gravity = (0.0, 0.0, 0.0)
    wl.iterations = 1
    wl.substeps = 1
    # compliances so large that the constraints move nothing: the particle stays
    # exactly on the centre until the push-out
    wl.compliance = W.constant_compliance(1, 1e30, 1e30)
    with make_batch(xp, wl) as b:
        b.step(1, tools)
        counts = b.read(xp.FIELD_CONTACT_COUNTS)
        x = b.positions()
    om = K.oracle_meshes(oracle_lib, wl)[0]
    ref = oracle_lib.run_env(om, wl.compliance[0], K.oracle_params(oracle_lib, wl), tools[:, 0],
                             1, want_contacts=True)
    assert counts[0] == ref.contact_count[0, 0] and counts[0] >= 1
    assert K.max_position_error(x, ref.x) <= K.POS_TOL
    np.testing.assert_allclose(x[i], m.rest_pos[i] + [0, 0, wl.tool_radius[0]], atol=1e-6)


def test_variants_agree(xp):
    """The two data placements run the same projections in the same order."""
    wl = W.batch_workload(64, seed=6, num_steps=50)
    tools = wl.tools(50)
    with make_batch(xp, wl, flags=xp.F_LAMBDA | xp.F_RESIDUAL, variant=1) as a, \
            make_batch(xp, wl, flags=xp.F_LAMBDA | xp.F_RESIDUAL, variant=2) as b:
        a.step(50, tools)
        b.step(50, tools)
        assert K.max_position_error(a.positions(), b.positions().astype(np.float64)) <= 0.1 * K.POS_TOL
        la, lb = a.read(xp.FIELD_LAMBDA), b.read(xp.FIELD_LAMBDA)
        assert np.max(np.abs(la - lb)) <= 1e-2 * np.max(np.abs(lb))
        ra, rb = a.read(xp.FIELD_RESIDUAL), b.read(xp.FIELD_RESIDUAL)
        np.testing.assert_allclose(ra, rb, rtol=0.05, atol=1e-6)
        np.testing.assert_array_equal(a.read(xp.FIELD_CONTACT_COUNTS), b.read(xp.FIELD_CONTACT_COUNTS))


def test_register_variant_refuses_oversized_schedules(xp):
    """64 threads cannot hold the 16x10x4 slab's rounds in registers."""
    wl = W.batch_workload(2, seed=0, num_steps=1)
    with pytest.raises(xp.XpbdError) as e:
        make_batch(xp, wl, block_size=64, variant=1)
    assert e.value.status == xp.XPBD_E_CAPACITY


@pytest.mark.parametrize("variant", VARIANTS, ids=VARIANT_IDS)
@pytest.mark.parametrize("packing", [1, 2, 3, 4])
def test_colour_packing_does_not_change_results(xp, packing, variant):
    """The order of constraints inside a colour is free: bitwise equal results."""
    wl = W.batch_workload(8, seed=7, num_steps=30)
    tools = W.tool_path(30, 8, 7, start_depth=6e-3)
    p_ref = K.lib_params(xp, wl, xp.F_LAMBDA)
    p_ref.solver_variant = variant
    p_ref.colour_packing = 1
    p = K.lib_params(xp, wl, xp.F_LAMBDA)
    p.solver_variant = variant
    p.colour_packing = packing
    with xp.Batch(K.lib_meshes(wl), wl.env_mesh, wl.compliance, p_ref) as a, \
            xp.Batch(K.lib_meshes(wl), wl.env_mesh, wl.compliance, p) as b:
        a.step(30, tools)
        b.step(30, tools)
        assert np.array_equal(a.positions(), b.positions())
        assert np.array_equal(a.velocities(), b.velocities())
        assert np.array_equal(a.read(xp.FIELD_LAMBDA), b.read(xp.FIELD_LAMBDA))


@pytest.mark.parametrize("variant", VARIANTS, ids=VARIANT_IDS)
def test_searched_packing_changes_only_rounding(xp, variant):
    """The searched packing also reorders the particles inside edges and (by even
    permutations) tetrahedra: the same projections, different rounding."""
    wl = W.batch_workload(8, seed=7, num_steps=30)
    tools = W.tool_path(30, 8, 7, start_depth=6e-3)
    p_ref = K.lib_params(xp, wl, xp.F_LAMBDA)
    p_ref.solver_variant = variant
    p_ref.colour_packing = xp.PACKING_ID_ORDER
    p = K.lib_params(xp, wl, xp.F_LAMBDA)
    p.solver_variant = variant
    p.colour_packing = xp.PACKING_SEARCH
    with xp.Batch(K.lib_meshes(wl), wl.env_mesh, wl.compliance, p_ref) as a, \
            xp.Batch(K.lib_meshes(wl), wl.env_mesh, wl.compliance, p) as b:
        a.step(30, tools)
        b.step(30, tools)
        assert K.max_position_error(b.positions(), a.positions()) <= K.POS_TOL
        la, lb = a.read(xp.FIELD_LAMBDA), b.read(xp.FIELD_LAMBDA)
        assert np.abs(la - lb).max() <= 1e-3 * np.abs(la).max()
        if variant == 2:   # the LDS variant ignores the register-only packings
            assert np.array_equal(a.positions(), b.positions())


def test_flags_can_change_between_steps(xp):
    """Residual and multipliers requested on a later step only."""
    wl = W.batch_workload(4, seed=8, num_steps=6)
    tools = wl.tools(6)
    with make_batch(xp, wl, flags=xp.F_RESIDUAL | xp.F_LAMBDA) as ref, make_batch(xp, wl) as b:
        ref.step(6, tools)
        with pytest.raises(xp.XpbdError) as e:
            b.read(xp.FIELD_RESIDUAL)
        assert e.value.status == xp.XPBD_E_STATE
        b.step(5, tools[:5])
        b.set_flags(xp.F_RESIDUAL | xp.F_LAMBDA)
        b.step(1, tools[5:])
        assert np.array_equal(b.positions(), ref.positions())
        np.testing.assert_array_equal(b.read(xp.FIELD_RESIDUAL), ref.read(xp.FIELD_RESIDUAL))
        np.testing.assert_array_equal(b.read(xp.FIELD_LAMBDA), ref.read(xp.FIELD_LAMBDA))
        b.set_flags(0)
        b.step(1, tools[5:])
        with pytest.raises(xp.XpbdError):
            b.read(xp.FIELD_LAMBDA)
        with pytest.raises(xp.XpbdError):
            b.set_flags(0x40)


@pytest.mark.parametrize("colouring", [0, 5], ids=["greedy", "capped-where-it-fits"])
def test_uneven_4096_sampled_parity(xp, oracle_lib, colouring):
    """The 4096-environment uneven workload (675 distinct slabs of 105 to 1911
    particles) as the benchmark launches it (one launch per step of every
    size class; the benchmark's per-mesh capped colouring, and the greedy
    one): the smallest and largest environments and four others follow the
    oracle after 100 steps; with the per-mesh colouring, the colours of every
    32nd mesh and of the sampled environments' meshes equal the oracle's."""
    steps = 100
    wl = W.uneven_workload(4096, seed=0, num_steps=steps)
    V = np.array([m.num_vertices for m in wl.meshes])[wl.env_mesh]
    sample = sorted({int(np.argmin(V)), int(np.argmax(V)), 0, 1000, 2047, 4095})
    tools = wl.tools(steps)
    om = [oracle_lib.prepare_mesh(m.rest_pos, m.inv_mass, m.tets, colouring=colouring)
          if k in {int(wl.env_mesh[e]) for e in sample} else None
          for k, m in enumerate(wl.meshes)]
    refs = oracle_lib.run_batch(om, wl.env_mesh, wl.compliance, K.oracle_params(oracle_lib, wl),
                                tools[:, sample], steps, env_ids=sample, threads=len(sample))
    with make_batch(xp, wl, colouring=colouring) as b:
        if colouring:
            assert b.info()["solver_variant"] == xp.VARIANT_REGISTERS
            col = b.read(xp.FIELD_COLOURS)
            # A mesh's colours are those of its edges, then of its tets;
            # constraints whose particles are all pinned are not kept.
            pairs = [0, 1, 0, 2, 0, 3, 1, 2, 1, 3, 2, 3]
            counts = []
            for m in wl.meshes:
                free = m.inv_mass.reshape(-1) > 0
                e = np.unique(np.sort(m.tets[:, pairs].reshape(-1, 2), axis=1), axis=0)
                counts.append(int(free[e].any(axis=1).sum()) + int(free[m.tets].any(axis=1).sum()))
            off = np.concatenate([[0], np.cumsum(counts)])
            assert off[-1] == len(col)
            for k in sorted(set(range(0, len(wl.meshes), 32)) | {int(wl.env_mesh[e]) for e in sample}):
                o = om[k] or oracle_lib.prepare_mesh(wl.meshes[k].rest_pos, wl.meshes[k].inv_mass,
                                                     wl.meshes[k].tets, colouring=colouring)
                assert np.array_equal(col[off[k]:off[k + 1]],
                                      np.concatenate([o.edge_colour, o.tet_colour])), f"mesh {k}"
        b.step(steps, tools)
        x = b.positions()
        for n, e in enumerate(sample):
            err = K.max_position_error(K.env_block(x, b.env_offsets, e), refs[n].x)
            assert err <= K.POS_TOL, f"env {e} ({V[e]} particles): {err:.3e}"


@pytest.mark.parametrize("case", ["single-4-iterations", "single-1-iteration", "batch-3-envs"])
def test_jacobi_follows_the_oracle(xp, oracle_lib, case):
    """The paper's Jacobi solver (XPBD_VARIANT_JACOBI) against the oracle's
    Jacobi iteration, with the tool pressing: positions within the tolerance,
    and a second run equal bit for bit (sums in a fixed order)."""
    if case.startswith("single"):
        wl = W.single_env_workload(seed=7)
        if case == "single-1-iteration":
            wl.iterations = 1
        steps, envs = 60, [0]
    else:
        wl = W.batch_workload(3, seed=8, num_steps=40)
        steps, envs = 40, [0, 1, 2]
    tools = W.tool_path(steps, wl.num_envs, wl.seed, start_depth=6e-3)
    om = K.oracle_meshes(oracle_lib, wl)
    refs = oracle_lib.run_batch(om, wl.env_mesh, wl.compliance, K.oracle_params(oracle_lib, wl),
                                tools, steps, threads=len(envs), jacobi=True)
    with make_batch(xp, wl, variant=xp.VARIANT_JACOBI) as b, \
            make_batch(xp, wl, variant=xp.VARIANT_JACOBI) as again:
        b.step(steps, tools)
        again.step(steps, tools)
        x = b.positions()
        assert np.array_equal(x, again.positions())
        for e in envs:
            err = K.max_position_error(K.env_block(x, b.env_offsets, e), refs[e].x)
            assert err <= K.POS_TOL, f"env {e}: {err:.3e}"
    plain = oracle_lib.run_batch(om, wl.env_mesh, wl.compliance, K.oracle_params(oracle_lib, wl),
                                 tools, steps, threads=len(envs))
    assert max(np.abs(plain[e].x - refs[e].x).max() for e in envs) > K.POS_TOL


def test_capsule_full_size_sampled(xp, oracle_lib):
    """Capsule tools on the benchmark's shape: 1024 environments of the
    16x10x4 slab under the colouring capped at 256 members (53 rounds, two
    multiplier banks), one launch per step for 30 steps.  16 sampled
    environments: the first step's candidate-face counts equal the oracle's,
    the positions follow its capsule driver."""
    steps = 30
    wl = W.batch_workload(1024, seed=4, num_steps=steps)
    sample = list(range(3, 1024, 64))
    caps = W.capsule_path(steps, wl.num_envs, wl.seed)
    m = wl.meshes[0]
    om = oracle_lib.prepare_mesh(m.rest_pos, m.inv_mass, m.tets,
                                 colouring=oracle_lib.COLOURING_CAPPED)
    op = K.oracle_params(oracle_lib, wl)
    refs = [oracle_lib.run_env_capsule(om, wl.compliance[e], op, caps[:, e].astype(np.float64),
                                       steps) for e in sample]
    assert sum(int(r.contact_count[0, 0]) for r in refs) > 0
    p = K.lib_params(xp, wl)
    p.tool_shape = xp.TOOL_CAPSULE
    p.colouring = 3   # XPBD_COLOURING_CAPPED
    with xp.Batch(K.lib_meshes(wl), wl.env_mesh, wl.compliance, p) as b:
        info = b.info()
        assert info["solver_variant"] == xp.VARIANT_REGISTERS and info["lambda_banks"] == 2
        # resident workgroups from the occupancy calculator: the capsule
        # kernel's registers allow no more than the LDS does
        lds_per_cu = 160 * 1024
        assert 1 <= info["workgroups_per_cu"] <= lds_per_cu // info["lds_bytes"]
        assert info["waves_per_cu"] == info["workgroups_per_cu"] * info["block_size"] // 64
        b.step(1, caps[:1])
        counts = b.read(xp.FIELD_CONTACT_COUNTS).reshape(wl.num_envs, 1)
        assert [int(counts[e, 0]) for e in sample] == [int(r.contact_count[0, 0]) for r in refs]
        for s in range(1, steps):
            b.step(1, caps[s:s + 1])
        x = b.positions()
        offs = b.env_offsets
    worst = max(K.max_position_error(K.env_block(x, offs, e), refs[n].x)
                for n, e in enumerate(sample))
    assert worst <= K.POS_TOL, f"max position error {worst:.3e} m"


@pytest.mark.parametrize("block", [0, 64])
def test_two_capsules_follow_the_oracle(xp, oracle_lib, block):
    """Two capsule tools on the register kernel (each tool's flagged faces
    listed and pushed on their own, tool by tool): a second capsule 2.5 cm
    along y from the first, radii 5 and 4 mm; 3 environments of the 16x10x4
    slab over 30 steps.  With 64-thread workgroups one wave lists both
    tools (on the 8x5x3 slab, whose colours fit 64 rounds of 64 lanes).
    First-step candidate counts equal the oracle's, positions within the
    tolerance."""
    import dataclasses
    steps = 30
    wl = dataclasses.replace(W.batch_workload(3, seed=11, num_steps=steps), num_tools=2,
                             tool_radius=(W.TOOL_RADIUS, 0.004))
    if block:
        wl = dataclasses.replace(wl, meshes=[W.slab_mesh(8, 5, 3)])
    one = W.capsule_path(steps, wl.num_envs, wl.seed)[:, :, 0]
    two = one.copy()
    two[..., 1] += 0.025
    two[..., 4] += 0.025
    caps = np.ascontiguousarray(np.stack([one, two], axis=2), dtype=np.float32)
    om = K.oracle_meshes(oracle_lib, wl)
    op = K.oracle_params(oracle_lib, wl)
    refs = [oracle_lib.run_env_capsule(om[0], wl.compliance[e], op, caps[:, e].astype(np.float64),
                                       steps) for e in range(wl.num_envs)]
    assert all(r.contact_count[0, 1] > 0 and r.contact_count[0, 0] > 0 for r in refs)
    p = K.lib_params(xp, wl, block_size=block)
    p.tool_shape = xp.TOOL_CAPSULE
    with xp.Batch(K.lib_meshes(wl), wl.env_mesh, wl.compliance, p) as b:
        assert b.info()["solver_variant"] == xp.VARIANT_REGISTERS
        if block:
            assert b.info()["block_size"] == block
        b.step(1, caps[:1])
        counts = b.read(xp.FIELD_CONTACT_COUNTS).reshape(wl.num_envs, 2)
        assert counts.tolist() == [[int(c) for c in r.contact_count[0]] for r in refs]
        b.step(steps - 1, caps[1:])
        x = b.positions()
    # all steps in one launch, on a fresh batch: the same bits
    with xp.Batch(K.lib_meshes(wl), wl.env_mesh, wl.compliance, p) as again:
        again.step(steps, caps)
        assert np.array_equal(again.positions(), x)
    for e in range(wl.num_envs):
        err = K.max_position_error(K.env_block(x, b.env_offsets, e), refs[e].x)
        assert err <= K.POS_TOL, f"env {e}: {err:.3e}"


def test_capsules_on_uneven_meshes(xp, oracle_lib):
    """Capsule tools on a batch of three slab sizes (8x5x3, 12x8x3, 20x12x6:
    size classes on their own streams, each mesh with its own face list and
    colours): every environment follows the oracle over 20 steps, with the
    first step's candidate counts equal."""
    steps = 20
    meshes = [W.slab_mesh(8, 5, 3), W.slab_mesh(12, 8, 3), W.slab_mesh(20, 12, 6)]
    wl = W.Workload("uneven-capsules", meshes, np.array([2, 0, 1, 2, 1], np.int32),
                    W.log_uniform_compliance(5, 1e-7, 1e-5, 13), iterations=4, num_steps=steps,
                    seed=13)
    caps = W.capsule_path(steps, wl.num_envs, wl.seed)
    om = K.oracle_meshes(oracle_lib, wl)
    op = K.oracle_params(oracle_lib, wl)
    refs = [oracle_lib.run_env_capsule(om[int(wl.env_mesh[e])], wl.compliance[e], op,
                                       caps[:, e].astype(np.float64), steps)
            for e in range(wl.num_envs)]
    assert all(r.contact_count[0, 0] > 0 for r in refs)
    p = K.lib_params(xp, wl)
    p.tool_shape = xp.TOOL_CAPSULE
    with xp.Batch(K.lib_meshes(wl), wl.env_mesh, wl.compliance, p) as b:
        info = b.info()
        assert info["solver_variant"] == xp.VARIANT_REGISTERS and info["size_classes"] >= 2
        b.step(1, caps[:1])
        counts = b.read(xp.FIELD_CONTACT_COUNTS).reshape(wl.num_envs, 1)
        assert [int(c) for c in counts[:, 0]] == [int(r.contact_count[0, 0]) for r in refs]
        b.step(steps - 1, caps[1:])
        x = b.positions()
    for e in range(wl.num_envs):
        err = K.max_position_error(K.env_block(x, b.env_offsets, e), refs[e].x)
        assert err <= K.POS_TOL, f"env {e}: {err:.3e}"


@pytest.mark.parametrize("case", ["single", "batch-3-envs", "single-lds", "batch-3-envs-lds",
                                  "jacobi"])
def test_capsule_tools_follow_the_oracle(xp, oracle_lib, case):
    """Capsule tools against the surface faces (XPBD_TOOL_CAPSULE): positions
    follow the oracle's capsule driver; the first step's candidate-face counts
    are equal.  The library's choice runs them on the register variant; the
    LDS and Jacobi variants are checked too."""
    if case.startswith("batch-3-envs"):
        wl = W.batch_workload(3, seed=9, num_steps=30)
    else:
        wl = W.single_env_workload(seed=9)
    steps = 30
    caps = W.capsule_path(steps, wl.num_envs, wl.seed)
    om = K.oracle_meshes(oracle_lib, wl)
    op = K.oracle_params(oracle_lib, wl)
    jacobi = case == "jacobi"
    refs = [oracle_lib.run_env_capsule(om[int(wl.env_mesh[e])], wl.compliance[e], op,
                                       caps[:, e].astype(np.float64), steps, jacobi=jacobi)
            for e in range(wl.num_envs)]
    assert sum(r.contact_count.sum() for r in refs) > 0
    p = K.lib_params(xp, wl)
    p.tool_shape = xp.TOOL_CAPSULE
    want = xp.VARIANT_REGISTERS
    if jacobi:
        p.solver_variant = want = xp.VARIANT_JACOBI
    elif case.endswith("-lds"):
        p.solver_variant = want = xp.VARIANT_LDS
    with xp.Batch(K.lib_meshes(wl), wl.env_mesh, wl.compliance, p) as b:
        assert b.info()["solver_variant"] == want
        b.step(1, caps[:1])
        counts = b.read(xp.FIELD_CONTACT_COUNTS).reshape(wl.num_envs, 1)
        assert [int(c) for c in counts[:, 0]] == [int(r.contact_count[0, 0]) for r in refs]
        b.step(steps - 1, caps[1:])
        x = b.positions()
    for e in range(wl.num_envs):
        err = K.max_position_error(K.env_block(x, b.env_offsets, e), refs[e].x)
        assert err <= K.POS_TOL, f"env {e}: {err:.3e}"
