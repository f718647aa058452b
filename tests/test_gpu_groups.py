"""GPU: several environments per workgroup (register variant).

Two environments of one mesh can share a workgroup, its LDS and its rounds
(a round's lanes then mix both environments).  With the packing fixed to
constraint-id order the arithmetic of every projection is unchanged, so the
grouped launch must reproduce the one-environment launch bit for bit,
including the filler that completes a group when a mesh has an odd number of
environments; with the searched packing it must stay within the oracle gate.
"""
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


def uneven_odd_workload(seed=3):
    """Three meshes; mesh 0 has three environments (one group plus a filler)."""
    grids = [(6, 4, 2), (8, 5, 3), (10, 6, 3)]
    meshes = [W.slab_mesh(*g) for g in grids]
    env_mesh = np.array([0, 1, 2, 2, 1, 0, 0], np.int32)
    return W.Workload("uneven-odd", meshes, env_mesh,
                      W.log_uniform_compliance(7, 1e-7, 1e-5, seed), iterations=8,
                      num_steps=60, seed=seed)


def grouped_batch(xp, wl, group, packing, flags=0):
    p = K.lib_params(xp, wl, flags)
    p.solver_variant = xp.VARIANT_REGISTERS
    p.colour_packing = packing
    p.envs_per_group = group
    return xp.Batch(K.lib_meshes(wl), wl.env_mesh, wl.compliance, p)


def test_groups_of_two_are_bitwise_equal_to_single_envs(xp):
    wl = uneven_odd_workload()
    steps = 60
    tools = W.tool_path(steps, wl.num_envs, wl.seed, start_depth=6e-3)
    flags = xp.F_LAMBDA | xp.F_RESIDUAL
    with grouped_batch(xp, wl, 1, xp.PACKING_ID_ORDER, flags) as a, \
            grouped_batch(xp, wl, 2, xp.PACKING_ID_ORDER, flags) as b:
        a.step(steps // 2, tools[:steps // 2])
        b.step(steps // 2, tools[:steps // 2])
        a.step(steps - steps // 2, tools[steps // 2:])
        b.step(steps - steps // 2, tools[steps // 2:])
        assert np.array_equal(a.positions(), b.positions())
        assert np.array_equal(a.velocities(), b.velocities())
        for f in (xp.FIELD_LAMBDA, xp.FIELD_CONTACTS, xp.FIELD_CONTACT_COUNTS,
                  xp.FIELD_RESIDUAL, xp.FIELD_NONFINITE):
            assert np.array_equal(a.read(f), b.read(f)), f
        assert b.read(xp.FIELD_CONTACT_COUNTS).sum() > 0


def small_meshes_workload(seed=5):
    """Slabs of 105 to 1911 particles with odd environment counts: the
    library's per-class choice runs the small ones two to a workgroup and the
    largest one alone."""
    grids = [(6, 4, 2), (7, 4, 2), (8, 5, 3), (11, 6, 5), (20, 12, 6)]
    meshes = [W.slab_mesh(*g) for g in grids]
    env_mesh = np.array([0, 1, 2, 3, 0, 0, 1, 2, 3, 3, 0, 4, 4, 4], np.int32)
    return W.Workload("small-meshes", meshes, env_mesh,
                      W.log_uniform_compliance(len(env_mesh), 1e-7, 1e-5, seed), iterations=8,
                      num_steps=40, seed=seed)


def test_per_class_groups_are_bitwise_equal_to_single_envs(xp):
    """Several meshes with the environments per workgroup left to the library:
    the small meshes' classes run two environments per workgroup, the others
    one (the batch reports the largest); with the packing fixed to id order
    the results equal one environment per workgroup bit for bit."""
    wl = small_meshes_workload()
    steps = 40
    tools = W.tool_path(steps, wl.num_envs, wl.seed, start_depth=6e-3)
    flags = xp.F_LAMBDA | xp.F_RESIDUAL
    with grouped_batch(xp, wl, 1, xp.PACKING_ID_ORDER, flags) as a, \
            grouped_batch(xp, wl, 0, xp.PACKING_ID_ORDER, flags) as b:
        assert a.info()["envs_per_group"] == 1
        assert b.info()["envs_per_group"] == 2 and b.info()["size_classes"] >= 2
        a.step(steps, tools)
        b.step(steps, tools)
        assert np.array_equal(a.positions(), b.positions())
        assert np.array_equal(a.velocities(), b.velocities())
        for f in (xp.FIELD_LAMBDA, xp.FIELD_CONTACTS, xp.FIELD_CONTACT_COUNTS,
                  xp.FIELD_RESIDUAL):
            assert np.array_equal(a.read(f), b.read(f)), f


def test_groups_of_two_oracle_parity(xp, oracle_lib):
    wl = uneven_odd_workload(seed=4)
    steps = 60
    tools = W.tool_path(steps, wl.num_envs, wl.seed, start_depth=5e-3)
    om = K.oracle_meshes(oracle_lib, wl)
    refs = oracle_lib.run_batch(om, wl.env_mesh, wl.compliance, K.oracle_params(oracle_lib, wl),
                                tools, steps, threads=7)
    with grouped_batch(xp, wl, 2, xp.PACKING_AUTO) as b:
        b.step(steps, tools)
        x = b.positions()
        for e in range(wl.num_envs):
            err = K.max_position_error(K.env_block(x, b.env_offsets, e), refs[e].x)
            assert err <= K.POS_TOL, f"env {e}: {err:.3e}"


def test_groups_of_two_report_nonfinite_per_env(xp):
    wl = W.batch_workload(3, seed=5, num_steps=1)
    with grouped_batch(xp, wl, 2, xp.PACKING_AUTO) as b:
        x = b.positions()
        x[b.env_offsets[1] + 500] = np.nan
        b.write(xp.FIELD_POS, x)
        b.step(1, wl.tools(1))
        flags = b.read(xp.FIELD_NONFINITE, raise_nonfinite=False)
        assert flags.tolist() == [0, 1, 0]


def test_groups_need_the_register_variant(xp):
    wl = W.batch_workload(4, seed=0, num_steps=1)
    p = K.lib_params(xp, wl)
    p.solver_variant = xp.VARIANT_LDS
    p.envs_per_group = 2
    with pytest.raises(xp.XpbdError) as e:
        xp.Batch(K.lib_meshes(wl), wl.env_mesh, wl.compliance, p)
    assert e.value.status == xp.XPBD_E_CAPACITY


def test_autotune_picks_a_configuration_that_runs(xp, oracle_lib):
    """The autotuner times its candidates on an uneven batch and returns the
    fastest (never slower than the default, which is one of them); a batch
    made with the choice follows the oracle."""
    import dataclasses
    grids = [(6, 4, 2), (12, 8, 3), (20, 12, 6)]
    meshes = [W.slab_mesh(*g) for g in grids]
    env_mesh = np.array([k % 3 for k in range(24)], np.int32)
    wl = W.Workload("tune", meshes, env_mesh, W.log_uniform_compliance(24, 1e-7, 1e-5, 5),
                    iterations=8, num_steps=10, seed=5)
    tools = W.tool_path(10, 24, 5, start_depth=5e-3)
    p = K.lib_params(xp, wl)
    best, default = xp.xpbd_autotune(K.lib_meshes(wl), wl.env_mesh, wl.compliance, p, 3,
                                     tools[:3])
    assert 0 < best <= default
    assert p.solver_variant in (0, 1, 2) and p.envs_per_group in (0, 1, 2)
    sample = [0, 1, 2, 23]
    om = K.oracle_meshes(oracle_lib, wl)
    refs = oracle_lib.run_batch(om, wl.env_mesh, wl.compliance, K.oracle_params(oracle_lib, wl),
                                tools[:, sample], 10, env_ids=sample, threads=4)
    with xp.Batch(K.lib_meshes(wl), wl.env_mesh, wl.compliance, p) as b:
        b.step(10, tools)
        x = b.positions()
        for n, e in enumerate(sample):
            err = K.max_position_error(K.env_block(x, b.env_offsets, e), refs[n].x)
            assert err <= K.POS_TOL, f"env {e}: {err:.3e}"


def test_batch_info_reports_the_chosen_launch(xp):
    """The occupancy model's choices: 256 threads and one environment per
    workgroup for the 16x10x4 slab (4 per CU), 128 threads for the 12x8x3
    slab (8 per CU), size classes for uneven meshes, and the LDS variant."""
    wl = W.batch_workload(1024, seed=0, num_steps=1)
    with xp.Batch(K.lib_meshes(wl), wl.env_mesh, wl.compliance, K.lib_params(xp, wl)) as b:
        i = b.info()
        assert (i["solver_variant"], i["block_size"], i["envs_per_group"], i["size_classes"]) == \
            (xp.VARIANT_REGISTERS, 256, 1, 1)
        assert (i["workgroups"], i["workgroups_per_cu"], i["waves_per_cu"], i["lambda_banks"]) == \
            (1024, 4, 16, 2)
    rl = W.rl_workload(8192, seed=0)
    with xp.Batch(K.lib_meshes(rl), rl.env_mesh, rl.compliance, K.lib_params(xp, rl)) as b:
        i = b.info()
        assert (i["block_size"], i["envs_per_group"], i["workgroups_per_cu"], i["waves_per_cu"]) == \
            (128, 1, 8, 16)
    # 64 environments fit one pass at any block: the fewest rounds win (256 threads)
    rl = W.rl_workload(64, seed=0)
    with xp.Batch(K.lib_meshes(rl), rl.env_mesh, rl.compliance, K.lib_params(xp, rl)) as b:
        assert b.info()["block_size"] == 256
    un = W.uneven_workload(64, seed=0, num_steps=1)
    with xp.Batch(K.lib_meshes(un), un.env_mesh, un.compliance, K.lib_params(xp, un)) as b:
        assert b.info()["size_classes"] >= 2
        assert b.info()["envs_per_group"] == 2      # the small meshes' classes
    p = K.lib_params(xp, wl)
    p.solver_variant = xp.VARIANT_LDS
    small = W.batch_workload(4, seed=0, num_steps=1)
    with xp.Batch(K.lib_meshes(small), small.env_mesh, small.compliance, p) as b:
        i = b.info()
        assert i["solver_variant"] == xp.VARIANT_LDS and i["size_classes"] == 1
