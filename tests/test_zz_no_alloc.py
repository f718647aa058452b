"""GPU: the allocation-free learned step (xpbd_step_learned_noalloc) against
the allocating one (xpbd_step_learned), through the C ABI.

Both run the same kernels, so the results must agree bit for bit: positions,
velocities, sweep counts and per-substep residuals.  Two calls in a row share
the library's fixed device array: a 64-environment batch of the 16x10x4 slab,
then one environment of the 8x5x3 slab (a smaller input on a different mesh,
which finds the first call's contents in the array).  Sizes beyond the array
and host tool poses are refused before any device work.
"""
import numpy as np
import pytest

from oracle import warmstart as ws
from paper_2503_18616_amd import workloads as W
from tests import cases as K

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def xp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2503_18616_amd import xpbd
    return xpbd


def network(xp, seed=8):
    """A seeded random network at the feature and output scales of the slabs."""
    rng = np.random.default_rng(seed)
    net = ws.init_net(seed, in_scale=np.ones(27), out_scale=np.full(3, 2e-6))
    for b in (net.b1, net.b2, net.b3):
        b[:] = rng.standard_normal(b.shape) * 0.05
    in_scale = 1.0 / np.array([2e-4] * 3 + [0.1] * 3 + [2e-3] * 3 + [2e-5] * 18)
    in_shift = rng.uniform(-0.3, 0.3, 27) / in_scale
    params = np.concatenate([p.reshape(-1) for p in net.params()]).astype(np.float32)
    return xp.Mlp(params, in_shift, in_scale, net.out_shift, net.out_scale)


def make_batch(xp, wl):
    p = K.lib_params(xp, wl)
    p.solver_variant = xp.VARIANT_REGISTERS
    return xp.Batch(K.lib_meshes(wl), wl.env_mesh, wl.compliance, p)


def run_both(xp, net, wl, tools, steps, threshold, stall):
    """The allocating and the allocation-free step from the same state;
    returns both sides' (positions, velocities, sweeps, residuals)."""
    import torch
    out = []
    for noalloc in (False, True):
        n = steps * wl.substeps * wl.num_envs
        its = torch.zeros(n, dtype=torch.int32, device="cuda")
        res = torch.zeros(n, dtype=torch.float32, device="cuda")
        with make_batch(xp, wl) as b:
            b.step(2, tools[:2])
            run = b.step_learned_noalloc if noalloc else b.step_learned
            run(net, steps, tools[2:], 2, 8, threshold, iterations=its, residuals=res,
                stall_ratio=stall)
            out.append((b.positions(), b.velocities(), its.cpu().numpy(), res.cpu().numpy()))
    return out


def test_noalloc_learned_step_equals_the_allocating_step_twice(xp):
    import torch
    steps = 3
    big = W.batch_workload(64, seed=4, num_steps=steps + 2)
    small = W.single_env_workload(seed=5)
    with network(xp) as net:
        for wl, stall in ((big, 0.0), (small, 0.9)):
            tools = torch.from_numpy(np.ascontiguousarray(wl.tools(steps + 2))).cuda()
            # a threshold between the residuals the substeps reach after two sweeps,
            # so that both decisions occur
            probe = run_both(xp, net, wl, tools, steps, np.inf, 0.0)[0][3]
            threshold = float(np.median(probe))
            (xa, va, ia, ra), (xb, vb, ib, rb) = run_both(xp, net, wl, tools, steps, threshold,
                                                         stall)
            assert np.array_equal(xa, xb) and np.array_equal(va, vb)
            assert np.array_equal(ia, ib) and np.array_equal(ra, rb)
            assert set(np.unique(ia)) <= {2, 8}
            if stall == 0.0:
                assert set(np.unique(ia)) == {2, 8}, np.unique(ia)


def test_noalloc_refuses_what_it_cannot_hold(xp):
    import torch
    steps = 1
    # 1200 environments of 935 particles: 1.12 M particles, 86 MB of workspace with
    # the correction, more than the 80 MiB array
    wl = W.batch_workload(1200, seed=0, num_steps=steps)
    tools = torch.from_numpy(np.ascontiguousarray(wl.tools(steps))).cuda()
    with network(xp) as net, make_batch(xp, wl) as b:
        x0 = b.positions()
        with pytest.raises(xp.XpbdError) as e:
            b.step_learned_noalloc(net, steps, tools, 2, 8, 1e-3)
        assert e.value.status == xp.XPBD_E_CAPACITY
        # without the correction the workspace (13 bytes per particle) fits
        b.step_learned_noalloc(None, steps, tools, 8, 8, np.inf, apply_correction=False)
        assert not np.array_equal(b.positions(), x0)
    small = W.single_env_workload(seed=5)
    with network(xp) as net, make_batch(xp, small) as b:
        host_tools = np.ascontiguousarray(small.tools(1))
        with pytest.raises(xp.XpbdError) as e:
            b.step_learned_noalloc(net, 1, host_tools, 2, 8, 1e-3)
        assert e.value.status == xp.XPBD_E_ARG
