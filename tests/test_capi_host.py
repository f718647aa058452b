"""Host-side checks of the C ABI (no GPU needed).

- the shared library loads and exports every function the headers in include/ declare;
- the library's mesh set-up (orientation, edges, greedy colours) is bit-exact
  with the oracle's, and its float32 rest values are the oracle's FP64 values
  rounded (within one unit in the last place);
- every validation error is returned before any device work.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2503_18616_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def xp():
    from paper_2503_18616_amd import xpbd
    return xpbd


def declared_functions():
    text = "".join(open(os.path.join(ROOT, "include", h)).read()
                   for h in sorted(os.listdir(os.path.join(ROOT, "include"))) if h.endswith(".h"))
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(xpbd_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol(xp):
    names = declared_functions()
    assert len(names) >= 8
    lib = ctypes.CDLL(xp.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), f"{n} declared in include/ but not exported"
    assert set(names) == set(xp.EXPORTED)


def ulp_close(a32, b64, ulps=1):
    a32 = np.asarray(a32, np.float32)
    b32 = np.asarray(b64, np.float64).astype(np.float32)
    spacing = np.spacing(np.abs(b32))
    return np.all(np.abs(a32.astype(np.float64) - b32.astype(np.float64)) <= ulps * spacing)


GRIDS = [(1, 1, 1), (2, 1, 1), (8, 5, 3), (16, 10, 4), (12, 8, 3), (20, 12, 6), (6, 4, 2)]


@pytest.mark.parametrize("grid", GRIDS)
def test_mesh_setup_bit_exact_with_oracle(xp, oracle_lib, grid):
    m = W.slab_mesh(*grid)
    lib = xp.xpbd_prepare_mesh(m.rest_pos, m.inv_mass, m.tets)
    om = oracle_lib.prepare_mesh(m.rest_pos, m.inv_mass, m.tets)
    assert np.array_equal(lib["edges"], om.edges)
    assert np.array_equal(lib["tets"], om.tets)
    assert np.array_equal(lib["edge_colour"], om.edge_colour)
    assert np.array_equal(lib["tet_colour"], om.tet_colour)
    assert lib["num_edge_colours"] == om.num_edge_colours
    assert lib["num_tet_colours"] == om.num_tet_colours
    assert ulp_close(lib["rest_length"], om.rest_length)
    assert ulp_close(lib["rest_volume"], om.rest_volume)


@pytest.mark.parametrize("colouring", [1, 2, 3, 4])
@pytest.mark.parametrize("grid", GRIDS)
def test_largest_first_colourings_bit_exact_with_oracle(xp, oracle_lib, grid, colouring):
    """The library's largest-first colourings (plain, with the cut of
    65..100-member colours to 64, and capped at 256 or 128 members) equal the
    oracle's, constraint by constraint."""
    m = W.slab_mesh(*grid)
    lib = xp.xpbd_prepare_mesh(m.rest_pos, m.inv_mass, m.tets, colouring=colouring)
    om = oracle_lib.prepare_mesh(m.rest_pos, m.inv_mass, m.tets, colouring=colouring)
    assert np.array_equal(lib["edge_colour"], om.edge_colour)
    assert np.array_equal(lib["tet_colour"], om.tet_colour)
    assert lib["num_edge_colours"] == om.num_edge_colours
    assert lib["num_tet_colours"] == om.num_tet_colours


@pytest.mark.parametrize("grid", [(16, 10, 4), (12, 8, 3), (20, 12, 6), (6, 4, 2)])
def test_capped_fit_colouring_bit_exact_with_oracle(xp, oracle_lib, grid):
    """The per-mesh CAPPED_FIT colouring equals the oracle's on slabs below
    the limit (the capped colouring) and above it (20x12x6: the uncapped
    largest-first colouring)."""
    m = W.slab_mesh(*grid)
    lib = xp.xpbd_prepare_mesh(m.rest_pos, m.inv_mass, m.tets, colouring=5)
    om = oracle_lib.prepare_mesh(m.rest_pos, m.inv_mass, m.tets, colouring=5)
    assert np.array_equal(lib["edge_colour"], om.edge_colour)
    assert np.array_equal(lib["tet_colour"], om.tet_colour)
    capped = oracle_lib.prepare_mesh(m.rest_pos, m.inv_mass, m.tets, colouring=3)
    fits = (capped.num_edge_colours + capped.num_edge_colours % 2 +
            capped.num_tet_colours + capped.num_tet_colours % 2) <= 64
    assert fits == (grid != (20, 12, 6))
    want = capped if fits else oracle_lib.prepare_mesh(m.rest_pos, m.inv_mass, m.tets, colouring=1)
    assert np.array_equal(lib["edge_colour"], want.edge_colour)
    assert np.array_equal(lib["tet_colour"], want.tet_colour)


def test_mesh_setup_on_perturbed_and_shuffled_meshes(xp, oracle_lib):
    rng = np.random.default_rng(5)
    for trial in range(5):
        m = W.slab_mesh(*rng.integers(1, 6, size=3))
        rest = m.rest_pos + rng.normal(scale=1e-3, size=m.rest_pos.shape).astype(np.float32)
        perm = rng.permutation(m.num_tets)
        tets = m.tets[perm]
        w = m.inv_mass * rng.uniform(0.5, 2.0, size=m.num_vertices).astype(np.float32)
        for colouring in (0, 1, 2, 3, 4, 5):
            lib = xp.xpbd_prepare_mesh(rest, w, tets, colouring=colouring)
            om = oracle_lib.prepare_mesh(rest, w, tets, colouring=colouring)
            assert np.array_equal(lib["edges"], om.edges)
            assert np.array_equal(lib["tets"], om.tets)
            assert np.array_equal(lib["edge_colour"], om.edge_colour)
            assert np.array_equal(lib["tet_colour"], om.tet_colour)


def test_prepare_mesh_errors(xp):
    m = W.slab_mesh(1, 1, 1)
    bad = m.tets.copy()
    bad[1, 2] = 8
    with pytest.raises(xp.XpbdError) as e:
        xp.xpbd_prepare_mesh(m.rest_pos, m.inv_mass, bad)
    assert e.value.status == xp.XPBD_E_MESH and "particle 8" in str(e.value)
    rep = m.tets.copy()
    rep[0, 1] = rep[0, 0]
    with pytest.raises(xp.XpbdError) as e:
        xp.xpbd_prepare_mesh(m.rest_pos, m.inv_mass, rep)
    assert e.value.status == xp.XPBD_E_MESH
    flat = m.rest_pos.copy()
    flat[:, 2] = 0
    with pytest.raises(xp.XpbdError) as e:
        xp.xpbd_prepare_mesh(flat, np.ones(8, np.float32), m.tets)
    assert e.value.status == xp.XPBD_E_MESH and "zero rest volume" in str(e.value)
    nanpos = m.rest_pos.copy()
    nanpos[3, 0] = np.nan
    with pytest.raises(xp.XpbdError) as e:
        xp.xpbd_prepare_mesh(nanpos, m.inv_mass, m.tets)
    assert e.value.status == xp.XPBD_E_MESH
    neg = m.inv_mass.copy()
    neg[5] = -1.0
    with pytest.raises(xp.XpbdError):
        xp.xpbd_prepare_mesh(m.rest_pos, neg, m.tets)
    big = np.zeros((70000, 3), np.float32)
    with pytest.raises(xp.XpbdError) as e:
        xp.xpbd_prepare_mesh(big, np.ones(70000, np.float32), m.tets)
    assert e.value.status == xp.XPBD_E_MESH


def _create_error(xp, meshes=None, env_mesh=None, compliance=None, **pkw):
    m = W.slab_mesh(2, 1, 1)
    meshes = meshes if meshes is not None else [(m.rest_pos, m.inv_mass, m.tets)]
    env_mesh = env_mesh if env_mesh is not None else np.zeros(2, np.int32)
    compliance = compliance if compliance is not None else np.full((len(env_mesh), 2), 1e-6, np.float32)
    kw = dict(dt=1 / 60, substeps=10, iterations=4)
    kw.update(pkw)
    p = xp.make_params(**kw)
    with pytest.raises(xp.XpbdError) as e:
        xp.xpbd_create_batch(meshes, env_mesh, compliance, p, stream=0)
    return e.value


@pytest.mark.parametrize("kw,status", [
    (dict(dt=0.0), -1), (dict(dt=float("nan")), -1), (dict(substeps=0), -1),
    (dict(iterations=-1), -1), (dict(num_tools=3), -1), (dict(tool_radius=(0.0, 0.0)), -1),
    (dict(flags=0x80), -1), (dict(block_size=96), -1), (dict(block_size=2048), -1),
    (dict(gravity=(0.0, float("inf"), 0.0)), -1), (dict(envs_per_group=3), -1),
    (dict(envs_per_group=-1), -1), (dict(colour_packing=6), -1), (dict(solver_variant=4), -1),
    (dict(colouring=6), -1), (dict(colouring=-1), -1),
])
def test_create_rejects_bad_params(xp, kw, status):
    assert _create_error(xp, **kw).status == status


def test_create_rejects_bad_batches(xp):
    m = W.slab_mesh(2, 1, 1)
    assert _create_error(xp, env_mesh=np.array([0, 1], np.int32)).status == xp.XPBD_E_ARG
    c = np.full((2, 2), 1e-6, np.float32)
    c[1, 1] = -1e-6
    assert _create_error(xp, compliance=c).status == xp.XPBD_E_ARG
    c[1, 1] = np.nan
    assert _create_error(xp, compliance=c).status == xp.XPBD_E_ARG
    bad = m.tets.copy()
    bad[0, 0] = -1
    e = _create_error(xp, meshes=[(m.rest_pos, m.inv_mass, bad)])
    assert e.status == xp.XPBD_E_MESH and "mesh 0" in str(e)
    assert _create_error(xp, meshes=[]).status == xp.XPBD_E_ARG
    assert _create_error(xp, env_mesh=np.zeros(0, np.int32),
                         compliance=np.zeros((0, 2), np.float32)).status == xp.XPBD_E_ARG


def test_last_error_is_cleared_by_success(xp):
    m = W.slab_mesh(1, 1, 1)
    bad = m.tets.copy()
    bad[0, 0] = 99
    with pytest.raises(xp.XpbdError):
        xp.xpbd_prepare_mesh(m.rest_pos, m.inv_mass, bad)
    assert xp.xpbd_last_error() != ""
    xp.xpbd_prepare_mesh(m.rest_pos, m.inv_mass, m.tets)
    assert xp.xpbd_last_error() == ""


@pytest.mark.parametrize("grid", [(1, 1, 1), (8, 5, 3), (16, 10, 4), (20, 12, 6)])
def test_axis_neighbours_bit_exact_with_oracle(xp, grid):
    from oracle import warmstart as ws
    m = W.slab_mesh(*grid)
    assert np.array_equal(xp.xpbd_axis_neighbours(m.rest_pos), ws.axis_neighbours(m.rest_pos))
    # a shuffled and duplicated point cloud: the smallest id among equals wins on both sides
    rng = np.random.default_rng(1)
    pts = m.rest_pos[rng.permutation(len(m.rest_pos))]
    pts = np.concatenate([pts, pts[:7]])
    assert np.array_equal(xp.xpbd_axis_neighbours(pts), ws.axis_neighbours(pts))


def test_network_create_rejects_bad_scales(xp):
    ones27, ones3 = np.ones(27, np.float32), np.ones(3, np.float32)
    for si, so in [(np.full(27, np.nan, np.float32), ones3), (ones27, np.zeros(3, np.float32)),
                   (ones27, -ones3)]:
        with pytest.raises(xp.XpbdError) as e:
            xp.xpbd_mlp_create(None, None, si, None, so, stream=0)
        assert e.value.status == xp.XPBD_E_ARG


def test_autotune_rejects_bad_arguments(xp):
    """Argument errors are reported before any device work."""
    m = W.slab_mesh(2, 1, 1)
    meshes = [(m.rest_pos, m.inv_mass, m.tets)]
    p = xp.make_params(dt=1 / 60, substeps=10, iterations=4, num_tools=0)
    for steps in (0, -3):
        with pytest.raises(xp.XpbdError) as e:
            xp.xpbd_autotune(meshes, np.zeros(2, np.int32), np.full((2, 2), 1e-6, np.float32), p,
                             steps, None, stream=0)
        assert e.value.status == xp.XPBD_E_ARG and "num_steps" in str(e.value)


@pytest.mark.parametrize("grid", [(1, 1, 1), (4, 3, 2), (16, 10, 4)])
def test_surface_faces_equal_the_oracle(xp, grid):
    import oracle
    m = W.slab_mesh(*grid)
    faces, colours, n_col = xp.xpbd_surface_faces(m.rest_pos, m.inv_mass, m.tets)
    om = oracle.prepare_mesh(m.rest_pos, m.inv_mass, m.tets)
    assert np.array_equal(faces, om.faces)
    assert np.array_equal(colours, om.face_colour)
    assert n_col == int(om.face_colour.max()) + 1


def test_policy_create_rejects_bad_parameters(xp):
    """Checked on the host before any device call."""
    import ctypes
    h = ctypes.c_void_p()
    p = np.zeros(xp.RL_POLICY_PARAMS, np.float32)
    assert xp._lib.xpbd_policy_create(p.ctypes.data, 10, None, ctypes.byref(h)) == xp.XPBD_E_ARG
    assert "parameters" in xp.xpbd_last_error()
    p[7] = np.inf
    assert xp._lib.xpbd_policy_create(p.ctypes.data, p.size, None, ctypes.byref(h)) == xp.XPBD_E_ARG
    assert "finite" in xp.xpbd_last_error()
    assert xp._lib.xpbd_policy_create(None, p.size, None, ctypes.byref(h)) == xp.XPBD_E_ARG


def test_rl_constants_match_the_oracle(xp):
    import oracle.rl as R
    assert (xp.RL_OBS, xp.RL_HIDDEN, xp.RL_ACTIONS, xp.RL_TRACKED, xp.RL_POLICY_PARAMS) == \
        (R.OBS, R.HIDDEN, R.ACTIONS, R.TRACKED, R.NUM_PARAMS)
    assert ctypes_sizeof_rl_params(xp) == 4 * (1 + 3 + 1 + 1 + 3 + 3 + 3) + 4 * 18


def ctypes_sizeof_rl_params(xp):
    import ctypes
    return ctypes.sizeof(xp.XpbdRlParams)


def test_batch_info_rejects_null(xp):
    import ctypes
    assert xp._lib.xpbd_get_batch_info(None, None) == xp.XPBD_E_ARG
    info = xp.XpbdBatchInfo()
    assert xp._lib.xpbd_get_batch_info(None, ctypes.byref(info)) == xp.XPBD_E_ARG


def test_binding_refuses_to_load_without_the_library(tmp_path):
    """The product path has no fallback: a package copy without libxpbd.so
    raises ImportError when the binding (or a module built on it) loads."""
    import shutil
    import subprocess
    import sys
    src = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_2503_18616_amd")
    dst = tmp_path / "paper_2503_18616_amd"
    dst.mkdir()
    for name in os.listdir(src):
        if name.endswith(".py"):
            shutil.copy(os.path.join(src, name), dst / name)
    for module in ("xpbd", "warmstart"):
        r = subprocess.run([sys.executable, "-c", f"import paper_2503_18616_amd.{module}"],
                           cwd=tmp_path, capture_output=True, text=True, timeout=120,
                           env={**os.environ, "PYTHONPATH": str(tmp_path)})
        assert r.returncode != 0
        assert "ImportError" in r.stderr and "libxpbd.so is missing" in r.stderr
