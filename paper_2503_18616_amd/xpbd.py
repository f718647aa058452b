"""ctypes binding of libxpbd.so (the C ABI in include/xpbd.h).

The functions below carry the C names and only marshal arguments: every step
of the simulation runs in the HIP library.  Arrays may be numpy arrays (host
memory) or torch tensors (host or GPU memory; GPU tensors are passed as
device pointers, which the library reads in place).

If the shared library has not been built this module raises on import:
there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libxpbd.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing; build it with "
                      "`python -m paper_2503_18616_amd.build` (hipcc, gfx950)")
_lib = ctypes.CDLL(LIB_PATH)

XPBD_OK = 0
XPBD_E_ARG = -1
XPBD_E_MESH = -2
XPBD_E_CAPACITY = -3
XPBD_E_HIP = -4
XPBD_E_NONFINITE = -5
XPBD_E_STATE = -6
STATUS_NAMES = {0: "XPBD_OK", -1: "XPBD_E_ARG", -2: "XPBD_E_MESH", -3: "XPBD_E_CAPACITY",
                -4: "XPBD_E_HIP", -5: "XPBD_E_NONFINITE", -6: "XPBD_E_STATE"}

FIELD_POS = 0
FIELD_VEL = 1
FIELD_LAMBDA = 2
FIELD_CONTACTS = 3
FIELD_CONTACT_COUNTS = 4
FIELD_COLOURS = 5
FIELD_RESIDUAL = 6
FIELD_ENV_OFFSETS = 7
FIELD_NONFINITE = 8

F_RESIDUAL = 0x1
F_LAMBDA = 0x2

VARIANT_AUTO = 0
VARIANT_REGISTERS = 1
VARIANT_LDS = 2
VARIANT_JACOBI = 3
TOOL_SPHERE = 0
TOOL_CAPSULE = 1

PACKING_AUTO = 0
PACKING_ID_ORDER = 1
PACKING_BANKS8 = 2
PACKING_BANKS16 = 3
PACKING_SCATTERED_BANKS16 = 4
PACKING_SEARCH = 5

# field -> numpy dtype of its elements
FIELD_DTYPES = {FIELD_POS: np.float32, FIELD_VEL: np.float32, FIELD_LAMBDA: np.float32,
                FIELD_CONTACTS: np.int32, FIELD_CONTACT_COUNTS: np.int32,
                FIELD_COLOURS: np.int32, FIELD_RESIDUAL: np.float32,
                FIELD_ENV_OFFSETS: np.int32, FIELD_NONFINITE: np.int32}

EXPORTED = ["xpbd_create_batch", "xpbd_step", "xpbd_read_state", "xpbd_write_state",
            "xpbd_set_flags", "xpbd_field_bytes", "xpbd_destroy_batch", "xpbd_last_error",
            "xpbd_prepare_mesh", "xpbd_mlp_create", "xpbd_mlp_get_params", "xpbd_mlp_set_params",
            "xpbd_mlp_forward", "xpbd_mlp_train_step", "xpbd_mlp_destroy", "xpbd_axis_neighbours",
            "xpbd_step_learned", "xpbd_autotune", "xpbd_surface_faces", "xpbd_policy_create",
            "xpbd_policy_destroy", "xpbd_rl_step", "xpbd_rl_step_learned",
            "xpbd_step_graph_create", "xpbd_rl_graph_create", "xpbd_graph_launch",
            "xpbd_graph_destroy", "xpbd_get_batch_info", "xpbd_lds_probe",
            "xpbd_prepare_mesh_coloured", "xpbd_mlp_normalisation",
            "xpbd_step_learned_noalloc", "xpbd_mlp_train_steps"]

# learned warm start (include/xpbd_learned.h)
MLP_FEATURES = 27
MLP_FEATURE_STRIDE = 32
MLP_HIDDEN = 128
MLP_OUTPUTS = 3
MLP_PARAMS = 20483


# RL-style step (include/xpbd_rl.h)
RL_OBS = 64
RL_HIDDEN = 256
RL_ACTIONS = 7
RL_TRACKED = 18
RL_POLICY_PARAMS = 84231


class XpbdMesh(ctypes.Structure):
    _fields_ = [("num_vertices", ctypes.c_int32), ("num_tets", ctypes.c_int32),
                ("rest_pos", ctypes.c_void_p), ("inv_mass", ctypes.c_void_p),
                ("tets", ctypes.c_void_p)]


class XpbdParams(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_float), ("substeps", ctypes.c_int32),
                ("iterations", ctypes.c_int32), ("gravity", ctypes.c_float * 3),
                ("num_tools", ctypes.c_int32), ("tool_radius", ctypes.c_float * 2),
                ("flags", ctypes.c_uint32), ("block_size", ctypes.c_int32),
                ("solver_variant", ctypes.c_int32), ("colour_packing", ctypes.c_int32),
                ("envs_per_group", ctypes.c_int32), ("tool_shape", ctypes.c_int32),
                ("colouring", ctypes.c_int32)]


class XpbdBatchInfo(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int32) for name in (
        "solver_variant", "block_size", "envs_per_group", "size_classes", "lambda_banks",
        "lds_bytes", "workgroups", "workgroups_per_cu", "waves_per_cu")]


_lib.xpbd_get_batch_info.restype = ctypes.c_int
_lib.xpbd_get_batch_info.argtypes = [ctypes.c_void_p, ctypes.POINTER(XpbdBatchInfo)]
_lib.xpbd_create_batch.restype = ctypes.c_int
_lib.xpbd_create_batch.argtypes = [ctypes.POINTER(XpbdMesh), ctypes.c_int32, ctypes.c_void_p,
                                   ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(XpbdParams),
                                   ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
_lib.xpbd_step.restype = ctypes.c_int
_lib.xpbd_step.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t]
_lib.xpbd_autotune.restype = ctypes.c_int
_lib.xpbd_autotune.argtypes = [ctypes.POINTER(XpbdMesh), ctypes.c_int32, ctypes.c_void_p,
                               ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
_lib.xpbd_read_state.restype = ctypes.c_int
_lib.xpbd_read_state.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t]
_lib.xpbd_write_state.restype = ctypes.c_int
_lib.xpbd_write_state.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t]
_lib.xpbd_set_flags.restype = ctypes.c_int
_lib.xpbd_set_flags.argtypes = [ctypes.c_void_p, ctypes.c_uint32]
_lib.xpbd_field_bytes.restype = ctypes.c_int
_lib.xpbd_field_bytes.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
_lib.xpbd_destroy_batch.restype = None
_lib.xpbd_destroy_batch.argtypes = [ctypes.c_void_p]
_lib.xpbd_last_error.restype = ctypes.c_char_p
_lib.xpbd_last_error.argtypes = []
_lib.xpbd_prepare_mesh.restype = ctypes.c_int
_lib.xpbd_prepare_mesh.argtypes = [ctypes.POINTER(XpbdMesh), ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
_lib.xpbd_prepare_mesh_coloured.restype = ctypes.c_int
_lib.xpbd_prepare_mesh_coloured.argtypes = [ctypes.POINTER(XpbdMesh), ctypes.c_int32,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p]


class XpbdLearnedParams(ctypes.Structure):
    _fields_ = [("apply_correction", ctypes.c_int32), ("min_iterations", ctypes.c_int32),
                ("max_iterations", ctypes.c_int32), ("threshold", ctypes.c_float),
                ("record_substep", ctypes.c_int32), ("record_features", ctypes.c_void_p),
                ("record_targets", ctypes.c_void_p), ("iterations", ctypes.c_void_p),
                ("stall_ratio", ctypes.c_float), ("residuals", ctypes.c_void_p)]


_V = ctypes.c_void_p
_lib.xpbd_mlp_create.restype = ctypes.c_int
_lib.xpbd_mlp_create.argtypes = [_V, _V, _V, _V, _V, _V, ctypes.POINTER(ctypes.c_void_p)]
_lib.xpbd_mlp_get_params.restype = ctypes.c_int
_lib.xpbd_mlp_get_params.argtypes = [_V, _V]
_lib.xpbd_mlp_set_params.restype = ctypes.c_int
_lib.xpbd_mlp_set_params.argtypes = [_V, _V]
_lib.xpbd_mlp_forward.restype = ctypes.c_int
_lib.xpbd_mlp_forward.argtypes = [_V, _V, ctypes.c_int32, _V]
_lib.xpbd_mlp_train_step.restype = ctypes.c_int
_lib.xpbd_mlp_train_step.argtypes = [_V, _V, _V, _V, ctypes.c_int32, ctypes.c_float, _V, _V]
_lib.xpbd_mlp_train_steps.restype = ctypes.c_int
_lib.xpbd_mlp_train_steps.argtypes = [_V, _V, _V, _V, ctypes.c_int64, _V, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_float, ctypes.c_float, _V]
_lib.xpbd_mlp_destroy.restype = None
_lib.xpbd_mlp_destroy.argtypes = [_V]
_lib.xpbd_axis_neighbours.restype = ctypes.c_int
_lib.xpbd_axis_neighbours.argtypes = [ctypes.POINTER(XpbdMesh), _V]
_lib.xpbd_step_learned.restype = ctypes.c_int
_lib.xpbd_step_learned.argtypes = [_V, _V, ctypes.c_int32, _V, ctypes.c_size_t,
                                   ctypes.POINTER(XpbdLearnedParams)]
_lib.xpbd_step_learned_noalloc.restype = ctypes.c_int
_lib.xpbd_step_learned_noalloc.argtypes = [_V, _V, ctypes.c_int32, _V, ctypes.c_size_t,
                                           ctypes.POINTER(XpbdLearnedParams)]
# bytes of the allocation-free learned step's device array
NOALLOC_SCRATCH_BYTES = 80 << 20

# handle -> (num_envs, num_tools), to check tool-pose buffers before a launch
_BATCHES = {}
_SUBSTEPS = {}


class XpbdError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _check(status):
    if status != XPBD_OK:
        raise XpbdError(status, xpbd_last_error())


def _nbytes(a):
    """Bytes of a numpy array or torch tensor (None -> 0)."""
    if a is None:
        return 0
    if isinstance(a, np.ndarray):
        return int(a.nbytes)
    return int(a.numel()) * int(a.element_size())


def _ptr(a):
    """Address of a contiguous numpy array or torch tensor (None -> NULL)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return a.ctypes.data
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return a.data_ptr()
    raise TypeError(f"unsupported buffer type {type(a)}")


def _mesh_struct(rest_pos, inv_mass, tets, keep):
    rest_pos = np.ascontiguousarray(rest_pos, dtype=np.float32).reshape(-1, 3)
    inv_mass = np.ascontiguousarray(inv_mass, dtype=np.float32).reshape(-1)
    tets = np.ascontiguousarray(tets, dtype=np.int32).reshape(-1, 4)
    keep.extend([rest_pos, inv_mass, tets])
    return XpbdMesh(rest_pos.shape[0], tets.shape[0], rest_pos.ctypes.data,
                    inv_mass.ctypes.data, tets.ctypes.data)


def make_params(dt, substeps, iterations, gravity=(0.0, 0.0, -9.81), num_tools=1,
                tool_radius=(0.005, 0.005), flags=0, block_size=0,
                solver_variant=VARIANT_AUTO, colour_packing=PACKING_AUTO,
                envs_per_group=0, tool_shape=0, colouring=0) -> XpbdParams:
    p = XpbdParams()
    p.dt = dt
    p.substeps = substeps
    p.iterations = iterations
    p.gravity[:] = list(gravity)
    p.num_tools = num_tools
    r = list(tool_radius) + [0.0] * (2 - len(tool_radius))
    p.tool_radius[:] = r[:2]
    p.flags = flags
    p.block_size = block_size
    p.solver_variant = solver_variant
    p.colour_packing = colour_packing
    p.envs_per_group = envs_per_group
    p.tool_shape = tool_shape
    p.colouring = colouring
    return p


def default_stream():
    """torch's current HIP stream as a raw pointer (0 without a GPU)."""
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except ImportError:
        pass
    return 0


# --------------------------------------------------------------------- C names
def xpbd_last_error() -> str:
    return _lib.xpbd_last_error().decode()


_lib.xpbd_surface_faces.restype = ctypes.c_int
_lib.xpbd_surface_faces.argtypes = [ctypes.POINTER(XpbdMesh), ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p]


def xpbd_surface_faces(rest_pos, inv_mass, tets):
    """Host-only surface triangles and their colours (include/xpbd.h)."""
    keep = []
    mesh = _mesh_struct(rest_pos, inv_mass, tets, keep)
    counts = np.zeros(2, np.int32)
    _check(_lib.xpbd_surface_faces(ctypes.byref(mesh), counts.ctypes.data, None, None))
    faces = np.zeros((max(int(counts[0]), 1), 3), np.int32)
    colours = np.zeros(max(int(counts[0]), 1), np.int32)
    _check(_lib.xpbd_surface_faces(ctypes.byref(mesh), counts.ctypes.data, faces.ctypes.data,
                                   colours.ctypes.data))
    F = int(counts[0])
    return faces[:F], colours[:F], int(counts[1])


def xpbd_prepare_mesh(rest_pos, inv_mass, tets, colouring=0):
    """Host-only set-up of one mesh: dict of edges, tets, colours and rest values."""
    keep = []
    m = _mesh_struct(rest_pos, inv_mass, tets, keep)
    counts = np.zeros(4, np.int32)
    _check(_lib.xpbd_prepare_mesh_coloured(ctypes.byref(m), int(colouring), counts.ctypes.data,
                                           None, None, None, None))
    E, T = int(counts[0]), int(counts[1])
    edges = np.zeros((E, 2), np.int32)
    tout = np.zeros((T, 4), np.int32)
    colours = np.zeros(E + T, np.int32)
    rest = np.zeros(E + T, np.float32)
    _check(_lib.xpbd_prepare_mesh_coloured(ctypes.byref(m), int(colouring), counts.ctypes.data,
                                           edges.ctypes.data, tout.ctypes.data,
                                           colours.ctypes.data, rest.ctypes.data))
    return {"edges": edges, "tets": tout, "edge_colour": colours[:E], "tet_colour": colours[E:],
            "num_edge_colours": int(counts[2]), "num_tet_colours": int(counts[3]),
            "rest_length": rest[:E], "rest_volume": rest[E:]}


def xpbd_create_batch(meshes, env_mesh, compliance, params: XpbdParams, stream=None):
    """meshes: list of (rest_pos [V,3], inv_mass [V], tets [T,4]).  Returns a handle."""
    keep = []
    arr = (XpbdMesh * len(meshes))(*[_mesh_struct(*m, keep) for m in meshes])
    env_mesh = np.ascontiguousarray(env_mesh, dtype=np.int32)
    compliance = np.ascontiguousarray(compliance, dtype=np.float32).reshape(-1, 2)
    if compliance.shape[0] != env_mesh.shape[0]:
        raise ValueError("compliance must be [num_envs, 2]")
    out = ctypes.c_void_p()
    s = default_stream() if stream is None else stream
    _check(_lib.xpbd_create_batch(arr, len(meshes), env_mesh.ctypes.data, env_mesh.shape[0],
                                  compliance.ctypes.data, ctypes.byref(params), s or None,
                                  ctypes.byref(out)))
    _BATCHES[out.value] = (int(env_mesh.shape[0]), int(params.num_tools),
                           6 if params.tool_shape == TOOL_CAPSULE else 3)
    _SUBSTEPS[out.value] = int(params.substeps)
    return out.value


# LDS bandwidth probe (include/xpbd_probe.h)
PROBE_LDS_READ_B128 = 0
PROBE_LDS_WRITE_B96 = 1
_lib.xpbd_lds_probe.restype = ctypes.c_int
_lib.xpbd_lds_probe.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                ctypes.c_void_p]


def xpbd_lds_probe(kind, workgroups, reps, stream=None):
    """(ms, bytes, cycles per workgroup, 100 MHz ticks per workgroup) of one timed
    probe launch; see include/xpbd_probe.h."""
    out = np.zeros(4, np.float64)
    _check(_lib.xpbd_lds_probe(int(kind), int(workgroups), int(reps), stream, out.ctypes.data))
    return tuple(float(v) for v in out)


def xpbd_autotune(meshes, env_mesh, compliance, params: XpbdParams, num_steps, tool_pos,
                  stream=None):
    """Time the candidate launch configurations (see include/xpbd.h) and write the
    fastest into params.  tool_pos: [num_steps][N][tools][3] (host or device).
    Returns (ms per step of the choice, ms per step of the default)."""
    keep = []
    arr = (XpbdMesh * len(meshes))(*[_mesh_struct(*m, keep) for m in meshes])
    env_mesh = np.ascontiguousarray(env_mesh, dtype=np.int32)
    compliance = np.ascontiguousarray(compliance, dtype=np.float32).reshape(-1, 2)
    if compliance.shape[0] != env_mesh.shape[0]:
        raise ValueError("compliance must be [num_envs, 2]")
    n = int(env_mesh.shape[0])
    if params.num_tools:
        want = num_steps * n * params.num_tools * 3
        if tool_pos is None or int(np.prod(tool_pos.shape)) != want:
            raise ValueError(f"tool_pos must hold {want} floats")
    ms = (ctypes.c_float * 2)()
    s = default_stream() if stream is None else stream
    _check(_lib.xpbd_autotune(arr, len(meshes), env_mesh.ctypes.data, n, compliance.ctypes.data,
                              ctypes.byref(params), s or None, int(num_steps), _ptr(tool_pos),
                              _nbytes(tool_pos), ms))
    return float(ms[0]), float(ms[1])


def xpbd_step(batch, num_steps, tool_pos):
    """tool_pos: [num_steps][N][tools][3] float32, numpy (host) or torch (host/GPU).

    The kernel reads exactly num_steps * N * tools * 3 floats, so the buffer's
    element count and dtype are checked here before the launch."""
    tool_pos = _check_tool_pos(batch, num_steps, tool_pos)
    _check(_lib.xpbd_step(batch, int(num_steps), _ptr(tool_pos), _nbytes(tool_pos)))


def xpbd_set_flags(batch, flags):
    _check(_lib.xpbd_set_flags(batch, int(flags)))


def xpbd_field_bytes(batch, field) -> int:
    n = ctypes.c_size_t(0)
    _check(_lib.xpbd_field_bytes(batch, int(field), ctypes.byref(n)))
    return int(n.value)


def xpbd_read_state(batch, field, dst=None, raise_nonfinite=True):
    """Read a field into dst (numpy or torch); allocates a numpy array if dst is None."""
    if dst is None:
        n = xpbd_field_bytes(batch, field)
        dt = FIELD_DTYPES[field]
        dst = np.zeros(n // np.dtype(dt).itemsize, dtype=dt)
    s = _lib.xpbd_read_state(batch, int(field), _ptr(dst), _nbytes(dst))
    if s == XPBD_E_NONFINITE and not raise_nonfinite:
        return dst
    _check(s)
    return dst


def xpbd_write_state(batch, field, src):
    if isinstance(src, np.ndarray):
        src = np.ascontiguousarray(src, dtype=np.float32)
    _check(_lib.xpbd_write_state(batch, int(field), _ptr(src), _nbytes(src)))


def xpbd_get_batch_info(batch) -> dict:
    """The launch configuration the batch runs with (include/xpbd.h)."""
    info = XpbdBatchInfo()
    _check(_lib.xpbd_get_batch_info(batch, ctypes.byref(info)))
    return {name: int(getattr(info, name)) for name, _ in XpbdBatchInfo._fields_}


def xpbd_destroy_batch(batch):
    _BATCHES.pop(batch, None)
    _SUBSTEPS.pop(batch, None)
    _lib.xpbd_destroy_batch(batch)


def _check_tool_pos(batch, num_steps, tool_pos):
    n_envs, n_tools, per_tool = _BATCHES.get(batch, (None, None, 3))
    if isinstance(tool_pos, np.ndarray):
        tool_pos = np.ascontiguousarray(tool_pos, dtype=np.float32)
    if n_tools and num_steps > 0:
        need = int(num_steps) * n_envs * n_tools * per_tool
        if tool_pos is None:
            raise ValueError("tool_pos is required when the batch has tools")
        numel = tool_pos.size if isinstance(tool_pos, np.ndarray) else tool_pos.numel()
        if numel != need:
            raise ValueError(f"tool_pos has {numel} elements; the launch reads {need}")
        if not isinstance(tool_pos, np.ndarray) and str(tool_pos.dtype) != "torch.float32":
            raise TypeError("tool_pos must be float32")
    return tool_pos


def _check_per_substep(batch, num_steps, t, dtype_name, what):
    """A per-substep output buffer [num_steps * substeps * N] (device, contiguous)."""
    if t is None:
        return
    n = _device_rows(t, 1, dtype_name, what)
    n_envs, subs = _BATCHES.get(batch, (None,))[0], _SUBSTEPS.get(batch)
    if n_envs is not None and subs is not None and n < int(num_steps) * subs * n_envs:
        raise ValueError(f"{what} holds {n} values; the launch writes {int(num_steps) * subs * n_envs}")


def xpbd_mlp_create(params, in_shift, in_scale, out_shift, out_scale, stream=None):
    """params: float32 [MLP_PARAMS] or None; in_shift, in_scale [27]; out_shift,
    out_scale [3] (shifts may be None).  Returns a handle."""
    p = None if params is None else np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
    if p is not None and p.size != MLP_PARAMS:
        raise ValueError(f"params must have {MLP_PARAMS} values")

    def vec(a, n, name, optional=False):
        if a is None and optional:
            return None
        a = np.ascontiguousarray(a, dtype=np.float32).reshape(-1)
        if a.size != n:
            raise ValueError(f"{name} needs {n} values")
        return a
    ish, isc = vec(in_shift, MLP_FEATURES, "in_shift", True), vec(in_scale, MLP_FEATURES, "in_scale")
    osh, osc = vec(out_shift, MLP_OUTPUTS, "out_shift", True), vec(out_scale, MLP_OUTPUTS, "out_scale")
    out = ctypes.c_void_p()
    s = default_stream() if stream is None else stream
    _check(_lib.xpbd_mlp_create(_ptr(p), _ptr(ish), _ptr(isc), _ptr(osh), _ptr(osc), s or None,
                                ctypes.byref(out)))
    return out.value


def xpbd_mlp_get_params(net):
    out = np.zeros(MLP_PARAMS, np.float32)
    _check(_lib.xpbd_mlp_get_params(net, out.ctypes.data))
    return out


def xpbd_mlp_set_params(net, params):
    p = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
    if p.size != MLP_PARAMS:
        raise ValueError(f"params must have {MLP_PARAMS} values")
    _check(_lib.xpbd_mlp_set_params(net, p.ctypes.data))


def _device_rows(t, cols, dtype_name, what):
    if not hasattr(t, "data_ptr") or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{what} must be a contiguous device tensor")
    if str(t.dtype) != dtype_name or t.numel() % cols:
        raise TypeError(f"{what} must be {dtype_name} with rows of {cols}")
    return t.numel() // cols


def xpbd_mlp_forward(net, features, y):
    """features: device bfloat16 [n, 32]; y: device float32 [n, 4]."""
    n = _device_rows(features, MLP_FEATURE_STRIDE, "torch.bfloat16", "features")
    if _device_rows(y, 4, "torch.float32", "y") != n:
        raise ValueError("y needs one row per feature row")
    _check(_lib.xpbd_mlp_forward(net, _ptr(features), n, _ptr(y)))


_lib.xpbd_mlp_normalisation.restype = ctypes.c_int
_lib.xpbd_mlp_normalisation.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p]


def xpbd_mlp_normalisation(features, targets, stream=None):
    """(in_shift [27], in_scale [27], out_shift [3], out_scale [3]) float32 of a
    recording (device bfloat16 [n, 32], float32 [n, 4]); see include/xpbd_learned.h."""
    n = _device_rows(features, MLP_FEATURE_STRIDE, "torch.bfloat16", "features")
    if _device_rows(targets, 4, "torch.float32", "targets") != n:
        raise ValueError("targets need one row per feature row")
    ish, isc = np.zeros(MLP_FEATURES, np.float32), np.zeros(MLP_FEATURES, np.float32)
    osh, osc = np.zeros(3, np.float32), np.zeros(3, np.float32)
    _check(_lib.xpbd_mlp_normalisation(_ptr(features), _ptr(targets), n, stream, ish.ctypes.data,
                                       isc.ctypes.data, osh.ctypes.data, osc.ctypes.data))
    return ish, isc, osh, osc


def check_rows(rows, n):
    """Raise unless every index of the device int32 tensor rows lies in [0, n)
    (reads the tensor back: one synchronisation)."""
    if rows.numel() and (int(rows.min()) < 0 or int(rows.max()) >= n):
        raise ValueError("rows must index the feature table")


def xpbd_mlp_train_steps(net, features, targets, rows, batch, num_steps, first_rate, last_rate,
                         starts=None, losses=None, rows_checked=False):
    """num_steps training steps in one library call: step s on the window of
    ``batch`` entries of the device int32 row list ``rows`` that begins at
    starts[s] (host int64 array; None: s * batch) and wraps around its end,
    with a learning rate decaying geometrically from first_rate to last_rate;
    each step's loss to losses[s] (device float32) if given.  The row list is
    checked here against the tables unless rows_checked."""
    n = _device_rows(features, MLP_FEATURE_STRIDE, "torch.bfloat16", "features")
    if _device_rows(targets, 4, "torch.float32", "targets") != n:
        raise ValueError("targets need one row per feature row")
    num_rows = _device_rows(rows, 1, "torch.int32", "rows")
    if not rows_checked:
        check_rows(rows, n)
    if losses is not None and _device_rows(losses, 1, "torch.float32", "losses") < num_steps:
        raise ValueError("losses needs num_steps values")
    st = None
    if starts is not None:
        st = np.ascontiguousarray(starts, dtype=np.int64)
        if st.size < num_steps:
            raise ValueError("starts needs num_steps values")
    _check(_lib.xpbd_mlp_train_steps(net, _ptr(features), _ptr(targets), _ptr(rows), int(num_rows),
                                     _ptr(st), int(batch), int(num_steps), float(first_rate),
                                     float(last_rate), _ptr(losses)))


def xpbd_mlp_train_step(net, features, targets, learning_rate, grad=None, rows=None,
                        loss_out=None, rows_checked=False):
    """One training step on every row, or on the rows listed in ``rows`` (device
    int32, each index checked here against the tables unless the caller has
    checked them, rows_checked).  Returns the mean loss; with ``loss_out`` (a
    device float32 tensor of one value) the loss goes there in stream order
    instead and nothing synchronises (returns None)."""
    n = _device_rows(features, MLP_FEATURE_STRIDE, "torch.bfloat16", "features")
    if _device_rows(targets, 4, "torch.float32", "targets") != n:
        raise ValueError("targets need one row per feature row")
    if grad is not None and _device_rows(grad, MLP_PARAMS, "torch.float32", "grad") != 1:
        raise ValueError("grad must hold MLP_PARAMS values")
    count = n
    if rows is not None:
        count = _device_rows(rows, 1, "torch.int32", "rows")
        if not rows_checked:
            check_rows(rows, n)
    if loss_out is not None:
        if _device_rows(loss_out, 1, "torch.float32", "loss_out") < 1:
            raise ValueError("loss_out needs one value")
        _check(_lib.xpbd_mlp_train_step(net, _ptr(features), _ptr(targets), _ptr(rows), count,
                                        float(learning_rate), _ptr(loss_out), _ptr(grad)))
        return None
    loss = ctypes.c_float(0.0)
    _check(_lib.xpbd_mlp_train_step(net, _ptr(features), _ptr(targets), _ptr(rows), count,
                                    float(learning_rate), ctypes.addressof(loss), _ptr(grad)))
    return float(loss.value)


def xpbd_mlp_destroy(net):
    _lib.xpbd_mlp_destroy(net)


def xpbd_axis_neighbours(rest_pos):
    keep = []
    V = int(np.asarray(rest_pos).reshape(-1, 3).shape[0])
    m = _mesh_struct(rest_pos, np.ones(V, np.float32), np.zeros((1, 4), np.int32), keep)
    out = np.zeros((V, 6), np.int32)
    _check(_lib.xpbd_axis_neighbours(ctypes.byref(m), out.ctypes.data))
    return out


def xpbd_step_learned(batch, net, num_steps, tool_pos, min_iterations, max_iterations,
                      threshold, apply_correction=True, record_substep=-1, record_features=None,
                      record_targets=None, iterations=None, stall_ratio=0.0, residuals=None):
    """One substep per launch with the network's correction; see include/xpbd_learned.h.
    record_features / record_targets / iterations / residuals: device tensors (bfloat16
    [NP, 32], float32 [NP, 4], int32 and float32 [num_steps * substeps * N]) or None."""
    tool_pos = _check_tool_pos(batch, num_steps, tool_pos)
    _check_per_substep(batch, num_steps, iterations, "torch.int32", "iterations")
    _check_per_substep(batch, num_steps, residuals, "torch.float32", "residuals")
    lp = XpbdLearnedParams(int(bool(apply_correction)), int(min_iterations), int(max_iterations),
                           float(threshold), int(record_substep), _ptr(record_features),
                           _ptr(record_targets), _ptr(iterations), float(stall_ratio),
                           _ptr(residuals))
    _check(_lib.xpbd_step_learned(batch, net, int(num_steps), _ptr(tool_pos), _nbytes(tool_pos),
                                  ctypes.byref(lp)))


def xpbd_step_learned_noalloc(batch, net, num_steps, tool_pos, min_iterations, max_iterations,
                              threshold, apply_correction=True, record_substep=-1,
                              record_features=None, record_targets=None, iterations=None,
                              stall_ratio=0.0, residuals=None):
    """xpbd_step_learned without device allocation (workspace in the library's
    fixed device array); tool_pos must be a device tensor.  See
    include/xpbd_learned.h."""
    tool_pos = _check_tool_pos(batch, num_steps, tool_pos)
    _check_per_substep(batch, num_steps, iterations, "torch.int32", "iterations")
    _check_per_substep(batch, num_steps, residuals, "torch.float32", "residuals")
    lp = XpbdLearnedParams(int(bool(apply_correction)), int(min_iterations), int(max_iterations),
                           float(threshold), int(record_substep), _ptr(record_features),
                           _ptr(record_targets), _ptr(iterations), float(stall_ratio),
                           _ptr(residuals))
    _check(_lib.xpbd_step_learned_noalloc(batch, net, int(num_steps), _ptr(tool_pos),
                                          _nbytes(tool_pos), ctypes.byref(lp)))


class XpbdRlParams(ctypes.Structure):
    _fields_ = [("grasp_radius", ctypes.c_float), ("grasp_offset", ctypes.c_float * 3),
                ("max_speed", ctypes.c_float), ("obs_scale", ctypes.c_float),
                ("obs_origin", ctypes.c_float * 3), ("box_lo", ctypes.c_float * 3),
                ("box_hi", ctypes.c_float * 3), ("tracked", ctypes.c_int32 * RL_TRACKED)]


_lib.xpbd_policy_create.restype = ctypes.c_int
_lib.xpbd_policy_create.argtypes = [_V, ctypes.c_int64, _V, ctypes.POINTER(ctypes.c_void_p)]
_lib.xpbd_policy_destroy.restype = None
_lib.xpbd_policy_destroy.argtypes = [_V]
_lib.xpbd_rl_step.restype = ctypes.c_int
_lib.xpbd_rl_step.argtypes = [_V, _V, ctypes.POINTER(XpbdRlParams), ctypes.c_int32, _V, _V, _V,
                              _V, _V]


_lib.xpbd_rl_step_learned.restype = ctypes.c_int
_lib.xpbd_rl_step_learned.argtypes = [_V, _V, ctypes.POINTER(XpbdRlParams), _V,
                                      ctypes.POINTER(XpbdLearnedParams), ctypes.c_int32, _V, _V,
                                      _V, _V, _V]


def make_rl_params(grasp_radius, grasp_offset, max_speed, obs_scale, obs_origin, box_lo, box_hi,
                   tracked) -> XpbdRlParams:
    p = XpbdRlParams()
    p.grasp_radius = grasp_radius
    p.grasp_offset[:] = [float(v) for v in grasp_offset]
    p.max_speed = max_speed
    p.obs_scale = obs_scale
    p.obs_origin[:] = [float(v) for v in obs_origin]
    p.box_lo[:] = [float(v) for v in box_lo]
    p.box_hi[:] = [float(v) for v in box_hi]
    tr = [int(v) for v in np.asarray(tracked).reshape(-1)]
    if len(tr) != RL_TRACKED:
        raise ValueError(f"tracked needs {RL_TRACKED} particle ids")
    p.tracked[:] = tr
    return p


def xpbd_policy_create(params, stream=None):
    p = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
    h = ctypes.c_void_p()
    _check(_lib.xpbd_policy_create(p.ctypes.data, int(p.size),
                                   stream if stream is not None else default_stream(),
                                   ctypes.byref(h)))
    return h.value


def xpbd_policy_destroy(policy):
    _lib.xpbd_policy_destroy(policy)


def _check_rl_buffers(batch, num_steps, tool_pos, grasped, target, obs, actions):
    n_envs = _BATCHES.get(batch, (None,))[0]
    steps = int(num_steps)
    need = [(tool_pos, "torch.float32", n_envs * 6, "tool_pos"),
            (grasped, "torch.int32", n_envs, "grasped"),
            (target, "torch.float32", n_envs * 3, "target"),
            (obs, "torch.float32", steps * n_envs * RL_OBS, "obs"),
            (actions, "torch.float32", steps * n_envs * RL_ACTIONS, "actions")]
    for t, dtype, count, what in need:
        if t is None and what in ("obs", "actions"):
            continue
        if not hasattr(t, "data_ptr") or not t.is_cuda or not t.is_contiguous():
            raise TypeError(f"{what} must be a contiguous device tensor")
        if str(t.dtype) != dtype or t.numel() != count:
            raise ValueError(f"{what} must be {dtype} with {count} elements")


def xpbd_rl_step(batch, policy, params: XpbdRlParams, num_steps, tool_pos, grasped, target,
                 obs=None, actions=None):
    """RL steps on the batch's stream; every array is a contiguous device tensor:
    tool_pos float32 [N, 2, 3], grasped int32 [N] (both updated in place),
    target float32 [N, 3], obs float32 [num_steps, N, 64] or None, actions
    float32 [num_steps, N, 7] or None (sizes checked here)."""
    _check_rl_buffers(batch, num_steps, tool_pos, grasped, target, obs, actions)
    _check(_lib.xpbd_rl_step(batch, policy, ctypes.byref(params), int(num_steps), _ptr(tool_pos),
                             _ptr(grasped), _ptr(target), _ptr(obs), _ptr(actions)))


def xpbd_rl_step_learned(batch, policy, params: XpbdRlParams, net, num_steps, tool_pos, grasped,
                         target, min_iterations, max_iterations, threshold, obs=None,
                         actions=None, apply_correction=True, iterations=None, stall_ratio=0.0,
                         record_substep=-1, record_features=None, record_targets=None,
                         residuals=None):
    """xpbd_rl_step with the learned warm start (see include/xpbd_rl.h);
    iterations / residuals: device int32 / float32 [num_steps * substeps * N] or None."""
    _check_rl_buffers(batch, num_steps, tool_pos, grasped, target, obs, actions)
    _check_per_substep(batch, num_steps, iterations, "torch.int32", "iterations")
    _check_per_substep(batch, num_steps, residuals, "torch.float32", "residuals")
    lp = XpbdLearnedParams(int(bool(apply_correction)), int(min_iterations), int(max_iterations),
                           float(threshold), int(record_substep), _ptr(record_features),
                           _ptr(record_targets), _ptr(iterations), float(stall_ratio),
                           _ptr(residuals))
    _check(_lib.xpbd_rl_step_learned(batch, policy, ctypes.byref(params), net, ctypes.byref(lp),
                                     int(num_steps), _ptr(tool_pos), _ptr(grasped), _ptr(target),
                                     _ptr(obs), _ptr(actions)))


# captured steps (include/xpbd_graph.h)
_lib.xpbd_step_graph_create.restype = ctypes.c_int
_lib.xpbd_step_graph_create.argtypes = [_V, _V, ctypes.POINTER(XpbdLearnedParams), _V,
                                        ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p)]
_lib.xpbd_rl_graph_create.restype = ctypes.c_int
_lib.xpbd_rl_graph_create.argtypes = [_V, _V, ctypes.POINTER(XpbdRlParams), _V,
                                      ctypes.POINTER(XpbdLearnedParams), _V, _V, _V, _V, _V,
                                      ctypes.POINTER(ctypes.c_void_p)]
_lib.xpbd_graph_launch.restype = ctypes.c_int
_lib.xpbd_graph_launch.argtypes = [_V, ctypes.c_int32]
_lib.xpbd_graph_destroy.restype = None
_lib.xpbd_graph_destroy.argtypes = [_V]


def make_learned_params(min_iterations, max_iterations, threshold, apply_correction=True,
                        record_substep=-1, record_features=None, record_targets=None,
                        iterations=None, stall_ratio=0.0, residuals=None) -> XpbdLearnedParams:
    return XpbdLearnedParams(int(bool(apply_correction)), int(min_iterations),
                             int(max_iterations), float(threshold), int(record_substep),
                             _ptr(record_features), _ptr(record_targets), _ptr(iterations),
                             float(stall_ratio), _ptr(residuals))


def xpbd_step_graph_create(batch, net, learned, tool_pos):
    """One step (learned: XpbdLearnedParams or None) reading tool_pos (a
    contiguous device tensor [N, tools, 3]) at every replay."""
    n_envs, n_tools, per_tool = _BATCHES.get(batch, (None, None, 3))
    if n_tools:
        if not hasattr(tool_pos, "data_ptr") or not tool_pos.is_cuda or \
                not tool_pos.is_contiguous() or str(tool_pos.dtype) != "torch.float32" or \
                tool_pos.numel() != n_envs * n_tools * per_tool:
            raise ValueError("tool_pos must be a contiguous float32 device tensor of one step")
    h = ctypes.c_void_p()
    _check(_lib.xpbd_step_graph_create(batch, net, ctypes.byref(learned) if learned else None,
                                       _ptr(tool_pos), _nbytes(tool_pos), ctypes.byref(h)))
    return h.value


def xpbd_rl_graph_create(batch, policy, params: XpbdRlParams, net, learned, tool_pos, grasped,
                         target, obs=None, actions=None):
    _check_rl_buffers(batch, 1, tool_pos, grasped, target, obs, actions)
    h = ctypes.c_void_p()
    _check(_lib.xpbd_rl_graph_create(batch, policy, ctypes.byref(params), net,
                                     ctypes.byref(learned) if learned else None, _ptr(tool_pos),
                                     _ptr(grasped), _ptr(target), _ptr(obs), _ptr(actions),
                                     ctypes.byref(h)))
    return h.value


def xpbd_graph_launch(graph, times=1):
    _check(_lib.xpbd_graph_launch(graph, int(times)))


def xpbd_graph_destroy(graph):
    _lib.xpbd_graph_destroy(graph)


# --------------------------------------------------------------------- convenience
class Graph:
    """Owning wrapper around a captured step; keeps the buffers it names alive."""

    def __init__(self, handle, keep):
        self.handle = handle
        self._keep = keep

    def launch(self, times=1):
        xpbd_graph_launch(self.handle, times)

    def close(self):
        if self.handle:
            xpbd_graph_destroy(self.handle)
            self.handle = None
        self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Policy:
    """Owning wrapper around a policy handle."""

    def __init__(self, params, stream=None):
        self.handle = xpbd_policy_create(params, stream)

    def close(self):
        if self.handle:
            xpbd_policy_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Mlp:
    """Owning wrapper around a network handle."""

    def __init__(self, params, in_shift, in_scale, out_shift, out_scale, stream=None):
        self.handle = xpbd_mlp_create(params, in_shift, in_scale, out_shift, out_scale, stream)

    def params(self):
        return xpbd_mlp_get_params(self.handle)

    def set_params(self, params):
        xpbd_mlp_set_params(self.handle, params)

    def forward(self, features, y):
        xpbd_mlp_forward(self.handle, features, y)

    def train_steps(self, features, targets, rows, batch, num_steps, first_rate, last_rate,
                    starts=None, losses=None, rows_checked=False):
        xpbd_mlp_train_steps(self.handle, features, targets, rows, batch, num_steps, first_rate,
                             last_rate, starts, losses, rows_checked)

    def train_step(self, features, targets, learning_rate, grad=None, rows=None, loss_out=None,
                   rows_checked=False):
        return xpbd_mlp_train_step(self.handle, features, targets, learning_rate, grad, rows,
                                   loss_out, rows_checked)

    def close(self):
        if self.handle:
            xpbd_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Owning wrapper around a batch handle with numpy read-back helpers."""

    def __init__(self, meshes, env_mesh, compliance, params: XpbdParams, stream=None):
        self.handle = xpbd_create_batch(meshes, env_mesh, compliance, params, stream)
        self.params = params
        self.num_envs = int(np.asarray(env_mesh).shape[0])
        self.env_offsets = xpbd_read_state(self.handle, FIELD_ENV_OFFSETS)

    def step(self, num_steps, tool_pos):
        xpbd_step(self.handle, num_steps, tool_pos)

    def step_learned(self, net, num_steps, tool_pos, min_iterations, max_iterations, threshold,
                     **kw):
        xpbd_step_learned(self.handle, net.handle if net is not None else None, num_steps,
                          tool_pos, min_iterations, max_iterations, threshold, **kw)

    def step_learned_noalloc(self, net, num_steps, tool_pos, min_iterations, max_iterations,
                             threshold, **kw):
        xpbd_step_learned_noalloc(self.handle, net.handle if net is not None else None,
                                  num_steps, tool_pos, min_iterations, max_iterations,
                                  threshold, **kw)

    def rl_step(self, policy, params: XpbdRlParams, num_steps, tool_pos, grasped, target,
                obs=None, actions=None):
        xpbd_rl_step(self.handle, policy.handle, params, num_steps, tool_pos, grasped, target,
                     obs, actions)

    def rl_step_learned(self, policy, params: XpbdRlParams, net, num_steps, tool_pos, grasped,
                        target, min_iterations, max_iterations, threshold, **kw):
        xpbd_rl_step_learned(self.handle, policy.handle, params,
                             net.handle if net is not None else None, num_steps, tool_pos,
                             grasped, target, min_iterations, max_iterations, threshold, **kw)

    def step_graph(self, tool_pos, net=None, learned: XpbdLearnedParams = None):
        """A captured step (see include/xpbd_graph.h); learned from make_learned_params."""
        h = xpbd_step_graph_create(self.handle, net.handle if net is not None else None, learned,
                                   tool_pos)
        return Graph(h, (tool_pos, net, learned))

    def rl_graph(self, policy, params: XpbdRlParams, tool_pos, grasped, target, obs=None,
                 actions=None, net=None, learned: XpbdLearnedParams = None):
        h = xpbd_rl_graph_create(self.handle, policy.handle, params,
                                 net.handle if net is not None else None, learned, tool_pos,
                                 grasped, target, obs, actions)
        return Graph(h, (policy, params, tool_pos, grasped, target, obs, actions, net, learned))

    def read(self, field, dst=None, raise_nonfinite=True):
        return xpbd_read_state(self.handle, field, dst, raise_nonfinite)

    def info(self):
        return xpbd_get_batch_info(self.handle)

    def positions(self):
        return self.read(FIELD_POS).reshape(-1, 3)

    def velocities(self):
        return self.read(FIELD_VEL).reshape(-1, 3)

    def write(self, field, src):
        xpbd_write_state(self.handle, field, src)

    def set_flags(self, flags):
        xpbd_set_flags(self.handle, flags)

    def env_slice(self, e):
        return slice(int(self.env_offsets[e]), int(self.env_offsets[e + 1]))

    def close(self):
        if self.handle:
            xpbd_destroy_batch(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
