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
            "xpbd_prepare_mesh"]


class XpbdMesh(ctypes.Structure):
    _fields_ = [("num_vertices", ctypes.c_int32), ("num_tets", ctypes.c_int32),
                ("rest_pos", ctypes.c_void_p), ("inv_mass", ctypes.c_void_p),
                ("tets", ctypes.c_void_p)]


class XpbdParams(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_float), ("substeps", ctypes.c_int32),
                ("iterations", ctypes.c_int32), ("gravity", ctypes.c_float * 3),
                ("num_tools", ctypes.c_int32), ("tool_radius", ctypes.c_float * 2),
                ("flags", ctypes.c_uint32), ("block_size", ctypes.c_int32),
                ("solver_variant", ctypes.c_int32), ("colour_packing", ctypes.c_int32)]


_lib.xpbd_create_batch.restype = ctypes.c_int
_lib.xpbd_create_batch.argtypes = [ctypes.POINTER(XpbdMesh), ctypes.c_int32, ctypes.c_void_p,
                                   ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(XpbdParams),
                                   ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
_lib.xpbd_step.restype = ctypes.c_int
_lib.xpbd_step.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
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


# handle -> (num_envs, num_tools), to check tool-pose buffers before a launch
_BATCHES = {}


class XpbdError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _check(status):
    if status != XPBD_OK:
        raise XpbdError(status, xpbd_last_error())


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


def _nbytes(a):
    if isinstance(a, np.ndarray):
        return a.nbytes
    return a.numel() * a.element_size()


def _mesh_struct(rest_pos, inv_mass, tets, keep):
    rest_pos = np.ascontiguousarray(rest_pos, dtype=np.float32).reshape(-1, 3)
    inv_mass = np.ascontiguousarray(inv_mass, dtype=np.float32).reshape(-1)
    tets = np.ascontiguousarray(tets, dtype=np.int32).reshape(-1, 4)
    keep.extend([rest_pos, inv_mass, tets])
    return XpbdMesh(rest_pos.shape[0], tets.shape[0], rest_pos.ctypes.data,
                    inv_mass.ctypes.data, tets.ctypes.data)


def make_params(dt, substeps, iterations, gravity=(0.0, 0.0, -9.81), num_tools=1,
                tool_radius=(0.005, 0.005), flags=0, block_size=0,
                solver_variant=VARIANT_AUTO, colour_packing=PACKING_AUTO) -> XpbdParams:
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


def xpbd_prepare_mesh(rest_pos, inv_mass, tets):
    """Host-only set-up of one mesh: dict of edges, tets, colours and rest values."""
    keep = []
    m = _mesh_struct(rest_pos, inv_mass, tets, keep)
    counts = np.zeros(4, np.int32)
    _check(_lib.xpbd_prepare_mesh(ctypes.byref(m), counts.ctypes.data, None, None, None, None))
    E, T = int(counts[0]), int(counts[1])
    edges = np.zeros((E, 2), np.int32)
    tout = np.zeros((T, 4), np.int32)
    colours = np.zeros(E + T, np.int32)
    rest = np.zeros(E + T, np.float32)
    _check(_lib.xpbd_prepare_mesh(ctypes.byref(m), counts.ctypes.data, edges.ctypes.data,
                                  tout.ctypes.data, colours.ctypes.data, rest.ctypes.data))
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
    _BATCHES[out.value] = (int(env_mesh.shape[0]), int(params.num_tools))
    return out.value


def xpbd_step(batch, num_steps, tool_pos):
    """tool_pos: [num_steps][N][tools][3] float32, numpy (host) or torch (host/GPU).

    The kernel reads exactly num_steps * N * tools * 3 floats, so the buffer's
    element count and dtype are checked here before the launch."""
    n_envs, n_tools = _BATCHES.get(batch, (None, None))
    if isinstance(tool_pos, np.ndarray):
        tool_pos = np.ascontiguousarray(tool_pos, dtype=np.float32)
    if n_tools and num_steps > 0:
        need = int(num_steps) * n_envs * n_tools * 3
        if tool_pos is None:
            raise ValueError("tool_pos is required when the batch has tools")
        numel = tool_pos.size if isinstance(tool_pos, np.ndarray) else tool_pos.numel()
        if numel != need:
            raise ValueError(f"tool_pos has {numel} elements; the launch reads {need}")
        if not isinstance(tool_pos, np.ndarray) and str(tool_pos.dtype) != "torch.float32":
            raise TypeError("tool_pos must be float32")
    _check(_lib.xpbd_step(batch, int(num_steps), _ptr(tool_pos)))


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


def xpbd_destroy_batch(batch):
    _BATCHES.pop(batch, None)
    _lib.xpbd_destroy_batch(batch)


# --------------------------------------------------------------------- convenience
class Batch:
    """Owning wrapper around a batch handle with numpy read-back helpers."""

    def __init__(self, meshes, env_mesh, compliance, params: XpbdParams, stream=None):
        self.handle = xpbd_create_batch(meshes, env_mesh, compliance, params, stream)
        self.params = params
        self.num_envs = int(np.asarray(env_mesh).shape[0])
        self.env_offsets = xpbd_read_state(self.handle, FIELD_ENV_OFFSETS)

    def step(self, num_steps, tool_pos):
        xpbd_step(self.handle, num_steps, tool_pos)

    def read(self, field, dst=None, raise_nonfinite=True):
        return xpbd_read_state(self.handle, field, dst, raise_nonfinite)

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
