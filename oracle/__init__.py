"""FP64 CPU oracle for the batched XPBD substep (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It compiles ``xpbd_oracle.c`` with gcc
(no fused multiply-add) and wraps it with ctypes.  It shares nothing with the
GPU library: mesh set-up (orientation, rest values, edge extraction, greedy
colouring) and the simulation are recomputed here from the raw input arrays.

The arithmetic lives in ``xpbd_oracle.c``; its header lists the paper
passages followed and the readings taken where the paper is silent or
garbled.  This wrapper only marshals arrays, builds the colour schedule
(a stable sort of constraint ids by colour) and spreads independent
environments over threads.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "xpbd_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = True) -> str:
    """Compile the oracle shared library in-tree with gcc."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                        "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
                build(force=True)
            lib = ctypes.CDLL(_LIB_PATH)
            lib.oracle_tet_volume.restype = ctypes.c_double
            lib.oracle_tet_volume.argtypes = [_D, _D, _D, _D]
            lib.oracle_tet_gradients.restype = ctypes.c_double
            lib.oracle_tet_gradients.argtypes = [_D, _D]
            lib.oracle_project_distance.restype = None
            lib.oracle_project_distance.argtypes = [_D, _D, ctypes.c_int, ctypes.c_int,
                                                    ctypes.c_double, ctypes.c_double, _D]
            lib.oracle_project_volume.restype = None
            lib.oracle_project_volume.argtypes = [_D, _D, _I, ctypes.c_double, ctypes.c_double, _D]
            lib.oracle_project_contact.restype = None
            lib.oracle_project_contact.argtypes = [_D, _D, ctypes.c_double]
            lib.oracle_setup_tets.restype = ctypes.c_int
            lib.oracle_setup_tets.argtypes = [ctypes.c_int, _D, _D, ctypes.c_int, _I, _I, _D,
                                              ctypes.POINTER(ctypes.c_int)]
            lib.oracle_setup_edges.restype = ctypes.c_int
            lib.oracle_setup_edges.argtypes = [ctypes.c_int, _D, _D, ctypes.c_int, _I, _I, _D,
                                               ctypes.POINTER(ctypes.c_int)]
            lib.oracle_greedy_colour.restype = ctypes.c_int
            lib.oracle_greedy_colour.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _I, _I]
            lib.oracle_largest_first_colour.restype = ctypes.c_int
            lib.oracle_largest_first_colour.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                        _I, ctypes.c_int, ctypes.c_int, _I]
            lib.oracle_residual.restype = None
            lib.oracle_residual.argtypes = [_D, ctypes.c_int, _I, _D, ctypes.c_int, _I, _D,
                                            ctypes.c_double, ctypes.c_double, _D, _D]
            lib.oracle_candidates.restype = ctypes.c_int
            lib.oracle_candidates.argtypes = [ctypes.c_int, _D, _D, _D, ctypes.c_double, _I]
            lib.oracle_predict.restype = None
            lib.oracle_predict.argtypes = [ctypes.c_int, _D, ctypes.c_double, _D, _D, _D, _D]
            lib.oracle_iterate.restype = None
            lib.oracle_iterate.argtypes = [
                _D, _D, ctypes.c_int, _I, _D, _D, _I,
                ctypes.c_int, _I, _I, ctypes.c_int, _I, _I,
                ctypes.c_double, ctypes.c_double, _D,
                ctypes.c_int, ctypes.c_int, _D, _D, _I, ctypes.POINTER(ctypes.c_int)]
            lib.oracle_iterate_jacobi.restype = None
            lib.oracle_iterate_jacobi.argtypes = [
                _D, _D, ctypes.c_int, _I, _D, ctypes.c_int, _I, _D,
                ctypes.c_double, ctypes.c_double, _D, _I, _D,
                ctypes.c_int, ctypes.c_int, _D, _D, _I, ctypes.POINTER(ctypes.c_int)]
            lib.oracle_segment_triangle.restype = ctypes.c_double
            lib.oracle_segment_triangle.argtypes = [_D, _D, _D, _D, _D, _D, _D, _D]
            lib.oracle_project_capsule_face.restype = None
            lib.oracle_project_capsule_face.argtypes = [_D, _D, _I, _D, _D, ctypes.c_double]
            lib.oracle_project_capsule_faces.restype = None
            lib.oracle_project_capsule_faces.argtypes = [_D, _D, _I, _I, ctypes.c_int, _D, _D,
                                                         ctypes.c_double]
            lib.oracle_face_candidates.restype = ctypes.c_int
            lib.oracle_face_candidates.argtypes = [_D, _D, ctypes.c_int, _I, _I, _D, _D,
                                                   ctypes.c_double, _I]
            lib.oracle_grasp_select.restype = ctypes.c_int
            lib.oracle_grasp_select.argtypes = [ctypes.c_int, _D, _D, _D, ctypes.c_double, _D]
            lib.oracle_project_drag.restype = None
            lib.oracle_project_drag.argtypes = [_D, _D, ctypes.c_int, _D]
            lib.oracle_velocity.restype = None
            lib.oracle_velocity.argtypes = [ctypes.c_int, ctypes.c_double, _D, _D, _D]
            lib.oracle_run.restype = ctypes.c_int
            lib.oracle_run.argtypes = [
                ctypes.c_int, _D,
                ctypes.c_int, _I, _D,
                ctypes.c_int, _I, _D,
                ctypes.c_int, _I, _I,
                ctypes.c_int, _I, _I,
                ctypes.c_double, ctypes.c_int, ctypes.c_int, _D,
                ctypes.c_double, ctypes.c_double,
                ctypes.c_int, _D,
                ctypes.c_int, _D,
                _D, _D,
                _D, _I, _I, _D, ctypes.c_int]
            _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(_I) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class OracleError(RuntimeError):
    pass


# ---------------------------------------------------------------- primitives
def tet_volume(p):
    """Signed volume of a tetrahedron p[4][3] (float64)."""
    p = _f64(p).reshape(4, 3)
    rows = [np.ascontiguousarray(p[i]) for i in range(4)]
    return _load().oracle_tet_volume(*[_dp(r) for r in rows])


def tet_gradients(p):
    """(volume, gradients[4][3]) of the volume constraint at p[4][3]."""
    p = _f64(p).reshape(4, 3).copy()
    g = np.zeros((4, 3))
    vol = _load().oracle_tet_gradients(_dp(p), _dp(g))
    return vol, g


def project_distance(x, w, a, b, rest_length, alpha_tilde, lam=0.0):
    """One distance projection; returns (new x, new lambda)."""
    x = _f64(x).copy()
    w = _f64(w)
    lam_arr = np.array([lam], dtype=np.float64)
    _load().oracle_project_distance(_dp(x), _dp(w), int(a), int(b), float(rest_length),
                                    float(alpha_tilde), _dp(lam_arr))
    return x, float(lam_arr[0])


def project_volume(x, w, q, rest_volume, alpha_tilde, lam=0.0):
    """One volume projection of tetrahedron q; returns (new x, new lambda)."""
    x = _f64(x).copy()
    w = _f64(w)
    q = _i32(q)
    lam_arr = np.array([lam], dtype=np.float64)
    _load().oracle_project_volume(_dp(x), _dp(w), _ip(q), float(rest_volume),
                                  float(alpha_tilde), _dp(lam_arr))
    return x, float(lam_arr[0])


def project_contact(xi, centre, radius):
    xi = _f64(xi).copy()
    c = _f64(centre)
    _load().oracle_project_contact(_dp(xi), _dp(c), float(radius))
    return xi


def greedy_colour(num_vertices, verts):
    """Greedy colours of constraints verts[n][k]; returns (colours, count)."""
    verts = _i32(verts)
    n, k = verts.shape if verts.size else (0, max(1, verts.shape[-1] if verts.ndim == 2 else 1))
    out = np.zeros(max(n, 1), dtype=np.int32)
    nc = _load().oracle_greedy_colour(int(num_vertices), int(n), int(k), _ip(verts), _ip(out))
    if nc < 0:
        raise OracleError(f"oracle_greedy_colour failed: {nc}")
    return out[:n], nc


# colourings of the edge and tetrahedron constraints (R10, R13)
(COLOURING_GREEDY, COLOURING_LARGEST_FIRST, COLOURING_WAVES, COLOURING_CAPPED,
 COLOURING_CAPPED_128, COLOURING_CAPPED_FIT) = 0, 1, 2, 3, 4, 5
WAVE_CUT_ABOVE = 100
COLOUR_CAP = 256
COLOUR_CAP_128 = 128
FIT_COLOURS = 64      # CAPPED_FIT keeps the cap up to this many colours (kinds rounded to even)


def largest_first_colour(num_vertices, verts, cut_above=0, cap=0):
    """Largest-first colours of constraints verts[n][k] (R13); returns (colours, count)."""
    verts = _i32(verts)
    n, k = verts.shape
    out = np.zeros(max(n, 1), dtype=np.int32)
    nc = _load().oracle_largest_first_colour(int(num_vertices), int(n), int(k), _ip(verts),
                                             int(cut_above), int(cap), _ip(out))
    if nc < 0:
        raise OracleError(f"oracle_largest_first_colour failed: {nc}")
    return out[:n], nc


def colour(num_vertices, verts, colouring=COLOURING_GREEDY):
    """Colours of constraints verts[n][k] by the named colouring; (colours, count).
    CAPPED_FIT decides over both kinds of a mesh: see ``mesh_colours``."""
    if colouring == COLOURING_CAPPED_FIT:
        raise ValueError("CAPPED_FIT colours a mesh's two kinds together (mesh_colours)")
    if len(verts) == 0:
        return np.zeros(0, np.int32), 0
    if colouring == COLOURING_GREEDY:
        return greedy_colour(num_vertices, verts)
    cut = WAVE_CUT_ABOVE if colouring == COLOURING_WAVES else 0
    cap = {COLOURING_CAPPED: COLOUR_CAP, COLOURING_CAPPED_128: COLOUR_CAP_128}.get(colouring, 0)
    return largest_first_colour(num_vertices, verts, cut, cap)


def mesh_colours(num_vertices, edges, tets, colouring=COLOURING_GREEDY):
    """Colours of a mesh's edges and tetrahedra: ((edge colours, count), (tet
    colours, count)).  CAPPED_FIT (R13): the CAPPED colouring if its edge and
    tetrahedron colour counts, each rounded up to an even number, sum to at
    most FIT_COLOURS, else LARGEST_FIRST."""
    if colouring != COLOURING_CAPPED_FIT:
        return colour(num_vertices, edges, colouring), colour(num_vertices, tets, colouring)
    e, t = colour(num_vertices, edges, COLOURING_CAPPED), colour(num_vertices, tets, COLOURING_CAPPED)
    if e[1] + e[1] % 2 + t[1] + t[1] % 2 <= FIT_COLOURS:
        return e, t
    return (colour(num_vertices, edges, COLOURING_LARGEST_FIRST),
            colour(num_vertices, tets, COLOURING_LARGEST_FIRST))


def schedule(colours, num_colours):
    """Processing order: colour ascending, constraint id ascending inside a colour."""
    colours = np.asarray(colours, dtype=np.int64)
    order = np.argsort(colours, kind="stable").astype(np.int32)
    ptr = np.zeros(num_colours + 1, dtype=np.int32)
    if colours.size:
        ptr[1:] = np.cumsum(np.bincount(colours, minlength=num_colours))
    return ptr, order


def surface_faces(rest, tets):
    """Boundary triangles of a tetrahedral mesh (faces of exactly one
    tetrahedron), each ordered so that (x1 - x0) x (x2 - x0) points away from
    its tetrahedron's fourth vertex; sorted by their ascending vertex triple.
    Returns int32 [F][3]."""
    rest = _f64(rest).reshape(-1, 3)
    tets = _i32(tets).reshape(-1, 4)
    seen = {}
    for t in tets:
        for skip in range(4):
            tri = tuple(int(t[k]) for k in range(4) if k != skip)
            key = tuple(sorted(tri))
            seen.setdefault(key, []).append((tri, int(t[skip])))
    out = []
    for key in sorted(seen):
        if len(seen[key]) != 1:
            continue
        (i, j, k), l = seen[key][0]
        normal = np.cross(rest[j] - rest[i], rest[k] - rest[i])
        if np.dot(normal, rest[l] - rest[i]) > 0.0:
            j, k = k, j
        out.append((i, j, k))
    return np.array(out, dtype=np.int32).reshape(-1, 3)


def segment_triangle(p0, p1, a, b, c):
    """Closest points of segment p0 p1 and triangle (a, b, c):
    (squared distance, triangle point, segment point, barycentrics)."""
    q, s_, bary = np.zeros(3), np.zeros(3), np.zeros(3)
    d2 = _load().oracle_segment_triangle(*(_dp(_f64(v)) for v in (p0, p1, a, b, c)), _dp(q),
                                         _dp(s_), _dp(bary))
    return d2, q, s_, bary


def capsule_push(x, w, face, p0, p1, radius):
    """One push-out of a face (x updated in place)."""
    _load().oracle_project_capsule_face(_dp(x), _dp(_f64(w)), _ip(_i32(face)), _dp(_f64(p0)),
                                        _dp(_f64(p1)), float(radius))
    return x


# ---------------------------------------------------------------- mesh set-up
@dataclass
class OracleMesh:
    num_vertices: int
    w: np.ndarray             # [V] float64 inverse masses
    rest: np.ndarray          # [V,3] float64
    tets: np.ndarray          # [T,4] int32, kept + oriented, input order
    rest_volume: np.ndarray   # [T] float64
    edges: np.ndarray         # [E,2] int32, sorted, free
    rest_length: np.ndarray   # [E] float64
    edge_colour: np.ndarray   # [E] int32
    tet_colour: np.ndarray    # [T] int32
    num_edge_colours: int
    num_tet_colours: int
    edge_ptr: np.ndarray
    edge_order: np.ndarray
    tet_ptr: np.ndarray
    tet_order: np.ndarray
    faces: np.ndarray = None       # [F,3] int32 outward surface triangles
    face_colour: np.ndarray = None # [F] int32 greedy colours (faces sharing a particle differ)
    face_ptr: np.ndarray = None
    face_order: np.ndarray = None

    @property
    def num_edges(self):
        return int(self.edges.shape[0])

    @property
    def num_tets(self):
        return int(self.tets.shape[0])


def prepare_mesh(rest_pos, inv_mass, tets, colouring=COLOURING_GREEDY) -> OracleMesh:
    """Orientation, rest values, edges and colours of one mesh, from raw input;
    colouring names the colouring of the edges and tetrahedra (R10, R13)."""
    lib = _load()
    rest = _f64(rest_pos).reshape(-1, 3)
    w = _f64(inv_mass).reshape(-1)
    tin = _i32(tets).reshape(-1, 4)
    V, T = rest.shape[0], tin.shape[0]
    tout = np.zeros((max(T, 1), 4), dtype=np.int32)
    vol = np.zeros(max(T, 1))
    kept = ctypes.c_int(0)
    rc = lib.oracle_setup_tets(V, _dp(rest), _dp(w), T, _ip(tin), _ip(tout), _dp(vol),
                               ctypes.byref(kept))
    if rc != 0:
        raise OracleError(f"oracle_setup_tets failed: {rc}")
    T = kept.value
    tout, vol = tout[:T].copy(), vol[:T].copy()
    edges = np.zeros((max(6 * T, 1), 2), dtype=np.int32)
    rl = np.zeros(max(6 * T, 1))
    ne = ctypes.c_int(0)
    rc = lib.oracle_setup_edges(V, _dp(rest), _dp(w), T, _ip(tout), _ip(edges), _dp(rl),
                                ctypes.byref(ne))
    if rc != 0:
        raise OracleError(f"oracle_setup_edges failed: {rc}")
    E = ne.value
    edges, rl = edges[:E].copy(), rl[:E].copy()
    (ecol, nec), (tcol, ntc) = mesh_colours(V, edges, tout, colouring)
    eptr, eorder = schedule(ecol, nec)
    tptr, torder = schedule(tcol, ntc)
    faces = surface_faces(rest, tout) if T else np.zeros((0, 3), np.int32)
    fcol, nfc = greedy_colour(V, faces) if len(faces) else (np.zeros(0, np.int32), 0)
    fptr, forder = schedule(fcol, nfc)
    return OracleMesh(V, w, rest, tout, vol, edges, rl, ecol, tcol, nec, ntc,
                      eptr, eorder, tptr, torder, faces, fcol, fptr, forder)


# ---------------------------------------------------------------- simulation
@dataclass
class OracleParams:
    dt: float
    substeps: int
    iterations: int
    gravity: tuple
    num_tools: int = 1
    tool_radius: tuple = (0.005, 0.005)


@dataclass
class OracleResult:
    x: np.ndarray
    v: np.ndarray
    lam: np.ndarray | None = None
    contacts: np.ndarray | None = None        # [steps][tools][V]
    contact_count: np.ndarray | None = None   # [steps][tools]
    residual: np.ndarray | None = None        # [steps][substeps][2]


def run_env(mesh: OracleMesh, compliance, params: OracleParams, tool_pos, num_steps,
            x0=None, v0=None, want_lambda=False, want_contacts=False, want_residual=False,
            edge_schedule=None, tet_schedule=None, jacobi=False) -> OracleResult:
    """Advance one environment by ``num_steps`` steps.

    tool_pos: [num_steps][num_tools][3]; compliance: (alpha_edge, alpha_tet).
    edge_schedule / tet_schedule: optional (ptr, order) overriding the default
    colour order (used to check independence of the order inside a colour).
    jacobi: the paper's own parallel solver (``oracle_iterate_jacobi``:
    every constraint from the same positions, corrections averaged by each
    particle's number of constraints) instead of coloured Gauss-Seidel.
    """
    lib = _load()
    V, E, T = mesh.num_vertices, mesh.num_edges, mesh.num_tets
    nt = int(params.num_tools)
    x = _f64(mesh.rest if x0 is None else x0).reshape(V, 3).copy()
    v = np.zeros((V, 3)) if v0 is None else _f64(v0).reshape(V, 3).copy()
    tp = _f64(tool_pos).reshape(num_steps, nt, 3) if nt else np.zeros((1, 1, 3))
    radius = _f64(np.asarray(params.tool_radius[:max(nt, 1)]))
    grav = _f64(params.gravity)
    eptr, eorder = edge_schedule if edge_schedule is not None else (mesh.edge_ptr, mesh.edge_order)
    tptr, torder = tet_schedule if tet_schedule is not None else (mesh.tet_ptr, mesh.tet_order)
    eptr, eorder, tptr, torder = _i32(eptr), _i32(eorder), _i32(tptr), _i32(torder)
    lam = np.zeros(max(E + T, 1)) if want_lambda else None
    contacts = np.zeros((max(num_steps, 1), max(nt, 1), V), np.int32) if want_contacts else None
    ccount = np.zeros((max(num_steps, 1), max(nt, 1)), np.int32) if want_contacts else None
    resid = np.zeros((max(num_steps, 1), params.substeps, 2)) if want_residual else None
    edges = mesh.edges if E else np.zeros((1, 2), np.int32)
    tets = mesh.tets if T else np.zeros((1, 4), np.int32)
    rl = mesh.rest_length if E else np.ones(1)
    rv = mesh.rest_volume if T else np.ones(1)
    rc = lib.oracle_run(V, _dp(mesh.w), E, _ip(_i32(edges)), _dp(_f64(rl)),
                        T, _ip(_i32(tets)), _dp(_f64(rv)),
                        len(eptr) - 1, _ip(eptr), _ip(eorder if eorder.size else np.zeros(1, np.int32)),
                        len(tptr) - 1, _ip(tptr), _ip(torder if torder.size else np.zeros(1, np.int32)),
                        float(params.dt), int(params.substeps), int(params.iterations), _dp(grav),
                        float(compliance[0]), float(compliance[1]),
                        nt, _dp(radius), int(num_steps), _dp(np.ascontiguousarray(tp)),
                        _dp(x), _dp(v), _dp(lam), _ip(contacts), _ip(ccount), _dp(resid),
                        int(bool(jacobi)))
    if rc != 0:
        raise OracleError(f"oracle_run failed: {rc}")
    return OracleResult(x, v,
                        lam[:E + T] if lam is not None else None,
                        contacts[:num_steps, :nt] if contacts is not None else None,
                        ccount[:num_steps, :nt] if ccount is not None else None,
                        resid[:num_steps] if resid is not None else None)


def iterate(mesh: OracleMesh, x, alpha_tilde_d, alpha_tilde_v, lam=None, centres=None,
            radii=None, candidates=None):
    """One Gauss-Seidel iteration of ``oracle_iterate`` on one environment:
    x [V][3] and the multipliers lam [E+T] are updated in place (lam zeros
    if None); centres [tools][3], radii [tools] and candidates (one id list
    per tool) describe the sphere tools (none if None).  Returns (x, lam)."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    V, E, T = mesh.num_vertices, mesh.num_edges, mesh.num_tets
    lam = np.zeros(max(E + T, 1)) if lam is None else lam
    nt = 0 if centres is None else len(centres)
    cand = np.zeros((max(nt, 1), V), np.int32)
    ncand = (ctypes.c_int * max(nt, 1))()
    for t in range(nt):
        ids = np.asarray(candidates[t], np.int32)
        cand[t, :len(ids)] = ids
        ncand[t] = len(ids)
    c = _f64(np.asarray(centres, float).reshape(-1, 3)) if nt else np.zeros((1, 3))
    r = _f64(np.asarray(radii, float).reshape(-1)) if nt else np.zeros(1)
    lib.oracle_iterate(_dp(x), _dp(mesh.w), E, _ip(mesh.edges), _dp(mesh.rest_length),
                       _dp(mesh.rest_volume), _ip(mesh.tets),
                       mesh.num_edge_colours, _ip(mesh.edge_ptr), _ip(mesh.edge_order),
                       mesh.num_tet_colours, _ip(mesh.tet_ptr), _ip(mesh.tet_order),
                       float(alpha_tilde_d), float(alpha_tilde_v), _dp(lam),
                       V, nt, _dp(c), _dp(r), _ip(cand), ncand)
    return x, lam


def iterate_jacobi(x, w, edges, rest_length, tets, rest_volume, alpha_tilde_d=0.0,
                   alpha_tilde_v=0.0, lam=None):
    """One iteration of ``oracle_iterate_jacobi`` without tools, on raw arrays:
    x [V][3] (updated in place), w [V], edges [E][2], tets [T][4] (oriented),
    rest lengths / volumes, multipliers lam [E+T] (updated; zeros if None).
    The particle counts n are those of the given constraints."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    V = x.shape[0]
    edges = _i32(np.asarray(edges).reshape(-1, 2))
    tets = _i32(np.asarray(tets).reshape(-1, 4))
    E, T = edges.shape[0], tets.shape[0]
    count = np.zeros(V, np.int32)
    np.add.at(count, edges.ravel(), 1)
    np.add.at(count, tets.ravel(), 1)
    lam = np.zeros(max(E + T, 1)) if lam is None else lam
    dx = np.zeros((V, 3))
    ncand = (ctypes.c_int * 1)()
    lib.oracle_iterate_jacobi(_dp(x), _dp(_f64(w)), E, _ip(edges if E else np.zeros((1, 2), np.int32)),
                              _dp(_f64(rest_length if E else np.ones(1))), T,
                              _ip(tets if T else np.zeros((1, 4), np.int32)),
                              _dp(_f64(rest_volume if T else np.ones(1))),
                              float(alpha_tilde_d), float(alpha_tilde_v), _dp(lam), _ip(count),
                              _dp(dx), V, 0, None, None, None, ncand)
    return x, lam


def run_env_capsule(mesh: OracleMesh, compliance, params: OracleParams, capsules, num_steps,
                    x0=None, v0=None, want_contacts=False, jacobi=False):
    """Advance one environment with capsule tools against the surface faces
    (Sec. III-A.3) instead of spheres against particles.  capsules:
    [num_steps][num_tools][6] axis end points (p0, p1), radii
    params.tool_radius.  Per step: face candidates on the start-of-step
    positions; per iteration: the deformation constraints (the plain sweep of
    ``oracle_iterate``), then, per tool, the candidate faces in face-colour
    order pushed out with k_c = 1.  jacobi: the deformation constraints by
    ``oracle_iterate_jacobi`` instead."""
    lib = _load()
    V, E, T = mesh.num_vertices, mesh.num_edges, mesh.num_tets
    nt = int(params.num_tools)
    F = len(mesh.faces)
    x = _f64(mesh.rest if x0 is None else x0).reshape(V, 3).copy()
    v = np.zeros((V, 3)) if v0 is None else _f64(v0).reshape(V, 3).copy()
    cp = _f64(capsules).reshape(num_steps, nt, 6)
    radius = [float(params.tool_radius[t]) for t in range(nt)]
    grav = _f64(params.gravity)
    eptr, eorder, tptr, torder = (_i32(mesh.edge_ptr), _i32(mesh.edge_order),
                                  _i32(mesh.tet_ptr), _i32(mesh.tet_order))
    edges = _i32(mesh.edges if E else np.zeros((1, 2), np.int32))
    tets = _i32(mesh.tets if T else np.zeros((1, 4), np.int32))
    faces = _i32(mesh.faces if F else np.zeros((1, 3), np.int32))
    forder = _i32(mesh.face_order if F else np.zeros(1, np.int32))
    rl = _f64(mesh.rest_length if E else np.ones(1))
    rv = _f64(mesh.rest_volume if T else np.ones(1))
    h = float(params.dt) / params.substeps
    atd, atv = float(compliance[0]) / (h * h), float(compliance[1]) / (h * h)
    lam = np.zeros(max(E + T, 1))
    x_prev = np.zeros((V, 3))
    ncand0 = (ctypes.c_int * 1)()
    lists = [np.zeros(max(F, 1), np.int32) for _ in range(max(nt, 1))]
    count = np.zeros(V, np.int32)
    np.add.at(count, mesh.edges.ravel(), 1)
    np.add.at(count, mesh.tets.ravel(), 1)
    dx = np.zeros((V, 3))
    counts = np.zeros((num_steps, max(nt, 1)), np.int32)
    contacts = [] if want_contacts else None
    for step in range(num_steps):
        for t in range(nt):
            p0, p1 = np.ascontiguousarray(cp[step, t, :3]), np.ascontiguousarray(cp[step, t, 3:])
            counts[step, t] = lib.oracle_face_candidates(_dp(x), _dp(mesh.w), F, _ip(faces),
                                                         _ip(forder), _dp(p0), _dp(p1),
                                                         radius[t], _ip(lists[t]))
        if want_contacts:
            contacts.append([lists[t][:counts[step, t]].copy() for t in range(nt)])
        for sub in range(params.substeps):
            lib.oracle_predict(V, _dp(mesh.w), h, _dp(grav), _dp(x), _dp(v), _dp(x_prev))
            lam[:] = 0.0
            for _ in range(params.iterations):
                if jacobi:
                    lib.oracle_iterate_jacobi(_dp(x), _dp(mesh.w), E, _ip(edges), _dp(rl), T,
                                              _ip(tets), _dp(rv), atd, atv, _dp(lam),
                                              _ip(count), _dp(dx), V, 0, None, None, None,
                                              ncand0)
                else:
                    lib.oracle_iterate(_dp(x), _dp(mesh.w), E, _ip(edges), _dp(rl), _dp(rv),
                                       _ip(tets), len(eptr) - 1, _ip(eptr),
                                       _ip(eorder if eorder.size else np.zeros(1, np.int32)),
                                       len(tptr) - 1, _ip(tptr),
                                       _ip(torder if torder.size else np.zeros(1, np.int32)),
                                       atd, atv, _dp(lam), V, 0, None, None, None, ncand0)
                for t in range(nt):
                    p0 = np.ascontiguousarray(cp[step, t, :3])
                    p1 = np.ascontiguousarray(cp[step, t, 3:])
                    lib.oracle_project_capsule_faces(_dp(x), _dp(mesh.w), _ip(faces),
                                                     _ip(lists[t]), int(counts[step, t]),
                                                     _dp(p0), _dp(p1), radius[t])
            lib.oracle_velocity(V, h, _dp(x), _dp(x_prev), _dp(v))
    return OracleResult(x, v, None, contacts, counts, None)


def run_batch(meshes, env_mesh, compliance, params: OracleParams, tool_pos, num_steps,
              env_ids=None, threads=1, **kw):
    """Run independent environments (optionally on several threads).

    tool_pos: [num_steps][len(env_ids)][tools][3] for the selected envs.
    Returns a list of OracleResult in env_ids order.
    """
    env_ids = list(range(len(env_mesh))) if env_ids is None else list(env_ids)

    def one(n):
        e = env_ids[n]
        tp = tool_pos[:, n] if params.num_tools else None
        return run_env(meshes[int(env_mesh[e])], compliance[e], params, tp, num_steps, **kw)

    if threads <= 1:
        return [one(n) for n in range(len(env_ids))]
    with ThreadPoolExecutor(max_workers=threads) as pool:
        return list(pool.map(one, range(len(env_ids))))


def contact_candidates_f32(x, inv_mass, centre, radius):
    """Contact-candidate rule (reading R6) evaluated in single precision with
    every product and sum rounded separately, as the GPU kernel takes it:
    d = x - c; d2 = (dx*dx + dy*dy) + dz*dz; candidate iff w > 0 and
    d2 < (2r)^2 with (2r)^2 rounded to float32."""
    x = np.asarray(x, dtype=np.float32).reshape(-1, 3)
    c = np.asarray(centre, dtype=np.float32).reshape(3)
    d = x - c
    d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    reach = np.float32(2.0) * np.float32(radius)
    reach2 = reach * reach
    ok = (np.asarray(inv_mass, dtype=np.float32) > 0) & (d2 < reach2)
    return np.nonzero(ok)[0].astype(np.int32)


# ------------------------------------------------- learned warm start (extension)
@dataclass
class LearnedResult:
    x: np.ndarray
    v: np.ndarray
    iterations: np.ndarray     # [num_steps][substeps] iterations run
    residual: np.ndarray       # [num_steps][substeps][2] (RMS, max) after the last iteration
    early_residual: np.ndarray # [num_steps][substeps] RMS after min_iterations
    checks: np.ndarray         # [num_steps][substeps][max_iterations + 1] RMS after n sweeps
                               # wherever the driver evaluated it, else NaN


def run_env_learned(mesh: OracleMesh, compliance, params: OracleParams, tool_pos, num_steps,
                    corrector, min_iterations, max_iterations, threshold, x0=None, v0=None,
                    nbr=None, stall_ratio=0.0) -> LearnedResult:
    """Advance one environment with the learned warm start (see ``warmstart``).

    corrector(x_prev, v, x_hat, nbr) -> [V, 3] correction of the predicted
    positions (zero rows for pinned particles), or None for the plain solver.
    Per substep: predict (Alg. 1), add the correction, reset the multipliers,
    run min_iterations sweeps, evaluate the residual RMS r; if r exceeds
    ``threshold``, run sweeps up to max_iterations; then the velocity update.
    With 0 < stall_ratio and min_iterations >= 1, the residual is also
    evaluated before the last of the min_iterations sweeps, and the further
    sweeps run only if that sweep lowered it to at most stall_ratio times the
    value before it: a sweep that no longer lowers the residual marks a state
    the further sweeps cannot improve (as where the tool pushes particles back
    out against the constraints).
    """
    from . import warmstart as ws
    lib = _load()
    V, E, T = mesh.num_vertices, mesh.num_edges, mesh.num_tets
    nt = int(params.num_tools)
    x = _f64(mesh.rest if x0 is None else x0).reshape(V, 3).copy()
    v = np.zeros((V, 3)) if v0 is None else _f64(v0).reshape(V, 3).copy()
    tp = _f64(tool_pos).reshape(num_steps, nt, 3) if nt else np.zeros((num_steps, 1, 3))
    radius = _f64(np.asarray(params.tool_radius[:max(nt, 1)]))
    grav = _f64(params.gravity)
    nbr = ws.axis_neighbours(mesh.rest) if nbr is None else nbr
    eptr, eorder, tptr, torder = (_i32(mesh.edge_ptr), _i32(mesh.edge_order),
                                  _i32(mesh.tet_ptr), _i32(mesh.tet_order))
    edges = _i32(mesh.edges if E else np.zeros((1, 2), np.int32))
    tets = _i32(mesh.tets if T else np.zeros((1, 4), np.int32))
    rl = _f64(mesh.rest_length if E else np.ones(1))
    rv = _f64(mesh.rest_volume if T else np.ones(1))
    h = float(params.dt) / params.substeps
    atd, atv = float(compliance[0]) / (h * h), float(compliance[1]) / (h * h)
    lam = np.zeros(max(E + T, 1))
    cand = np.zeros((max(nt, 1), V), np.int32)
    ncand = (ctypes.c_int * max(nt, 1))()
    x_prev = np.zeros((V, 3))
    its = np.zeros((num_steps, params.substeps), np.int32)
    res = np.zeros((num_steps, params.substeps, 2))
    early = np.zeros((num_steps, params.substeps))
    checks = np.full((num_steps, params.substeps, max_iterations + 1), np.nan)
    r2 = np.zeros(2)

    def sweep(centres):
        lib.oracle_iterate(_dp(x), _dp(mesh.w), E, _ip(edges), _dp(rl), _dp(rv), _ip(tets),
                           len(eptr) - 1, _ip(eptr), _ip(eorder if eorder.size else np.zeros(1, np.int32)),
                           len(tptr) - 1, _ip(tptr), _ip(torder if torder.size else np.zeros(1, np.int32)),
                           atd, atv, _dp(lam), V, nt, _dp(centres), _dp(radius), _ip(cand), ncand)

    def residual():
        lib.oracle_residual(_dp(x), E, _ip(edges), _dp(rl), T, _ip(tets), _dp(rv), atd, atv,
                            _dp(lam), _dp(r2))
        return float(r2[0]), float(r2[1])

    for step in range(num_steps):
        centres = np.ascontiguousarray(tp[step])
        for t in range(nt):
            row = np.ascontiguousarray(cand[t])
            ncand[t] = lib.oracle_candidates(V, _dp(mesh.w), _dp(x), _dp(np.ascontiguousarray(centres[t])),
                                             float(radius[t]), _ip(row))
            cand[t] = row
        for sub in range(params.substeps):
            v_start = v.copy()
            lib.oracle_predict(V, _dp(mesh.w), h, _dp(grav), _dp(x), _dp(v), _dp(x_prev))
            if corrector is not None:
                x += corrector(x_prev, v_start, x, nbr)
            lam[:] = 0.0
            n_it = 0
            stall_check = stall_ratio > 0.0 and min_iterations >= 1
            for _ in range(min_iterations):
                if stall_check and n_it == min_iterations - 1:
                    checks[step, sub, n_it] = residual()[0]
                sweep(centres)
                n_it += 1
            r = early[step, sub] = checks[step, sub, n_it] = residual()[0]
            go_on = r > threshold
            if go_on and stall_check:
                go_on = r <= stall_ratio * checks[step, sub, n_it - 1]
            if go_on:
                while n_it < max_iterations:
                    sweep(centres)
                    n_it += 1
            its[step, sub] = n_it
            res[step, sub] = residual()
            lib.oracle_velocity(V, h, _dp(x), _dp(x_prev), _dp(v))
    return LearnedResult(x, v, its, res, early, checks)
