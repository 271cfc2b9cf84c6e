"""FP64 CPU oracle of the coupled LB / immersed-membrane step (test infrastructure).

This package is test infrastructure: only ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import it.  The product package
(``paper_1312_3426_amd``) never imports it, and it imports nothing from the
product package.  The numerical work is the plain C in ``oif_oracle.c``; this
module only marshals numpy arrays and applies object placement (rotation then
translation of template coordinates) on the oracle side.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
import threading
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oif_oracle.c")
_HDR = os.path.join(_HERE, "oif_oracle.h")
_LIB = os.path.join(_HERE, "liboif_oracle.so")
_LIB_OMP = os.path.join(_HERE, "liboif_oracle_omp.so")
_lock = threading.Lock()
_lib = None

D3Q19_E = np.array(
    [[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
     [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1], [1, 0, -1],
     [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], dtype=np.int64)
D3Q19_W = np.array([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12)


def build(force: bool = False, openmp: bool = False) -> str:
    """Compile the oracle with gcc (IEEE FP64, no fast-math, no FMA contraction).
    openmp=True builds the variant whose two lattice sweeps run on several host
    threads (same results bit for bit, see orc_threads); both are built when
    either is stale."""
    with _lock:
        stale = any((not os.path.exists(lib_)) or any(
            os.path.getmtime(p) > os.path.getmtime(lib_) for p in (_SRC, _HDR)) for lib_ in (_LIB, _LIB_OMP))
        if force or stale:
            for lib_, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
                tmp = lib_ + f".tmp{os.getpid()}"
                cmd = ["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-fPIC", "-shared",
                       "-ffp-contract=off", "-Wall", "-Wno-unknown-pragmas", *extra, "-o", tmp, _SRC, "-lm"]
                subprocess.run(cmd, check=True)
                os.replace(tmp, lib_)
    return _LIB_OMP if openmp else _LIB


class _Lattice(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("walls_z", C.c_int),
                ("tau", C.c_double), ("rho0", C.c_double), ("g", C.c_double * 3),
                ("xi", C.c_double), ("solid", C.c_void_p), ("wall_u", C.c_void_p),
                ("collision", C.c_int), ("gamma_shear", C.c_double), ("gamma_bulk", C.c_double),
                ("gamma_odd", C.c_double), ("gamma_even", C.c_double)]

BGK, MRT = 0, 1
EULER, VERLET = 0, 1


class _Mesh(C.Structure):
    _fields_ = [("n_tmpl", C.c_int), ("t_nv", C.c_void_p), ("t_nt", C.c_void_p),
                ("t_tri_off", C.c_void_p), ("tri", C.c_void_p), ("t_k", C.c_void_p),
                ("t_linear", C.c_void_p), ("n_obj", C.c_int), ("o_tmpl", C.c_void_p),
                ("o_node_off", C.c_void_p), ("o_mass", C.c_void_p), ("o_fext", C.c_void_p),
                ("t_model", C.c_void_p), ("integrator", C.c_int), ("o_type", C.c_void_p),
                ("n_pair", C.c_int), ("pair", C.c_void_p), ("n_wall", C.c_int), ("wall", C.c_void_p),
                ("n_shape", C.c_int), ("shape", C.c_void_p)]


class _SoftSphere(C.Structure):
    _fields_ = [("type_a", C.c_int), ("type_b", C.c_int), ("a", C.c_double), ("n", C.c_double),
                ("cutoff", C.c_double), ("offset", C.c_double)]


class _Shape(C.Structure):
    _fields_ = [("kind", C.c_int), ("corner", C.c_double * 3), ("a", C.c_double * 3), ("b", C.c_double * 3),
                ("c", C.c_double * 3), ("normal", C.c_double * 3), ("dist", C.c_double)]


def _shape(b) -> _Shape:
    sh = _Shape()
    sh.kind = 0 if b.kind == "rhomboid" else 1
    for c in range(3):
        sh.corner[c], sh.a[c], sh.b[c], sh.c[c] = b.corner[c], b.a[c], b.b[c], b.c[c]
        sh.normal[c] = b.normal[c]
    sh.dist = float(b.dist)
    return sh


def shape_distance(boundary, x) -> Optional[Tuple[float, np.ndarray]]:
    """(distance, unit direction from the closest surface point) of a point
    outside a boundary shape, None inside."""
    sh = _shape(boundary)
    d = C.c_double()
    u = np.zeros(3)
    ok = lib().orc_shape_distance(C.byref(sh), _p(_f64(x)), C.byref(d), _p(u))
    return (d.value, u) if ok else None

# force models (orc_membrane_forces)
MODEL_PAPER = 0
MODEL_CONSERVATIVE = 1


def model_code(model) -> int:
    """'paper' / 'conservative' (or the integer code) -> integer code."""
    if isinstance(model, str):
        return {"paper": MODEL_PAPER, "conservative": MODEL_CONSERVATIVE}[model]
    return int(model)


def lib():
    global _lib
    if _lib is None:
        # OIF_ORACLE_LIB lets the mutation test load a deliberately broken copy;
        # OIF_ORACLE_OPENMP=1 loads the build whose lattice sweeps use several
        # host threads (identical results)
        path = os.environ.get("OIF_ORACLE_LIB") or build(
            openmp=os.environ.get("OIF_ORACLE_OPENMP") == "1")
        L = C.CDLL(path)
        dp, ip, vp = C.c_void_p, C.c_void_p, C.c_void_p
        L.orc_kappa.restype = C.c_double
        L.orc_kappa.argtypes = [C.c_double]
        L.orc_topology.restype = C.c_int
        L.orc_topology.argtypes = [C.c_int, C.c_int, ip, ip, ip, ip]
        L.orc_geometry.restype = None
        L.orc_geometry.argtypes = [C.c_int, dp, C.c_int, ip, dp, dp, dp]
        L.orc_dihedral.restype = C.c_double
        L.orc_dihedral.argtypes = [dp, dp, dp, dp]
        L.orc_relaxed.restype = None
        L.orc_relaxed.argtypes = [C.c_int, dp, C.c_int, ip, C.c_int, ip, ip, dp, dp, dp, dp, dp]
        L.orc_membrane_forces.restype = None
        L.orc_wing_height.restype = None
        L.orc_wing_height.argtypes = [C.c_int, dp, C.c_int, ip, dp]
        L.orc_force_bend_gradient.restype = None
        L.orc_force_bend_gradient.argtypes = [C.c_int, dp, C.c_int, ip, dp, dp, C.c_double, dp]
        L.orc_force_local_area_balanced.restype = None
        L.orc_force_local_area_balanced.argtypes = [C.c_int, dp, C.c_int, ip, dp, C.c_double, dp]
        L.orc_force_global_area_balanced.restype = None
        L.orc_force_global_area_balanced.argtypes = [C.c_int, dp, C.c_int, ip, C.c_double, C.c_double, dp]
        L.orc_membrane_forces.argtypes = [C.c_int, dp, C.c_int, ip, C.c_int, ip, ip, dp, dp, dp,
                                          C.c_double, C.c_double, dp, C.c_int, C.c_int, dp, dp]
        L.orc_force_stretch.argtypes = [C.c_int, dp, C.c_int, ip, dp, C.c_double, C.c_int, dp]
        L.orc_force_bend.argtypes = [C.c_int, dp, C.c_int, ip, dp, C.c_double, dp]
        L.orc_force_local_area.argtypes = [C.c_int, dp, C.c_int, ip, dp, C.c_double, dp]
        L.orc_force_global_area.argtypes = [C.c_int, dp, C.c_int, ip, C.c_double, C.c_double, dp]
        L.orc_force_volume.argtypes = [C.c_int, dp, C.c_int, ip, C.c_double, C.c_double, dp]
        for f in (L.orc_force_stretch, L.orc_force_bend, L.orc_force_local_area,
                  L.orc_force_global_area, L.orc_force_volume):
            f.restype = None
        L.orc_moments.restype = None
        L.orc_moments.argtypes = [vp, dp, dp, dp, dp]
        L.orc_mark_rhomboid.restype = None
        L.orc_mark_rhomboid.argtypes = [vp, vp, C.c_int, dp, dp, dp, dp]
        L.orc_mark_wall.restype = None
        L.orc_mark_wall.argtypes = [vp, vp, C.c_int, dp, C.c_double]
        L.orc_lb_step.restype = None
        L.orc_lb_step.argtypes = [vp, dp, dp, dp]
        L.orc_stencil.restype = C.c_int
        L.orc_stencil.argtypes = [vp, dp, vp, dp]
        L.orc_couple_point.restype = C.c_int
        L.orc_couple_point.argtypes = [vp, dp, dp, dp, dp, dp]
        L.orc_system_create.restype = C.c_void_p
        L.orc_system_create.argtypes = [vp, vp, ip, dp]
        L.orc_system_destroy.restype = None
        L.orc_system_destroy.argtypes = [vp]
        L.orc_system_run.restype = C.c_int
        L.orc_system_run.argtypes = [vp, dp, dp, dp, C.c_int, dp]
        L.orc_system_geometry.restype = None
        L.orc_system_geometry.argtypes = [vp, dp, dp, dp]
        L.orc_system_forces.restype = None
        L.orc_system_forces.argtypes = [vp, dp, dp]
        L.orc_system_touched.restype = C.c_long
        L.orc_system_touched.argtypes = [vp, dp]
        L.orc_shape_distance.restype = C.c_int
        L.orc_shape_distance.argtypes = [vp, dp, vp, dp]
        L.orc_system_repulsion.restype = None
        L.orc_system_repulsion.argtypes = [vp, dp, dp]
        L.orc_system_get_force.restype = None
        L.orc_system_get_force.argtypes = [vp, dp]
        L.orc_system_set_force.restype = None
        L.orc_system_set_force.argtypes = [vp, dp]
        L.orc_threads.restype = C.c_int
        L.orc_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def threads(n: int = 0) -> int:
    """Host threads of the lattice sweeps (n > 0 sets them; 1 for the serial
    build); returns the number in use."""
    return int(lib().orc_threads(int(n)))


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


# ---------------------------------------------------------------------------
# mesh-level functions
# ---------------------------------------------------------------------------

def kappa(lam: float) -> float:
    return lib().orc_kappa(float(lam))


def topology(nv: int, tris) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(edges (ne,2), hinges (ne,4) = A,B,C,D, hinge_tri (ne,2)); raises on a
    non-manifold or inconsistently oriented mesh."""
    tris = _i32(tris)
    nt = len(tris)
    cap = 3 * nt // 2 + 1
    e = np.zeros((cap, 2), np.int32)
    h = np.zeros((cap, 4), np.int32)
    ht = np.zeros((cap, 2), np.int32)
    ne = lib().orc_topology(int(nv), nt, _p(tris), _p(e), _p(h), _p(ht))
    if ne < 0:
        raise ValueError("mesh is not closed, manifold and consistently oriented")
    return e[:ne].copy(), h[:ne].copy(), ht[:ne].copy()


def geometry(x, tris) -> Tuple[np.ndarray, float, float]:
    """(triangle areas, total area, volume) -- volume positive for inward orientation."""
    x = _f64(x)
    tris = _i32(tris)
    S = np.zeros(len(tris))
    A = C.c_double()
    V = C.c_double()
    lib().orc_geometry(len(x), _p(x), len(tris), _p(tris), _p(S), C.byref(A), C.byref(V))
    return S, A.value, V.value


def dihedral(xa, xb, xc, xd) -> float:
    a, b, c, d = (_f64(v) for v in (xa, xb, xc, xd))
    return lib().orc_dihedral(_p(a), _p(b), _p(c), _p(d))


class Relaxed:
    """Topology and relaxed values of one template."""

    def __init__(self, x, tris):
        x = _f64(x)
        self.tris = _i32(tris)
        self.nv = len(x)
        self.edges, self.hinges, self.hinge_tri = topology(self.nv, self.tris)
        ne = len(self.edges)
        self.L0 = np.zeros(ne)
        self.theta0 = np.zeros(ne)
        self.S0 = np.zeros(len(self.tris))
        Sg0 = C.c_double()
        V0 = C.c_double()
        lib().orc_relaxed(self.nv, _p(x), len(self.tris), _p(self.tris), ne, _p(self.edges),
                          _p(self.hinges), _p(self.L0), _p(self.theta0), _p(self.S0),
                          C.byref(Sg0), C.byref(V0))
        self.Sg0 = Sg0.value
        self.V0 = V0.value
        self.hbar = wing_height(x, self.hinges)

    def forces(self, x, ks=0.0, kb=0.0, kal=0.0, kag=0.0, kv=0.0, linear=False,
               model="paper") -> np.ndarray:
        x = _f64(x)
        F = np.zeros((self.nv, 3))
        k = _f64([ks, kb, kal, kag, kv])
        lib().orc_membrane_forces(self.nv, _p(x), len(self.tris), _p(self.tris), len(self.edges),
                                  _p(self.edges), _p(self.hinges), _p(self.L0), _p(self.theta0),
                                  _p(self.S0), self.Sg0, self.V0, _p(k), int(linear),
                                  model_code(model), _p(self.hbar), _p(F))
        return F

    def force_family(self, which: str, x, k: float, linear: bool = False) -> np.ndarray:
        x = _f64(x)
        F = np.zeros((self.nv, 3))
        L = lib()
        nt, ne = len(self.tris), len(self.edges)
        if which == "stretch":
            L.orc_force_stretch(self.nv, _p(x), ne, _p(self.edges), _p(self.L0), k, int(linear), _p(F))
        elif which == "bend":
            L.orc_force_bend(self.nv, _p(x), ne, _p(self.hinges), _p(self.theta0), k, _p(F))
        elif which == "local_area":
            L.orc_force_local_area(self.nv, _p(x), nt, _p(self.tris), _p(self.S0), k, _p(F))
        elif which == "global_area":
            L.orc_force_global_area(self.nv, _p(x), nt, _p(self.tris), self.Sg0, k, _p(F))
        elif which == "volume":
            L.orc_force_volume(self.nv, _p(x), nt, _p(self.tris), self.V0, k, _p(F))
        elif which == "bend_gradient":
            L.orc_force_bend_gradient(self.nv, _p(x), ne, _p(self.hinges), _p(self.theta0),
                                      _p(self.hbar), k, _p(F))
        elif which == "local_area_balanced":
            L.orc_force_local_area_balanced(self.nv, _p(x), nt, _p(self.tris), _p(self.S0), k, _p(F))
        elif which == "global_area_balanced":
            L.orc_force_global_area_balanced(self.nv, _p(x), nt, _p(self.tris), self.Sg0, k, _p(F))
        else:
            raise ValueError(which)
        return F


def wing_height(x, hinges) -> np.ndarray:
    """Mean relaxed wing height (S(A,B,C) + S(D,C,B)) / |C - B| of each hinge."""
    x, h = _f64(x), _i32(hinges)
    hbar = np.zeros(len(h))
    lib().orc_wing_height(len(x), _p(x), len(h), _p(h), _p(hbar))
    return hbar


def force_bend_gradient_hinges(x, hinges, theta0, hbar, kb) -> np.ndarray:
    """Gradient-form bending forces of an explicit hinge list (A, B, C, D)."""
    x, h, th, hb = _f64(x), _i32(hinges), _f64(theta0), _f64(hbar)
    F = np.zeros((len(x), 3))
    lib().orc_force_bend_gradient(len(x), _p(x), len(h), _p(h), _p(th), _p(hb), float(kb), _p(F))
    return F


def force_stretch_edges(x, edges, L0, ks, linear=False) -> np.ndarray:
    """Stretching forces of an explicit edge list (no closed mesh needed)."""
    x, e, L0 = _f64(x), _i32(edges), _f64(L0)
    F = np.zeros((len(x), 3))
    lib().orc_force_stretch(len(x), _p(x), len(e), _p(e), _p(L0), float(ks), int(linear), _p(F))
    return F


def force_bend_hinges(x, hinges, theta0, kb) -> np.ndarray:
    """Bending forces of an explicit hinge list (A, B, C, D)."""
    x, h, th = _f64(x), _i32(hinges), _f64(theta0)
    F = np.zeros((len(x), 3))
    lib().orc_force_bend(len(x), _p(x), len(h), _p(h), _p(th), float(kb), _p(F))
    return F


def force_triangles(which: str, x, tris, k, S0=None, Sg0=None, V0=None) -> np.ndarray:
    """Local-area, global-area or volume forces of an explicit triangle list."""
    x, t = _f64(x), _i32(tris)
    F = np.zeros((len(x), 3))
    L = lib()
    if which == "local_area":
        S0 = _f64(S0)
        L.orc_force_local_area(len(x), _p(x), len(t), _p(t), _p(S0), float(k), _p(F))
    elif which == "global_area":
        L.orc_force_global_area(len(x), _p(x), len(t), _p(t), float(Sg0), float(k), _p(F))
    elif which == "volume":
        L.orc_force_volume(len(x), _p(x), len(t), _p(t), float(V0), float(k), _p(F))
    elif which == "local_area_balanced":
        S0 = _f64(S0)
        L.orc_force_local_area_balanced(len(x), _p(x), len(t), _p(t), _p(S0), float(k), _p(F))
    elif which == "global_area_balanced":
        L.orc_force_global_area_balanced(len(x), _p(x), len(t), _p(t), float(Sg0), float(k), _p(F))
    else:
        raise ValueError(which)
    return F


# ---------------------------------------------------------------------------
# lattice-level functions
# ---------------------------------------------------------------------------

def _lattice(nx, ny, nz, tau=1.0, rho0=1.0, g=(0.0, 0.0, 0.0), xi=0.0, walls_z=False,
             obstacles=None, mrt=None) -> _Lattice:
    """Lattice descriptor; obstacles = (solid uint8 [N], wall_u float64 [nb+1][3])
    from ``boundary_field`` (the caller keeps the arrays alive); mrt = None (BGK
    with tau) or the rates (gamma_shear, gamma_bulk, gamma_odd, gamma_even) of
    the multiple-relaxation-time operator."""
    L = _Lattice()
    L.nx, L.ny, L.nz, L.walls_z = int(nx), int(ny), int(nz), int(bool(walls_z))
    L.tau, L.rho0, L.xi = float(tau), float(rho0), float(xi)
    if mrt is not None:
        L.collision = MRT
        L.gamma_shear, L.gamma_bulk, L.gamma_odd, L.gamma_even = (float(v) for v in mrt)
    for c in range(3):
        L.g[c] = float(g[c])
    if obstacles is not None:
        L.solid, L.wall_u = obstacles[0].ctypes.data, obstacles[1].ctypes.data
    return L


def boundary_field(nx, ny, nz, boundaries) -> Tuple[np.ndarray, np.ndarray]:
    """Solid-node field and wall velocities of a list of boundary descriptions
    (``synth.Boundary``-like: kind 'rhomboid' with corner, a, b, c or kind
    'wall' with normal, dist; velocity).  Boundary k (1-based, in list order)
    overwrites earlier ones where they overlap."""
    if len(boundaries) > 255:
        raise ValueError("at most 255 boundaries")
    solid = np.zeros((nz, ny, nx), dtype=np.uint8)
    wall_u = np.zeros((len(boundaries) + 1, 3))
    L = _lattice(nx, ny, nz)
    for k, b in enumerate(boundaries, start=1):
        wall_u[k] = b.velocity
        if b.kind == "rhomboid":
            lib().orc_mark_rhomboid(C.byref(L), solid.ctypes.data, k, _p(_f64(b.corner)), _p(_f64(b.a)),
                                    _p(_f64(b.b)), _p(_f64(b.c)))
        elif b.kind == "wall":
            lib().orc_mark_wall(C.byref(L), solid.ctypes.data, k, _p(_f64(b.normal)), float(b.dist))
        else:
            raise ValueError(b.kind)
    return solid, wall_u


def equilibrium_populations(nx, ny, nz, rho0=1.0) -> np.ndarray:
    """Rest state n_i = w_i rho0, layout (19, nz, ny, nx)."""
    return np.broadcast_to((D3Q19_W * rho0)[:, None, None, None], (19, nz, ny, nx)).copy()


def lb_step(n: np.ndarray, tau=1.0, g=(0.0, 0.0, 0.0), G: Optional[np.ndarray] = None,
            walls_z=False, obstacles=None, rho0=1.0, mrt=None) -> np.ndarray:
    n = _f64(n)
    _, nz, ny, nx = n.shape
    L = _lattice(nx, ny, nz, tau=tau, g=g, walls_z=walls_z, obstacles=obstacles, rho0=rho0, mrt=mrt)
    out = np.empty_like(n)
    Gp = None if G is None else _f64(G)
    lib().orc_lb_step(C.byref(L), _p(n), None if Gp is None else _p(Gp), _p(out))
    return out


def moments(n: np.ndarray, g=(0.0, 0.0, 0.0), G: Optional[np.ndarray] = None, obstacles=None,
            rho0=1.0) -> Tuple[np.ndarray, np.ndarray]:
    """(rho (nz,ny,nx), u (3,nz,ny,nx)) with u = (sum n e + F/2)/rho, F = g + G
    (rho0 and the wall velocity at solid nodes)."""
    n = _f64(n)
    _, nz, ny, nx = n.shape
    L = _lattice(nx, ny, nz, g=g, obstacles=obstacles, rho0=rho0)
    rho = np.empty((nz, ny, nx))
    u = np.empty((3, nz, ny, nx))
    Gp = None if G is None else _f64(G)
    lib().orc_moments(C.byref(L), _p(n), None if Gp is None else _p(Gp), _p(rho), _p(u))
    return rho, u


def stencil(X, dims, walls_z=False) -> Tuple[np.ndarray, np.ndarray, int]:
    nx, ny, nz = dims
    L = _lattice(nx, ny, nz, walls_z=walls_z)
    X = _f64(X)
    idx = np.zeros(8, np.int64)
    w = np.zeros(8)
    cl = lib().orc_stencil(C.byref(L), _p(X), _p(idx), _p(w))
    return idx, w, cl


def couple_point(u: np.ndarray, X, V, xi: float, walls_z=False, obstacles=None
                 ) -> Tuple[np.ndarray, np.ndarray]:
    """(G (3, nz, ny, nx) spread by one point, drag xi (V - u(X)))."""
    u = _f64(u)
    _, nz, ny, nx = u.shape
    L = _lattice(nx, ny, nz, xi=xi, walls_z=walls_z, obstacles=obstacles)
    G = np.zeros_like(u)
    drag = np.zeros(3)
    X, V = _f64(X), _f64(V)
    lib().orc_couple_point(C.byref(L), _p(u), _p(X), _p(V), _p(G), _p(drag))
    return G, drag


# ---------------------------------------------------------------------------
# coupled system
# ---------------------------------------------------------------------------

def euler_to_rot(rx: float, ry: float, rz: float) -> np.ndarray:
    """Rotation by rx about x, then ry about y, then rz about z (fixed axes):
    R = Rz Ry Rx."""
    cx, sx, cy, sy, cz, sz = math.cos(rx), math.sin(rx), math.cos(ry), math.sin(ry), math.cos(rz), math.sin(rz)
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


class System:
    """Coupled oracle system built from a ``synth.Box``-like description
    (duck-typed: nx, ny, nz, tau, rho0, g, friction, walls_z, templates, objects)."""

    def __init__(self, box):
        self.box = box
        bnd = list(getattr(box, "boundaries", []) or [])
        self.obstacles = boundary_field(box.nx, box.ny, box.nz, bnd) if bnd else None
        L = self._L = _lattice(box.nx, box.ny, box.nz, tau=box.tau, rho0=box.rho0, g=box.g,
                               xi=box.friction, walls_z=box.walls_z, obstacles=self.obstacles,
                               mrt=getattr(box, "mrt", None))
        # templates: apply the per-axis stretch to the node coordinates
        t_x, t_nv, t_nt, t_off, t_tri_off, tri, t_k, t_lin, t_mod = [], [], [], [], [], [], [], [], []
        noff = toff = 0
        self.t_nodes = []
        for t in box.templates:
            x = _f64(t.nodes) * _f64(t.stretch)[None, :]
            self.t_nodes.append(x)
            t_x.append(x)
            t_nv.append(len(x))
            t_nt.append(len(t.tris))
            t_off.append(noff)
            t_tri_off.append(toff)
            tri.append(_i32(t.tris))
            t_k.append([t.ks, t.kb, t.kal, t.kag, t.kv])
            t_lin.append(int(t.linear))
            t_mod.append(model_code(getattr(t, "model", "paper")))
            noff += len(x)
            toff += len(t.tris)
        self._keep = dict(
            t_x=_f64(np.concatenate(t_x) if t_x else np.zeros((1, 3))),
            t_nv=_i32(t_nv or [0]), t_nt=_i32(t_nt or [0]), t_off=_i32(t_off or [0]),
            t_tri_off=_i32(t_tri_off or [0]),
            tri=_i32(np.concatenate(tri) if tri else np.zeros((1, 3))),
            t_k=_f64(t_k or [[0] * 5]), t_lin=_i32(t_lin or [0]), t_mod=_i32(t_mod or [0]))
        # objects: X = origin + R x_template
        o_t, o_off, o_m, o_f, X0 = [], [], [], [], []
        off = 0
        for o in box.objects:
            R = np.eye(3) if o.rot is None else _f64(o.rot)
            xt = self.t_nodes[o.tid]
            X0.append(xt @ R.T + _f64(o.origin)[None, :])
            o_t.append(o.tid)
            o_off.append(off)
            o_m.append(o.mass if o.mass > 0 else 1.0)
            o_f.append(list(o.fext))
            off += len(xt)
        self.M = off
        self.obj_off = list(o_off)
        self._keep.update(o_t=_i32(o_t or [0]), o_off=_i32(o_off or [0]), o_m=_f64(o_m or [1]),
                          o_f=_f64(o_f or [[0, 0, 0]]))
        k = self._keep
        m = _Mesh()
        m.n_tmpl = len(box.templates)
        m.t_nv, m.t_nt, m.t_tri_off, m.tri = _p(k["t_nv"]), _p(k["t_nt"]), _p(k["t_tri_off"]), _p(k["tri"])
        m.t_k, m.t_linear, m.t_model = _p(k["t_k"]), _p(k["t_lin"]), _p(k["t_mod"])
        m.n_obj = len(box.objects)
        m.integrator = VERLET if getattr(box, "integrator", "euler") == "verlet" else EULER
        # soft-sphere repulsion
        rep = list(getattr(box, "repulsion", []) or [])
        pairs = [r for r in rep if r.type_b is not None]
        walls = [r for r in rep if r.type_b is None]
        PairArr = _SoftSphere * max(len(pairs), 1)
        WallArr = _SoftSphere * max(len(walls), 1)
        ShapeArr = _Shape * max(len(bnd), 1)
        pa, wa, sa = PairArr(), WallArr(), ShapeArr()
        for arr, lst in ((pa, pairs), (wa, walls)):
            for i, r in enumerate(lst):
                arr[i].type_a, arr[i].type_b = int(r.type_a), int(r.type_b if r.type_b is not None else -1)
                arr[i].a, arr[i].n, arr[i].cutoff, arr[i].offset = float(r.a), float(r.n), float(r.cutoff), float(r.offset)
        for i, b in enumerate(bnd):
            sa[i] = _shape(b)
        self._keep.update(o_type=_i32([getattr(o, "ptype", 0) for o in box.objects] or [0]), pa=pa, wa=wa, sa=sa)
        m.o_type = _p(self._keep["o_type"])
        m.n_pair, m.pair = len(pairs), C.addressof(pa)
        m.n_wall, m.wall = len(walls), C.addressof(wa)
        m.n_shape, m.shape = len(bnd), C.addressof(sa)
        m.o_tmpl, m.o_node_off, m.o_mass, m.o_fext = _p(k["o_t"]), _p(k["o_off"]), _p(k["o_m"]), _p(k["o_f"])
        self._mesh = m
        h = lib().orc_system_create(C.byref(L), C.byref(m), _p(k["t_off"]), _p(k["t_x"]))
        if not h:
            raise ValueError("oracle: mesh error in a template")
        self._h = h
        self.X = _f64(np.concatenate(X0)) if X0 else np.zeros((0, 3))
        self.V = np.zeros_like(self.X)
        self.n = equilibrium_populations(box.nx, box.ny, box.nz, box.rho0)
        self.last_diag = np.zeros(13)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_system_destroy(h)
            self._h = None

    def run(self, n_steps: int) -> None:
        d = np.zeros(13)
        Xp = self.X if self.M else np.zeros((1, 3))
        Vp = self.V if self.M else np.zeros((1, 3))
        rc = lib().orc_system_run(self._h, _p(self.n), _p(Xp), _p(Vp), int(n_steps), _p(d))
        self.last_diag = d
        if rc != 0:
            raise FloatingPointError(f"oracle: non-finite mesh state at step {-rc - 1}")

    @property
    def F(self) -> np.ndarray:
        """Total force of the last step per mesh node (carried by velocity Verlet)."""
        F = np.zeros((max(self.M, 1), 3))
        lib().orc_system_get_force(self._h, _p(F))
        return F[:self.M]

    @F.setter
    def F(self, value) -> None:
        F = np.ascontiguousarray(np.broadcast_to(_f64(value), (self.M, 3)))
        if self.M:
            lib().orc_system_set_force(self._h, _p(F))

    def geometry(self) -> Tuple[np.ndarray, np.ndarray]:
        no = len(self.box.objects)
        Sg = np.zeros(max(no, 1))
        Vo = np.zeros(max(no, 1))
        lib().orc_system_geometry(self._h, _p(self.X if self.M else np.zeros((1, 3))), _p(Sg), _p(Vo))
        return Sg[:no], Vo[:no]

    def repulsion(self) -> np.ndarray:
        """Soft-sphere forces on every mesh node at the current positions."""
        F = np.zeros((max(self.M, 1), 3))
        lib().orc_system_repulsion(self._h, _p(self.X if self.M else np.zeros((1, 3))), _p(F))
        return F[:self.M]

    def forces(self) -> np.ndarray:
        F = np.zeros((max(self.M, 1), 3))
        lib().orc_system_forces(self._h, _p(self.X if self.M else np.zeros((1, 3))), _p(F))
        return F[:self.M]

    def touched(self) -> int:
        if not self.M:
            return 0
        return int(lib().orc_system_touched(self._h, _p(self.X)))

    def fields(self) -> Dict[str, np.ndarray]:
        """Canonical output fields: populations, deviations from rest, density,
        velocity (with half the body force), mesh positions and velocities."""
        rho, u = moments(self.n, g=self.box.g, obstacles=self.obstacles, rho0=self.box.rho0)
        delta = self.n - (D3Q19_W * self.box.rho0)[:, None, None, None]
        return dict(n=self.n.copy(), delta=delta, rho=rho, u=u, X=self.X.copy(), V=self.V.copy())
