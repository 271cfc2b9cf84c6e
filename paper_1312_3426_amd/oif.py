"""ctypes binding of liboif.so (C ABI in include/oif.h).

Argument marshalling only: every step of the coupled lattice-Boltzmann /
membrane update runs in the HIP kernels of the library.  There is no CPU
fallback; loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboif.so")

OIF_OK = 0
ERRORS = {-1: "OIF_E_ARG", -2: "OIF_E_ID", -3: "OIF_E_MESH", -4: "OIF_E_STATE", -5: "OIF_E_NOMEM",
          -6: "OIF_E_HIP", -7: "OIF_E_NONFINITE", -8: "OIF_E_OVERFLOW", -9: "OIF_E_UNSUPPORTED"}
E_ARG, E_ID, E_MESH, E_STATE, E_NOMEM, E_HIP, E_NONFINITE, E_OVERFLOW, E_UNSUPPORTED = range(-1, -10, -1)

PREC_FP64, PREC_FP32, PREC_FP32_ST_FP16, PREC_FP32_ST_BF16 = 0, 1, 2, 3
PRECISIONS = {"fp64": PREC_FP64, "fp32": PREC_FP32, "fp16": PREC_FP32_ST_FP16, "bf16": PREC_FP32_ST_BF16}
STRETCH_NEOHOOKE, STRETCH_LINEAR = 0, 1
FORCES_PAPER, FORCES_CONSERVATIVE = 0, 1
_MODELS = {"paper": FORCES_PAPER, "conservative": FORCES_CONSERVATIVE}


class OifError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class LatticeDesc(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("walls_z", C.c_int),
                ("tau", C.c_double), ("rho0", C.c_double), ("body_force", C.c_double * 3),
                ("friction", C.c_double), ("precision", C.c_int), ("fp16_scale_exp", C.c_int),
                ("fixed_point_exp", C.c_int), ("device", C.c_int)]


class Moduli(C.Structure):
    _fields_ = [("ks", C.c_double), ("kb", C.c_double), ("kal", C.c_double), ("kag", C.c_double),
                ("kv", C.c_double), ("stretch_law", C.c_int), ("force_model", C.c_int)]


class Analysis(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("bounds", C.c_double * 6), ("volume", C.c_double),
                ("area", C.c_double), ("velocity", C.c_double * 3)]


class Info(C.Structure):
    _fields_ = [("n_templates", C.c_int), ("n_objects", C.c_int), ("precision", C.c_int),
                ("walls_z", C.c_int), ("n_nodes", C.c_longlong), ("n_mesh_nodes", C.c_longlong),
                ("steps_done", C.c_longlong), ("device_bytes", C.c_longlong), ("lb_block", C.c_int),
                ("mesh_block", C.c_int), ("xcd_remap", C.c_int), ("graph_steps", C.c_int),
                ("max_lds", C.c_longlong), ("lds_objects", C.c_int), ("overlap", C.c_int),
                ("integrator", C.c_int), ("lb_nontemporal", C.c_int), ("cpl_objects", C.c_int),
                ("cpl_lds_bytes", C.c_longlong), ("split_objects", C.c_int), ("split_workgroups", C.c_int),
                ("split_lds_bytes", C.c_longlong), ("force_clear_by_membrane", C.c_int)]


class Diag(C.Structure):
    _fields_ = [("mass", C.c_double), ("momentum_fluid", C.c_double * 3),
                ("momentum_mesh", C.c_double * 3), ("nonfinite", C.c_int), ("clamped", C.c_int),
                ("overflow", C.c_int)]


class Timing(C.Structure):
    _fields_ = [("total_ms", C.c_double), ("lb_ms", C.c_double), ("mesh_ms", C.c_double),
                ("lb_launches", C.c_int), ("mesh_launches", C.c_int), ("lb_touched_ms", C.c_double),
                ("mark_ms", C.c_double), ("overlap", C.c_int)]


_lib = None

# name -> (restype, argtypes); void pointers for arrays and handles
_vp, _i, _d, _ll = C.c_void_p, C.c_int, C.c_double, C.c_longlong
SIGNATURES = {
    "oif_lattice_desc_init": (_i, [_vp]),
    "oif_create": (_i, [_vp, _vp]),
    "oif_destroy": (_i, [_vp]),
    "oif_last_error": (C.c_char_p, [_vp]),
    "oif_bind_stream": (_i, [_vp, _vp]),
    "oif_population_bytes": (_i, [_vp, _vp]),
    "oif_bind_device_buffers": (_i, [_vp, _vp, _vp, C.c_size_t]),
    "oif_template_create": (_i, [_vp, _i, _vp, _i, _vp, _i, _vp, _vp]),
    "oif_object_add": (_i, [_vp, _i, _i, _vp, _vp, _d, _i]),
    "oif_euler_to_rot": (_i, [_d, _d, _d, _vp]),
    "oif_object_set_force": (_i, [_vp, _i, _vp]),
    "oif_object_set_origin": (_i, [_vp, _i, _vp]),
    "oif_object_set_nodes": (_i, [_vp, _i, _vp]),
    "oif_step": (_i, [_vp, _i]),
    "oif_step_timed": (_i, [_vp, _i, _vp]),
    "oif_set_graph": (_i, [_vp, _i]),
    "oif_set_overlap": (_i, [_vp, _i]),
    "oif_set_launch": (_i, [_vp, _i, _i, _i]),
    "oif_set_lb_loads": (_i, [_vp, _i]),
    "oif_set_force_clear": (_i, [_vp, _i]),
    "oif_set_mrt": (_i, [_vp, _vp]),
    "oif_set_integrator": (_i, [_vp, _i]),
    "oif_set_soft_sphere": (_i, [_vp, _i, _i, _d, _d, _d, _d]),
    "oif_set_wall_soft_sphere": (_i, [_vp, _i, _d, _d, _d, _d]),
    "oif_read_force": (_i, [_vp, _i, _vp]),
    "oif_write_force": (_i, [_vp, _i, _vp]),
    "oif_autotune": (_i, [_vp, C.c_char_p]),
    "oif_read_populations": (_i, [_vp, _vp]),
    "oif_write_populations": (_i, [_vp, _vp]),
    "oif_read_deviations": (_i, [_vp, _vp]),
    "oif_write_deviations": (_i, [_vp, _vp]),
    "oif_read_density": (_i, [_vp, _vp]),
    "oif_read_velocity": (_i, [_vp, _vp]),
    "oif_read_mesh": (_i, [_vp, _i, _vp, _vp]),
    "oif_write_mesh": (_i, [_vp, _i, _vp, _vp]),
    "oif_object_analyze": (_i, [_vp, _i, _vp]),
    "oif_info": (_i, [_vp, _vp]),
    "oif_diagnostics": (_i, [_vp, _vp]),
    "oif_diagnostics_noalloc": (_i, [_vp, _vp]),
    "oif_touched_nodes": (_i, [_vp, _vp]),
    "oif_boundary_rhomboid": (_i, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "oif_boundary_wall": (_i, [_vp, _vp, C.c_double, _vp, _vp]),
    "oif_boundary_clear": (_i, [_vp]),
    "oif_read_boundary": (_i, [_vp, _vp]),
    "oif_copy_bandwidth": (_i, [_i, _ll, _i, _vp]),
    "oif_batch_create": (_i, [_vp, _i, _vp]),
    "oif_batch_destroy": (_i, [_vp]),
    "oif_batch_step": (_i, [_vp, _i]),
    "oif_batch_set_graph": (_i, [_vp, _i]),
    "oif_batch_set_launch": (_i, [_vp, _i, _i, _i]),
    "oif_batch_set_lb_loads": (_i, [_vp, _i]),
    "oif_batch_set_persistent": (_i, [_vp, _i, _i]),
    "oif_batch_autotune": (_i, [_vp, C.c_char_p]),
    "oif_batch_step_timed": (_i, [_vp, _i, _vp]),
    "oif_batch_last_error": (C.c_char_p, [_vp]),
}


def lib():
    """Load liboif.so; raises if it was not built (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(paper_1312_3426_amd/build.py); there is no CPU fallback")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def copy_bandwidth(nbytes: int, reps: int = 20, device: int = 0) -> float:
    """GB/s (read + write) of a plain device copy kernel: the achievable-bandwidth reference."""
    v = C.c_double()
    rc = lib().oif_copy_bandwidth(int(device), int(nbytes), int(reps), C.byref(v))
    if rc != OIF_OK:
        raise OifError(rc, "oif_copy_bandwidth failed")
    return v.value


def euler_to_rot(rx: float, ry: float, rz: float) -> np.ndarray:
    R = np.zeros(9)
    lib().oif_euler_to_rot(rx, ry, rz, _p(R))
    return R.reshape(3, 3)


class Context:
    """One fluid box with its templates and objects (an ``oif_ctx``)."""

    def __init__(self, nx: int, ny: int, nz: int, *, tau: float = 1.0, rho0: float = 1.0,
                 body_force: Sequence[float] = (0.0, 0.0, 0.0), friction: float = 0.0,
                 walls_z: bool = False, precision="fp32", fp16_scale_exp: int = 12,
                 fixed_point_exp: int = 40, device: int = 0):
        L = lib()
        d = LatticeDesc()
        L.oif_lattice_desc_init(C.byref(d))
        d.nx, d.ny, d.nz, d.walls_z = int(nx), int(ny), int(nz), int(bool(walls_z))
        d.tau, d.rho0, d.friction = float(tau), float(rho0), float(friction)
        for k in range(3):
            d.body_force[k] = float(body_force[k])
        d.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        d.fp16_scale_exp, d.fixed_point_exp, d.device = int(fp16_scale_exp), int(fixed_point_exp), int(device)
        self.desc = d
        h = C.c_void_p()
        rc = L.oif_create(C.byref(d), C.byref(h))
        if rc != OIF_OK:
            raise OifError(rc, "oif_create failed")
        self.h = h
        self.shape = (nz, ny, nx)
        self.N = nx * ny * nz
        self._obj_nv = []
        self._tmpl_nv = []

    # -- plumbing --
    def _chk(self, rc: int):
        if rc != OIF_OK:
            raise OifError(rc, lib().oif_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib().oif_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def bind_stream(self, stream_ptr: Optional[int]):
        self._chk(lib().oif_bind_stream(self.h, stream_ptr))

    def population_bytes(self) -> int:
        """Bytes of each of the two population buffers."""
        n = C.c_size_t()
        self._chk(lib().oif_population_bytes(self.h, C.byref(n)))
        return n.value

    def bind_device_buffers(self, f0, f1, nbytes: Optional[int] = None):
        """Keep the population buffers in caller-owned device memory: two
        objects with ``data_ptr()`` and ``nbytes`` (e.g. PyTorch tensors on
        the context's device), or two addresses with ``nbytes`` given; both
        None returns them to the context.  The caller keeps the memory alive
        while it is bound."""
        if f0 is None and f1 is None:
            self._chk(lib().oif_bind_device_buffers(self.h, None, None, 0))
            self._bound = None
            return
        if (f0 is None) != (f1 is None):  # the library refuses it too
            raise ValueError("bind both population buffers or neither")
        ptrs = [t if isinstance(t, int) else t.data_ptr() for t in (f0, f1)]
        if nbytes is None:
            nbytes = min(int(t.nbytes) for t in (f0, f1))
        self._chk(lib().oif_bind_device_buffers(self.h, ptrs[0], ptrs[1], int(nbytes)))
        self._bound = (f0, f1)  # keeps Python-owned buffers alive while bound

    # -- templates and objects --
    def template_create(self, tid: int, nodes, tris, stretch=None, ks=0.0, kb=0.0, kal=0.0, kag=0.0,
                        kv=0.0, linear: bool = False, model="paper"):
        nodes = _f64(nodes)
        tris = np.ascontiguousarray(tris, dtype=np.int32)
        m = _MODELS[model] if isinstance(model, str) else int(model)
        k = Moduli(ks, kb, kal, kag, kv, STRETCH_LINEAR if linear else STRETCH_NEOHOOKE, m)
        st = None if stretch is None else _f64(stretch)
        self._chk(lib().oif_template_create(self.h, tid, _p(nodes), len(nodes), _p(tris), len(tris),
                                            _p(st), C.byref(k)))
        self._tmpl_nv.append(len(nodes))

    def object_add(self, oid: int, tid: int, origin, rot=None, mass: float = 1.0, part_type: int = 0):
        o = _f64(origin)
        R = None if rot is None else _f64(rot).reshape(9)
        self._chk(lib().oif_object_add(self.h, oid, tid, _p(o), _p(R), float(mass), int(part_type)))
        self._obj_nv.append(self._tmpl_nv[tid])

    def object_set_force(self, oid: int, f):
        self._chk(lib().oif_object_set_force(self.h, oid, _p(_f64(f))))

    def object_set_origin(self, oid: int, o):
        self._chk(lib().oif_object_set_origin(self.h, oid, _p(_f64(o))))

    def object_set_nodes(self, oid: int, x):
        self._chk(lib().oif_object_set_nodes(self.h, oid, _p(_f64(x))))

    # -- stepping --
    def step(self, n: int = 1):
        self._chk(lib().oif_step(self.h, int(n)))

    def step_timed(self, n: int) -> Timing:
        t = Timing()
        self._chk(lib().oif_step_timed(self.h, int(n), C.byref(t)))
        return t

    def set_graph(self, steps_per_graph: int):
        self._chk(lib().oif_set_graph(self.h, int(steps_per_graph)))

    def set_launch(self, lb_block: int = -1, mesh_block: int = -1, xcd_remap: int = -1):
        self._chk(lib().oif_set_launch(self.h, int(lb_block), int(mesh_block), int(xcd_remap)))

    def set_lb_loads(self, nontemporal: bool):
        """Population reads of the lattice kernel non-temporal (True) or ordinary."""
        self._chk(lib().oif_set_lb_loads(self.h, int(bool(nontemporal))))

    def set_force_clear(self, by_membrane: bool):
        """Coupling force cleared by the membrane kernel from its slot lists
        (True) or by the lattice kernel where it reads it (False)."""
        self._chk(lib().oif_set_force_clear(self.h, int(bool(by_membrane))))

    def set_mrt(self, gamma=None):
        """Multiple-relaxation-time collision with the factors (shear, bulk,
        odd, even); None returns to BGK."""
        if gamma is None:
            self._chk(lib().oif_set_mrt(self.h, None))
        else:
            g = np.ascontiguousarray(np.asarray(gamma, dtype=np.float64).reshape(4))
            self._chk(lib().oif_set_mrt(self.h, g.ctypes.data))

    def set_soft_sphere(self, type_a: int, type_b: int, a: float, n: float, cutoff: float, offset: float = 0.0):
        self._chk(lib().oif_set_soft_sphere(self.h, int(type_a), int(type_b), float(a), float(n), float(cutoff),
                                            float(offset)))

    def set_wall_soft_sphere(self, ptype: int, a: float, n: float, cutoff: float, offset: float = 0.0):
        self._chk(lib().oif_set_wall_soft_sphere(self.h, int(ptype), float(a), float(n), float(cutoff),
                                                 float(offset)))

    def set_integrator(self, name: str):
        """Mesh integrator: "euler" (default) or "verlet"."""
        code = {"euler": 0, "verlet": 1}[name]
        self._chk(lib().oif_set_integrator(self.h, code))

    def read_force(self, oid: int = -1) -> np.ndarray:
        """Force carried into the next step by velocity Verlet, (n, 3)."""
        n = self._nv(oid)
        F = np.empty((n, 3))
        self._chk(lib().oif_read_force(self.h, int(oid), F.ctypes.data))
        return F

    def write_force(self, oid: int, F) -> None:
        n = self._nv(oid)
        F = np.ascontiguousarray(np.broadcast_to(np.asarray(F, dtype=np.float64), (n, 3)))
        self._chk(lib().oif_write_force(self.h, int(oid), F.ctypes.data))

    def set_overlap(self, on: bool):
        self._chk(lib().oif_set_overlap(self.h, int(bool(on))))

    def autotune(self, cache_path: Optional[str] = None):
        self._chk(lib().oif_autotune(self.h, None if cache_path is None else cache_path.encode()))

    # -- read-back --
    def read_populations(self) -> np.ndarray:
        out = np.empty((19,) + self.shape)
        self._chk(lib().oif_read_populations(self.h, _p(out)))
        return out

    def write_populations(self, n) -> None:
        n = _f64(n)
        assert n.size == 19 * self.N
        self._chk(lib().oif_write_populations(self.h, _p(n)))

    def read_deviations(self) -> np.ndarray:
        """The stored deviations n_i - w_i rho0, exact in every storage form
        (the checkpoint form of the lattice state)."""
        out = np.empty((19,) + self.shape)
        self._chk(lib().oif_read_deviations(self.h, _p(out)))
        return out

    def write_deviations(self, d) -> None:
        d = _f64(d)
        assert d.size == 19 * self.N
        self._chk(lib().oif_write_deviations(self.h, _p(d)))

    def read_density(self) -> np.ndarray:
        out = np.empty(self.shape)
        self._chk(lib().oif_read_density(self.h, _p(out)))
        return out

    def read_velocity(self) -> np.ndarray:
        out = np.empty((3,) + self.shape)
        self._chk(lib().oif_read_velocity(self.h, _p(out)))
        return out

    def _nv(self, oid: int) -> int:
        return sum(self._obj_nv) if oid < 0 else self._obj_nv[oid]

    def read_mesh(self, oid: int = -1):
        n = self._nv(oid)
        X = np.empty((n, 3))
        V = np.empty((n, 3))
        self._chk(lib().oif_read_mesh(self.h, int(oid), _p(X), _p(V)))
        return X, V

    def write_mesh(self, oid: int = -1, X=None, V=None):
        Xp = None if X is None else _f64(X)
        Vp = None if V is None else _f64(V)
        self._chk(lib().oif_write_mesh(self.h, int(oid), _p(Xp), _p(Vp)))

    def object_analyze(self, oid: int) -> Analysis:
        a = Analysis()
        self._chk(lib().oif_object_analyze(self.h, oid, C.byref(a)))
        return a

    def info(self) -> Info:
        i = Info()
        self._chk(lib().oif_info(self.h, C.byref(i)))
        return i

    def diagnostics(self) -> Diag:
        d = Diag()
        self._chk(lib().oif_diagnostics(self.h, C.byref(d)))
        return d

    def diagnostics_noalloc(self) -> Diag:
        """oif_diagnostics without device allocation (fixed per-device scratch)."""
        d = Diag()
        self._chk(lib().oif_diagnostics_noalloc(self.h, C.byref(d)))
        return d

    def touched_nodes(self) -> int:
        v = C.c_longlong()
        self._chk(lib().oif_touched_nodes(self.h, C.byref(v)))
        return v.value

    # -- obstacles --
    def boundary_rhomboid(self, corner, a, b, c, velocity=None) -> int:
        bid = C.c_int()
        v = None if velocity is None else _p(_f64(velocity))
        self._chk(lib().oif_boundary_rhomboid(self.h, _p(_f64(corner)), _p(_f64(a)), _p(_f64(b)),
                                              _p(_f64(c)), v, C.byref(bid)))
        return bid.value

    def boundary_wall(self, normal, dist, velocity=None) -> int:
        bid = C.c_int()
        v = None if velocity is None else _p(_f64(velocity))
        self._chk(lib().oif_boundary_wall(self.h, _p(_f64(normal)), float(dist), v, C.byref(bid)))
        return bid.value

    def boundary_clear(self):
        self._chk(lib().oif_boundary_clear(self.h))

    def read_boundary(self) -> np.ndarray:
        out = np.empty(self.shape, dtype=np.uint8)
        self._chk(lib().oif_read_boundary(self.h, out.ctypes.data))
        return out

    # -- convenience: build from a workload description --
    @classmethod
    def from_box(cls, box, precision="fp32", **kw) -> "Context":
        """Create a context from a ``synth.Box``-like description (duck-typed)."""
        c = cls(box.nx, box.ny, box.nz, tau=box.tau, rho0=box.rho0, body_force=box.g,
                friction=box.friction, walls_z=box.walls_z, precision=precision, **kw)
        if getattr(box, "mrt", None) is not None:
            c.set_mrt(box.mrt)
        if getattr(box, "integrator", "euler") != "euler":
            c.set_integrator(box.integrator)
        for bnd in getattr(box, "boundaries", []) or []:
            if bnd.kind == "rhomboid":
                c.boundary_rhomboid(bnd.corner, bnd.a, bnd.b, bnd.c, bnd.velocity)
            else:
                c.boundary_wall(bnd.normal, bnd.dist, bnd.velocity)
        for tid, t in enumerate(box.templates):
            c.template_create(tid, t.nodes, t.tris, stretch=t.stretch, ks=t.ks, kb=t.kb, kal=t.kal,
                              kag=t.kag, kv=t.kv, linear=t.linear, model=getattr(t, "model", "paper"))
        for r in getattr(box, "repulsion", []) or []:
            if r.type_b is None:
                c.set_wall_soft_sphere(r.type_a, r.a, r.n, r.cutoff, r.offset)
            else:
                c.set_soft_sphere(r.type_a, r.type_b, r.a, r.n, r.cutoff, r.offset)
        for oid, o in enumerate(box.objects):
            c.object_add(oid, o.tid, o.origin, o.rot, o.mass, getattr(o, "ptype", 0))
            if any(o.fext):
                c.object_set_force(oid, o.fext)
        return c


class Batch:
    """Many boxes advanced together (``oif_batch``); the contexts stay owned by
    the caller and must outlive the batch."""

    def __init__(self, contexts: Sequence[Context]):
        self.contexts = list(contexts)
        arr = (C.c_void_p * len(contexts))(*[c.h for c in contexts])
        h = C.c_void_p()
        rc = lib().oif_batch_create(arr, len(contexts), C.byref(h))
        if rc != OIF_OK:
            raise OifError(rc, "oif_batch_create failed")
        self.h = h

    def _chk(self, rc):
        if rc != OIF_OK:
            raise OifError(rc, lib().oif_batch_last_error(self.h).decode())

    def step(self, n: int = 1):
        self._chk(lib().oif_batch_step(self.h, int(n)))

    def step_timed(self, n: int) -> Timing:
        t = Timing()
        self._chk(lib().oif_batch_step_timed(self.h, int(n), C.byref(t)))
        return t

    def set_graph(self, steps_per_graph: int):
        self._chk(lib().oif_batch_set_graph(self.h, int(steps_per_graph)))

    def set_launch(self, lb_block: int = -1, mesh_block: int = -1, xcd_remap: int = -1):
        self._chk(lib().oif_batch_set_launch(self.h, int(lb_block), int(mesh_block), int(xcd_remap)))

    def set_lb_loads(self, nontemporal: bool):
        self._chk(lib().oif_batch_set_lb_loads(self.h, int(bool(nontemporal))))

    def set_persistent(self, on: bool, lattice_blocks_per_task: int = 0):
        self._chk(lib().oif_batch_set_persistent(self.h, int(bool(on)), int(lattice_blocks_per_task)))

    def autotune(self, cache_path: Optional[str] = None):
        self._chk(lib().oif_batch_autotune(self.h, None if cache_path is None else cache_path.encode()))

    def close(self):
        if getattr(self, "h", None):
            lib().oif_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
