"""Seeded synthetic inputs: membrane meshes, cell placements and box configurations.

This module only *generates inputs*.  It holds none of the method's arithmetic
(no lattice-Boltzmann update, no coupling, no membrane force, no relaxed-value
computation), so the FP64 oracle and the HIP path can both be fed from it
without sharing any of the computation they are compared on.

Meshes follow the file convention of the paper's template section (one node
per row, triangles as three node ids whose cross product AB x AC points *into*
the object).  All random numbers come from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

# ----------------------------------------------------------------------------
# meshes
# ----------------------------------------------------------------------------


def _orient_inward(nodes: np.ndarray, tris: np.ndarray) -> np.ndarray:
    """Flip every triangle whose normal points away from the mesh centroid.

    Only valid for star-shaped meshes around their centroid (all generated
    meshes here are).  Returns a new (nt, 3) int32 array.
    """
    c = nodes.mean(axis=0)
    a, b, cc = nodes[tris[:, 0]], nodes[tris[:, 1]], nodes[tris[:, 2]]
    n = np.cross(b - a, cc - a)
    centroid = (a + b + cc) / 3.0
    outward = np.einsum("ij,ij->i", n, centroid - c) > 0.0
    out = tris.copy()
    out[outward, 1], out[outward, 2] = tris[outward, 2], tris[outward, 1]
    return out.astype(np.int32)


def icosahedron(edge: float = 1.0) -> Tuple[np.ndarray, np.ndarray]:
    """Regular icosahedron with the given edge length, centred at the origin,
    triangles oriented with inward normals."""
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array(
        [[-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
         [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
         [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1]], dtype=np.float64)
    v *= edge / 2.0  # the construction above has edge length 2
    f = np.array(
        [[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
         [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
         [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
         [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int32)
    return v, _orient_inward(v, f)


def tetrahedron(edge: float = 1.0) -> Tuple[np.ndarray, np.ndarray]:
    """Regular tetrahedron, inward-oriented."""
    v = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64)
    v *= edge / (2.0 * math.sqrt(2.0))
    f = np.array([[0, 1, 2], [0, 1, 3], [0, 2, 3], [1, 2, 3]], dtype=np.int32)
    return v, _orient_inward(v, f)


def octahedron(edge: float = 1.0) -> Tuple[np.ndarray, np.ndarray]:
    """Regular octahedron, inward-oriented."""
    r = edge / math.sqrt(2.0)
    v = np.array([[r, 0, 0], [-r, 0, 0], [0, r, 0], [0, -r, 0], [0, 0, r], [0, 0, -r]])
    f = np.array([[0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4],
                  [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5]], dtype=np.int32)
    return v, _orient_inward(v, f)


def cube(edge: float = 1.0) -> Tuple[np.ndarray, np.ndarray]:
    """Axis-aligned cube as 12 triangles, centred at the origin, inward-oriented."""
    h = edge / 2.0
    v = np.array([[x, y, z] for x in (-h, h) for y in (-h, h) for z in (-h, h)])
    # index = 4*ix + 2*iy + iz
    quads = [(0, 1, 3, 2), (4, 6, 7, 5), (0, 4, 5, 1), (2, 3, 7, 6), (0, 2, 6, 4), (1, 5, 7, 3)]
    f = []
    for a, b, c, d in quads:
        f.append((a, b, c))
        f.append((a, c, d))
    return v, _orient_inward(v, np.array(f, dtype=np.int32))


def icosphere(level: int, radius: float = 1.0) -> Tuple[np.ndarray, np.ndarray]:
    """Geodesic sphere: icosahedron subdivided ``level`` times (each triangle into
    four), nodes projected to the sphere.  Node counts 12, 42, 162, 642, 2562 for
    levels 0..4; triangle count 20 * 4**level.  Inward-oriented."""
    v, f = icosahedron(2.0)
    verts = [tuple(x / np.linalg.norm(x)) for x in v]
    faces = [tuple(t) for t in f]
    for _ in range(level):
        cache = {}

        def mid(i, j):
            key = (min(i, j), max(i, j))
            if key not in cache:
                m = np.add(verts[i], verts[j]) / 2.0
                m = m / np.linalg.norm(m)
                cache[key] = len(verts)
                verts.append(tuple(m))
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    nodes = np.array(verts, dtype=np.float64) * radius
    return nodes, _orient_inward(nodes, np.array(faces, dtype=np.int32))


def fibonacci_sphere(n: int, radius: float = 1.0) -> Tuple[np.ndarray, np.ndarray]:
    """``n`` quasi-uniform points on a sphere (golden-angle spiral), triangulated
    by their convex hull (2n - 4 triangles), inward-oriented."""
    from scipy.spatial import ConvexHull

    i = np.arange(n, dtype=np.float64) + 0.5
    z = 1.0 - 2.0 * i / n
    r = np.sqrt(1.0 - z * z)
    phi = math.pi * (3.0 - math.sqrt(5.0)) * i
    pts = np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)
    hull = ConvexHull(pts)
    nodes = pts * radius
    return nodes, _orient_inward(nodes, hull.simplices.astype(np.int32))


# Evans & Fung (1972) red-cell profile coefficients, C0, C1, C2 divided by R0
# (C0 = 0.81, C1 = 7.83, C2 = -4.39 um at R0 = 3.91 um).
EVANS_FUNG = (0.81 / 3.91, 7.83 / 3.91, -4.39 / 3.91)


def biconcave_from_sphere(nodes_unit: np.ndarray, tris: np.ndarray, radius: float
                          ) -> Tuple[np.ndarray, np.ndarray]:
    """Map a unit-sphere mesh onto the Evans-Fung biconcave disc of the given
    radius: X = R x, Y = R y, Z = (R/2) z (c0 + c1 rho^2 + c2 rho^4), rho^2 = x^2 + y^2.

    The mapping preserves the sign of z, so orientation is kept; it is re-checked
    against the centroid anyway.
    """
    c0, c1, c2 = EVANS_FUNG
    u = nodes_unit / np.linalg.norm(nodes_unit, axis=1, keepdims=True)
    rho2 = u[:, 0] ** 2 + u[:, 1] ** 2
    out = np.empty_like(u)
    out[:, 0] = radius * u[:, 0]
    out[:, 1] = radius * u[:, 1]
    out[:, 2] = 0.5 * radius * u[:, 2] * (c0 + c1 * rho2 + c2 * rho2 * rho2)
    return out, tris.copy()


def rbc_393(radius: float = 4.0) -> Tuple[np.ndarray, np.ndarray]:
    """393-node biconcave red-cell mesh (782 triangles): Fibonacci sphere mapped
    by the Evans-Fung profile."""
    n, t = fibonacci_sphere(393, 1.0)
    return biconcave_from_sphere(n, t, radius)


def rbc_642(radius: float) -> Tuple[np.ndarray, np.ndarray]:
    """642-node biconcave red-cell mesh (1280 triangles): level-3 icosphere
    mapped by the Evans-Fung profile."""
    n, t = icosphere(3, 1.0)
    return biconcave_from_sphere(n, t, radius)


def write_mesh_files(nodes: np.ndarray, tris: np.ndarray, nfile: str, tfile: str) -> None:
    """Write the two text files of the paper's template format."""
    np.savetxt(nfile, nodes, fmt="%.17g")
    np.savetxt(tfile, tris, fmt="%d")


def read_mesh_files(nfile: str, tfile: str) -> Tuple[np.ndarray, np.ndarray]:
    nodes = np.loadtxt(nfile, dtype=np.float64, ndmin=2)
    tris = np.loadtxt(tfile, dtype=np.int64, ndmin=2).astype(np.int32)
    return nodes, tris


# ----------------------------------------------------------------------------
# random rotations and placement
# ----------------------------------------------------------------------------


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation matrix from a normalised Gaussian quaternion."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def random_centres(rng: np.random.Generator, n: int, lo: Sequence[float], hi: Sequence[float],
                   min_dist: float, box: Optional[Sequence[float]] = None,
                   max_tries: int = 200000) -> np.ndarray:
    """Random sequential addition: ``n`` centres uniform in [lo, hi) with pairwise
    distance >= ``min_dist`` (minimum-image distance when ``box`` is given)."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    boxv = None if box is None else np.asarray(box, dtype=np.float64)
    out = np.empty((0, 3))
    tries = 0
    while len(out) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError(f"could only place {len(out)} of {n} centres")
        c = lo + (hi - lo) * rng.random(3)
        if len(out):
            d = out - c
            if boxv is not None:
                d -= boxv * np.round(d / boxv)
            if np.min(np.einsum("ij,ij->i", d, d)) < min_dist * min_dist:
                continue
        out = np.vstack([out, c])
    return out


# ----------------------------------------------------------------------------
# workload descriptions
# ----------------------------------------------------------------------------

MODULI_DEFAULT = dict(ks=0.1, kb=0.03, kal=0.1, kag=0.4, kv=1.0)

# Friction used by the workloads.  The explicit drag coupling with unit mass
# and unit time step diverges for xi >= 1 on the 642-node sphere (its fluid
# back-reaction makes the relative velocity grow by |1 - xi (1/m + 1/m_f)|
# per step), so the stated xi = 1.5 cannot be run; 0.5 is stable for the
# 162/393/642-node meshes, 0.25 is needed where 2562-node meshes occur.
WORKING_FRICTION = 0.5
WORKING_FRICTION_FINE = 0.25
# The level-4 (2562-node) icosphere is too stiff at the default moduli with
# m = 1, dt = 1; its template takes the moduli scaled by 642/2562 ~ 1/4
# (moduli are calibrated per mesh density).
FINE_MODULI_SCALE = 0.25


@dataclasses.dataclass
class Template:
    nodes: np.ndarray  # (nv, 3) float64
    tris: np.ndarray   # (nt, 3) int32, inward-oriented
    ks: float = 0.0
    kb: float = 0.0
    kal: float = 0.0
    kag: float = 0.0
    kv: float = 0.0
    linear: bool = False
    stretch: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    model: str = "paper"   # force model: "paper" or "conservative"


@dataclasses.dataclass
class ObjectSpec:
    tid: int
    origin: np.ndarray                 # (3,)
    rot: Optional[np.ndarray] = None   # (3, 3) or None for identity
    mass: float = 1.0
    fext: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    ptype: int = 0                     # part type (selects repulsion partners)


@dataclasses.dataclass
class SoftSphere:
    """Soft-sphere repulsion a (d - offset)^-n for offset < d < offset + cutoff
    between mesh nodes of part types type_a and type_b, or (type_b = None)
    between nodes of type_a and every obstacle shape / z wall."""
    type_a: int
    type_b: Optional[int]
    a: float
    n: float
    cutoff: float
    offset: float = 0.0


@dataclasses.dataclass
class Boundary:
    """Obstacle (the lbboundary shapes of the paper's scripts): kind "rhomboid"
    (corner, edge vectors a, b, c) or "wall" (half-space normal . x < dist),
    moving with `velocity` (0 = at rest; a moving boundary drives the fluid,
    e.g. as a velocity inlet)."""
    kind: str
    corner: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    a: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    b: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    c: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    normal: Tuple[float, float, float] = (0.0, 0.0, 1.0)
    dist: float = 0.0
    velocity: Tuple[float, float, float] = (0.0, 0.0, 0.0)


@dataclasses.dataclass
class Box:
    nx: int
    ny: int
    nz: int
    tau: float = 1.0
    rho0: float = 1.0
    g: Tuple[float, float, float] = (1e-5, 0.0, 0.0)
    friction: float = WORKING_FRICTION
    walls_z: bool = False
    templates: List[Template] = dataclasses.field(default_factory=list)
    objects: List[ObjectSpec] = dataclasses.field(default_factory=list)
    steps: int = 1
    name: str = ""
    boundaries: List[Boundary] = dataclasses.field(default_factory=list)
    # collision: None = BGK with tau; else the multiple-relaxation-time rates
    # (gamma_shear, gamma_bulk, gamma_odd, gamma_even)
    mrt: Optional[Tuple[float, float, float, float]] = None
    integrator: str = "euler"  # mesh integrator: "euler" or "verlet"
    repulsion: List["SoftSphere"] = dataclasses.field(default_factory=list)

    @property
    def n_nodes(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_mesh_nodes(self) -> int:
        return sum(len(self.templates[o.tid].nodes) for o in self.objects)


def config_sphere_fp64(steps: int = 100) -> Box:
    """Plain FP64 method case: 20^3 periodic box, one level-3 icosphere
    (642 nodes / 1280 triangles) of radius 4 centred at (10, 10, 10), body
    force 1e-5 in x, friction WORKING_FRICTION (the stated 1.5 diverges)."""
    n, t = icosphere(3, 4.0)
    tm = Template(n, t, **MODULI_DEFAULT)
    return Box(20, 20, 20, templates=[tm], objects=[ObjectSpec(0, np.array([10.0, 10.0, 10.0]))],
               steps=steps, name="sphere642_20cube_fp64")


def config_channel_rbc(steps: int = 1000, seed: int = 2, n_cells: int = 10) -> Box:
    """FP32 channel case: 64x32x32, bounce-back walls at z = 0 and z = 32,
    body force 1e-5 in x, ten 393-node biconcave cells (diameter 8) at random
    non-overlapping centres (distance >= 9, centre z in [5, 27]) with uniform
    random rotations."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    n, t = rbc_393(4.0)
    tm = Template(n, t, **MODULI_DEFAULT)
    cs = random_centres(rng, n_cells, (0.0, 0.0, 5.0), (64.0, 32.0, 27.0), 9.0, box=None)
    objs = [ObjectSpec(0, c, random_rotation(rng)) for c in cs]
    return Box(64, 32, 32, walls_z=True, templates=[tm], objects=objs, steps=steps,
               name="rbc393x10_64x32x32_walls")


def obstacle_channel_boundaries(nx: int = 96, ny: int = 48, inlet: float = 0.01) -> List[Boundary]:
    """S-shaped channel from obstacles: side walls at y < 2 and y > ny - 2, a
    baffle from the low side (x in [0.31, 0.375] nx, y < 2/3 ny) and one from the
    high side (x in [0.625, 0.69] nx, y > ny/3), and a velocity inlet: a slab
    at x < 2 moving along +x with `inlet` (periodic in x, so the slab's far
    face is the outlet)."""
    fx = lambda f: round(f * nx)  # noqa: E731
    return [
        Boundary("wall", normal=(0, 1, 0), dist=2.0),
        Boundary("wall", normal=(0, -1, 0), dist=-(ny - 2.0)),
        Boundary("rhomboid", corner=(fx(0.3125), 0, 0), a=(fx(0.0625), 0, 0), b=(0, round(2 * ny / 3), 0),
                 c=(0, 0, 1e4)),
        Boundary("rhomboid", corner=(fx(0.625), round(ny / 3), 0), a=(fx(0.0625), 0, 0),
                 b=(0, ny - round(ny / 3), 0), c=(0, 0, 1e4)),
        Boundary("rhomboid", corner=(0, 0, 0), a=(2, 0, 0), b=(0, ny, 0), c=(0, 0, 1e4),
                 velocity=(inlet, 0.0, 0.0)),
    ]


def config_obstacle_channel(steps: int = 200, seed: int = 6, n_cells: int = 10, nx: int = 96, ny: int = 48,
                            nz: int = 16) -> Box:
    """Obstacle case (stand-in for the paper's S-channel script): the channel
    of ``obstacle_channel_boundaries`` with bounce-back walls at z = 0 and
    z = nz, no body force (the inlet drives the flow), ten 393-node cells
    (diameter 8) at random rotations, centres at least 5.5 from every solid
    node and 5 from the z walls, pairwise distance >= 9."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    bnd = obstacle_channel_boundaries(nx, ny)
    # solid nodes of the shapes (a plain membership test, independent of both
    # the oracle and the library, used only to keep the cells clear)
    cx, cy = np.meshgrid(np.arange(nx) + 0.5, np.arange(ny) + 0.5, indexing="xy")
    solid2d = (cy < 2.0) | (cy > ny - 2.0) | (cx < 2.0)
    for b in bnd[2:4]:
        x0, y0 = b.corner[0], b.corner[1]
        solid2d |= (cx >= x0) & (cx <= x0 + b.a[0]) & (cy >= y0) & (cy <= y0 + b.b[1])
    sy, sx = np.nonzero(solid2d)
    pts = np.stack([sx + 0.5, sy + 0.5], axis=1)
    n, t = rbc_393(4.0)
    tm = Template(n, t, **MODULI_DEFAULT)
    cs = np.empty((0, 3))
    tries = 0
    while len(cs) < n_cells:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not place the cells")
        c = np.array([nx, ny, nz - 10.0]) * rng.random(3) + [0.0, 0.0, 5.0]
        dxy = pts - c[:2]
        dxy[:, 0] -= nx * np.round(dxy[:, 0] / nx)
        if np.min(np.einsum("ij,ij->i", dxy, dxy)) < 5.5 ** 2:
            continue
        if len(cs):
            d = cs - c
            d[:, 0] -= nx * np.round(d[:, 0] / nx)
            if np.min(np.einsum("ij,ij->i", d, d)) < 81.0:
                continue
        cs = np.vstack([cs, c])
    objs = [ObjectSpec(0, c, random_rotation(rng)) for c in cs]
    return Box(nx, ny, nz, g=(0.0, 0.0, 0.0), walls_z=True, templates=[tm], objects=objs, steps=steps,
               name=f"rbc393x{n_cells}_schannel_{nx}x{ny}x{nz}", boundaries=bnd)


def config_precision(steps: int = 500, seed: int = 3, nx: int = 256, ny: int = 128, nz: int = 128,
                     n_cells: int = 500) -> Box:
    """Precision-form case: 256x128x128 periodic, 500 level-3 icospheres of
    radius 4 at random centres (periodic distance >= 9)."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    n, t = icosphere(3, 4.0)
    tm = Template(n, t, **MODULI_DEFAULT)
    cs = random_centres(rng, n_cells, (0.0, 0.0, 0.0), (nx, ny, nz), 9.0, box=(nx, ny, nz))
    objs = [ObjectSpec(0, c) for c in cs]
    return Box(nx, ny, nz, templates=[tm], objects=objs, steps=steps,
               name=f"sphere642x{n_cells}_{nx}x{ny}x{nz}")


def config_precision_subbox(steps: int = 500, seed: int = 3) -> Box:
    """64^3 sub-run of the precision case at the same number density (31 cells)."""
    return config_precision(steps=steps, seed=seed, nx=64, ny=64, nz=64, n_cells=31)


def config_batch(seed: int = 4, steps: int = 200, n_boxes: int = 32) -> List[Box]:
    """Batching case: 32 periodic boxes of uneven sizes (box 0 = 32^3, last =
    64x48x48, others nx ~ U{32..64}, ny, nz ~ U{32..48}), each holding U{1..20}
    icospheres of radius 4 whose level is drawn from {2, 3, 4}."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    lv_mesh = {lv: icosphere(lv, 4.0) for lv in (2, 3, 4)}
    boxes = []
    for b in range(n_boxes):
        if b == 0:
            dims = (32, 32, 32)
        elif b == n_boxes - 1:
            dims = (64, 48, 48)
        else:
            dims = (int(rng.integers(32, 65)), int(rng.integers(32, 49)), int(rng.integers(32, 49)))
        ncell = int(rng.integers(1, 21))
        levels = rng.integers(2, 5, size=ncell)
        fine = {k: v * FINE_MODULI_SCALE for k, v in MODULI_DEFAULT.items()}
        tmpls = [Template(*lv_mesh[lv], **(fine if lv == 4 else MODULI_DEFAULT)) for lv in (2, 3, 4)]
        cs = random_centres(rng, ncell, (0, 0, 0), dims, 9.0, box=dims)
        objs = [ObjectSpec(int(lv) - 2, c) for lv, c in zip(levels, cs)]
        boxes.append(Box(*dims, templates=tmpls, objects=objs, steps=steps, name=f"batch{b}",
                         friction=WORKING_FRICTION_FINE))
    return boxes


def config_scale(steps: int = 200, seed: int = 5, nx: int = 512, ny: int = 256, nz: int = 256,
                 n_cells: int = 5000, diameter: float = 15.0) -> Box:
    """Scale case: 512x256x256 periodic, 5000 biconcave 642-node cells of
    diameter 15 placed on a jittered 26x14x14 grid (5000 of 5096 sites, jitter
    <= 1 per axis) with random rotations."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    n, t = rbc_642(diameter / 2.0)
    tm = Template(n, t, **MODULI_DEFAULT)
    gx, gy, gz = 26, 14, 14
    sites = np.array([[(i + 0.5) * nx / gx, (j + 0.5) * ny / gy, (k + 0.5) * nz / gz]
                      for i in range(gx) for j in range(gy) for k in range(gz)])
    pick = rng.choice(len(sites), size=n_cells, replace=False)
    cs = sites[np.sort(pick)] + rng.uniform(-1.0, 1.0, size=(n_cells, 3))
    objs = [ObjectSpec(0, c, random_rotation(rng)) for c in cs]
    return Box(nx, ny, nz, templates=[tm], objects=objs, steps=steps,
               name=f"rbc642x{n_cells}_{nx}x{ny}x{nz}")


def config_scale_share(ranks: int = 8, rank: int = 0, steps: int = 200, seed: int = 5) -> Box:
    """One GPU's share of the scale case split into `ranks` slabs along x: the
    (512 / ranks) x 256 x 256 slab of rank `rank` with the cells whose centres
    lie in it, shifted to the slab's origin.  The slab is periodic in x as
    well, standing in for the populations and forces its faces would exchange
    with the neighbouring ranks (the per-rank work is the same)."""
    full = config_scale(steps=steps, seed=seed)
    if full.nx % ranks or not 0 <= rank < ranks:
        raise ValueError("ranks must divide nx and 0 <= rank < ranks")
    w = full.nx // ranks
    x0 = rank * w
    objs = [dataclasses.replace(o, origin=o.origin - np.array([x0, 0.0, 0.0]))
            for o in full.objects if x0 <= o.origin[0] < x0 + w]
    return Box(w, full.ny, full.nz, templates=full.templates, objects=objs, steps=steps,
               name=f"rbc642x{len(objs)}_{w}x{full.ny}x{full.nz}_slab{rank + 1}of{ranks}")


def random_populations(rng: np.random.Generator, box: Box, amp: float = 1e-3) -> np.ndarray:
    """Full D3Q19 populations (19, nz, ny, nx) close to rest: weights times rho0
    plus uniform noise of the given amplitude.  Used to start parity runs from a
    non-trivial state; the weights are the standard D3Q19 ones (1/3, 1/18, 1/36)."""
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    base = (w * box.rho0)[:, None, None, None]
    noise = amp * (rng.random((19, box.nz, box.ny, box.nx)) - 0.5) * base * 18.0
    return base + noise
