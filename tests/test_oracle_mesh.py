"""Pins of the oracle's mesh geometry and membrane forces against closed forms,
hand values, finite differences and invariants (no GPU).

Each test states which passage of the paper it pins ("Elastic interactions"
subsections, the template-creation rules) and which plausible mistake it would
catch.
"""
import math

import numpy as np
import pytest

from paper_1312_3426_amd import synth

K5 = dict(ks=0.1, kb=0.03, kal=0.1, kag=0.4, kv=1.0)


def rand_rot(seed):
    return synth.random_rotation(np.random.default_rng(seed))


# --------------------------------------------------------------------------
# kappa(lambda) ("Stretching force")
# --------------------------------------------------------------------------

def test_kappa_hand_values(orc):
    assert orc.kappa(1.0) == pytest.approx(1.0, abs=1e-15)
    # (sqrt 2 + 2^-2.5) / (2 + 2^-3), worked by hand
    hand = (1.4142135623730951 + 0.17677669529663687) / 2.125
    assert orc.kappa(2.0) == pytest.approx(hand, rel=1e-15)
    assert orc.kappa(0.5) == pytest.approx(hand, rel=1e-15)


@pytest.mark.parametrize("lam", [0.3, 0.77, 1.2, 1.9, 3.5])
def test_kappa_inversion_symmetry(orc, lam):
    # kappa(lambda) = kappa(1/lambda) holds for the stated exponents only
    assert orc.kappa(lam) == pytest.approx(orc.kappa(1.0 / lam), rel=1e-14)


# --------------------------------------------------------------------------
# topology and orientation (template section)
# --------------------------------------------------------------------------

def test_topology_counts_and_hinge_convention(orc):
    for lv, nv in [(0, 12), (1, 42), (2, 162), (3, 642)]:
        x, t = synth.icosphere(lv, 1.0)
        assert len(x) == nv and len(t) == 2 * nv - 4
        e, h, ht = orc.topology(len(x), t)
        assert len(e) == 3 * nv - 6
        # hinge (A, B, C, D): T1 holds A, B, C with B -> C in cyclic order
        for (A, B, C, D), (t1, t2) in zip(h, ht):
            tri1 = list(t[t1])
            k = tri1.index(B)
            assert tri1[(k + 1) % 3] == C and tri1[(k + 2) % 3] == A
            tri2 = list(t[t2])
            k = tri2.index(C)
            assert tri2[(k + 1) % 3] == B and tri2[(k + 2) % 3] == D


def test_topology_rejects_bad_meshes(orc):
    x, t = synth.icosphere(1, 1.0)
    bad = t.copy()
    bad[3] = bad[3][[0, 2, 1]]  # one triangle flipped: inconsistent orientation
    with pytest.raises(ValueError):
        orc.topology(len(x), bad)
    with pytest.raises(ValueError):
        orc.topology(len(x), t[:-1])  # open mesh


def test_orientation_worked_example(orc):
    """The template rule: for ids 3, 5, 8 with AB x AC pointing outward the
    file must hold "3 8 5" (fixture tests/golden/orientation_358.txt)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "orientation_358.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    wrong, right = [int(v) for v in rows[0]], [int(v) for v in rows[1]]
    assert wrong == [3, 5, 8] and right == [3, 8, 5]
    # a tetrahedron on nodes 0, 3, 5, 8 whose face (3, 5, 8) has AB x AC outward
    x = np.zeros((9, 3))
    x[3], x[5], x[8] = [0, 0, 0], [1, 0, 0], [0, 1, 0]
    x[0] = [0.2, 0.2, -1.0]  # apex below: AB x AC = +z points away from it
    n = np.cross(x[5] - x[3], x[8] - x[3])
    assert n @ (x[0] - x[3]) < 0  # outward
    others = [[0, 3, 8], [0, 8, 5], [0, 5, 3]]  # fixed to be consistent with (3, 8, 5)
    t_right = np.array([right] + others)
    _, _, V = orc.geometry(x, t_right)
    assert V > 0  # inward orientation -> positive enclosed volume
    t_wrong = np.array([wrong] + [o[::-1] for o in others])
    _, _, Vw = orc.geometry(x, t_wrong)
    assert Vw == pytest.approx(-V, rel=1e-15)


# --------------------------------------------------------------------------
# areas and volumes ("Global area conservation", "Volume conservation")
# --------------------------------------------------------------------------

@pytest.mark.parametrize("a", [0.7, 1.0, 2.3])
def test_platonic_area_volume(orc, a):
    s5 = math.sqrt(5.0)
    cases = [
        (synth.icosahedron(a), 5 * math.sqrt(3) * a * a, 5.0 / 12.0 * (3 + s5) * a ** 3),
        (synth.tetrahedron(a), math.sqrt(3) * a * a, a ** 3 / (6 * math.sqrt(2))),
        (synth.octahedron(a), 2 * math.sqrt(3) * a * a, math.sqrt(2) / 3 * a ** 3),
        (synth.cube(a), 6 * a * a, a ** 3),
    ]
    for (x, t), A, V in cases:
        S, Ag, Vg = orc.geometry(x, t)
        assert Ag == pytest.approx(A, rel=1e-14)
        assert Vg == pytest.approx(V, rel=1e-14)
        assert S.sum() == pytest.approx(A, rel=1e-14)


def test_volume_invariance_and_sign(orc):
    x, t = synth.icosphere(2, 3.0)
    _, A, V = orc.geometry(x, t)
    R = rand_rot(7)
    y = x @ R.T + np.array([101.3, -55.2, 7.7])
    _, A2, V2 = orc.geometry(y, t)
    assert A2 == pytest.approx(A, rel=1e-13) and V2 == pytest.approx(V, rel=1e-12)
    _, _, Vf = orc.geometry(x, t[:, [0, 2, 1]])
    assert Vf == pytest.approx(-V, rel=1e-14)


def test_icosphere_volume_converges(orc):
    errs = []
    for lv in (1, 2, 3, 4):
        x, t = synth.icosphere(lv, 1.0)
        _, _, V = orc.geometry(x, t)
        errs.append(abs(V - 4.0 * math.pi / 3.0))
    assert all(e2 < e1 / 3.0 for e1, e2 in zip(errs, errs[1:]))


# --------------------------------------------------------------------------
# dihedral angle ("Bending force": inner angle, > pi for concave)
# --------------------------------------------------------------------------

def test_dihedral_platonic(orc):
    for (x, t), want in [(synth.tetrahedron(1.0), math.acos(1.0 / 3.0)),
                         (synth.octahedron(1.0), math.acos(-1.0 / 3.0)),
                         (synth.icosahedron(1.0), math.acos(-math.sqrt(5.0) / 3.0))]:
        r = orc.Relaxed(x, t)
        assert np.allclose(r.theta0, want, rtol=0, atol=1e-14)


def test_dihedral_cube_and_flat(orc):
    x, t = synth.cube(1.0)
    r = orc.Relaxed(x, t)
    th = np.sort(r.theta0)
    assert np.allclose(th[:12], math.pi / 2, atol=1e-14)   # cube edges
    assert np.allclose(th[12:], math.pi, atol=1e-14)       # face diagonals are flat


@pytest.mark.parametrize("h", [0.05, 0.4, 1.7])
def test_dihedral_tent_convex_and_concave(orc, h):
    B, C = np.array([1.0, 0, 0]), np.array([0.0, 0, 0])
    # ridge tent over the interior (below): inner angle pi - 2 atan(h)
    A, D = np.array([0.5, 1, -h]), np.array([0.5, -1, -h])
    assert orc.dihedral(A, B, C, D) == pytest.approx(math.pi - 2 * math.atan(h), abs=1e-14)
    # valley (wings above the edge): concave, pi + 2 atan(h)
    A2, D2 = np.array([0.5, 1, h]), np.array([0.5, -1, h])
    assert orc.dihedral(A2, B, C, D2) == pytest.approx(math.pi + 2 * math.atan(h), abs=1e-14)


# --------------------------------------------------------------------------
# rest shape: no force (every subsection: no force in the relaxed state)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("mesh", ["ico2", "rbc393", "cube"])
def test_rest_mesh_zero_force(orc, mesh):
    x, t = {"ico2": lambda: synth.icosphere(2, 4.0), "rbc393": lambda: synth.rbc_393(4.0),
            "cube": lambda: synth.cube(2.0)}[mesh]()
    r = orc.Relaxed(x, t)
    for seed in range(3):
        R = rand_rot(seed)
        y = x @ R.T + np.array([12.5, -3.0, 40.25]) * seed
        F = r.forces(y, **K5)
        assert np.abs(F).max() < 1e-13


# --------------------------------------------------------------------------
# stretching: force = -grad of the energy whose derivative is the paper's law
# --------------------------------------------------------------------------

def _stretch_energy(x, edges, L0, ks, linear):
    """E = sum ks L0 int_1^lambda kappa(s)(s - 1) ds (20-point Gauss-Legendre);
    dE/dL = ks kappa(lambda)(L - L0)/L0 by construction."""
    gx, gw = np.polynomial.legendre.leggauss(20)
    E = 0.0
    for (a, b), l0 in zip(edges, L0):
        L = np.linalg.norm(x[b] - x[a])
        lam = L / l0
        if linear:
            E += ks * (L - l0) ** 2 / (2 * l0)
            continue
        s = 1.0 + (lam - 1.0) * (gx + 1.0) / 2.0
        kap = (s ** 0.5 + s ** -2.5) / (s + s ** -3)
        E += ks * l0 * np.sum(gw * kap * (s - 1.0)) * (lam - 1.0) / 2.0
    return E


@pytest.mark.parametrize("linear", [False, True])
def test_stretch_is_energy_gradient(orc, linear):
    x, t = synth.octahedron(1.0)
    r = orc.Relaxed(x, t)
    rng = np.random.default_rng(11)
    y = x + 0.15 * rng.standard_normal(x.shape)
    F = orc.force_stretch_edges(y, r.edges, r.L0, 0.37, linear)
    eps = 1e-6
    G = np.zeros_like(y)
    for i in range(len(y)):
        for c in range(3):
            yp, ym = y.copy(), y.copy()
            yp[i, c] += eps
            ym[i, c] -= eps
            G[i, c] = -(_stretch_energy(yp, r.edges, r.L0, 0.37, linear)
                        - _stretch_energy(ym, r.edges, r.L0, 0.37, linear)) / (2 * eps)
    assert np.abs(F - G).max() <= 1e-7 * np.abs(F).max()
    assert np.abs(F.sum(axis=0)).max() < 1e-15  # pair forces: symmetric


# --------------------------------------------------------------------------
# bending
# --------------------------------------------------------------------------

def _inner_angle_by_projection(A, B, C, D, n1):
    """Dihedral angle from the wing vectors projected perpendicular to the edge
    (independent of the oracle's normals-based atan2); measured through the
    side the inward normal n1 of T1 points to."""
    e = (C - B) / np.linalg.norm(C - B)
    a = (A - B) - ((A - B) @ e) * e
    d = (D - B) - ((D - B) @ e) * e
    ang = math.atan2(np.linalg.norm(np.cross(a, d)), a @ d)
    return ang if n1 @ d > 0 else 2 * math.pi - ang


def _sym_hinge(fold, h=0.8, half=0.6):
    B, C = np.array([-half, 0.0, 0.0]), np.array([half, 0.0, 0.0])
    A = np.array([0.0, h * math.cos(fold), -h * math.sin(fold)])
    D = np.array([0.0, -h * math.cos(fold), -h * math.sin(fold)])
    return np.array([A, B, C, D])


@pytest.mark.parametrize("fold,theta0", [(0.3, 2.2), (0.3, 3.0), (-0.2, 2.9), (0.6, 1.4)])
def test_bend_symmetric_hinge_is_energy_gradient(orc, fold, theta0):
    """On a symmetric hinge (wings at equal height, feet at the edge midpoint)
    the rule F_A = f n1, F_D = f n2, F_B = F_C = -(F_A + F_D)/2 equals
    -grad [kb h (theta - theta0)^2 / (2 theta0)] with the wing height h frozen."""
    x = _sym_hinge(fold)
    hinge = np.array([[0, 1, 2, 3]])
    kb = 0.45
    F = orc.force_bend_hinges(x, hinge, [theta0], kb)

    def n1_of(y):
        n = np.cross(y[1] - y[0], y[2] - y[0])
        return n / np.linalg.norm(n)

    h0 = np.linalg.norm(x[0] - 0.5 * (x[1] + x[2]))

    def energy(y):
        th = _inner_angle_by_projection(y[0], y[1], y[2], y[3], n1_of(y))
        return kb * h0 * (th - theta0) ** 2 / (2 * theta0)

    th_here = _inner_angle_by_projection(*x, n1_of(x))
    assert orc.dihedral(*x) == pytest.approx(th_here, abs=1e-14)
    eps = 1e-6
    G = np.zeros_like(x)
    for i in range(4):
        for c in range(3):
            yp, ym = x.copy(), x.copy()
            yp[i, c] += eps
            ym[i, c] -= eps
            G[i, c] = -(energy(yp) - energy(ym)) / (2 * eps)
    assert np.abs(F - G).max() <= 1e-7 * np.abs(F).max()


def test_bend_general_hinge_invariants(orc):
    rng = np.random.default_rng(5)
    for _ in range(5):
        x = rng.standard_normal((4, 3))
        F = orc.force_bend_hinges(x, [[0, 1, 2, 3]], [2.0], 0.3)
        assert np.abs(F.sum(axis=0)).max() < 1e-15
        n1 = np.cross(x[1] - x[0], x[2] - x[0])
        n2 = np.cross(x[2] - x[3], x[1] - x[3])
        assert np.linalg.norm(np.cross(F[0], n1)) < 1e-14 * np.linalg.norm(n1)
        assert np.linalg.norm(np.cross(F[3], n2)) < 1e-14 * np.linalg.norm(n2)
        assert np.allclose(F[1], F[2], atol=1e-16)


def test_bend_restores_towards_theta0(orc):
    # a convex ridge folded tighter than its rest angle is pushed open
    x = _sym_hinge(0.5)
    th = orc.dihedral(*x)
    F = orc.force_bend_hinges(x, [[0, 1, 2, 3]], [th + 0.3], 1.0)
    x2 = x + 1e-4 * F
    assert orc.dihedral(*x2) > th


# --------------------------------------------------------------------------
# local and global area
# --------------------------------------------------------------------------

_POLY = {
    # name: (mesh ctor, faces per vertex * cos(angle between centroid->vertex
    #        and centre->vertex), same for the face normal (volume force))
    "tetra": (synth.tetrahedron, math.sqrt(8.0), 3 * (1.0 / 3.0)),
    "octa": (synth.octahedron, 8.0 / math.sqrt(6.0), 4 / math.sqrt(3.0)),
    "icosa": (synth.icosahedron, 5 * math.sqrt(2.0 / 3.0 * (1 - 1 / math.sqrt(5.0))),
              5 * ((math.sqrt(3) / 12 * (3 + math.sqrt(5))) / (math.sqrt(10 + 2 * math.sqrt(5)) / 4))),
}


@pytest.mark.parametrize("name", list(_POLY))
@pytest.mark.parametrize("s", [0.8, 1.0, 1.25])
def test_area_forces_on_scaled_platonic(orc, name, s):
    """Uniform scaling by s: every triangle has dS/S = 1 - 1/s^2, so each vertex
    receives -k (1 - 1/s^2) c_poly v_hat (local and global alike)."""
    ctor, cw, _ = _POLY[name]
    x, t = ctor(1.3)
    r = orc.Relaxed(x, t)
    R = rand_rot(3)
    y = (s * x) @ R.T + np.array([5.0, 6.0, -7.0])
    vhat = (x / np.linalg.norm(x, axis=1, keepdims=True)) @ R.T
    for fam, k in (("local_area", 0.21), ("global_area", 0.37)):
        F = r.force_family(fam, y, k)
        want = -k * (1 - 1 / s ** 2) * cw * vhat
        assert np.abs(F - want).max() < 1e-14
        assert np.abs(F.sum(axis=0)).max() < 1e-14
        assert np.abs(np.cross(y - y.mean(axis=0), F).sum(axis=0)).max() < 1e-13


def test_global_area_uses_object_total(orc):
    """Move the top vertex of a regular octahedron: the bottom vertex's four
    faces are unchanged, so its local-area force vanishes while its
    global-area force is -kag (dSg/Sg) (8/sqrt 6) v_hat."""
    a = 1.0
    x, t = synth.octahedron(a)
    r = orc.Relaxed(x, t)
    R0 = a / math.sqrt(2)
    top = int(np.argmax(x[:, 2]))
    bot = int(np.argmin(x[:, 2]))
    Rp = 1.3 * R0
    y = x.copy()
    y[top, 2] = Rp
    top_face = 0.5 * R0 * math.sqrt(2) * math.sqrt(R0 ** 2 / 2 + Rp ** 2)
    Sg0 = 4 * math.sqrt(3) * R0 ** 2
    Sg = 4 * (math.sqrt(3) / 2) * R0 ** 2 + 4 * top_face
    Fl = r.force_family("local_area", y, 0.3)
    assert np.abs(Fl[bot]).max() < 1e-15
    Fg = r.force_family("global_area", y, 0.4)
    want = -0.4 * (Sg - Sg0) / Sg * (8 / math.sqrt(6)) * np.array([0, 0, -1.0])
    assert np.abs(Fg[bot] - want).max() < 1e-15


def test_local_area_sign_uses_current_area(orc):
    # dS/S with the *current* S: doubling the scale gives 3/4, not 3
    x, t = synth.tetrahedron(1.0)
    r = orc.Relaxed(x, t)
    F = r.force_family("local_area", 2 * x, 1.0)
    v = x[0] / np.linalg.norm(x[0])
    assert F[0] @ v == pytest.approx(-0.75 * math.sqrt(8.0), rel=1e-14)


# --------------------------------------------------------------------------
# volume
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["octa", "icosa"])
@pytest.mark.parametrize("s", [0.9, 1.2])
def test_volume_force_scaled_platonic(orc, name, s):
    ctor, _, cn = _POLY[name]
    a = 1.1
    x, t = ctor(a)
    r = orc.Relaxed(x, t)
    y = s * x
    F = r.force_family("volume", y, 0.8)
    S_face = s * s * math.sqrt(3) / 4 * a * a
    vhat = x / np.linalg.norm(x, axis=1, keepdims=True)
    want = -0.8 * (s ** 3 - 1) * S_face * cn / 3.0 * vhat
    assert np.abs(F - want).max() < 1e-14
    if s > 1:
        assert np.all(np.einsum("ij,ij->i", F, vhat) < 0)  # inflated -> pushed inward


def test_volume_force_zero_net_force_and_torque(orc):
    x, t = synth.icosphere(2, 3.0)
    r = orc.Relaxed(x, t)
    rng = np.random.default_rng(3)
    y = 1.1 * x + 0.2 * rng.standard_normal(x.shape) + 4.0
    F = r.force_family("volume", y, 1.0)
    scale = np.abs(F).max()
    assert np.abs(F.sum(axis=0)).max() < 1e-14 * scale * len(x)
    tq = np.cross(y - y.mean(axis=0), F).sum(axis=0)
    assert np.abs(tq).max() < 1e-13 * scale * len(x)


def test_net_force_residuals_stated(orc):
    """Bending and area forces are not torque-free on a general mesh (the
    paper's rules are not gradients); only their net force vanishes for
    bending.  This records the sizes so a change in convention is noticed."""
    x, t = synth.rbc_393(4.0)
    r = orc.Relaxed(x, t)
    rng = np.random.default_rng(9)
    y = x + 0.05 * rng.standard_normal(x.shape)
    Fb = r.force_family("bend", y, 0.03)
    assert np.abs(Fb.sum(axis=0)).max() < 1e-15 * len(x)
    Fs = r.force_family("stretch", y, 0.1)
    assert np.abs(Fs.sum(axis=0)).max() < 1e-15 * len(x)
    assert np.abs(np.cross(y, Fs).sum(axis=0)).max() < 1e-13 * len(x)
