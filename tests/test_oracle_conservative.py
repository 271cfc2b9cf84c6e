"""Pins of the oracle's conservative force model (gradient bending, balanced
local/global area), a per-template alternative to the paper's printed rules
that the paper's force-based framework admits ("Elastic interactions": the
model is a set of forces per mesh element).  Pinned against finite
differences of an independently computed energy, the paper's own rules where
they coincide (symmetric hinges, equilateral triangles), hand values and the
invariants the variant exists for (no net force, no torque)."""
import math

import numpy as np
import pytest

from paper_1312_3426_amd import synth


def _inner_angle_by_projection(A, B, C, D, n1):
    """Dihedral angle from the wing vectors projected perpendicular to the edge
    (independent of the oracle's normals-based atan2)."""
    e = (C - B) / np.linalg.norm(C - B)
    a = (A - B) - ((A - B) @ e) * e
    d = (D - B) - ((D - B) @ e) * e
    ang = math.atan2(np.linalg.norm(np.cross(a, d)), a @ d)
    return ang if n1 @ d > 0 else 2 * math.pi - ang


def _dist_to_line(P, B, C):
    e = (C - B) / np.linalg.norm(C - B)
    r = (P - B) - ((P - B) @ e) * e
    return np.linalg.norm(r)


def _random_hinge(rng):
    """Asymmetric hinge with wings well away from the edge line and the angle
    away from 0 and 2 pi."""
    while True:
        B = np.array([-0.5, 0.0, 0.0]) + 0.1 * rng.standard_normal(3)
        C = np.array([0.6, 0.0, 0.0]) + 0.1 * rng.standard_normal(3)
        A = np.array([rng.uniform(-0.8, 0.9), rng.uniform(0.4, 1.2), rng.uniform(-0.5, 0.5)])
        D = np.array([rng.uniform(-0.8, 0.9), rng.uniform(-1.2, -0.4), rng.uniform(-0.5, 0.5)])
        x = np.array([A, B, C, D])
        n1 = np.cross(B - A, C - A)
        th = _inner_angle_by_projection(A, B, C, D, n1 / np.linalg.norm(n1))
        if 0.6 < th < 2 * math.pi - 0.6:
            return x


def test_wing_height_closed_forms(orc):
    # regular tetrahedron of edge a: every wing height is the face height a sqrt(3)/2
    for a in (1.0, 2.5):
        x = a * np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float) / math.sqrt(8)
        t = np.array([[0, 1, 2], [0, 2, 3], [0, 3, 1], [1, 3, 2]])
        _, V = orc.geometry(x, t)[1:]
        if V < 0:
            t = t[:, [0, 2, 1]]
        R = orc.Relaxed(x, t)
        assert np.allclose(R.hbar, a * math.sqrt(3) / 2, rtol=1e-14)
    # asymmetric hinges: mean of the two distances to the edge line
    rng = np.random.default_rng(11)
    for _ in range(5):
        x = _random_hinge(rng)
        hb = orc.wing_height(x, [[0, 1, 2, 3]])[0]
        ref = 0.5 * (_dist_to_line(x[0], x[1], x[2]) + _dist_to_line(x[3], x[1], x[2]))
        assert hb == pytest.approx(ref, rel=1e-14)


@pytest.mark.parametrize("seed", range(6))
def test_bend_gradient_is_energy_gradient(orc, seed):
    """F = -grad [kb hbar (theta - theta0)^2 / (2 theta0)] on asymmetric hinges,
    all 12 components, hbar a fixed constant of the hinge."""
    rng = np.random.default_rng(100 + seed)
    x = _random_hinge(rng)
    kb, hbar = 0.3, 0.7 + 0.5 * rng.random()
    n1_here = np.cross(x[1] - x[0], x[2] - x[0])
    th_here = _inner_angle_by_projection(*x, n1_here / np.linalg.norm(n1_here))
    theta0 = th_here + rng.choice([-1, 1]) * (0.1 + 0.4 * rng.random())
    F = orc.force_bend_gradient_hinges(x, [[0, 1, 2, 3]], [theta0], [hbar], kb)

    def energy(y):
        n1 = np.cross(y[1] - y[0], y[2] - y[0])
        th = _inner_angle_by_projection(y[0], y[1], y[2], y[3], n1 / np.linalg.norm(n1))
        return kb * hbar * (th - theta0) ** 2 / (2 * theta0)

    assert orc.dihedral(*x) == pytest.approx(th_here, abs=1e-13)
    eps = 1e-6
    G = np.zeros_like(x)
    for i in range(4):
        for c in range(3):
            yp, ym = x.copy(), x.copy()
            yp[i, c] += eps
            ym[i, c] -= eps
            G[i, c] = -(energy(yp) - energy(ym)) / (2 * eps)
    assert np.abs(F - G).max() <= 1e-7 * np.abs(F).max()


def test_bend_gradient_no_net_force_or_torque(orc):
    rng = np.random.default_rng(7)
    for _ in range(8):
        x = _random_hinge(rng) + rng.standard_normal(3)
        F = orc.force_bend_gradient_hinges(x, [[0, 1, 2, 3]], [2.0], [0.8], 0.3)
        scale = np.abs(F).max()
        assert np.abs(F.sum(axis=0)).max() < 1e-14 * scale
        assert np.abs(np.cross(x, F).sum(axis=0)).max() < 1e-14 * scale * np.abs(x).max()


@pytest.mark.parametrize("fold,theta0", [(0.3, 2.2), (-0.2, 2.9), (0.6, 1.4)])
def test_bend_gradient_is_paper_rule_on_symmetric_hinge(orc, fold, theta0):
    """Wings at equal height h = hbar with their feet at the edge midpoint: the
    gradient form is the paper's rule (f n on the wings, minus half the sum on
    the edge vertices)."""
    h, half = 0.8, 0.6
    B, C = np.array([-half, 0.0, 0.0]), np.array([half, 0.0, 0.0])
    A = np.array([0.0, h * math.cos(fold), -h * math.sin(fold)])
    D = np.array([0.0, -h * math.cos(fold), -h * math.sin(fold)])
    x = np.array([A, B, C, D])
    Fp = orc.force_bend_hinges(x, [[0, 1, 2, 3]], [theta0], 0.3)
    Fg = orc.force_bend_gradient_hinges(x, [[0, 1, 2, 3]], [theta0], [h], 0.3)
    assert np.abs(Fg - Fp).max() <= 1e-14 * np.abs(Fp).max()


def test_balanced_area_hand_values(orc):
    """Triangle (0,0,0), (3,0,0), (0,3,0): centroid (1,1,0), t = (-1,-1,0),
    (2,-1,0), (-1,2,0), t_rms^2 = (2 + 5 + 5)/3 = 4."""
    x = np.array([[0.0, 0, 0], [3, 0, 0], [0, 3, 0]])
    t = [[0, 1, 2]]
    S = 4.5
    S0, kal = 4.0, 0.2
    F = orc.force_triangles("local_area_balanced", x, t, kal, S0=[S0])
    coef = -kal * (S - S0) / S
    assert np.allclose(F, coef * np.array([[-1, -1, 0], [2, -1, 0], [-1, 2, 0]]) / 2.0, rtol=1e-15, atol=0)
    Fg = orc.force_triangles("global_area_balanced", x, t, 0.4, Sg0=5.0)
    cg = -0.4 * (S - 5.0) / S
    assert np.allclose(Fg, cg * np.array([[-1, -1, 0], [2, -1, 0], [-1, 2, 0]]) / 2.0, rtol=1e-15, atol=0)


def test_balanced_area_no_net_force_or_torque_per_triangle(orc):
    rng = np.random.default_rng(3)
    for _ in range(10):
        x = rng.standard_normal((3, 3)) * [1.0, 0.5, 2.0] + rng.standard_normal(3)
        for which, kw in (("local_area_balanced", dict(S0=[0.3])), ("global_area_balanced", dict(Sg0=0.3))):
            F = orc.force_triangles(which, x, [[0, 1, 2]], 0.5, **kw)
            scale = np.abs(F).max()
            assert np.abs(F.sum(axis=0)).max() < 1e-15 * max(scale, 1)
            assert np.abs(np.cross(x, F).sum(axis=0)).max() < 1e-14 * scale * np.abs(x).max()
        # while the paper's unit directions do not balance on this triangle
        Fp = orc.force_triangles("local_area", x, [[0, 1, 2]], 0.5, S0=[0.3])
        assert np.abs(Fp.sum(axis=0)).max() > 1e-6 * np.abs(Fp).max()


def test_balanced_area_is_paper_rule_on_equilateral_mesh(orc):
    """Every face of a (rotated, scaled) icosahedron is equilateral, where t_v /
    t_rms is the unit centroid-to-vertex vector."""
    x, t = synth.icosahedron()
    rng = np.random.default_rng(5)
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    R = np.array([[a*a+b*b-c*c-d*d, 2*(b*c-a*d), 2*(b*d+a*c)],
                  [2*(b*c+a*d), a*a-b*b+c*c-d*d, 2*(c*d-a*b)],
                  [2*(b*d-a*c), 2*(c*d+a*b), a*a-b*b-c*c+d*d]])
    x = 2.3 * x @ R.T + 1.7
    S, _, _ = orc.geometry(x, t)
    S0 = 0.9 * S
    Fp = orc.force_triangles("local_area", x, t, 0.2, S0=S0)
    Fb = orc.force_triangles("local_area_balanced", x, t, 0.2, S0=S0)
    assert np.abs(Fb - Fp).max() <= 1e-14 * np.abs(Fp).max()
    Fp = orc.force_triangles("global_area", x, t, 0.4, Sg0=0.8 * S.sum())
    Fb = orc.force_triangles("global_area_balanced", x, t, 0.4, Sg0=0.8 * S.sum())
    assert np.abs(Fb - Fp).max() <= 1e-14 * np.abs(Fp).max()


@pytest.mark.parametrize("mesh", ["ico2", "rbc393"])
def test_conservative_model_no_net_force_or_torque(orc, mesh):
    """The point of the variant: on an arbitrary deformed closed mesh all five
    forces together exert no net force and no torque (the paper's printed
    rules leave residuals, stated in the mesh pins)."""
    x, t = synth.icosphere(2, 3.0) if mesh == "ico2" else synth.rbc_393(4.0)
    R = orc.Relaxed(x, t)
    rng = np.random.default_rng(21)
    xd = x + 0.05 * rng.standard_normal(x.shape) + 10.0
    F = R.forces(xd, ks=0.1, kb=0.03, kal=0.1, kag=0.4, kv=1.0, model="conservative")
    scale = np.abs(F).max()
    assert np.abs(F.sum(axis=0)).max() < 1e-13 * scale
    assert np.abs(np.cross(xd, F).sum(axis=0)).max() < 1e-12 * scale * np.abs(xd).max()
    Fp = R.forces(xd, ks=0.1, kb=0.03, kal=0.1, kag=0.4, kv=1.0, model="paper")
    assert np.abs(Fp.sum(axis=0)).max() > 1e-4 * np.abs(Fp).max()


def test_conservative_model_zero_at_rest(orc):
    x, t = synth.rbc_393(4.0)
    R = orc.Relaxed(x, t)
    rot = orc.euler_to_rot(0.4, -0.2, 1.1)
    for y in (x, x @ rot.T + [3.0, -2.0, 5.0]):
        F = R.forces(y, ks=0.1, kb=0.03, kal=0.1, kag=0.4, kv=1.0, model="conservative")
        assert np.abs(F).max() < 1e-13


def test_conservative_model_is_sum_of_its_families(orc):
    x, t = synth.icosphere(2, 3.0)
    R = orc.Relaxed(x, t)
    xd = x + 0.03 * np.random.default_rng(2).standard_normal(x.shape)
    F = R.forces(xd, ks=0.1, kb=0.03, kal=0.1, kag=0.4, kv=1.0, model="conservative")
    parts = (R.force_family("stretch", xd, 0.1) + R.force_family("bend_gradient", xd, 0.03)
             + R.force_family("local_area_balanced", xd, 0.1)
             + R.force_family("global_area_balanced", xd, 0.4) + R.force_family("volume", xd, 1.0))
    assert np.abs(F - parts).max() <= 1e-15 * np.abs(F).max() * 10
