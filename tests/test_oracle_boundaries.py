"""Pins of the oracle's obstacles: rhomboid and wall shapes (the lbboundary
shapes of the paper's scripts, "Implementation details"), bounce-back from
resting and moving obstacle nodes, the velocity they impose, and the coupling
next to them.  Checked against node counts by hand, the built-in halfway
bounce-back walls, the exact linear Couette profile, conservation laws and
the coupling's weights."""
import math

import numpy as np
import pytest

from paper_1312_3426_amd import synth

B = synth.Boundary


def test_rhomboid_axis_aligned_counts(orc):
    solid, wu = orc.boundary_field(8, 8, 8, [B("rhomboid", corner=(2, 2, 2), a=(3, 0, 0), b=(0, 2, 0), c=(0, 0, 1))])
    assert solid.sum() == 3 * 2 * 1
    zz, yy, xx = np.nonzero(solid)
    assert set(xx) == {2, 3, 4} and set(yy) == {2, 3} and set(zz) == {2}
    assert wu.shape == (2, 3) and np.all(wu == 0)


def test_rhomboid_faces_through_node_centres_are_inside(orc):
    """A face through node centres (corner at 1.5) counts those centres inside:
    2 units along each axis cover 3 centres."""
    solid, _ = orc.boundary_field(8, 8, 8, [B("rhomboid", corner=(1.5, 1.5, 1.5), a=(2, 0, 0), b=(0, 2, 0), c=(0, 0, 2))])
    assert solid.sum() == 27


def test_rhomboid_sheared_membership(orc):
    """Sheared rhomboid corner (0,0,0), a = (4,0,0), b = (2,2,0), c = (0,0,1):
    in the plane z = 1/2 a centre (x, y) is inside iff 0 <= y <= 2 and
    y <= x <= y + 4."""
    solid, _ = orc.boundary_field(8, 4, 2, [B("rhomboid", corner=(0, 0, 0), a=(4, 0, 0), b=(2, 2, 0), c=(0, 0, 1))])
    for y in range(4):
        for x in range(8):
            cx, cy = x + 0.5, y + 0.5
            inside = 0 <= cy <= 2 and cy <= cx <= cy + 4
            assert bool(solid[0, y, x]) == inside, (x, y)
    assert solid[1].sum() == 0


def test_wall_half_space(orc):
    solid, _ = orc.boundary_field(4, 4, 6, [B("wall", normal=(0, 0, 2.0), dist=2.0)])
    assert solid.sum() == 4 * 4 * 2  # centres z = 0.5, 1.5 below the plane z = 2
    solid, _ = orc.boundary_field(4, 4, 6, [B("wall", normal=(0, 0, -1.0), dist=-2.5)])
    assert solid.sum() == 4 * 4 * 3  # -z < -2.5: z = 3.5, 4.5, 5.5; the centre on the plane is fluid
    # diagonal plane x + y < 4 (normal not unit)
    solid, _ = orc.boundary_field(4, 4, 1, [B("wall", normal=(1, 1, 0), dist=4 / math.sqrt(2))])
    hand = sum(1 for x in range(4) for y in range(4) if (x + 0.5) + (y + 0.5) < 4)
    assert solid.sum() == hand


def test_later_boundary_overwrites(orc):
    solid, wu = orc.boundary_field(6, 6, 6, [B("wall", normal=(0, 0, 1), dist=3, velocity=(0.1, 0, 0)),
                                             B("rhomboid", corner=(0, 0, 0), a=(6, 0, 0), b=(0, 6, 0), c=(0, 0, 1))])
    assert np.all(solid[0] == 2) and np.all(solid[1:3] == 1) and np.all(solid[3:] == 0)
    assert np.allclose(wu[1], (0.1, 0, 0))


def test_obstacle_layers_reproduce_builtin_walls(orc):
    """Solid layers at z = 0 and z = nz + 1 (at rest) make the fluid between
    them evolve exactly as the built-in halfway bounce-back walls of a box of
    height nz (random populations, body force)."""
    rng = np.random.default_rng(3)
    nx, ny, nz = 5, 4, 6
    n = orc.equilibrium_populations(nx, ny, nz) + 2e-3 * rng.standard_normal((19, nz, ny, nx))
    big = orc.equilibrium_populations(nx, ny, nz + 2)
    big[:, 1:-1] = n
    obst = orc.boundary_field(nx, ny, nz + 2, [B("wall", normal=(0, 0, 1), dist=1.0),
                                               B("wall", normal=(0, 0, -1), dist=-(nz + 1.0))])
    assert obst[0][0].all() and obst[0][-1].all() and not obst[0][1:-1].any()
    g = (2e-5, -1e-5, 3e-5)
    for _ in range(7):
        n = orc.lb_step(n, tau=0.8, g=g, walls_z=True)
        big = orc.lb_step(big, tau=0.8, g=g, obstacles=obst)
    assert np.abs(big[:, 1:-1] - n).max() < 1e-15


@pytest.mark.parametrize("tau", [1.0, 0.7])
def test_couette_profile_exact(orc, tau):
    """Resting solid layer below, a layer moving with U along x above: the
    steady flow is linear between the walls, which sit halfway between the
    solid and the first fluid nodes: u_x(z) = U (z - 1)/H, H = nz - 2."""
    nz, U = 10, 0.01
    H = nz - 2
    obst = orc.boundary_field(1, 1, nz, [B("wall", normal=(0, 0, 1), dist=1.0),
                                         B("wall", normal=(0, 0, -1), dist=-(nz - 1.0), velocity=(U, 0, 0))])
    n = orc.equilibrium_populations(1, 1, nz)
    for _ in range(6000):
        n = orc.lb_step(n, tau=tau, obstacles=obst)
    rho, u = orc.moments(n, obstacles=obst)
    z = np.arange(1, nz - 1) + 0.5
    assert np.abs(u[0, 1:-1, 0, 0] - U * (z - 1.0) / H).max() < 1e-10 * U
    assert np.abs(u[1:, 1:-1]).max() < 1e-14
    assert np.allclose(u[0, -1, 0, 0], U) and u[0, 0, 0, 0] == 0.0   # walls report their velocity
    # tangential motion adds no mass: the wall terms cancel per node; what is
    # left is rounding, about 1e-15 per step over the 6000 steps
    assert abs(rho[1:-1].sum() - H) < 1e-11


def test_static_obstacles_conserve_mass_and_move_nothing(orc):
    rng = np.random.default_rng(9)
    nx, ny, nz = 8, 7, 6
    bnd = [B("rhomboid", corner=(1.2, 1.7, 0.3), a=(3.1, 0.4, 0), b=(0.5, 2.2, 0.3), c=(0.2, 0.1, 3.3)),
           B("wall", normal=(-1, 0.5, -0.3), dist=-5.0)]
    obst = orc.boundary_field(nx, ny, nz, bnd)
    fluid = obst[0] == 0
    assert 0 < (~fluid).sum() < fluid.sum()
    n = orc.equilibrium_populations(nx, ny, nz) + 1e-3 * rng.standard_normal((19, nz, ny, nx))
    m0 = n.sum(axis=0)[fluid].sum()
    solid_pops = n[:, ~fluid].copy()
    for _ in range(10):
        n = orc.lb_step(n, tau=0.9, obstacles=obst)
    assert abs(n.sum(axis=0)[fluid].sum() - m0) < 1e-12 * m0
    assert np.array_equal(n[:, ~fluid], solid_pops)


def test_moving_slab_is_a_velocity_source(orc):
    """A solid slab across the box moving along its normal (+x) pushes fluid
    out of its +x face and draws it in at its -x face: in the periodic box the
    mass is conserved, and the fluid gains +x momentum."""
    nx, ny, nz, U = 12, 3, 3, 0.01
    obst = orc.boundary_field(nx, ny, nz, [B("rhomboid", corner=(0, 0, 0), a=(2, 0, 0), b=(0, ny, 0),
                                                 c=(0, 0, nz), velocity=(U, 0, 0))])
    fluid = obst[0] == 0
    n = orc.equilibrium_populations(nx, ny, nz)
    m0 = n.sum(axis=0)[fluid].sum()
    for _ in range(50):
        n = orc.lb_step(n, tau=1.0, obstacles=obst)
    rho, u = orc.moments(n, obstacles=obst)
    assert abs(rho[fluid].sum() - m0) < 1e-12 * m0
    assert (rho * u[0])[fluid].sum() > 0
    # first fluid layer after the slab: pushed along +x, density raised
    assert u[0][:, :, 2].mean() > 0 and rho[:, :, 2].mean() > 1.0 and rho[:, :, nx - 1].mean() < 1.0


def test_coupling_next_to_obstacle(orc):
    """Interpolation reads the wall velocity at solid corners; spreading leaves
    them out (the obstacle absorbs that share)."""
    nx = ny = nz = 6
    obst = orc.boundary_field(nx, ny, nz, [B("wall", normal=(1, 0, 0), dist=2.0, velocity=(0, 0.05, 0))])
    rng = np.random.default_rng(4)
    n = orc.equilibrium_populations(nx, ny, nz) + 1e-3 * rng.standard_normal((19, nz, ny, nx))
    rho, u = orc.moments(n, obstacles=obst)
    assert np.allclose(u[:, :, :, :2], np.array([0, 0.05, 0])[:, None, None, None])
    X, V = np.array([2.3, 3.1, 2.8]), np.array([0.01, -0.02, 0.03])
    G, drag = orc.couple_point(u, X, V, 0.5, obstacles=obst)
    idx, w, _ = orc.stencil(X, (nx, ny, nz))
    fl = np.array([obst[0].ravel()[i] == 0 for i in idx])
    uref = sum(w[k] * u.reshape(3, -1)[:, idx[k]] for k in range(8))
    assert np.allclose(drag, 0.5 * (V - uref), rtol=1e-15, atol=0)
    assert np.allclose(G.reshape(3, -1).sum(axis=1), drag * w[fl].sum(), rtol=1e-14, atol=0)
    assert 0 < w[fl].sum() < 1
    assert np.all(G.reshape(3, -1)[:, obst[0].ravel() != 0] == 0)
