"""Obstacles on the GPU against the oracle: shapes (bit-exact node sets),
the lattice update with resting and moving obstacles, the coupled step next to
obstacles (the S-shaped channel stand-in), batching, and clearing."""
import numpy as np
import pytest

from paper_1312_3426_amd import synth

from gpu_util import check, fmt, gpu_fields, oracle_fields, rel, say

pytestmark = pytest.mark.gpu
B = synth.Boundary


@pytest.fixture(scope="module")
def oif():
    from paper_1312_3426_amd import oif as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build()
    return oracle


SHAPES = [
    [B("rhomboid", corner=(1.5, 1.5, 1.5), a=(2, 0, 0), b=(0, 2, 0), c=(0, 0, 2))],
    [B("rhomboid", corner=(0.3, 0.2, 0.1), a=(4.1, 0.3, 0), b=(1.7, 2.9, 0.2), c=(0.1, 0.4, 3.3))],
    [B("wall", normal=(1, 1, 0.5), dist=4.2), B("wall", normal=(0, 0, -1), dist=-6.0, velocity=(0.01, 0, 0))],
]


@pytest.mark.parametrize("k", range(len(SHAPES)))
def test_boundary_shapes_match_oracle(oif, orc, k):
    nx, ny, nz = 9, 8, 7
    c = oif.Context(nx, ny, nz, precision="fp32")
    for b in SHAPES[k]:
        if b.kind == "rhomboid":
            c.boundary_rhomboid(b.corner, b.a, b.b, b.c, b.velocity)
        else:
            c.boundary_wall(b.normal, b.dist, b.velocity)
    mine = c.read_boundary()
    ref, _ = orc.boundary_field(nx, ny, nz, SHAPES[k])
    c.close()
    assert np.array_equal(mine, ref)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("nx", [14, 128])
def test_lattice_with_obstacles_vs_oracle(oif, orc, prec, walls, nx):
    """Random populations, a resting sheared rhomboid, a sliding wall and a
    moving slab, body force; 12 steps of the lattice alone (rows of 14 nodes,
    and rows of two whole 64-node tiles)."""
    ny, nz = 11, 9
    bnd = [B("rhomboid", corner=(3.2, 2.1, 1.3), a=(4.0, 0.6, 0), b=(0.8, 3.9, 0.4), c=(0.2, 0.3, 4.1)),
           B("wall", normal=(0, 1, 0), dist=1.0, velocity=(0.02, 0, 0.01)),
           B("rhomboid", corner=(11, 0, 0), a=(2, 0, 0), b=(0, ny, 0), c=(0, 0, nz), velocity=(0.015, 0, 0))]
    box = synth.Box(nx, ny, nz, g=(1e-5, 2e-6, -3e-6), walls_z=walls, friction=0.5, boundaries=bnd)
    rng = np.random.default_rng(5)
    n0 = synth.random_populations(rng, box, amp=1e-3)
    s = orc.System(box)
    s.n[:] = n0
    c = oif.Context.from_box(box, precision=prec)
    c.write_populations(n0)
    c.step(12)
    s.run(12)
    res = check(gpu_fields(c, box.rho0, None), oracle_fields(s, None), prec, box.rho0, nx)
    say(f"[obstacles] lattice {prec} walls={walls} nx={nx}: {fmt(res)}")
    c.close()
    assert all(v[3] for v in res.values()), fmt(res)


@pytest.mark.parametrize("prec,steps", [("fp64", (1, 20)), ("fp32", (1, 100))])
def test_obstacle_channel_vs_oracle(oif, orc, prec, steps):
    """S-shaped obstacle channel with a velocity inlet and ten cells."""
    box = synth.config_obstacle_channel(max(steps))
    say(f"[obstacles] {box.name} {prec}")
    s = orc.System(box)
    X0 = s.X.copy()
    c = oif.Context.from_box(box, precision=prec)
    solid, _ = orc.boundary_field(box.nx, box.ny, box.nz, box.boundaries)
    assert np.array_equal(c.read_boundary(), solid)
    done = 0
    for k in steps:
        c.step(k - done)
        s.run(k - done)
        done = k
        res = check(gpu_fields(c, box.rho0, X0), oracle_fields(s, X0), prec, box.rho0, box.nx)
        say(f"   step {k}: {fmt(res)}")
        assert all(v[3] for v in res.values()), fmt(res)
    c.close()


@pytest.mark.parametrize("prec,bound", [("fp16", 5e-3), ("bf16", 5e-2)])
@pytest.mark.parametrize("mrt", [False, True])
def test_obstacle_channel_storage_forms_vs_oracle(oif, orc, prec, bound, mrt):
    """The obstacle channel (bounce-back from solid nodes, the moving inlet's
    wall term, ten cells) with FP16 / BF16 storage of the deviations, BGK and
    MRT collision: velocity error after 100 steps (MRT: 10, the oracle's
    mode-space collision is slow) against the FP64 oracle, relative to max |u|,
    within the bounds the plain channel meets in these forms."""
    steps = 10 if mrt else 100
    box = synth.config_obstacle_channel(steps)
    if mrt:
        box.mrt = (0.25, -0.4, 0.0, 0.0)
    say(f"[obstacles] {box.name} {prec}{' mrt' if mrt else ''}")
    s = orc.System(box)
    X0 = s.X.copy()
    c = oif.Context.from_box(box, precision=prec)
    c.step(steps)
    s.run(steps)
    g, o = gpu_fields(c, box.rho0, X0), oracle_fields(s, X0)
    c.close()
    e = {k: rel(g[k], o[k]) for k in ("u", "delta", "dX", "V")}
    say(f"   step {steps}: " + ", ".join(f"{a}={b:.2e}" for a, b in e.items()))
    assert e["u"] <= bound


def test_obstacle_batch_matches_single_boxes(oif):
    boxes = [synth.config_obstacle_channel(10, seed=6), synth.config_channel_rbc(10)]
    singles = []
    for b in boxes:
        c = oif.Context.from_box(b, precision="fp32")
        c.step(10)
        singles.append((c.read_populations(), c.read_mesh(-1)[0]))
        c.close()
    ctxs = [oif.Context.from_box(b, precision="fp32") for b in boxes]
    bt = oif.Batch(ctxs)
    bt.step(10)
    for c, (n, X) in zip(ctxs, singles):
        assert np.array_equal(c.read_populations(), n) and np.array_equal(c.read_mesh(-1)[0], X)
    bt.close()
    for c in ctxs:
        c.close()


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_obstacle_kernel_without_solid_nodes_is_bitwise_plain(oif, prec):
    """A boundary that contains no node centre switches the box to the lattice
    kernel with the obstacle code; with nothing solid the update must be the
    plain one bit for bit (same collision arithmetic in both kernels)."""
    say(f"[obstacles] empty boundary vs none, {prec}")
    box = synth.config_channel_rbc(10)
    outs = []
    for empty in (False, True):
        c = oif.Context.from_box(box, precision=prec)
        if empty:
            # half-space z < 0.25: below the first node centre (z = 0.5)
            c.boundary_wall((0.0, 0.0, 1.0), 0.25)
            assert not c.read_boundary().any()
        c.step(10)
        outs.append((c.read_populations(), c.read_mesh(-1)[0]))
        c.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_boundary_clear_restores_plain_step(oif):
    box = synth.config_channel_rbc(10)
    outs = []
    for with_obstacle in (False, True):
        c = oif.Context.from_box(box, precision="fp32")
        if with_obstacle:
            c.boundary_rhomboid((5, 5, 5), (3, 0, 0), (0, 3, 0), (0, 0, 3), (0.01, 0, 0))
            c.boundary_clear()
            assert not c.read_boundary().any()
        c.step(10)
        outs.append(c.read_populations())
        c.close()
    assert np.array_equal(*outs)


def test_boundary_validation(oif):
    c = oif.Context(8, 8, 8, precision="fp32")
    with pytest.raises(oif.OifError) as ei:
        c.boundary_rhomboid((0, 0, 0), (1, 0, 0), (2, 0, 0), (0, 0, 1))   # degenerate
    assert ei.value.code == oif.E_ARG
    with pytest.raises(oif.OifError) as ei:
        c.boundary_wall((0, 0, 0), 1.0)                                   # no normal
    assert ei.value.code == oif.E_ARG
    with pytest.raises(oif.OifError) as ei:
        c.boundary_wall((0, 0, 1), 1.0, (np.nan, 0, 0))
    assert ei.value.code == oif.E_ARG
    assert c.boundary_wall((0, 0, 1), 1.0) == 1
    c.close()
