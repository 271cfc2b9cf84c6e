"""GPU parity of the optional engine variants through the C ABI: the
multiple-relaxation-time collision (the LB operator of the paper's
references) and the velocity Verlet mesh integrator (the paper's engine),
against the FP64 oracle on the same seeded inputs."""
import dataclasses

import numpy as np
import pytest

from paper_1312_3426_amd import synth

from gpu_util import W, check, fmt, gpu_fields, oracle_fields, rel, say

pytestmark = pytest.mark.gpu

RATES = {
    "shear_bulk": (0.25, -0.4, 0.0, 0.0),
    "ghosts": (-0.3, 0.5, 0.6, -0.7),
}


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


def assert_ok(res, what):
    bad = {k: v for k, v in res.items() if not v[3]}
    assert not bad, f"{what}: {fmt(bad)}"


LB_CASES = [
    # (nx, ny, nz, walls)
    (20, 20, 20, False),   # 8000 nodes: 31.25 blocks of 256
    (9, 7, 11, True),      # ragged, bounce-back walls
    (2, 2, 2, False),      # every neighbour wraps onto the box
    (128, 2, 3, True),     # rows of two whole tiles: x pushes cross tiles
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("rates", sorted(RATES))
@pytest.mark.parametrize("case", LB_CASES, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}{'w' if c[3] else ''}")
def test_mrt_lattice_vs_oracle(oif, orc, prec, rates, case):
    nx, ny, nz, walls = case
    gam = RATES[rates]
    say(f"[mrt] lattice {prec} {rates} {case}")
    rng = np.random.default_rng(nx * 100 + ny * 10 + nz)
    box = synth.Box(nx, ny, nz, g=(1e-5, -2e-5, 3e-5), walls_z=walls, mrt=gam)
    n0 = synth.random_populations(rng, box, amp=1e-3)
    ctx = oif.Context.from_box(box, precision=prec)
    ctx.write_populations(n0)
    n_or = n0.copy()
    for step in (1, 9):
        ctx.step(step)
        for _ in range(step):
            n_or = orc.lb_step(n_or, g=box.g, walls_z=walls, mrt=gam)
        _, u_or = orc.moments(n_or, g=box.g)
        g = dict(delta=ctx.read_populations() - W[:, None, None, None], u=ctx.read_velocity())
        o = dict(delta=n_or - W[:, None, None, None], u=u_or)
        res = check(g, o, prec, 1.0, max(nx, ny, nz), keys=("delta", "u"))
        say(f"   after {step}: {fmt(res)}")
        assert_ok(res, f"step {step}")
    ctx.close()


def test_mrt_equal_rates_matches_bgk(oif):
    """All factors 1 - 1/tau: the MRT kernel reproduces the BGK kernel (FP64,
    up to the different rounding order of the two operators)."""
    say("[mrt] equal rates vs BGK, fp64")
    tau = 0.8
    gam = 1 - 1 / tau
    box = synth.config_sphere_fp64(10)
    box.tau = tau
    out = []
    for mrt in (None, (gam,) * 4):
        c = oif.Context.from_box(box, precision="fp64")
        c.set_mrt(mrt)
        c.step(10)
        out.append((c.read_populations(), c.read_mesh(-1)[0]))
        c.close()
    dn = np.abs(out[0][0] - out[1][0]).max()
    dx = np.abs(out[0][1] - out[1][1]).max()
    say(f"   max |n_mrt - n_bgk| = {dn:.2e}, |X| {dx:.2e}")
    assert dn < 1e-14 and dx < 1e-12


def _deformed_sphere(orc, box, seed=21):
    rng = np.random.default_rng(seed)
    sysm = orc.System(box)
    X0 = sysm.X + 0.012 * rng.standard_normal(sysm.X.shape)
    V0 = 2e-4 * rng.standard_normal(sysm.X.shape)
    n0 = synth.random_populations(rng, box, amp=2e-3)
    sysm.X[:] = X0
    sysm.V[:] = V0
    sysm.n[:] = n0
    return sysm, X0, V0, n0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_mrt_coupled_sphere_vs_oracle(oif, orc, prec):
    """Coupled step with the MRT collision: 20^3 box, 642-node sphere,
    deformed moving start, random populations."""
    say(f"[mrt] coupled sphere642 {prec}")
    box = synth.config_sphere_fp64(20)
    box.mrt = RATES["ghosts"]
    sysm, X0, V0, n0 = _deformed_sphere(orc, box)
    ctx = oif.Context.from_box(box, precision=prec)
    ctx.write_mesh(-1, X0, V0)
    ctx.write_populations(n0)
    done = 0
    for k in (1, 20):
        ctx.step(k - done)
        sysm.run(k - done)
        done = k
        res = check(gpu_fields(ctx, box.rho0, X0), oracle_fields(sysm, X0), prec, box.rho0, 20)
        say(f"   step {k}: {fmt(res)}")
        assert_ok(res, f"step {k}")
    ctx.close()


def test_mrt_obstacle_channel_vs_oracle(oif, orc):
    """MRT collision with obstacles and a moving inlet (the obstacle kernel's
    MRT variant), ten cells, FP64."""
    say("[mrt] obstacle channel fp64")
    box = synth.config_obstacle_channel(10, seed=6)
    box.mrt = RATES["shear_bulk"]
    sysm = orc.System(box)
    X0 = sysm.X.copy()
    ctx = oif.Context.from_box(box, precision="fp64")
    ctx.step(10)
    sysm.run(10)
    res = check(gpu_fields(ctx, box.rho0, X0), oracle_fields(sysm, X0), "fp64", box.rho0, box.nx)
    say(f"   step 10: {fmt(res)}")
    assert_ok(res, "step 10")
    ctx.close()


def test_mrt_batch_matches_single_boxes(oif):
    """A batch mixing BGK and MRT boxes (one lattice launch per variant)
    equals the boxes stepped one by one, bit for bit."""
    say("[mrt] batch of BGK and MRT boxes vs single")
    boxes = synth.config_batch(n_boxes=3, steps=10)
    boxes[1].mrt = RATES["ghosts"]
    singles = []
    for bx in boxes:
        c = oif.Context.from_box(bx, precision="fp32")
        c.step(10)
        singles.append((c.read_populations(), c.read_mesh(-1)[0]))
        c.close()
    ctxs = [oif.Context.from_box(bx, precision="fp32") for bx in boxes]
    B = oif.Batch(ctxs)
    B.step(10)
    for c, (n, X) in zip(ctxs, singles):
        assert np.array_equal(c.read_populations(), n) and np.array_equal(c.read_mesh(-1)[0], X)
    B.close()
    for c in ctxs:
        c.close()


def test_mrt_rejects_unstable_factors(oif):
    c = oif.Context(8, 8, 8, precision="fp32")
    for bad in ((1.0, 0, 0, 0), (0, -1.0, 0, 0), (0, 0, float("nan"), 0), (0, 0, 0, 1.5)):
        with pytest.raises(oif.OifError):
            c.set_mrt(bad)
    c.set_mrt((0.1, 0.2, 0.3, 0.4))
    c.set_mrt(None)
    c.close()


# ---------------------------------------------------------------------------
# velocity Verlet
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec,mrt", [("fp64", None), ("fp32", None), ("fp64", "ghosts")])
def test_verlet_coupled_sphere_vs_oracle(oif, orc, prec, mrt):
    """Velocity Verlet on the 20^3 sphere case from a deformed moving start:
    fields and the carried force against the oracle (optionally with MRT)."""
    say(f"[verlet] coupled sphere642 {prec} mrt={mrt}")
    box = synth.config_sphere_fp64(20)
    box.integrator = "verlet"
    box.mrt = RATES[mrt] if mrt else None
    sysm, X0, V0, n0 = _deformed_sphere(orc, box, seed=22)
    ctx = oif.Context.from_box(box, precision=prec)
    assert ctx.info().integrator == 1
    ctx.write_mesh(-1, X0, V0)
    ctx.write_populations(n0)
    done = 0
    for k in (1, 20):
        ctx.step(k - done)
        sysm.run(k - done)
        done = k
        g, o = gpu_fields(ctx, box.rho0, X0), oracle_fields(sysm, X0)
        g["F"], o["F"] = ctx.read_force(-1), sysm.F
        res = check(g, o, prec, box.rho0, 20)
        fF = check(dict(V=g["F"]), dict(V=o["F"]), prec, box.rho0, 20, keys=("V",))
        say(f"   step {k}: {fmt(res)}; F: {fmt(fF)}")
        assert_ok(res, f"step {k}")
        assert_ok(fF, f"force, step {k}")
    ctx.close()


def test_verlet_checkpoint_graph_and_batch_bitwise(oif):
    """Verlet state = populations (as stored deviations) + positions +
    velocities + carried force: restoring all four continues bit for bit; graph replay and a batch that
    mixes Verlet and Euler boxes equal eager single-box stepping."""
    say("[verlet] checkpoint / graph / batch, fp32 channel")
    box = synth.config_channel_rbc(20)
    box.integrator = "verlet"
    a = oif.Context.from_box(box, precision="fp32")
    a.step(5)
    n, (X, V), F = a.read_deviations(), a.read_mesh(-1), a.read_force(-1)
    assert np.abs(F).max() > 0
    b = oif.Context.from_box(box, precision="fp32")
    b.write_deviations(n)
    b.write_mesh(-1, X, V)
    b.write_force(-1, F)
    a.step(7)
    b.step(7)
    assert np.array_equal(a.read_populations(), b.read_populations())
    assert np.array_equal(a.read_mesh(-1)[0], b.read_mesh(-1)[0])
    assert np.array_equal(a.read_force(-1), b.read_force(-1))
    a.close()
    b.close()
    # graph replay vs eager
    out = []
    for graph in (0, 4):
        c = oif.Context.from_box(box, precision="fp32")
        c.set_graph(graph)
        c.step(12)
        out.append((c.read_populations(), c.read_mesh(-1)[0], c.read_force(-1)))
        c.close()
    assert all(np.array_equal(p, q) for p, q in zip(*out))
    # batch mixing integrators
    boxes = synth.config_batch(n_boxes=3, steps=10)
    boxes[0].integrator = "verlet"
    boxes[2].integrator = "verlet"
    singles = []
    for bx in boxes:
        c = oif.Context.from_box(bx, precision="fp32")
        c.step(10)
        singles.append((c.read_populations(), c.read_mesh(-1)[0]))
        c.close()
    ctxs = [oif.Context.from_box(bx, precision="fp32") for bx in boxes]
    B = oif.Batch(ctxs)
    B.step(10)
    for c, (n, X) in zip(ctxs, singles):
        assert np.array_equal(c.read_populations(), n) and np.array_equal(c.read_mesh(-1)[0], X)
    B.close()
    for c in ctxs:
        c.close()


def test_verlet_state_errors(oif):
    box = synth.config_channel_rbc(1)
    c = oif.Context.from_box(box, precision="fp32")
    with pytest.raises(oif.OifError):
        c.write_force(-1, np.zeros((box.n_mesh_nodes, 3)))  # Euler carries no force
    c.set_overlap(True)
    with pytest.raises(oif.OifError):
        c.set_integrator("verlet")
    c.set_overlap(False)
    c.set_integrator("verlet")
    with pytest.raises(oif.OifError):
        c.set_overlap(True)
    with pytest.raises(oif.OifError):
        c.write_force(-1, np.full((box.n_mesh_nodes, 3), np.nan))
    c.close()


# ---------------------------------------------------------------------------
# soft-sphere repulsion
# ---------------------------------------------------------------------------
def _contact_box(n_box=16, sep=4.18, walls=False, integrator="euler", mrt=None, bnd=(), extra=(), same=False,
                 cut=0.5):
    """Two level-2 icospheres (162 nodes, radius 2) whose surfaces nearly touch,
    types 0 and 1 (or both 0), pair and wall repulsion in range."""
    x, t = synth.icosphere(2, 2.0)
    tm = synth.Template(x, t, ks=0.05, kb=0.01, kv=0.5)
    rng = np.random.default_rng(41)
    c = n_box / 2
    objs = [synth.ObjectSpec(0, np.array([c - sep / 2, c, c]), rot=synth.random_rotation(rng), ptype=0),
            synth.ObjectSpec(0, np.array([c + sep / 2, c + 0.1, c - 0.05]), rot=synth.random_rotation(rng),
                             ptype=0 if same else 1)]
    objs += list(extra)
    rep = [synth.SoftSphere(0, 0 if same else 1, a=2e-6, n=2.0, cutoff=cut, offset=0.02),
           synth.SoftSphere(0, None, a=1e-6, n=1.5, cutoff=0.8)]
    if not same:
        rep.append(synth.SoftSphere(1, None, a=1e-6, n=1.5, cutoff=0.8))
    return synth.Box(n_box, n_box, n_box, g=(1e-5, 0, 0), friction=0.5, walls_z=walls, templates=[tm],
                     objects=objs, repulsion=rep, boundaries=list(bnd), integrator=integrator, mrt=mrt)


def _run_vs_oracle(oif, orc, box, prec, steps, label):
    sysm = orc.System(box)
    X0 = sysm.X.copy()
    Fr = sysm.repulsion()
    assert np.abs(Fr).max() > 1e-5, "the configuration must put pairs in range"
    ctx = oif.Context.from_box(box, precision=prec)
    done = 0
    for k in steps:
        ctx.step(k - done)
        sysm.run(k - done)
        done = k
        res = check(gpu_fields(ctx, box.rho0, X0), oracle_fields(sysm, X0), prec, box.rho0, box.nx)
        say(f"   {label} step {k}: {fmt(res)}")
        assert_ok(res, f"{label} step {k}")
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_repulsion_pairs_vs_oracle(oif, orc, prec):
    """Two cells in contact in a periodic box (cells hashed into buckets)."""
    say(f"[repulsion] pair contact {prec}")
    _run_vs_oracle(oif, orc, _contact_box(), prec, (1, 10), "pairs")


def test_repulsion_walls_shapes_and_verlet_vs_oracle(oif, orc):
    """Cells against the z walls, a sheared block and a half-space wall, with
    velocity Verlet and MRT, FP64; a second box small enough that every cell
    has its own bucket."""
    say("[repulsion] walls, shapes, verlet, mrt fp64")
    block = synth.Boundary("rhomboid", corner=(1.0, 9.9, 2.0), a=(5.0, 0.0, 0.5), b=(0.5, 3.0, 0.0),
                           c=(0.0, 0.3, 4.0))
    wall = synth.Boundary("wall", normal=(0.0, -1.0, 0.0), dist=-13.6)  # solid for y > 13.6
    box = _contact_box(sep=4.2, walls=True, integrator="verlet", mrt=RATES["ghosts"], bnd=(block, wall))
    box.objects[0].origin = np.array([5.0, 8.0, 2.6])   # near z = 0 and the block
    box.objects[1].origin = np.array([9.2, 11.5, 2.7])  # near the half-space wall
    _run_vs_oracle(oif, orc, box, "fp64", (1, 8), "walls")
    # pair range 1.62: 9^3 cells of edge 16/9, fewer than the 1024 buckets, one bucket each
    direct = _contact_box(sep=4.6, cut=1.6)
    _run_vs_oracle(oif, orc, direct, "fp64", (1, 6), "direct")


def test_refused_boundary_leaves_no_shape(oif):
    """A boundary call refused for its velocity leaves the obstacle shapes
    that the wall repulsion acts against as they were: steps afterwards give
    the bits of a context that never made the call (the refused half-space
    and block would lie next to the cells)."""
    say("[repulsion] refused boundaries leave no shape")
    box = _contact_box(walls=True)
    ref = oif.Context.from_box(box, precision="fp32")
    c = oif.Context.from_box(box, precision="fp32")
    with pytest.raises(oif.OifError) as ei:
        c.boundary_wall((1.0, 0.0, 0.0), 7.5, (np.nan, 0.0, 0.0))
    assert ei.value.code == oif.E_ARG
    with pytest.raises(oif.OifError) as ei:
        c.boundary_rhomboid((7.0, 9.8, 7.0), (2.0, 0.0, 0.0), (0.0, 2.0, 0.0), (0.0, 0.0, 2.0), (0.0, np.inf, 0.0))
    assert ei.value.code == oif.E_ARG
    ref.step(5)
    c.step(5)
    (X1, V1), (X2, V2) = ref.read_mesh(-1), c.read_mesh(-1)
    ref.close()
    c.close()
    assert np.array_equal(X1, X2) and np.array_equal(V1, V2)


@pytest.mark.parametrize("prec,bound", [("fp16", 5e-3), ("bf16", 5e-2)])
def test_mixed_feature_batch_storage_forms_vs_oracle(oif, orc, prec, bound):
    """One batch in FP16 / BF16 storage whose boxes each switch on other
    options: velocity Verlet (channel), soft-sphere repulsion with MRT (two
    cells in contact), the conservative force model (sphere).  Each box
    against the FP64 oracle after 20 steps: velocity error relative to max |u|
    within the storage form's bound for the plain channel, and the mesh
    fields close to the oracle's."""
    say(f"[batch] mixed options, {prec} storage")
    chan = synth.config_channel_rbc(20, n_cells=4)
    chan.integrator = "verlet"
    contact = _contact_box(mrt=RATES["ghosts"])
    contact.name = "contact_repulsion_mrt"
    sph = synth.config_sphere_fp64(20)
    sph.templates[0].model = "conservative"
    boxes = [chan, contact, sph]
    systems = [orc.System(b) for b in boxes]
    X0s = [s.X.copy() for s in systems]
    ctxs = [oif.Context.from_box(b, precision=prec) for b in boxes]
    B = oif.Batch(ctxs)
    B.step(20)
    B.close()
    for b, s, X0, c in zip(boxes, systems, X0s, ctxs):
        s.run(20)
        g, o = gpu_fields(c, b.rho0, X0), oracle_fields(s, X0)
        c.close()
        e = {k: rel(g[k], o[k]) for k in ("u", "delta", "dX", "V")}
        say(f"   {b.name}: " + ", ".join(f"{a}={v:.2e}" for a, v in e.items()))
        assert e["u"] <= bound and e["dX"] <= bound and e["V"] <= bound, (b.name, e)


def test_repulsion_same_type_and_minimum_image(oif, orc):
    """Both cells of type 0 with a 0-0 interaction (also acting inside each
    cell), placed across the periodic x boundary."""
    say("[repulsion] same type across the periodic boundary fp64")
    box = _contact_box(sep=4.16, same=True)
    box.objects[0].origin = np.array([1.9, 8.0, 8.0])
    box.objects[1].origin = np.array([-2.26 + 16.0, 8.1, 7.95])
    _run_vs_oracle(oif, orc, box, "fp64", (1, 6), "periodic")


def test_repulsion_modes_bitwise(oif):
    """Repulsion is deterministic: rerun, graph replay and a batch with a
    plain box give the same bits."""
    say("[repulsion] determinism, graph, batch fp32")
    box = _contact_box()
    out = []
    for graph in (0, 0, 4):
        c = oif.Context.from_box(box, precision="fp32")
        c.set_graph(graph)
        c.step(12)
        out.append((c.read_populations(), c.read_mesh(-1)[0]))
        c.close()
    assert all(np.array_equal(out[0][i], o[i]) for o in out[1:] for i in range(2))
    other = synth.config_batch(n_boxes=1, steps=12)[0]
    ref = []
    for bx in (box, other):
        c = oif.Context.from_box(bx, precision="fp32")
        c.step(12)
        ref.append((c.read_populations(), c.read_mesh(-1)[0]))
        c.close()
    ctxs = [oif.Context.from_box(bx, precision="fp32") for bx in (box, other)]
    B = oif.Batch(ctxs)
    B.step(12)
    for c, (n, X) in zip(ctxs, ref):
        assert np.array_equal(c.read_populations(), n) and np.array_equal(c.read_mesh(-1)[0], X)
    B.close()
    for c in ctxs:
        c.close()


def test_repulsion_duplicate_settings_last_one_holds(oif):
    """A pair and a wall interaction set twice (the pair the second time with
    its types swapped): the same bits as the later settings alone."""
    say("[repulsion] duplicate settings fp32")
    box = _contact_box(walls=True)
    dup = synth.Box(**{f.name: getattr(box, f.name) for f in dataclasses.fields(box)})
    dup.repulsion = [synth.SoftSphere(1, 0, a=7e-6, n=3.0, cutoff=0.45, offset=0.0),
                     synth.SoftSphere(0, None, a=5e-6, n=2.0, cutoff=0.7),
                     synth.SoftSphere(0, 1, a=2e-6, n=2.0, cutoff=0.5, offset=0.02)] + box.repulsion[1:]
    out = []
    for b in (box, dup):
        c = oif.Context.from_box(b, precision="fp32")
        c.step(6)
        X, V = c.read_mesh(-1)
        out.append((c.read_populations(), X, V))
        c.close()
    assert all(np.array_equal(p, q) for p, q in zip(*out))


def test_repulsion_argument_errors(oif):
    c = oif.Context(8, 8, 8, precision="fp32")
    for args in ((16, 0, 1e-6, 2.0, 0.5), (0, -1, 1e-6, 2.0, 0.5), (0, 1, -1.0, 2.0, 0.5),
                 (0, 1, 1e-6, 0.0, 0.5), (0, 1, 1e-6, 2.0, 0.0), (0, 1, 1e-6, 2.0, 4.5)):
        with pytest.raises(oif.OifError):
            c.set_soft_sphere(*args)
    with pytest.raises(oif.OifError):
        c.set_wall_soft_sphere(16, 1e-6, 2.0, 0.5)
    c.set_soft_sphere(0, 1, 1e-6, 2.0, 0.5)
    c.close()
