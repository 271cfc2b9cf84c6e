"""GPU tests of the execution modes and the auxiliary subsystems, through the
C ABI: overlapped vs sequential steps, graph replay vs eager launches,
autotuning, checkpoint/restore, the batching form, object analysis,
conservation diagnostics, the watchdog and input validation."""
import dataclasses
import json
import os
import re

import numpy as np
import pytest

from paper_1312_3426_amd import synth

from gpu_util import ATOL, W, check, fmt, gpu_fields, oracle_fields, rel, say

pytestmark = pytest.mark.gpu


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


def state(ctx):
    X, V = ctx.read_mesh(-1)
    return ctx.read_populations(), X, V


def same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


def channel(steps=40):
    return synth.config_channel_rbc(steps)


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_overlap_matches_sequential_bitwise(oif, prec):
    """Split stepping runs other instantiations of the lattice kernel (touch
    masks, populations loaded after the mask) than the sequential step; the
    collision is rounded as written in all of them, so the bits agree."""
    say(f"[modes] overlap vs sequential, {prec} channel")
    box = channel()
    outs = []
    for ov in (False, True):
        c = oif.Context.from_box(box, precision=prec)
        c.set_overlap(ov)
        c.step(40)
        assert c.info().overlap == int(ov)
        outs.append(state(c))
        c.close()
    assert same(*outs)


@pytest.mark.parametrize("prec,overlap,case", [("fp32", False, "channel"), ("fp16", False, "channel"),
                                               ("fp64", False, "channel"), ("fp32", True, "channel"),
                                               ("fp32", False, "obstacles"), ("fp32", False, "mrt")])
def test_nontemporal_loads_bitwise(oif, prec, overlap, case):
    """The cache policy of the population reads changes no value, in either
    form (the spreading is exact fixed point in both)."""
    say(f"[modes] non-temporal vs ordinary population reads, {prec} {case}, overlap={overlap}")
    box = synth.config_obstacle_channel(40) if case == "obstacles" else channel()
    if case == "mrt":
        box.mrt = (0.25, -0.4, 0.6, -0.7)
    outs = []
    for nt in (False, True):
        c = oif.Context.from_box(box, precision=prec)
        c.set_overlap(overlap)
        c.set_lb_loads(nt)
        assert c.info().lb_nontemporal == int(nt)
        c.step(40)
        outs.append(state(c))
        if nt:
            assert oif.lib().oif_set_lb_loads(c.h, 2) == -1  # OIF_E_ARG
        c.close()
    assert same(*outs)


@pytest.mark.parametrize("prec,overlap", [("fp32", False), ("fp32", True), ("fp64", False), ("fp16", False),
                                          ("bf16", True)])
def test_graph_matches_eager_bitwise(oif, prec, overlap):
    say(f"[modes] graph vs eager, {prec}, overlap={overlap}")
    box = channel()
    outs = []
    for g in (0, 8):
        c = oif.Context.from_box(box, precision=prec)
        c.set_overlap(overlap)
        c.set_graph(g)
        c.step(3)    # odd: the graph path must first realign to parity 0
        c.step(37)   # 4 replays of 8 steps + 5 eager
        outs.append(state(c))
        c.close()
    assert same(*outs)


@pytest.mark.parametrize("overlap", [False, True])
def test_step_timed_matches_step(oif, overlap):
    say(f"[modes] timed vs plain stepping, overlap={overlap}")
    box = channel()
    outs = []
    for timed in (False, True):
        c = oif.Context.from_box(box, precision="fp32")
        c.set_overlap(overlap)
        if timed:
            t = c.step_timed(40)
            assert t.total_ms > 0 and t.lb_ms > 0 and t.mesh_ms > 0 and t.overlap == int(overlap)
        else:
            c.step(40)
        outs.append(state(c))
        c.close()
    assert same(*outs)


def test_autotune_leaves_state_unchanged(oif, tmp_path):
    say("[modes] autotune mid-run")
    box = channel()
    outs = []
    cache = str(tmp_path / "tune.json")
    for tune in (False, True):
        c = oif.Context.from_box(box, precision="fp32")
        c.step(20)
        if tune:
            c.autotune(cache)
            i = c.info()
            assert i.lb_block in (128, 256, 512, 1024) and i.mesh_block % 64 == 0 and 64 <= i.mesh_block <= 1024
            chosen = (i.lb_block, i.mesh_block, i.xcd_remap, i.lb_nontemporal, i.force_clear_by_membrane)
        c.step(20)
        outs.append(state(c))
        c.close()
    # tuning changes launch shapes: FP32 results are independent of them except
    # for the FP64 area/volume block sums, which differ only by round-off
    for a, b in zip(*outs):
        assert rel(a, b) < 1e-6
    assert os.path.exists(cache) and "gfx950" in open(cache).read()
    # a second context finds the shapes, the read policy and who clears the
    # coupling force in the cache
    entries = json.load(open(cache))
    assert all(len(v) == 5 for v in entries.values())
    c = oif.Context.from_box(box, precision="fp32")
    c.set_lb_loads(not chosen[3])
    c.set_force_clear(not chosen[4])
    c.autotune(cache)
    i = c.info()
    assert (i.lb_block, i.mesh_block, i.xcd_remap, i.lb_nontemporal, i.force_clear_by_membrane) == chosen
    c.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16", "bf16"])
def test_checkpoint_restore_bitwise(oif, prec):
    """Checkpoint = stored deviations + mesh positions and velocities:
    restoring them into a new context continues bit for bit in every form,
    also early in a run, when many deviations are too small for full FP64
    populations near w_i rho0 to carry all their bits."""
    say(f"[modes] checkpoint / restore, {prec}")
    box = channel()
    for first in (3, 30):
        a = oif.Context.from_box(box, precision=prec)
        a.step(first)
        d = a.read_deviations()
        X, V = a.read_mesh(-1)
        a.step(20)
        ref = state(a)
        a.close()
        b = oif.Context.from_box(box, precision=prec)
        b.write_deviations(d)
        assert np.array_equal(b.read_deviations(), d)
        b.write_mesh(-1, X, V)
        b.step(20)
        got = state(b)
        assert same(ref, got)
        b.close()


def test_population_round_trip(oif):
    """Full populations through FP64 and back: the stored deviations come
    back exactly wherever w_i rho0 + d_i carries all bits of d_i, and never
    off by more than the FP64 rounding of that sum."""
    say("[modes] population round trip")
    box = channel()
    a = oif.Context.from_box(box, precision="fp32")
    a.step(3)
    d = a.read_deviations()
    a.write_populations(a.read_populations())
    d2 = a.read_deviations()
    wr = (W * box.rho0)[:, None, None, None]
    assert np.all(np.abs(d2 - d) <= 2.0 ** -52 * wr)
    a.close()


def test_batch_matches_single_boxes(oif):
    say("[modes] batch of 3 boxes vs single contexts")
    boxes = synth.config_batch(n_boxes=3, steps=20)
    singles = []
    for bx in boxes:
        c = oif.Context.from_box(bx, precision="fp32")
        c.set_overlap(False)
        c.step(20)
        singles.append(state(c))
        c.close()
    ctxs = [oif.Context.from_box(bx, precision="fp32") for bx in boxes]
    B = oif.Batch(ctxs)
    B.set_graph(4)
    B.set_lb_loads(not ctxs[0].info().lb_nontemporal)  # the other read policy than the singles
    B.step(1)
    B.step(19)
    for c, ref in zip(ctxs, singles):
        assert same(ref, state(c))
    t = B.step_timed(4)
    assert t.total_ms > 0
    B.close()
    for c in ctxs:
        c.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_box_vs_oracle(oif, orc, prec):
    """Two batched boxes with 162/642/2562-node spheres (the largest split over
    several workgroups) against the oracle, 30 steps."""
    say(f"[modes] batch boxes 0-1 vs oracle ({prec})")
    boxes = synth.config_batch(n_boxes=2, steps=30)
    ctxs = [oif.Context.from_box(bx, precision=prec) for bx in boxes]
    B = oif.Batch(ctxs)
    B.step(30)
    for bx, c in zip(boxes, ctxs):
        s = orc.System(bx)
        X0 = s.X.copy()
        s.run(30)
        res = check(gpu_fields(c, bx.rho0, X0), oracle_fields(s, X0), prec, bx.rho0, max(bx.nx, bx.ny, bx.nz))
        say(f"   {bx.name} ({len(bx.objects)} cells): {fmt(res)}")
        assert all(v[3] for v in res.values())
    B.close()
    for c in ctxs:
        c.close()



@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_large_meshes_vs_oracle(oif, orc, prec):
    """A box whose 2562-node spheres do not fit LDS against the oracle: each is
    split over several workgroups (triangle and edge slices, then node patches
    with their positions, forces and coupling area in LDS, the element arrays
    in the global scratch)."""
    say(f"[modes] large meshes vs oracle ({prec})")
    bx = synth.config_batch(n_boxes=1, steps=30)[0]
    c = oif.Context.from_box(bx, precision=prec)
    c.step(30)
    i = c.info()  # objects are placed at the first step
    assert 0 < i.lds_objects < i.n_objects
    # the meshes outside LDS run split, four patches each
    assert i.lds_objects + i.split_objects == i.n_objects and i.split_lds_bytes > 0
    assert i.split_workgroups == 4 * i.split_objects
    s = orc.System(bx)
    X0 = s.X.copy()
    s.run(30)
    res = check(gpu_fields(c, bx.rho0, X0), oracle_fields(s, X0), prec, bx.rho0, max(bx.nx, bx.ny, bx.nz))
    say(f"   {bx.name} ({len(bx.objects)} cells, {i.lds_objects} in LDS): {fmt(res)}")
    assert all(v[3] for v in res.values())
    c.close()

@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("case", ["batchbox", "pulled"])
def test_force_clear_modes_bitwise(oif, case, prec):
    """The coupling force cleared by the lattice kernel (the default), by the
    membrane kernel from its lists of slots one step later, or by one and then
    the other, switching every two steps: the same bits (FP32, and FP64 with
    its 64-byte slots), eagerly, under graph capture and in a batch.  The batching box has 2562-node spheres split
    over several workgroups (a list per slice) beside spheres in LDS; in the
    pulled case one node 16 units out sends the sphere's coupling corner by
    corner (no list: the lattice kernel clears G in that step)."""
    say(f"[modes] force clear by lattice / membrane kernel, {case} {prec}")
    box = synth.config_batch(n_boxes=1, steps=12)[0] if case == "batchbox" else synth.config_sphere_fp64(12)

    def make(by_membrane=False):
        c = oif.Context.from_box(box, precision=prec)
        if case == "pulled":
            X, V = c.read_mesh(-1)
            X[0, 0] += 16.0
            c.write_mesh(-1, X, V)
        c.set_force_clear(by_membrane)
        assert c.info().force_clear_by_membrane == int(by_membrane)
        return c

    def state(c):
        X, V = c.read_mesh(-1)
        return c.read_deviations(), X, V

    def same(a, b):
        return all(np.array_equal(p, q) for p, q in zip(a, b))

    ref = make()
    ref.step(12)
    want = state(ref)
    ref.close()
    a = make(True)
    a.step(12)
    assert same(want, state(a)), "membrane-side clearing differs"
    a.close()
    b = make()
    for mode in (1, 0, 1, 1, 0, 0):
        b.set_force_clear(bool(mode))
        b.step(2)
    assert same(want, state(b)), "switching between the two differs"
    b.close()
    g = make(True)
    g.set_graph(4)
    g.step(12)
    assert same(want, state(g)), "membrane-side clearing under graph capture differs"
    g.close()
    c = make(True)
    B = oif.Batch([c])
    B.step(12)
    B.close()
    assert same(want, state(c)), "membrane-side clearing in a batch differs"
    c.close()
    if case == "pulled":  # the persistent form runs meshes whole, as the single box does here
        c = make(True)
        B = oif.Batch([c])
        B.set_persistent(True)
        B.step(12)
        B.close()
        assert same(want, state(c)), "membrane-side clearing in the persistent form differs"
        c.close()


def test_split_meshes_overlap_bitwise(oif):
    """Split stepping (the lattice update of the nodes outside every stencil
    concurrent with the membrane launches) with 2562-node spheres split into
    patches: each patch workgroup marks its own nodes' stencils for the next
    step, and the result is the sequential step's, bit for bit (FP32)."""
    say("[modes] overlap vs sequential, batching box with split meshes")
    box = synth.config_batch(n_boxes=1, steps=20)[0]
    outs = []
    for ov in (False, True):
        c = oif.Context.from_box(box, precision="fp32")
        c.set_overlap(ov)
        c.step(20)
        assert c.info().split_objects > 0 and c.info().overlap == int(ov)
        outs.append(state(c))
        c.close()
    assert same(*outs)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_split_meshes_verlet_vs_oracle(oif, orc, prec):
    """Velocity Verlet with 2562-node spheres split into patches (the staged
    half-step positions, the carried force written per patch) against the
    oracle."""
    say(f"[modes] split meshes with velocity Verlet vs oracle ({prec})")
    bx = synth.config_batch(n_boxes=1, steps=20)[0]
    bx.integrator = "verlet"
    c = oif.Context.from_box(bx, precision=prec)
    c.step(20)
    i = c.info()
    assert i.split_objects > 0 and i.integrator == 1
    s = orc.System(bx)
    X0 = s.X.copy()
    s.run(20)
    res = check(gpu_fields(c, bx.rho0, X0), oracle_fields(s, X0), prec, bx.rho0, max(bx.nx, bx.ny, bx.nz))
    say(f"   {bx.name}: {fmt(res)}")
    assert all(v[3] for v in res.values())
    c.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_split_meshes_conservative_vs_oracle(oif, orc, prec):
    """The conservative force model (gradient bending, balanced area forces)
    on every template of a batching box whose 2562-node spheres do not fit
    LDS: split into patches in the FP32 form (the model's per-hinge wing
    factors and feet gathered per patch), whole in global scratch in the FP64
    form (whose patches, with four FP64 words per edge, would not fit LDS);
    from a deformed moving
    start, against the oracle after 10 steps."""
    say(f"[modes] split meshes with the conservative model vs oracle ({prec})")
    bx = synth.config_batch(n_boxes=1, steps=10)[0]
    for t in bx.templates:
        t.model = "conservative"
    rng = np.random.default_rng(103)
    s = orc.System(bx)
    X0 = s.X + 0.01 * rng.standard_normal(s.X.shape)
    V0 = 1e-4 * rng.standard_normal(s.X.shape)
    s.X[:] = X0
    s.V[:] = V0
    c = oif.Context.from_box(bx, precision=prec)
    c.write_mesh(-1, X0, V0)
    c.step(10)
    i = c.info()
    s.run(10)
    res = check(gpu_fields(c, bx.rho0, X0), oracle_fields(s, X0), prec, bx.rho0, max(bx.nx, bx.ny, bx.nz))
    c.close()
    say(f"   {bx.name}: objects {i.n_objects}, in LDS {i.lds_objects}, split {i.split_objects}; {fmt(res)}")
    assert all(v[3] for v in res.values()), fmt(res)
    assert i.lds_objects < i.n_objects
    if prec == "fp32":
        assert i.split_objects > 0


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_oversize_meshes_vs_oracle(oif, orc, prec):
    """A 10242-node sphere, whose positions alone exceed LDS, runs in one
    workgroup with its mesh arrays in the global scratch and its coupling area
    in LDS; a 162-node sphere beside it stays in LDS.  Against the oracle."""
    say(f"[modes] oversize mesh vs oracle ({prec})")
    fine = {k: v * synth.FINE_MODULI_SCALE for k, v in synth.MODULI_DEFAULT.items()}
    big = synth.Template(*synth.icosphere(5, 6.0), **fine)
    small = synth.Template(*synth.icosphere(2, 3.0), **synth.MODULI_DEFAULT)
    bx = synth.Box(28, 24, 24, templates=[big, small], friction=synth.WORKING_FRICTION_FINE,
                   objects=[synth.ObjectSpec(0, np.array([10.3, 12.1, 11.7])),
                            synth.ObjectSpec(1, np.array([22.6, 11.4, 12.2]))],
                   steps=8, name="sphere10242_28x24x24")
    c = oif.Context.from_box(bx, precision=prec)
    c.step(8)
    i = c.info()
    assert i.lds_objects == 1 and i.cpl_objects == 1 and i.split_objects == 0 and i.cpl_lds_bytes > 0
    s = orc.System(bx)
    X0 = s.X.copy()
    s.run(8)
    res = check(gpu_fields(c, bx.rho0, X0), oracle_fields(s, X0), prec, bx.rho0, max(bx.nx, bx.ny, bx.nz))
    say(f"   {bx.name}: {fmt(res)}")
    assert all(v[3] for v in res.values())
    c.close()


@pytest.mark.parametrize("case", ["sphere20", "precision256"])
def test_touched_nodes_vs_oracle(oif, orc, case):
    """oif_touched_nodes (the count of distinct lattice nodes inside some mesh
    node's 2x2x2 stencil, the coupling term of the byte model) equals the
    oracle's count, at the start and after the meshes have moved."""
    box = synth.config_sphere_fp64(20) if case == "sphere20" else synth.config_precision(2)
    prec = "fp64" if case == "sphere20" else "fp32"
    say(f"[aux] touched nodes vs oracle, {box.name}")
    c = oif.Context.from_box(box, precision=prec)
    s = orc.System(box)
    if case == "sphere20":
        s.V[:] = 0.05 * np.random.default_rng(3).standard_normal(s.V.shape)
        c.write_mesh(-1, None, s.V)
    counts = []
    for steps in (0, 2):
        if steps:
            c.step(steps)
            s.run(steps)
            X, _ = c.read_mesh(-1)
            assert np.abs(X - s.X).max() < 1e-9
        g, o = c.touched_nodes(), s.touched()
        counts.append((g, o))
        assert g == o, (steps, g, o)
    say(f"   (gpu, oracle) at steps 0 and 2: {counts}")
    c.close()


def test_object_analysis_vs_oracle(oif, orc):
    say("[aux] object analysis")
    box = synth.config_sphere_fp64(30)
    c = oif.Context.from_box(box, precision="fp64")
    c.step(30)
    s = orc.System(box)
    s.run(30)
    Sg, Vol = s.geometry()
    a = c.object_analyze(0)
    assert a.volume == pytest.approx(Vol[0], rel=1e-12)
    assert a.area == pytest.approx(Sg[0], rel=1e-12)
    assert np.allclose(a.origin, s.X.mean(axis=0), rtol=0, atol=1e-12)
    assert np.allclose(a.velocity, s.V.mean(axis=0), rtol=1e-9, atol=1e-16)
    assert a.bounds[0] == pytest.approx(s.X[:, 0].min(), abs=1e-12)
    assert a.bounds[5] == pytest.approx(s.X[:, 2].max(), abs=1e-12)
    info = c.info()
    assert (info.n_objects, info.n_templates, info.n_mesh_nodes, info.steps_done) == (1, 1, 642, 30)
    c.close()


def test_fp64_momentum_budget_and_mass(oif):
    """Stretching and volume forces sum to zero on a closed mesh, so with an
    external force the total momentum grows by steps x (N g + M f_ext)."""
    say("[aux] FP64 diagnostics: momentum budget")
    box = synth.config_sphere_fp64(25)
    t = box.templates[0]
    t.kb = t.kal = t.kag = 0.0
    box.objects[0].fext = (3e-6, -1e-6, 2e-6)
    c = oif.Context.from_box(box, precision="fp64")
    d0 = c.diagnostics()
    c.step(25)
    d1 = c.diagnostics()
    P0 = np.array(d0.momentum_fluid) + np.array(d0.momentum_mesh)
    P1 = np.array(d1.momentum_fluid) + np.array(d1.momentum_mesh)
    want = 25 * (box.n_nodes * np.array(box.g) + box.n_mesh_nodes * np.array(box.objects[0].fext))
    assert np.abs((P1 - P0) - want).max() < 1e-12 * np.abs(want).max() + 1e-15
    assert d1.mass == pytest.approx(box.n_nodes * box.rho0, rel=1e-14)
    assert d1.nonfinite == 0 and d1.clamped == 0 and d1.overflow == 0
    c.close()


def test_watchdog_nonfinite_population(oif):
    say("[aux] watchdog: NaN written from the host")
    box = synth.Box(16, 8, 8)
    c = oif.Context.from_box(box, precision="fp32")
    n = c.read_populations()
    n[3, 2, 1, 5] = np.nan
    c.write_populations(n)
    with pytest.raises(oif.OifError) as ei:
        c.step(1)
    assert ei.value.code == oif.E_NONFINITE
    c.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_watchdog_fixed_point_overflow(oif, prec):
    """A spread force beyond the fixed-point range: 2^55 units of
    2^-fixed_point_exp in the FP32 forms, 2^25 in the FP64 form (room for sums
    of 256 such values; a huge external force gives the mesh a huge velocity
    in step 1, the drag of step 2 overflows)."""
    say(f"[aux] watchdog: fixed-point range, {prec}")
    box = synth.config_sphere_fp64(2)
    if prec == "fp32":
        box.objects[0].fext = (1e6, 0.0, 0.0)
        c = oif.Context.from_box(box, precision="fp32", fixed_point_exp=56)
    else:
        box.objects[0].fext = (2e6, 0.0, 0.0)
        box.friction = 1e5
        c = oif.Context.from_box(box, precision="fp64")
    c.step(1)
    with pytest.raises(oif.OifError) as ei:
        c.step(1)
    assert ei.value.code == oif.E_OVERFLOW
    c.close()


def test_input_validation(oif):
    say("[aux] validation of templates and objects")
    x, t = synth.icosphere(2, 3.0)
    c = oif.Context(16, 16, 16, precision="fp32")
    with pytest.raises(oif.OifError) as ei:
        c.template_create(0, x, t[:, [0, 2, 1]], ks=0.1)   # outward normals
    assert ei.value.code == oif.E_MESH
    with pytest.raises(oif.OifError) as ei:
        c.template_create(1, x, t, ks=0.1)                 # ids start at 0
    assert ei.value.code == oif.E_ID
    with pytest.raises(oif.OifError) as ei:
        c.template_create(0, x, t[:-1], ks=0.1)           # open mesh
    assert ei.value.code == oif.E_MESH
    with pytest.raises(oif.OifError) as ei:
        c.template_create(0, x, t, ks=0.1, model=5)       # unknown force model
    assert ei.value.code == oif.E_ARG
    c.template_create(0, x, t, ks=0.1, stretch=(1.0, 1.0, 1.5))
    with pytest.raises(oif.OifError) as ei:
        c.object_add(1, 0, (8, 8, 8))
    assert ei.value.code == oif.E_ID
    c.object_add(0, 0, (8, 8, 8), rot=oif.euler_to_rot(0.3, 0.2, 0.1), mass=2.0)
    with pytest.raises(oif.OifError) as ei:
        c.template_create(1, x, t, ks=0.1)                 # after objects exist
    assert ei.value.code == oif.E_STATE
    # stretched template: relaxed volume scales by 1.5; object placement keeps it
    a = c.object_analyze(0)
    import oracle
    _, _, V0 = oracle.geometry(x, t)
    assert a.volume == pytest.approx(1.5 * V0, rel=1e-12)
    assert np.allclose(a.origin, 8.0, atol=1e-12)
    c.object_set_origin(0, (5.0, 6.0, 7.0))
    assert np.allclose(c.object_analyze(0).origin, (5, 6, 7), atol=1e-12)
    # refused arguments leave the state as it was
    for bad in ((np.nan, 0.0, 0.0), (0.0, 2e6, 0.0)):
        with pytest.raises(oif.OifError) as ei:
            c.object_set_origin(0, bad)
        assert ei.value.code == oif.E_ARG
    with pytest.raises(oif.OifError) as ei:
        c.object_set_origin(1, (5.0, 6.0, 7.0))
    assert ei.value.code == oif.E_ARG
    Xb = c.read_mesh(0)[0]
    Xbad = Xb.copy()
    Xbad[3, 1] = np.inf
    with pytest.raises(oif.OifError) as ei:
        c.object_set_nodes(0, Xbad)
    assert ei.value.code == oif.E_ARG
    assert np.array_equal(c.read_mesh(0)[0], Xb)
    assert np.allclose(c.object_analyze(0).origin, (5, 6, 7), atol=1e-12)
    with pytest.raises(oif.OifError) as ei:
        c.object_set_force(0, (0.0, np.inf, 0.0))
    assert ei.value.code == oif.E_ARG
    with pytest.raises(oif.OifError) as ei:
        c.step(-1)
    assert ei.value.code == oif.E_ARG
    c.step(0)
    assert c.info().steps_done == 0
    # launch shapes: lattice blocks are powers of two, membrane blocks multiples of 64
    for lb, mb in ((100, -1), (2048, -1), (-1, 100), (-1, 1088), (-1, 32)):
        with pytest.raises(oif.OifError) as ei:
            c.set_launch(lb, mb, -1)
        assert ei.value.code == oif.E_ARG
    c.set_launch(-1, 640, -1)
    assert c.info().mesh_block == 640
    c.step(2)
    c.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_set_nodes_and_density_vs_oracle(oif, orc, prec):
    """oif_object_set_nodes (absolute positions of one object's nodes; here the
    third of four cells, so the node offset of an object counts) and
    oif_read_density, against the oracle: FP64 channel from random populations
    with that cell's nodes displaced, 5 steps; the density compared as a field
    of its own (rho - rho0, at the deviations' bar)."""
    say(f"[aux] object_set_nodes + read_density vs oracle ({prec})")
    box = synth.config_channel_rbc(5, n_cells=4)
    s = orc.System(box)
    rng = np.random.default_rng(71)
    s.n[:] = synth.random_populations(rng, box, amp=1e-3)
    nvs = [len(box.templates[o.tid].nodes) for o in box.objects]
    a = sum(nvs[:2])
    Xn = s.X[a:a + nvs[2]] + 0.05 * rng.standard_normal((nvs[2], 3))
    s.X[a:a + nvs[2]] = Xn
    c = oif.Context.from_box(box, precision=prec)
    c.write_populations(s.n)
    c.object_set_nodes(2, Xn)
    X2, _ = c.read_mesh(2)
    assert np.abs(X2 - Xn).max() <= 4 * np.finfo(float).eps * box.nx
    X0 = s.X.copy()
    c.step(5)
    s.run(5)
    g, o = gpu_fields(c, box.rho0, X0), oracle_fields(s, X0)
    g["drho"] = c.read_density() - box.rho0
    o["drho"] = s.fields()["rho"] - box.rho0
    c.close()
    res = check(g, o, prec, box.rho0, box.nx, keys=("delta", "u", "dX", "V", "drho"))
    say(f"   {fmt(res)}")
    assert set(res) == {"delta", "u", "dX", "V", "drho"}
    assert all(v[3] for v in res.values()), fmt(res)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_zero_friction_decouples(oif, orc, prec):
    """xi = 0 switches the coupling off (eq. dragforce with a zero
    coefficient): the fluid evolves bit for bit as the same box without
    objects, while the deformed, moving cells follow their elastic forces
    alone, as in the oracle.  Channel, random start, 10 steps."""
    say(f"[aux] zero friction decouples fluid and cells ({prec})")
    box = dataclasses.replace(synth.config_channel_rbc(10, n_cells=4), friction=0.0)
    rng = np.random.default_rng(73)
    s = orc.System(box)
    n0 = synth.random_populations(rng, box, amp=1e-3)
    s.n[:] = n0
    s.X += 0.02 * rng.standard_normal(s.X.shape)
    s.V[:] = 1e-4 * rng.standard_normal(s.X.shape)
    X0 = s.X.copy()
    c = oif.Context.from_box(box, precision=prec)
    c.write_populations(n0)
    c.write_mesh(-1, s.X, s.V)
    bare = oif.Context.from_box(dataclasses.replace(box, objects=[]), precision=prec)
    bare.write_populations(n0)
    c.step(10)
    bare.step(10)
    s.run(10)
    assert np.array_equal(c.read_deviations(), bare.read_deviations()), "the cells moved the fluid"
    g, o = gpu_fields(c, box.rho0, X0), oracle_fields(s, X0)
    c.close()
    bare.close()
    res = check(g, o, prec, box.rho0, box.nx)
    say(f"   {fmt(res)}")
    assert all(v[3] for v in res.values()), fmt(res)
    assert np.abs(o["dX"]).max() > 1e-3  # the cells did move


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_template_options_vs_oracle(oif, orc, prec):
    """Template and object options against the oracle, one cell each: the
    linear stretching law alone; bending and local area without stretching,
    on a template stretched by (1.2, 1, 0.8) (relaxed values taken after the
    stretch); global area and volume alone (no edge forces at all); no moduli
    (a passive cell, drag only).  Masses 1, 2, 0.5, 3, an external force on
    the second and fourth cell, rotated placements, deformed moving start,
    random populations, 20 steps."""
    say(f"[aux] template options vs oracle ({prec})")
    x, t = synth.icosphere(2, 3.0)
    tms = [synth.Template(x, t, ks=0.1, linear=True),
           synth.Template(x, t, kb=0.03, kal=0.1, stretch=(1.2, 1.0, 0.8)),
           synth.Template(x, t, kag=0.4, kv=1.0),
           synth.Template(x, t)]
    centres = [(8.0, 8.0, 8.0), (24.0, 8.5, 8.0), (8.5, 24.0, 24.0), (24.0, 24.0, 15.5)]
    masses = [1.0, 2.0, 0.5, 3.0]
    rng = np.random.default_rng(79)
    fext = [(0.0, 0.0, 0.0), (2e-5, -1e-5, 5e-6), (0.0, 0.0, 0.0), (-1e-5, 0.0, 3e-5)]
    objs = [synth.ObjectSpec(k, np.array(c), synth.random_rotation(rng), m, f)
            for k, (c, m, f) in enumerate(zip(centres, masses, fext))]
    box = synth.Box(32, 32, 32, templates=tms, objects=objs, steps=20, name="template_options")
    s = orc.System(box)
    s.n[:] = synth.random_populations(rng, box, amp=1e-3)
    s.X += 0.02 * rng.standard_normal(s.X.shape)
    s.V[:] = 1e-4 * rng.standard_normal(s.X.shape)
    X0 = s.X.copy()
    c = oif.Context.from_box(box, precision=prec)
    c.write_populations(s.n)
    c.write_mesh(-1, s.X, s.V)
    c.step(20)
    s.run(20)
    res = check(gpu_fields(c, box.rho0, X0), oracle_fields(s, X0), prec, box.rho0, box.nx)
    c.close()
    say(f"   {fmt(res)}")
    assert all(v[3] for v in res.values()), fmt(res)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("path", ["compact", "per-corner"])
def test_stencils_clamped_at_walls_vs_oracle(oif, orc, prec, path):
    """A cell whose lowest nodes lie below the first node centre of a z wall
    (z < 1/2): their stencils reach past the wall and are clamped to the
    first fluid layer, on both sides the same way (both z corners then take
    the layer k = 0), and the diagnostics report it.  Compact numbering of the
    stencil box, and the per-corner path (one node pulled far out of the cell
    makes the box too large; two steps, as that node snaps back fast).
    Channel 32x24x16, 5 steps."""
    say(f"[aux] stencils clamped at a z wall vs oracle ({prec}, {path})")
    x, t = synth.icosphere(2, 3.0)
    tm = synth.Template(x, t, **synth.MODULI_DEFAULT)
    box = synth.Box(32, 24, 16, walls_z=True, templates=[tm],
                    objects=[synth.ObjectSpec(0, np.array([12.0, 12.0, 3.2]))], steps=5, name="wall_contact")
    s = orc.System(box)
    rng = np.random.default_rng(83)
    s.n[:] = synth.random_populations(rng, box, amp=1e-3)
    if path == "per-corner":
        s.X[int(np.argmax(s.X[:, 2])), 0] += 16.0
    assert s.X[:, 2].min() < 0.5
    X0 = s.X.copy()
    c = oif.Context.from_box(box, precision=prec)
    c.write_populations(s.n)
    c.write_mesh(-1, s.X, s.V)
    steps = 5 if path == "compact" else 2
    c.step(steps)
    s.run(steps)
    d = c.diagnostics()
    res = check(gpu_fields(c, box.rho0, X0), oracle_fields(s, X0), prec, box.rho0, box.nx)
    c.close()
    say(f"   clamped={d.clamped}; {fmt(res)}")
    assert d.clamped == 1 and d.nonfinite == 0 and d.overflow == 0
    assert all(v[3] for v in res.values()), fmt(res)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("path", ["compact", "per-corner"])
def test_cell_across_periodic_corner_vs_oracle(oif, orc, prec, path):
    """A cell centred on a corner of the periodic box, so that its stencils
    wrap in x, y and z at once (unwrapped positions on both sides of a
    periodic face on every axis); compact stencil box and per-corner path (one node
    pulled out of the cell).  24x20x16, random start, 5 / 2 steps."""
    say(f"[aux] cell across the periodic corner vs oracle ({prec}, {path})")
    x, t = synth.icosphere(2, 3.0)
    tm = synth.Template(x, t, **synth.MODULI_DEFAULT)
    box = synth.Box(24, 20, 16, templates=[tm], objects=[synth.ObjectSpec(0, np.array([0.3, 19.8, 0.1]))],
                    steps=5, name="periodic_corner")
    s = orc.System(box)
    rng = np.random.default_rng(89)
    s.n[:] = synth.random_populations(rng, box, amp=1e-3)
    s.V[:] = 1e-4 * rng.standard_normal(s.X.shape)
    if path == "per-corner":
        s.X[int(np.argmax(s.X[:, 0])), 0] += 16.0
    lo, hi = s.X.min(axis=0), s.X.max(axis=0)
    assert lo[0] < 0 < hi[0] and lo[1] < box.ny < hi[1] and lo[2] < 0 < hi[2]
    X0 = s.X.copy()
    c = oif.Context.from_box(box, precision=prec)
    c.write_populations(s.n)
    c.write_mesh(-1, s.X, s.V)
    steps = 5 if path == "compact" else 2
    c.step(steps)
    s.run(steps)
    res = check(gpu_fields(c, box.rho0, X0), oracle_fields(s, X0), prec, box.rho0, box.nx)
    c.close()
    say(f"   {fmt(res)}")
    assert all(v[3] for v in res.values()), fmt(res)


def test_readme_c_example_runs(oif, tmp_path):
    """The C example of README.md, built with gcc against the C ABI alone:
    100 steps of one octahedral cell in a fluid driven along x; it exits 0 and
    the cell has been carried along +x."""
    import subprocess
    from example_util import build_readme_example
    say("[aux] README C example")
    exe = build_readme_example(tmp_path)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    say("   " + r.stdout.strip() + r.stderr.strip())
    assert r.returncode == 0, r.stderr
    m = re.search(r"node 0 at \(([-0-9.]+), ([-0-9.]+), ([-0-9.]+)\), moving at ([-0-9.e+]+) along x", r.stdout)
    assert m, r.stdout
    x0, v0 = float(m.group(1)), float(m.group(4))
    assert 19.0 < x0 < 19.5 and v0 > 0.0


def test_readme_python_example_runs(oif):
    """The Python example of README.md runs in a child process and prints a
    rate, the kernel times and finite fields."""
    import subprocess
    import sys
    from example_util import ROOT, readme_python_example
    say("[aux] README Python example")
    r = subprocess.run([sys.executable, "-c", readme_python_example()], capture_output=True, text=True,
                       timeout=300, cwd=ROOT, env=dict(os.environ, PYTHONPATH=ROOT))
    say("   " + r.stdout.strip().replace("\n", " | ") + r.stderr[-2000:])
    assert r.returncode == 0, r.stderr[-2000:]
    assert re.search(r"^\d+ MLUPS$", r.stdout, re.M) and "lattice kernel" in r.stdout and "max |u|" in r.stdout


@pytest.mark.parametrize("mb", [192, 640, 768])
def test_membrane_block_sizes_match_oracle(oif, orc, mb):
    """Membrane workgroups of any multiple of 64 (not only powers of two) give
    the oracle's result: FP32 channel, 20 steps."""
    say(f"[modes] membrane block {mb} vs oracle")
    box = channel(20)
    s = orc.System(box)
    X0 = s.X.copy()
    c = oif.Context.from_box(box, precision="fp32")
    c.set_launch(-1, mb, -1)
    c.step(20)
    s.run(20)
    res = check(gpu_fields(c, box.rho0, X0), oracle_fields(s, X0), "fp32", box.rho0, box.nx)
    c.close()
    say(f"   {fmt(res)}")
    assert all(v[3] for v in res.values()), fmt(res)


@pytest.mark.parametrize("prec,chunk,meshes", [("fp32", 0, "lds"), ("fp64", 0, "lds"), ("fp32", 1, "lds"),
                                               ("fp32", 3, "lds"), ("fp32", 0, "all"), ("fp64", 0, "all")])
def test_persistent_batch_matches_launch_pairs(oif, prec, chunk, meshes):
    """The persistent form of a batch (one launch per step, device task list,
    per-box waits) against the launch-per-phase form, eagerly, under graph
    capture, and from either step parity; lattice tasks of one block, of the
    default count, and of three blocks (a box's last task then runs past its
    nodes).  With the 162- and 642-node spheres of the batching case only (all
    meshes in LDS) the results agree bit for bit (fixed-point spreading in
    every form).  With its 2562-node
    spheres as well, which the launch-per-phase form splits over several
    workgroups and the persistent form runs whole (coupling area in LDS), the
    area and volume sums are rounded in another order, so the two agree to the
    parity tolerance."""
    say(f"[modes] persistent batch vs launch pairs, {prec}, lattice blocks per task {chunk}, meshes {meshes}")
    boxes = synth.config_batch(n_boxes=6, steps=12)
    if meshes == "lds":
        boxes = [dataclasses.replace(b, objects=[o for o in b.objects if o.tid < 2]) for b in boxes]
    ref, got = [], []
    for persistent, out in ((False, ref), (True, got)):
        ctxs = [oif.Context.from_box(bx, precision=prec) for bx in boxes]
        ctxs[0].step(1)  # the batch then starts at odd parity in every box
        for c in ctxs[1:]:
            c.step(1)
        if not persistent and meshes == "all":
            assert sum(c.info().split_objects for c in ctxs) > 0
        B = oif.Batch(ctxs)
        B.set_persistent(persistent, chunk)
        B.step(3)
        B.set_graph(4)
        B.step(8)
        for c in ctxs:
            X, V = c.read_mesh(-1)
            out.append((c.read_deviations(), X, V))
        B.close()
        for c in ctxs:
            c.close()
    rtol = 1e-5 if prec == "fp32" else 1e-12
    for bx, (d0, X0, V0), (d1, X1, V1) in zip(boxes, ref, got):
        if meshes == "all":
            # the parity criterion's relative bar and absolute floors (box length
            # for the mesh fields)
            L = max(bx.nx, bx.ny, bx.nz)
            for a, b, floor in ((d0, d1, ATOL["delta"] * bx.rho0), (X0, X1, ATOL["dX"] * L),
                                (V0, V1, ATOL["V"] * L)):
                if a.size:
                    assert np.abs(a - b).max() <= rtol * np.abs(a).max() + floor
        else:
            assert np.array_equal(d0, d1) and np.array_equal(X0, X1) and np.array_equal(V0, V1)


def test_persistent_batch_refuses_obstacles_and_mrt(oif):
    say("[modes] persistent batch: unsupported boxes")
    for case in ("obstacles", "mrt"):
        box = synth.config_obstacle_channel(4) if case == "obstacles" else synth.config_batch(n_boxes=1, steps=4)[0]
        if case == "mrt":
            box.mrt = (0.0, -0.5, 0.3, -0.3)
        c = oif.Context.from_box(box, precision="fp32")
        B = oif.Batch([c])
        B.set_persistent(True)
        with pytest.raises(oif.OifError) as e:
            B.step(1)
        assert e.value.code == oif.E_UNSUPPORTED
        B.set_persistent(False)
        B.step(1)
        B.close()
        c.close()
