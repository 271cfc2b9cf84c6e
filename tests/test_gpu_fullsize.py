"""Full-size parity: the workloads bench.py times, at their full sizes and in
the autotuned launch configuration, against the FP64 oracle on the same
seeded inputs (random near-rest populations, randomly deformed moving meshes)
for a few steps.  Every field is compared, not a sample: one oracle step of
the 4.2 M-node case takes ~2 s on the host, of the 33.5 M-node case ~20 s."""
import numpy as np
import pytest

from paper_1312_3426_amd import synth

from gpu_util import check, fmt, gpu_fields, oracle_fields, rel, say

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


def seeded_start(box, orc, seed):
    """Oracle system with random populations and perturbed, moving meshes."""
    rng = np.random.default_rng(seed)
    s = orc.System(box)
    s.n[:] = synth.random_populations(rng, box, amp=1e-3)
    s.X += 0.01 * rng.standard_normal(s.X.shape)
    s.V[:] = 1e-4 * rng.standard_normal(s.X.shape)
    return s


def run_case(oif, orc, box, prec, steps, seed, tune_path):
    say(f"[fullsize] {box.name} {prec}: N={box.n_nodes} M={box.n_mesh_nodes}, {steps} steps")
    s = seeded_start(box, orc, seed)
    X0 = s.X.copy()
    c = oif.Context.from_box(box, precision=prec)
    c.write_populations(s.n)
    c.write_mesh(-1, s.X, s.V)
    c.autotune(tune_path)
    i = c.info()
    say(f"   launch: lb_block={i.lb_block} mesh_block={i.mesh_block} remap={i.xcd_remap} "
        f"lds_objects={i.lds_objects}/{i.n_objects}")
    c.step(steps)
    s.run(steps)
    g, o = gpu_fields(c, box.rho0, X0), oracle_fields(s, X0)
    c.close()
    return g, o


def test_precision_case_full_size_fp32(oif, orc, tmp_path):
    box = synth.config_precision(2)
    g, o = run_case(oif, orc, box, "fp32", 2, 31, str(tmp_path / "t.json"))
    res = check(g, o, "fp32", box.rho0, box.nx)
    say(f"   {fmt(res)}")
    assert all(v[3] for v in res.values()), fmt(res)


def test_precision_case_full_size_fp16(oif, orc, tmp_path):
    """FP16 storage (deviations x 2^12): velocity within 1e-3 of max|u| after
    two steps from the random start (each step rounds every stored deviation)."""
    box = synth.config_precision(2)
    g, o = run_case(oif, orc, box, "fp16", 2, 31, str(tmp_path / "t.json"))
    e = {k: rel(g[k], o[k]) for k in ("delta", "u", "dX", "V")}
    say("   " + ", ".join(f"{a}={b:.2e}" for a, b in e.items()))
    assert e["u"] < 1e-3 and e["delta"] < 1e-3


@pytest.mark.timeout(600)
def test_scale_case_full_size_fp32(oif, orc, tmp_path):
    """512x256x256 box, 5000 biconcave cells of 642 nodes, one step."""
    box = synth.config_scale(1)
    g, o = run_case(oif, orc, box, "fp32", 1, 53, str(tmp_path / "t.json"))
    res = check(g, o, "fp32", box.rho0, box.nx)
    say(f"   {fmt(res)}")
    assert all(v[3] for v in res.values()), fmt(res)


@pytest.mark.timeout(600)
def test_scale_slab_full_size_fp32(oif, orc, tmp_path):
    """One GPU's share of the scale case split into eight x-slabs: the slab
    with the most cells (64x256x256, periodic in x), as timed, two steps."""
    share = max((synth.config_scale_share(8, k, 2) for k in range(8)), key=lambda b: len(b.objects))
    g, o = run_case(oif, orc, share, "fp32", 2, 67, str(tmp_path / "t.json"))
    res = check(g, o, "fp32", share.rho0, max(share.nx, share.ny, share.nz))
    say(f"   {fmt(res)}")
    assert all(v[3] for v in res.values()), fmt(res)


@pytest.mark.timeout(600)
def test_scale_case_full_size_fp64(oif, orc, tmp_path):
    """The same box in the FP64 form: each population buffer holds 19 x 33.5 M
    doubles (5.1 GB), so every population address lies beyond 32-bit byte
    offsets somewhere; one step against the oracle at the FP64 bar."""
    box = synth.config_scale(1)
    g, o = run_case(oif, orc, box, "fp64", 1, 59, str(tmp_path / "t.json"))
    res = check(g, o, "fp64", box.rho0, box.nx)
    say(f"   {fmt(res)}")
    assert all(v[3] for v in res.values()), fmt(res)


@pytest.mark.timeout(600)
def test_scale_case_fp64_momentum_budget_and_mass(oif):
    """512x256x256, 5000 cells, FP64 form, with the stretching and volume
    moduli only (forces that sum to zero over each closed mesh): after three
    steps from rest the fluid's and the meshes' momentum together grew by
    3 N g and the mass is unchanged, in the FP64 sums of the diagnostics over
    33.5 M lattice nodes and 3.2 M mesh nodes."""
    box = synth.config_scale(3)
    t = box.templates[0]
    t.kb = t.kal = t.kag = 0.0
    say(f"[fullsize] {box.name} fp64: momentum budget and mass, 3 steps")
    c = oif.Context.from_box(box, precision="fp64")
    d0 = c.diagnostics()
    c.step(3)
    d1 = c.diagnostics()
    c.close()
    P0 = np.array(d0.momentum_fluid) + np.array(d0.momentum_mesh)
    P1 = np.array(d1.momentum_fluid) + np.array(d1.momentum_mesh)
    want = 3 * box.n_nodes * np.array(box.g)
    err = np.abs((P1 - P0) - want).max()
    say(f"   momentum change {P1 - P0} against {want}: error {err:.2e}; mesh momentum {np.array(d1.momentum_mesh)}; "
        f"mass {d1.mass!r} against {box.n_nodes * box.rho0!r}")
    assert np.abs(np.array(d1.momentum_mesh)).max() > 0.0  # the fluid has dragged the cells
    assert err <= 1e-12 * np.abs(want).max()
    assert d1.mass == pytest.approx(box.n_nodes * box.rho0, rel=1e-14)
    assert d1.nonfinite == 0 and d1.clamped == 0 and d1.overflow == 0


@pytest.mark.timeout(600)
def test_scale_case_full_size_fp16(oif, orc, tmp_path):
    """512x256x256 box, 5000 cells, FP16 storage of the deviations (x 2^12),
    one step from the random start.  Each stored deviation is rounded once to
    11 significant bits (unit roundoff 2^-11 = 4.9e-4 of its value, the scale
    keeps them clear of the subnormal range): deviations and velocity within
    1e-3 of their maximum, mesh fields at the FP32 bar (the mesh arithmetic is
    FP32 and reads the velocity only through the interpolation, which uses the
    step's starting populations written from the same FP64 start)."""
    box = synth.config_scale(1)
    g, o = run_case(oif, orc, box, "fp16", 1, 61, str(tmp_path / "t.json"))
    e = {k: rel(g[k], o[k]) for k in ("delta", "u", "dX", "V")}
    say("   " + ", ".join(f"{a}={b:.2e}" for a, b in e.items()))
    assert e["u"] < 1e-3 and e["delta"] < 1e-3
    res = check(g, o, "fp32", box.rho0, box.nx, keys=("dX", "V"))
    say(f"   {fmt(res)}")


def test_precision_case_full_size_bf16(oif, orc, tmp_path):
    """256x128x128 box, 500 cells, BF16 storage of the deviations, two steps
    from the random start.  BF16 keeps 8 significant bits (unit roundoff
    2^-9 = 2.0e-3 of a value); two roundings of each stored deviation bound
    the deviations' and the velocity's error by 2 x 2^-9 of their maximum."""
    box = synth.config_precision(2)
    g, o = run_case(oif, orc, box, "bf16", 2, 37, str(tmp_path / "t.json"))
    e = {k: rel(g[k], o[k]) for k in ("delta", "u", "dX", "V")}
    say("   " + ", ".join(f"{a}={b:.2e}" for a, b in e.items()))
    assert e["u"] < 2 * 2.0 ** -9 and e["delta"] < 2 * 2.0 ** -9


@pytest.mark.timeout(900)
def test_batch_case_all_boxes_vs_oracle(oif, orc, tmp_path):
    """The whole batching case (32 boxes, 2.6 M nodes, 1-20 spheres of
    162/642/2562 nodes each) stepped through one batch in its autotuned launch
    configuration, from random starts, against the oracle box by box after 3
    steps, at the FP32 bar."""
    boxes = synth.config_batch(steps=3)
    say(f"[fullsize] batching case: {len(boxes)} boxes, {sum(b.n_nodes for b in boxes)} nodes, "
        f"{sum(b.n_mesh_nodes for b in boxes)} mesh nodes, 3 steps")
    systems, ctxs = [], []
    for k, bx in enumerate(boxes):
        s = seeded_start(bx, orc, 1000 + k)
        c = oif.Context.from_box(bx, precision="fp32")
        c.write_populations(s.n)
        c.write_mesh(-1, s.X, s.V)
        systems.append((s, s.X.copy()))
        ctxs.append(c)
    B = oif.Batch(ctxs)
    B.autotune(str(tmp_path / "t.json"))
    B.step(3)
    worst = {}
    for k, (bx, c, (s, X0)) in enumerate(zip(boxes, ctxs, systems)):
        s.run(3)
        res = check(gpu_fields(c, bx.rho0, X0), oracle_fields(s, X0), "fp32", bx.rho0,
                    max(bx.nx, bx.ny, bx.nz))
        for f, v in res.items():
            r = v[0] / v[1] if v[1] else 0.0
            worst[f] = max(worst.get(f, 0.0), r)
        assert all(v[3] for v in res.values()), f"{bx.name}: {fmt(res)}"
    say("   worst relative error over the 32 boxes: " + ", ".join(f"{f}={v:.2e}" for f, v in worst.items()))
    B.close()
    for c in ctxs:
        c.close()
