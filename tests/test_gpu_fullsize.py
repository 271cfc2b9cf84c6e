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
def test_scale_case_full_size_fp64(oif, orc, tmp_path):
    """The same box in the FP64 form: each population buffer holds 19 x 33.5 M
    doubles (5.1 GB), so every population address lies beyond 32-bit byte
    offsets somewhere; one step against the oracle at the FP64 bar."""
    box = synth.config_scale(1)
    g, o = run_case(oif, orc, box, "fp64", 1, 59, str(tmp_path / "t.json"))
    res = check(g, o, "fp64", box.rho0, box.nx)
    say(f"   {fmt(res)}")
    assert all(v[3] for v in res.values()), fmt(res)
