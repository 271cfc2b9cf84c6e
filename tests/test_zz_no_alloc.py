"""oif_diagnostics_noalloc, the allocation-free variant of oif_diagnostics
(partial sums in a fixed per-device array), through the C ABI: the same sums
bit for bit as oif_diagnostics, on two calls in a row, the second on a
smaller input (fewer objects, a smaller box, another precision) while the
array still holds the first call's partials; and its two refusals."""
import numpy as np
import pytest

from paper_1312_3426_amd import synth

from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def oif():
    from paper_1312_3426_amd import oif as m
    m.lib()
    return m


def as_tuple(d):
    return (d.mass, tuple(d.momentum_fluid), tuple(d.momentum_mesh), d.nonfinite, d.clamped, d.overflow)


def test_noalloc_diagnostics_match_twice_second_smaller(oif):
    say("[noalloc] diagnostics: channel (10 cells, fp32), then 20^3 sphere (1 cell, fp64)")
    big = oif.Context.from_box(synth.config_channel_rbc(6), precision="fp32")
    big.step(6)
    small = oif.Context.from_box(synth.config_sphere_fp64(4), precision="fp64")
    small.step(4)
    for c, n in ((big, 10), (small, 1)):
        got = as_tuple(c.diagnostics_noalloc())
        ref = as_tuple(c.diagnostics())
        say(f"   {n} objects: mass {got[0]:.17g}, momentum {got[1]}, {got[2]}")
        assert got == ref
        assert np.isfinite(got[0]) and got[3] == 0
    # once more on the larger input after the smaller one
    assert as_tuple(big.diagnostics_noalloc()) == as_tuple(big.diagnostics())
    big.close()
    small.close()


def test_noalloc_diagnostics_refusals(oif):
    say("[noalloc] refusals: changed mesh, too many objects")
    c = oif.Context.from_box(synth.config_sphere_fp64(2), precision="fp64")
    c.step(1)
    X, _ = c.read_mesh(-1)
    c.write_mesh(-1, X + 0.01, None)  # the device arrays must be rebuilt by a step
    with pytest.raises(oif.OifError) as e:
        c.diagnostics_noalloc()
    assert e.value.code == oif.E_STATE
    c.step(1)
    c.diagnostics_noalloc()
    c.close()
    # 25953 objects: one more than the fixed array holds partials for
    n, t = synth.tetrahedron(0.8)
    box = synth.Box(96, 96, 96, templates=[synth.Template(n, t)], g=(0.0, 0.0, 0.0))
    k = np.arange(25953)
    centres = np.stack([k % 96, (k // 96) % 96, 10 + 8 * (k // 9216)], axis=1) + 0.5
    box.objects = [synth.ObjectSpec(0, ctr) for ctr in centres]
    c = oif.Context.from_box(box, precision="fp32")
    c.step(1)
    with pytest.raises(oif.OifError) as e:
        c.diagnostics_noalloc()
    assert e.value.code == oif.E_ARG and "25952" in str(e.value)
    c.close()
