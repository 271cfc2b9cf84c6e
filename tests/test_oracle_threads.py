"""The oracle's OpenMP build (lattice sweeps over several host threads, used
for the all-core CPU baseline and for long reference runs) gives the serial
build's results bit for bit (no GPU)."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys, numpy as np
sys.path.insert(0, {root!r})
import oracle
from paper_1312_3426_amd import synth
oracle.threads({threads})
b = synth.config_channel_rbc(3, n_cells=3)
b.objects[0].fext = (1e-6, 0.0, -2e-6)
s = oracle.System(b)
s.n[:] = synth.random_populations(np.random.default_rng(5), b, amp=1e-3)
s.run(3)
np.savez({out!r}, n=s.n, X=s.X, V=s.V, t=oracle.threads())
"""


def run(tmp_path, openmp, threads):
    out = str(tmp_path / f"r{int(openmp)}.npz")
    env = dict(os.environ, OIF_ORACLE_OPENMP="1" if openmp else "0", PYTHONPATH=ROOT)
    env.pop("OIF_ORACLE_LIB", None)
    subprocess.run([sys.executable, "-c", SCRIPT.format(root=ROOT, threads=threads, out=out)], env=env,
                   check=True, timeout=300)
    return np.load(out)


def test_openmp_build_matches_serial_bitwise(orc, tmp_path):
    a = run(tmp_path, False, 0)
    b = run(tmp_path, True, 4)
    assert int(a["t"]) == 1 and int(b["t"]) == 4
    for k in ("n", "X", "V"):
        assert np.array_equal(a[k], b[k]), k
