"""The C-ABI library loads and exports every entry point include/oif.h
declares; host-only calls behave as documented.  No compute calls (no GPU)."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "oif.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(oif_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def oiflib():
    from paper_1312_3426_amd import oif
    return oif


def test_library_exports_every_declared_symbol(oiflib):
    L = oiflib.lib()
    names = declared_symbols()
    assert len(names) >= 30
    for n in names:
        assert hasattr(L, n), n
    # and the binding declares a signature for each of them
    assert set(names) == set(oiflib.SIGNATURES)


def test_library_exports_nothing_else(oiflib):
    """The dynamic symbol table holds the declared calls and no internal
    symbol (hidden visibility, version script)."""
    import shutil
    import subprocess
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm not available")
    out = subprocess.run([nm, "-D", "--defined-only", oiflib.lib()._name], capture_output=True, text=True,
                         check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    assert exported == set(declared_symbols()), sorted(exported ^ set(declared_symbols()))[:10]


def test_readme_c_example_compiles_and_links(oiflib, tmp_path):
    """The C example of README.md builds against oif.h and links liboif.so
    (it runs in the GPU tests)."""
    from example_util import build_readme_example
    oiflib.lib()
    try:
        exe = build_readme_example(tmp_path)
    except FileNotFoundError:
        pytest.skip("gcc not available")
    assert os.path.exists(exe)


def test_desc_defaults(oiflib):
    d = oiflib.LatticeDesc()
    assert oiflib.lib().oif_lattice_desc_init(C.byref(d)) == 0
    assert (d.tau, d.rho0, d.precision, d.fp16_scale_exp, d.fixed_point_exp) == (1.0, 1.0, 1, 12, 40)
    assert oiflib.lib().oif_lattice_desc_init(None) == oiflib.E_ARG


def test_euler_rotation_order(oiflib):
    rx, ry, rz = 0.3, -1.1, 2.2
    R = oiflib.euler_to_rot(rx, ry, rz)
    Rx = np.array([[1, 0, 0], [0, math.cos(rx), -math.sin(rx)], [0, math.sin(rx), math.cos(rx)]])
    Ry = np.array([[math.cos(ry), 0, math.sin(ry)], [0, 1, 0], [-math.sin(ry), 0, math.cos(ry)]])
    Rz = np.array([[math.cos(rz), -math.sin(rz), 0], [math.sin(rz), math.cos(rz), 0], [0, 0, 1]])
    assert np.allclose(R, Rz @ Ry @ Rx, atol=1e-15)
    assert np.allclose(R @ R.T, np.eye(3), atol=1e-15)


@pytest.mark.parametrize("field,value", [("nx", 0), ("tau", 0.5), ("rho0", -1.0), ("precision", 7),
                                         ("fixed_point_exp", 60), ("friction", float("nan"))])
def test_create_rejects_bad_desc(oiflib, field, value):
    d = oiflib.LatticeDesc()
    oiflib.lib().oif_lattice_desc_init(C.byref(d))
    d.nx = d.ny = d.nz = 4
    setattr(d, field, value)
    h = C.c_void_p()
    assert oiflib.lib().oif_create(C.byref(d), C.byref(h)) == oiflib.E_ARG
    assert not h.value


def test_product_does_not_import_oracle():
    """The product package never reaches into the oracle (and vice versa)."""
    pkg = os.path.join(ROOT, "paper_1312_3426_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "oif_oracle" not in txt, f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".py", ".c", ".h")):
            txt = open(os.path.join(ROOT, "oracle", f)).read()
            assert "import paper_1312_3426_amd" not in txt and "from paper_1312_3426_amd" not in txt, f
            assert "oif_device" not in txt and "kernels.hip" not in txt, f


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits with a message and
    status 2 before touching any device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
