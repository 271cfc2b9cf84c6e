"""Helpers shared by the GPU parity tests: run a workload on the HIP path and
on the oracle from the same seeded inputs, and compare fields.

Parity criterion per field f (populations as deviations n_i - w_i rho0,
velocity u, displacement X - X0, mesh velocity V):

    max |gpu - oracle| <= RTOL * max |oracle| + ATOL * scale_f

RTOL is 1e-12 (FP64 form) or 1e-5 (FP32 form).  The absolute term is the
round-off floor of the FP64 representation both sides share: the oracle stores
full populations (~rho0, ulp 5.6e-17) and both store absolute positions
(~box length L, ulp ~2.2e-16 L), so deviations that are tiny next to those
carry a few ulps of representation error that no implementation can remove.
scale_f = rho0 for populations, 1 (lattice units) for velocities, the box
length for positions and mesh velocities (the elastic forces turn the
positions' round-off into velocity differences of the same size).  ATOL is
about four times the largest such floor measured over the GPU parity tests
(|gpu - oracle| / scale_f where the relative bar alone would not hold):
deviations 2.2e-15, fluid velocity 2.2e-15, displacement 5.3e-16 L, mesh
velocity 6.2e-16 L; the density's deviation rho - rho0 (a sum of 19
deviations) takes the deviations' floor.  The FP32 form shares these floors: its positions are
FP64 as well, and the relative bar covers everything above them.
"""
import json
import os
import sys

import numpy as np

W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
RTOL = {"fp64": 1e-12, "fp32": 1e-5}
ATOL = {"delta": 1e-14, "u": 1e-14, "dX": 2.5e-15, "V": 2.5e-15, "drho": 1e-14}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    """max |a - b| / max |b| (0 if both vanish)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max() if b.size else 0.0
    num = np.abs(a - b).max() if a.size else 0.0
    if den == 0.0:
        return num
    return num / den


def gpu_fields(ctx, rho0, X0=None):
    n = ctx.read_populations()
    X, V = ctx.read_mesh(-1)
    out = dict(delta=n - (W * rho0)[:, None, None, None], u=ctx.read_velocity(), X=X, V=V)
    if X0 is not None:
        out["dX"] = X - X0
    return out


def oracle_fields(sys_, X0=None):
    f = sys_.fields()
    out = dict(delta=f["delta"], u=f["u"], X=f["X"], V=f["V"])
    if X0 is not None:
        out["dX"] = f["X"] - X0
    return out


def compare(g, o, keys=("delta", "u", "dX", "V")):
    return {k: rel(g[k], o[k]) for k in keys if k in g and k in o and o[k].size}


def check(g, o, prec, rho0, box_len, keys=("delta", "u", "dX", "V")):
    """Apply the parity criterion; returns {field: (abs_err, ref_max, bound, ok)}."""
    # mesh velocities inherit the positions' representation floor (~1e-16 of
    # the box length) through the elastic forces, so both take the box length
    scale = {"delta": rho0, "drho": rho0, "u": 1.0, "dX": box_len, "V": box_len}
    out = {}
    for k in keys:
        if k not in g or k not in o or not o[k].size:
            continue
        err = float(np.abs(np.asarray(g[k]) - np.asarray(o[k])).max())
        ref = float(np.abs(o[k]).max())
        bound = RTOL[prec] * ref + ATOL[k] * scale[k]
        out[k] = (err, ref, bound, err <= bound)
    log = os.environ.get("OIF_PARITY_LOG")
    if log:  # measured errors, for the record of the absolute floors
        with open(log, "a") as fh:
            for k, (err, ref, bound, ok) in out.items():
                fh.write(json.dumps({"test": os.environ.get("PYTEST_CURRENT_TEST", ""), "prec": prec,
                                     "field": k, "err": err, "ref": ref, "scale": scale[k],
                                     "ok": ok}) + "\n")
    return out


def fmt(res):
    return ", ".join(f"{k}: {e:.2e}/{r:.2e} (rel {e / r if r else 0:.1e}) {'ok' if ok else 'FAIL'}"
                     for k, (e, r, b, ok) in res.items())
