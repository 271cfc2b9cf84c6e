"""Pins of the oracle's soft-sphere repulsion (no GPU): the collisions the
paper's scripts switch on between part types and with the channel walls
(Section "Implementation details", the script's inter ... soft-sphere lines),
with the potential a (d - offset)^-n for offset < d < offset + cutoff.

Expected values come from independent code: closed forms for one pair and
for flat walls, a numpy brute-force energy differentiated by central
differences, a bounded numerical minimisation for distances to a sheared
rhomboid, conservation of momentum and angular momentum."""
import numpy as np
import pytest
from scipy.optimize import minimize

from paper_1312_3426_amd import synth


def _tetra_objects(centres, ptypes, rot=None):
    x, t = synth.tetrahedron(1.0)
    tm = synth.Template(x, t)  # no moduli: the nodes are free
    return tm, [synth.ObjectSpec(0, np.asarray(c, float), rot=rot, ptype=p) for c, p in zip(centres, ptypes)]


def _box(objs, tm, rep, n=16, walls=False, bnd=()):
    return synth.Box(n, n, n, g=(0.0, 0.0, 0.0), friction=0.0, walls_z=walls, templates=[tm], objects=objs,
                     repulsion=list(rep), boundaries=list(bnd))


def pair_energy(X, types, rep, box_len, periodic):
    """Brute-force soft-sphere energy of all distinct node pairs."""
    E = 0.0
    for j in range(len(X)):
        for k in range(j + 1, len(X)):
            for r in rep:
                if r.type_b is None or {types[j], types[k]} != {r.type_a, r.type_b}:
                    continue
                dv = X[j] - X[k]
                for c in range(3):
                    if periodic[c]:
                        dv[c] -= box_len[c] * np.floor(dv[c] / box_len[c] + 0.5)
                d = np.linalg.norm(dv) - r.offset
                if 0 < d < r.cutoff:
                    E += r.a * d ** (-r.n)
    return E


def test_single_pair_closed_form(orc):
    """One cross pair inside the range: force a n (d - offset)^-(n+1) along the
    line, equal and opposite; nothing for types without an interaction."""
    tm, objs = _tetra_objects([(5.0, 5.0, 5.0), (5.0, 5.0, 5.0)], [0, 1])
    rep = [synth.SoftSphere(0, 1, a=2e-4, n=1.5, cutoff=0.4, offset=0.05)]
    s = orc.System(_box(objs, tm, rep))
    X = s.X.copy()
    # move object 1 far away, then bring its node 0 next to object 0's node 2
    X[4:] += np.array([4.0, 0.0, 0.0])
    sep = np.array([0.12, -0.2, 0.1])
    X[4] = X[2] + sep
    s.X[:] = X
    F = s.repulsion()
    d = np.linalg.norm(sep)
    f = 2e-4 * 1.5 * (d - 0.05) ** -2.5
    want = np.zeros_like(X)
    want[4] = f * sep / d
    want[2] = -f * sep / d
    # all other cross pairs are out of range (checked), so this is the whole force
    dist = np.linalg.norm(X[:4, None, :] - X[None, 4:, :], axis=2)
    assert (dist < 0.45).sum() == 1
    assert np.abs(F - want).max() < 1e-14 * f
    # one step (no friction, unit mass): the nodes take exactly this force
    s.run(1)
    assert np.abs(s.V - want).max() < 1e-14 * f
    assert np.abs(s.X - (X + want)).max() < 1e-14
    # the same geometry with the pair defined for other types: no force
    rep2 = [synth.SoftSphere(0, 2, a=2e-4, n=1.5, cutoff=0.4, offset=0.05)]
    s2 = orc.System(_box(objs, tm, rep2))
    s2.X[:] = X
    assert np.abs(s2.repulsion()).max() == 0.0


def test_duplicate_settings_last_one_holds(orc):
    """A pair of types set twice (the second time with the types swapped) and
    a type's wall interaction set twice: the later setting replaces the
    earlier one, pinned by the closed form of the later one."""
    tm, objs = _tetra_objects([(5.0, 5.0, 1.0), (5.0, 5.0, 1.0)], [0, 1])
    last = synth.SoftSphere(1, 0, a=2e-4, n=1.5, cutoff=0.4, offset=0.05)
    first = synth.SoftSphere(0, 1, a=9e-4, n=3.0, cutoff=0.45, offset=0.0)
    s = orc.System(_box(objs, tm, [first, last]))
    X = s.X.copy()
    X[4:] += np.array([4.0, 0.0, 3.0])  # object 1 away from object 0 and from the z walls
    sep = np.array([0.12, -0.2, 0.1])
    X[4] = X[2] + sep
    s.X[:] = X
    d = np.linalg.norm(sep)
    f = 2e-4 * 1.5 * (d - 0.05) ** -2.5
    want = np.zeros_like(X)
    want[4] = f * sep / d
    want[2] = -f * sep / d
    dist = np.linalg.norm(X[:4, None, :] - X[None, 4:, :], axis=2)
    assert (dist < 0.46).sum() == 1
    assert np.abs(s.repulsion() - want).max() < 1e-14 * f
    # walls: node 0 of object 0 near z = 0 (the wall at z = 0 sits half a
    # lattice spacing below the first node layer); type 0 set twice
    wfirst = synth.SoftSphere(0, None, a=5e-4, n=2.0, cutoff=1.5)
    wlast = synth.SoftSphere(0, None, a=1e-4, n=1.5, cutoff=1.5)
    sw = orc.System(_box(objs, tm, [wfirst, wlast], walls=True))
    so = orc.System(_box(objs, tm, [wlast], walls=True))
    sw.X[:] = X
    so.X[:] = X
    Fw, Fo = sw.repulsion(), so.repulsion()
    assert np.abs(Fo).max() > 0.0
    assert np.array_equal(Fw, Fo)


def test_pair_forces_are_minus_gradient_and_conserve(orc):
    """Random close packing of three objects (types 0, 1, 0; pairs 0-1 and
    0-0, the latter also inside an object): forces = -grad of the brute-force
    energy (central differences), zero net force and zero net torque."""
    rng = np.random.default_rng(31)
    tm, objs = _tetra_objects([(5.0, 5.0, 5.0), (5.4, 5.3, 5.2), (4.7, 5.5, 5.4)], [0, 1, 0])
    rep = [synth.SoftSphere(0, 1, a=1e-4, n=2.0, cutoff=0.8, offset=0.1),
           synth.SoftSphere(0, 0, a=3e-5, n=1.2, cutoff=0.9, offset=0.0)]
    s = orc.System(_box(objs, tm, rep))
    s.X[:] += 0.1 * rng.standard_normal(s.X.shape)
    X = s.X.copy()
    types = [0] * 4 + [1] * 4 + [0] * 4
    F = s.repulsion()
    L3 = (16.0, 16.0, 16.0)
    per = (True, True, True)
    E0 = pair_energy(X, types, rep, L3, per)
    assert E0 > 0 and np.count_nonzero(np.abs(F).sum(axis=1)) >= 6
    eps = 1e-6
    G = np.zeros_like(X)
    for j in range(len(X)):
        for c in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[j, c] += eps
            Xm[j, c] -= eps
            G[j, c] = -(pair_energy(Xp, types, rep, L3, per) - pair_energy(Xm, types, rep, L3, per)) / (2 * eps)
    assert np.abs(F - G).max() < 1e-7 * np.abs(F).max()
    assert np.abs(F.sum(axis=0)).max() < 1e-16 * np.abs(F).sum()
    torque = np.cross(X, F).sum(axis=0)
    assert np.abs(torque).max() < 1e-14 * np.abs(F).sum()


def test_pair_minimum_image(orc):
    """Two nodes on either side of the periodic x boundary interact over the
    0.2 gap, not over the box length."""
    tm, objs = _tetra_objects([(5.0, 5.0, 5.0), (9.0, 9.0, 9.0)], [0, 1])
    rep = [synth.SoftSphere(0, 1, a=1e-4, n=2.0, cutoff=0.3)]
    s = orc.System(_box(objs, tm, rep, n=12))
    X = s.X.copy()
    X[0] = (0.1, 6.0, 6.0)
    X[4] = (11.9 + 12.0, 6.0, 6.0)  # unwrapped: one box further
    s.X[:] = X
    F = s.repulsion()
    f = 1e-4 * 2.0 * 0.2 ** -3.0
    assert F[0] == pytest.approx([f, 0.0, 0.0], rel=1e-9)
    assert F[4] == pytest.approx([-f, 0.0, 0.0], rel=1e-9)


def _box_distance(lo, hi, x):
    """Distance from x to an axis-aligned box (independent formula)."""
    q = np.maximum(np.maximum(lo - x, 0.0), x - hi)
    return np.linalg.norm(q)


def test_shape_distances(orc):
    rng = np.random.default_rng(32)
    box = synth.Boundary("rhomboid", corner=(2.0, 3.0, 1.0), a=(3.0, 0, 0), b=(0, 2.0, 0), c=(0, 0, 1.5))
    lo, hi = np.array([2.0, 3.0, 1.0]), np.array([5.0, 5.0, 2.5])
    for _ in range(200):
        x = rng.uniform(0, 8, 3)
        r = orc.shape_distance(box, x)
        inside = np.all(x >= lo) and np.all(x <= hi)
        assert (r is None) == inside
        if r is not None:
            assert r[0] == pytest.approx(_box_distance(lo, hi, x), rel=1e-13, abs=1e-14)
            # the direction points from the closest surface point to x
            assert _box_distance(lo, hi, x - r[0] * r[1]) < 1e-12
    # sheared rhomboid against a bounded minimisation over (s, t, u)
    sh = synth.Boundary("rhomboid", corner=(1.0, 1.0, 1.0), a=(3.0, 0.5, 0.0), b=(0.8, 2.0, 0.3),
                        c=(0.2, -0.4, 1.7))
    A = np.array([sh.a, sh.b, sh.c]).T
    for _ in range(40):
        x = rng.uniform(-1, 7, 3)
        r = orc.shape_distance(sh, x)
        stu = np.linalg.solve(A, x - np.array(sh.corner))
        assert (r is None) == bool(np.all((stu >= 0) & (stu <= 1)))
        if r is None:
            continue
        best = min((minimize(lambda p: np.sum((x - sh.corner - A @ p) ** 2), p0, method="L-BFGS-B",
                             bounds=[(0, 1)] * 3, options=dict(ftol=1e-15, gtol=1e-12)).fun
                    for p0 in rng.uniform(0, 1, (4, 3))))
        assert r[0] == pytest.approx(np.sqrt(best), rel=1e-6, abs=1e-7)
    # half-space wall n.x < dist (n not normalised)
    w = synth.Boundary("wall", normal=(0.0, 3.0, 4.0), dist=2.0)
    x = np.array([1.0, 2.0, 3.0])
    r = orc.shape_distance(w, x)
    assert r[0] == pytest.approx((3 * 2 + 4 * 3) / 5 - 2.0, rel=1e-15)
    assert r[1] == pytest.approx([0.0, 0.6, 0.8], rel=1e-15)
    assert orc.shape_distance(w, np.array([0.0, 0.0, 0.1])) is None


def test_wall_forces_closed_form_and_gradient(orc):
    """Nodes near the z walls, a half-space wall and an axis-aligned block:
    forces are a n (d - offset)^-(n+1) along the outward direction, the sum of
    -grad of the wall energies (central differences on independent
    distances)."""
    tm, objs = _tetra_objects([(6.0, 6.0, 6.0)], [3])
    wall = synth.Boundary("wall", normal=(1.0, 0.0, 0.0), dist=1.0)          # solid for x < 1
    block = synth.Boundary("rhomboid", corner=(8.0, 2.0, 2.0), a=(2.0, 0, 0), b=(0, 9.0, 0), c=(0, 0, 9.0))
    rep = [synth.SoftSphere(3, None, a=1e-4, n=1.2, cutoff=0.6, offset=0.05)]
    s = orc.System(_box(objs, tm, rep, walls=True, bnd=(wall, block)))
    X = np.array([[3.0, 6.0, 0.3],    # near z = 0
                  [4.0, 6.0, 15.55],  # near z = 16
                  [1.35, 6.0, 6.0],   # near the half-space wall
                  [7.6, 3.0, 3.0]])   # near the block face x = 8
    s.X[:] = X

    def energy(P):
        E = 0.0
        for p in P:
            for d in (p[2], 16.0 - p[2], p[0] - 1.0, _box_distance(np.array([8.0, 2.0, 2.0]),
                                                                    np.array([10.0, 11.0, 11.0]), p)):
                e = d - 0.05
                if 0 < e < 0.6:
                    E += 1e-4 * e ** -1.2
        return E

    F = s.repulsion()
    eps = 1e-6
    G = np.zeros_like(X)
    for j in range(4):
        for c in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[j, c] += eps
            Xm[j, c] -= eps
            G[j, c] = -(energy(Xp) - energy(Xm)) / (2 * eps)
    assert np.abs(F - G).max() < 1e-7 * np.abs(F).max()
    f = lambda d: 1e-4 * 1.2 * (d - 0.05) ** -2.2  # noqa: E731
    assert F[0] == pytest.approx([0, 0, f(0.3)], rel=1e-13)
    assert F[2] == pytest.approx([f(0.35), 0, 0], rel=1e-13)
    assert F[3] == pytest.approx([-f(0.4), 0, 0], rel=1e-13)


def test_repulsion_momentum_budget(orc):
    """Coupled run with pair repulsion in a periodic box: every step
    dP_fluid + sum m dV = N g + sum F_el + sum F_ext + sum F_rep, the pair part
    summing to zero.  With the wall interaction in a channel the step adds
    exactly the wall forces at the step-start positions (z only)."""
    x, t = synth.icosphere(2, 2.0)
    tm = synth.Template(x, t, ks=0.05, kv=0.5)
    objs = [synth.ObjectSpec(0, np.array([6.0, 6.0, 4.3]), ptype=0),
            synth.ObjectSpec(0, np.array([6.0, 6.0, 8.55]), ptype=1)]
    pair = synth.SoftSphere(0, 1, a=1e-6, n=2.0, cutoff=0.4)
    b = synth.Box(12, 12, 13, g=(1e-5, 0, 0), friction=0.3, templates=[tm], objects=objs, repulsion=[pair])
    s = orc.System(b)
    assert np.abs(s.repulsion()).max() > 1e-6
    E = orc.D3Q19_E.astype(float)
    for step in range(4):
        P0 = E.T @ s.n.reshape(19, -1).sum(axis=1)
        mV0 = s.V.sum(axis=0)
        s.run(1)
        d = s.last_diag
        P1 = E.T @ s.n.reshape(19, -1).sum(axis=1)
        lhs = (P1 - P0) + (s.V.sum(axis=0) - mV0)
        rhs = b.n_nodes * np.array(b.g) + d[1:4] + d[7:10] + d[10:13]
        assert np.abs(lhs - rhs).max() < 1e-12  # round-off of sums over 1872 nodes
        assert np.abs(d[10:13]).max() < 1e-17
    b.walls_z = True
    b.repulsion = [pair, synth.SoftSphere(0, None, a=1e-6, n=1.5, cutoff=2.5)]
    s = orc.System(b)
    Fr = s.repulsion()
    s.run(1)
    assert np.abs(s.last_diag[10:13] - Fr.sum(axis=0)).max() < 1e-18
    assert np.abs(Fr.sum(axis=0)[:2]).max() < 1e-18 and abs(Fr.sum(axis=0)[2]) > 1e-8
