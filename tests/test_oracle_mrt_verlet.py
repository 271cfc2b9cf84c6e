"""Pins of the oracle's optional engine variants (no GPU): the
multiple-relaxation-time collision of the paper's LB references (Section
"Method", the collision operator deferred to Ahlrichs & Duenweg and Duenweg &
Ladd) and the velocity Verlet mesh integrator of the paper's engine (eq. newton
integrated as the engine does, drag taken at the half-step velocity).

Every expected value here is computed from its own definition: moments and
projections with plain numpy, closed forms of uniformly accelerated motion,
time reversal, the BGK operator (itself pinned in test_oracle_lb.py)."""
import math

import numpy as np
import pytest

from paper_1312_3426_amd import synth

E = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
              [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1], [1, 0, -1],
              [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], dtype=float)
W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
OPP = [0] + [i + 1 if i % 2 else i - 1 for i in range(1, 19)]


def total_momentum(n):
    """Sum over nodes of each population first (pairwise summation), then the
    velocity moments: keeps the round-off of large opposite sums small."""
    return E.T @ n.reshape(19, -1).sum(axis=1)


def nu_of(gamma):
    """Kinematic viscosity of a shear relaxation factor gamma: the BGK relation
    nu = (tau - 1/2)/3 with gamma = 1 - 1/tau."""
    tau = 1 / (1 - gamma)
    return (tau - 0.5) / 3


# ---------------------------------------------------------------------------
# multiple-relaxation-time collision
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("tau", [0.55, 0.8, 1.0, 1.7])
@pytest.mark.parametrize("walls", [False, True])
def test_mrt_with_equal_rates_is_bgk(orc, tau, walls):
    """All rates 1 - 1/tau: the mode-space operator is the BGK operator."""
    rng = np.random.default_rng(11)
    n = W.reshape(19, 1, 1, 1) * (1 + 0.05 * rng.standard_normal((19, 4, 3, 5)))
    G = 1e-4 * rng.standard_normal((3, 4, 3, 5))
    g = (1e-5, -2e-5, 3e-5)
    gam = 1 - 1 / tau
    a = orc.lb_step(n, tau=tau, g=g, G=G, walls_z=walls)
    b = orc.lb_step(n, tau=tau, g=g, G=G, walls_z=walls, mrt=(gam, gam, gam, gam))
    assert np.abs(a - b).max() < 1e-15


def _hydro_projection(v):
    """Projection of a population vector onto the hydrodynamic subspace
    {w_i p(e_i), p of degree <= 2}, orthogonal in sum_i a_i b_i / w_i: a
    weighted least-squares fit of v/w by the ten quadratic monomials."""
    x, y, z = E.T
    P = np.stack([np.ones(19), x, y, z, x * x, y * y, z * z, x * y, x * z, y * z], axis=1)
    sw = np.sqrt(W)
    coef, *_ = np.linalg.lstsq(P * sw[:, None], (v / W) * sw, rcond=None)
    return W * (P @ coef)


@pytest.mark.parametrize("rates", [(0.3, -0.2, 0.5, -0.6), (-0.7, 0.4, 0.0, 0.9), (0.0, 0.0, 0.0, 0.0)])
def test_mrt_single_node_moments(orc, rates):
    """1x1x1 periodic box: one step is one collision.  Mass kept; momentum
    gains F; the trace and the traceless part of the second moment relax by
    gamma_bulk and gamma_shear towards rho/3 I + rho u u and take (1 + gamma)/2
    of u F + F u; the non-hydrodynamic remainder, split into its parts odd and
    even under e -> -e, is scaled by gamma_odd and gamma_even."""
    gs, gb, go, ge = rates
    rng = np.random.default_rng(12)
    iso = lambda A: np.trace(A) / 3 * np.eye(3)  # noqa: E731
    for _ in range(4):
        n = W * (1 + 0.2 * rng.standard_normal(19))
        F = 1e-3 * rng.standard_normal(3)
        out = orc.lb_step(n.reshape(19, 1, 1, 1), g=F, mrt=rates).ravel()
        rho = n.sum()
        j = E.T @ n
        assert out.sum() == pytest.approx(rho, rel=1e-15)
        assert np.abs(E.T @ out - (j + F)).max() < 1e-16
        u = (j + 0.5 * F) / rho
        Pi = np.einsum("i,ia,ib->ab", n, E, E)
        Pi1 = np.einsum("i,ia,ib->ab", out, E, E)
        Peq = rho * (np.eye(3) / 3 + np.outer(u, u))
        Phi = np.outer(u, F) + np.outer(F, u)
        D = Pi - Peq
        want = (Peq + gs * (D - iso(D)) + gb * iso(D)
                + 0.5 * (1 + gs) * (Phi - iso(Phi)) + 0.5 * (1 + gb) * iso(Phi))
        assert np.abs(Pi1 - want).max() < 2e-15
        gh0 = n - _hydro_projection(n)
        gh1 = out - _hydro_projection(out)
        odd = 0.5 * (gh0 - gh0[OPP])
        even = 0.5 * (gh0 + gh0[OPP])
        assert np.abs(gh1 - (go * odd + ge * even)).max() < 2e-15
        assert np.abs(odd).max() > 1e-3 and np.abs(even).max() > 1e-3  # both present


def test_mrt_conserves_total_mass_and_momentum(orc):
    rng = np.random.default_rng(13)
    n = W.reshape(19, 1, 1, 1) * (1 + 0.05 * rng.standard_normal((19, 5, 4, 6)))
    G = 1e-4 * rng.standard_normal((3, 5, 4, 6))
    g = np.array([1e-5, 0, -2e-5])
    out = orc.lb_step(n, g=g, G=G, mrt=(0.2, -0.5, 0.7, -0.3))
    assert out.sum() == pytest.approx(n.sum(), rel=1e-15)
    j0 = total_momentum(n)
    j1 = total_momentum(out)
    assert np.abs(j1 - (j0 + G.sum(axis=(1, 2, 3)) + g * n[0].size)).max() < 1e-14


def _shear_rate(orc, L, rates, steps=(40, 240)):
    z = np.arange(L) + 0.5
    A = 1e-4
    u = np.zeros(3)
    n = np.empty((19, L, 1, 1))
    for k in range(L):
        u[0] = A * math.sin(2 * math.pi * z[k] / L)
        eu = E @ u
        n[:, k, 0, 0] = W * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * u @ u)
    amps = {}
    for t in range(1, steps[1] + 1):
        n = orc.lb_step(n, mrt=rates)
        if t in steps:
            _, uu = orc.moments(n)
            amps[t] = 2 / L * np.sum(uu[0, :, 0, 0] * np.sin(2 * math.pi * z / L))
    k = 2 * math.pi / L
    return -math.log(amps[steps[1]] / amps[steps[0]]) / (k * k * (steps[1] - steps[0]))


def test_mrt_shear_wave_viscosity(orc):
    """A decaying shear wave measures nu = (1 + gamma_shear)/(6 (1 - gamma_shear))
    up to O(k^2).  The bulk and the even ghost rates do not enter a shear wave
    at all (same decay to round-off); a slowly relaxing odd ghost (third
    moments) changes only the O(k^2) correction, which still vanishes as L^-2.
    (Same decay: up to the O(u^2) coupling of the wave into the bulk modes,
    amplitude 1e-4.)"""
    gs = 0.25
    base = [_shear_rate(orc, L, (gs, 0.0, 0.0, 0.0)) for L in (16, 32)]
    other = [_shear_rate(orc, L, (gs, 0.6, 0.0, -0.8)) for L in (16, 32)]
    assert max(abs(a / b - 1) for a, b in zip(base, other)) < 1e-7
    errs = [abs(r / nu_of(gs) - 1) for r in base]
    assert errs[1] < 2e-3 and errs[1] < errs[0] / 3
    odd = [abs(_shear_rate(orc, L, (gs, 0.0, 0.8, 0.0)) / nu_of(gs) - 1) for L in (16, 32, 64)]
    assert odd[1] < odd[0] / 3.5 and odd[2] < odd[1] / 3.5 and odd[2] < 0.03


# ---------------------------------------------------------------------------
# velocity Verlet integrator
# ---------------------------------------------------------------------------
def _free_box(xi, m, integrator, nx=8, fext=(0.0, 0.0, 0.0)):
    x, t = synth.icosahedron(1.0)
    tm = synth.Template(x, t)  # all moduli zero: the nodes move independently
    return synth.Box(nx, nx, nx, g=(0.0, 0.0, 0.0), friction=xi, templates=[tm], integrator=integrator,
                     objects=[synth.ObjectSpec(0, np.array([3.3, 4.1, 3.7]), mass=m, fext=fext)])


@pytest.mark.parametrize("integrator", ["euler", "verlet"])
def test_constant_force_closed_form(orc, integrator):
    """No friction, a constant external force: after n steps, with no force
    carried into the first step, velocity Verlet gives X_n = X_0 + n V_0 +
    a n (n - 1)/2 and V_n = V_0 + a (n - 1/2); symplectic Euler gives
    X_n = X_0 + n V_0 + a n (n + 1)/2 and V_n = V_0 + a n (a = F/m)."""
    m = 2.0
    f = np.array([3e-4, -1e-4, 2e-4])
    s = orc.System(_free_box(0.0, m, integrator, fext=f))
    v0 = np.array([0.01, 0.02, -0.015])
    s.V[:] = v0
    X0 = s.X.copy()
    a = f / m
    done = 0
    for n in (1, 2, 7):
        s.run(n - done)
        done = n
        if integrator == "verlet":
            dx, v = n * v0 + a * n * (n - 1) / 2, v0 + a * (n - 0.5)
        else:
            dx, v = n * v0 + a * n * (n + 1) / 2, v0 + a * n
        assert np.abs(s.X - X0 - dx).max() < 1e-14
        assert np.abs(s.V - v).max() < 1e-16


def test_verlet_step_with_drag_at_rest_fluid(orc):
    """Fluid at rest (u = 0 at every node): the drag is xi times the half-step
    velocity V_h = V_t + F_t/(2m); X_{t+1} = X_t + V_h and
    V_{t+1} = V_h + (F_ext - xi V_h)/(2m); the force carried on is F_ext - xi V_h."""
    xi, m = 0.3, 2.0
    fext = np.array([1e-4, 0.0, -2e-4])
    s = orc.System(_free_box(xi, m, "verlet", fext=fext))
    rng = np.random.default_rng(14)
    V0 = 0.01 * rng.standard_normal(s.X.shape)
    F0 = 1e-3 * rng.standard_normal(s.X.shape)
    s.V[:] = V0
    s.F = F0
    X0 = s.X.copy()
    s.run(1)
    Vh = V0 + F0 / (2 * m)
    assert np.abs(s.X - (X0 + Vh)).max() < 1e-15
    Ft = fext - xi * Vh
    assert np.abs(s.V - (Vh + Ft / (2 * m))).max() < 1e-17
    assert np.abs(s.F - Ft).max() < 1e-18
    d = s.last_diag
    assert np.abs(d[4:7] - (-xi * Vh.sum(axis=0))).max() < 1e-16  # coupling on the mesh
    # the fluid received the opposite momentum
    P = total_momentum(s.n)
    assert np.abs(P - xi * Vh.sum(axis=0)).max() < 1e-13  # sum over 512 nodes: round-off only


def test_verlet_is_time_reversible(orc):
    """Elastic forces only (no friction): running n steps, reversing the
    velocities and running n steps more returns the start state (velocity
    Verlet is time-reversible; symplectic Euler is not)."""
    box = synth.config_sphere_fp64(1)
    box.friction = 0.0
    rng = np.random.default_rng(15)
    dX = V0 = None
    res = {}
    for integ in ("verlet", "euler"):
        box.integrator = integ
        s = orc.System(box)
        if dX is None:
            dX = 0.05 * rng.standard_normal(s.X.shape)
            V0 = 1e-3 * rng.standard_normal(s.X.shape)
        s.X += dX
        X0 = s.X.copy()
        s.V[:] = V0
        if integ == "verlet":
            s.F = s.forces()  # the force at the start state
        s.run(25)
        s.V[:] = -s.V
        s.run(25)
        res[integ] = (np.abs(s.X - X0).max(), np.abs(s.V + V0).max())
    assert res["verlet"][0] < 1e-12 and res["verlet"][1] < 1e-13
    assert res["euler"][0] > 1e-6  # the other integrator does not retrace its path


def test_verlet_momentum_budget(orc):
    """With the force carried into the next step, R = sum (m V + F/2) closes the
    budget every step: dP_fluid + dR = N g + sum F_el + sum F_ext."""
    b = synth.config_sphere_fp64(10)
    b.integrator = "verlet"
    b.objects[0].fext = (2e-6, -1e-6, 0.0)
    s = orc.System(b)
    N = b.n_nodes
    g = np.array(b.g)
    rng = np.random.default_rng(17)
    s.X += 0.05 * rng.standard_normal(s.X.shape)
    m = b.objects[0].mass
    for step in range(6):
        P0 = total_momentum(s.n)
        R0 = (m * s.V + 0.5 * s.F).sum(axis=0)
        s.run(1)
        d = s.last_diag
        P1 = total_momentum(s.n)
        R1 = (m * s.V + 0.5 * s.F).sum(axis=0)
        assert np.abs((P1 - P0) + (R1 - R0) - (N * g + d[1:4] + d[7:10])).max() < 1e-12
        assert np.abs(d[1:4]).max() > 1e-8
