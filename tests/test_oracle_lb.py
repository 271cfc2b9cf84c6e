"""Pins of the oracle's lattice-Boltzmann update (paper, Section "Method",
eq. lbequation and the moment definitions) against conservation laws, closed
forms and textbook flows (no GPU)."""
import math

import numpy as np
import pytest

E = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
              [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1], [1, 0, -1],
              [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], dtype=float)
W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def textbook_equilibrium(rho, u):
    """Second-order D3Q19 equilibrium, rho (...), u (3, ...) -> (19, ...)."""
    eu = np.einsum("ic,c...->i...", E, u)
    usq = np.einsum("c...,c...->...", u, u)
    return W.reshape((19,) + (1,) * rho.ndim) * rho * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * usq)


def mom(n):
    return np.einsum("i...->...", n), np.einsum("ic,i...->c...", E, n)


def test_velocity_set_is_d3q19(orc):
    # the oracle's tables, checked through its own moments: isotropy up to 4th order
    assert np.allclose(orc.D3Q19_E, E) and np.allclose(orc.D3Q19_W, W)
    assert W.sum() == pytest.approx(1.0, abs=1e-16)
    assert np.allclose(np.einsum("i,ia,ib->ab", W, E, E), np.eye(3) / 3, atol=1e-16)


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
def test_collision_conserves_and_forces_single_node(orc, tau):
    """1x1x1 periodic box: streaming is the identity, so one step is one
    collision.  Mass is conserved, momentum gains F, and the second moment
    relaxes as Pi' = Pi - (Pi - Pi_eq)/tau + (1 - 1/(2 tau))(u F + F u)."""
    rng = np.random.default_rng(1)
    for _ in range(5):
        n = (W * (1 + 0.2 * rng.standard_normal(19))).reshape(19, 1, 1, 1)
        g = 1e-3 * rng.standard_normal(3)
        out = orc.lb_step(n, tau=tau, g=g)
        r0, j0 = mom(n)
        r1, j1 = mom(out)
        assert r1.item() == pytest.approx(r0.item(), rel=1e-15)
        assert np.allclose(j1.ravel(), j0.ravel() + g, rtol=0, atol=1e-16)
        rho = r0.item()
        u = (j0.ravel() + 0.5 * g) / rho
        Pi = np.einsum("i,ia,ib->ab", n.ravel(), E, E)
        Pi1 = np.einsum("i,ia,ib->ab", out.ravel(), E, E)
        Pi_eq = rho * (np.eye(3) / 3 + np.outer(u, u))
        want = Pi - (Pi - Pi_eq) / tau + (1 - 0.5 / tau) * (np.outer(u, g) + np.outer(g, u))
        assert np.abs(Pi1 - want).max() < 2e-15


def test_collision_conserves_total_mass_momentum(orc):
    rng = np.random.default_rng(2)
    n = W.reshape(19, 1, 1, 1) * (1 + 0.05 * rng.standard_normal((19, 5, 4, 6)))
    G = 1e-4 * rng.standard_normal((3, 5, 4, 6))
    g = np.array([1e-5, 0, -2e-5])
    out = orc.lb_step(n, tau=0.9, g=g, G=G)
    r0, j0 = mom(n)
    r1, j1 = mom(out)
    assert r1.sum() == pytest.approx(r0.sum(), rel=1e-15)
    want = j0.sum(axis=(1, 2, 3)) + G.sum(axis=(1, 2, 3)) + g * n[0].size
    assert np.allclose(j1.sum(axis=(1, 2, 3)), want, rtol=0, atol=1e-14)


@pytest.mark.parametrize("walls", [False, True])
def test_streaming_moves_local_equilibria(orc, walls):
    """With every node at its own equilibrium and no force, collision is the
    identity and each population moves one link along e_i (periodic), or
    returns reversed at a wall."""
    rng = np.random.default_rng(3)
    nz, ny, nx = 4, 3, 5
    rho = 1 + 0.1 * rng.random((nz, ny, nx))
    u = 0.05 * rng.standard_normal((3, nz, ny, nx))
    n = textbook_equilibrium(rho, u)
    out = orc.lb_step(n, tau=0.8, walls_z=walls)
    for i in range(19):
        ex, ey, ez = E[i].astype(int)
        for z in range(nz):
            zd = z + ez
            if walls and not 0 <= zd < nz:
                opp = i + 1 if i % 2 else i - 1
                assert np.allclose(out[opp, z], n[i, z], rtol=1e-14, atol=0)
                continue
            zd %= nz
            shifted = np.roll(np.roll(n[i, z], ey, axis=0), ex, axis=1)
            assert np.allclose(out[i, zd], shifted, rtol=1e-14, atol=0)


def test_equilibrium_is_fixed_point(orc):
    rho = np.full((3, 4, 5), 1.1)
    u = np.broadcast_to(np.array([0.02, -0.01, 0.03])[:, None, None, None], (3, 3, 4, 5)).copy()
    n = textbook_equilibrium(rho, u)
    out = orc.lb_step(n, tau=0.7)
    assert np.abs(out - n).max() < 1e-16


@pytest.mark.parametrize("tau", [0.55, 1.0, 1.9])
def test_uniform_body_force_closed_form(orc, tau):
    """Periodic box at rest under uniform g: after n steps rho = 1 and the
    momentum is n g at every node, the velocity (n + 1/2) g."""
    g = np.array([1e-5, -2e-5, 3e-5])
    n = orc.equilibrium_populations(4, 3, 5)
    for step in range(1, 31):
        n = orc.lb_step(n, tau=tau, g=g)
    rho, j = mom(n)
    assert np.abs(rho - 1).max() < 1e-14
    assert np.abs(j - 30 * g[:, None, None, None]).max() < 1e-16 * 30 * 10
    _, u = orc.moments(n, g=g)
    assert np.abs(u - 30.5 * g[:, None, None, None]).max() < 1e-15


def _shear_rate(orc, L, tau, steps=(40, 240)):
    z = np.arange(L) + 0.5
    A = 1e-4
    u = np.zeros((3, L, 1, 1))
    u[0, :, 0, 0] = A * np.sin(2 * math.pi * z / L)
    n = textbook_equilibrium(np.ones((L, 1, 1)), u)
    amps = {}
    for t in range(1, steps[1] + 1):
        n = orc.lb_step(n, tau=tau)
        if t in steps:
            _, uu = orc.moments(n)
            amps[t] = 2 / L * np.sum(uu[0, :, 0, 0] * np.sin(2 * math.pi * z / L))
    k = 2 * math.pi / L
    return -math.log(amps[steps[1]] / amps[steps[0]]) / (k * k * (steps[1] - steps[0]))


def test_shear_wave_viscosity(orc):
    """A decaying shear wave measures nu = (tau - 1/2)/3 with O(k^2) error."""
    tau = 0.8
    nu = (tau - 0.5) / 3
    errs = [abs(_shear_rate(orc, L, tau) / nu - 1) for L in (16, 32, 64)]
    assert errs[2] < 2e-3
    assert errs[1] < errs[0] / 3 and errs[2] < errs[1] / 3


@pytest.mark.parametrize("tau", [1.0, 0.5 + math.sqrt(3) / 4])
def test_poiseuille_with_halfway_bounce_back(orc, tau):
    """Channel between bounce-back walls at z = 0 and z = H under force g:
    u(z) = g/(2 nu) z (H - z) + (g/nu)(16 L - 3)/24, L = (tau - 1/2)^2, at the
    node centres z = k + 1/2 (no slip term at L = 3/16)."""
    H = 16
    g = np.array([1e-5, 0, 0])
    n = orc.equilibrium_populations(1, 1, H)
    for _ in range(12000):
        n = orc.lb_step(n, tau=tau, g=g, walls_z=True)
    _, u = orc.moments(n, g=g)
    nu = (tau - 0.5) / 3
    Lam = (tau - 0.5) ** 2
    z = np.arange(H) + 0.5
    want = g[0] / (2 * nu) * z * (H - z) + g[0] / nu * (16 * Lam - 3) / 24
    # the linear analysis is exact for this flow: agreement to round-off
    assert np.abs(u[0, :, 0, 0] - want).max() < 1e-10 * want.max()
    assert np.abs(u[1:]).max() < 1e-14  # round-off only
