"""Pins of the oracle's central-difference scheme (the finite-difference
equation of Section "Explicit time integration"): the harmonic oscillator's
exact discrete solution (the scheme and velocity Verlet share the recurrence
w_{n+1} = 2 w_n - w_{n-1} - (omega dt)^2 w_n), agreement with velocity Verlet
up to rounding for the linear and NP laws, and boundary data."""
import numpy as np
import pytest

from paper_1806_06917_amd import inputs


@pytest.mark.parametrize("rho,dt", [(1.0, 0.05), (2.5, 0.11)])
def test_oscillator_exact_discrete_solution(orc, rho, dt):
    L, c, A = 0.5, 3.0, 1e-3
    m = orc.LawMesh(np.array([[0.0, 0.0], [L, 0.0]]), np.array([0.2, 0.3]), 1.1 * L,
                    method="brute")
    u0 = np.array([[-A / 2, 0.0], [A / 2, 0.0]])
    omega2 = c * (m.V[0] + m.V[1]) / (rho * L)
    theta = np.arccos(1 - omega2 * dt * dt / 2)
    for nsteps in (1, 2, 37, 200):
        st = m.start_law(u0, np.zeros((2, 2)), c, orc.LAW_LINEAR, 1.0)
        m.central_law(st, c, rho, 0.0, dt, nsteps, orc.LAW_LINEAR)
        w = st["u"][1, 0] - st["u"][0, 0]
        assert abs(w - A * np.cos(nsteps * theta)) <= 1e-12 * A
        # the returned velocity is the velocity-Verlet velocity of step n
        sv = m.start(u0, np.zeros((2, 2)), c)
        m.verlet(sv, c, rho, 0.0, dt, nsteps)
        np.testing.assert_allclose(st["v"], sv["v"], rtol=1e-9, atol=1e-15)


@pytest.mark.parametrize("law", [0, 1])
def test_central_equals_verlet_up_to_rounding(orc, law):
    w = inputs.plate_2d(20, 3, seed=1, steps=0)
    mesh = orc.LawMesh(w.X, w.V, w.delta)
    c = orc.micromodulus(2, w.E, w.delta)
    v0 = inputs.random_field(mesh.n, 2, 121, scale=5e-2)
    beta = 2e4
    a = mesh.start_law(w.u0, v0, c, law, beta)
    b = mesh.start_law(w.u0, v0, c, law, beta)
    mesh.verlet_law(a, c, w.rho, 0.0, w.dt, 150, law, beta)
    mesh.central_law(b, c, w.rho, 0.0, w.dt, 150, law, beta)
    assert np.linalg.norm(b["u"] - a["u"]) <= 1e-11 * np.linalg.norm(a["u"])
    assert np.linalg.norm(b["v"] - a["v"]) <= 1e-9 * np.linalg.norm(a["v"])
    assert not np.array_equal(b["u"], a["u"])          # a different rounding, not a copy


def test_central_boundary_data(orc):
    w = inputs.notched_plate_2d(N=24, m=3, s_c=0.0, v0=2e-3, steps=0, ramp_steps=10)
    mesh = orc.LawMesh(w.X, w.V, w.delta)
    c = orc.micromodulus(2, w.E, w.delta)
    st = mesh.start_law(w.u0, w.v0, c, orc.LAW_LINEAR, 1.0)
    mesh.central_law(st, c, w.rho, 0.0, w.dt, 30, orc.LAW_LINEAR, 1.0, bc_kind=w.bc_kind,
                     bc_vel=w.bc_vel, ramp=w.ramp_steps)
    sel = w.bc_kind == 2
    # prescribed-velocity nodes: u = dt * sum of r(k + 1/2) vbar, v = r(30) vbar
    ramp = sum(min(1.0, (k + 0.5) / 10) for k in range(30))
    np.testing.assert_allclose(st["u"][sel], w.dt * ramp * w.bc_vel[sel], rtol=1e-12, atol=1e-18)
    np.testing.assert_allclose(st["v"][sel], w.bc_vel[sel], rtol=1e-15)
