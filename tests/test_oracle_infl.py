"""Pins of the oracle's influence function (the 1-d validation's
J(r) = c1 r exp(-r^2/c2) of r = |xi|/delta, a factor of each bond's force and
energy): switched off it changes nothing; on a line of nodes under a
quadratic displacement the interior force is a one-dimensional sum written
out here and tends to the continuum integral as h -> 0; the force is minus
the gradient of the energy with J on; Verlet steps with J conserve energy to
second order."""
import math

import numpy as np
import pytest
from scipy import integrate

from paper_1806_06917_amd import inputs

J = (1.0, 0.4)     # c1, c2 of the 1-d validation


def line(N, h, delta, orc):
    """N + 1 nodes x_k = k h on the x axis (2-d coordinates, y = 0), V = h."""
    X = np.zeros((N + 1, 2))
    X[:, 0] = h * np.arange(N + 1)
    return orc.LawMesh(X, np.full(N + 1, h), delta, method="brute")


def test_off_changes_nothing(orc):
    h = 1.0 / 14
    X = inputs.grid_coords((14, 14), h, jitter=0.05, seed=171)
    m = orc.LawMesh(X, np.full(len(X), h * h), 3 * h)
    u = inputs.random_field(len(X), 2, 172, scale=3e-3)
    for law, st in ((orc.LAW_LINEAR, orc.STRETCH_LINEARISED), (orc.LAW_NP, orc.STRETCH_EXACT)):
        f0, U0 = m.force_law(u, 2.0, law, 50.0, st, energy=True)
        f1, U1 = m.force_law(u, 2.0, law, 50.0, st, energy=True, j=(1.0, 0.0))
        assert np.array_equal(f0, f1) and np.array_equal(U0, U1)


@pytest.mark.parametrize("m", [3, 5])
def test_line_quadratic_field(orc, m):
    """u = (x^2, 0): by the symmetry of the neighbours of an interior node,
    S e_x = 2 x_i sign(s) + |s| sums to f_x = 2 c V sum_k J(k h/delta) k h
    over k = 1..m, and f_y = 0."""
    h = 0.01
    delta = (m + 0.5) * h
    N = 40
    mesh = line(N, h, delta, orc)
    u = np.zeros_like(mesh.X)
    u[:, 0] = mesh.X[:, 0] ** 2
    c = 3.0
    f = mesh.force_law(u, c, orc.LAW_LINEAR, 1.0, j=J)
    c1, c2 = J
    ref = 2.0 * c * h * sum(c1 * (k * h / delta) * math.exp(-(k * h / delta) ** 2 / c2) * (k * h)
                            for k in range(1, m + 1))
    inner = slice(m + 1, N - m)
    np.testing.assert_allclose(f[inner, 0], ref, rtol=1e-11)
    assert np.all(f[:, 1] == 0.0)
    # J off: the same sum without the factor
    f0 = mesh.force_law(u, c, orc.LAW_LINEAR, 1.0)
    np.testing.assert_allclose(f0[inner, 0], 2.0 * c * h * sum(k * h for k in range(1, m + 1)),
                               rtol=1e-11)


def test_line_quadratic_continuum_limit(orc):
    """As h -> 0 at fixed delta the interior force of u = x^2 tends to
    2 c delta^2 int_0^1 c1 t^2 exp(-t^2/c2) dt."""
    c, delta = 3.0, 0.05
    c1, c2 = J
    cont = 2.0 * c * delta ** 2 * integrate.quad(lambda t: c1 * t * t * math.exp(-t * t / c2),
                                                 0.0, 1.0, epsabs=1e-14)[0]
    errs = []
    for m in (4, 8, 16, 32):
        h = delta / m
        N = 4 * m + 8
        mesh = line(N, h, delta * (1 + 1e-9), orc)
        u = np.zeros_like(mesh.X)
        u[:, 0] = mesh.X[:, 0] ** 2
        f = mesh.force_law(u, c, orc.LAW_LINEAR, 1.0, j=J)
        errs.append(abs(f[N // 2, 0] / cont - 1.0))
    assert errs[-1] < 0.02
    assert all(b < 0.7 * a for a, b in zip(errs, errs[1:]))


@pytest.mark.parametrize("law,stretch", [(0, 0), (1, 0), (1, 1)])
def test_force_is_minus_energy_gradient(orc, law, stretch):
    h = 1.0 / 16
    X = inputs.grid_coords((16, 16), h, jitter=0.05, seed=173)
    V = h * h * np.random.Generator(np.random.PCG64(174)).uniform(0.8, 1.2, len(X))
    mesh = orc.LawMesh(X, V, 3 * h)
    u = inputs.random_field(len(X), 2, 175, scale=3e-3)
    w = inputs.random_field(len(X), 2, 176, scale=1.0)
    c, beta, eps = 2.0, 200.0, 1e-7
    P = lambda x: mesh.energy_law(x, c, law, beta, stretch, j=J)  # noqa: E731
    dpi = (P(u + eps * w) - P(u - eps * w)) / (2 * eps)
    f = mesh.force_law(u, c, law, beta, stretch, j=J)
    rhs = -np.sum(V[:, None] * f * w)
    assert abs(dpi - rhs) <= 1e-6 * abs(rhs)
    # and J does change the force
    assert not np.allclose(f, mesh.force_law(u, c, law, beta, stretch), rtol=1e-3)


def test_verlet_with_influence_second_order(orc):
    h = 1.0 / 12
    X = inputs.grid_coords((12, 12), h, jitter=0.05, seed=177)
    mesh = orc.LawMesh(X, np.full(len(X), h * h), 3 * h)
    v0 = inputs.random_field(len(X), 2, 178, scale=1e-2)
    c, beta = 2.0, 100.0

    def drift(dt, steps):
        st = mesh.start_law(np.zeros_like(v0), v0, c, orc.LAW_NP, beta)
        st["f"] = mesh.force_law(st["u"], c, orc.LAW_NP, beta, j=J)
        e0 = mesh.kinetic(st["v"], 1.0) + mesh.energy_law(st["u"], c, orc.LAW_NP, beta, j=J)
        mesh.steps_j(st, c, 1.0, 0.0, dt, steps, J, orc.LAW_NP, beta)
        e1 = mesh.kinetic(st["v"], 1.0) + mesh.energy_law(st["u"], c, orc.LAW_NP, beta, j=J)
        return abs(e1 - e0) / e0

    d1, d2 = drift(0.1 * h, 40), drift(0.05 * h, 80)
    assert d1 < 1e-3
    assert 2.5 < d1 / d2 < 6.0


@pytest.mark.parametrize("m", [2, 4, 8])
def test_line_meshes_nest(m):
    """The 1-d study's meshes: cell-centred on [-delta, 1+delta], each coarse
    cell the union of two fine cells (the fine centres straddle the coarse
    centre), collars of delta/h clamped cells at each end, the pulses inside
    (0, 1) only, motion along x only; coarsen_line averages the pairs."""
    a, b = inputs.convergence_line(m, 2), inputs.convergence_line(2 * m, 2)
    assert b.n == 2 * a.n and a.n == int(round(1.02 * m / 0.01))
    np.testing.assert_allclose(0.5 * (b.X[0::2, 0] + b.X[1::2, 0]), a.X[:, 0], atol=1e-15)
    assert np.all(a.X[:, 1] == 0.0) and np.all(a.u0[:, 1] == 0.0)
    clamped = a.bc_kind == inputs.BC_CLAMPED
    assert clamped.sum() == 2 * m and np.all(a.u0[clamped] == 0.0)
    assert np.all((a.X[~clamped, 0] > 0) & (a.X[~clamped, 0] < 1))
    u = np.arange(2.0 * b.n).reshape(b.n, 2)
    np.testing.assert_array_equal(inputs.coarsen_line(u, a.n), 0.5 * (u[0::2] + u[1::2]))
    # IC 2: two pulses of amplitude a at 0.25 and 0.75
    i1, i2 = np.argmin(abs(b.X[:, 0] - 0.25)), np.argmin(abs(b.X[:, 0] - 0.75))
    assert abs(b.u0[i1, 0] - 1e-3) < 1e-5 and abs(b.u0[i2, 0] - 1e-3) < 1e-5


@pytest.mark.parametrize("rho,dt", [(1.0, 0.05), (2.5, 0.11)])
def test_central_with_influence_oscillator(orc, rho, dt):
    """Central-difference steps with J on a two-node bond: J multiplies the
    bond's stiffness by J(L/delta), so the discrete solution is
    A cos(n theta) with cos theta = 1 - omega^2 dt^2/2,
    omega^2 = c J(L/delta) (V1 + V2)/(rho L); the returned velocity is the
    velocity-Verlet one of the same steps."""
    L, c, A = 0.5, 3.0, 1e-3
    X = np.array([[0.0, 0.0], [L, 0.0]])
    m = orc.LawMesh(X, np.array([0.2, 0.3]), 1.1 * L, method="brute")
    delta = m.delta
    c1, c2 = J
    t = L / delta
    jv = c1 * t * math.exp(-t * t / c2)
    u0 = np.array([[-A / 2, 0.0], [A / 2, 0.0]])
    omega2 = c * jv * (m.V[0] + m.V[1]) / (rho * L)
    theta = math.acos(1 - omega2 * dt * dt / 2)
    for nsteps in (1, 2, 37, 200):
        st = m.start_law(u0, np.zeros((2, 2)), c, orc.LAW_LINEAR, 1.0)
        st["f"] = m.force_law(st["u"], c, orc.LAW_LINEAR, 1.0, j=J)
        m.steps_j(st, c, rho, 0.0, dt, nsteps, J, central=True)
        w = st["u"][1, 0] - st["u"][0, 0]
        assert abs(w - A * math.cos(nsteps * theta)) <= 1e-12 * A
        sv = m.start_law(u0, np.zeros((2, 2)), c, orc.LAW_LINEAR, 1.0)
        sv["f"] = m.force_law(sv["u"], c, orc.LAW_LINEAR, 1.0, j=J)
        m.steps_j(sv, c, rho, 0.0, dt, nsteps, J)
        np.testing.assert_allclose(st["v"], sv["v"], rtol=1e-9, atol=1e-15)


@pytest.mark.parametrize("law", [0, 1])
def test_central_with_influence_equals_verlet(orc, law):
    """On the 1-d study's line (h = delta/4, IC 2, clamped collars) the
    central-difference and velocity-Verlet steps with J share one
    recurrence, so they agree to rounding, but not bit for bit."""
    w = inputs.convergence_line(4, 2)
    c = 2.0 / w.delta ** 2
    mesh = orc.LawMesh(w.X, w.V, w.delta)
    runs = []
    for central in (False, True):
        st = mesh.start_law(w.u0, w.v0, c, law, 1.0)
        st["f"] = mesh.force_law(st["u"], c, law, 1.0, j=J)
        mesh.steps_j(st, c, 1.0, 0.0, w.dt, 400, J, law, 1.0, central=central,
                     bc_kind=w.bc_kind, bc_vel=w.bc_vel)
        runs.append(st)
    a, b = runs
    assert np.linalg.norm(b["u"] - a["u"]) <= 1e-11 * np.linalg.norm(a["u"])
    assert np.linalg.norm(b["v"] - a["v"]) <= 1e-9 * np.linalg.norm(a["v"])
    assert not np.array_equal(b["u"], a["u"])
    assert np.all(b["u"][w.bc_kind == inputs.BC_CLAMPED] == 0.0)
    # J is applied: without it the trajectory differs
    st = mesh.start_law(w.u0, w.v0, c, law, 1.0)
    mesh.central_law(st, c, 1.0, 0.0, w.dt, 400, law, 1.0, bc_kind=w.bc_kind, bc_vel=w.bc_vel)
    assert np.linalg.norm(st["u"] - b["u"]) > 1e-3 * np.linalg.norm(b["u"])


def test_central_with_influence_prescribed_velocity(orc):
    """Prescribed-velocity nodes under the central-difference steps with J
    follow their ramped velocity in closed form (J acts on forces only)."""
    w = inputs.notched_plate_2d(N=24, m=3, s_c=0.0, v0=2e-3, steps=0, ramp_steps=10)
    mesh = orc.LawMesh(w.X, w.V, w.delta)
    c = orc.micromodulus(2, w.E, w.delta)
    st = mesh.start_law(w.u0, w.v0, c, orc.LAW_LINEAR, 1.0)
    st["f"] = mesh.force_law(st["u"], c, orc.LAW_LINEAR, 1.0, j=J)
    mesh.steps_j(st, c, w.rho, 0.0, w.dt, 30, J, central=True, bc_kind=w.bc_kind,
                 bc_vel=w.bc_vel, ramp=w.ramp_steps)
    sel = w.bc_kind == 2
    ramp = sum(min(1.0, (k + 0.5) / 10) for k in range(30))
    np.testing.assert_allclose(st["u"][sel], w.dt * ramp * w.bc_vel[sel], rtol=1e-12, atol=1e-18)
    np.testing.assert_allclose(st["v"][sel], w.bc_vel[sel], rtol=1e-15)
