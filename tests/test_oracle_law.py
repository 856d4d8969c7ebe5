"""Pins of the oracle's general pairwise law (Algorithm 1 with the NP potential
psi(r) = C (1 - exp(-beta r)) of the validation section, and the exact-stretch
variant): the force is minus the gradient of the strain energy for every law
and stretch, the NP law tends to the linearised law for small beta r, the
exact stretch vanishes under a finite rigid rotation, the NP tangent equals the
paper's central-difference tangent of the force, and Newton's method reaches
the NP equilibrium."""
import math

import numpy as np
import pytest

from paper_1806_06917_amd import inputs


def jittered(orc, dim, N, seed, m=3):
    h = 1.0 / N
    X = inputs.grid_coords((N,) * dim, h, jitter=0.05, seed=seed)
    rng = np.random.Generator(np.random.PCG64(seed + 100))
    V = h ** dim * rng.uniform(0.8, 1.2, X.shape[0])
    return orc.LawMesh(X, V, m * h)


def bond_r(mesh, u, stretch=0):
    """r = |xi| S^2 of every bond (for choosing beta r ranges in the tests)."""
    i = np.repeat(np.arange(mesh.n), np.diff(mesh.row_ptr))
    j = mesh.col.astype(np.int64)
    xi = mesh.X[j] - mesh.X[i]
    eta = u[j] - u[i]
    L = np.linalg.norm(xi, axis=1)
    if stretch == 0:
        S = np.sum(xi * eta, axis=1) / L ** 2
    else:
        S = (np.linalg.norm(xi + eta, axis=1) - L) / L
    return L * S * S


def test_np_two_nodes_by_hand(orc):
    # xi = (0.3, 0.4), |xi| = 0.5, eta = (0.003, 0.004): S = 0.01, r = 5e-5;
    # beta = 1000: beta r = 0.05.  c = 2, V1 = 0.25, V2 = 0.5, e = (0.6, 0.8)
    m = orc.LawMesh(np.array([[0.0, 0.0], [0.3, 0.4]]), np.array([0.25, 0.5]), 0.6,
                    method="brute")
    u = np.array([[0.001, -0.002], [0.004, 0.002]])
    f, U = m.force_law(u, 2.0, orc.LAW_NP, 1000.0, energy=True)
    g = 2.0 * math.exp(-0.05) * 0.01                  # c exp(-beta r) S
    np.testing.assert_allclose(f[0], [g * 0.6 * 0.5, g * 0.8 * 0.5], rtol=1e-14)
    np.testing.assert_allclose(f[1], [-g * 0.6 * 0.25, -g * 0.8 * 0.25], rtol=1e-14)
    w = 2.0 / (4 * 1000.0) * (1 - math.exp(-0.05))    # c/(4 beta) (1 - exp(-beta r))
    np.testing.assert_allclose(U, [w * 0.5, w * 0.25], rtol=1e-13)
    # exact stretch of the same bond: |xi + eta| = 0.505, S = 0.01 exactly in
    # real arithmetic, direction (0.303, 0.404)/0.505 = (0.6, 0.8)
    fe = m.force_law(u, 2.0, orc.LAW_NP, 1000.0, orc.STRETCH_EXACT)
    np.testing.assert_allclose(fe, f, rtol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_linear_law_is_the_linearised_oracle(orc, dim):
    mesh = jittered(orc, dim, 14 if dim == 2 else 7, seed=31)
    u = inputs.random_field(mesh.n, dim, 32)
    f, U = mesh.force_law(u, 1.3, orc.LAW_LINEAR, 5.0, energy=True)
    f0, U0 = mesh.force(u, 1.3, energy=True)
    assert np.array_equal(f, f0)
    np.testing.assert_allclose(U, U0, rtol=1e-14)
    w = inputs.random_field(mesh.n, dim, 33, scale=1.0)
    assert np.array_equal(mesh.tangent_law(w, 1.3, orc.LAW_LINEAR, 5.0, ulin=u),
                          mesh.apply_tangent(w, 1.3))


@pytest.mark.parametrize("dim,law,stretch", [(2, 1, 0), (3, 1, 0), (2, 1, 1), (3, 1, 1),
                                             (2, 0, 1), (3, 0, 1)])
def test_force_is_minus_energy_gradient(orc, dim, law, stretch):
    """-dPi/du . w = sum_i V_i f_i . w with Pi = sum_i V_i U_i, by central
    differences, for the NP law (beta r up to about 1) and the exact stretch."""
    mesh = jittered(orc, dim, 16 if dim == 2 else 8, seed=41)
    u = inputs.random_field(mesh.n, dim, 42, scale=2e-3)
    beta = 1.0 / bond_r(mesh, u, stretch).max()       # beta r in (0, 1]
    w = inputs.random_field(mesh.n, dim, 43, scale=1.0)
    c, eps = 1.7, 1e-7
    P = lambda x: mesh.energy_law(x, c, law, beta, stretch)  # noqa: E731
    dpi = (P(u + eps * w) - P(u - eps * w)) / (2 * eps)
    f = mesh.force_law(u, c, law, beta, stretch)
    rhs = -np.sum(mesh.V[:, None] * f * w)
    assert abs(dpi - rhs) <= 1e-6 * abs(rhs)


@pytest.mark.parametrize("dim", [2, 3])
def test_np_tends_to_linear_for_small_beta(orc, dim):
    mesh = jittered(orc, dim, 14 if dim == 2 else 7, seed=51)
    u = inputs.random_field(mesh.n, dim, 52)
    beta = 1e-6 / bond_r(mesh, u).max()               # beta r <= 1e-6
    f, U = mesh.force_law(u, 1.0, orc.LAW_NP, beta, energy=True)
    f0, U0 = mesh.force(u, 1.0, energy=True)
    assert np.linalg.norm(f - f0) <= 2e-6 * np.linalg.norm(f0)
    assert np.linalg.norm(U - U0) <= 2e-6 * np.linalg.norm(U0)
    # and NP softens: each bond force is smaller in magnitude than the linear one
    beta = 1.0 / bond_r(mesh, u).max()
    e_np = mesh.energy_law(u, 1.0, orc.LAW_NP, beta)
    assert e_np < mesh.potential(u, 1.0)


@pytest.mark.parametrize("dim", [2, 3])
def test_exact_stretch_rigid_rotation_is_force_free(orc, dim):
    """A finite rigid rotation leaves every bond length unchanged: the exact
    stretch gives no force, the linearised one does."""
    mesh = jittered(orc, dim, 14 if dim == 2 else 7, seed=61)
    a = 0.5                                           # radians
    R = np.eye(dim)
    R[0, 0], R[0, 1], R[1, 0], R[1, 1] = math.cos(a), -math.sin(a), math.sin(a), math.cos(a)
    u = mesh.X @ R.T - mesh.X
    f_lin = mesh.force_law(u, 1.0, orc.LAW_LINEAR, 1.0, orc.STRETCH_LINEARISED)
    f_ex = mesh.force_law(u, 1.0, orc.LAW_LINEAR, 1.0, orc.STRETCH_EXACT)
    scale = np.abs(f_lin).max()
    assert scale > 0.0
    assert np.abs(f_ex).max() <= 1e-12 * scale


def small_bar(orc, nx=14, ny=4, m=3, clamp=3, traction=1e-3):
    w = inputs.bar_2d(nx, ny, m, traction=traction, clamp_cols=clamp)
    mesh = orc.LawMesh(w.X, w.V, w.delta, method="brute")
    c = orc.micromodulus(2, w.E, w.delta)
    return w, mesh, c


def test_np_tangent_equals_central_difference_of_force(orc):
    """The analytic NP tangent c exp(-beta r)(1 - 2 beta r) per bond against the
    paper's tangent equation K = (f(u + eps) - f(u - eps))/(2 eps), column by
    column, at a strained state."""
    w, mesh, c = small_bar(orc)
    ulin, _ = mesh.solve_implicit(w.u0, c, w.b, w.fixed, rtol=1e-12)
    ulin = 30.0 * ulin                                # a state well into the nonlinear range
    beta = 0.3 / bond_r(mesh, ulin).max()
    n, d = mesh.n, 2
    eps = 1e-7 * np.abs(ulin).max()
    H = np.zeros((n * d, n * d))
    for q in range(n * d):
        e = np.zeros(n * d)
        e[q] = eps
        fp = mesh.force_law(ulin + e.reshape(n, d), c, orc.LAW_NP, beta).reshape(-1)
        fm = mesh.force_law(ulin - e.reshape(n, d), c, orc.LAW_NP, beta).reshape(-1)
        H[:, q] = -(np.repeat(mesh.V, d) * (fp - fm) / (2 * eps))
    fx = np.repeat(w.fixed.astype(bool), d)
    H[fx, :] = 0.0
    H[:, fx] = 0.0
    H[fx, fx] = 1.0
    rng = np.random.Generator(np.random.PCG64(9))
    for _ in range(3):
        x = rng.standard_normal((n, d))
        y = mesh.tangent_law(x, c, orc.LAW_NP, beta, ulin=ulin, fixed=w.fixed)
        np.testing.assert_allclose(y.reshape(-1), H @ x.reshape(-1), rtol=1e-6,
                                   atol=1e-6 * np.abs(y).max())
    # symmetric, as the Hessian of the energy
    z = rng.standard_normal((n, d))
    Hz = mesh.tangent_law(z, c, orc.LAW_NP, beta, ulin=ulin, fixed=w.fixed)
    Hx = mesh.tangent_law(x, c, orc.LAW_NP, beta, ulin=ulin, fixed=w.fixed)
    assert abs(np.sum(z * Hx) - np.sum(Hz * x)) <= 1e-12 * np.sqrt(np.sum(z * z) * np.sum(Hx * Hx))


def test_np_newton_reaches_equilibrium(orc):
    w, mesh, c = small_bar(orc, nx=16, ny=4, traction=3e-2)
    u_lin, info_lin = mesh.solve_implicit(w.u0, c, w.b, w.fixed, rtol=1e-12)
    assert info_lin["status"] == 0
    # the linear law through the general solver: the same answer in one step
    u0, info0 = mesh.solve_law(w.u0, c, w.b, w.fixed, orc.LAW_LINEAR, 1.0, rtol=1e-12)
    assert info0["status"] == 0 and info0["outer"] == 1
    assert np.linalg.norm(u0 - u_lin) <= 1e-10 * np.linalg.norm(u_lin)
    # NP with beta r about 0.1 at the linear solution: a few Newton steps
    beta = 0.1 / bond_r(mesh, u_lin).max()
    u, info = mesh.solve_law(w.u0, c, w.b, w.fixed, orc.LAW_NP, beta, rtol=1e-12)
    assert info["status"] == 0 and 2 <= info["outer"] <= 8, info
    _, rn = mesh.residual_law(u, c, w.b, orc.LAW_NP, beta, w.fixed)
    bn = np.linalg.norm((mesh.V[:, None] * w.b)[w.fixed == 0])
    assert rn <= 1e-12 * bn
    # the softening law yields more under the same load, by O(beta r)
    grow = np.linalg.norm(u) / np.linalg.norm(u_lin) - 1.0
    assert 1e-3 < grow < 0.2
    # the linear solution is not an NP equilibrium
    _, r_lin = mesh.residual_law(u_lin, c, w.b, orc.LAW_NP, beta, w.fixed)
    assert r_lin > 1e-4 * bn


def test_verlet_law_linear_is_verlet_and_np_conserves_energy(orc):
    """The integrator with the general law: the linear law reproduces the
    linearised integrator bit for bit; with the NP law (no damage, free
    plate) the total energy KE + sum V_i U_i drifts at second order in dt."""
    w = inputs.plate_2d(20, 3, seed=1, steps=0)
    mesh = orc.LawMesh(w.X, w.V, w.delta)
    c = orc.micromodulus(2, w.E, w.delta)
    v0 = inputs.random_field(mesh.n, 2, 71, scale=5e-2)
    a = mesh.start(w.u0, v0, c)
    b = mesh.start_law(w.u0, v0, c, orc.LAW_LINEAR, 1.0)
    mesh.verlet(a, c, w.rho, 0.0, w.dt, 40)
    mesh.verlet_law(b, c, w.rho, 0.0, w.dt, 40, orc.LAW_LINEAR, 1.0)
    assert np.array_equal(a["u"], b["u"]) and np.array_equal(a["v"], b["v"])
    # NP: beta set so that beta r reaches about 1 during the run
    probe = mesh.start(w.u0, v0, c)
    mesh.verlet(probe, c, w.rho, 0.0, w.dt, 40)
    beta = 1.0 / bond_r(mesh, probe["u"]).max()

    def drift(dt, steps):
        st = mesh.start_law(w.u0, v0, c, orc.LAW_NP, beta)
        e0 = mesh.kinetic(st["v"], w.rho) + mesh.energy_law(st["u"], c, orc.LAW_NP, beta)
        mesh.verlet_law(st, c, w.rho, 0.0, dt, steps, orc.LAW_NP, beta)
        e1 = mesh.kinetic(st["v"], w.rho) + mesh.energy_law(st["u"], c, orc.LAW_NP, beta)
        return abs(e1 - e0) / e0

    d1, d2 = drift(w.dt, 40), drift(w.dt / 2, 80)
    assert d1 < 1e-3
    assert 2.5 < d1 / d2 < 6.0                         # second order: ratio about 4
