"""Pins of the oracle's linear peridynamic solid (Algorithm 2, 3-d): under an
isotropic expansion the dilatation equals 3 eps at every node and the energy
density the classical (9/2) K eps^2; simple shear gives mu gamma^2/2 up to the
lattice error; the force is minus the gradient of the total strain energy
(which pins the scatter force against the energy written separately); the net
force vanishes; a finite rigid motion produces nothing; the Verlet steps
conserve energy to second order."""
import math

import numpy as np
import pytest

from paper_1806_06917_amd import inputs


def lattice(orc, m, N=None):
    N = N or (2 * m + 5)
    h = 1.0 / N
    X = inputs.grid_coords((N,) * 3, h)
    mesh = orc.LpsMesh(X, np.full(X.shape[0], h ** 3), m * h)
    centre = int(np.argmin(np.sum((X - X.mean(0)) ** 2, axis=1)))
    return mesh, centre


def jittered(orc, N, seed, m=3):
    h = 1.0 / N
    X = inputs.grid_coords((N,) * 3, h, jitter=0.05, seed=seed)
    rng = np.random.Generator(np.random.PCG64(seed + 100))
    V = h ** 3 * rng.uniform(0.8, 1.2, X.shape[0])
    return orc.LpsMesh(X, V, m * h)


@pytest.mark.parametrize("m", [3, 4])
def test_isotropic_expansion_is_exact(orc, m):
    K, mu = orc.lps_moduli(1.0, 0.3)
    mesh, c = lattice(orc, m)
    eps = 1e-3
    mm, th, f, W = mesh.lps(eps * mesh.X, K, mu)
    np.testing.assert_allclose(th, 3 * eps, rtol=1e-11)           # every node
    np.testing.assert_allclose(W, 4.5 * K * eps * eps, rtol=1e-10)
    assert np.abs(f[c]).max() <= 1e-12 * np.abs(f).max()          # interior balance
    # the weighted volume is the plain sum of |xi|^2 V_j
    i = np.repeat(np.arange(mesh.n), np.diff(mesh.row_ptr))
    xi = mesh.X[mesh.col] - mesh.X[i]
    np.testing.assert_allclose(mm, np.bincount(i, np.sum(xi * xi, 1) * mesh.V[mesh.col],
                                               minlength=mesh.n), rtol=1e-13)


@pytest.mark.parametrize("m", [3, 4, 5])
def test_simple_shear_energy_near_classical(orc, m):
    K, mu = orc.lps_moduli(1.0, 0.3)
    mesh, c = lattice(orc, m)
    g = 1e-4
    u = np.zeros_like(mesh.X)
    u[:, 0] = g * mesh.X[:, 1]
    _, th, _, W = mesh.lps(u, K, mu)
    assert 0.85 < W[c] / (mu * g * g / 2) < 1.15                   # lattice error only
    assert abs(th[c]) < 1e-4 * g                                  # no volume change


@pytest.mark.parametrize("dead", [0.0, 0.1])
def test_force_is_minus_energy_gradient(orc, dead):
    K, mu = orc.lps_moduli(1.0, 0.25)
    mesh = jittered(orc, 8, seed=91)
    rng = np.random.Generator(np.random.PCG64(92))
    alive = (rng.uniform(size=mesh.nnz) >= dead).astype(np.uint8)
    u = inputs.random_field(mesh.n, 3, 93, scale=2e-3)
    w = inputs.random_field(mesh.n, 3, 94, scale=1.0)
    eps = 1e-7
    P = lambda x: mesh.energy_lps(x, K, mu, alive)  # noqa: E731
    dpi = (P(u + eps * w) - P(u - eps * w)) / (2 * eps)
    f = mesh.lps(u, K, mu, alive)[2]
    rhs = -np.sum(mesh.V[:, None] * f * w)
    assert abs(dpi - rhs) <= 1e-6 * abs(rhs)


def test_net_force_zero_and_rigid_motion(orc):
    K, mu = orc.lps_moduli(1.0, 0.3)
    mesh = jittered(orc, 8, seed=95)
    u = inputs.random_field(mesh.n, 3, 96, scale=2e-3)
    f = mesh.lps(u, K, mu)[2]
    net = np.abs((mesh.V[:, None] * f).sum(0))
    assert np.all(net <= 1e-13 * np.sum(mesh.V[:, None] * np.abs(f), axis=0))
    a = 0.5
    R = np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1]])
    ur = mesh.X @ R.T - mesh.X + np.array([0.1, -0.2, 0.3])
    _, th, fr, W = mesh.lps(ur, K, mu)
    assert np.abs(th).max() < 1e-13
    assert np.abs(fr).max() <= 1e-10 * np.abs(f).max()
    assert np.abs(W).max() < 1e-20


def test_verlet_lps_second_order_energy(orc):
    K, mu = orc.lps_moduli(1.0, 0.3)
    mesh = jittered(orc, 8, seed=97)
    v0 = inputs.random_field(mesh.n, 3, 98, scale=1e-2)
    h = 1.0 / 8

    def drift(dt, steps):
        st = mesh.start_lps(np.zeros_like(v0), v0, K, mu)
        e0 = mesh.kinetic(st["v"], 1.0) + mesh.energy_lps(st["u"], K, mu)
        mesh.verlet_lps(st, K, mu, 1.0, dt, steps)
        e1 = mesh.kinetic(st["v"], 1.0) + mesh.energy_lps(st["u"], K, mu)
        return abs(e1 - e0) / e0

    d1, d2 = drift(0.02 * h, 40), drift(0.01 * h, 80)
    assert d1 < 1e-3
    assert 2.5 < d1 / d2 < 6.0
