"""Pins of the oracle's partial volumes (the correction the paper names; the
partial-area reading: neighbours out to R = delta + h/2, V_j scaled by
clamp((R - |xi|)/h, 0, 1)): hand values of the weight on a two-node mesh,
no change when switched off, a better worst-case quadrature of the horizon
ball, and the force-energy identity for the pairwise law and the solid."""
import numpy as np
import pytest

from paper_1806_06917_amd import inputs


def test_weight_by_hand(orc):
    # delta = 1, h = 0.2: neighbours out to R = 1.1; weights at |xi| = 0.85,
    # 0.95, 1.05 are 1, 0.75 and 0.25
    for d, wgt in ((0.85, 1.0), (0.95, 0.75), (1.05, 0.25)):
        X = np.array([[0.0, 0.0], [0.6 * d, 0.8 * d]])
        m = orc.LawMesh(X, np.array([0.3, 0.5]), 1.1, method="brute")
        u = np.array([[0.0, 0.0], [0.6e-3, 0.8e-3]])
        f0 = m.force_law(u, 2.0, orc.LAW_LINEAR, 1.0)
        f1 = m.force_law(u, 2.0, orc.LAW_LINEAR, 1.0, pv_h=0.2)
        np.testing.assert_allclose(f1, wgt * f0, rtol=1e-13)
        assert np.array_equal(m.force_law(u, 2.0, orc.LAW_LINEAR, 1.0, pv_h=0.0), f0)


@pytest.mark.parametrize("dim,ms", [(2, (3, 4, 5, 6)), (3, (3, 4))])
def test_ball_quadrature_improves(orc, dim, ms):
    """Energy density of an isotropic expansion at an interior lattice node
    against the continuum value: the worst relative error over the horizons
    is smaller with partial volumes."""
    errs_pv, errs = [], []
    for m in ms:
        N = 2 * m + 7
        h = 1.0 / N
        delta = m * h
        X = inputs.grid_coords((N,) * dim, h)
        V = np.full(len(X), h ** dim)
        c = orc.micromodulus(dim, 1.0, delta)
        eps = 1e-3
        cen = int(np.argmin(np.sum((X - X.mean(0)) ** 2, 1)))
        W = 1.5 * eps * eps if dim == 2 else 4.5 * (1.0 / 1.5) * eps * eps
        _, Up = orc.LawMesh(X, V, delta + h / 2).force_law(eps * X, c, orc.LAW_LINEAR, 1.0,
                                                           energy=True, pv_h=h)
        _, U0 = orc.LawMesh(X, V, delta).force_law(eps * X, c, orc.LAW_LINEAR, 1.0, energy=True)
        errs_pv.append(abs(Up[cen] / W - 1))
        errs.append(abs(U0[cen] / W - 1))
    assert max(errs_pv) < 0.7 * max(errs)
    assert max(errs_pv) < (0.03 if dim == 2 else 0.07)


@pytest.mark.parametrize("kind", ["np", "lps"])
def test_force_is_minus_energy_gradient_with_pv(orc, kind):
    dim = 3 if kind == "lps" else 2
    N = 8 if dim == 3 else 16
    h = 1.0 / N
    X = inputs.grid_coords((N,) * dim, h, jitter=0.05, seed=151)
    V = h ** dim * np.random.Generator(np.random.PCG64(152)).uniform(0.8, 1.2, len(X))
    R = 3 * h + h / 2
    u = inputs.random_field(len(X), dim, 153, scale=2e-3)
    w = inputs.random_field(len(X), dim, 154, scale=1.0)
    eps = 1e-7
    if kind == "lps":
        mesh = orc.LpsMesh(X, V, R)
        K, mu = orc.lps_moduli(1.0, 0.3)
        P = lambda x: mesh.energy_lps(x, K, mu, pv_h=h)  # noqa: E731
        f = mesh.lps(u, K, mu, pv_h=h)[2]
        # the isotropic expansion stays exact: theta = 3 eps with the same weights in m
        th = mesh.lps(1e-3 * X, K, mu, pv_h=h)[1]
        np.testing.assert_allclose(th, 3e-3, rtol=1e-10)
    else:
        mesh = orc.LawMesh(X, V, R)
        c = 1.7
        beta = 2e4
        P = lambda x: mesh.energy_law(x, c, orc.LAW_NP, beta, pv_h=h)  # noqa: E731
        f = mesh.force_law(u, c, orc.LAW_NP, beta, pv_h=h)
    dpi = (P(u + eps * w) - P(u - eps * w)) / (2 * eps)
    rhs = -np.sum(V[:, None] * f * w)
    assert abs(dpi - rhs) <= 1e-6 * abs(rhs)
