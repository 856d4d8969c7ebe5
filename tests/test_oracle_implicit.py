"""Pins of the oracle's implicit path: the tangent operator against the
paper's central-difference tangent of the force, its symmetry and
definiteness, CG against a dense direct solve, and the quasi-static bar
against the classical linear-elastic solution (Section "Implicit time
integration", tangent equation and flow chart)."""
import json
import os

import numpy as np
import pytest

from paper_1806_06917_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small_bar(orc, nx=12, ny=4, m=3, clamp=3):
    w = inputs.bar_2d(nx, ny, m, traction=1e-3, clamp_cols=clamp)
    mesh = orc.Mesh(w.X, w.V, w.delta, method="brute")
    c = orc.micromodulus(2, w.E, w.delta)
    return w, mesh, c


def fd_tangent_dense(mesh, c, fixed, eps=1e-3):
    """K = df/du by the central difference of the force (tangent equation),
    then H = -V K on free rows, identity on fixed rows, zero fixed columns."""
    n, d = mesh.n, mesh.dim
    H = np.zeros((n * d, n * d))
    for q in range(n * d):
        e = np.zeros(n * d)
        e[q] = eps
        fp = mesh.force(e.reshape(n, d), c).reshape(-1)
        fm = mesh.force(-e.reshape(n, d), c).reshape(-1)
        H[:, q] = -(np.repeat(mesh.V, d) * (fp - fm) / (2 * eps))
    fx = np.repeat(fixed.astype(bool), d)
    H[fx, :] = 0.0
    H[:, fx] = 0.0
    H[fx, fx] = 1.0
    return H


def test_tangent_equals_central_difference_of_force(orc):
    w, mesh, c = small_bar(orc)
    H = fd_tangent_dense(mesh, c, w.fixed)
    rng = np.random.Generator(np.random.PCG64(3))
    for _ in range(3):
        x = rng.standard_normal((mesh.n, 2))
        y = mesh.apply_tangent(x, c, w.fixed)
        np.testing.assert_allclose(y.reshape(-1), H @ x.reshape(-1), rtol=1e-9,
                                   atol=1e-9 * np.abs(y).max())


def test_tangent_symmetric_positive(orc):
    wk = inputs.bar_2d(30, 8, 3, clamp_cols=3)
    mesh = orc.Mesh(wk.X, wk.V, wk.delta)
    c = orc.micromodulus(2, 1.0, wk.delta)
    rng = np.random.Generator(np.random.PCG64(4))
    z = rng.standard_normal((mesh.n, 2))
    x = rng.standard_normal((mesh.n, 2))
    Hz = mesh.apply_tangent(z, c, wk.fixed)
    Hx = mesh.apply_tangent(x, c, wk.fixed)
    assert abs(np.sum(z * Hx) - np.sum(Hz * x)) <= 1e-12 * np.sqrt(np.sum(z * z) * np.sum(Hx * Hx))
    free = wk.fixed == 0
    x[~free] = 0
    assert np.sum(x * mesh.apply_tangent(x, c, wk.fixed)) > 0
    # a rigid translation of the free nodes alone is resisted only through the
    # bonds to fixed nodes, so it is still positive
    t = np.zeros_like(x)
    t[free] = [1.0, 0.0]
    assert np.sum(t * mesh.apply_tangent(t, c, wk.fixed)) > 0
    # without any fixed node, rigid translations are in the null space
    assert np.abs(mesh.apply_tangent(np.ones_like(x), c)).max() == 0.0


def test_cg_matches_dense_solve(orc):
    w, mesh, c = small_bar(orc, nx=14, ny=5)
    H = fd_tangent_dense(mesh, c, w.fixed)
    rng = np.random.Generator(np.random.PCG64(8))
    rhs = rng.standard_normal((mesh.n, 2))
    rhs[w.fixed.astype(bool)] = 0.0
    ref = np.linalg.solve(H, rhs.reshape(-1)).reshape(mesh.n, 2)
    x, info = mesh.cg(rhs, c, w.fixed, rtol=1e-14)
    assert info["status"] == 0
    assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)


def test_implicit_solution_dense_and_residual(orc):
    w, mesh, c = small_bar(orc, nx=16, ny=4)
    u, info = mesh.solve_implicit(w.u0, c, w.b, w.fixed, rtol=1e-12)
    assert info["status"] == 0 and info["relres"] <= 1e-12
    # dense: H u = V b on free DOFs
    H = fd_tangent_dense(mesh, c, w.fixed)
    rhs = (mesh.V[:, None] * w.b)
    rhs[w.fixed.astype(bool)] = 0
    ref = np.linalg.solve(H, rhs.reshape(-1)).reshape(mesh.n, 2)
    assert np.linalg.norm(u - ref) <= 1e-8 * np.linalg.norm(ref)


def test_ccm_golden_constants():
    """The classical 1-d bar values printed in the paper's implicit validation."""
    with open(os.path.join(GOLDEN, "ccm_1d_bar.json")) as fh:
        g = json.load(fh)
    stress = g["F"] / g["A"]
    strain = stress / g["E"]
    energy = stress ** 2 / (2 * g["E"])
    assert np.isclose(stress, g["stress"], rtol=1e-15)
    assert np.isclose(strain, g["strain"], rtol=1e-15)
    assert np.isclose(energy, g["energy_density"], rtol=1e-15)


@pytest.mark.slow
def test_bar_interior_strain_matches_classical(orc):
    """Bar under end traction t, clamped at the left: away from both ends
    the axial strain approaches t/E (modelling error of the bond-based
    discretisation, surface effects near the ends, a few percent)."""
    wk = inputs.bar_2d(120, 12, 3, traction=1e-3)
    mesh = orc.Mesh(wk.X, wk.V, wk.delta)
    c = orc.micromodulus(2, wk.E, wk.delta)
    u, info = mesh.solve_implicit(wk.u0, c, wk.b, wk.fixed, rtol=1e-10)
    assert info["status"] == 0
    x = wk.X[:, 0]
    H = 1.0
    sel = (x > 3 * wk.h + 2 * H) & (x < x.max() - 2 * H)
    slope = np.polyfit(x[sel], u[sel, 0], 1)[0]
    assert abs(slope / (wk.traction / wk.E) - 1) < 0.10
