"""GPU parity of the influence function (the 1-d validation's
J(r) = c1 r exp(-r^2/c2), r = |xi|/delta, on every bond) against the FP64
oracle: force and energy on a 2-d plate for the linear and NP laws and the
exact stretch, with and without partial volumes; explicit steps on the 1-d
study's line; the 1-d convergence study itself, whose rates must match what
the quadrature of the horizon integral predicts; the calls that do not take
J reject it.  Bars: rel-L2 1e-12 FP64, 1e-5 mixed."""
import math

import numpy as np
import pytest

from conftest import say
from paper_1806_06917_amd import inputs
from test_gpu_parity import TOL64, TOLMIX, dev, host, read_state, relL2

pytestmark = pytest.mark.gpu

J = inputs.INFLUENCE_1D


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("kind,pv", [("linear", False), ("np", False), ("exact", False),
                                     ("np", True)])
def test_force_energy_parity(gpu, orc, kind, pv, prec):
    torch, pd, ctx = gpu
    N = 40
    h = 1.0 / N
    X = inputs.grid_coords((N, N), h, jitter=0.05, seed=181)
    V = h * h * np.random.Generator(np.random.PCG64(182)).uniform(0.9, 1.1, len(X))
    u = inputs.random_field(len(X), 2, 183, scale=2e-2 * h)
    delta = 3 * h
    pv_h = h if pv else 0.0
    R = delta + pv_h / 2
    c = orc.micromodulus(2, 1.0, delta)
    law = orc.LAW_NP if kind == "np" else orc.LAW_LINEAR
    sk = orc.STRETCH_EXACT if kind == "exact" else orc.STRETCH_LINEARISED
    beta = 3e3
    ref_f, ref_U = orc.LawMesh(X, V, R).force_law(u, c, law, beta, sk, energy=True, pv_h=pv_h,
                                                   j=J)
    say("influence function", kind, "pv" if pv else "", prec)
    nb = pd.Neighbors(ctx, dev(torch, X), R)
    mat = pd.material(2, c, 1.0, 0.0, prec, law="np" if kind == "np" else "linear", beta=beta,
                      stretch="exact" if kind == "exact" else "linearised", pv_h=pv_h, j=J)
    f = torch.zeros((len(X), 2), dtype=torch.float64, device="cuda")
    U = torch.zeros(len(X), dtype=torch.float64, device="cuda")
    pd.internal_force(ctx, nb, mat, dev(torch, X), dev(torch, V), dev(torch, u), f, U=U)
    torch.cuda.synchronize()
    nb.close()
    tol = TOL64 if prec == "fp64" else TOLMIX
    assert relL2(host(f), ref_f) <= tol
    assert relL2(host(U), ref_U) <= tol
    # J is really applied
    f0 = orc.LawMesh(X, V, R).force_law(u, c, law, beta, sk, pv_h=pv_h)
    assert relL2(ref_f, f0) > 0.1


@pytest.mark.parametrize("law", ["linear", "np"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_line_steps_parity(gpu, orc, law, prec):
    """300 Verlet steps of the 1-d study's line (h = delta/4, IC 2) against
    the oracle's steps with J."""
    torch, pd, ctx = gpu
    w = inputs.convergence_line(4, 2)
    c = 2.0 / w.delta ** 2
    lw = orc.LAW_NP if law == "np" else orc.LAW_LINEAR
    mesh = orc.LawMesh(w.X, w.V, w.delta)
    st = mesh.start_law(w.u0, w.v0, c, lw, 1.0)
    st["f"] = mesh.force_law(st["u"], c, lw, 1.0, j=J)
    steps = 300
    mesh.steps_j(st, c, 1.0, 0.0, w.dt, steps, J, lw, 1.0, bc_kind=w.bc_kind, bc_vel=w.bc_vel)
    say("line steps", law, prec)
    nb = pd.Neighbors(ctx, dev(torch, w.X), w.delta)
    sim = pd.Simulation(ctx, nb, pd.material(2, c, 1.0, 0.0, prec, law=law, beta=1.0, j=J),
                        dev(torch, w.X), dev(torch, w.V), dev(torch, w.u0), dev(torch, w.v0),
                        bc_kind=dev(torch, w.bc_kind), bc_vel=dev(torch, w.bc_vel))
    assert sim.info()["kernel"] == "gather"
    sim.step(steps, w.dt)
    u, v, _, _ = read_state(torch, sim, w.n, 2, nb.nnz)
    sim.close()
    nb.close()
    tol = TOL64 if prec == "fp64" else TOLMIX
    assert relL2(u, st["u"]) <= tol
    assert relL2(v, st["v"]) <= tol
    assert np.all(u[:, 1] == 0.0)                          # motion along the line only
    assert np.all(u[w.bc_kind == inputs.BC_CLAMPED] == 0.0)


@pytest.mark.parametrize("law", ["linear", "np"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_line_central_steps_parity(gpu, orc, law, prec):
    """300 central-difference steps (pd_central_step) of the 1-d study's line
    with J (h = delta/4, IC 2, clamped collars) against the oracle's
    central-difference steps with J."""
    torch, pd, ctx = gpu
    w = inputs.convergence_line(4, 2)
    c = 2.0 / w.delta ** 2
    lw = orc.LAW_NP if law == "np" else orc.LAW_LINEAR
    mesh = orc.LawMesh(w.X, w.V, w.delta)
    st = mesh.start_law(w.u0, w.v0, c, lw, 1.0)
    st["f"] = mesh.force_law(st["u"], c, lw, 1.0, j=J)
    steps = 300
    mesh.steps_j(st, c, 1.0, 0.0, w.dt, steps, J, lw, 1.0, central=True, bc_kind=w.bc_kind,
                 bc_vel=w.bc_vel)
    say("line central steps", law, prec)
    nb = pd.Neighbors(ctx, dev(torch, w.X), w.delta)
    sim = pd.Simulation(ctx, nb, pd.material(2, c, 1.0, 0.0, prec, law=law, beta=1.0, j=J),
                        dev(torch, w.X), dev(torch, w.V), dev(torch, w.u0), dev(torch, w.v0),
                        bc_kind=dev(torch, w.bc_kind), bc_vel=dev(torch, w.bc_vel))
    sim.central_step(steps, w.dt)
    u, v, _, info = read_state(torch, sim, w.n, 2, nb.nnz)
    sim.close()
    nb.close()
    assert info["step"] == steps
    tol = TOL64 if prec == "fp64" else TOLMIX
    assert relL2(u, st["u"]) <= tol
    assert relL2(v, st["v"]) <= tol
    assert np.all(u[:, 1] == 0.0)
    assert np.all(u[w.bc_kind == inputs.BC_CLAMPED] == 0.0)


def quadrature_rates(pv):
    """Rates of the two mesh sets predicted by the bond sum's quadrature of
    the horizon integral: for smooth u the line's operator is 2 u'' R(m),
    R(m) = (1/m) sum_k w_k g(k/m) with g(t) = J(t) t, m = delta/h, all
    weights 1 (no partial volumes: a right-endpoint rule, whose error is
    g(1)/(2m) + O(1/m^2), with g(1) = J(1) != 0) or the node at distance
    delta weighted 1/2 (partial volumes: the trapezoidal rule, O(1/m^2)).
    The meshes differ mainly through this effective modulus, so the rate
    of a set is log2 of the ratio of successive differences of R."""
    c1, c2 = J
    g = lambda t: c1 * t * math.exp(-t * t / c2) * t  # noqa: E731
    R = [sum((0.5 if (pv and k == m) else 1.0) * g(k / m) for k in range(1, m + 1)) / m
         for m in (2, 4, 8, 16)]
    d = [R[k] - R[k + 1] for k in range(3)]
    return math.log2(d[0] / d[1]), math.log2(d[1] / d[2])


@pytest.mark.parametrize("pv", [False, True])
@pytest.mark.parametrize("law,ic", [("linear", 1), ("np", 2)])
def test_line_convergence_rates(gpu, law, ic, pv):
    """The 1-d study on the GPU: rates at t = 0.25 and 0.5 within 0.12 of the
    quadrature prediction (about 0.57 and 0.84 without partial volumes, 2.07
    and 2.02 with them), and set 2 above set 1 without them, as the paper
    observes."""
    torch, pd, _ = gpu
    import bench
    p1, p2 = quadrature_rates(pv)
    say("1-d convergence", law, ic, "pv" if pv else "", "predicted", round(p1, 3), round(p2, 3))
    res = bench.convergence_1d(torch, pd, law, ic, t_end=0.5, every=0.25, pv=pv)
    assert res["steps"] == 50000 and len(res["rates"]) == 2
    for r in res["rates"]:
        assert all(d > 0.0 for d in r["diff"])             # the meshes do differ
        assert abs(r["alpha_set1"] - p1) < 0.12, (r, p1)
        assert abs(r["alpha_set2"] - p2) < 0.12, (r, p2)
        if not pv:
            assert r["alpha_set2"] > r["alpha_set1"]


def test_rejections(gpu):
    torch, pd, ctx = gpu
    N = 12
    h = 1.0 / N
    X = inputs.grid_coords((N, N), h)
    V = np.full(len(X), h * h)
    nb = pd.Neighbors(ctx, dev(torch, X), 3 * h)
    y = torch.zeros((len(X), 2), dtype=torch.float64, device="cuda")
    say("influence rejections")
    for bad in (dict(j=J), ):
        mat = pd.material(2, 1.0, **bad)
        with pytest.raises(pd.PDError) as e:
            pd.apply_tangent(ctx, nb, mat, dev(torch, X), dev(torch, V), y, torch.zeros_like(y))
        assert e.value.status == pd.PD_EINVAL
        b = torch.zeros_like(y)
        with pytest.raises(pd.PDError) as e:
            pd.solve_implicit(ctx, nb, mat, dev(torch, X), dev(torch, V), b, torch.zeros_like(y))
        assert e.value.status == pd.PD_EINVAL
    with pytest.raises(pd.PDError) as e:      # c2 must be >= 0
        pd.internal_force(ctx, nb, pd.material(2, 1.0, j=(1.0, -0.4)), dev(torch, X),
                          dev(torch, V), torch.zeros_like(y), y)
    assert e.value.status == pd.PD_EINVAL
    nb.close()
    X3 = inputs.grid_coords((6, 6, 6), 1.0 / 6)
    nb3 = pd.Neighbors(ctx, dev(torch, X3), 0.5)
    y3 = torch.zeros((len(X3), 3), dtype=torch.float64, device="cuda")
    with pytest.raises(pd.PDError) as e:      # not for the solid
        pd.internal_force(ctx, nb3, pd.material(3, 0.0, law="lps", bulk=1.0, shear=0.5, j=J),
                          dev(torch, X3), dev(torch, np.full(len(X3), 1.0 / 216)),
                          torch.zeros_like(y3), y3)
    assert e.value.status == pd.PD_EINVAL
    nb3.close()
