"""Degenerate cases: zero-step requests and calls, an isolated node in the
peridynamic solid, a zero-load NP solve, an all-zero batch chunk, empty and
bondless meshes (rejected), and the smallest mesh with a bond (two nodes)."""
import numpy as np
import pytest

from conftest import say
from paper_1806_06917_amd import inputs
from test_gpu_parity import TOL64, TOLMIX, dev, host, read_state, relL2

pytestmark = pytest.mark.gpu


def test_zero_step_request_and_calls(gpu):
    torch, pd, ctx = gpu
    w = inputs.notched_plate_2d(N=24, m=3, steps=0, ramp_steps=0)
    w.u0 = inputs.random_field(w.n, 2, 141)
    w.v0 = inputs.random_field(w.n, 2, 142)
    say("zero-step request")
    srv = pd.Server(ctx, 1 << 30, chunk_steps=10)
    c = pd.micromodulus(2, w.E, w.delta)
    rid = srv.submit(w.X, w.V, pd.material(2, c, w.rho, w.s_c, "fp64"), w.delta, w.dt, 0,
                     u0=w.u0, v0=w.v0, keep_state=True)
    while srv.pump() != (0, 0):
        pass
    assert srv.info(rid)["state"] == pd.PD_REQ_DONE
    u, v = srv.result(rid, w.n, 2)
    assert np.array_equal(u, w.u0) and np.array_equal(v, w.v0)
    srv.close()
    # zero steps through every stepping call leave the state untouched
    nb = pd.Neighbors(ctx, dev(torch, w.X), w.delta)
    s = pd.Simulation(ctx, nb, pd.material(2, c, w.rho, 0.0, "fp64"), dev(torch, w.X),
                      dev(torch, w.V), dev(torch, w.u0), dev(torch, w.v0))
    s.step(0, w.dt)
    s.central_step(0, w.dt)
    b = pd.Batch(ctx)
    b.step([s], [0], [w.dt], 5)              # a chunk in which the instance takes no step
    b.close()
    u2, v2, _, info = read_state(torch, s, w.n, 2, nb.nnz)
    assert info["step"] == 0
    assert np.array_equal(u2, w.u0) and np.array_equal(v2, w.v0)
    s.close()
    nb.close()


def test_lps_isolated_node(gpu, orc):
    torch, pd, ctx = gpu
    X = inputs.grid_coords((6, 6, 6), 1.0 / 6)
    X = np.vstack([X, [[5.0, 5.0, 5.0]]])       # far from everything: no bonds
    V = np.full(X.shape[0], 1.0 / 216)
    u = inputs.random_field(X.shape[0], 3, 143, scale=1e-3)
    K, mu = orc.lps_moduli(1.0, 0.3)
    mesh = orc.LpsMesh(X, V, 2.0 / 6)
    _, th, ref_f, ref_W = mesh.lps(u, K, mu)
    say("LPS isolated node")
    nb = pd.Neighbors(ctx, dev(torch, X), 2.0 / 6)
    f = torch.zeros((X.shape[0], 3), dtype=torch.float64, device="cuda")
    W = torch.zeros(X.shape[0], dtype=torch.float64, device="cuda")
    pd.internal_force(ctx, nb, pd.material(3, 0.0, law="lps", bulk=K, shear=mu),
                      dev(torch, X), dev(torch, V), dev(torch, u), f, U=W)
    torch.cuda.synchronize()
    f, W = host(f), host(W)
    assert np.all(f[-1] == 0.0) and W[-1] == 0.0 and th[-1] == 0.0
    assert np.allclose(f, ref_f, rtol=0, atol=1e-12 * np.abs(ref_f).max())
    nb.close()


def test_np_solve_zero_load(gpu):
    torch, pd, ctx = gpu
    w = inputs.bar_2d(30, 6, 3, traction=0.0)
    nb = pd.Neighbors(ctx, dev(torch, w.X), w.delta)
    u = dev(torch, w.u0)
    say("NP zero load")
    res = pd.solve_implicit(ctx, nb, pd.material(2, pd.micromodulus(2, 1.0, w.delta), law="np",
                                                 beta=10.0),
                            dev(torch, w.X), dev(torch, w.V), dev(torch, w.b), u,
                            fixed=dev(torch, w.fixed), rtol=1e-10)
    assert res.outer == 0 and res.rel_residual == 0.0
    assert np.all(host(u) == 0.0)
    nb.close()


def test_empty_and_bondless_meshes_rejected(gpu):
    """No nodes: the neighbour build reports PD_EINVAL.  Nodes none of which
    lies within delta of another: the build gives nnz = 0, and every call
    that would compute on it (force, tangent, implicit solve, simulation)
    reports PD_EINVAL before any launch; the context stays usable."""
    torch, pd, ctx = gpu
    say("empty and bondless meshes")
    for dim in (2, 3):
        with pytest.raises(pd.PDError) as e:
            pd.Neighbors(ctx, torch.zeros((0, dim), dtype=torch.float64, device="cuda"), 1.0)
        assert e.value.status == pd.PD_EINVAL
        X = np.zeros((3, dim))
        X[:, 0] = [0.0, 1.0, 2.5]
        Xd, Vd = dev(torch, X), dev(torch, np.full(3, 0.1))
        y = torch.zeros((3, dim), dtype=torch.float64, device="cuda")
        mat = pd.material(dim, 1.0, 1.0, 0.0, "fp64")
        nb = pd.Neighbors(ctx, Xd, 0.9)
        assert nb.nnz == 0
        calls = [
            lambda: pd.internal_force(ctx, nb, mat, Xd, Vd, torch.zeros_like(y), y),
            lambda: pd.apply_tangent(ctx, nb, mat, Xd, Vd, torch.zeros_like(y), y),
            lambda: pd.solve_implicit(ctx, nb, mat, Xd, Vd, torch.ones_like(y), y),
            lambda: pd.Simulation(ctx, nb, mat, Xd, Vd, torch.zeros_like(y), torch.zeros_like(y)),
        ]
        for call in calls:
            with pytest.raises(pd.PDError) as e:
                call()
            assert e.value.status == pd.PD_EINVAL and "no bonds" in str(e.value)
        nb.close()
        # the same nodes with a horizon that reaches one neighbour each way
        nb = pd.Neighbors(ctx, Xd, 1.5)
        assert nb.nnz == 4
        pd.internal_force(ctx, nb, mat, Xd, Vd, torch.ones_like(y), y)
        torch.cuda.synchronize()
        assert np.all(host(y) == 0.0)            # a rigid translation
        nb.close()


def two_nodes(dim):
    X = np.array([[0.1, 0.2, 0.3][:dim], [0.13, 0.24, 0.3 + 0.012 * (dim == 3)][:dim]])
    V = np.array([0.7e-3, 1.3e-3])
    return X, V, 1.2 * np.linalg.norm(X[1] - X[0])


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("prec", ["fp64", "mixed", "fp32"])
def test_two_node_bond(gpu, orc, dim, prec):
    """The smallest mesh with a bond: two nodes.  Force and energy density
    against their closed form f_0 = c S e V_1, f_1 = -c S e V_0,
    U_i = (c/4) S^2 |xi| V_j; then 40 Verlet steps against the oracle, and a
    bond stretched past s_c that breaks at the first force evaluation, after
    which both nodes fly freely (u = u_0 + t v_0)."""
    torch, pd, ctx = gpu
    X, V, delta = two_nodes(dim)
    rng = np.random.Generator(np.random.PCG64(191 + dim))
    u = rng.uniform(-1e-3, 1e-3, (2, dim))
    c, rho = 2.0, 1.0
    xi, eta = X[1] - X[0], u[1] - u[0]
    L = np.linalg.norm(xi)
    S = eta @ xi / L ** 2
    e = xi / L
    f_ref = np.array([c * S * e * V[1], -c * S * e * V[0]])
    U_ref = np.array([c / 4 * S * S * L * V[1], c / 4 * S * S * L * V[0]])
    say("two-node bond", dim, prec)
    nb = pd.Neighbors(ctx, dev(torch, X), delta)
    assert nb.nnz == 2
    f = torch.zeros((2, dim), dtype=torch.float64, device="cuda")
    U = torch.zeros(2, dtype=torch.float64, device="cuda")
    pd.internal_force(ctx, nb, pd.material(dim, c, rho, 0.0, prec), dev(torch, X), dev(torch, V),
                      dev(torch, u), f, U=U)
    torch.cuda.synchronize()
    tol = TOL64 if prec == "fp64" else TOLMIX
    assert relL2(host(f), f_ref) <= tol and relL2(host(U), U_ref) <= tol
    # Verlet steps of the pair against the oracle
    v0 = rng.uniform(-1e-2, 1e-2, (2, dim))
    dt, steps = 1e-3, 40
    mesh = orc.Mesh(X, V, delta)
    st = mesh.start(u, v0, c)
    mesh.verlet(st, c, rho, 0.0, dt, steps)
    sim = pd.Simulation(ctx, nb, pd.material(dim, c, rho, 0.0, prec), dev(torch, X),
                        dev(torch, V), dev(torch, u), dev(torch, v0))
    sim.step(steps, dt)
    ug, vg, ag, _ = read_state(torch, sim, 2, dim, 2)
    sim.close()
    assert relL2(ug, st["u"]) <= tol and relL2(vg, st["v"]) <= tol and np.all(ag == 1)
    # a bond stretched to S + 0.05 > 0 breaks at the first force evaluation
    # when s_c is half that: free flight from then on
    ub = u.copy()
    ub[1] += 0.05 * xi
    Sb = (ub[1] - ub[0]) @ xi / L ** 2
    s_c = 0.5 * Sb
    assert Sb > s_c > 0.0
    sim = pd.Simulation(ctx, nb, pd.material(dim, c, rho, s_c, prec), dev(torch, X),
                        dev(torch, V), dev(torch, ub), dev(torch, v0))
    sim.step(steps, dt)
    ug, vg, ag, _ = read_state(torch, sim, 2, dim, 2)
    sim.close()
    nb.close()
    assert np.all(ag == 0)
    np.testing.assert_array_equal(vg, v0)
    np.testing.assert_allclose(ug, ub + steps * dt * v0, rtol=1e-12, atol=1e-15)


def test_server_fails_bondless_request_only(gpu):
    """A served request whose mesh has no bonds fails at admission with
    PD_EINVAL (the simulation cannot be created); the request behind it is
    served as usual."""
    torch, pd, ctx = gpu
    say("served bondless request")
    w = inputs.notched_plate_2d(N=24, m=3, steps=20, ramp_steps=0)
    c = pd.micromodulus(2, w.E, w.delta)
    Xb = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    srv = pd.Server(ctx, 1 << 30, chunk_steps=10)
    bad = srv.submit(Xb, np.full(3, 1e-2), pd.material(2, c, w.rho, 0.0, "fp64"), 0.5, w.dt, 20)
    good = srv.submit(w.X, w.V, pd.material(2, c, w.rho, 0.0, "fp64"), w.delta, w.dt, 20)
    while srv.pump() != (0, 0):
        pass
    fb, fg = srv.info(bad), srv.info(good)
    srv.close()
    assert fb["state"] == pd.PD_REQ_FAILED and fb["status"] == pd.PD_EINVAL
    assert fb["bonds"] == 0
    assert fg["state"] == pd.PD_REQ_DONE and fg["status"] == pd.PD_OK and fg["bonds"] > 0


def test_fp32_scope(gpu):
    """PD_FP32 covers the linearised law: the NP law, the exact stretch and the
    solid are rejected with PD_EINVAL, as are the tangent in FP32 and the
    register-staged tile kernel forced for an FP32 simulation (PD_ECAPACITY);
    the implicit solve accepts it as the mixed solve."""
    torch, pd, ctx = gpu
    X, V, delta = two_nodes(2)
    Xd, Vd = dev(torch, X), dev(torch, V)
    nb = pd.Neighbors(ctx, Xd, delta)
    u = torch.zeros((2, 2), dtype=torch.float64, device="cuda")
    f = torch.zeros_like(u)
    for kw in ({"law": "np", "beta": 1.0}, {"stretch": "exact"}):
        with pytest.raises(pd.PDError) as e:
            pd.internal_force(ctx, nb, pd.material(2, 1.0, 1.0, 0.0, "fp32", **kw), Xd, Vd, u, f)
        assert e.value.status == pd.PD_EINVAL
    with pytest.raises(pd.PDError) as e:
        pd.apply_tangent(ctx, nb, pd.material(2, 1.0, 1.0, 0.0, "fp32"), Xd, Vd, u, f)
    assert e.value.status == pd.PD_EINVAL
    ctx.set_tuning("tile", 0, 0)
    try:
        with pytest.raises(pd.PDError) as e:
            pd.Simulation(ctx, nb, pd.material(2, 1.0, 1.0, 0.0, "fp32"), Xd, Vd, None, None)
        assert e.value.status == pd.PD_ECAPACITY
    finally:
        ctx.set_tuning(0, 0, 0)
    nb.close()
    X3, V3, d3 = two_nodes(3)
    nb3 = pd.Neighbors(ctx, dev(torch, X3), d3)
    with pytest.raises(pd.PDError) as e:
        pd.Simulation(ctx, nb3, pd.material(3, 0.0, 1.0, 0.0, "fp32", law="lps", bulk=1.0,
                                            shear=0.5), dev(torch, X3), dev(torch, V3),
                      None, None)
    assert e.value.status == pd.PD_EINVAL
    nb3.close()
