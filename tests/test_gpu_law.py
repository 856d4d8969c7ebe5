"""GPU parity of the general pairwise law (the NP potential of the paper's
validation section in Algorithm 1, and the exact-stretch variant) against the
FP64 oracle: force and energy, damage under the exact stretch, explicit
steps, the tangent linearised at a strained state, and the Newton-Krylov
quasi-static solve.  Bars as in the linear parity tests: rel-L2 1e-12 in
FP64 and 1e-5 mixed, flags equal outside the 1e-6 band."""
import numpy as np
import pytest

from conftest import say
from paper_1806_06917_amd import inputs
from test_gpu_parity import TOL64, TOLMIX, bar_case, dev, force_case, host, read_state, relL2
from test_oracle_law import bond_r

pytestmark = pytest.mark.gpu


def codes(orc, law, stretch):
    return ({"np": orc.LAW_NP, "linear": orc.LAW_LINEAR}[law],
            {"linearised": orc.STRETCH_LINEARISED, "exact": orc.STRETCH_EXACT}[stretch])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("dim,law,stretch", [(2, "np", "linearised"), (3, "np", "linearised"),
                                             (2, "np", "exact"), (3, "linear", "exact"),
                                             (2, "linear", "exact")])
def test_law_force_energy_parity(gpu, orc, dim, law, stretch, prec):
    torch, pd, ctx = gpu
    X, V, u, delta = force_case(81, dim, 40 if dim == 2 else 14, 3, 0.05, scale=2e-2)
    mesh = orc.LawMesh(X, V, delta)
    lw, sk = codes(orc, law, stretch)
    beta = 1.0 / bond_r(mesh, u, sk).max()            # beta r up to 1
    c = orc.micromodulus(dim, 1.0, delta)
    ref_f, ref_U = mesh.force_law(u, c, lw, beta, sk, energy=True)
    say("law force", dim, law, stretch, prec)
    nb = pd.Neighbors(ctx, dev(torch, X), delta)
    mat = pd.material(dim, pd.micromodulus(dim, 1.0, delta), 1.0, 0.0, prec, law=law,
                      beta=beta, stretch=stretch)
    f = torch.zeros((mesh.n, dim), dtype=torch.float64, device="cuda")
    U = torch.zeros(mesh.n, dtype=torch.float64, device="cuda")
    pd.internal_force(ctx, nb, mat, dev(torch, X), dev(torch, V), dev(torch, u), f, U=U)
    torch.cuda.synchronize()
    tol = TOL64 if prec == "fp64" else TOLMIX
    assert relL2(host(f), ref_f) <= tol
    assert relL2(host(U), ref_U) <= tol


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_exact_stretch_damage_parity(gpu, orc, prec):
    torch, pd, ctx = gpu
    X, V, u, delta = force_case(83, 2, 48, 3, 0.05, scale=0.05)
    mesh = orc.LawMesh(X, V, delta)
    c = orc.micromodulus(2, 1.0, delta)
    i = np.repeat(np.arange(mesh.n), np.diff(mesh.row_ptr))
    j = mesh.col.astype(np.int64)
    xi = X[j] - X[i]
    L = np.linalg.norm(xi, axis=1)
    S = (np.linalg.norm(xi + u[j] - u[i], axis=1) - L) / L
    s_c = float(np.quantile(S, 0.9))
    band = np.abs(S / s_c - 1) <= 1e-6
    ref_alive = mesh.all_alive().copy()
    ref_f = mesh.force_law(u, c, orc.LAW_LINEAR, 1.0, orc.STRETCH_EXACT, s_c, ref_alive)
    assert 0 < np.count_nonzero(ref_alive == 0) < mesh.nnz
    say("exact-stretch damage", prec)
    nb = pd.Neighbors(ctx, dev(torch, X), delta)
    mat = pd.material(2, pd.micromodulus(2, 1.0, delta), 1.0, s_c, prec, stretch="exact")
    f = torch.zeros((mesh.n, 2), dtype=torch.float64, device="cuda")
    al = dev(torch, mesh.all_alive())
    pd.internal_force(ctx, nb, mat, dev(torch, X), dev(torch, V), dev(torch, u), f, alive=al)
    torch.cuda.synchronize()
    got = host(al)
    assert np.array_equal(got[~band], ref_alive[~band])
    if np.array_equal(got, ref_alive):
        assert relL2(host(f), ref_f) <= (TOL64 if prec == "fp64" else TOLMIX)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("law,stretch", [("np", "linearised"), ("linear", "exact"),
                                         ("np", "exact")])
def test_law_explicit_steps(gpu, orc, law, stretch, prec):
    """A free-moving plate (no damage) for 40 steps under the general law."""
    torch, pd, ctx = gpu
    w = inputs.plate_2d(36, 3, seed=4, steps=0)
    w.v0 = inputs.random_field(w.n, 2, 85, scale=5e-2)
    mesh = orc.LawMesh(w.X, w.V, w.delta)
    c = orc.micromodulus(2, w.E, w.delta)
    lw, sk = codes(orc, law, stretch)
    probe = mesh.start(w.u0, w.v0, c)
    mesh.verlet(probe, c, w.rho, 0.0, w.dt, 40)
    beta = 1.0 / bond_r(mesh, probe["u"], sk).max()
    st = mesh.start_law(w.u0, w.v0, c, lw, beta, sk)
    mesh.verlet_law(st, c, w.rho, 0.0, w.dt, 40, lw, beta, sk)
    say("law steps", law, stretch, prec)
    nb = pd.Neighbors(ctx, dev(torch, w.X), w.delta)
    mat = pd.material(2, pd.micromodulus(2, w.E, w.delta), w.rho, 0.0, prec, law=law,
                      beta=beta, stretch=stretch)
    sim = pd.Simulation(ctx, nb, mat, dev(torch, w.X), dev(torch, w.V), dev(torch, w.u0),
                        dev(torch, w.v0))
    # the NP law (linearised stretch, no damage) runs on the streamed kernel
    assert sim.info()["kernel"] == ("stream" if (law, stretch) == ("np", "linearised")
                                    else "gather")
    sim.step(40, w.dt)
    u, v, _, info = read_state(torch, sim, w.n, 2, nb.nnz)
    sim.close()
    nb.close()
    assert info["step"] == 40
    tol = TOL64 if prec == "fp64" else TOLMIX
    assert relL2(u, st["u"]) <= tol
    assert relL2(v, st["v"]) <= tol


@pytest.mark.parametrize("prec,tol", [("fp64", TOL64), ("mixed", TOLMIX)])
def test_np_tangent_at_parity(gpu, orc, prec, tol):
    torch, pd, ctx = gpu
    w = bar_case(61, 9)
    mesh = orc.LawMesh(w.X, w.V, w.delta)
    c = orc.micromodulus(2, 1.0, w.delta)
    ulin, _ = mesh.solve_implicit(w.u0, c, w.b, w.fixed, rtol=1e-12)
    ulin = 30.0 * ulin
    beta = 0.3 / bond_r(mesh, ulin).max()
    x = inputs.random_field(w.n, 2, 87, scale=1.0)
    alive = (np.random.Generator(np.random.PCG64(5)).uniform(size=mesh.nnz) > 0.05).astype(np.uint8)
    ref = mesh.tangent_law(x, c, orc.LAW_NP, beta, ulin=ulin, fixed=w.fixed, alive=alive)
    say("NP tangent", prec)
    nb = pd.Neighbors(ctx, dev(torch, w.X), w.delta)
    mat = pd.material(2, pd.micromodulus(2, 1.0, w.delta), 1.0, 0.0, prec, law="np", beta=beta)
    y = torch.zeros((w.n, 2), dtype=torch.float64, device="cuda")
    pd.apply_tangent_at(ctx, nb, mat, dev(torch, w.X), dev(torch, w.V), dev(torch, ulin),
                        dev(torch, x), y, alive=dev(torch, alive), fixed=dev(torch, w.fixed))
    torch.cuda.synchronize()
    assert relL2(host(y), ref) <= tol
    # the linear law ignores the linearisation point
    lin = pd.material(2, pd.micromodulus(2, 1.0, w.delta), 1.0, 0.0, prec)
    y2 = torch.zeros_like(y)
    pd.apply_tangent_at(ctx, nb, lin, dev(torch, w.X), dev(torch, w.V), dev(torch, ulin),
                        dev(torch, x), y2, alive=dev(torch, alive), fixed=dev(torch, w.fixed))
    torch.cuda.synchronize()
    assert relL2(host(y2), mesh.apply_tangent(x, c, w.fixed, alive)) <= tol


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_np_newton_krylov_solve(gpu, orc, prec):
    """NP quasi-static bar: the GPU Newton-Krylov solution has the FP64
    residual 1e-10 (evaluated by the oracle) and matches the oracle's Newton
    solution."""
    torch, pd, ctx = gpu
    w = inputs.bar_2d(120, 12, 3, traction=1e-2)
    mesh = orc.LawMesh(w.X, w.V, w.delta)
    c = orc.micromodulus(2, 1.0, w.delta)
    u_lin, _ = mesh.solve_implicit(w.u0, c, w.b, w.fixed, rtol=1e-12)
    beta = 0.1 / bond_r(mesh, u_lin).max()
    ref, rinfo = mesh.solve_law(w.u0, c, w.b, w.fixed, orc.LAW_NP, beta, rtol=1e-12)
    assert rinfo["status"] == 0 and rinfo["outer"] >= 2
    say("NP Newton-Krylov", prec)
    nb = pd.Neighbors(ctx, dev(torch, w.X), w.delta)
    mat = pd.material(2, pd.micromodulus(2, 1.0, w.delta), 1.0, 0.0, prec, law="np", beta=beta)
    u = dev(torch, w.u0)
    res = pd.solve_implicit(ctx, nb, mat, dev(torch, w.X), dev(torch, w.V), dev(torch, w.b), u,
                            fixed=dev(torch, w.fixed), rtol=1e-10)
    got = host(u)
    _, rn = mesh.residual_law(got, c, w.b, orc.LAW_NP, beta, w.fixed)
    bn = np.linalg.norm((w.V[:, None] * w.b)[w.fixed == 0])
    assert res.rel_residual <= 1e-10 and res.outer >= 2
    assert rn / bn <= 2e-10
    assert relL2(got, ref) <= 1e-6
    assert relL2(got, u_lin) > 1e-4                   # the law did change the answer


def test_law_argument_errors(gpu):
    torch, pd, ctx = gpu
    w = bar_case(30, 6)
    nb = pd.Neighbors(ctx, dev(torch, w.X), w.delta)
    X, V = dev(torch, w.X), dev(torch, w.V)
    x = dev(torch, np.ones((w.n, 2)))
    y = torch.zeros_like(x)
    c = pd.micromodulus(2, 1.0, w.delta)
    for bad in (pd.material(2, c, law="np", beta=0.0), pd.material(2, c, law=7),
                pd.material(2, c, stretch=3)):
        with pytest.raises(pd.PDError) as e:
            pd.internal_force(ctx, nb, bad, X, V, x, y)
        assert e.value.status == pd.PD_EINVAL
    exact = pd.material(2, c, stretch="exact")
    with pytest.raises(pd.PDError) as e:
        pd.apply_tangent(ctx, nb, exact, X, V, x, y)
    assert e.value.status == pd.PD_EINVAL
    with pytest.raises(pd.PDError) as e:
        pd.solve_implicit(ctx, nb, exact, X, V, dev(torch, w.b), x, fixed=dev(torch, w.fixed))
    assert e.value.status == pd.PD_EINVAL
    ctx.set_tuning("stream", 0, 0)
    try:
        with pytest.raises(pd.PDError) as e:
            pd.Simulation(ctx, nb, pd.material(2, c, law="np", beta=1.0, stretch="exact"), X, V)
        assert e.value.status == pd.PD_ECAPACITY
    finally:
        ctx.set_tuning(0, 0, 0)
    ctx.set_tuning("tile", 0, 0)
    try:
        with pytest.raises(pd.PDError) as e:
            pd.Simulation(ctx, nb, pd.material(2, c, law="np", beta=1.0), X, V)
        assert e.value.status == pd.PD_ECAPACITY
    finally:
        ctx.set_tuning(0, 0, 0)
    nb.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_np_stream_equals_gather_within_tolerance_and_batches(gpu, orc, prec):
    """The NP law on the streamed kernel against the same law forced onto the
    gather kernel and against the oracle, and NP simulations batched in one
    launch equal the same simulations stepped alone, bit for bit."""
    torch, pd, ctx = gpu
    ws = [inputs.plate_2d(N, 3, seed=s, steps=0) for N, s in ((36, 4), (28, 5))]
    for k, w in enumerate(ws):
        w.v0 = inputs.random_field(w.n, 2, 110 + k, scale=5e-2)
    beta = 2e4
    ctx.set_lanes(4)
    try:
        alone, sims = [], []
        for k, w in enumerate(ws):
            nb = pd.Neighbors(ctx, dev(torch, w.X), w.delta)
            mat = pd.material(2, pd.micromodulus(2, w.E, w.delta), w.rho, 0.0, prec, law="np",
                              beta=beta)
            s = pd.Simulation(ctx, nb, mat, dev(torch, w.X), dev(torch, w.V), None,
                              dev(torch, w.v0))
            assert s.info()["kernel"] == "stream"
            s.step(30, w.dt)
            alone.append(read_state(torch, s, w.n, 2, nb.nnz)[:2])
            s.close()
            sims.append((nb, pd.Simulation(ctx, nb, mat, dev(torch, w.X), dev(torch, w.V), None,
                                           dev(torch, w.v0))))
        say("NP batch", prec)
        b = pd.Batch(ctx)
        b.step([s for _, s in sims], [30, 30], [w.dt for w in ws], 30)
        b.close()
        for (nb, s), w, ref in zip(sims, ws, alone):
            got = read_state(torch, s, w.n, 2, nb.nnz)[:2]
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
            s.close()
        # the same law on the gather kernel, and the oracle
        w = ws[0]
        ctx.set_tuning("gather", 0, 0)
        nb, _ = sims[0]
        mat = pd.material(2, pd.micromodulus(2, w.E, w.delta), w.rho, 0.0, prec, law="np",
                          beta=beta)
        s = pd.Simulation(ctx, nb, mat, dev(torch, w.X), dev(torch, w.V), None, dev(torch, w.v0))
        assert s.info()["kernel"] == "gather"
        s.step(30, w.dt)
        gat = read_state(torch, s, w.n, 2, nb.nnz)[:2]
        s.close()
    finally:
        ctx.set_lanes(0)
        ctx.set_tuning(0, 0, 0)
    for nb, _ in sims:
        nb.close()
    mesh = orc.LawMesh(w.X, w.V, w.delta)
    c = orc.micromodulus(2, w.E, w.delta)
    st = mesh.start_law(w.u0, w.v0, c, orc.LAW_NP, beta)
    mesh.verlet_law(st, c, w.rho, 0.0, w.dt, 30, orc.LAW_NP, beta)
    tol = TOL64 if prec == "fp64" else TOLMIX
    for got in (alone[0], gat):
        assert relL2(got[0], st["u"]) <= tol
        assert relL2(got[1], st["v"]) <= tol


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_np_streamed_full_size_steps(gpu, orc, prec):
    """The NP law's explicit steps on the benchmark's mesh (the 512^2 notched
    plate, beta = 1e3, no damage) on the streamed kernel at the benchmark's
    launch shape, where every persistent workgroup walks several tiles (the
    next tile's copies are issued during the current one's sums): 3 steps
    from a random velocity against the oracle's NP steps (notch and collars
    included)."""
    torch, pd, ctx = gpu
    w = inputs.CONFIGS["notched512"]()
    v0 = inputs.random_field(w.n, 2, 97, scale=2e-2)
    v0[w.bc_kind == inputs.BC_VELOCITY] = 0.0
    beta, steps = 1e3, 3
    mesh = orc.LawMesh(w.X, w.V, w.delta)
    c = orc.micromodulus(2, w.E, w.delta)
    alive0 = mesh.notch_cut(w.notch, mesh.all_alive())
    st = mesh.start_law(w.u0, v0, c, orc.LAW_NP, beta, alive=alive0)
    mesh.verlet_law(st, c, w.rho, 0.0, w.dt, steps, orc.LAW_NP, beta, bc_kind=w.bc_kind,
                    bc_vel=w.bc_vel, ramp=w.ramp_steps)
    say("NP streamed full size", prec)
    ctx.tune_clear()
    nb = pd.Neighbors(ctx, dev(torch, w.X), w.delta)
    mat = pd.material(2, pd.micromodulus(2, w.E, w.delta), w.rho, 0.0, prec, law="np",
                      beta=beta)
    sim = pd.Simulation(ctx, nb, mat, dev(torch, w.X), dev(torch, w.V), dev(torch, w.u0),
                        dev(torch, v0), bc_kind=dev(torch, w.bc_kind),
                        bc_vel=dev(torch, w.bc_vel), notch=w.notch, ramp_steps=w.ramp_steps)
    info = sim.info()
    assert info["kernel"] == "stream"
    # even at the most workgroups a CU can hold, each walks two tiles or more
    ntiles = -(-w.n // info["tile"])
    assert ntiles >= 2 * 256 * (2048 // info["block"])
    sim.step(steps, w.dt)
    u, v, a, _ = read_state(torch, sim, w.n, 2, nb.nnz)
    sim.close()
    nb.close()
    assert np.array_equal(a, alive0)
    tol = TOL64 if prec == "fp64" else TOLMIX
    assert relL2(u, st["u"]) <= tol
    assert relL2(v, st["v"]) <= tol
