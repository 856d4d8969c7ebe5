"""Degenerate cases of the newer entry points: zero-step requests and calls,
an isolated node in the peridynamic solid, a zero-load NP solve, an
all-zero batch chunk."""
import numpy as np
import pytest

from conftest import say
from paper_1806_06917_amd import inputs
from test_gpu_parity import dev, host, read_state

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
