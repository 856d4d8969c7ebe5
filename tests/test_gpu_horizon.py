"""Long-horizon runs of the two explicit workloads under their own edge
loading (no artificial initial velocity): the 512^2 notched plate for its
10k steps and the 1M-node jittered cube for its 2k steps, each with the
boundary velocity ramp of the workload.  The whole horizon runs on the GPU;
at checkpoints spread over it (before the crack starts, while it grows and
at the end) the oracle restarts from the GPU state and must match the GPU
after a window of steps (velocity-Verlet equations with the critical-stretch
test of the explicit-integration section): rel-L2 1e-12 in FP64 and 1e-5 in
the other modes, flags equal outside the band.  A second test compares the
reduced-precision runs with the FP64 run at the end of the horizon."""
import numpy as np
import pytest

from conftest import say
from paper_1806_06917_amd import inputs
from test_gpu_parity import (TOL64, cached_mesh, dev, eta_band, read_state, relL2,
                             sim_from_workload, tol_of)

pytestmark = pytest.mark.gpu

# checkpoint steps and window length per workload: the plate's ramp ends at
# step 1000, the cube's at step 200
HORIZON = {
    "notched512": (list(range(0, 10000, 1250)) + [9980], 20),
    "cube100": ([0, 300, 700, 1100, 1500, 1995], 5),
}


def start_alive(mesh, w):
    return mesh.notch_cut(w.notch, mesh.all_alive()) if w.notch is not None else mesh.all_alive()


@pytest.mark.parametrize("prec", ["fp64", "mixed", "fp32"])
@pytest.mark.parametrize("wl", ["notched512", "cube100"])
def test_loaded_horizon_windows(gpu, orc, wl, prec):
    torch, pd, ctx = gpu
    w = inputs.CONFIGS[wl]()
    marks, W = HORIZON[wl]
    say("horizon", wl, prec, "steps", w.steps)
    mesh = cached_mesh(orc, wl, w)
    c = orc.micromodulus(w.dim, w.E, w.delta)
    tol = tol_of(prec)
    alive0 = start_alive(mesh, w)
    nb = pd.Neighbors(ctx, dev(torch, w.X), w.delta)
    sim = sim_from_workload(torch, pd, ctx, nb, w, pd.micromodulus(w.dim, w.E, w.delta), prec)
    try:
        step = 0
        broken = []
        for k, m in enumerate(marks):
            if m > step:
                sim.step(m - step, w.dt)
                step = m
            u, v, a, info = read_state(torch, sim, w.n, w.dim, nb.nnz)
            assert info["step"] == step
            st = mesh.start(u, v, c, w.s_c, a)
            st["step"] = step
            band = mesh.verlet_banded(st, c, w.rho, w.s_c, w.dt, W, w.bc_kind, w.bc_vel, None,
                                      w.ramp_steps, tol_eta=eta_band(prec)).astype(bool)
            sim.step(W, w.dt)
            step += W
            u, v, a, info = read_state(torch, sim, w.n, w.dim, nb.nnz)
            assert np.array_equal(a[~band], st["alive"][~band]), f"window at {m}"
            same = np.array_equal(a, st["alive"])
            eu, ev = relL2(u, st["u"]), relL2(v, st["v"])
            broken.append(int(np.count_nonzero(a == 0) - np.count_nonzero(alive0 == 0)))
            say("window at", m, "broken", broken[-1], "same flags", same, "relL2 u", eu, "v", ev)
            if same:
                assert eu <= tol and ev <= 10 * tol, f"window at {m}"
            else:                                   # a bond inside the band went the other way
                assert prec != "fp64"
                assert eu <= 100 * tol, f"window at {m}"
        # the load breaks bonds during the horizon, and the damage only grows
        assert broken[-1] > 0
        assert all(b0 <= b1 for b0, b1 in zip(broken, broken[1:]))
    finally:
        sim.close()
        nb.close()


@pytest.mark.parametrize("wl", ["notched512", "cube100"])
def test_loaded_horizon_precisions(gpu, wl):
    """The mixed and FP32 runs against the FP64 run on the same GPU at the end
    of the whole horizon, beside FP64 runs whose micromodulus is raised by 4
    units in the last place, by 2^-22 (the bound on the mixed mode's
    reciprocal square root estimate) and by 2^-20.

    A bond whose stretch comes within a relative 1e-7 of s_c may break a step
    earlier or later under any change at that level, and the fracture that
    follows spreads the difference: on the cube, which shatters (9 % of its
    bonds break), a 2^-22 change of the stiffness moves the displacement
    field by about 1e-2 after 2k steps.  The bar: on the plate, whose crack
    takes no such turn under the reduced modes, flags equal to the FP64 run's
    and the displacement within the mode's tolerance; on both workloads, a
    drift (displacement, velocity, flags) at most twice that of the 2^-22
    control and the same damage and energies to 1e-3 and 1e-2."""
    torch, pd, ctx = gpu
    w = inputs.CONFIGS[wl]()
    c = pd.micromodulus(w.dim, w.E, w.delta)
    nb = pd.Neighbors(ctx, dev(torch, w.X), w.delta)
    out = {}
    try:
        for key, prec, cc in [("fp64", "fp64", c), ("fp64+4ulp", "fp64", c * (1 + 4 * 2.0 ** -52)),
                              ("fp64+2^-22", "fp64", c * (1 + 2.0 ** -22)),
                              ("fp64+2^-20", "fp64", c * (1 + 2.0 ** -20)),
                              ("mixed", "mixed", c), ("fp32", "fp32", c)]:
            say(wl, key, "steps", w.steps)
            sim = sim_from_workload(torch, pd, ctx, nb, w, cc, prec)
            sim.step(w.steps, w.dt)
            out[key] = read_state(torch, sim, w.n, w.dim, nb.nnz)
            sim.close()
    finally:
        nb.close()
    u64, v64, a64, i64 = out["fp64"]
    drift = {}
    for key in list(out)[1:]:
        u, v, a, info = out[key]
        drift[key] = (relL2(u, u64), relL2(v, v64), int(np.count_nonzero(a != a64)))
        say(wl, key, "vs fp64: relL2 u", drift[key][0], "v", drift[key][1], "dead",
            int(np.count_nonzero(a == 0)), "fp64 dead", int(np.count_nonzero(a64 == 0)),
            "flags differ", drift[key][2], "ke", info["ke"], i64["ke"], "pe", info["pe"], i64["pe"])
    ctl = drift["fp64+2^-22"]
    assert drift["fp64+4ulp"][2] == 0 and drift["fp64+4ulp"][0] <= TOL64
    for key in ["mixed", "fp32"]:
        u, v, a, info = out[key]
        du, dv, dflags = drift[key]
        if wl == "notched512":
            assert dflags == 0 and du <= tol_of(key) and dv <= 10 * tol_of(key), key
        assert du <= 2 * ctl[0] and dv <= 2 * ctl[1] and dflags <= 2 * max(ctl[2], 1), key
        dead, dead64 = np.count_nonzero(a == 0), np.count_nonzero(a64 == 0)
        assert abs(int(dead) - int(dead64)) <= 1e-3 * dead64, key
        assert abs(info["ke"] - i64["ke"]) <= 1e-2 * i64["ke"], key
        assert abs(info["pe"] - i64["pe"]) <= 1e-2 * i64["pe"], key


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_loaded_horizon_np_windows(gpu, orc, prec):
    """The NP law of the validation section in Algorithm 1 (beta = 1e3, no
    damage) on the 512^2 notched plate for the whole 10k steps under its
    collar loading, on the streamed kernel: at checkpoints the oracle's NP
    steps restart from the GPU state and must match it after 20 steps."""
    torch, pd, ctx = gpu
    w = inputs.CONFIGS["notched512"]()
    beta, W = 1e3, 20
    marks = list(range(0, 10000, 2500)) + [9980]
    mesh = orc.LawMesh(w.X, w.V, w.delta)
    c = orc.micromodulus(2, w.E, w.delta)
    alive0 = mesh.notch_cut(w.notch, mesh.all_alive())
    tol = TOL64 if prec == "fp64" else tol_of(prec)
    nb = pd.Neighbors(ctx, dev(torch, w.X), w.delta)
    mat = pd.material(2, pd.micromodulus(2, w.E, w.delta), w.rho, 0.0, prec, law="np",
                      beta=beta)
    sim = pd.Simulation(ctx, nb, mat, dev(torch, w.X), dev(torch, w.V), dev(torch, w.u0),
                        dev(torch, w.v0), bc_kind=dev(torch, w.bc_kind),
                        bc_vel=dev(torch, w.bc_vel), notch=w.notch, ramp_steps=w.ramp_steps)
    try:
        assert sim.info()["kernel"] == "stream"
        step = 0
        for m in marks:
            sim.step(m - step, w.dt)
            step = m
            u, v, a, info = read_state(torch, sim, w.n, 2, nb.nnz)
            assert info["step"] == step and np.array_equal(a, alive0)
            st = mesh.start_law(u, v, c, orc.LAW_NP, beta, alive=a)
            st["step"] = step
            mesh.verlet_law(st, c, w.rho, 0.0, w.dt, W, orc.LAW_NP, beta, bc_kind=w.bc_kind,
                            bc_vel=w.bc_vel, ramp=w.ramp_steps)
            sim.step(W, w.dt)
            step += W
            u, v, a, info = read_state(torch, sim, w.n, 2, nb.nnz)
            eu, ev = relL2(u, st["u"]), relL2(v, st["v"])
            say("NP window at", m, "relL2 u", eu, "v", ev)
            assert eu <= tol and ev <= 10 * tol, f"window at {m}"
        assert np.abs(u).max() > 1e-4          # the collars have moved the plate
    finally:
        sim.close()
        nb.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_loaded_horizon_solid_windows(gpu, orc, prec):
    """The linear peridynamic solid of Algorithm 2 (nu = 1/4, no damage) on the
    1M-node cube for the whole 2k steps under its uniaxial collar loading, on
    the streamed kernel's two passes: at checkpoints the oracle's solid steps
    restart from the GPU state and must match it after 2 steps."""
    torch, pd, ctx = gpu
    w = inputs.CONFIGS["cube100"]()
    K, mu = orc.lps_moduli(w.E, 0.25)
    marks, W = [0, 700, 1400, 1998], 2
    mesh = orc.LpsMesh(w.X, w.V, w.delta)
    tol = TOL64 if prec == "fp64" else tol_of(prec)
    ctx.tune_clear()
    nb = pd.Neighbors(ctx, dev(torch, w.X), w.delta)
    mat = pd.material(3, 0.0, w.rho, 0.0, prec, law="lps", bulk=K, shear=mu)
    sim = pd.Simulation(ctx, nb, mat, dev(torch, w.X), dev(torch, w.V), dev(torch, w.u0),
                        dev(torch, w.v0), bc_kind=dev(torch, w.bc_kind),
                        bc_vel=dev(torch, w.bc_vel), ramp_steps=w.ramp_steps)
    try:
        assert sim.info()["kernel"] == "stream"
        step = 0
        for m in marks:
            sim.step(m - step, w.dt)
            step = m
            u, v, _, info = read_state(torch, sim, w.n, 3, nb.nnz)
            assert info["step"] == step
            st = mesh.start_lps(u, v, K, mu)
            st["step"] = step
            mesh.verlet_lps(st, K, mu, w.rho, w.dt, W, bc_kind=w.bc_kind, bc_vel=w.bc_vel,
                            ramp=w.ramp_steps)
            sim.step(W, w.dt)
            step += W
            u, v, _, info = read_state(torch, sim, w.n, 3, nb.nnz)
            eu, ev = relL2(u, st["u"]), relL2(v, st["v"])
            say("solid window at", m, "relL2 u", eu, "v", ev)
            assert eu <= tol and ev <= 10 * tol, f"window at {m}"
        assert np.abs(u).max() > 1e-4          # the collars have stretched the cube
    finally:
        sim.close()
        nb.close()
