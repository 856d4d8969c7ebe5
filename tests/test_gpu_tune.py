"""The autotuner (pd_autotune): every candidate launch shape it can pick
steps in parity with the FP64 oracle, the fastest lands in the context's
cache, and simulations created afterwards on meshes of the same kind use it
and step bit for bit like the same shape chosen by hand."""
import numpy as np
import pytest

from conftest import say
from paper_1806_06917_amd import inputs
from test_gpu_parity import TOL64, TOLMIX, dev, read_state, relL2, sim_from_workload

pytestmark = pytest.mark.gpu

CANDIDATES = [(32, 8), (32, 16), (64, 4), (64, 8), (64, 16), (128, 2),
              (128, 4), (128, 8), (192, 4), (240, 4), (256, 2), (256, 4)]


def moving_plate(N, m):
    # notched plate with a random initial velocity and no breaks: every launch
    # shape differs from the oracle only in the order of each node's sum
    w = inputs.notched_plate_2d(N=N, m=m, s_c=1.0, v0=2e-3, steps=0, ramp_steps=5)
    w.v0 = inputs.random_field(w.n, 2, 11, scale=2e-3)
    w.v0[w.bc_kind == 2] = 0
    return w


@pytest.mark.parametrize("prec,tol", [("fp64", TOL64), ("mixed", TOLMIX), ("fp32", TOLMIX)])
def test_every_candidate_matches_oracle(gpu, orc, prec, tol):
    torch, pd, ctx = gpu
    w = moving_plate(64, 3)
    mesh = orc.Mesh(w.X, w.V, w.delta)
    c = orc.micromodulus(2, w.E, w.delta)
    st = mesh.start(w.u0, w.v0, c, w.s_c, mesh.notch_cut(w.notch, mesh.all_alive()))
    mesh.verlet(st, c, w.rho, w.s_c, w.dt, 20, w.bc_kind, w.bc_vel, None, w.ramp_steps)
    for tile, lanes in CANDIDATES:
        say("candidate", prec, tile, lanes)
        ctx.set_lanes(lanes)
        ctx.set_tuning("auto", tile, 0)
        try:
            nb = pd.Neighbors(ctx, dev(torch, w.X), w.delta)
            s = sim_from_workload(torch, pd, ctx, nb, w, pd.micromodulus(2, w.E, w.delta), prec)
            info = s.info()
            assert info["kernel"] in ("stream", "tile")
            assert (info["tile"], info["lanes"]) == (tile, lanes)
            s.step(20, w.dt)
            u, v, _, _ = read_state(torch, s, w.n, 2, nb.nnz)
            s.close()
            nb.close()
        finally:
            ctx.set_lanes(0)
            ctx.set_tuning(0, 0, 0)
        assert relL2(u, st["u"]) <= tol, (tile, lanes)
        assert relL2(v, st["v"]) <= tol, (tile, lanes)


def test_autotune_cache_and_use(gpu):
    torch, pd, _ = gpu
    ctx = pd.Context(0)                 # a context of its own: the cache is per context
    try:
        w = moving_plate(64, 3)
        say("autotune search")
        best, table = ctx.autotune(dev(torch, w.X), dev(torch, w.V), w.delta, "mixed", steps=5)
        assert [(r["tile"], r["lanes"]) for r in table] == CANDIDATES
        ran = [r for r in table if r["us_per_step"] > 0]
        assert ran and all(r["kernel"] in (2, 3) for r in ran)
        assert best["us_per_step"] == min(r["us_per_step"] for r in ran)
        nb0 = pd.Neighbors(ctx, dev(torch, w.X), w.delta)
        k = nb0.nnz / w.n
        nb0.close()
        assert ctx.tune_lookup(2, k, "mixed") == (best["tile"], best["lanes"])
        assert ctx.tune_lookup(2, k, "fp64") is None
        assert ctx.tune_lookup(3, k, "mixed") is None
        # another mesh of the same kind (2-d, delta = 3h) takes the tuned shape
        w2 = moving_plate(80, 3)
        c = pd.micromodulus(2, w2.E, w2.delta)
        say("tuned simulation", best["tile"], best["lanes"])
        nb = pd.Neighbors(ctx, dev(torch, w2.X), w2.delta)
        s = sim_from_workload(torch, pd, ctx, nb, w2, c, "mixed")
        info = s.info()
        assert (info["tile"], info["lanes"]) == (best["tile"], best["lanes"])
        s.step(30, w2.dt)
        tuned = read_state(torch, s, w2.n, 2, nb.nnz)[:3]
        s.close()
        nb.close()
        # the same shape by hand: bit for bit
        ctx.tune_clear()
        assert ctx.tune_lookup(2, k, "mixed") is None
        ctx.set_lanes(best["lanes"])
        ctx.set_tuning("auto", best["tile"], 0)
        nb = pd.Neighbors(ctx, dev(torch, w2.X), w2.delta)
        s = sim_from_workload(torch, pd, ctx, nb, w2, c, "mixed")
        s.step(30, w2.dt)
        by_hand = read_state(torch, s, w2.n, 2, nb.nnz)[:3]
        s.close()
        nb.close()
        for x, y in zip(tuned, by_hand):
            assert np.array_equal(x, y)
        ctx.set_lanes(0)
        ctx.set_tuning(0, 0, 0)
        # an installed choice is used the same way; non-candidates are refused
        ctx.tune_set(2, k, 128, 2, "mixed")
        assert ctx.tune_lookup(2, k, "mixed") == (128, 2)
        with pytest.raises(pd.PDError):
            ctx.tune_set(2, k, 48, 3, "mixed")
    finally:
        ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_large_tiles_stream_with_gather_side_calls(gpu, prec):
    """240-node tiles with 4 lanes on a 3-d cube under tension with damage:
    the steps stream (whether or not the LDS tile kernel can be resident at
    that shape, in which case the closing half-kick and the energy read-back
    run on the gather kernel with the bond flags synchronised), and the
    trajectory, the breaks and the energies equal the gather kernel's bit for
    bit through a read-back in the middle of the run."""
    torch, pd, ctx = gpu
    w = inputs.cube_3d(N=26, s_c=2e-4, v0=2e-2, steps=0, ramp_steps=5)
    out = []
    for kern, tile, lanes in (("stream", 240, 4), ("gather", 0, 4)):
        say("large tiles", kern, prec)
        ctx.set_lanes(lanes)
        ctx.set_tuning(kern, tile, 0)
        try:
            nb = pd.Neighbors(ctx, dev(torch, w.X), w.delta)
            s = sim_from_workload(torch, pd, ctx, nb, w, pd.micromodulus(3, w.E, w.delta), prec)
            info = s.info()
            assert info["kernel"] == kern
            if kern == "stream":
                assert (info["tile"], info["lanes"]) == (240, 4)
            s.step(20, w.dt)
            mid = s.get(energies=True)
            s.step(20, w.dt)
            u, v, alive, end = read_state(torch, s, w.n, 3, nb.nnz)
            out.append((u, v, alive, mid["ke"], mid["pe"], end["ke"], end["pe"]))
            s.close()
            nb.close()
        finally:
            ctx.set_lanes(0)
            ctx.set_tuning(0, 0, 0)
    a, b = out
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], b[2])
    assert a[3:] == b[3:]
    assert np.count_nonzero(a[2] == 0) > 0          # bonds did break


def test_tuned_shape_applies_whole_or_not_at_all(gpu):
    """A tuned (tile size, lanes) pair is taken as a whole: a simulation runs
    either at the tuned shape or, if it cannot use the tuned tile size (its
    material's streamed layout does not fit, or the mesh's tiles are held at
    another size), at the automatic shape, the one a context without tuning
    picks -- never with the tuned lanes on other tiles or the other way
    round.  The solid under a 240 x 4 entry (mixed then FP64), then a
    linear-law simulation on tiles held at 128 nodes."""
    torch, pd, _ = gpu
    N = 22
    h = 1.0 / N
    X = inputs.grid_coords((N,) * 3, h, jitter=0.05, seed=201)
    n = len(X)
    V = np.full(n, h ** 3)
    plain, tuned = pd.Context(0), pd.Context(0)
    ref = {}
    try:
        for c in (plain, tuned):
            nb = pd.Neighbors(c, dev(torch, X), 3 * h)
            if c is tuned:
                for prec in ("mixed", "fp64"):
                    c.tune_set(3, nb.nnz / n, 240, 4, prec)
            for prec in ("mixed", "fp64"):
                say("solid under a tuned shape", "tuned" if c is tuned else "plain", prec)
                sim = pd.Simulation(c, nb, pd.material(3, 0.0, 1.0, 0.0, prec, law="lps",
                                                       bulk=1.0, shear=0.5),
                                    dev(torch, X), dev(torch, V), None, None)
                info = sim.info()
                sim.close()
                if c is plain:
                    ref[prec] = info
                else:
                    whole = (info["tile"], info["lanes"]) == (240, 4)
                    say("solid under 240 x 4:", info)
                    assert whole or info == ref[prec], (prec, info, ref[prec])
            nb.close()
        # tiles held at 128 nodes by a live simulation: a linear-law simulation
        # created under the 240 x 4 entry takes the automatic shape on them,
        # not the tuned 4 lanes
        nbp = pd.Neighbors(plain, dev(torch, X), 3 * h)
        auto = pd.Simulation(plain, nbp, pd.material(3, 1.0, 1.0, 0.0, "mixed"), dev(torch, X),
                             dev(torch, V), None, None)
        want = auto.info()
        auto.close()
        nbp.close()
        assert want["tile"] == 128 and want["lanes"] != 4
        nb = pd.Neighbors(tuned, dev(torch, X), 3 * h)
        tuned.set_tuning("auto", 128, 0)
        holder = pd.Simulation(tuned, nb, pd.material(3, 1.0, 1.0, 0.0, "fp64"), dev(torch, X),
                               dev(torch, V), None, None)
        tuned.set_tuning(0, 0, 0)
        assert holder.info()["tile"] == 128
        say("linear law under a tuned shape on held tiles")
        sim = pd.Simulation(tuned, nb, pd.material(3, 1.0, 1.0, 0.0, "mixed"), dev(torch, X),
                            dev(torch, V), None, None)
        got = sim.info()
        sim.close()
        holder.close()
        nb.close()
        assert (got["tile"], got["lanes"]) == (want["tile"], want["lanes"]), (got, want)
    finally:
        tuned.close()
        plain.close()
