"""Handle lifetimes through the C ABI: a context or neighbour list destroyed
before the handles built on it stays valid memory until the last of them is
destroyed; calls through a destroyed context fail with PD_EINVAL."""
import numpy as np
import pytest

from conftest import say
from paper_1806_06917_amd import inputs

pytestmark = pytest.mark.gpu


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _sim(torch, pd, ctx, nb, w):
    c = pd.micromodulus(w.dim, w.E, w.delta)
    return pd.Simulation(ctx, nb, pd.material(w.dim, c, w.rho, 0.0, "fp64"), _dev(torch, w.X),
                         _dev(torch, w.V), _dev(torch, w.u0), _dev(torch, w.v0))


def test_destroy_order(gpu):
    torch, pd, _ = gpu
    w = inputs.plate_2d(16, 3, seed=4, steps=0)
    say("handles: list destroyed before its simulation")
    ctx = pd.Context(0)
    nb = pd.Neighbors(ctx, _dev(torch, w.X), w.delta)
    s = _sim(torch, pd, ctx, nb, w)
    nb.close()
    s.step(3, w.dt)                      # the simulation keeps its list alive
    assert s.get()["step"] == 3
    say("handles: context destroyed before its simulation")
    ctx.close()
    with pytest.raises(pd.PDError) as e:
        s.step(1, w.dt)
    assert e.value.status == pd.PD_EINVAL
    s.close()                            # frees the list, then the context
    assert pd.lib.pd_ctx_destroy(None) == pd.PD_EINVAL
