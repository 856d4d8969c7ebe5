"""The C ABI used from a host program with no Python or PyTorch in it
(tests/c/abi_force.cpp, built by __graft_entry__.build()): on a jittered
2-d lattice and a jittered 3-d cube, with the three left columns clamped and
a body force on the right column, the program calls every entry point of
the hot path in FP64.  Against the oracle: neighbour lists bit-exact; the
force (Algorithm 1, linearised law), the tangent applied to a vector and a
velocity-Verlet trajectory within rel-L2 1e-12; the quasi-static solution
with a relative residual of 1e-10 (evaluated by the oracle: at most 2e-10)
and within 1e-6 of the oracle's own solution."""
import os
import subprocess

import numpy as np
import pytest

from conftest import say
from paper_1806_06917_amd import inputs
from test_gpu_parity import TOL64, relL2

pytestmark = pytest.mark.gpu

PROG = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c", "abi_force")

CASES = {
    "lattice2d_41x29": ((41, 29), 1 / 32, 3),
    "cube3d_17": ((17, 17, 17), 1 / 16, 3),
}


@pytest.mark.parametrize("name", list(CASES))
def test_c_program_matches_oracle(orc, tmp_path, name):
    assert os.path.exists(PROG), "the C-ABI test program is not built"
    shape, h, m = CASES[name]
    dim = len(shape)
    X = inputs.grid_coords(shape, h, jitter=0.05, seed=11)
    n = X.shape[0]
    V = np.full(n, h ** dim)
    u = inputs.random_field(n, dim, 12, scale=1e-3 * h)
    delta, dt, nsteps = m * h, 0.1 * h, 20
    ij = inputs.lattice_index(shape)
    fixed = (ij[:, 0] < 3).astype(np.uint8)
    b = np.zeros((n, dim))
    b[ij[:, 0] == shape[0] - 1, 0] = 1e-3 / h
    c = orc.micromodulus(dim, 1.0, delta)
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as fh:
        np.array([n, dim, nsteps], np.int64).tofile(fh)
        np.array([delta, c, dt], np.float64).tofile(fh)
        for a in (X, V, u, b):
            np.ascontiguousarray(a, np.float64).tofile(fh)
        fixed.tofile(fh)
    say("C program", name, n)
    r = subprocess.run([PROG, str(inp), str(out)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    raw = np.fromfile(out, np.uint8)
    nnz = int(raw[:8].view(np.int64)[0])
    off = 8

    def take(dtype, count):
        nonlocal off
        a = raw[off:off + np.dtype(dtype).itemsize * count].view(dtype)
        off += np.dtype(dtype).itemsize * count
        return a

    row_ptr = take(np.int64, n + 1)
    col = take(np.int32, nnz)
    f, y, uT, vT, us = (take(np.float64, n * dim).reshape(n, dim) for _ in range(5))
    rel = float(take(np.float64, 1)[0])
    assert off == raw.size

    mesh = orc.Mesh(X, V, delta)
    assert nnz == mesh.nnz
    assert np.array_equal(row_ptr, mesh.row_ptr)
    assert np.array_equal(col, mesh.col)
    ef = relL2(f, mesh.force(u, c))
    ey = relL2(y, mesh.apply_tangent(u, c, fixed))
    st = mesh.start(u, np.zeros_like(u), c)
    mesh.verlet(st, c, 1.0, 0.0, dt, nsteps)
    eu, ev = relL2(uT, st["u"]), relL2(vT, st["v"])
    ref, info = mesh.solve_implicit(np.zeros_like(u), c, b, fixed, rtol=1e-12)
    assert info["status"] == 0
    _, rn = mesh.residual(us, c, b, fixed)
    bn = np.linalg.norm((V[:, None] * b)[fixed == 0])
    say("C program", name, "nnz", nnz, "force", ef, "tangent", ey, "steps u", eu, "v", ev,
        "solve", relL2(us, ref), "residual", rel, rn / bn)
    assert ef <= TOL64 and ey <= TOL64 and eu <= TOL64 and ev <= TOL64
    assert rel <= 1e-10 and rn / bn <= 2e-10
    assert relL2(us, ref) <= 1e-6
