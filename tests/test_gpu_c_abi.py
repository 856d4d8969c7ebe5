"""The C ABI used from a host program with no Python or PyTorch in it
(tests/c/abi_force.cpp, built by __graft_entry__.build()): on a jittered
2-d lattice and a jittered 3-d cube the program builds the neighbour lists
(bit-exact against the oracle's) and evaluates the internal force once in
FP64 (Algorithm 1, linearised law: rel-L2 1e-12 against the oracle)."""
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
    delta = m * h
    c = orc.micromodulus(dim, 1.0, delta)
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as fh:
        np.array([n, dim], np.int64).tofile(fh)
        np.array([delta, c], np.float64).tofile(fh)
        for a in (X, V, u):
            np.ascontiguousarray(a, np.float64).tofile(fh)
    say("C program", name, n)
    r = subprocess.run([PROG, str(inp), str(out)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    raw = np.fromfile(out, np.uint8)
    nnz = int(raw[:8].view(np.int64)[0])
    off = 8
    row_ptr = raw[off:off + 8 * (n + 1)].view(np.int64)
    off += 8 * (n + 1)
    col = raw[off:off + 4 * nnz].view(np.int32)
    off += 4 * nnz
    f = raw[off:off + 8 * n * dim].view(np.float64).reshape(n, dim)
    assert off + 8 * n * dim == raw.size
    mesh = orc.Mesh(X, V, delta)
    assert nnz == mesh.nnz
    assert np.array_equal(row_ptr, mesh.row_ptr)
    assert np.array_equal(col, mesh.col)
    ref = mesh.force(u, c)
    say("C program", name, "nnz", nnz, "relL2 f", relL2(f, ref))
    assert relL2(f, ref) <= TOL64
