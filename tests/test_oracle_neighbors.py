"""Pins of the oracle's neighbour search against brute force, integer lattice
counts and the closed-ball definition of the horizon (Section
"Discretization of peridynamics equations")."""
import json
import os

import numpy as np
import pytest

from paper_1806_06917_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def lattice_count(dim, m):
    """Integer vectors a != 0 with |a| <= m (exact integer arithmetic)."""
    r = range(-m, m + 1)
    if dim == 2:
        return sum(1 for a in r for b in r if (a, b) != (0, 0) and a * a + b * b <= m * m)
    return sum(1 for a in r for b in r for c in r
               if (a, b, c) != (0, 0, 0) and a * a + b * b + c * c <= m * m)


def test_lattice_counts_golden():
    with open(os.path.join(GOLDEN, "lattice_counts.json")) as fh:
        g = json.load(fh)
    for key, val in g["counts"].items():
        dim, m = int(key[0]), int(key.split("_m")[1])
        assert lattice_count(dim, m) == val


@pytest.mark.parametrize("dim,N,m,h", [(2, 16, 3, 1.0 / 16), (2, 16, 4, 1.0 / 16),
                                       (2, 20, 3, 0.01), (2, 40, 3, 1.0 / 40),
                                       (3, 10, 3, 0.01), (3, 9, 3, 1.0 / 8)])
def test_interior_counts_match_closed_ball(orc, dim, N, m, h):
    """Interior nodes of a lattice have exactly the closed-ball count; exact
    ties at |xi| = delta are kept also for non-dyadic h (relative slack)."""
    X = inputs.grid_coords((N,) * dim, h)
    rp, col = orc.neighbors(X, m * h)
    ij = inputs.lattice_index((N,) * dim)
    inner = np.all((ij >= m) & (ij < N - m), axis=1)
    counts = np.diff(rp)
    assert inner.any()
    assert np.all(counts[inner] == lattice_count(dim, m))
    # the strict (open-ball) count would be smaller: the ties are really present
    strict = lattice_count(dim, m) - sum(
        1 for v in np.ndindex(*(2 * m + 1,) * dim)
        if sum((x - m) ** 2 for x in v) == m * m)
    assert strict < lattice_count(dim, m)


@pytest.mark.parametrize("dim,n,seed", [(2, 700, 1), (3, 900, 2), (2, 1, 3), (3, 2, 4)])
def test_binned_equals_brute(orc, dim, n, seed):
    X = inputs.random_cloud(n, dim, seed)
    delta = 0.11 if dim == 2 else 0.2
    a = orc.neighbors(X, delta, "brute")
    b = orc.neighbors(X, delta, "binned")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_binned_equals_brute_on_grid_ties(orc):
    X = inputs.grid_coords((17, 13), 0.01)
    a = orc.neighbors(X, 0.03, "brute")
    b = orc.neighbors(X, 0.03, "binned")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_symmetric_sorted_no_self(orc):
    X = inputs.grid_coords((12, 12, 12), 1.0 / 12, jitter=0.05, seed=7)
    rp, col = orc.neighbors(X, 3.0 / 12)
    n = X.shape[0]
    pairs = set()
    for i in range(n):
        row = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) > 0)
        assert i not in row
        pairs.update((i, int(j)) for j in row)
    assert all((j, i) in pairs for (i, j) in pairs)


def test_hand_chain(orc):
    X = np.array([[0.0, 0.0], [0.5, 0.0], [1.0, 0.0], [3.0, 0.0]])
    rp, col = orc.neighbors(X, 0.5, "brute")
    assert rp.tolist() == [0, 1, 3, 4, 4]
    assert col.tolist() == [1, 0, 2, 1]


def test_coincident_nodes_rejected(orc):
    X = np.array([[0.0, 0.0], [0.1, 0.0], [0.1, 0.0]])
    with pytest.raises(ValueError):
        orc.neighbors(X, 0.5, "brute")
    with pytest.raises(ValueError):
        orc.neighbors(X, 0.5, "binned")


def test_threshold_reading(orc):
    d = 0.03
    assert orc.threshold(d) == (d * d) * (1.0 + 1e-10)
