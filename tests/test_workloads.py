"""Pins of the sequential deposition that builds the settled column: no two
spheres overlap beyond rounding, every sphere rests on the floor or on
contacts whose normals carry its weight (checked by nonnegative least
squares, a method of its own), the packing fraction and coordination lie at
the values random deposition with rolling is known for (about 0.58 and 6),
and the result is reproducible from the seed."""
import numpy as np
import pytest
from scipy.optimize import nnls
from scipy.spatial import cKDTree

import workloads as W


@pytest.fixture(scope="module")
def pile():
    rng = np.random.default_rng(5)
    R = np.exp(0.2 * rng.standard_normal(4000))  # lognormal radii, median 1 (mm)
    L = 24.0
    x, stuck = W.deposit(R, L, L, 11)
    return R, L, x, stuck


def periodic_pairs(R, L, x):
    tree = cKDTree(x, boxsize=[L, L, 1e9])
    pairs = tree.query_pairs(2.0 * R.max() + 1e-9, output_type="ndarray")
    d = x[pairs[:, 0]] - x[pairs[:, 1]]
    d[:, :2] = (d[:, :2] + 0.5 * L) % L - 0.5 * L
    gap = np.linalg.norm(d, axis=1) - (R[pairs[:, 0]] + R[pairs[:, 1]])
    return pairs, d, gap


def test_no_overlap_and_inside_the_cell(pile):
    R, L, x, stuck = pile
    assert stuck == 0
    assert np.all(x[:, :2] >= 0.0) and np.all(x[:, :2] < L)
    assert np.all(x[:, 2] - R >= -1e-12)
    _, _, gap = periodic_pairs(R, L, x)
    assert gap.min() > -1e-12 * R.max()


def test_every_sphere_carried(pile):
    """Weight (0, 0, 1) in the cone of the contact normals, or the floor."""
    R, L, x, _ = pile
    pairs, d, gap = periodic_pairs(R, L, x)
    touch = np.abs(gap) < 1e-9
    normals = [[] for _ in range(len(R))]
    for (a, b), dv in zip(pairs[touch], d[touch]):
        u = dv / np.linalg.norm(dv)  # from b to a
        normals[a].append(u)
        normals[b].append(-u)
    on_floor = np.abs(x[:, 2] - R) < 1e-9
    worst = 0.0
    for i in range(len(R)):
        if on_floor[i]:
            continue
        N = np.array(normals[i]).T
        assert N.shape[1] >= 2, i
        _, res = nnls(N, np.array([0.0, 0.0, 1.0]))
        worst = max(worst, res)
    assert worst < 1e-6, worst


def test_fraction_and_coordination(pile):
    R, L, x, _ = pile
    _, _, gap = periodic_pairs(R, L, x)
    ntouch = int(np.sum(np.abs(gap) < 1e-9))
    coordination = 2.0 * ntouch / len(R)
    assert 5.5 < coordination < 6.5, coordination
    top = x[:, 2].max()
    lo, hi = 0.25 * top, 0.6 * top
    # volume of the spheres in the slab, counting each by the part inside
    zc, r = x[:, 2], R
    a = np.clip(lo - zc, -r, r)
    b = np.clip(hi - zc, -r, r)
    part = np.pi * ((r * r * b - b ** 3 / 3.0) - (r * r * a - a ** 3 / 3.0))
    phi = part.sum() / (L * L * (hi - lo))
    assert 0.55 < phi < 0.62, phi


def test_reproducible_from_the_seed(pile):
    R, L, x, _ = pile
    x2, _ = W.deposit(R, L, L, 11)
    assert np.array_equal(x, x2)
    x3, _ = W.deposit(R, L, L, 12)
    assert not np.array_equal(x, x3)
