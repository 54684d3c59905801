"""Pins of the oracle's particle spawning (Section 3.1): the counter-based
generator against published known answers and an independent library
implementation; the spawn sequence replayed attempt by attempt with an
independent contact predicate; uniformity of centres and radii; the cap
N_max; the initial state of new particles; lower-dimensional spawn boxes.
"""
import json
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

import oracle as O
import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
KAT = json.load(open(os.path.join(HERE, "golden", "philox4x32_10_kat.json")))


def P(**kw):
    base = dict(rho=2500.0, E=1e6, nu=0.3, e_n=0.5, mu_s=0.5, mu_r=0.1, mu_t=0.1, eta=0.0,
                g=(0.0, 0.0, 0.0), dt=1e-6)
    base.update(kw)
    return O.make_params(**base)


def empty(params=None, **mesh):
    return O.Sim(params or P(), np.zeros((0, 3)), R=np.zeros(0), **mesh)


def unit_open(k):
    return (k + 0.5) / 4294967296.0


def draws(seed, a):
    """Centre and radius fractions of attempt a, from the oracle's generator
    (pinned by the two tests below)."""
    o = O.philox4x32_10([a & 0xFFFFFFFF, a >> 32, 0, 0], [seed & 0xFFFFFFFF, seed >> 32])
    return [unit_open(k) for k in o]


# --------------------------------------------------------------------------
# the generator
# --------------------------------------------------------------------------
def test_philox_known_answer_vectors():
    for v in KAT["vectors"]:
        got = O.philox4x32_10([int(c, 16) for c in v["ctr"]], [int(k, 16) for k in v["key"]])
        assert got == [int(c, 16) for c in v["out"]]


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand_engine():
    """rocRAND's header-only philox4x32_10 engine (an independent
    implementation) gives the same words for counters 0, 1, 2, ... under a
    64-bit seed split into the two key words."""
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "philox_rocrand")
        subprocess.run(["hipcc", "-O1", "-o", exe, os.path.join(HERE, "golden",
                                                                  "philox_rocrand.cpp")],
                       check=True, capture_output=True, timeout=600)
        for seed in (0, 0x0123456789ABCDEF, 2 ** 64 - 1):
            out = subprocess.run([exe, hex(seed), "300"], check=True, capture_output=True,
                                 text=True).stdout.split("\n")
            for i in (0, 1, 2, 17, 255, 299):
                want = [int(t) for t in out[i].split()]
                assert O.philox4x32_10([i, 0, 0, 0], [seed & 0xFFFFFFFF, seed >> 32]) == want


# --------------------------------------------------------------------------
# the spawn sequence, replayed
# --------------------------------------------------------------------------
def touches(c, r, X, R, els, rm):
    """Independent contact predicate of a candidate sphere: any particle or
    rounded element with (R_j + r) - d >= 0."""
    for x, Rj in zip(X, R):
        dx, dy, dz = (x[0] - c[0]), (x[1] - c[1]), (x[2] - c[2])
        d = math.sqrt((dx * dx + dy * dy) + dz * dz)
        if (Rj + r) - d >= 0.0:
            return True
    for e, Rm in zip(els, rm):
        cp = O.closest_point_element(c, e)
        dx, dy, dz = (c[0] - cp[0]), (c[1] - cp[1]), (c[2] - cp[2])
        d = math.sqrt((dx * dx + dy * dy) + dz * dz)
        if (r + Rm) - d >= 0.0:
            return True
    return False


@pytest.mark.parametrize("with_mesh", [False, True])
def test_spawn_sequence_replayed(with_mesh):
    """A crowded box, no gravity, new particles at rest (nothing moves):
    every spawned particle sits at the centre drawn by one attempt; its
    radius is the draw of the attempt after the previous success (the radius
    carries over failures); each attempt in between would have touched a
    particle present then, or an element, and the successful one touches
    nothing."""
    seed = 77
    smin, smax, Rmin, Rmax = (0.0, 0.0, 0.0), (8e-3, 8e-3, 6e-3), 0.6e-3, 1.6e-3
    els, rm = ([[[4e-3, 4e-3, 3e-3]], [[0.0, 2e-3, 1e-3], [8e-3, 6e-3, 5e-3]]], [1.0e-3, 0.4e-3]) \
        if with_mesh else ([], [])
    s = empty(elements=els if with_mesh else None, rmesh=rm if with_mesh else None)
    s.set_spawn(smin=smin, smax=smax, Rmin=Rmin, Rmax=Rmax, n_spawn=40, n_max=10 ** 6, seed=seed)
    s.step(6)
    attempts, carried = s.spawn_status()
    assert attempts == 240
    X, R = s.state()["x"], s.radii
    assert 15 < len(R) < 200
    box = np.array(smax) - np.array(smin)
    a = 0
    for i in range(len(R)):
        r_new = Rmin + draws(seed, a)[3] * (Rmax - Rmin)
        assert R[i] == r_new, i
        while True:
            u = draws(seed, a)
            c = [smin[k] + u[k] * box[k] for k in range(3)]
            blocked = touches(c, R[i], X[:i], R[:i], els, rm)
            a += 1
            if not blocked:
                assert np.array_equal(X[i], c), i
                break
            assert a < attempts
    # the attempts after the last success all failed with one carried radius
    if a < attempts:
        r_c = Rmin + draws(seed, a)[3] * (Rmax - Rmin)
        assert carried == r_c
        for b in range(a, attempts):
            u = draws(seed, b)
            assert touches([smin[k] + u[k] * box[k] for k in range(3)], r_c, X, R, els, rm)
    else:
        assert carried == 0.0


def test_spawn_avoids_existing_particles_and_mesh():
    """Particles spawned among existing ones and a floor never start in
    contact: the first step's contacts hold none of the new ids."""
    w = W.random_cluster(150, 3, box=12e-3, overlap=0.1)
    tri = W.floor_mesh(6e-3, 6e-3, 0.02, 0.0)
    s = O.Sim(P(), w["x"], R=w["R"], tri=tri)
    n0 = s.n
    s.set_spawn(smin=(0.0, 0.0, 0.0), smax=(12e-3, 12e-3, 24e-3), Rmin=0.5e-3, Rmax=1.0e-3,
                n_spawn=300, n_max=10 ** 6, seed=5)
    s.step(1)
    assert s.n > n0 + 20
    c = s.contacts()
    assert not np.any(c["ki"] >= n0) and not np.any(c["kj"] >= n0)
    # and the independent predicate agrees for every new particle
    X, R = s.state()["x"], s.radii
    for i in range(n0, s.n):
        others = np.r_[0:i]
        assert not touches(X[i], R[i], X[others], R[others], [t for t in tri], [0.0, 0.0])


# --------------------------------------------------------------------------
# distribution, cap and initial state
# --------------------------------------------------------------------------
def test_uniform_centres_and_radii_in_an_open_box():
    """Where rejections are rare, centres are uniform in the box and radii
    uniform in [R_min, R_max] (Kolmogorov-Smirnov)."""
    s = empty()
    s.set_spawn(smin=(-0.5, 0.0, 1.0), smax=(0.5, 2.0, 1.5), Rmin=1e-3, Rmax=3e-3, n_spawn=500,
                n_max=4000, seed=11)
    s.step(10)
    assert s.n == 4000
    X, R = s.state()["x"], s.radii
    for k, (lo, hi) in enumerate(((-0.5, 0.5), (0.0, 2.0), (1.0, 1.5))):
        assert stats.kstest(X[:, k], "uniform", args=(lo, hi - lo)).pvalue > 1e-3
        assert X[:, k].min() > lo and X[:, k].max() < hi
    assert stats.kstest(R, "uniform", args=(1e-3, 2e-3)).pvalue > 1e-3


def test_carried_radius_keeps_sizes_unbiased_in_a_crowd():
    """In a crowded box most attempts fail, yet the placed radii stay
    uniform: every drawn radius waits until it fits (Section 3.1).  A
    redraw after each failure would favour small radii."""
    s = empty()
    s.set_spawn(smin=(0.0, 0.0, 0.0), smax=(20e-3, 20e-3, 20e-3), Rmin=0.3e-3, Rmax=2.0e-3,
                n_spawn=200, n_max=10 ** 6, seed=21)
    s.step(60)
    attempts, _ = s.spawn_status()
    R = s.radii
    assert attempts > 3 * len(R) > 600  # mostly failures
    assert stats.kstest(R, "uniform", args=(0.3e-3, 1.7e-3)).pvalue > 1e-3


def test_stops_at_n_max_and_counts_only_attempts_made():
    s = empty()
    s.set_spawn(smin=(0.0, 0.0, 0.0), smax=(1.0, 1.0, 1.0), Rmin=1e-3, Rmax=1e-3, n_spawn=50,
                n_max=130, seed=3)
    s.step(2)
    assert s.n == 100 and s.spawn_status()[0] == 100
    s.step(1)
    assert s.n == 130 and s.spawn_status()[0] == 130
    s.step(2)
    assert s.n == 130 and s.spawn_status()[0] == 130
    assert np.all(s.radii == 1e-3)


def test_new_particle_state():
    """v0, w0 and the identity orientation at creation; after the one step
    that created it (no contacts, no gravity), v = v0, w = w0 and q is the
    SPIRAL rotation of the identity by dt |w0| (Eq. spiral)."""
    dt = 1e-5
    v0, w0 = (0.1, -0.2, -1.0), (3.0, 0.0, 4.0)
    s = empty(P(dt=dt))
    s.set_spawn(smin=(0.0, 0.0, 0.0), smax=(1.0, 1.0, 1.0), Rmin=1e-3, Rmax=2e-3, v0=v0, w0=w0,
                n_spawn=5, n_max=5, seed=9)
    s.step(1)
    st = s.state()
    assert np.array_equal(st["v"], np.tile(v0, (5, 1)))
    assert np.array_equal(st["w"], np.tile(w0, (5, 1)))
    phi = dt * 5.0 / 2
    q = np.array([math.cos(phi), *(math.sin(phi) * np.array(w0) / 5.0)])
    assert np.allclose(st["q"], np.tile(q, (5, 1)), rtol=0, atol=1e-16)
    # the position advanced by one semi-implicit step from the drawn centre
    u = draws(9, 0)
    c0 = np.array(u[:3])
    assert np.allclose(st["x"][0], c0 + dt * np.array(v0), rtol=0, atol=1e-15)


def test_flat_spawn_region_pins_one_coordinate():
    """Only centres are confined: a box with s_min,z = s_max,z puts every
    centre exactly at that height (the lower-dimensional use of Section 3.1)."""
    s = empty()
    s.set_spawn(smin=(0.0, 0.0, 0.25), smax=(0.1, 0.1, 0.25), Rmin=1e-3, Rmax=2e-3, n_spawn=80,
                n_max=80, seed=4)
    s.step(1)
    assert s.n > 60
    assert np.all(s.state()["x"][:, 2] == 0.25)


def test_seeds_and_validation():
    def run(seed):
        s = empty()
        s.set_spawn(smin=(0.0, 0.0, 0.0), smax=(0.01, 0.01, 0.01), Rmin=5e-4, Rmax=1e-3,
                    n_spawn=30, n_max=1000, seed=seed)
        s.step(3)
        return s.state()["x"], s.radii
    a, b, c = run(1), run(1), run(2)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert not np.array_equal(a[1][:5], c[1][:5])
    s = empty()
    for bad in (dict(smin=(0, 0, 1.0), smax=(1, 1, 0.0), Rmin=1e-3, Rmax=2e-3),
                dict(smin=(0, 0, 0), smax=(1, 1, 1), Rmin=0.0, Rmax=2e-3),
                dict(smin=(0, 0, 0), smax=(1, 1, 1), Rmin=3e-3, Rmax=2e-3),
                dict(smin=(0, 0, 0), smax=(1, 1, 1), Rmin=1e-3, Rmax=2e-3, n_spawn=-1)):
        with pytest.raises(ValueError):
            s.set_spawn(**bad)


@pytest.mark.parametrize("gap_ulps", [0, 1])
def test_exact_touching_blocks_a_spawn(gap_ulps):
    """A candidate exactly touching a particle or a rounded element
    (delta = 0, a contact by the inclusive test) is rejected; one ulp
    farther it is placed.  A point-like spawn box and R_min = R_max fix the
    candidate: centre (0, 0, 0), radius 1 mm."""
    d = 2e-3
    for _ in range(gap_ulps):
        d = np.nextafter(d, 1.0)
    s = O.Sim(P(), [[d, 0.0, 0.0]], R=[1e-3])
    s.set_spawn(smin=(0.0, 0.0, 0.0), smax=(0.0, 0.0, 0.0), Rmin=1e-3, Rmax=1e-3, n_spawn=1,
                n_max=10, seed=1)
    s.step(1)
    assert s.n == 1 + gap_ulps
    dm = 1.5e-3
    for _ in range(gap_ulps):
        dm = np.nextafter(dm, 1.0)
    s = empty(elements=[[[0.0, dm, 0.0]]], rmesh=[0.5e-3])
    s.set_spawn(smin=(0.0, 0.0, 0.0), smax=(0.0, 0.0, 0.0), Rmin=1e-3, Rmax=1e-3, n_spawn=1,
                n_max=10, seed=1)
    s.step(1)
    assert s.n == gap_ulps
