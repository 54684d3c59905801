"""GPU parity of particle spawning (Section 3.1) through the C ABI against the
FP64 oracle: the same generator words, the same accepted attempts, the same
carried radius, the same new ids and radii (bit for bit), then the usual
parity of keys (bit-exact) and states (1e-12 FP64, 1e-5 mixed)."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.parity_util import force_err, keys, rel, rel_w, spring_err

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def hopper(n_max=1000, n_spawn=100, low=False, seed=2507):
    els, rm = W.hopper_elements()
    w = W._finish("hopper", W.hopper_params(), np.zeros((0, 3)), np.zeros(0),
                  np.random.default_rng(0), None, 1)
    w["elements"], w["rmesh"] = els, rm
    sp = W.hopper_spawn(n_max=n_max, n_spawn=n_spawn, seed=seed)
    if low:  # a box inside the funnel: wall contacts from the first steps
        sp.update(smin=(-0.06, -0.06, 0.15), smax=(0.06, 0.06, 0.22))
    return w, sp


def solver(w, sp, **kw):
    from paper_2507_12610_amd import Solver
    return Solver(w, device="cuda:0", spawn=sp, **kw)


def oracle_sim(w, sp):
    o = oracle.Sim(w["params"], np.zeros((0, 3)), R=np.zeros(0), elements=w["elements"],
                   rmesh=w["rmesh"])
    o.set_spawn(**sp)
    return o


def oracle_resync(w, sp, g):
    """Oracle started from the GPU's state, springs, clock and spawn
    sequence position."""
    st, c = g.state(forces=False), g.contacts()
    n, attempts, carried = g.spawn_status()
    o = oracle.Sim(w["params"], st["x"], v=st["v"], w=st["w"], q=st["q"], R=g.radii(),
                   elements=w["elements"], rmesh=w["rmesh"])
    o.set_time(g.stats()["steps"] * w["params"]["dt"])
    if len(c["ki"]):
        o.set_history(c["ki"], c["kj"], c["us"], c["ur"], c["ut"])
    o.set_spawn(**sp)
    o.set_spawn_status(attempts, carried)
    return o


def compare(g, o, tol, what):
    n, attempts, carried = g.spawn_status()
    assert n == o.n, what
    assert (attempts, carried) == o.spawn_status(), what
    assert np.array_equal(g.radii(), o.radii), what
    cg, co = g.contacts(), o.contacts()
    assert np.array_equal(keys(cg), keys(co)), what
    if len(co["ki"]):
        assert max(spring_err(cg, co).values()) < tol, what
    sg, so = g.state(), o.state()
    fo = o.forces()
    assert force_err(sg["F"], fo["F"], fo["Fscale"]) < tol, what
    for k in ("v", "q"):
        assert rel(sg[k], so[k]) < tol, (what, k)
    assert rel_w(sg["w"], so["w"], o.radii, so["v"]) < tol, what
    assert rel(sg["x"], so["x"]) < tol, what
    return len(co["ki"]), int((co["kj"] <= 0).sum())


def test_spawn_sequence_free_running():
    """From an empty hopper (Table 2 spawn defaults), 40 steps: the spawn
    decisions of every step are the oracle's."""
    w, sp = hopper()
    g, o = solver(w, sp), oracle_sim(w, sp)
    for k in range(4):
        g.step(10)
        o.step(10)
        compare(g, o, TOL64, k)
    assert 400 < g.n <= 1000


@pytest.mark.parametrize("skin,lanes", [(0.0, 0), (0.05, 0), (0.05, 1)])
def test_spawn_resynced_in_the_funnel(skin, lanes):
    """A spawn box inside the funnel, 2,000 particles at most: every 100 of
    700 steps the oracle takes the GPU's state, springs and spawn position
    and both advance one step (spawning while particles and funnel walls
    collide; later, attempts failing with a carried radius)."""
    w, sp = hopper(n_max=2000, low=True)
    g = solver(w, sp, skin=skin, detect_lanes=lanes)
    pp = pw = 0
    carried_seen = False
    for t in range(0, 700, 100):
        if t:
            g.step(99)
        o = oracle_resync(w, sp, g)
        g.step(1)
        o.step(1)
        a, b = compare(g, o, TOL64, t)
        pp, pw = pp + a - b, pw + b
        carried_seen |= o.spawn_status()[1] > 0.0
    assert pp > 200 and pw > 50
    assert carried_seen


def test_spawn_mixed_precision_step():
    w, sp = hopper(n_max=1500, low=True)
    g = solver(w, sp, precision="mixed")
    g.step(150)
    o = oracle_resync(w, sp, g)
    g.step(1)
    o.step(1)
    n, attempts, carried = g.spawn_status()
    assert n == o.n and (attempts, carried) == o.spawn_status()
    assert np.array_equal(keys(g.contacts()), keys(o.contacts()))
    sg, so, fo = g.state(), o.state(), o.forces()
    assert force_err(sg["F"], fo["F"], fo["Fscale"]) < TOL32
    assert rel(sg["v"], so["v"]) < TOL32


@pytest.mark.parametrize("gap_ulps", [0, 1])
def test_exact_touching_blocks_a_spawn(gap_ulps):
    """A point-like spawn box and R_min = R_max: the candidate (centre 0,
    radius 1 mm) exactly touches a particle 2 mm away and is rejected; one
    ulp farther it is placed (the inclusive contact test)."""
    d = 2e-3
    for _ in range(gap_ulps):
        d = np.nextafter(d, 1.0)
    w = W._finish("touch", W.default_params(dt=1e-6, g=(0, 0, 0)), np.array([[d, 0.0, 0.0]]),
                  np.array([1e-3]), np.random.default_rng(0), None, 1)
    sp = dict(smin=(0.0, 0.0, 0.0), smax=(0.0, 0.0, 0.0), Rmin=1e-3, Rmax=1e-3, n_spawn=1,
              n_max=10, seed=1)
    g = solver(w, sp)
    g.step(1)
    assert g.n == 1 + gap_ulps
    assert g.spawn_status()[2] == (1e-3 if gap_ulps == 0 else 0.0)


def test_spawn_counts_and_errors():
    from paper_2507_12610_amd import SdemError, Solver
    w, sp = hopper(n_max=300, n_spawn=100)
    g, o = solver(w, sp), oracle_sim(w, sp)
    g.step(2)
    o.step(2)
    assert g.spawn_status() == (o.n, *o.spawn_status())
    assert 150 < g.n < 300
    g.step(5)
    o.step(5)
    assert g.n == 300  # capped; attempts stop once the cap is reached
    assert g.spawn_status() == (o.n, *o.spawn_status())
    assert g.spawn_status()[1] < 100 * 7
    with pytest.raises(SdemError) as ei:
        g.set_spawn(**dict(sp, n_max=10 ** 6))  # above the context's capacity
    assert "ECAPACITY" in str(ei.value)
    with pytest.raises(SdemError) as ei:
        g.set_spawn(**dict(sp, Rmin=0.0))
    assert "EINVAL" in str(ei.value)
    two = [W.random_cluster(20, 1), W.random_cluster(20, 2)]
    s2 = Solver(two, device="cuda:0")
    with pytest.raises(SdemError) as ei:
        s2.set_spawn(**sp)
    assert "EINVAL" in str(ei.value)
