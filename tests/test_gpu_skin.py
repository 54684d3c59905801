"""Cells kept between steps (skin > 0): the contact set and the results must
be those of the paper's every-step rebuild.  The oracle rebuilds every step
(brute force or fresh linked cells), so any pair missed because a particle
drifted out of reach of a kept cell shows up as a key mismatch."""
import numpy as np
import pytest

import workloads as W
from tests.parity_util import (force_err, keys, oracle_from, oracle_resync, rel, rel_w,
                               spring_err, torque_err)

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def solver(w, **kw):
    from paper_2507_12610_amd import Solver
    return Solver(w, device="cuda:0", **kw)


def check_resync(g, w, every, checks, t0=0.0):
    """Every `every` steps: oracle from the GPU state and springs, one step on
    both, keys bit for bit and forces/states within the FP64 tolerance."""
    dt = w["params"]["dt"]
    done = 0
    total = 0
    for _ in range(checks):
        g.step(every - 1)
        done += every - 1
        st, c = g.state(forces=False), g.contacts()
        o = oracle_resync(w, st, c, t0 + done * dt)
        g.step(1)
        o.step(1)
        done += 1
        cg, co = g.contacts(), o.contacts()
        assert np.array_equal(keys(cg), keys(co)), done
        total += len(co["ki"])
        if len(co["ki"]):
            assert max(spring_err(cg, co).values()) < TOL64, done
        sg, so, fo = g.state(), o.state(), o.forces()
        assert force_err(sg["F"], fo["F"], fo["Fscale"]) < TOL64, done
        assert torque_err(sg["T"], fo["T"], fo["Tscale"], fo["Fscale"], w["R"]) < TOL64, done
        for k in ("v", "q"):
            assert rel(sg[k], so[k]) < TOL64, (done, k)
        assert rel_w(sg["w"], so["w"], w["R"], so["v"]) < TOL64, done
    return total


@pytest.mark.parametrize("skin,lanes", [(0.02, 1), (0.05, 0), (0.2, 1)])
def test_fast_cluster_rebuilds_when_needed(skin, lanes):
    """Polydisperse spheres at up to ~2 m/s in a box (4 um per step): with a
    half skin of 14 um the cells are rebuilt every few steps, with 140 um
    rarely; the contacts are those of the every-step rebuild throughout."""
    tri = W.cube_mesh([-0.2e-3] * 3, [18.2e-3] * 3)
    w = W.random_cluster(600, 41, box=18e-3, overlap=0.2, r_lo=0.4e-3, r_hi=1.4e-3, vel=0.5,
                         spin=200.0, tri=tri)
    w["params"].update(g=(0.0, 0.0, -9.81), dt=2e-6)
    g = solver(w, cell_factor=0.5, detect_lanes=lanes, skin=skin)
    total = check_resync(g, w, every=25, checks=12)
    assert total > 2000
    st = g.stats()
    assert st["steps"] == 300
    if skin < 0.1:
        assert 10 < st["rebuilds"] < 300, st
    else:
        assert 1 <= st["rebuilds"] < 30, st


def test_free_running_cfg1_with_skin():
    """Configuration 1 over 200 free-running steps with the cells kept: the
    same keys and, within the chaos bound, the same states as the oracle."""
    w = W.cfg1()
    g = solver(w, skin=0.1)
    o = oracle_from(w)
    g.step(200)
    o.step(200)
    sg, so = g.state(), o.state()
    assert np.array_equal(keys(g.contacts()), keys(o.contacts()))
    for k in ("v", "w", "q"):
        assert rel(sg[k], so[k]) < TOL64, k
    assert g.stats()["rebuilds"] < 200


def test_batch_with_skin():
    """Uneven box drops in one context with the cells kept per simulation."""
    sims = [W.cfg4_sim(s, n) for s, n in ((3, 700), (120, 1300), (250, 520))]
    for s in sims:
        s["x"][:, 2] -= s["x"][:, 2].min() - 1.1e-3
    g = solver(sims, skin=0.05)
    g.step(800)
    st, c = g.state(forces=False), g.contacts()
    g.step(1)
    sg, cg = g.state(), g.contacts()
    off = g.offsets
    total = 0
    for k, w in enumerate(sims):
        lo, hi = off[k], off[k + 1]
        m = (c["ki"] >= lo) & (c["ki"] < hi)
        kj = c["kj"][m].copy()
        kj[kj > 0] -= lo
        hist = {"ki": c["ki"][m] - lo, "kj": kj, "us": c["us"][m], "ur": c["ur"][m],
                "ut": c["ut"][m]}
        sub = {kk: st[kk][lo:hi] for kk in ("x", "v", "w", "q")}
        o = oracle_resync(w, sub, hist, 800 * w["params"]["dt"])
        o.step(1)
        co, so = o.contacts(), o.state()
        mm = (cg["ki"] >= lo) & (cg["ki"] < hi)
        kg = np.stack([cg["ki"][mm] - lo, np.where(cg["kj"][mm] > 0, cg["kj"][mm] - lo,
                                                     cg["kj"][mm])], 1)
        assert np.array_equal(kg, keys(co)), k
        total += len(co["ki"])
        for key in ("v", "q"):
            assert rel(sg[key][lo:hi], so[key]) < TOL64, (k, key)
        fo = o.forces()
        assert force_err(sg["F"][lo:hi], fo["F"], fo["Fscale"]) < TOL64, k
    assert total > 300
    assert g.stats()["rebuilds"] < 801


def test_drift_past_the_skin_within_one_call():
    """A skin far too small for the speeds and no scheduled rebuild inside one
    call of 60 steps: after the first step every search must widen by the
    measured drift beyond half the skin.  The contact set and the state at the
    end match the oracle, and only the first step rebuilt the cells."""
    tri = W.cube_mesh([-0.2e-3] * 3, [18.2e-3] * 3)
    w = W.random_cluster(600, 43, box=18e-3, overlap=0.2, r_lo=0.4e-3, r_hi=1.4e-3, vel=0.5,
                         spin=200.0, tri=tri)
    w["params"].update(g=(0.0, 0.0, -9.81), dt=2e-6)
    g = solver(w, cell_factor=0.5, detect_lanes=1, skin=0.001, rebuild_every=100000)
    o = oracle_from(w)
    g.step(60)
    o.step(60)
    assert g.stats()["rebuilds"] == 1
    cg, co = g.contacts(), o.contacts()
    assert np.array_equal(keys(cg), keys(co))
    assert len(co["ki"]) > 200
    sg, so = g.state(), o.state()
    for k in ("v", "q"):
        assert rel(sg[k], so[k]) < TOL64, k
    assert rel_w(sg["w"], so["w"], w["R"], so["v"]) < TOL64
    # the next call starts with a rebuild and stays exact
    check_resync(g, w, every=10, checks=3, t0=60 * w["params"]["dt"])
    assert g.stats()["rebuilds"] >= 2


def test_profiled_steps_rebuild_like_plain_steps():
    """Steps timed phase by phase take the same rebuild decisions as plain
    steps (period adapted at its end, drift past the skin seen): the same
    rebuild count and the same state bit for bit after 300 steps."""
    tri = W.cube_mesh([-0.2e-3] * 3, [18.2e-3] * 3)
    w = W.random_cluster(600, 41, box=18e-3, overlap=0.2, r_lo=0.4e-3, r_hi=1.4e-3, vel=0.5,
                         spin=200.0, tri=tri)
    w["params"].update(g=(0.0, 0.0, -9.81), dt=2e-6)
    a = solver(w, cell_factor=0.5, detect_lanes=1, skin=0.02)
    b = solver(w, cell_factor=0.5, detect_lanes=1, skin=0.02)
    a.step(300)
    ph = b.step_profiled(300)
    assert all(v >= 0.0 for v in ph.values())
    ra, rb = a.stats()["rebuilds"], b.stats()["rebuilds"]
    assert ra == rb and 10 < ra < 300, (ra, rb)
    sa, sb = a.state(), b.state()
    for k in ("x", "v", "w", "q", "F", "T"):
        assert np.array_equal(sa[k], sb[k]), k


def test_static_walls_found_between_rebuilds():
    """With a skin, a rebuild lists every static element within
    R_i + R_m + half skin of each particle, taken from the element bin of its
    centre, so the bins must reach R_max + R_m + half skin.  Spheres of R_max
    start half a half skin away from contact with the +x, +y and +z faces of
    a cube, whose element bins (bin edge half the face) have a boundary right
    where a reach of R_max alone would end, and move onto the faces between
    rebuilds: the contact keys equal the oracle's at every step."""
    L, R = 20e-3, 1e-3
    tri = W.cube_mesh([0.0] * 3, [L] * 3)
    skin = 1.0
    gap = 0.25 * skin * R  # half of the half skin
    c = 0.5 * L
    x = np.array([[L - R - gap, c, c], [c, L - R - gap, c], [c, c, L - R - gap],
                  [c - 3e-3, c - 3e-3, c - 3e-3]])
    v = np.array([[2.0, 0, 0], [0, 2.0, 0], [0, 0, 2.0], [0.1, 0.1, 0.1]])
    n = len(x)
    w = {"name": "walls_between_rebuilds", "params": W.default_params(g=(0.0, 0.0, 0.0), dt=2e-6),
         "x": x, "v": v, "w": np.zeros((n, 3)), "q": np.tile([1.0, 0, 0, 0], (n, 1)),
         "R": np.full(n, R), "tri": tri, "rmesh": np.zeros(len(tri)), "steps": 0, "R_max": R}
    g = solver(w, skin=skin, rebuild_every=100000)
    o = oracle_from(w)
    rebuilds_at_touch = None
    for step in range(150):
        g.step(1)
        o.step(1)
        kg, ko = keys(g.contacts()), keys(o.contacts())
        assert np.array_equal(kg, ko), step
        if rebuilds_at_touch is None and len(ko) >= 3:
            rebuilds_at_touch = g.stats()["rebuilds"]
    # the walls were reached on steps that kept the cells of the first step
    assert rebuilds_at_touch == 1
