"""Mixed precision (FP32 contact force and torque arithmetic, FP64 positions,
differences, contact test, spring updates, sums and integration; springs kept
as floats between steps) against the FP64 oracle: keys bit-exact, every quantity within 1e-5 normwise relative after one
step and over a short horizon; the per-quantity errors are printed."""
import numpy as np
import pytest

import workloads as W
from tests.parity_util import force_err, keys, torque_err, oracle_from, oracle_resync, rel, rel_w, spring_err

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


def solver(w, **kw):
    from paper_2507_12610_amd import Solver
    return Solver(w, device="cuda:0", precision="mixed", **kw)


def errors(g, o, w):
    cg, co = g.contacts(), o.contacts()
    assert np.array_equal(keys(cg), keys(co))
    sg, so, fo = g.state(), o.state(), o.forces()
    e = dict(spring_err(cg, co))
    e["F"] = force_err(sg["F"], fo["F"], fo["Fscale"])
    e["T"] = torque_err(sg["T"], fo["T"], fo["Tscale"], fo["Fscale"], w["R"])
    e["v"] = rel(sg["v"], so["v"])
    e["w"] = rel_w(sg["w"], so["w"], w["R"], so["v"])
    e["q"] = rel(sg["q"], so["q"])
    e["dx"] = rel(sg["x"] - w["x"], so["x"] - w["x"])
    return e


@pytest.mark.parametrize("case", ["cluster", "cfg1"])
def test_mixed_one_step(case):
    if case == "cluster":
        w = W.random_cluster(500, 4, box=16e-3, overlap=0.15,
                             tri=W.cube_mesh([-0.2e-3] * 3, [16.2e-3] * 3))
        w["params"].update(g=(0.0, 0.0, -9.81))
    else:
        w = W.cfg1()
    g, o = solver(w), oracle_from(w)
    g.step(1)
    o.step(1)
    e = errors(g, o, w)
    print(case, {k: f"{v:.2e}" for k, v in e.items()})
    assert max(e.values()) < TOL32, e


@pytest.mark.parametrize("skin", [0.0, 0.1])
def test_mixed_resynced_horizon_cfg1(skin):
    """Every 50 of 500 steps of configuration 1: keys bit-exact and all
    quantities within 1e-5 one step after a resync.  With a skin and one
    search lane, the steps that keep the cells run the FP32 contact law in
    the same kernel as the search."""
    w = W.cfg1()
    g = solver(w, skin=skin, detect_lanes=1) if skin else solver(w)
    worst = {}
    for t in range(0, 500, 50):
        if t:
            g.step(49)
        st, c = g.state(forces=False), g.contacts()
        o = oracle_resync(w, st, c, g.stats()["steps"] * w["params"]["dt"])
        g.step(1)
        o.step(1)
        w2 = dict(w)
        w2["x"] = st["x"]
        e = errors(g, o, w2)
        for k, v in e.items():
            worst[k] = max(worst.get(k, 0.0), v)
    print("worst over the horizon", {k: f"{v:.2e}" for k, v in worst.items()})
    assert max(worst.values()) < TOL32, worst


def test_mixed_free_running_short_horizon():
    """Free-running 20 steps from the same start: the FP32 force rounding
    stays within 1e-5 of the FP64 oracle."""
    w = W.cfg1()
    g, o = solver(w), oracle_from(w)
    g.step(20)
    o.step(20)
    e = errors(g, o, w)
    print("20 steps", {k: f"{v:.2e}" for k, v in e.items()})
    assert max(e.values()) < TOL32, e


def test_mixed_springs_kept_as_floats():
    """Between steps the mixed path keeps each contact's springs as floats:
    springs loaded through sdem_set_history read back rounded to the nearest
    float, and after a step every spring is a float value, within 1e-5 of the
    oracle's step from the same (unrounded) history.  The FP64 path reads
    them back bit for bit."""
    from paper_2507_12610_amd import Solver
    w = W.random_cluster(300, 4, box=14e-3, overlap=0.15,
                         tri=W.cube_mesh([-0.2e-3] * 3, [14.2e-3] * 3))
    o = oracle_from(w)
    o.step(3)
    co, st = o.contacts(), o.state()
    assert len(co["ki"]) > 100
    w2 = dict(w)
    w2.update(x=st["x"], v=st["v"], w=st["w"], q=st["q"])
    as_f32 = (lambda a: np.asarray(a, np.float64).astype(np.float32).astype(np.float64))
    for precision in ("fp64", "mixed"):
        g = Solver(w2, device="cuda:0", precision=precision)
        g.set_history(co["ki"], co["kj"], co["us"], co["ur"], co["ut"])
        cg = g.contacts()
        assert np.array_equal(keys(cg), keys(co))
        for k in ("us", "ur", "ut"):
            want = co[k] if precision == "fp64" else as_f32(co[k])
            assert np.array_equal(cg[k], want), (precision, k)
        if precision == "mixed":
            o2 = oracle_resync(w, st, co, 3 * w["params"]["dt"])
            g.step(1)
            o2.step(1)
            cg, c2 = g.contacts(), o2.contacts()
            assert np.array_equal(keys(cg), keys(c2))
            for k in ("us", "ur", "ut"):
                assert np.array_equal(cg[k], as_f32(cg[k])), k
            assert max(spring_err(cg, c2).values()) < TOL32
        g.close()
