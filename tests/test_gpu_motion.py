"""GPU parity of moving meshes (motion groups: an extension generalising the
rotating drum; the vibrated base of the segregation example of Section 4)
through sdem_set_mesh_motion, against the FP64 oracle.  Keys bit-exact,
springs, forces and states within 1e-12 (FP64) or 1e-5 (mixed)."""
import numpy as np
import pytest

import workloads as W
from tests.parity_util import (force_err, keys, oracle_from, oracle_resync, rel, rel_w,
                               spring_err)

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def solver(w, **kw):
    from paper_2507_12610_amd import Solver
    return Solver(w, device="cuda:0", **kw)


def errors(g, o, w):
    cg, co = g.contacts(), o.contacts()
    assert np.array_equal(keys(cg), keys(co))
    sg, so, fo = g.state(), o.state(), o.forces()
    e = dict(spring_err(cg, co)) if len(co["ki"]) else {}
    e["F"] = force_err(sg["F"], fo["F"], fo["Fscale"])
    e["v"] = rel(sg["v"], so["v"])
    e["w"] = rel_w(sg["w"], so["w"], w["R"], so["v"])
    e["q"] = rel(sg["q"], so["q"])
    return e, len(co["ki"]), int((co["kj"] == -(len(w["elements"]) - 1)).sum())


@pytest.mark.parametrize("skin,lanes", [(0.0, 0), (0.05, 0), (0.05, 1)])
def test_vibrated_floor_resynced(skin, lanes):
    """Spheres landing on a floor vibrated at 3 g (walls fixed): every 100 of
    800 steps the oracle takes the GPU state, springs and clock and both
    advance one step.  With a skin and one search lane the steps that keep
    the cells read the wall motion in the fused search and contact law."""
    w = W.vibrated_box()
    g = solver(w, skin=skin, detect_lanes=lanes)
    floor = 0
    for t in range(0, 800, 100):
        if t:
            g.step(99)
        st, c = g.state(forces=False), g.contacts()
        o = oracle_resync(w, st, c, g.stats()["steps"] * w["params"]["dt"])
        g.step(1)
        o.step(1)
        e, n, nf = errors(g, o, w)
        floor += nf
        assert max(e.values()) < TOL64, (t, e)
    assert floor >= 5


def test_vibrated_floor_free_running():
    """The same scene over 400 free-running steps from the start: the floor's
    motion and wall velocity follow the oracle's."""
    w = W.vibrated_box()
    g, o = solver(w), oracle_from(w)
    for _ in range(4):
        g.step(100)
        o.step(100)
        assert np.array_equal(keys(g.contacts()), keys(o.contacts()))
    e, _, _ = errors(g, o, w)
    assert max(e.values()) < 1e-10, e


def test_turning_and_vibrating_groups():
    """Three motion groups in one element mesh (turning, vibrating, both)
    with spheres among them: 60 free-running steps."""
    from tests.test_gpu_primitives import primitive_case
    w = primitive_case(n=400, seed=4)
    w["params"].update(dt=1e-6)
    els = w["elements"]
    w["motion"] = [dict(omega=(0.0, 0.0, 30.0), center=(0.01, 0.01, 0.0)),
                   dict(amp=(1e-3, 0.0, 2e-3), freq=40.0, phase=0.4),
                   dict(omega=(10.0, -20.0, 5.0), center=(0.0, 0.02, 0.01), amp=(0.0, 5e-4, 0.0),
                        freq=25.0, phase=-1.0)]
    w["motion_groups"] = np.arange(len(els), dtype=np.int32) % 3
    g, o = solver(w), oracle_from(w)
    for _ in range(3):
        g.step(20)
        o.step(20)
        assert np.array_equal(keys(g.contacts()), keys(o.contacts()))
    e, n, _ = errors(g, o, w)
    assert n > 50
    assert max(e.values()) < 1e-10, e


def test_vibrated_floor_mixed_precision():
    w = W.vibrated_box()
    g = solver(w, precision="mixed")
    g.step(500)
    st, c = g.state(forces=False), g.contacts()
    o = oracle_resync(w, st, c, g.stats()["steps"] * w["params"]["dt"])
    g.step(1)
    o.step(1)
    e, _, _ = errors(g, o, w)
    assert max(e.values()) < TOL32, e


def test_motion_errors():
    from paper_2507_12610_amd import SdemError
    w = W.vibrated_box(n=50)
    g = solver(w)
    with pytest.raises(SdemError) as ei:
        g.set_mesh_motion(0, [dict()], groups=np.full(len(w["elements"]), 1))
    assert "EINVAL" in str(ei.value)
    with pytest.raises(SdemError) as ei:
        g.set_mesh_motion(0, [dict()] * 17)
    assert "EINVAL" in str(ei.value)
    with pytest.raises(SdemError) as ei:
        g.set_mesh_motion(0, [dict(freq=-1.0)])
    assert "EINVAL" in str(ei.value)
