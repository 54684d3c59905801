"""GPU parity of the other mesh primitives (Section 3.3, Fig. 4A-E): points,
segments, triangles and rectangles, each with its own radius R_m, given
through sdem_add_mesh_elements, against the FP64 oracle.  Keys bit-exact;
springs, forces and states within 1e-12 (FP64) or 1e-5 (mixed)."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.parity_util import (force_err, keys, oracle_from, oracle_resync, rel, rel_w,
                               spring_err, torque_err)

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5
BOX = 20e-3


def solver(w, **kw):
    from paper_2507_12610_amd import Solver
    return Solver(w, device="cuda:0", **kw)


def primitive_case(n=600, seed=0, omega=None):
    """Spheres at random in a container built from all four kinds of element
    (rounded points, rails, tilted rounded triangles and rectangle, walls of
    rectangles and triangles), under gravity; spheres that start more than
    0.2 R_i inside an element are dropped."""
    els, rm = W.primitive_mesh(BOX, seed)
    w = W.random_cluster(n, 50 + seed, box=BOX, overlap=0.15, r_lo=0.6e-3, r_hi=1.2e-3)
    keep = np.ones(len(w["R"]), bool)
    for i, (x, R) in enumerate(zip(w["x"], w["R"])):
        for e, r in zip(els, rm):
            d = np.linalg.norm(x - oracle.closest_point_element(x, e))
            if d < r + 0.8 * R:
                keep[i] = False
                break
    for k in ("x", "v", "w", "q", "R"):
        w[k] = np.ascontiguousarray(w[k][keep])
    w["elements"], w["rmesh"] = els, rm
    w["params"].update(g=(0.0, 0.0, -9.81))
    if omega is not None:
        w["params"].update(mesh_omega=tuple(omega), mesh_center=(BOX / 2, BOX / 2, BOX / 2))
    return w


def element_kinds(w, kj):
    return {len(w["elements"][-k]) for k in np.asarray(kj).tolist() if k <= 0}


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


@pytest.mark.parametrize("seed,cf", [(0, 1.0), (1, 0.4), (2, 0.7)])
def test_one_step_every_primitive(seed, cf):
    w = primitive_case(seed=seed)
    g, o = solver(w, cell_factor=cf), oracle_from(w)
    g.step(1)
    o.step(1)
    co = o.contacts()
    assert element_kinds(w, co["kj"]) == {1, 2, 3, 4}
    e = errors(g, o, w)
    assert max(e.values()) < TOL64, e


@pytest.mark.parametrize("skin", [0.0, 0.05])
def test_resynced_steps_every_primitive(skin):
    """600 steps of spheres falling onto and rolling over the elements: every
    100 steps the oracle takes the GPU state and springs and both advance
    one step.  With a skin the elements come from the candidate lists made
    at rebuilds."""
    w = primitive_case(seed=3)
    g = solver(w, skin=skin)
    kinds = set()
    for t in range(0, 600, 100):
        if t:
            g.step(99)
        st, c = g.state(forces=False), g.contacts()
        o = oracle_resync(w, st, c, g.stats()["steps"] * w["params"]["dt"])
        g.step(1)
        o.step(1)
        kinds |= element_kinds(w, o.contacts()["kj"])
        e = errors(g, o, w)
        assert max(e.values()) < TOL64, (t, e)
    assert kinds == {1, 2, 3, 4}


def test_mixed_one_step_every_primitive():
    w = primitive_case(seed=4)
    g, o = solver(w, precision="mixed"), oracle_from(w)
    g.step(1)
    o.step(1)
    e = errors(g, o, w)
    print({k: f"{v:.2e}" for k, v in e.items()})
    assert max(e.values()) < TOL32, e


def test_rotating_primitive_mesh():
    """Every kind of element turning rigidly about the container centre
    (the rotating-mesh extension): keys and states follow the oracle."""
    w = primitive_case(seed=5, omega=(0.0, 2.0, 0.5))
    g, o = solver(w), oracle_from(w)
    for _ in range(3):
        g.step(10)
        o.step(10)
        assert np.array_equal(keys(g.contacts()), keys(o.contacts()))
    sg, so = g.state(), o.state()
    for k in ("v", "w"):
        assert rel(sg[k], so[k]) < 1e-11, k


def test_batch_mixing_element_and_triangle_meshes():
    """Simulations with element meshes and with triangle meshes in one
    context: keys count elements from 0 in each simulation."""
    a = primitive_case(n=300, seed=6)
    b = W.random_cluster(250, 61, box=16e-3, overlap=0.15,
                         tri=W.cube_mesh([-0.2e-3] * 3, [16.2e-3] * 3))
    b["params"].update(g=(0.0, 0.0, -9.81))
    c = primitive_case(n=200, seed=7)
    sims = [a, b, c]
    g = solver(sims)
    g.step(3)
    st, cg = g.state(), g.contacts()
    off = g.offsets
    for k, w in enumerate(sims):
        o = oracle_from(w)
        o.step(3)
        so = o.state()
        sl = slice(off[k], off[k + 1])
        for key in ("v", "q"):
            assert rel(st[key][sl], so[key]) < TOL64, (k, key)
        m = (cg["ki"] >= off[k]) & (cg["ki"] < off[k + 1])
        kg = np.stack([cg["ki"][m] - off[k],
                       np.where(cg["kj"][m] > 0, cg["kj"][m] - off[k], cg["kj"][m])], 1)
        assert np.array_equal(kg[np.lexsort((kg[:, 1], kg[:, 0]))], keys(o.contacts()))


def test_single_elements_and_exact_touching():
    """One sphere and one element of each kind placed so that
    R_i + R_m - d is exactly 0 (a contact) or one ulp of the distance
    negative (none)."""
    R, Rm = 1e-3, 0.5e-3
    cases = {
        1: [[0.0, 0.0, 0.0]],
        2: [[-4e-3, 0.0, 0.0], [4e-3, 0.0, 0.0]],
        3: [[-4e-3, -4e-3, 0.0], [4e-3, -4e-3, 0.0], [0.0, 4e-3, 0.0]],
        4: [[-4e-3, -4e-3, 0.0], [4e-3, -4e-3, 0.0], [4e-3, 4e-3, 0.0], [-4e-3, 4e-3, 0.0]],
    }
    for nv, el in cases.items():
        for z, touching in ((R + Rm, True), (np.nextafter(R + Rm, 1.0), False)):
            w = W._finish("one", W.default_params(dt=1e-6, g=(0, 0, 0)),
                          np.array([[0.0, 0.0, z]]), np.array([R]), np.random.default_rng(0),
                          None, 1)
            w["elements"], w["rmesh"] = [el], np.array([Rm])
            g, o = solver(w), oracle_from(w)
            g.step(1)
            o.step(1)
            assert keys(g.contacts()).tolist() == keys(o.contacts()).tolist()
            assert (len(g.contacts()["ki"]) == 1) == touching, (nv, z)


def test_bad_elements_rejected():
    from paper_2507_12610_amd import SdemError
    base = primitive_case(n=50, seed=8)
    bads = [
        ([[[0.0, 0, 0], [1e-3, 0, 0], [1.3e-3, 2e-3, 0], [0.3e-3, 2e-3, 0]]], [0.0], "rectangle"),
        ([[[0.0, 0, 0], [1e-3, 0, 0], [1e-3, 2e-3, 1e-4], [0.0, 2e-3, 0]]], [0.0], "rectangle"),
        ([[[0.0, 0, np.inf]]], [0.0], "finite"),
        ([[[0.0, 0, 0]]], [-1e-3], "radius"),
    ]
    for els, rm, word in bads:
        w = dict(base)
        w["elements"], w["rmesh"] = els, np.array(rm)
        with pytest.raises(SdemError) as ei:
            solver(w)
        assert "EINVAL" in str(ei.value) and word in str(ei.value), word
