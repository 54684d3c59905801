"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle on
the same seeded inputs.  Contact keys must match bit for bit; forces, springs
and states within 1e-12 (FP64 path), normwise relative, per-particle forces
scaled by the sum of the contact contributions (dense packings cancel)."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads as W
from tests.parity_util import (force_err, keys, torque_err, oracle_from, oracle_resync, rel, rel_w,
                               spring_err)

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def solver(w, **kw):
    from paper_2507_12610_amd import Solver
    return Solver(w, device="cuda:0", **kw)


def test_device_sqrt_and_division_correctly_rounded():
    """The contact test is bit-reproducible only if the device square root and
    division round like the host's (IEEE correctly rounded)."""
    from paper_2507_12610_amd import selftest_rounding
    rng = np.random.default_rng(0)
    n = 1 << 20
    a = np.concatenate([rng.uniform(1e-12, 1e-4, n // 2),
                        np.exp(rng.uniform(-700, 700, n // 2))])
    b = np.concatenate([rng.uniform(1e-6, 1e-2, n // 2), np.exp(rng.uniform(-300, 300, n // 2))])
    s, q = selftest_rounding(a, b)
    with np.errstate(over="ignore", under="ignore"):
        ref_q = a / b
    assert np.array_equal(s.view(np.int64), np.sqrt(a).view(np.int64))
    assert np.array_equal(q.view(np.int64), ref_q.view(np.int64))


@pytest.mark.parametrize("nbytes", [16, 48 << 10, (3 << 20) + 16 * 37])
def test_copy_probe_copies_and_rejects_bad_arguments(nbytes):
    """The bench's bandwidth probe moves every byte (sizes below one
    workgroup's share, and ragged past a whole number of them) and refuses
    sizes that are not whole 16-byte words and overlapping buffers, before
    launching anything."""
    import torch

    from paper_2507_12610_amd import SdemError, copy_probe, lib
    g = torch.Generator().manual_seed(nbytes)
    src = torch.randint(0, 1 << 30, (nbytes // 4,), dtype=torch.int32, generator=g).to("cuda:0")
    dst = torch.zeros_like(src)
    ms = copy_probe(src, dst, reps=3)
    assert ms > 0.0
    assert torch.equal(src.cpu(), dst.cpu())
    with pytest.raises(SdemError, match="EINVAL"):
        copy_probe(src, src, reps=1)
    out = ctypes.c_double()
    stream = torch.cuda.current_stream("cuda:0").cuda_stream
    assert lib().sdem_copy_probe(src.data_ptr(), dst.data_ptr(), nbytes - 8, 1, stream,
                                 ctypes.byref(out)) != 0


@pytest.mark.parametrize("skin", [0.0, 0.5])
def test_step_graphs_made_once(skin):
    """Every HIP graph a context replays is instantiated at the start of its
    first sdem_step call; later calls of any length (with rebuilds) make
    none, so a timed window after a warm-up call holds no instantiation."""
    w = W.cfg1()
    g = solver(w, skin=skin, detect_lanes=1) if skin else solver(w)
    assert g.graph_stats()["instantiated"] == 0
    g.step(3)
    first = g.graph_stats()
    assert first["instantiated"] > 0 and not first["failed"]
    r0 = g.stats()["rebuilds"]
    for k in (1, 8, 30, 200):
        g.step(k)
    assert g.stats()["rebuilds"] > r0
    assert g.graph_stats() == first
    g.close()


def cluster_case(n=400, seed=1, mesh=True, **pk):
    tri = W.cube_mesh([-0.2e-3] * 3, [16.2e-3] * 3) if mesh else None
    w = W.random_cluster(n, seed, box=16e-3, overlap=0.15, tri=tri)
    w["params"].update(g=(0.0, 0.0, -9.81), **pk)
    return w


def compare_one_step(w, tol=TOL64, **skw):
    g = solver(w, **skw)
    o = oracle_from(w)
    g.step(1)
    o.step(1)
    cg, co = g.contacts(), o.contacts()
    assert np.array_equal(keys(cg), keys(co))
    assert len(co["ki"]) > 0
    se = spring_err(cg, co)
    assert max(se.values()) < tol, se
    sg, so = g.state(), o.state()
    fo = o.forces()
    assert force_err(sg["F"], fo["F"], fo["Fscale"]) < tol
    assert torque_err(sg["T"], fo["T"], fo["Tscale"], fo["Fscale"], w["R"]) < tol
    for k in ("v", "w", "q"):
        assert rel(sg[k], so[k]) < tol, k
    assert rel(sg["x"] - w["x"], so["x"] - w["x"]) < tol
    return g, o


def test_one_step_cluster_with_box():
    compare_one_step(cluster_case())


@pytest.mark.parametrize("n", [1, 63, 64, 65, 257, 1000])
def test_one_step_ragged_sizes(n):
    w = W.random_cluster(n, 100 + n, box=max(4e-3, (n * 8e-9 / 0.2) ** (1 / 3)), overlap=0.2,
                         tri=None)
    if n == 1:
        g = solver(w)
        g.step(3)
        o = oracle_from(w)
        o.step(3)
        assert rel(g.state()["v"], o.state()["v"]) < TOL64
        return
    compare_one_step(w)


def test_exact_touching_counts_as_contact():
    """delta = 0 is a contact (inclusive test), found on the GPU as in the
    oracle; a pair a hair apart is not."""
    R = 1e-3
    x = np.array([[0.0, 0, 0], [2e-3, 0, 0], [4e-3 + 1e-12, 0, 0], [4e-3 + 1e-12, 2.5e-3, 0]])
    w = W._finish("touch", W.default_params(dt=1e-6, g=(0, 0, 0)), x, np.full(4, R),
                  np.random.default_rng(0), None, 1)
    g = solver(w)
    g.step(1)
    assert keys(g.contacts()).tolist() == [[0, 1]]


def test_free_running_horizon_cfg1():
    """Configuration 1 (1,000 spheres dropped in a 12-triangle box) over a
    horizon H for which two oracle runs 1 ulp apart stay 10x inside the
    tolerance; keys bit-exact at the end."""
    w = W.cfg1()
    H = 200
    # intrinsic divergence (chaos bound): oracle vs oracle with x perturbed by 1 ulp
    o1 = oracle_from(w)
    w2 = dict(w)
    w2["x"] = np.nextafter(w["x"], np.inf)
    o2 = oracle_from(w2)
    o1.step(H)
    o2.step(H)
    s1, s2 = o1.state(), o2.state()
    chaos = max(rel(s2["v"], s1["v"]), rel(s2["w"], s1["w"]))
    assert chaos < 0.1 * TOL64, chaos
    g = solver(w)
    g.step(H)
    sg = g.state()
    for k in ("v", "w", "q"):
        assert rel(sg[k], s1[k]) < TOL64, k
    assert rel(sg["x"] - w["x"], s1["x"] - w["x"]) < TOL64
    assert np.array_equal(keys(g.contacts()), keys(o1.contacts()))
    c1, cg = o1.contacts(), g.contacts()
    assert max(spring_err(cg, c1).values()) < 1e-10


def test_resynced_steps_cfg1():
    """Re-synced regime over 2,000 steps of configuration 1: every 100 steps
    the oracle takes the GPU state and springs, both advance one step, and
    keys, springs, forces and states must agree."""
    w = W.cfg1()
    g = solver(w)
    total = 0
    for t in range(0, 2000, 100):
        if t:
            g.step(99)
        st = g.state(forces=False)
        c = g.contacts()
        o = oracle_resync(w, st, c, g.stats()["steps"] * w["params"]["dt"])
        g.step(1)
        o.step(1)
        cg, co = g.contacts(), o.contacts()
        assert np.array_equal(keys(cg), keys(co)), t
        total += len(co["ki"])
        if len(co["ki"]):
            assert max(spring_err(cg, co).values()) < TOL64, t
        sg, so, fo = g.state(), o.state(), o.forces()
        assert force_err(sg["F"], fo["F"], fo["Fscale"]) < TOL64, t
        for k in ("v", "w", "q"):
            assert rel(sg[k], so[k]) < TOL64, (t, k)
    assert total > 1000


def check_batch_against_oracle(g, sims, steps):
    """Each simulation of batch context g (stepped `steps` times) against
    its own oracle run: states within the tolerance, contact keys bit for
    bit."""
    st = g.state()
    c = g.contacts()
    off = g.offsets
    for k, w in enumerate(sims):
        assert off[k + 1] - off[k] == len(w["R"])
        if not len(w["R"]):
            continue
        o = oracle_from(w)
        o.step(steps)
        so = o.state()
        sl = slice(off[k], off[k + 1])
        for key in ("v", "q"):
            assert rel(st[key][sl], so[key]) < TOL64, (k, key)
        assert rel_w(st["w"][sl], so["w"], w["R"], so["v"]) < TOL64, k
        m = (c["ki"] >= off[k]) & (c["ki"] < off[k + 1])
        kg = np.stack([c["ki"][m] - off[k], np.where(c["kj"][m] > 0, c["kj"][m] - off[k],
                                                       c["kj"][m])], 1)
        ko = keys(o.contacts())
        assert np.array_equal(kg[np.lexsort((kg[:, 1], kg[:, 0]))], ko)


@pytest.mark.parametrize("skin", [0.0, 0.5])
def test_batch_with_an_empty_simulation(skin):
    """A batch whose middle simulation has a mesh but no particles steps the
    others as separate oracle runs do (with and without kept cells)."""
    a, c = W.cfg4_sim(3, 300), W.cfg4_sim(200, 700)
    for w in (a, c):
        w["x"][:, 2] -= w["x"][:, 2].min() - 0.9e-3
    e = W._finish("empty_in_batch", W.default_params(dt=a["params"]["dt"]), np.zeros((0, 3)),
                  np.zeros(0), np.random.default_rng(1), W.cube_mesh([0, 0, 0], [10e-3] * 3), 5)
    sims = [a, e, c]
    g = solver(sims, skin=skin, detect_lanes=1) if skin else solver(sims)
    g.step(6)
    check_batch_against_oracle(g, sims, 6)
    g.close()


def test_batch_of_uneven_simulations():
    """Several independent simulations in one context (different sizes,
    friction and meshes) match separate oracle runs."""
    sims = [W.cfg4_sim(s, n) for s, n in ((0, 500), (77, 1400), (255, 830))]
    for s in sims:  # start them in contact with each other and the floor
        s["x"][:, 2] -= s["x"][:, 2].min() - 0.9e-3
    g = solver(sims)
    g.step(5)
    check_batch_against_oracle(g, sims, 5)


def test_empty_system():
    w = W._finish("empty", W.default_params(), np.zeros((0, 3)), np.zeros(0),
                  np.random.default_rng(0), W.cube_mesh([0] * 3, [1e-2] * 3), 1)
    g = solver(w)
    g.step(4)
    assert g.stats()["steps"] == 4
    assert len(g.contacts()["ki"]) == 0


def test_contact_capacity_error_leaves_previous_state():
    from paper_2507_12610_amd import SdemError
    w = cluster_case(n=300)
    g = solver(w, contacts_max=16)
    with pytest.raises(SdemError) as ei:
        g.step(3)
    assert "ECAPACITY" in str(ei.value) and "contacts" in str(ei.value)
    st = g.state(forces=False)
    assert np.array_equal(st["x"], w["x"])  # the failed first step is abandoned
    with pytest.raises(SdemError):
        g.step(1)  # no further steps on a failed context


def test_nonfinite_input_is_reported():
    from paper_2507_12610_amd import SdemError
    w = cluster_case(n=50)
    w["x"][7, 1] = np.nan
    g = solver(w)
    with pytest.raises(SdemError) as ei:
        g.step(1)
    assert "ENONFINITE" in str(ei.value)


def test_grid_capacity_error_for_far_particle():
    from paper_2507_12610_amd import SdemError
    w = cluster_case(n=50, mesh=False)
    g = solver(w, cells_max=4096)
    w2 = dict(w)
    w2["x"] = w["x"].copy()
    w2["x"][0] = [1e3, 1e3, 1e3]
    g2 = solver(w2, cells_max=4096)
    g.step(1)
    with pytest.raises(SdemError) as ei:
        g2.step(1)
    assert "ECAPACITY" in str(ei.value) and "cells" in str(ei.value)


def test_bad_parameters_rejected():
    from paper_2507_12610_amd import SdemError
    for bad in (dict(nu=0.7), dict(e_n=1.5), dict(mu_s=-1.0), dict(dt=0.0), dict(rho=-1.0)):
        w = cluster_case(n=10, mesh=False)
        w["params"].update(bad)
        with pytest.raises(SdemError) as ei:
            solver(w)
        assert "EINVAL" in str(ei.value)
    w = cluster_case(n=10, mesh=False)
    w["R"][3] = 0.0
    with pytest.raises(SdemError):
        solver(w)


def test_set_history_round_trip():
    """Springs loaded through sdem_set_history are carried like the oracle's."""
    w = cluster_case(n=300)
    o = oracle_from(w)
    o.step(3)
    co = o.contacts()
    st = o.state()
    w2 = dict(w)
    w2.update(x=st["x"], v=st["v"], w=st["w"], q=st["q"])
    g = solver(w2)
    # resync the oracle from the same inputs, same history
    o2 = oracle_resync(w, st, co, 3 * w["params"]["dt"])
    g.set_history(co["ki"], co["kj"], co["us"], co["ur"], co["ut"])
    # the GPU mesh clock starts at 0: use a static mesh (it is static here)
    g.step(1)
    o2.step(1)
    cg, c2 = g.contacts(), o2.contacts()
    assert np.array_equal(keys(cg), keys(c2))
    assert max(spring_err(cg, c2).values()) < TOL64


def test_rotating_mesh_drum_segment():
    """Extension for the rotating drum: a small drum (rotating mesh) with
    particles resting in it, against the oracle's rotating mesh."""
    tri = W.drum_mesh(0.012, 0.02, nseg=32, nring=4)
    rng = np.random.default_rng(3)
    n = 200
    R = rng.uniform(0.9e-3, 1.1e-3, n)
    x = W.rsa_place(0.93 * R, [-0.011, -0.009, -0.011], [0.011, 0.009, 0.0], 5, shape=1,
                    cyl=(0.0, 0.0, 0.0108, 0.0))
    p = W.default_params(dt=2e-6, mesh_omega=(0.0, 3.0, 0.0))
    w = W._finish("drum", p, x, R, rng, tri, 1)
    g = solver(w)
    o = oracle_from(w)
    for _ in range(3):
        g.step(10)
        o.step(10)
        assert np.array_equal(keys(g.contacts()), keys(o.contacts()))
    sg, so = g.state(), o.state()
    for k in ("v", "w"):
        assert rel(sg[k], so[k]) < 1e-11, k


@pytest.mark.parametrize("cf", [0.25, 0.4, 0.7, 1.0, 1.6])
def test_contact_set_independent_of_cell_size(cf):
    """Strongly polydisperse spheres (radii 0.3-1.5 mm): the per-particle
    search box finds the same contacts for any cell edge, smaller or larger
    than the largest diameter, and the step matches the oracle."""
    w = W.random_cluster(600, 31, box=18e-3, overlap=0.2, r_lo=0.3e-3, r_hi=1.5e-3,
                         tri=W.cube_mesh([-0.2e-3] * 3, [18.2e-3] * 3))
    w["params"].update(g=(0.0, 0.0, -9.81))
    compare_one_step(w, cell_factor=cf)


def test_contact_capacity_error_on_a_step_that_keeps_the_cells():
    """One slot group (at most 256 spheres), cells kept between rebuilds and
    one search lane, so steps that keep the cells run the search and the
    contact law in one kernel: with room for exactly the most contacts of
    the steps before, the first step that needs more, one that keeps the
    cells, fails with ECAPACITY and leaves the previous step's state."""
    from paper_2507_12610_amd import SdemError
    w = W.random_cluster(220, 5, box=9e-3, overlap=0.1, r_lo=0.4e-3, r_hi=0.9e-3, vel=0.4,
                         spin=50.0, tri=W.cube_mesh([-0.2e-3] * 3, [9.2e-3] * 3))
    w["params"].update(g=(0.0, 0.0, -9.81), dt=2e-6)
    kw = dict(cell_factor=0.5, detect_lanes=1, skin=0.3)
    ref = solver(w, **kw)
    counts, rebuilt, states = [], [], [ref.state(forces=False)["x"]]
    for _ in range(300):
        a = ref.stats()
        ref.step(1)
        b = ref.stats()
        counts.append((b["pp"] - a["pp"]) + (b["pw"] - a["pw"]))
        rebuilt.append(b["rebuilds"] > a["rebuilds"])
        states.append(ref.state(forces=False)["x"])
    t = next(t for t in range(1, len(counts))
             if counts[t] > max(counts[:t]) and not rebuilt[t])
    cap = max(counts[:t])
    g = solver(w, contacts_max=cap, **kw)
    for k in range(t):
        g.step(1)
    assert np.array_equal(g.state(forces=False)["x"], states[t])
    with pytest.raises(SdemError) as ei:
        g.step(1)
    assert "ECAPACITY" in str(ei.value) and "contacts" in str(ei.value)
    assert np.array_equal(g.state(forces=False)["x"], states[t])
