"""GPU checks of the file formats and of resuming a run: the CSV state read
back exactly; a hopper whose mesh comes from an OFF file (face radius indices
into Table 2's radius list) saved mid-run (state, springs, clock, spawn
position) and resumed in a fresh context, which then follows the original:
keys bit for bit, states within 1e-12 (the resumed context sums a particle's
contacts in its own slot order); and the same resume from files that hold
the oracle's run, against the oracle going on."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.parity_util import keys, rel, rel_w, spring_err

pytestmark = pytest.mark.gpu

RADII = [0.0, 0.002, 0.02, 0.01]  # 0 for the walls, then Table 2's R_mesh list


def write_off(path, els, rm):
    verts, faces = [], []
    for e, r in zip(els, rm):
        e = np.asarray(e).reshape(-1, 3)
        idx = list(range(len(verts), len(verts) + len(e)))
        verts += e.tolist()
        faces.append("%d %s %d" % (len(e), " ".join(map(str, idx)), RADII.index(r)))
    with open(path, "w") as f:
        f.write("OFF\n%d %d 0\n" % (len(verts), len(faces)))
        for v in verts:
            f.write("%.17g %.17g %.17g\n" % tuple(v))
        f.write("\n".join(faces) + "\n")


def scene(tmp_path):
    from paper_2507_12610_amd import sdem
    els, rm = W.hopper_elements()
    write_off(tmp_path / "hopper.off", els, rm)
    els2, rm2 = sdem.read_off(str(tmp_path / "hopper.off"), RADII)
    assert len(els2) == len(els)
    for a, b in zip(els, els2):
        assert np.array_equal(np.asarray(a), b)
    assert np.array_equal(rm, rm2)
    w = W._finish("hopper", W.hopper_params(), np.zeros((0, 3)), np.zeros(0),
                  np.random.default_rng(0), None, 1)
    w["elements"], w["rmesh"] = els2, rm2
    sp = W.hopper_spawn(n_max=1500)
    sp.update(smin=(-0.06, -0.06, 0.15), smax=(0.06, 0.06, 0.22))
    return w, sp


def test_csv_state_round_trip(tmp_path):
    from paper_2507_12610_amd import Solver, sdem
    w, sp = scene(tmp_path)
    g = Solver(w, device="cuda:0", spawn=sp)
    g.step(120)
    g.write_csv(str(tmp_path / "frame.csv"))
    st, back = g.state(forces=False), sdem.read_csv(str(tmp_path / "frame.csv"))
    for k in ("x", "v", "w", "q"):
        assert np.array_equal(back[k], st[k]), k
    assert np.array_equal(back["R"], g.radii())


def test_resume_from_files(tmp_path):
    from paper_2507_12610_amd import Solver, sdem
    w, sp = scene(tmp_path)
    a = Solver(w, device="cuda:0", spawn=sp)
    a.step(300)
    a.write_csv(str(tmp_path / "state.csv"))
    a.write_contacts_csv(str(tmp_path / "contacts.csv"))
    steps = a.stats()["steps"]
    n, attempts, carried = a.spawn_status()
    # a fresh context from the files
    st = sdem.read_csv(str(tmp_path / "state.csv"))
    w2 = dict(w)
    w2.update(x=st["x"], v=st["v"], w=st["w"], q=st["q"], R=st["R"])
    b = Solver(w2, device="cuda:0", spawn=sp)
    c = sdem.read_contacts_csv(str(tmp_path / "contacts.csv"))
    assert len(c["ki"]) > 30
    b.set_history(c["ki"], c["kj"], c["us"], c["ur"], c["ut"])
    b.set_clock(steps)
    b.set_spawn_status(attempts, carried)
    for k in range(5):
        a.step(10)
        b.step(10)
        assert a.spawn_status() == b.spawn_status(), k
        assert np.array_equal(a.radii(), b.radii()), k
        ca, cb = a.contacts(), b.contacts()
        assert np.array_equal(keys(ca), keys(cb)), k
        assert max(spring_err(cb, ca).values()) < 1e-12, k
        sa, sb = a.state(), b.state()
        for q in ("x", "v", "w", "q"):
            assert rel(sb[q], sa[q]) < 1e-12, (k, q)
    assert b.stats()["steps"] == steps + 50


def write_state_csv(path, st, R):
    """A state file in the library's column layout, from host arrays."""
    with open(path, "w") as f:
        f.write("id,x,y,z,vx,vy,vz,wx,wy,wz,q0,q1,q2,q3,R\n")
        for i in range(len(R)):
            vals = [*st["x"][i], *st["v"][i], *st["w"][i], *st["q"][i], R[i]]
            f.write("%d," % i + ",".join("%.17g" % v for v in vals) + "\n")


def write_contacts_csv(path, c):
    with open(path, "w") as f:
        f.write("ki,kj,usx,usy,usz,urx,ury,urz,ut\n")
        for e in range(len(c["ki"])):
            vals = [*c["us"][e], *c["ur"][e], c["ut"][e]]
            f.write("%d,%d," % (c["ki"][e], c["kj"][e]) + ",".join("%.17g" % v for v in vals)
                    + "\n")


def test_resume_from_oracle_files(tmp_path):
    """The oracle runs the hopper for 300 steps (spawning from an empty
    container); its state and springs are written in the library's file
    formats by this test, read by the library's parsers, and a fresh GPU
    context resumes from them with the clock and the spawn position.  It then
    follows the oracle, which goes on from its own run: spawn status, radii
    and keys bit for bit, springs and states within 1e-12, every 10 of 50
    steps."""
    from paper_2507_12610_amd import Solver, sdem
    w, sp = scene(tmp_path)
    o = oracle.Sim(w["params"], np.zeros((0, 3)), R=np.zeros(0), elements=w["elements"],
                   rmesh=w["rmesh"])
    o.set_spawn(**sp)
    o.step(300)
    attempts, carried = o.spawn_status()
    c0 = o.contacts()
    assert o.n > 100 and len(c0["ki"]) > 30
    write_state_csv(tmp_path / "state.csv", o.state(), o.radii)
    write_contacts_csv(tmp_path / "contacts.csv", c0)
    st = sdem.read_csv(str(tmp_path / "state.csv"))
    w2 = dict(w)
    w2.update(x=st["x"], v=st["v"], w=st["w"], q=st["q"], R=st["R"])
    g = Solver(w2, device="cuda:0", spawn=sp)
    c = sdem.read_contacts_csv(str(tmp_path / "contacts.csv"))
    g.set_history(c["ki"], c["kj"], c["us"], c["ur"], c["ut"])
    g.set_clock(300)
    g.set_spawn_status(attempts, carried)
    for k in range(5):
        o.step(10)
        g.step(10)
        n, ga, gc = g.spawn_status()
        assert (n, ga, gc) == (o.n, *o.spawn_status()), k
        assert np.array_equal(g.radii(), o.radii), k
        cg, co = g.contacts(), o.contacts()
        assert np.array_equal(keys(cg), keys(co)), k
        assert max(spring_err(cg, co).values()) < 1e-12, k
        sg, so = g.state(forces=False), o.state()
        for q in ("x", "v", "q"):
            assert rel(sg[q], so[q]) < 1e-12, (k, q)
        assert rel_w(sg["w"], so["w"], o.radii, so["v"]) < 1e-12, k
    assert g.stats()["steps"] == 350
