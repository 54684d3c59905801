"""Pins of the oracle's moving meshes (an extension generalising the rotating
drum; the vibrated base of the segregation example of Section 4): vertices
against scipy rotations, the default group against the rotating mesh, and
two closed forms of a sphere on a vibrated floor (rolling without slip at
2/7 of the floor's speed; the quasi-static Hertz overlap under the floor's
acceleration)."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle as O
import workloads as W


def mass(rho, R):
    return 4.0 / 3.0 * math.pi * rho * R ** 3


def P(**kw):
    base = dict(rho=2500.0, E=1e6, nu=0.3, e_n=0.3, mu_s=0.5, mu_r=0.0, mu_t=0.0, eta=0.0,
                g=(0.0, 0.0, -9.81), dt=2e-6)
    base.update(kw)
    return O.make_params(**base)


def delta_eq(R, accel=9.81, rho=2500.0, E=1e6, nu=0.3):
    Ew = E / (1 - nu ** 2)
    return (mass(rho, R) * accel / (4.0 / 3.0 * Ew * math.sqrt(R))) ** (2.0 / 3.0)


def floor_rect(h=0.05):
    return [[-h, -h, 0.0], [h, -h, 0.0], [h, h, 0.0], [-h, h, 0.0]]


def test_vertices_follow_rotation_and_displacement():
    els, rm = W.primitive_mesh(20e-3, 4)
    groups = np.arange(len(els)) % 3
    mo = [dict(omega=(0.0, 0.0, 3.0), center=(0.01, 0.01, 0.0)),
          dict(amp=(1e-3, 0.0, 2e-3), freq=15.0, phase=0.4),
          dict(omega=(1.0, -2.0, 0.5), center=(0.0, 0.02, 0.01), amp=(0.0, 5e-4, 0.0), freq=7.0,
               phase=-1.0)]
    s = O.Sim(P(g=(0, 0, 0)), np.array([[1.0, 1.0, 1.0]]), R=[1e-3], elements=els, rmesh=rm)
    s.set_mesh_motion(mo, groups)
    s.step(1234)
    t = s.time
    got = s.mesh()
    for m, e in enumerate(els):
        g = mo[groups[m]]
        e = np.asarray(e).reshape(-1, 3)
        d = np.array(g.get("amp", (0, 0, 0))) * (math.sin(2 * math.pi * g.get("freq", 0) * t +
                                                          g.get("phase", 0)) -
                                                 math.sin(g.get("phase", 0)))
        c = np.array(g.get("center", (0, 0, 0)))
        ref = Rotation.from_rotvec(np.array(g.get("omega", (0, 0, 0))) * t).apply(e - c) + c + d
        assert np.allclose(got[m, :len(e)], ref, rtol=0, atol=1e-15), m


def test_default_group_is_the_rotating_mesh():
    """A one-group table with the parameters' rotation gives the same run
    bit for bit as no table (the rotating-mesh reading)."""
    tri = W.drum_mesh(0.012, 0.02, nseg=16, nring=3)
    w = W.random_cluster(80, 5, box=10e-3, overlap=0.1)
    x = w["x"] - 5e-3
    p = P(mesh_omega=(0.0, 4.0, 0.0), mesh_center=(0.0, 0.0, 0.0))
    a = O.Sim(p, x, v=w["v"], R=w["R"], tri=tri)
    b = O.Sim(p, x, v=w["v"], R=w["R"], tri=tri)
    b.set_mesh_motion([dict(omega=(0.0, 4.0, 0.0), center=(0.0, 0.0, 0.0))])
    a.step(300)
    b.step(300)
    assert np.array_equal(a.state()["v"], b.state()["v"])
    assert np.array_equal(a.mesh(), b.mesh())
    assert len(a.contacts()["ki"]) > 10


def test_rolling_on_a_horizontally_vibrated_floor():
    """No slip, no rolling friction: the bottom point moves with the floor,
    so v = v_floor - w R and (7/2) m dv/dt = m a_floor: v(t) = (2/7) v_floor(t)
    when both start at rest (phase pi/2, so v_floor(0) = 0)."""
    R, f = 1e-3, 10.0
    w_ = 2 * math.pi * f
    A = 0.5 * 9.81 / w_ ** 2  # peak floor acceleration g/2 < (7/2) mu_s g
    s = O.Sim(P(), [[0.0, 0.0, R - delta_eq(R)]], R=[R], elements=[floor_rect()])
    s.set_mesh_motion([dict(amp=(A, 0.0, 0.0), freq=f, phase=math.pi / 2)])
    vmax = A * w_
    worst = 0.0
    dt = 2e-6
    for k in range(1, 101):
        s.step(500)  # 1 ms
        t = s.time
        vf = A * w_ * math.cos(w_ * t + math.pi / 2)
        worst = max(worst, abs(s.state()["v"][0, 0] - 2.0 / 7.0 * vf))
    assert worst < 0.01 * (2.0 / 7.0) * vmax
    assert abs(s.state()["x"][0, 1]) < 1e-15


def test_resting_on_a_vertically_vibrated_floor():
    """Ex. F's agitated base at a peak acceleration below g: the sphere
    stays on the floor and, the floor being slow next to the contact's own
    oscillation, its overlap is the Hertz overlap under g + a_floor(t)."""
    R, f = 1e-3, 20.0
    w_ = 2 * math.pi * f
    A = 0.5 * 9.81 / w_ ** 2
    s = O.Sim(P(e_n=0.3), [[0.0, 0.0, R - delta_eq(R)]], R=[R], elements=[floor_rect()])
    s.set_mesh_motion([dict(amp=(0.0, 0.0, A), freq=f, phase=math.pi / 2)])
    s.step(10000)  # let the start transient decay (20 ms)
    d0 = delta_eq(R)
    worst = 0.0
    for k in range(50):
        s.step(200)
        t = s.time
        zf = A * (math.sin(w_ * t + math.pi / 2) - 1.0)
        af = -A * w_ ** 2 * math.sin(w_ * t + math.pi / 2)
        assert len(s.contacts()["ki"]) == 1
        delta = (zf + R) - s.state()["x"][0, 2]
        worst = max(worst, abs(delta - delta_eq(R, 9.81 + af)))
    assert worst < 0.03 * d0


def test_motion_validation():
    s = O.Sim(P(), np.array([[0.0, 0.0, 1.0]]), R=[1e-3], elements=[floor_rect()])
    with pytest.raises(ValueError):
        s.set_mesh_motion([dict(freq=-1.0)])
    with pytest.raises(ValueError):
        s.set_mesh_motion([dict()], groups=[1])
    with pytest.raises(ValueError):
        s.set_mesh_motion([dict(amp=(np.nan, 0, 0))])


def test_wall_velocity_is_the_vertex_velocity():
    """The material velocity of the wall at a vertex equals the time
    derivative of that vertex's trajectory (central differences of the
    moved vertices, step h = 1e-6 s), for a group that turns and vibrates at
    once (the rotation centre moves with the displacement)."""
    el = [[0.01, 0.0, 0.0], [0.02, 0.005, 0.0], [0.01, 0.01, 0.003]]
    mo = [dict(omega=(0.5, -1.0, 2.0), center=(0.002, -0.001, 0.004), amp=(2e-3, -1e-3, 3e-3),
               freq=12.0, phase=0.3)]
    h = 1e-6

    def sim_at(k):
        s = O.Sim(P(dt=h, g=(0, 0, 0)), np.array([[1.0, 1.0, 1.0]]), R=[1e-3], elements=[el])
        s.set_mesh_motion(mo)
        s.set_time(k * h)
        return s
    mid = sim_at(5000)
    xm, xp = sim_at(4999).mesh()[0], sim_at(5001).mesh()[0]
    for v in range(3):
        vw, ww = mid.wall_velocity(0, mid.mesh()[0, v])
        fd = (xp[v] - xm[v]) / (2 * h)
        assert np.allclose(vw, fd, rtol=1e-6, atol=1e-9), v
        assert np.array_equal(ww, mo[0]["omega"])
