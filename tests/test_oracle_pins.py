"""Pins of the FP64 CPU oracle against facts that do not come from the oracle
itself: values the paper prints, textbook closed forms (Hertz impact time,
Hertz equilibrium, rigid-body rolling), exact conservation laws, discrete
closed forms of the integrator, library routines (scipy rotations, k-d
trees) and brute force on tiny inputs.  Each test names the passage it pins.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.spatial import cKDTree
from scipy.spatial.transform import Rotation

import oracle as O
import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def mass(rho, R):
    return 4.0 / 3.0 * math.pi * rho * R ** 3


def inertia(rho, R):
    return 0.4 * mass(rho, R) * R ** 2


def P(**kw):
    base = dict(rho=2500.0, E=1e6, nu=0.3, e_n=0.5, mu_s=0.5, mu_r=0.1, mu_t=0.1, eta=0.0,
                g=(0.0, 0.0, 0.0), dt=1e-6)
    base.update(kw)
    return O.make_params(**base)


# --------------------------------------------------------------------------
# printed values (Section 2.3, Table 2, Section 2.2)
# --------------------------------------------------------------------------
def test_dt_worked_example():
    g = GOLD["dt_worked_example"]
    dt = O.dt_default(g["R"], g["rho"], g["E"], g["nu"])
    assert abs(dt - g["dt_about"]) / g["dt_about"] < 0.02
    assert abs(60.0 / dt - g["steps_per_minute_about"]) / g["steps_per_minute_about"] < 0.01
    d = GOLD["default_run"]
    t = d["N_frames"] * d["N_steps"] * O.dt_default(d["R_min"], d["rho"], d["E"], d["nu"])
    assert abs(t - d["physical_time_about"]) / d["physical_time_about"] < 0.01


def test_beta_special_values():
    # e_n = 1: no damping (beta = 0); e_n = 0: beta = 1 (Section 2.2, Eq. cn)
    assert O.beta(1.0) == 0.0
    assert O.beta(0.0) == 1.0
    # monotone decreasing in e_n
    e = np.linspace(0.01, 0.99, 50)
    b = np.array([O.beta(x) for x in e])
    assert np.all(np.diff(b) < 0)


@pytest.mark.parametrize("nu", [-0.9, -0.5, 0.0, 0.3, 0.5])
def test_damping_ratio_equal_spheres(nu):
    """c_s/c_n = sqrt((1-nu)/(10(2-nu))) in (0.18, 0.26) (Section 2.2)."""
    rng = GOLD["damping_ratio_range"]
    p = P(nu=nu)
    o = O.eval_pp(p, [1.9e-3, 0, 0], [0, 0, 0], [0, 0, 0], 1e-3, [0, 0, 0], [0, 0, 0], [0, 0, 0],
                  1e-3)
    ratio = o["cs"] / o["cn"]
    assert ratio == pytest.approx(math.sqrt((1 - nu) / (10 * (2 - nu))), rel=1e-13)
    assert rng["lo"] < ratio < rng["hi"]


@pytest.mark.parametrize("wall", [False, True])
def test_effective_moduli_general_definition(wall):
    """k_n = 4/3 E* a, k_s = 8 G* a, a = sqrt(R* delta) with the general
    two-body E*, G*, R* of Section 2.2, and the rigid-wall limits
    R_j = E_j = m_j = inf."""
    E, nu, Ri, Rj = 2.3e6, 0.27, 1.1e-3, 0.7e-3
    p = P(E=E, nu=nu)
    G = E / (2 * (1 + nu))
    if wall:
        o = O.eval_pw(p, [0, 0, 1.0e-3], [0, 0, 0], [0, 0, 0], Ri, [0, 0, 0])
        Es, Gs, Rs = 1 / ((1 - nu ** 2) / E), 1 / ((2 - nu) / G), Ri
    else:
        o = O.eval_pp(p, [1.7e-3, 0, 0], [0, 0, 0], [0, 0, 0], Ri, [0, 0, 0], [0, 0, 0], [0, 0, 0], Rj)
        Es = 1 / ((1 - nu ** 2) / E + (1 - nu ** 2) / E)
        Gs = 1 / ((2 - nu) / G + (2 - nu) / G)
        Rs = 1 / (1 / Ri + 1 / Rj)
    a = math.sqrt(Rs * o["delta"])
    assert o["kn"] == pytest.approx(4.0 / 3.0 * Es * a, rel=1e-13)
    assert o["ks"] == pytest.approx(8.0 * Gs * a, rel=1e-13)


# --------------------------------------------------------------------------
# head-on collisions: restitution definition and Hertz impact time
# --------------------------------------------------------------------------
def collide(e_n, v0, Ri=1e-3, Rj=1e-3, dt=2e-7):
    p = P(e_n=e_n, dt=dt)
    x = np.array([[0.0, 0, 0], [Ri + Rj + 1e-12, 0, 0]])
    mi, mj = mass(2500.0, Ri), mass(2500.0, Rj)
    v = np.array([[v0 * mj / (mi + mj), 0, 0], [-v0 * mi / (mi + mj), 0, 0]])
    s = O.Sim(p, x, v=v, R=[Ri, Rj])
    started, tc = False, 0.0
    for _ in range(100000):
        s.step(1)
        nc = O.lib().orc_num_contacts(s._h)
        if nc:
            started, tc = True, tc + dt
        elif started:
            break
    st = s.state()
    return (st["v"][1, 0] - st["v"][0, 0]) / v0, tc


@pytest.mark.parametrize("e_n", GOLD["restitution_definition"]["e_n"])
def test_restitution_equals_e_n(e_n):
    """v_n' = -e_n v_n (Section 2.2) for Hertz contact with c_n =
    sqrt(5 m* k_n) beta, independent of the impact speed and of the size
    ratio."""
    for v0, Rj in ((0.1, 1e-3), (1.0, 1e-3), (0.5, 0.6e-3)):
        e_out, _ = collide(e_n, v0, Rj=Rj)
        assert e_out == pytest.approx(e_n, abs=2e-3), (v0, Rj)


@pytest.mark.parametrize("v0,Rj", [(0.1, 1e-3), (1.0, 0.6e-3)])
def test_hertz_impact_duration(v0, Rj):
    """Elastic (e_n = 1) Hertz impact lasts 2.868 (m*^2/(R* E*^2 v0))^(1/5)
    (textbook Hertz collision time, e.g. Johnson, Contact Mechanics)."""
    Ri = 1e-3
    _, tc = collide(1.0, v0, Rj=Rj)
    ms = 1 / (1 / mass(2500.0, Ri) + 1 / mass(2500.0, Rj))
    Rs = 1 / (1 / Ri + 1 / Rj)
    Es = 1e6 / (2 * (1 - 0.09))
    t_hertz = 2.868 * (ms ** 2 / (Rs * Es ** 2 * v0)) ** 0.2
    assert tc == pytest.approx(t_hertz, rel=2e-3)


# --------------------------------------------------------------------------
# single sphere on a floor: Hertz equilibrium, sliding, rolling, twisting
# --------------------------------------------------------------------------
def floor():
    return W.floor_mesh(0.0, 0.0, 0.2, 0.0)


def delta_eq(R, rho=2500.0, E=1e6, nu=0.3, g=9.81):
    # Hertz sphere on a rigid half-space: m g = 4/3 E_w sqrt(R) delta^(3/2)
    Ew = E / (1 - nu ** 2)
    return (mass(rho, R) * g / (4.0 / 3.0 * Ew * math.sqrt(R))) ** (2.0 / 3.0)


def sphere_on_floor(R=1e-3, v=(0, 0, 0), w=(0, 0, 0), dt=2e-6, **kw):
    p = P(g=(0, 0, -9.81), dt=dt, **kw)
    x = np.array([[0.013, 0.007, R - delta_eq(R)]])
    return O.Sim(p, x, v=[v], w=[w], R=[R], tri=floor())


def test_hertz_static_equilibrium():
    s = sphere_on_floor(e_n=0.3)
    s.x0 = None
    st0 = s.state()
    s.step(20000)
    R = 1e-3
    z = s.state()["x"][0, 2]
    assert (R - z) == pytest.approx(delta_eq(R), rel=1e-6)
    F = s.forces()["F"][0]
    assert F[2] == pytest.approx(mass(2500.0, R) * 9.81, rel=1e-6)
    assert st0["x"][0, 2] < R


def run_series(s, chunks, every):
    out = []
    for _ in range(chunks):
        s.step(every)
        st = s.state()
        out.append((s.time, st["v"][0].copy(), st["w"][0].copy()))
    return out


def test_sliding_to_rolling_transition():
    """Kinetic Coulomb sliding decelerates at mu_s g and spins the sphere up
    until v = r_i w, then it rolls at v0/(1 + I/(m r_i^2)) (rigid body with a
    kinetic friction force mu_s m g at lever r_i; Eq. Coulombs, tau_s)."""
    R, v0, mu = 1e-3, 0.3, 0.3
    s = sphere_on_floor(R=R, v=(v0, 0, 0), mu_s=mu, mu_r=0.0, mu_t=0.0, e_n=0.5, dt=2e-6)
    ri = R - delta_eq(R) / 2
    m, I = mass(2500.0, R), inertia(2500.0, R)
    t_star = v0 / (mu * 9.81 * (1 + m * ri * ri / I))
    series = run_series(s, 80, 500)
    t = np.array([a[0] for a in series])
    v = np.array([a[1][0] for a in series])
    # kinetic phase: dv/dt = -mu g
    early = t < 0.6 * t_star
    slope = np.polyfit(t[early], v[early], 1)[0]
    assert slope == pytest.approx(-mu * 9.81, rel=2e-3)
    v_f = v0 / (1 + I / (m * ri * ri))
    assert v[-1] == pytest.approx(v_f, rel=2e-3)
    # rolling without slip at the end: v = r_i w_y
    assert series[-1][2][1] * ri == pytest.approx(v[-1], rel=2e-3)


def test_rolling_friction_deceleration():
    """Kinetic rolling resistance |f_r| = mu_r |f_n| with torque R* n x f_r
    (R* = R for a wall) decelerates a sphere rolling without slip at
    mu_r g (R/r_i) / (1 + I/(m r_i^2))."""
    R, v0, mu_r = 1e-3, 0.2, 0.05
    ri = R - delta_eq(R) / 2
    s = sphere_on_floor(R=R, v=(v0, 0, 0), w=(0, v0 / ri, 0), mu_s=2.0, mu_r=mu_r, mu_t=0.0,
                        e_n=0.5, dt=2e-6)
    m, I = mass(2500.0, R), inertia(2500.0, R)
    series = run_series(s, 40, 500)
    t = np.array([a[0] for a in series])[5:]
    v = np.array([a[1][0] for a in series])[5:]
    slope = np.polyfit(t, v, 1)[0]
    assert slope == pytest.approx(-mu_r * 9.81 * (R / ri) / (1 + I / (m * ri * ri)), rel=5e-3)


def test_twisting_friction_spin_down():
    """Kinetic twisting torque mu_t |f_n| R* about n: I dw/dt = -mu_t m g R,
    i.e. dw/dt = -(5/2) mu_t g / R (Eq. ft, Coulombt, tau_t)."""
    R, mu_t = 1e-3, 0.2
    s = sphere_on_floor(R=R, w=(0, 0, 60.0), mu_s=0.5, mu_r=0.5, mu_t=mu_t, e_n=0.5, dt=2e-6)
    series = run_series(s, 20, 200)
    t = np.array([a[0] for a in series])[3:]
    wz = np.array([a[2][2] for a in series])[3:]
    slope = np.polyfit(t, wz, 1)[0]
    assert slope == pytest.approx(-2.5 * mu_t * 9.81 / R, rel=2e-3)


def test_twisting_static_below_threshold():
    """Below mu_t, a twisting spring holds: a small spin is stopped and the
    twist stays static."""
    s = sphere_on_floor(w=(0, 0, 0.5), mu_t=0.5, e_n=0.5, dt=2e-6)
    s.step(4000)
    c = s.contacts()
    assert len(c["ki"]) == 1
    o_w = s.state()["w"][0, 2]
    assert abs(o_w) < 0.5


# --------------------------------------------------------------------------
# conservation laws (Section 3.2 antisymmetry, Section 2.3 symplectic Euler)
# --------------------------------------------------------------------------
def cluster(n=60, seed=3, **kw):
    w = W.random_cluster(n, seed, box=8e-3, overlap=0.12)
    p = P(**kw)
    return O.Sim(p, w["x"], v=w["v"], w=w["w"], q=w["q"], R=w["R"]), w


def momenta(s, R, rho=2500.0):
    st = s.state()
    m = mass(rho, R)[:, None]
    I = inertia(rho, R)[:, None]
    Pm = (m * st["v"]).sum(0)
    L = (np.cross(st["x"], m * st["v"]) + I * st["w"]).sum(0)
    scaleP = (m * np.abs(st["v"])).sum()
    scaleL = np.abs(np.cross(st["x"], m * st["v"])).sum() + (I * np.abs(st["w"])).sum()
    return Pm, L, scaleP, scaleL


def test_momentum_and_angular_momentum_conserved():
    """Single-evaluation antisymmetry (Eq. antisymm_normal..antisymm_sliding)
    conserves linear momentum and, because r_i + r_j = d, angular momentum
    exactly under the semi-implicit update (g = 0, eta = 0, no mesh)."""
    s, w = cluster(e_n=0.7, mu_s=0.5, mu_r=0.2, mu_t=0.3, dt=2e-6)
    P0, L0, sP, sL = momenta(s, w["R"])
    total = 0
    for _ in range(20):
        s.step(10)
        total += len(s.contacts()["ki"])
    P1, L1, _, _ = momenta(s, w["R"])
    assert total > 100  # contacts were exercised
    assert np.abs(P1 - P0).max() <= 1e-13 * sP
    assert np.abs(L1 - L0).max() <= 1e-12 * sL


def hertz_energy(s, R, tri, rho=2500.0, E=1e6, nu=0.3):
    st = s.state()
    g = np.array(s.params.g[:])
    m = mass(rho, R)
    I = inertia(rho, R)
    e = (0.5 * m * (st["v"] ** 2).sum(1) + 0.5 * I * (st["w"] ** 2).sum(1)
         - m * (st["x"] @ g)).sum()
    # elastic energy of each contact: integral of 4/3 E* sqrt(R*) delta^(3/2)
    x = st["x"]
    tree = cKDTree(x)
    for i, j in tree.query_pairs(2 * R.max(), output_type="ndarray"):
        d = np.linalg.norm(x[i] - x[j])
        de = R[i] + R[j] - d
        if de > 0:
            Rs = 1 / (1 / R[i] + 1 / R[j])
            e += 8.0 / 15.0 * (E / (2 * (1 - nu ** 2))) * math.sqrt(Rs) * de ** 2.5
    for i in range(len(R)):
        for t in tri:
            cp = closest_point_numpy(x[i], t)
            de = R[i] - np.linalg.norm(x[i] - cp)
            if de > 0:
                e += 8.0 / 15.0 * (E / (1 - nu ** 2)) * math.sqrt(R[i]) * de ** 2.5
    return e


@pytest.mark.parametrize("dt", [2e-6, 1e-6])
def test_energy_bounded_elastic_frictionless(dt):
    """e_n = 1, mu = eta = 0: the semi-implicit Euler scheme keeps the total
    energy (kinetic + gravitational + Hertz elastic) bounded with O(dt)
    fluctuation and no drift (Section 2.3)."""
    w = W.random_cluster(40, 11, box=10e-3, overlap=0.1, vel=0.2)
    tri = W.cube_mesh([-0.5e-3] * 3, [10.5e-3] * 3)
    p = P(e_n=1.0, mu_s=0.0, mu_r=0.0, mu_t=0.0, g=(0, 0, -9.81), dt=dt)
    s = O.Sim(p, w["x"], v=w["v"], w=w["w"], R=w["R"], tri=tri)
    e0 = hertz_energy(s, w["R"], tri)
    scale = abs(e0)
    es = []
    steps = int(round(2e-3 / dt))
    for _ in range(20):
        s.step(steps // 20)
        es.append(hertz_energy(s, w["R"], tri))
    dev = np.max(np.abs(np.array(es) - e0)) / scale
    test_energy_bounded_elastic_frictionless.devs[dt] = dev
    assert dev < 2e-3
    if len(test_energy_bounded_elastic_frictionless.devs) == 2:
        d = test_energy_bounded_elastic_frictionless.devs
        # first order in dt: halving the step roughly halves the excursion
        assert 1.3 < d[2e-6] / d[1e-6] < 3.2


test_energy_bounded_elastic_frictionless.devs = {}


# --------------------------------------------------------------------------
# friction sign (reading R1), spring projection and continuity
# --------------------------------------------------------------------------
def test_meshing_spheres_no_sliding():
    """Two equal spheres counter-rotating like gears have contact points with
    equal velocity: no slip, so no sliding force at first contact."""
    R = 1e-3
    o = O.eval_pp(P(), [1.99e-3, 0, 0], [0, 0, 0], [0, 0, 10.0], R, [0, 0, 0], [0, 0, 0],
                  [0, 0, -10.0], R)
    assert np.linalg.norm(o["fs"]) <= 1e-12 * np.linalg.norm(o["fn"])
    # co-rotating spheres do slip
    o2 = O.eval_pp(P(), [1.99e-3, 0, 0], [0, 0, 0], [0, 0, 10.0], R, [0, 0, 0], [0, 0, 0],
                   [0, 0, 10.0], R)
    assert np.linalg.norm(o2["fs"]) > 1e-3 * np.linalg.norm(o2["fn"])


def test_sliding_power_identity():
    """At first contact (u_s = 0, static) the power of the sliding force and
    its two torques equals f_s . v_s = -c_s |v_s|^2 <= 0 when v_s is the true
    slip velocity of the contact points (rigid-body kinematics)."""
    rng = np.random.default_rng(5)
    for _ in range(50):
        Ri, Rj = rng.uniform(0.7e-3, 1.3e-3, 2)
        nvec = rng.normal(size=3)
        nvec /= np.linalg.norm(nvec)
        d = (Ri + Rj) * (1 - rng.uniform(0.001, 0.05))
        xi = nvec * d
        vi, vj = rng.normal(0, 0.1, 3), rng.normal(0, 0.1, 3)
        wi, wj = rng.normal(0, 50, 3), rng.normal(0, 50, 3)
        o = O.eval_pp(P(mu_s=1e3), xi, vi, wi, Ri, [0, 0, 0], vj, wj, Rj)
        fs, n = o["fs"], o["n"]
        fxn = np.cross(fs, n)
        power = fs @ (vi - vj) + (o["ri"] * fxn) @ wi + (o["rj"] * fxn) @ wj
        scale = np.linalg.norm(fs) * (np.linalg.norm(vi - vj) + Ri * np.linalg.norm(wi)
                                      + Rj * np.linalg.norm(wj))
        assert power == pytest.approx(fs @ o["vs"], abs=1e-12 * scale)
        assert power == pytest.approx(-o["cs"] * (o["vs"] @ o["vs"]), abs=1e-12 * scale)
        assert o["kinetic"][0] == 0


def test_spring_projection_keeps_length():
    """Springs from the previous step are rotated onto the tangent plane and
    keep their length (Eq. um projection); R4 edge cases."""
    rng = np.random.default_rng(7)
    for _ in range(30):
        u = rng.normal(0, 1e-5, 3)
        ur = rng.normal(0, 1e-5, 3)
        o = O.eval_pp(P(mu_s=1e3, mu_r=1e3), [1.95e-3, 0.1e-3, 0], [0.01, 0, 0], [0, 3, 0], 1e-3,
                      [0, 0, 0], [0, 0, 0], [0, 0, 0], 1e-3, us=u, ur=ur)
        n = o["n"]
        for key, vel, old in (("us", "vs", u), ("ur", "vr", ur)):
            proj = o[key] - 1e-6 * o[vel]
            assert abs(proj @ n) <= 1e-12 * np.linalg.norm(old)
            assert np.linalg.norm(proj) == pytest.approx(np.linalg.norm(old), rel=1e-12)
    # a spring exactly along n (n = x here) collapses to zero (reading R4)
    o = O.eval_pp(P(mu_s=1e3), [1.95e-3, 0, 0], [0, 0, 0], [0, 0, 0], 1e-3, [0, 0, 0],
                  [0, 0, 0], [0, 0, 0], 1e-3, us=[3e-5, 0, 0])
    assert np.array_equal(o["n"], [1.0, 0.0, 0.0])
    assert np.array_equal(o["us"], [0.0, 0.0, 0.0])


def test_kinetic_reset_continuity():
    """After a kinetic reset, -k u - c v reproduces the clipped force
    (Eq. fm_kinetic, um_kinetic), for sliding, rolling and twisting."""
    rng = np.random.default_rng(9)
    hits = [0, 0, 0]
    for _ in range(60):
        o = O.eval_pp(P(mu_s=0.2, mu_r=0.05, mu_t=0.1), [1.9e-3, 0.2e-3, 0.1e-3],
                      rng.normal(0, 0.3, 3), rng.normal(0, 300, 3), 1e-3, [0, 0, 0],
                      rng.normal(0, 0.3, 3), rng.normal(0, 300, 3), 1.1e-3,
                      us=rng.normal(0, 1e-4, 3), ur=rng.normal(0, 1e-4, 3),
                      ut=float(rng.normal(0, 1e-4)))
        fnl = np.linalg.norm(o["fn"])
        if o["kinetic"][0]:
            hits[0] += 1
            assert np.linalg.norm(o["fs"]) == pytest.approx(0.2 * fnl, rel=1e-13)
            assert np.allclose(-o["ks"] * o["us"] - o["cs"] * o["vs"], o["fs"],
                               rtol=0, atol=1e-12 * np.linalg.norm(o["fs"]))
        if o["kinetic"][1]:
            hits[1] += 1
            assert np.linalg.norm(o["fr"]) == pytest.approx(0.05 * fnl, rel=1e-13)
            assert np.allclose(-o["kn"] * o["ur"] - o["cn"] * o["vr"], o["fr"],
                               rtol=0, atol=1e-12 * np.linalg.norm(o["fr"]))
        if o["kinetic"][2]:
            hits[2] += 1
            assert abs(o["ft"]) == pytest.approx(0.1 * fnl, rel=1e-13)
            assert -o["ks"] * o["ut"] - o["cs"] * o["vt"] == pytest.approx(o["ft"], rel=1e-12)
    assert min(hits) >= 10


def test_static_spring_increment():
    """In the static regime the spring grows by dt v_m (Eq. um_static)."""
    o = O.eval_pp(P(mu_s=1e3, mu_r=1e3, mu_t=1e3, dt=3e-6), [1.9e-3, 0, 0], [0, 0.02, 0],
                  [1.0, 2.0, 3.0], 1e-3, [0, 0, 0], [0, 0, 0], [0, 0, 0], 1e-3)
    assert o["kinetic"] == [0, 0, 0]
    assert np.allclose(o["us"], 3e-6 * o["vs"], rtol=1e-14, atol=0)
    assert np.allclose(o["ur"], 3e-6 * o["vr"], rtol=1e-14, atol=0)
    assert o["ut"] == pytest.approx(3e-6 * o["vt"], rel=1e-14)


def test_torque_bookkeeping():
    """tau_s = r_i f_s x n on i and r_j f_s x n on j; rolling and twisting
    torques are antisymmetric (Eq. antisymm_*): the pair's total torque
    about the origin vanishes."""
    rng = np.random.default_rng(2)
    for _ in range(20):
        xi = rng.normal(0, 1e-3, 3) + [1.8e-3, 0, 0]
        xj = rng.normal(0, 1e-5, 3)
        if np.linalg.norm(xi - xj) > 2e-3:
            continue
        o = O.eval_pp(P(), xi, rng.normal(0, 0.1, 3), rng.normal(0, 30, 3), 1e-3, xj,
                      rng.normal(0, 0.1, 3), rng.normal(0, 30, 3), 1.05e-3,
                      us=rng.normal(0, 1e-6, 3), ur=rng.normal(0, 1e-6, 3))
        tot = o["ti"] + o["tj"] + np.cross(xi, o["fi"]) + np.cross(xj, o["fj"])
        scale = np.linalg.norm(o["ti"]) + np.linalg.norm(np.cross(xi, o["fi"]))
        assert np.abs(tot).max() <= 1e-12 * scale
        assert np.allclose(o["fi"], -o["fj"], rtol=0, atol=0)


# --------------------------------------------------------------------------
# integrator closed forms (Eq. v, x, spiral, w; Stokes drag Section 2.1)
# --------------------------------------------------------------------------
def test_free_fall_discrete():
    p = P(g=(0.3, -1.0, -9.81), dt=1e-4)
    v0 = np.array([0.1, 0.2, 0.3])
    x0 = np.array([1.0, 2.0, 3.0])
    s = O.Sim(p, [x0], v=[v0], R=[1e-3])
    n = 777
    s.step(n)
    st = s.state()
    g = np.array(p.g[:])
    dt = 1e-4
    assert np.allclose(st["v"][0], v0 + n * dt * g, rtol=1e-12)
    assert np.allclose(st["x"][0], x0 + n * dt * v0 + dt * dt * g * n * (n + 1) / 2, rtol=1e-12)


def to_rot(q):
    return Rotation.from_quat([q[1], q[2], q[3], q[0]])


def test_quat_mul_matches_rotation_composition():
    rng = np.random.default_rng(4)
    for _ in range(20):
        a = rng.normal(size=4)
        b = rng.normal(size=4)
        a /= np.linalg.norm(a)
        b /= np.linalg.norm(b)
        c = O.quat_mul(a, b)
        assert np.allclose((to_rot(a) * to_rot(b)).as_matrix(), to_rot(c).as_matrix(), atol=1e-14)


def test_spiral_constant_spin():
    """alpha = 0, constant w: q_n = q_0 (cos n phi, sin n phi w/|w|)."""
    p = P(dt=1e-4)
    w = np.array([30.0, -20.0, 50.0])
    q0 = np.array([0.5, 0.5, -0.5, 0.5])
    s = O.Sim(p, [[0, 0, 0]], w=[w], q=[q0], R=[1e-3])
    n = 300
    s.step(n)
    q = s.state()["q"][0]
    ang = n * 1e-4 * np.linalg.norm(w)
    expect = to_rot(q0) * Rotation.from_rotvec(w / np.linalg.norm(w) * ang)
    assert np.allclose(to_rot(q).as_matrix(), expect.as_matrix(), atol=1e-12)
    assert np.linalg.norm(q) == pytest.approx(1.0, abs=1e-12)


def test_spiral_constant_torque_order():
    """w_0 = 0 and a constant torque about a fixed axis: the quaternion is
    advanced with the old w before w is updated, with the second factor
    angle (dt/2)^2 |alpha|, so the accumulated angle is exactly
    alpha t^2 / 2 (alpha = T/I, I = 2/5 m R^2)."""
    R = 1e-3
    p = P(dt=1e-4)
    T = np.array([1e-9, 2e-9, -1.5e-9])
    q = np.array([1.0, 0, 0, 0])
    x = v = w = np.zeros(3)
    n = 250
    for _ in range(n):
        x, v, w, q = O.integrate(p, R, [0, 0, 0], T, x, v, w, q)
    alpha = np.linalg.norm(T) / inertia(2500.0, R)
    t = n * 1e-4
    expect = Rotation.from_rotvec(T / np.linalg.norm(T) * alpha * t * t / 2)
    assert np.allclose(to_rot(q).as_matrix(), expect.as_matrix(), atol=1e-11)
    assert np.allclose(w, T / inertia(2500.0, R) * t, rtol=1e-12)


def test_stokes_drag_decay():
    """c = 6 pi eta R / m and gamma = 8 pi eta R^3 / I (Stokes' law): free
    particle, g = 0, v_n = v_0 (1 - dt c)^n, w_n = w_0 (1 - dt gamma)^n."""
    R, eta, rho, dt = 0.8e-3, 1e-3, 2500.0, 1e-4
    p = P(eta=eta, dt=dt, rho=rho)
    v0, w0 = np.array([0.3, -0.1, 0.2]), np.array([5.0, 1.0, -2.0])
    s = O.Sim(p, [[0, 0, 0]], v=[v0], w=[w0], R=[R])
    n = 400
    s.step(n)
    st = s.state()
    c = 6 * math.pi * eta * R / mass(rho, R)
    gam = 8 * math.pi * eta * R ** 3 / inertia(rho, R)
    assert np.allclose(st["v"][0], v0 * (1 - dt * c) ** n, rtol=1e-11)
    assert np.allclose(st["w"][0], w0 * (1 - dt * gam) ** n, rtol=1e-11)


# --------------------------------------------------------------------------
# geometry and contact sets (Section 3.3, Fig. 4C)
# --------------------------------------------------------------------------
def closest_point_numpy(p, tri):
    """Independent point-triangle closest point: orthogonal projection if it
    falls inside, else the best of the three edge segments."""
    a, b, c = tri
    n = np.cross(b - a, c - a)
    n = n / np.linalg.norm(n)
    proj = p - ((p - a) @ n) * n
    # barycentric inside test
    v0, v1, v2 = b - a, c - a, proj - a
    d00, d01, d11, d20, d21 = v0 @ v0, v0 @ v1, v1 @ v1, v2 @ v0, v2 @ v1
    den = d00 * d11 - d01 * d01
    bv = (d11 * d20 - d01 * d21) / den
    bw = (d00 * d21 - d01 * d20) / den
    if bv >= 0 and bw >= 0 and bv + bw <= 1:
        return proj
    best, bd = None, np.inf
    for s, e in ((a, b), (b, c), (c, a)):
        t = np.clip((p - s) @ (e - s) / ((e - s) @ (e - s)), 0, 1)
        q = s + t * (e - s)
        dq = np.linalg.norm(p - q)
        if dq < bd:
            best, bd = q, dq
    return best


def test_closest_point_triangle_vs_independent_method():
    rng = np.random.default_rng(1)
    for _ in range(2000):
        tri = rng.normal(size=(3, 3))
        p = rng.normal(size=3) * 2
        got = O.closest_point_triangle(p, *tri)
        ref = closest_point_numpy(p, tri)
        assert np.linalg.norm(p - got) == pytest.approx(np.linalg.norm(p - ref), rel=1e-9, abs=1e-12)
        assert np.allclose(got, ref, atol=1e-9)


def test_closest_point_interior_is_projection():
    tri = np.array([[0.0, 0, 0], [1.0, 0, 0], [0, 1.0, 0]])
    got = O.closest_point_triangle([0.2, 0.3, 0.7], *tri)
    assert np.allclose(got, [0.2, 0.3, 0.0], rtol=0, atol=1e-15)


def test_closest_point_dense_sampling():
    """Brute force: no sampled point of the triangle is closer."""
    rng = np.random.default_rng(8)
    k = 200
    uu, vv = np.meshgrid(np.linspace(0, 1, k), np.linspace(0, 1, k))
    m = uu + vv <= 1
    bary = np.stack([uu[m], vv[m]], 1)
    for _ in range(50):
        tri = rng.normal(size=(3, 3))
        p = rng.normal(size=3)
        pts = tri[0] + bary[:, :1] * (tri[1] - tri[0]) + bary[:, 1:] * (tri[2] - tri[0])
        dmin = np.linalg.norm(pts - p, axis=1).min()
        got = np.linalg.norm(p - O.closest_point_triangle(p, *tri))
        assert got <= dmin + 1e-12
        assert got >= dmin - 0.02 * np.linalg.norm(tri[1] - tri[0])


def reference_contact_set(x, R, tri):
    """Contact keys by an independent route: k-d tree pairs, and an
    independent point-triangle distance."""
    tree = cKDTree(x)
    keys = set()
    for i, j in tree.query_pairs(2 * R.max() + 1e-9, output_type="ndarray"):
        i, j = min(i, j), max(i, j)
        dv = x[i] - x[j]
        d = math.sqrt((dv[0] * dv[0] + dv[1] * dv[1]) + dv[2] * dv[2])
        if (R[i] + R[j]) - d >= 0:
            keys.add((i, j))
    for i in range(len(R)):
        for m, t in enumerate(tri):
            d = np.linalg.norm(x[i] - closest_point_numpy(x[i], t))
            if R[i] - d >= 0:
                keys.add((i, -m))
    return keys


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_contact_set_brute_force_and_cells(seed):
    w = W.random_cluster(300, seed, box=20e-3, overlap=0.2, r_lo=0.5e-3, r_hi=1.5e-3)
    tri = W.cube_mesh([0.3e-3] * 3, [19.7e-3] * 3)
    s = O.Sim(P(), w["x"], R=w["R"], tri=tri)
    ref = reference_contact_set(w["x"], w["R"], tri)
    assert len(ref) > 100
    for mode, cf in ((0, 1.0), (1, 1.0), (1, 1.7)):
        s.set_search(mode, cf)
        ki, kj = s.contact_keys()
        assert set(zip(ki.tolist(), kj.tolist())) == ref
        # key order: i ascending, then j ascending (signed)
        order = np.lexsort((kj, ki))
        assert np.array_equal(order, np.arange(len(ki)))


def test_sampled_keys_are_the_brute_force_set_per_particle():
    """The per-particle key lists used for full-size checks are the
    brute-force contact set restricted to each listed particle, in key
    order (Section 3.3 contact definition)."""
    w = W.random_cluster(300, 4, box=20e-3, overlap=0.2, r_lo=0.5e-3, r_hi=1.5e-3)
    tri = W.cube_mesh([0.3e-3] * 3, [19.7e-3] * 3)
    s = O.Sim(P(), w["x"], R=w["R"], tri=tri)
    ref = reference_contact_set(w["x"], w["R"], tri)
    idx = np.arange(300)[::-1]
    ki, kj, cnt = s.sample_keys(idx)
    assert cnt.sum() == len(ki) > 200
    pos = 0
    for a, p in enumerate(idx):
        mine = sorted(k for k in ref if k[0] == p or (k[1] > 0 and k[1] == p))
        got = list(zip(ki[pos:pos + cnt[a]].tolist(), kj[pos:pos + cnt[a]].tolist()))
        assert got == mine, p
        pos += cnt[a]


def test_sampled_step_equals_the_full_step():
    """The sampled one-step evaluation gives each listed particle the net
    force, torque and next state of a full step (Section 2.3 forces with the
    carried springs, Section 2.1 integration), here after 30 steps so that
    the springs are loaded and some contacts are kinetic."""
    tri = W.cube_mesh([-0.2e-3] * 3, [14.2e-3] * 3)
    w = W.random_cluster(200, 7, box=14e-3, tri=tri)
    s = O.Sim(w["params"], w["x"], v=w["v"], w=w["w"], q=w["q"], R=w["R"], tri=tri)
    s.step(30)
    assert len(s.contacts()["ki"]) > 100
    idx = np.array([0, 3, 50, 99, 150, 199])
    smp = s.sample_step(idx)
    s.step(1)
    f, st = s.forces(), s.state()
    for k, key in (("F", "Fscale"), ("T", "Tscale")):
        d = np.linalg.norm(smp[k] - f[k][idx], axis=1)
        sc = f[key][idx] + (f["Fscale"][idx] * w["R"][idx] if k == "T" else 0.0)
        assert np.all(d <= 1e-13 * sc), k
    assert np.array_equal(smp["ncont"] > 0, np.linalg.norm(f["F"][idx], axis=1) > 0)
    for k in ("x", "v", "w", "q"):
        sc = np.abs(st[k]).max()
        assert np.abs(smp[k] - st[k][idx]).max() <= 1e-13 * sc, k


def test_contact_set_edge_cases():
    # exactly touching (delta = 0) counts; a hair apart does not
    s = O.Sim(P(), [[0, 0, 0], [2e-3, 0, 0], [4e-3 + 1e-12, 0, 0]], R=[1e-3, 1e-3, 1e-3])
    ki, kj = s.contact_keys()
    assert list(zip(ki, kj)) == [(0, 1)]
    # empty system
    s = O.Sim(P(), np.zeros((0, 3)), R=np.zeros(0))
    s.step(3)
    assert s.contact_keys()[0].size == 0


def test_ghost_double_contact_on_seam():
    """A sphere resting on the shared edge of two coplanar triangles touches
    both (no de-duplication), each carrying m g / 2 at rest (Section 3.3)."""
    R = 1e-3
    tri = W.floor_mesh(0.0, 0.0, 0.02, 0.0)  # diagonal seam along x = y
    p = P(g=(0, 0, -9.81), dt=2e-6, e_n=0.3)
    # equilibrium with two contacts each carrying half the weight
    de = (mass(2500.0, R) * 9.81 / 2 / (4.0 / 3.0 * 1e6 / (1 - 0.09) * math.sqrt(R))) ** (2 / 3)
    s = O.Sim(p, [[0.005, 0.005, R - de]], R=[R], tri=tri)
    s.step(10000)
    c = s.contacts()
    assert sorted(c["kj"].tolist()) == [-1, 0]
    for f in c["f"]:
        assert f[2] == pytest.approx(mass(2500.0, R) * 9.81 / 2, rel=1e-5)


# --------------------------------------------------------------------------
# history lifecycle (Section 3.2) and parameter validation (Table 2)
# --------------------------------------------------------------------------
def test_history_lifecycle_restart_from_zero():
    """A contact that ends loses its springs; when it forms again the springs
    start from zero (Section 2.3: initialised to zero at a new collision;
    Section 3.2: inactive contacts are destroyed)."""
    R = 1e-3
    p = P(g=(0, 0, -9.81), dt=2e-6, e_n=0.95, mu_s=5.0, mu_r=5.0, mu_t=5.0)
    s = O.Sim(p, [[0, 0, R + 2e-5]], v=[[0.05, 0, -0.1]], w=[[3.0, 0, 0]], R=[R],
              tri=W.floor_mesh(0, 0, 0.2))
    phase, carried = 0, 0.0
    for _ in range(40000):
        pre = s.state()
        s.step(1)
        c = s.contacts()
        if phase == 0 and len(c["ki"]):
            phase = 1
        elif phase == 1 and len(c["ki"]):
            carried = max(carried, np.linalg.norm(c["us"][0]))
        elif phase == 1 and not len(c["ki"]):
            phase = 2
        elif phase == 2 and len(c["ki"]):
            break
    else:
        pytest.fail("no second contact")
    x, v, w = pre["x"][0], pre["v"][0], pre["w"][0]
    fresh = O.eval_pw(p, x, v, w, R, [x[0], x[1], 0.0])
    assert carried > 10 * np.linalg.norm(fresh["us"])  # a carried spring would show
    assert np.allclose(c["us"][0], fresh["us"], rtol=0, atol=1e-12 * np.linalg.norm(fresh["us"]))
    assert np.allclose(c["ur"][0], fresh["ur"], rtol=0, atol=1e-12 * np.linalg.norm(fresh["ur"]))
    assert c["ut"][0] == pytest.approx(fresh["ut"], rel=1e-12)


def test_rigid_rotation_of_a_pair_has_no_relative_motion():
    """Two touching spheres moving as one rigid body (v = Omega x x,
    w_i = w_j = Omega) have zero sliding, rolling and twisting velocity
    (reading R1 plus the relative angular velocity w_i - w_j)."""
    rng = np.random.default_rng(12)
    for _ in range(20):
        Om = rng.normal(0, 20, 3)
        Ri, Rj = rng.uniform(0.6e-3, 1.4e-3, 2)
        nvec = rng.normal(size=3)
        nvec /= np.linalg.norm(nvec)
        xj = rng.normal(0, 1e-3, 3)
        xi = xj + nvec * (Ri + Rj) * 0.98
        o = O.eval_pp(P(), xi, np.cross(Om, xi), Om, Ri, xj, np.cross(Om, xj), Om, Rj)
        scale = np.linalg.norm(Om) * 3e-3
        assert np.linalg.norm(o["vs"]) <= 1e-13 * scale
        assert np.linalg.norm(o["vr"]) == 0.0
        assert o["vt"] == 0.0


def test_set_history_drops_stale_keys():
    R = 1e-3
    s = O.Sim(P(), [[0, 0, 0], [1.9e-3, 0, 0], [9e-3, 0, 0]], R=[R, R, R])
    s.set_history([0, 0], [1, 2], [[0, 1e-6, 0], [0, 2e-6, 0]], [[0, 0, 0], [0, 0, 0]], [0, 0])
    s.step(1)
    c = s.contacts()
    assert list(zip(c["ki"], c["kj"])) == [(0, 1)]


@pytest.mark.parametrize("bad", [dict(nu=0.6), dict(nu=-1.0), dict(e_n=1.1), dict(e_n=-0.1),
                                 dict(mu_s=-0.1), dict(mu_r=-1), dict(mu_t=-1), dict(eta=-1),
                                 dict(dt=0.0), dict(rho=0.0), dict(E=-1.0)])
def test_validation_table2_requirements(bad):
    assert not O.validate(P(**bad))
    with pytest.raises(ValueError):
        O.Sim(P(**bad), [[0, 0, 0]], R=[1e-3])


def test_validation_radius():
    with pytest.raises(ValueError):
        O.Sim(P(), [[0, 0, 0]], R=[0.0])


# --------------------------------------------------------------------------
# rotating mesh extension (reading R14)
# --------------------------------------------------------------------------
def test_rotating_mesh_vertices_and_drag_direction():
    """Vertices rotate rigidly by |Omega| t; a resting sphere on a spinning
    floor is dragged along Omega x r by the sliding damper."""
    tri = W.floor_mesh(0.0, 0.0, 0.05, 0.0)
    om = np.array([0.0, 0.0, 2.0])
    p = P(g=(0, 0, -9.81), dt=1e-6, mesh_omega=tuple(om), mesh_center=(0, 0, 0))
    R = 1e-3
    x0 = np.array([0.01, 0.0, R - delta_eq(R)])
    s = O.Sim(p, [x0], R=[R], tri=tri)
    s.step(5)
    t = s.time
    rot = Rotation.from_rotvec(om * t)
    assert np.allclose(s.mesh()[:, :3].reshape(-1, 3), rot.apply(tri.reshape(-1, 3)), atol=1e-15)
    F = s.forces()["F"][0]
    drag_dir = np.cross(om, x0)
    assert F[:2] @ drag_dir[:2] > 1e-6 * mass(2500.0, R) * 9.81 * np.linalg.norm(drag_dir)
    # a static mesh gives no tangential force beyond rounding of the normal
    s2 = O.Sim(P(g=(0, 0, -9.81), dt=1e-6), [x0], R=[R], tri=tri)
    s2.step(5)
    assert np.abs(s2.forces()["F"][0][:2]).max() < 1e-12 * mass(2500.0, R) * 9.81
