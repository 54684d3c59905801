"""Pins of the oracle's rolling and twisting kinematics (Section 2.2): the
rolling velocity v_r = (1/r_i + 1/r_j)^-1 w x n, the twisting velocity
v_t = R* w.n, and the levers of the rolling torque R* n x f_r and of the
twisting torque f_t R* n.

Kinetic friction alone cannot pin these: there |f_m| = mu_m |f_n| whatever
v_r, v_t are, and on a wall R* = R_i differs from r_i only by delta/2.  The
pins below therefore use
  - static springs, whose stiffness times the kinematic factor sets a
    vibration frequency (a twisting oscillator, and the two coupled rocking
    modes of a sphere on a floor), on a soft material so that delta/R is a
    few per cent and the levers R* and r_i are told apart;
  - pair collisions, where R* = R/2 for equal spheres is far from r_i ~ R
    and the spin change follows from the normal impulse.
Every expected value is derived here from rigid-body mechanics and the
constitutive laws of Section 2.2, not taken from the oracle.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W

RHO, R = 2500.0, 1e-3


def mass(R=R):
    return 4.0 / 3.0 * math.pi * RHO * R ** 3


def inertia(R=R):
    return 0.4 * mass(R) * R ** 2


def wall_moduli(E, nu):
    """Effective moduli of a sphere against a rigid wall (Section 2.2 with
    the second body's radius, mass and stiffness taken to infinity)."""
    return E / (1.0 - nu ** 2), E / (2.0 * (1.0 + nu) * (2.0 - nu))


def delta_eq(E, nu, g=9.81):
    """Hertz overlap of a sphere resting on a rigid floor:
    m g = 4/3 E* sqrt(R) delta^(3/2)."""
    Ew, _ = wall_moduli(E, nu)
    return (mass() * g / (4.0 / 3.0 * Ew * math.sqrt(R))) ** (2.0 / 3.0)


def on_floor(E, nu, w0, v0=(0.0, 0.0, 0.0), dt=5e-6, **mu):
    """One sphere resting at its Hertz overlap on a flat two-triangle floor,
    e_n = 1 (no damping, so the normal force stays exactly m g)."""
    p = O.make_params(rho=RHO, E=E, nu=nu, e_n=1.0, eta=0.0, g=(0.0, 0.0, -9.81), dt=dt, **mu)
    x = np.array([[0.013, 0.007, R - delta_eq(E, nu)]])
    return O.Sim(p, x, v=[v0], w=[w0], R=[R], tri=W.floor_mesh(0.0, 0.0, 0.2, 0.0))


def record(sim, steps, pick):
    out = np.empty(steps)
    for k in range(steps):
        sim.step(1)
        out[k] = pick(sim.state())
    return out


def period_from_zero_crossings(y, dt):
    """Oscillation period of a sampled signal from its zero crossings
    (linear interpolation between samples)."""
    t = dt * np.arange(1, len(y) + 1)
    s = np.sign(y)
    k = np.nonzero(s[:-1] * s[1:] < 0)[0]
    tc = t[k] - y[k] * (t[k + 1] - t[k]) / (y[k + 1] - y[k])
    assert len(tc) >= 4, "fewer than two periods recorded"
    # half periods between successive crossings; a least-squares line through
    # the crossing times gives the mean half period
    hp = np.polyfit(np.arange(len(tc)), tc, 1)[0]
    return 2.0 * hp


# soft material: delta/R ~ 3.7 % on a 1 mm sphere under gravity
E_SOFT, NU = 1e4, 0.3


def test_twisting_oscillation_period():
    """Static twist on a floor is a torsional oscillator.  The twist spring
    grows as du_t/dt = v_t = R* w_z and acts with torque f_t R* about n
    (f_t = -k_t u_t, k_t = k_s = 8 G* sqrt(R* delta), c_t = 0 at e_n = 1), so
    I d2u/dt2 = -k_t R*^2 u: period 2 pi sqrt(I / (k_t R*^2)), with
    R* = R against a wall.  A wrong v_t changes the period by its factor;
    the lever r_i = R - delta/2 instead of R* would change it by 0.9 %."""
    d = delta_eq(E_SOFT, NU)
    _, Gw = wall_moduli(E_SOFT, NU)
    kt = 8.0 * Gw * math.sqrt(R * d)
    T = 2.0 * math.pi * math.sqrt(inertia() / (kt * R * R))
    dt = 5e-6
    # amplitude: the twist force k_t R w0 / omega stays below mu_t m g
    w0 = 2.0
    assert kt * R * w0 * T / (2 * math.pi) < 0.1 * mass() * 9.81
    s = on_floor(E_SOFT, NU, (0.0, 0.0, w0), dt=dt, mu_s=10.0, mu_r=10.0, mu_t=0.5)
    wz = record(s, int(3.2 * T / dt), lambda st: st["w"][0, 2])
    c = s.contacts()
    assert len(c["ki"]) == 1 and c["kj"][0] <= 0
    assert abs(c["ut"][0]) > 0
    # the spring and the spin are advanced from the same start-of-step
    # values (Section 2.3), an explicit step of the oscillator that grows its
    # amplitude by sqrt(1 + (omega dt)^2) per step
    steps = len(wz)
    grow = (1.0 + (2.0 * math.pi * dt / T) ** 2) ** (0.5 * steps)
    assert np.abs(wz[-int(T / dt):]).max() == pytest.approx(w0 * grow, rel=1e-2)
    assert period_from_zero_crossings(wz, dt) == pytest.approx(T, rel=1e-4)


def rocking_modes(E, nu):
    """Small rocking of a sphere on a floor with static sliding and rolling
    springs (Section 2.2, e_n = 1 so c_s = c_r = 0).  With the centre moved
    by x and the sphere turned by theta about y (n = +z):
      sliding:  v_s = dx/dt - r_i dtheta/dt  ->  u_s = x - r_i theta,
                f_s = -k_s u_s, torque r_i f_s x n gives +r_i k_s u_s about y;
      rolling:  v_r = r_i (w x n) = r_i dtheta/dt (the wall's r_j is
                infinite) -> u_r = r_i theta, f_r = -k_r u_r, torque
                R* n x f_r gives -R* k_r r_i theta about y;
      m d2x/dt2 = -k_s (x - r_i theta),
      I d2theta/dt2 = r_i k_s (x - r_i theta) - R* k_r r_i theta,
    with k_s = 8 G* a, k_r = k_n = 4/3 E* a, a = sqrt(R* delta), R* = R.
    Returns the two angular frequencies (ascending) and the mode shapes
    (columns: dx/dt, dtheta/dt)."""
    d = delta_eq(E, nu)
    Ew, Gw = wall_moduli(E, nu)
    a = math.sqrt(R * d)
    ks, kr = 8.0 * Gw * a, 4.0 / 3.0 * Ew * a
    ri = R - d / 2.0
    K = np.array([[ks, -ks * ri], [-ks * ri, ks * ri * ri + R * kr * ri]])
    M = np.diag([mass(), inertia()])
    # symmetric form M^-1/2 K M^-1/2
    Mh = np.diag(1.0 / np.sqrt(np.diag(M)))
    lam, V = np.linalg.eigh(Mh @ K @ Mh)
    return np.sqrt(lam), Mh @ V


@pytest.mark.parametrize("mode", [0, 1])
def test_rocking_mode_frequencies(mode):
    """Each rocking mode, excited alone through its mode shape, oscillates
    at its own frequency.  The rolling spring's rate r_i w x n enters the
    stiffness of theta: doubling v_r moves both frequencies by tens of per
    cent, the lever r_i instead of R* in the rolling torque by ~0.4 %."""
    om, V = rocking_modes(E_SOFT, NU)
    T = 2.0 * math.pi / om[mode]
    dt = 5e-6
    amp = 1e-4 / abs(V[0, mode])  # horizontal speed 0.1 mm/s
    xdot, thdot = amp * V[0, mode], amp * V[1, mode]
    s = on_floor(E_SOFT, NU, (0.0, thdot, 0.0), v0=(xdot, 0.0, 0.0), dt=dt, mu_s=1e3, mu_r=1e3,
                 mu_t=1e3)
    vx = record(s, int(4.2 * T / dt), lambda st: st["v"][0, 0])
    assert period_from_zero_crossings(vx, dt) == pytest.approx(T, rel=1e-4)
    # the other mode stays unexcited: v_x keeps its amplitude (up to the slow
    # growth of the explicit spring update)
    assert np.abs(vx[: int(T / dt)]).max() == pytest.approx(abs(xdot), rel=5e-2)


def collide_spinning_pair(w1, w2, v0=0.1, **mu):
    """Two equal spheres on the x axis closing at 2 v0, elastic (e_n = 1),
    no gravity; returns (normal impulse on sphere 0 from its momentum change,
    change of sphere 0's spin, change of sphere 1's spin)."""
    p = O.make_params(rho=RHO, E=1e6, nu=0.3, e_n=1.0, eta=0.0, g=(0.0, 0.0, 0.0), dt=2e-7,
                      **mu)
    x = np.array([[-R - 2e-6, 0.0, 0.0], [R + 2e-6, 0.0, 0.0]])
    s = O.Sim(p, x, v=[[v0, 0, 0], [-v0, 0, 0]], w=[w1, w2], R=[R, R])
    st0 = s.state()
    touched = False
    for _ in range(400):
        s.step(50)
        if len(s.contacts()["ki"]):
            touched = True
        elif touched:
            break
    assert touched and len(s.contacts()["ki"]) == 0, "the collision did not end"
    st = s.state()
    J = mass() * abs(st["v"][0, 0] - st0["v"][0, 0])
    assert J == pytest.approx(2.0 * mass() * v0, rel=1e-2)  # elastic: J = 2 m* (2 v0)
    return J, st["w"][0] - st0["w"][0], st["w"][1] - st0["w"][1]


def test_pair_twist_lever_counter_spin():
    """Spheres spinning in opposite senses about the line of centres slip in
    twist throughout: each takes the kinetic twisting torque mu_t |f_n| R*
    about n, so its spin changes by mu_t R* J / I towards the other's, with
    R* = R/2 for equal spheres (the lever r_i ~ R would double it)."""
    Om, mu_t = 2000.0, 0.2
    J, dw0, dw1 = collide_spinning_pair((Om, 0, 0), (-Om, 0, 0), mu_s=0.5, mu_r=0.1, mu_t=mu_t)
    expect = mu_t * (R / 2.0) * J / inertia()
    assert dw0[0] == pytest.approx(-expect, rel=3e-2)
    assert dw1[0] == pytest.approx(+expect, rel=3e-2)
    assert np.abs(dw0[1:]).max() <= 1e-9 * expect


def test_pair_rolling_lever_meshing_spin():
    """Spins perpendicular to the line of centres, equal and opposite
    ("meshing gears"): the contact points move together (no sliding, R1) but
    the relative spin 2 Om gives a rolling velocity, kinetic throughout, so
    each sphere takes the torque R* n x f_r of magnitude mu_r |f_n| R* and
    its spin drops by mu_r R* J / I, R* = R/2 (the lever r_i would double
    it)."""
    Om, mu_r = 2000.0, 0.1
    J, dw0, dw1 = collide_spinning_pair((0, Om, 0), (0, -Om, 0), mu_s=0.5, mu_r=mu_r, mu_t=0.1)
    expect = mu_r * (R / 2.0) * J / inertia()
    assert dw0[1] == pytest.approx(-expect, rel=3e-2)
    assert dw1[1] == pytest.approx(+expect, rel=3e-2)
    assert abs(dw0[0]) + abs(dw0[2]) <= 1e-9 * expect
