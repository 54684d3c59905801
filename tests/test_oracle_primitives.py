"""Pins of the oracle's other mesh primitives (Section 3.3, Fig. 4A, B, D):
points, line segments and rectangles, each rounded by its own radius
R_m >= 0 (a vertex acts as a sphere, an edge as a spherocylinder).

Each check rests on something other than the oracle's own formulas: dense
sampling of the element, first-order optimality of the closest point, the
triangle routine (pinned on its own) on the two halves of a rectangle,
Hertz equilibrium and impact closed forms, and the ghost-contact argument
the paper gives for rectangles.
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize_scalar
from scipy.spatial.transform import Rotation

import oracle as O
import workloads as W


def mass(rho, R):
    return 4.0 / 3.0 * math.pi * rho * R ** 3


def P(**kw):
    base = dict(rho=2500.0, E=1e6, nu=0.3, e_n=0.5, mu_s=0.5, mu_r=0.1, mu_t=0.1, eta=0.0,
                g=(0.0, 0.0, 0.0), dt=1e-6)
    base.update(kw)
    return O.make_params(**base)


def delta_eq(R, rho=2500.0, E=1e6, nu=0.3, g=9.81):
    # Hertz sphere on a rigid body of infinite curvature radius (the wall
    # reading of the effective radius): m g = 4/3 E_w sqrt(R) delta^(3/2)
    Ew = E / (1 - nu ** 2)
    return (mass(rho, R) * g / (4.0 / 3.0 * Ew * math.sqrt(R))) ** (2.0 / 3.0)


def rect_corners(rng, scale=1.0):
    """A random rectangle in 3D: corner a, orthogonal edges e1, e2."""
    a = rng.normal(size=3) * scale
    e1 = rng.normal(size=3)
    e2 = np.cross(e1, rng.normal(size=3))
    e1 *= scale * rng.uniform(0.2, 2.0) / np.linalg.norm(e1)
    e2 *= scale * rng.uniform(0.2, 2.0) / np.linalg.norm(e2)
    return np.array([a, a + e1, a + e1 + e2, a + e2])


# --------------------------------------------------------------------------
# closest points (Fig. 4A, B, D)
# --------------------------------------------------------------------------
def test_segment_closest_point_dense_sampling_and_optimality():
    rng = np.random.default_rng(11)
    t = np.linspace(0.0, 1.0, 20001)[:, None]
    for _ in range(300):
        a, b, p = rng.normal(size=(3, 3))
        c = O.closest_point_segment(p, a, b)
        pts = a + t * (b - a)
        dmin = np.linalg.norm(pts - p, axis=1).min()
        d = np.linalg.norm(p - c)
        assert d <= dmin + 1e-12
        assert d >= dmin - 1e-4 * np.linalg.norm(b - a)
        # on the segment, and first-order optimal: an interior point sees
        # p along the normal plane of the segment; an end point sees p
        # outside the segment's slab on its own side
        u = (c - a) @ (b - a) / ((b - a) @ (b - a))
        assert -1e-12 <= u <= 1 + 1e-12
        assert np.linalg.norm(c - (a + u * (b - a))) <= 1e-12
        g = (p - c) @ (b - a)
        if 1e-9 < u < 1 - 1e-9:
            assert abs(g) <= 1e-12 * np.linalg.norm(p - c) * np.linalg.norm(b - a) + 1e-14
        elif u <= 1e-9:
            assert g <= 1e-12
        else:
            assert g >= -1e-12


def test_segment_closest_point_special_cases():
    a, b = np.array([-1.0, 0, 0]), np.array([1.0, 0, 0])
    assert np.array_equal(O.closest_point_segment([0.25, 3.0, -4.0], a, b), [0.25, 0.0, 0.0])
    assert np.array_equal(O.closest_point_segment([5.0, 1.0, 0.0], a, b), b)
    assert np.array_equal(O.closest_point_segment([-5.0, 1.0, 0.0], a, b), a)
    # zero length: the segment is its vertex
    assert np.array_equal(O.closest_point_segment([3.0, 2.0, 1.0], a, a), a)


def test_rectangle_closest_point_is_the_closer_half():
    """A rectangle is the union of the triangles (a, b, c) and (a, c, d):
    its closest point is the closer of theirs (the triangle routine is
    pinned by its own tests), and it is unique (convex set)."""
    rng = np.random.default_rng(12)
    for _ in range(2000):
        a, b, c, d = rect_corners(rng)
        p = rng.normal(size=3) * 2
        got = O.closest_point_rectangle(p, a, b, c, d)
        h1 = O.closest_point_triangle(p, a, b, c)
        h2 = O.closest_point_triangle(p, a, c, d)
        ref = h1 if np.linalg.norm(p - h1) <= np.linalg.norm(p - h2) else h2
        assert np.linalg.norm(p - got) == pytest.approx(np.linalg.norm(p - ref), rel=1e-9,
                                                        abs=1e-12)
        assert np.allclose(got, ref, atol=1e-9)


def test_rectangle_closest_point_dense_sampling():
    rng = np.random.default_rng(13)
    k = 201
    uu, vv = np.meshgrid(np.linspace(0, 1, k), np.linspace(0, 1, k))
    st = np.stack([uu.ravel(), vv.ravel()], 1)
    for _ in range(50):
        a, b, c, d = rect_corners(rng)
        p = rng.normal(size=3)
        pts = a + st[:, :1] * (b - a) + st[:, 1:] * (d - a)
        dmin = np.linalg.norm(pts - p, axis=1).min()
        got = np.linalg.norm(p - O.closest_point_rectangle(p, a, b, c, d))
        assert got <= dmin + 1e-12
        assert got >= dmin - 0.01 * (np.linalg.norm(b - a) + np.linalg.norm(d - a))


def test_rectangle_closest_point_special_cases():
    a, b, c, d = np.array([[0.0, 0, 0], [2.0, 0, 0], [2.0, 1.0, 0], [0.0, 1.0, 0]])
    # above the interior: the orthogonal projection
    assert np.array_equal(O.closest_point_rectangle([0.5, 0.25, 7.0], a, b, c, d),
                          [0.5, 0.25, 0.0])
    # beyond a corner: that corner; beside an edge: the foot on that edge
    assert np.array_equal(O.closest_point_rectangle([3.0, 2.0, -1.0], a, b, c, d), c)
    assert np.array_equal(O.closest_point_rectangle([1.5, -4.0, 1.0], a, b, c, d),
                          [1.5, 0.0, 0.0])


def test_element_dispatch():
    rng = np.random.default_rng(14)
    for _ in range(200):
        v = rng.normal(size=(3, 3))
        p = rng.normal(size=3)
        assert np.array_equal(O.closest_point_element(p, v[:1]), v[0])
        assert np.array_equal(O.closest_point_element(p, v[:2]), O.closest_point_segment(p, *v[:2]))
        assert np.array_equal(O.closest_point_element(p, v), O.closest_point_triangle(p, *v))
        r = rect_corners(rng)
        assert np.array_equal(O.closest_point_element(p, r), O.closest_point_rectangle(p, *r))


# --------------------------------------------------------------------------
# contact sets with rounded elements (Section 3.3)
# --------------------------------------------------------------------------
def dist_segment_independent(p, a, b):
    """Distance to a segment by bounded scalar minimisation."""
    f = lambda t: float(np.sum((a + t * (b - a) - p) ** 2))
    r = minimize_scalar(f, bounds=(0.0, 1.0), method="bounded", options={"xatol": 1e-13})
    return math.sqrt(min(r.fun, f(0.0), f(1.0)))


def dist_element_independent(p, e):
    e = np.asarray(e).reshape(-1, 3)
    if len(e) == 1:
        return float(np.linalg.norm(p - e[0]))
    if len(e) == 2:
        return dist_segment_independent(p, e[0], e[1])
    if len(e) == 3:
        return float(np.linalg.norm(p - O.closest_point_triangle(p, *e)))
    return min(float(np.linalg.norm(p - O.closest_point_triangle(p, e[0], e[1], e[2]))),
               float(np.linalg.norm(p - O.closest_point_triangle(p, e[0], e[2], e[3]))))


@pytest.mark.parametrize("seed", [0, 1])
def test_contact_set_with_rounded_primitives(seed):
    """Key set = brute force over every (particle, element) pair with the
    rounded-element predicate R_i + R_m - dist >= 0, with dist computed by
    independent routes (bounded minimisation for segments, the two
    triangles for rectangles)."""
    els, rm = W.primitive_mesh(20e-3, seed)
    w = W.random_cluster(300, 10 + seed, box=20e-3, overlap=0.2, r_lo=0.5e-3, r_hi=1.5e-3)
    x, R = w["x"], w["R"]
    s = O.Sim(P(), x, R=R, elements=els, rmesh=rm)
    ki, kj = s.contact_keys()
    got = {(i, j) for i, j in zip(ki.tolist(), kj.tolist()) if j <= 0}
    ref = set()
    margin_hits = 0
    for i in range(len(R)):
        for m, e in enumerate(els):
            gap = (R[i] + rm[m]) - dist_element_independent(x[i], e)
            if abs(gap) < 1e-9:
                margin_hits += 1
            if gap >= 0:
                ref.add((i, -m))
    assert margin_hits == 0
    assert len(ref) > 40
    kinds = {len(els[-k]) for _, k in ref}
    assert kinds == {1, 2, 3, 4}
    assert got == ref


# --------------------------------------------------------------------------
# dynamics on rounded primitives
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["point", "segment", "rectangle"])
def test_rest_on_rounded_primitive(kind):
    """A sphere resting on top of a point, a horizontal segment (a rounded
    rail) or a rectangle of radius R_m sinks to the Hertz equilibrium
    overlap below R_i + R_m above the element and carries its weight on one
    contact whose force is vertical."""
    R, Rm = 1e-3, 2e-3
    el = {"point": [[0.0, 0.0, 0.0]],
          "segment": [[-0.02, 0.0, 0.0], [0.02, 0.0, 0.0]],
          "rectangle": [[-0.02, -0.01, 0.0], [0.02, -0.01, 0.0], [0.02, 0.01, 0.0],
                        [-0.02, 0.01, 0.0]]}[kind]
    p = P(g=(0, 0, -9.81), dt=2e-6, e_n=0.3)
    x0 = [[0.0015 if kind != "point" else 0.0, 0.0, R + Rm - 0.9 * delta_eq(R)]]
    s = O.Sim(p, x0, R=[R], elements=[el], rmesh=[Rm])
    s.step(20000)
    st, c = s.state(), s.contacts()
    assert c["kj"].tolist() == [0]
    assert (R + Rm) - st["x"][0, 2] == pytest.approx(delta_eq(R), rel=1e-6)
    assert c["f"][0][2] == pytest.approx(mass(2500.0, R) * 9.81, rel=1e-6)
    assert np.abs(c["f"][0][:2]).max() <= 1e-9 * c["f"][0][2]
    if kind == "point":
        assert np.abs(st["x"][0, :2]).max() < 1e-12


def test_rectangle_removes_the_seam_ghost():
    """The reason rectangles exist (Section 3.3): a sphere on the diagonal
    seam of a floor made of two triangles touches both and carries m g / 2
    on each, while the same floor as one rectangle gives one contact with
    the whole weight at the Hertz equilibrium overlap."""
    R = 1e-3
    p = P(g=(0, 0, -9.81), dt=2e-6, e_n=0.3)
    rect = [[0.0, 0.0, 0.0], [0.02, 0.0, 0.0], [0.02, 0.02, 0.0], [0.0, 0.02, 0.0]]
    s = O.Sim(p, [[0.005, 0.005, R - delta_eq(R)]], R=[R], elements=[rect])
    s.step(10000)
    c = s.contacts()
    assert c["kj"].tolist() == [0]
    assert c["f"][0][2] == pytest.approx(mass(2500.0, R) * 9.81, rel=1e-5)
    assert R - s.state()["x"][0, 2] == pytest.approx(delta_eq(R), rel=1e-5)
    # the same floor as two triangles (seam along x = y)
    s2 = O.Sim(p, [[0.005, 0.005, R - delta_eq(R)]], R=[R], tri=W.floor_mesh(0.0, 0.0, 0.02, 0.0))
    s2.step(10000)
    assert sorted(s2.contacts()["kj"].tolist()) == [-1, 0]


@pytest.mark.parametrize("Rm", [0.0, 1.5e-3])
def test_head_on_impact_on_a_rounded_vertex(Rm):
    """A sphere shot at a point element: contact starts when the centre is
    R_i + R_m from the vertex, and leaves with e_n times its speed (Hertz
    contact with the damping of Eq. cn restores e_n whatever the curvature,
    Section 2.2)."""
    R, v0, dt = 1e-3, 0.5, 2e-7
    p = P(e_n=0.6, dt=dt)
    gap0 = 20 * v0 * dt
    s = O.Sim(p, [[R + Rm + gap0, 0.0, 0.0]], v=[[-v0, 0.0, 0.0]], R=[R],
              elements=[[[0.0, 0.0, 0.0]]], rmesh=[Rm])
    first, started = None, False
    for k in range(200000):
        x_before = s.state()["x"][0, 0]
        s.step(1)
        if O.lib().orc_num_contacts(s._h):
            if first is None:
                first = x_before
            started = True
        elif started:
            break
    # the first step in contact started inside R_i + R_m, the one before not
    assert first <= R + Rm < first + v0 * dt * 1.0000001
    assert s.state()["v"][0, 0] == pytest.approx(0.6 * v0, abs=2e-3 * v0)
    assert np.abs(s.state()["v"][0, 1:]).max() == 0.0


def test_rolling_along_a_rounded_rail_keeps_its_line():
    """A sphere rolling along a horizontal rounded segment, started on top of
    it with the rolling velocity, stays in the vertical plane of the rail:
    the contact normal and every force lie in that plane."""
    R, Rm = 1e-3, 0.5e-3
    p = P(g=(0, 0, -9.81), dt=2e-6, e_n=0.3, mu_r=0.0, mu_t=0.0)
    v = 0.05
    s = O.Sim(p, [[-0.01, 0.0, R + Rm - delta_eq(R)]], v=[[v, 0.0, 0.0]],
              w=[[0.0, v / (R - delta_eq(R) / 2), 0.0]], R=[R],
              elements=[[[-0.03, 0.0, 0.0], [0.03, 0.0, 0.0]]], rmesh=[Rm])
    s.step(2000)
    st = s.state()
    assert abs(st["x"][0, 1]) < 1e-15
    assert st["x"][0, 0] > -0.01 + 0.9 * v * 2000 * 2e-6
    assert s.contacts()["kj"].tolist() == [0]


# --------------------------------------------------------------------------
# validation and rotation
# --------------------------------------------------------------------------
def test_validation_of_elements():
    s = O.Sim(P(), np.zeros((1, 3)) + 1.0, R=[1e-3])
    good = [[0.0, 0, 0], [1.0, 0, 0], [1.0, 2.0, 0], [0.0, 2.0, 0]]
    s.set_mesh_elements([good])
    for bad in ([[0.0, 0, 0], [1.0, 0, 0], [1.3, 2.0, 0], [0.3, 2.0, 0]],   # parallelogram
                [[0.0, 0, 0], [1.0, 0, 0], [1.0, 2.0, 0.1], [0.0, 2.0, 0]],  # warped
                [[0.0, 0, 0], [1.0, 0, 0], [1.0, 2.0, 0], [0.0, 2.0, 0], [0, 0, 1.0]],
                [[0.0, 0, np.nan]]):
        with pytest.raises(ValueError):
            s.set_mesh_elements([bad])
    with pytest.raises(ValueError):
        s.set_mesh_elements([good], rmesh=[-1e-3])
    # a rectangle within the tolerance (printed to 8 digits) is accepted
    s.set_mesh_elements([np.round(Rotation.from_rotvec([0.3, 0.2, 0.1]).apply(good), 8)])


def test_rotating_elements_move_rigidly():
    """Every vertex of every kind of element follows the rigid rotation
    about the mesh centre (the rotating-mesh extension), checked with
    scipy's rotations."""
    els, rm = W.primitive_mesh(20e-3, 3)
    om = np.array([0.5, -1.0, 2.0])
    ctr = np.array([0.01, 0.01, 0.01])
    s = O.Sim(P(mesh_omega=tuple(om), mesh_center=tuple(ctr)), np.array([[0.5, 0.5, 0.5]]),
              R=[1e-3], elements=els, rmesh=rm)
    s.step(7)
    rot = Rotation.from_rotvec(om * s.time)
    got = s.mesh()
    for m, e in enumerate(els):
        e = np.asarray(e).reshape(-1, 3)
        assert np.allclose(got[m, :len(e)], rot.apply(e - ctr) + ctr, atol=1e-15)
