"""Seeded synthetic inputs for the DEM hot path (both the GPU solver's tests
and the CPU oracle read these; neither side's arithmetic lives here).

Every generator draws from NumPy's PCG64 with a fixed seed, except sphere
placement by random sequential addition, which runs in ``pack.c`` with its own
SplitMix64 stream seeded from the same seed.  A workload is a dict::

    {"name", "params": {rho, E, nu, e_n, mu_s, mu_r, mu_t, eta, g, dt,
                        mesh_omega, mesh_center},
     "x", "v", "w" (n,3), "q" (n,4) scalar first, "R" (n,),
     "tri" (m,3,3), "rmesh" (m,), "steps", "R_max"}

Units are SI.  Parameters not stated by a configuration take Table 2's
values (E = 1 MPa, nu = 0.3, eta = 0, g = (0,0,-9.81)) and the first
configuration's contact parameters (e_n = 0.7, mu = 0.5/0.1/0.1).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_PACK_SRC = os.path.join(_HERE, "pack.c")
_PACK_LIB = os.path.join(_HERE, "libpack.so")

MM = 1e-3


def build(force: bool = True) -> str:
    if force or not os.path.exists(_PACK_LIB):
        tmp = _PACK_LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _PACK_SRC, "-lm"],
                       check=True)
        os.replace(tmp, _PACK_LIB)
    return _PACK_LIB


_pack = None


def _packlib():
    global _pack
    if _pack is None:
        if not os.path.exists(_PACK_LIB):
            build()
        L = C.CDLL(_PACK_LIB)
        D = C.POINTER(C.c_double)
        L.pack_rsa.restype = C.c_int64
        L.pack_rsa.argtypes = [C.c_int64, D, D, D, C.c_int32, D, C.c_uint64, C.c_int64, D]
        L.pack_deposit.restype = C.c_int64
        L.pack_deposit.argtypes = [C.c_int64, D, C.c_double, C.c_double, C.c_uint64, D,
                                   C.POINTER(C.c_int64)]
        _pack = L
    return _pack


def rsa_place(R, lo, hi, seed, shape=0, cyl=(0.0, 0.0, 0.0, 0.0), max_attempts=100000):
    """Random sequential addition of spheres with radii R, largest first (a
    late large sphere would otherwise find no room); returns centres in the
    order of R."""
    R_in = np.asarray(R, dtype=np.float64)
    order = np.argsort(-R_in, kind="stable")
    R = np.ascontiguousarray(R_in[order])
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    cyl = np.ascontiguousarray(cyl, dtype=np.float64)
    x = np.zeros((len(R), 3))
    D = C.POINTER(C.c_double)
    got = _packlib().pack_rsa(len(R), R.ctypes.data_as(D), lo.ctypes.data_as(D),
                              hi.ctypes.data_as(D), int(shape), cyl.ctypes.data_as(D),
                              C.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), int(max_attempts),
                              x.ctypes.data_as(D))
    if got != len(R):
        raise RuntimeError(f"random sequential addition placed {got} of {len(R)} spheres")
    out = np.empty_like(x)
    out[order] = x
    return out


def deposit(R, Lx, Ly, seed):
    """Sequential deposition with rolling (Visscher and Bolsterli, 1972) of
    spheres with radii R, in the given order, onto the floor z = 0 of the
    cell [0, Lx) x [0, Ly), periodic in x and y: each sphere falls from above
    the pile at a random (x, y) and rolls downhill over the spheres below
    until it rests on the floor or on supports that carry its weight.
    Returns the centres (x and y in [0, L)) and the number of spheres whose
    rolling hit the step limit (left where they were)."""
    R = np.ascontiguousarray(R, dtype=np.float64)
    x = np.zeros((len(R), 3))
    stuck = C.c_int64(0)
    D = C.POINTER(C.c_double)
    got = _packlib().pack_deposit(len(R), R.ctypes.data_as(D), float(Lx), float(Ly),
                                  C.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), x.ctypes.data_as(D),
                                  C.byref(stuck))
    if got != len(R):
        raise RuntimeError(f"deposition failed ({got}): radii must be positive, the cell at "
                           f"least 6 R_max wide, and the radii not so unequal that a "
                           f"neighbour query overflows")
    return x, int(stuck.value)


# ---------------------------------------------------------------------------
# parameters
# ---------------------------------------------------------------------------
def default_params(**kw) -> dict:
    p = dict(rho=2500.0, E=1e6, nu=0.3, e_n=0.7, mu_s=0.5, mu_r=0.1, mu_t=0.1, eta=0.0,
             g=(0.0, 0.0, -9.81), dt=1e-6, mesh_omega=(0.0, 0.0, 0.0),
             mesh_center=(0.0, 0.0, 0.0))
    p.update(kw)
    return p


def dt_eq(R_min, rho, E, nu):
    """Eq. dt time step (needed where a configuration gives no step)."""
    return R_min * math.sqrt(rho * (1.0 - nu * nu) / E)


# ---------------------------------------------------------------------------
# geometry
# ---------------------------------------------------------------------------
def shoemake_quaternions(rng, n):
    """Uniformly random unit quaternions (Shoemake 1992), scalar first."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    q = np.stack([a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2),
                  b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3)], axis=1)
    return np.ascontiguousarray(q)


def cube_mesh(lo, hi):
    """12 triangles: each face of the box split along its min->max diagonal."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    tris = []
    for ax in range(3):
        u, v = [a for a in range(3) if a != ax]
        for side in (lo[ax], hi[ax]):
            def P(a, b):
                p = np.zeros(3)
                p[ax] = side
                p[u] = a
                p[v] = b
                return p
            p00, p11 = P(lo[u], lo[v]), P(hi[u], hi[v])
            p10, p01 = P(hi[u], lo[v]), P(lo[u], hi[v])
            tris.append([p00, p10, p11])
            tris.append([p00, p11, p01])
    return np.ascontiguousarray(np.array(tris))


def floor_mesh(cx, cy, half, z=0.0):
    """Square floor at height z from two triangles."""
    a = np.array([cx - half, cy - half, z])
    b = np.array([cx + half, cy - half, z])
    c = np.array([cx + half, cy + half, z])
    d = np.array([cx - half, cy + half, z])
    return np.ascontiguousarray(np.array([[a, b, c], [a, c, d]]))


def primitive_mesh(box, seed):
    """A container of side `box` built from every kind of mesh element
    (Section 3.3, Fig. 4A-E), each with its own radius R_m:
      - floor z = 0: four rectangles (R_m = 0);
      - walls x = 0 and x = box: one rectangle each; walls y = 0 and
        y = box: two triangles each (R_m = 0);
      - a tilted rounded rectangle (R_m = 1 mm) and two tilted rounded
        triangles (R_m = 0.8 mm) inside;
      - six rounded segments (rails, R_m ~ U[0.3, 1.5] mm) and eight rounded
        points (R_m ~ U[0.5, 2] mm) at random inside.
    Returns (elements, rmesh): a list of 1..4-vertex arrays (rectangle
    corners in cyclic order) and their radii."""
    rng = np.random.Generator(np.random.PCG64(seed + 9000))
    L = float(box)
    h = L / 2
    els, rm = [], []

    def add(v, r):
        els.append(np.asarray(v, float).reshape(-1, 3))
        rm.append(float(r))

    for x0 in (0.0, h):
        for y0 in (0.0, h):
            add([[x0, y0, 0], [x0 + h, y0, 0], [x0 + h, y0 + h, 0], [x0, y0 + h, 0]], 0.0)
    for xw in (0.0, L):
        add([[xw, 0, 0], [xw, L, 0], [xw, L, L], [xw, 0, L]], 0.0)
    for yw in (0.0, L):
        a, b, c, d = [0, yw, 0], [L, yw, 0], [L, yw, L], [0, yw, L]
        add([a, b, c], 0.0)
        add([a, c, d], 0.0)
    # tilted rounded rectangle: corner, two orthogonal edges
    c0 = np.array([0.3, 0.25, 0.45]) * L
    e1 = np.array([0.4, 0.0, 0.1]) * L
    e2 = np.cross(e1, [0.1, 1.0, 0.2])
    e2 *= 0.3 * L / np.linalg.norm(e2)
    add([c0, c0 + e1, c0 + e1 + e2, c0 + e2], 1.0 * MM)
    for k in range(2):
        t0 = rng.uniform(0.15, 0.85, 3) * L
        add([t0, t0 + rng.normal(0, 0.2, 3) * L, t0 + rng.normal(0, 0.2, 3) * L], 0.8 * MM)
    for k in range(6):
        s0 = rng.uniform(0.1, 0.9, 3) * L
        add([s0, np.clip(s0 + rng.normal(0, 0.3, 3) * L, 0.05 * L, 0.95 * L)],
            rng.uniform(0.3, 1.5) * MM)
    for k in range(8):
        add([rng.uniform(0.1, 0.9, 3) * L], rng.uniform(0.5, 2.0) * MM)
    return els, np.array(rm)


def hopper_elements():
    """A hopper in the spirit of the default scene of Section 4 (a container
    with a narrowing throat and a spherical and a cylindrical obstacle),
    built from every kind of element, with the radii of Table 2's R_mesh list
    {2, 20, 10} mm:
      - floor z = 0, |x|, |y| <= 0.15: one rectangle (R_m = 0);
      - four side walls up to z = 0.12: rectangles (R_m = 0);
      - a square funnel from half width 0.04 at z = 0.12 to 0.16 at
        z = 0.28: eight triangles (R_m = 2 mm);
      - a spherical obstacle below the throat: a point at z = 0.07
        (R_m = 20 mm), and a cylindrical one: a segment along y at
        x = 0.07, z = 0.04 (R_m = 10 mm).
    Particles spawn in the box (-0.1, -0.1, 0.3) .. (0.1, 0.1, 0.4) above it.
    Returns (elements, rmesh)."""
    els, rm = [], []
    h = 0.15
    els.append([[-h, -h, 0.0], [h, -h, 0.0], [h, h, 0.0], [-h, h, 0.0]])
    rm.append(0.0)
    for a, b in (((-h, -h), (h, -h)), ((h, -h), (h, h)), ((h, h), (-h, h)), ((-h, h), (-h, -h))):
        els.append([[a[0], a[1], 0.0], [b[0], b[1], 0.0], [b[0], b[1], 0.12], [a[0], a[1], 0.12]])
        rm.append(0.0)
    lo, hi = 0.04, 0.16
    ring = lambda s, z: [[-s, -s, z], [s, -s, z], [s, s, z], [-s, s, z]]
    r0, r1 = ring(lo, 0.12), ring(hi, 0.28)
    for k in range(4):
        a0, b0, a1, b1 = r0[k], r0[(k + 1) % 4], r1[k], r1[(k + 1) % 4]
        els.append([a0, b0, b1])
        els.append([a0, b1, a1])
        rm += [0.002, 0.002]
    els.append([[0.0, 0.0, 0.07]])
    rm.append(0.02)
    els.append([[0.07, -0.1, 0.04], [0.07, 0.1, 0.04]])
    rm.append(0.01)
    return [np.asarray(e, float) for e in els], np.array(rm)


def hopper_spawn(n_max=1000, n_spawn=100, seed=2507):
    """Spawn settings of Table 2's defaults: box (-0.1, -0.1, 0.3) ..
    (0.1, 0.1, 0.4), R in [2, 10] mm, v0 = (0, 0, -1) m/s, w0 = 0."""
    return dict(smin=(-0.1, -0.1, 0.3), smax=(0.1, 0.1, 0.4), Rmin=0.002, Rmax=0.01,
                v0=(0.0, 0.0, -1.0), w0=(0.0, 0.0, 0.0), n_spawn=n_spawn, n_max=n_max,
                seed=seed)


def hopper_params():
    """Table 2 defaults: rho 1000, E 1e6, nu 0.3, e_n 0.5, mu_s 0.3,
    mu_r 0.3, mu_t 2 mu_s / 3, eta 0, g = (0, 0, -9.81), dt by Eq. dt for
    R_min = 2 mm."""
    return default_params(rho=1000.0, E=1e6, nu=0.3, e_n=0.5, mu_s=0.3, mu_r=0.3, mu_t=0.2,
                          eta=0.0, g=(0.0, 0.0, -9.81), dt=dt_eq(0.002, 1000.0, 1e6, 0.3))


def vibrated_box(n=400, seed=61, box=16 * MM):
    """The agitated bath of the segregation example of Section 4 in a box:
    spheres R ~ U[0.8, 1.2] mm at random in a cube of side `box`, walls of
    two triangles each (fixed, motion group 0), and a floor rectangle
    vibrated vertically (group 1) with amplitude A = R_min and frequency f
    such that A (2 pi f)^2 = 3 g, phase pi/2 (at rest at t = 0)."""
    w = random_cluster(n, seed, box=box, overlap=0.1, vel=0.02, spin=5.0)
    lo, hi = -0.3 * MM, box + 0.3 * MM
    tri = cube_mesh([lo] * 3, [hi] * 3)
    walls = [t for t in tri if not np.allclose(np.asarray(t)[:, 2], lo)]
    els = [np.asarray(t, float) for t in walls]
    els.append(np.array([[lo, lo, lo], [hi, lo, lo], [hi, hi, lo], [lo, hi, lo]]))
    A = 0.8 * MM
    f = math.sqrt(3.0 * 9.81 / A) / (2.0 * math.pi)
    w["tri"] = np.zeros((0, 3, 3))
    w["elements"], w["rmesh"] = els, np.zeros(len(els))
    w["motion"] = [dict(), dict(amp=(0.0, 0.0, A), freq=f, phase=math.pi / 2)]
    w["motion_groups"] = np.array([0] * (len(els) - 1) + [1], np.int32)
    w["params"].update(g=(0.0, 0.0, -9.81), dt=2e-6)
    return w


def drum_mesh(radius, length, nseg=128, nring=31):
    """Closed drum around the y axis: nseg x nring x 2 shell triangles plus
    two end-cap fans of nseg triangles (8,192 for the defaults)."""
    th = np.linspace(0, 2 * np.pi, nseg + 1)[:-1]
    ys = np.linspace(-length / 2, length / 2, nring + 1)
    ring = np.stack([radius * np.cos(th), np.zeros(nseg), radius * np.sin(th)], axis=1)
    tris = []
    for r in range(nring):
        for s in range(nseg):
            s2 = (s + 1) % nseg
            p00 = ring[s] + [0, ys[r], 0]
            p10 = ring[s2] + [0, ys[r], 0]
            p01 = ring[s] + [0, ys[r + 1], 0]
            p11 = ring[s2] + [0, ys[r + 1], 0]
            tris.append([p00, p10, p11])
            tris.append([p00, p11, p01])
    for y in (ys[0], ys[-1]):
        ctr = np.array([0.0, y, 0.0])
        for s in range(nseg):
            s2 = (s + 1) % nseg
            tris.append([ctr, ring[s] + [0, y, 0], ring[s2] + [0, y, 0]])
    return np.ascontiguousarray(np.array(tris))


def _finish(name, params, x, R, rng, tri, steps, v=None, w=None, q=None, R_max=None):
    n = len(R)
    if v is None:
        v = np.zeros((n, 3))
    if w is None:
        w = np.zeros((n, 3))
    if q is None:
        q = shoemake_quaternions(rng, n)
    tri = np.zeros((0, 3, 3)) if tri is None else np.ascontiguousarray(tri, dtype=np.float64)
    return {"name": name, "params": params, "x": np.ascontiguousarray(x, dtype=np.float64),
            "v": np.ascontiguousarray(v, dtype=np.float64),
            "w": np.ascontiguousarray(w, dtype=np.float64),
            "q": np.ascontiguousarray(q, dtype=np.float64),
            "R": np.ascontiguousarray(R, dtype=np.float64), "tri": tri,
            "rmesh": np.zeros(len(tri)), "steps": int(steps),
            "R_max": float((R.max() if len(R) else 0.0) if R_max is None else R_max)}


# ---------------------------------------------------------------------------
# the five configurations
# ---------------------------------------------------------------------------
def cfg1(seed=101, pitch=2.2 * MM):
    """1,000 spheres, R ~ U[0.8, 1.2] mm, rho 2500, jittered 10^3 lattice
    (centres 1.1 + k*pitch mm, +-0.05 mm jitter) in the lower corner of a
    closed 12-triangle cube of side 30 mm; zero velocity, random orientation;
    mu 0.5/0.1/0.1, e_n 0.7, dt = 1e-6 s, 2,000 steps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n1 = 10
    R = rng.uniform(0.8 * MM, 1.2 * MM, n1 ** 3)
    k = np.arange(n1)
    g = np.stack(np.meshgrid(k, k, k, indexing="ij"), axis=-1).reshape(-1, 3)
    x = 1.1 * MM + g * pitch + rng.uniform(-0.05 * MM, 0.05 * MM, (n1 ** 3, 3))
    tri = cube_mesh([0, 0, 0], [30 * MM] * 3)
    return _finish("cfg1_box_drop_1k", default_params(dt=1e-6), x, R, rng, tri, 2000, R_max=1.2 * MM)


def cfg2(seed=202, n=200_000, shrink=0.999):
    """200,000 spheres, R = 1 mm * exp(0.2 Z), granular column on a
    600 x 600 mm two-triangle floor, full friction, dt = 5e-7 s, 20,000 steps.

    The settled column before its side walls are taken away: the spheres are
    poured, one after another in random order, into a 60 x 60 mm column
    (sequential deposition with rolling at radii shrink*R, periodic across
    the column's sides so that no side wall shapes the packing), each coming
    to rest on the floor or on three spheres that carry it (packing fraction
    about 0.59, about 6 contacts per sphere, a column about 475 mm high).
    At the true radii every such contact is pressed by (1 - shrink) of the
    two radii (about 2 micrometres), the bottom layer into the floor alike.
    The run starts with the column standing free (the collapse)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    R = MM * np.exp(0.2 * rng.standard_normal(n))
    L = 60 * MM
    x, stuck = deposit(shrink * R, L, L, seed)
    if stuck:
        raise RuntimeError(f"deposition left {stuck} spheres unsettled")
    x[:, 0] -= 0.5 * L
    x[:, 1] -= 0.5 * L
    tri = floor_mesh(0.0, 0.0, 300 * MM, 0.0)
    return _finish("cfg2_column_collapse_200k", default_params(dt=5e-7), x, R, rng, tri, 20000)


def fcc_sites(lo, hi, a_nn):
    """Face-centred cubic lattice sites (nearest-neighbour distance a_nn)
    inside the box [lo, hi], in (k, j, i, basis) generation order."""
    a = a_nn * math.sqrt(2.0)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    cnt = np.floor((hi - lo) / a).astype(np.int64) + 1
    g = np.stack(np.meshgrid(np.arange(cnt[0]), np.arange(cnt[1]), np.arange(cnt[2]),
                             indexing="ij"), axis=-1).reshape(-1, 3)
    basis = np.array([[0, 0, 0], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])
    pts = (lo + a * (g[:, None, :] + basis[None, :, :])).reshape(-1, 3)
    inside = np.all((pts >= lo) & (pts <= hi), axis=1)
    return pts[inside]


def cfg3(seed=303, n=2_000_000, a_nn=2.22 * MM, jitter=0.005 * MM):
    """2,000,000 spheres, R ~ U[0.9, 1.1] mm, in a rotating drum (radius
    0.15 m, axis y, length 0.40 m, 8,192 triangles, 1 rad/s about y through
    the origin); dt from Eq. dt at R_min = 0.9 mm.

    Start: the n lowest sites of a face-centred cubic lattice (nearest
    neighbours 2.22 mm apart, +-0.005 mm jitter per coordinate, so no two
    spheres touch) that lie at least R_max + 0.05 mm inside the drum's
    polygonal shell and end caps; zero velocity, random orientation.  The bed
    fills about half the drum and settles onto the shell within ~50 steps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Rd, Ld, nseg = 0.15, 0.40, 128
    R = rng.uniform(0.9 * MM, 1.1 * MM, n)
    clear = 1.1 * MM + 0.05 * MM
    r_in = Rd * math.cos(math.pi / nseg) - clear  # inscribed radius of the shell
    pts = fcc_sites([-r_in, -Ld / 2 + clear, -r_in], [r_in, Ld / 2 - clear, r_in], a_nn)
    pts = pts[pts[:, 0] ** 2 + pts[:, 2] ** 2 <= r_in * r_in]
    if len(pts) < n:
        raise ValueError(f"the drum holds {len(pts)} lattice sites, fewer than {n}")
    pts = pts[np.argsort(pts[:, 2], kind="stable")[:n]]
    x = pts + rng.uniform(-jitter, jitter, (n, 3))
    tri = drum_mesh(Rd, Ld, nseg)
    p = default_params(dt=dt_eq(0.9 * MM, 2500.0, 1e6, 0.3), mesh_omega=(0.0, 1.0, 0.0))
    return _finish("cfg3_rotating_drum_2M", p, x, R, rng, tri, 2000, R_max=1.1 * MM)


def cfg4_sim(s, n_s, seed=404):
    """One simulation of the batched sweep: a 'box drop' of n_s spheres,
    R ~ U[0.8, 1.2] mm, on an n x n lattice of pitch 2.5 mm (n = ceil(n_s^1/3))
    layered upward from 1.5 mm above the floor of a 12-triangle cube of side
    5n mm, horizontally centred, so the layers land one after another within
    the first ~1,500 steps; mu_s = 0.1 + 0.8 s/255, mu_r = mu_t = 0.1."""
    rng = np.random.Generator(np.random.PCG64(404_000 + s))
    nl = int(math.ceil(n_s ** (1.0 / 3.0) - 1e-9))
    Ls = 5.0 * nl * MM
    R = rng.uniform(0.8 * MM, 1.2 * MM, n_s)
    k = np.arange(n_s)
    ix, iy, iz = k % nl, (k // nl) % nl, k // (nl * nl)
    off = (Ls - (nl - 1) * 2.5 * MM) / 2.0
    x = np.stack([off + ix * 2.5 * MM, off + iy * 2.5 * MM, 1.5 * MM + iz * 2.5 * MM], axis=1)
    tri = cube_mesh([0, 0, 0], [Ls] * 3)
    p = default_params(dt=dt_eq(0.8 * MM, 2500.0, 1e6, 0.3), mu_s=0.1 + 0.8 * s / 255.0)
    return _finish(f"cfg4_sim{s}", p, x, R, rng, tri, 5000, R_max=1.2 * MM)


def cfg4(nsims=256, seed=404, sizes=None):
    """256 independent box drops of uneven size N_s ~ U{500..20,000}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if sizes is None:
        sizes = rng.integers(500, 20_000, size=nsims, endpoint=True)
    return [cfg4_sim(s, int(sizes[s]), seed) for s in range(nsims)]


def cfg5(seed=505, n=8_000_000, dims=(152, 161, 165), d_ls=2.38 * MM, jitter=0.001 * MM):
    """8,000,000 spheres, half R = 1.4 mm and half 1.0 mm, a pre-compressed
    static packing in a closed 12-triangle box; full friction, no gravity,
    eta = 0, dt from Eq. dt at 1.0 mm, 10,000 relaxation steps.

    Start: a body-centred (CsCl-type) arrangement.  Large spheres sit on a
    cubic lattice of dims[0] x dims[1] x dims[2] sites, small ones at the
    centres of its cells; the lattice constant puts every large-small pair
    at d_ls (overlap 0.02 mm), which presses the six axial large-large
    neighbours together by 0.052 mm.  Each small sphere touches 8 large
    ones, each large sphere 8 small and 6 large ones.  With these radii no
    body-centred packing keeps large-small contacts without large-large ones
    (that needs R_small >= 0.732 R_large), and in a rock-salt arrangement
    every lattice line ends at one wall with a small sphere 0.4 mm short of
    it, so it cannot be held in place by flat walls.

    The walls stand at the outermost large spheres with the overlap whose
    textbook Hertz force (4/3 E* sqrt(R*) delta^1.5; E* doubled for a rigid
    wall, R* = R) balances the contacts a boundary sphere lacks on its outer
    side: one large-large and four large-small ones at 1/sqrt(3) of their
    force.  Interior spheres are balanced by symmetry, so the packing starts
    in equilibrium up to +-jitter per coordinate (uniform); it then relaxes
    the small imbalances this leaves.  The surplus of the box over n (120
    sites) are small spheres removed at random (vacancies); n=None keeps
    every site (a smaller box of the same packing: dims sites per axis).

    Gravity is off: under gravity a column of 160 layers of this soft
    material (E = 1 MPa) loads its bottom contacts with several times the
    pre-compression force and sags by millimetres instead of relaxing in
    place."""
    rng = np.random.Generator(np.random.PCG64(seed))
    RL, RS = 1.4 * MM, 1.0 * MM
    a = 2.0 * d_ls / math.sqrt(3.0)
    nx, ny, nz = dims
    gl = np.stack(np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij"),
                  axis=-1).reshape(-1, 3)[:, ::-1].astype(float)
    gs = np.stack(np.meshgrid(np.arange(nz - 1), np.arange(ny - 1), np.arange(nx - 1),
                              indexing="ij"), axis=-1).reshape(-1, 3)[:, ::-1] + 0.5
    if n is None:
        n = len(gl) + len(gs)
    surplus = len(gl) + len(gs) - n
    if surplus < 0 or surplus > len(gs):
        raise ValueError("the box does not hold n spheres")
    if surplus:
        gs = np.delete(gs, rng.choice(len(gs), surplus, replace=False), axis=0)
    g = np.concatenate([gl, gs])
    R = np.concatenate([np.full(len(gl), RL), np.full(len(gs), RS)])
    order = np.lexsort((g[:, 0], g[:, 1], g[:, 2]))  # (z, y, x) order of sites
    g, R = g[order], R[order]
    x = g * a + rng.uniform(-jitter, jitter, (n, 3))
    # wall overlap: Hertz force on a boundary large sphere from the wall equal
    # to the outward sum of its missing contacts (the 4/3 factors cancel)
    E_pair = 1.0 / (2.0 * (1.0 - 0.3 * 0.3))  # E* / E of two spheres; a wall's is twice this
    d_ll = 2.0 * RL - a
    f_ll = E_pair * math.sqrt(RL * RL / (2 * RL)) * d_ll ** 1.5
    f_ls = E_pair * math.sqrt(RL * RS / (RL + RS)) * (RL + RS - d_ls) ** 1.5
    d_w = ((f_ll + 4.0 * f_ls / math.sqrt(3.0)) / (2.0 * E_pair * math.sqrt(RL))) ** (2.0 / 3.0)
    lo = np.full(3, -(RL - d_w))
    hi = (np.array(dims, float) - 1.0) * a + (RL - d_w)
    tri = cube_mesh(lo, hi)
    p = default_params(dt=dt_eq(1.0 * MM, 2500.0, 1e6, 0.3), g=(0.0, 0.0, 0.0))
    name = "cfg5_dense_packing_8M" if n == 8_000_000 else f"dense_packing_{n}"
    return _finish(name, p, x, R, rng, tri, 10000, R_max=RL)


# ---------------------------------------------------------------------------
# small cases for tests
# ---------------------------------------------------------------------------
def crowded_sphere(n_small=64, seed=77, R_big=10 * MM, r_small=2 * MM, overlap=0.01 * MM,
                   v_in=0.05, vel=0.005):
    """One sphere of radius R_big with n_small spheres of radius r_small pressed
    on it (the ends of Table 2's radius range, 2 and 10 mm): the small ones at
    the points of a Fibonacci lattice on the sphere of radius R_big + r_small -
    overlap (directions jittered by 2 degrees), so the large one has n_small
    contacts at once, more than a particle's search holds on chip (24) and more
    than the least per-particle capacity a context may ask for (32).
    The small ones move towards the centre at v_in (plus random velocities
    and spins of scale vel), so the contacts last about 20 steps; no gravity,
    a closed 12-triangle box well clear of the cluster; dt from Eq. dt at
    r_small."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = np.arange(n_small) + 0.5
    ph = np.arccos(1.0 - 2.0 * k / n_small)
    th = np.pi * (1.0 + 5.0 ** 0.5) * k
    d = np.stack([np.sin(ph) * np.cos(th), np.sin(ph) * np.sin(th), np.cos(ph)], axis=1)
    d += rng.normal(0.0, math.radians(2.0), d.shape)
    d /= np.linalg.norm(d, axis=1)[:, None]
    x = np.concatenate([np.zeros((1, 3)), d * (R_big + r_small - overlap)])
    R = np.concatenate([[R_big], np.full(n_small, r_small)])
    half = R_big + 3.0 * r_small
    tri = cube_mesh([-half] * 3, [half] * 3)
    p = default_params(dt=dt_eq(r_small, 2500.0, 1e6, 0.3), g=(0.0, 0.0, 0.0))
    v = rng.normal(0.0, vel, (len(R), 3))
    v[1:] -= v_in * d
    w = rng.normal(0.0, vel / r_small, (len(R), 3))
    return _finish(f"crowded_sphere{n_small}_{seed}", p, x, R, rng, tri, 200, v=v, w=w)


def random_cluster(n, seed, box=10 * MM, r_lo=0.8 * MM, r_hi=1.2 * MM, vel=0.05, spin=20.0,
                   overlap=0.15, params=None, tri=None):
    """n spheres at random in a cube (packing by random sequential addition at
    radii (1-overlap)R, so some neighbours start overlapped), with random
    velocities and spins.  Used for small parity and edge cases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    R = rng.uniform(r_lo, r_hi, n)
    x = rsa_place((1.0 - overlap) * R, [0, 0, 0], [box] * 3, seed + 17)
    v = rng.normal(0.0, vel, (n, 3))
    w = rng.normal(0.0, spin, (n, 3))
    p = default_params(dt=2e-6) if params is None else params
    return _finish(f"cluster{n}_{seed}", p, x, R, rng, tri, 100, v=v, w=w)
