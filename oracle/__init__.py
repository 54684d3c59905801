"""Plain FP64 CPU oracle of the TinyDEM time step (arXiv 2507.12610).

TEST INFRASTRUCTURE ONLY.  This package wraps ``dem_oracle.c`` (a slow,
serial, double-precision C implementation written from the paper's
equations) with ctypes.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark import it; the GPU solver never does.  It
shares no code with the GPU library.

Arrays follow the C side: vectors ``(n, 3)``, quaternions ``(n, 4)`` scalar
first, triangles ``(m, 3, 3)``, all float64 C-contiguous.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dem_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [("rho", C.c_double), ("E", C.c_double), ("nu", C.c_double),
                ("e_n", C.c_double), ("mu_s", C.c_double), ("mu_r", C.c_double),
                ("mu_t", C.c_double), ("eta", C.c_double), ("g", C.c_double * 3),
                ("dt", C.c_double), ("mesh_omega", C.c_double * 3),
                ("mesh_center", C.c_double * 3)]


class Motion(C.Structure):
    _fields_ = [("omega", C.c_double * 3), ("center", C.c_double * 3), ("amp", C.c_double * 3),
                ("freq", C.c_double), ("phase", C.c_double)]


def make_motion(omega=(0.0, 0.0, 0.0), center=(0.0, 0.0, 0.0), amp=(0.0, 0.0, 0.0), freq=0.0,
                phase=0.0) -> Motion:
    return Motion((C.c_double * 3)(*omega), (C.c_double * 3)(*center), (C.c_double * 3)(*amp),
                  float(freq), float(phase))


class Spawn(C.Structure):
    _fields_ = [("smin", C.c_double * 3), ("smax", C.c_double * 3), ("Rmin", C.c_double),
                ("Rmax", C.c_double), ("v0", C.c_double * 3), ("w0", C.c_double * 3),
                ("n_spawn", C.c_int64), ("n_max", C.c_int64), ("seed", C.c_uint64)]


def make_spawn(smin, smax, Rmin, Rmax, v0=(0.0, 0.0, 0.0), w0=(0.0, 0.0, 0.0), n_spawn=100,
               n_max=1000, seed=0) -> Spawn:
    return Spawn((C.c_double * 3)(*smin), (C.c_double * 3)(*smax), float(Rmin), float(Rmax),
                 (C.c_double * 3)(*v0), (C.c_double * 3)(*w0), int(n_spawn), int(n_max),
                 int(seed))


def philox4x32_10(ctr, key):
    """Philox4x32-10 output words for counter ctr[4] and key key[2]."""
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


class Contact(C.Structure):
    _fields_ = [("delta", C.c_double), ("d", C.c_double), ("ri", C.c_double), ("rj", C.c_double),
                ("n", C.c_double * 3), ("kn", C.c_double), ("ks", C.c_double),
                ("cn", C.c_double), ("cs", C.c_double),
                ("fn", C.c_double * 3), ("fs", C.c_double * 3), ("fr", C.c_double * 3),
                ("ft", C.c_double),
                ("vn", C.c_double * 3), ("vs", C.c_double * 3), ("vr", C.c_double * 3),
                ("vt", C.c_double),
                ("fi", C.c_double * 3), ("ti", C.c_double * 3),
                ("fj", C.c_double * 3), ("tj", C.c_double * 3),
                ("us", C.c_double * 3), ("ur", C.c_double * 3), ("ut", C.c_double),
                ("kinetic", C.c_int32 * 3)]

    def as_dict(self) -> dict:
        out = {}
        for name, _ in self._fields_:
            val = getattr(self, name)
            out[name] = np.array(val[:]) if hasattr(val, "__len__") else float(val)
        out["kinetic"] = [int(k) for k in self.kinetic]
        return out


_lib = None
_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)
_I64 = C.POINTER(C.c_int64)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        L.orc_beta.restype = C.c_double
        L.orc_beta.argtypes = [C.c_double]
        L.orc_dt_default.restype = C.c_double
        L.orc_dt_default.argtypes = [C.c_double] * 4
        L.orc_closest_point_triangle.argtypes = [_D] * 5
        L.orc_closest_point_segment.argtypes = [_D] * 4
        L.orc_closest_point_rectangle.argtypes = [_D] * 6
        L.orc_closest_point_element.argtypes = [_D, C.c_int32, _D, _D]
        L.orc_set_mesh_elements.argtypes = [C.c_void_p, C.c_int64, _I32, _D, _D]
        L.orc_quat_mul.argtypes = [_D] * 3
        L.orc_validate.argtypes = [C.POINTER(Params)]
        L.orc_eval_pp.restype = C.c_int
        L.orc_eval_pp.argtypes = [C.POINTER(Params), _D, _D, _D, C.c_double, _D, _D, _D, C.c_double,
                                  _D, _D, C.c_double, C.POINTER(Contact)]
        L.orc_eval_pw.restype = C.c_int
        L.orc_eval_pw.argtypes = [C.POINTER(Params), _D, _D, _D, C.c_double, _D, C.c_double, _D, _D,
                                  _D, _D, C.c_double, C.POINTER(Contact)]
        L.orc_integrate.argtypes = [C.POINTER(Params), C.c_double, _D, _D, _D, _D, _D, _D]
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(Params), C.c_int64, _D, _D, _D, _D, _D]
        L.orc_free.argtypes = [C.c_void_p]
        L.orc_set_mesh.argtypes = [C.c_void_p, C.c_int64, _D, _D]
        L.orc_set_history.argtypes = [C.c_void_p, C.c_int64, _I32, _I32, _D, _D, _D]
        L.orc_set_time.argtypes = [C.c_void_p, C.c_double]
        L.orc_get_time.restype = C.c_double
        L.orc_get_time.argtypes = [C.c_void_p]
        L.orc_set_search.argtypes = [C.c_void_p, C.c_int32, C.c_double]
        L.orc_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc_get_state.argtypes = [C.c_void_p, _D, _D, _D, _D]
        L.orc_get_forces.argtypes = [C.c_void_p, _D, _D, _D, _D]
        L.orc_num_particles.restype = C.c_int64
        L.orc_num_particles.argtypes = [C.c_void_p]
        L.orc_get_radii.argtypes = [C.c_void_p, _D]
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32)] * 3
        L.orc_set_spawn.argtypes = [C.c_void_p, C.POINTER(Spawn)]
        L.orc_set_mesh_motion.argtypes = [C.c_void_p, C.c_int32, C.POINTER(Motion), _I32]
        L.orc_wall_velocity.argtypes = [C.c_void_p, C.c_int64, _D, _D, _D]
        L.orc_spawn_status.argtypes = [C.c_void_p, C.POINTER(C.c_uint64), C.POINTER(C.c_double)]
        L.orc_set_spawn_status.argtypes = [C.c_void_p, C.c_uint64, C.c_double]
        L.orc_num_contacts.restype = C.c_int64
        L.orc_num_contacts.argtypes = [C.c_void_p]
        L.orc_get_contacts.argtypes = [C.c_void_p, _I32, _I32, _D, _D, _D, _D, _D, _D]
        L.orc_get_mesh.argtypes = [C.c_void_p, _D]
        L.orc_sample_step.argtypes = [C.c_void_p, C.c_int64, _I64, _D, _D, _D, _D, _I64, _D, _D,
                                      _D, _D]
        L.orc_sample_keys.restype = C.c_int64
        L.orc_sample_keys.argtypes = [C.c_void_p, C.c_int64, _I64, C.c_int64, _I64, _I32, _I32]
        L.orc_contact_keys.restype = C.c_int64
        L.orc_contact_keys.argtypes = [C.c_void_p, C.c_int64, _I32, _I32]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_D)


def _vec(a, n=None, k=3):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if n is not None:
        a = a.reshape(n, k)
    return a


def make_params(rho=1e3, E=1e6, nu=0.3, e_n=0.5, mu_s=0.3, mu_r=0.3, mu_t=None, eta=0.0,
                g=(0.0, 0.0, -9.81), dt=1e-5, mesh_omega=(0.0, 0.0, 0.0),
                mesh_center=(0.0, 0.0, 0.0)) -> Params:
    """Parameter struct; defaults follow Table 2 (mu_t = 2 mu_s / 3)."""
    if mu_t is None:
        mu_t = 2.0 * mu_s / 3.0
    return Params(rho, E, nu, e_n, mu_s, mu_r, mu_t, eta, (C.c_double * 3)(*g), dt,
                  (C.c_double * 3)(*mesh_omega), (C.c_double * 3)(*mesh_center))


def params_from_dict(d: dict) -> Params:
    keys = ("rho", "E", "nu", "e_n", "mu_s", "mu_r", "mu_t", "eta", "g", "dt", "mesh_omega",
            "mesh_center")
    return make_params(**{k: d[k] for k in keys if k in d})


def beta(e_n: float) -> float:
    return lib().orc_beta(e_n)


def dt_default(R_min, rho, E, nu) -> float:
    return lib().orc_dt_default(R_min, rho, E, nu)


def closest_point_triangle(p, a, b, c) -> np.ndarray:
    out = np.zeros(3)
    args = [_vec(v) for v in (p, a, b, c)]
    lib().orc_closest_point_triangle(*[_p(v) for v in args], _p(out))
    return out


def closest_point_segment(p, a, b) -> np.ndarray:
    out = np.zeros(3)
    args = [_vec(v) for v in (p, a, b)]
    lib().orc_closest_point_segment(*[_p(v) for v in args], _p(out))
    return out


def closest_point_rectangle(p, a, b, c, d) -> np.ndarray:
    out = np.zeros(3)
    args = [_vec(v) for v in (p, a, b, c, d)]
    lib().orc_closest_point_rectangle(*[_p(v) for v in args], _p(out))
    return out


def closest_point_element(p, verts) -> np.ndarray:
    """Closest point on an element given by its 1..4 vertices."""
    v = np.asarray(verts, np.float64).reshape(-1, 3)
    nv = len(v)
    buf = np.zeros((4, 3))
    buf[:nv] = v
    buf[nv:] = v[-1]
    out = np.zeros(3)
    lib().orc_closest_point_element(_p(_vec(p)), nv, _p(buf), _p(out))
    return out


def pack_elements(elements):
    """(nv [m] int32, verts [m][4][3]) from a list of 1..4-vertex arrays."""
    m = len(elements)
    nv = np.zeros(m, np.int32)
    verts = np.zeros((m, 4, 3))
    for k, e in enumerate(elements):
        e = np.asarray(e, np.float64).reshape(-1, 3)
        nv[k] = len(e)
        verts[k, :len(e)] = e
        verts[k, len(e):] = e[-1]
    return nv, verts


def quat_mul(a, b) -> np.ndarray:
    out = np.zeros(4)
    a = _vec(a)
    b = _vec(b)
    lib().orc_quat_mul(_p(a), _p(b), _p(out))
    return out


def validate(params: Params) -> bool:
    return lib().orc_validate(C.byref(params)) == 0


def eval_pp(params, xi, vi, wi, Ri, xj, vj, wj, Rj, us=(0, 0, 0), ur=(0, 0, 0), ut=0.0):
    """One particle-particle contact; returns a dict or None if not touching."""
    o = Contact()
    a = [_vec(v) for v in (xi, vi, wi, xj, vj, wj, us, ur)]
    hit = lib().orc_eval_pp(C.byref(params), _p(a[0]), _p(a[1]), _p(a[2]), float(Ri), _p(a[3]),
                            _p(a[4]), _p(a[5]), float(Rj), _p(a[6]), _p(a[7]), float(ut),
                            C.byref(o))
    return o.as_dict() if hit else None


def eval_pw(params, xi, vi, wi, Ri, cp, Rm=0.0, vwall=(0, 0, 0), wwall=(0, 0, 0), us=(0, 0, 0),
            ur=(0, 0, 0), ut=0.0):
    o = Contact()
    a = [_vec(v) for v in (xi, vi, wi, cp, vwall, wwall, us, ur)]
    hit = lib().orc_eval_pw(C.byref(params), _p(a[0]), _p(a[1]), _p(a[2]), float(Ri), _p(a[3]),
                            float(Rm), _p(a[4]), _p(a[5]), _p(a[6]), _p(a[7]), float(ut),
                            C.byref(o))
    return o.as_dict() if hit else None


def integrate(params, R, F, T, x, v, w, q):
    """One particle's integration step; returns the new (x, v, w, q)."""
    F, T = _vec(F), _vec(T)
    x, v, w, q = _vec(x).copy(), _vec(v).copy(), _vec(w).copy(), _vec(q).copy()
    lib().orc_integrate(C.byref(params), float(R), _p(F), _p(T), _p(x), _p(v), _p(w), _p(q))
    return x, v, w, q


class Sim:
    """One simulation held by the oracle."""

    def __init__(self, params, x, v=None, w=None, q=None, R=None, tri=None, rmesh=None,
                 elements=None):
        x = _vec(x)
        n = x.shape[0]
        self.n = n
        v = _vec(np.zeros((n, 3)) if v is None else v, n)
        w = _vec(np.zeros((n, 3)) if w is None else w, n)
        if q is None:
            q = np.zeros((n, 4))
            q[:, 0] = 1.0
        q = _vec(q, n, 4)
        R = np.ascontiguousarray(np.asarray(R, dtype=np.float64).reshape(n))
        if isinstance(params, dict):
            params = params_from_dict(params)
        self.params = params
        self._h = lib().orc_create(C.byref(params), n, _p(x.reshape(n, 3)), _p(v), _p(w), _p(q),
                                   _p(R))
        if not self._h:
            raise ValueError("oracle rejected the parameters or radii (Table 2 requirements)")
        self.ntri = 0
        if tri is not None:
            self.set_mesh(tri, rmesh)
        if elements is not None:
            self.set_mesh_elements(elements, rmesh)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_free(h)
            self._h = None

    def set_mesh(self, tri, rmesh=None):
        tri = np.ascontiguousarray(np.asarray(tri, dtype=np.float64).reshape(-1, 9))
        m = tri.shape[0]
        rm = None if rmesh is None else np.ascontiguousarray(np.asarray(rmesh, np.float64).reshape(m))
        if lib().orc_set_mesh(self._h, m, _p(tri), _p(rm) if rm is not None else None) != 0:
            raise ValueError("bad mesh")
        self.ntri = m

    def set_mesh_elements(self, elements, rmesh=None):
        """Mesh of points, segments, triangles and rectangles: a list of
        1..4-vertex arrays, or a pair (nv [m], verts [m][4][3])."""
        if isinstance(elements, tuple):
            nv, verts = elements
            nv = np.ascontiguousarray(nv, np.int32)
            verts = np.ascontiguousarray(np.asarray(verts, np.float64).reshape(len(nv), 12))
        else:
            nv, verts = pack_elements(elements)
            verts = np.ascontiguousarray(verts.reshape(len(nv), 12))
        m = len(nv)
        rm = None if rmesh is None else np.ascontiguousarray(np.asarray(rmesh, np.float64).reshape(m))
        if lib().orc_set_mesh_elements(self._h, m, nv.ctypes.data_as(_I32), _p(verts),
                                       _p(rm) if rm is not None else None) != 0:
            raise ValueError("bad mesh")
        self.ntri = m

    def set_history(self, ki, kj, us, ur, ut):
        ki = np.ascontiguousarray(ki, dtype=np.int32)
        kj = np.ascontiguousarray(kj, dtype=np.int32)
        us = _vec(us, len(ki))
        ur = _vec(ur, len(ki))
        ut = np.ascontiguousarray(ut, dtype=np.float64)
        lib().orc_set_history(self._h, len(ki), ki.ctypes.data_as(_I32), kj.ctypes.data_as(_I32),
                              _p(us), _p(ur), _p(ut))

    def set_time(self, t):
        lib().orc_set_time(self._h, float(t))

    @property
    def time(self):
        return lib().orc_get_time(self._h)

    def set_search(self, mode: int, cell_factor: float = 1.0):
        lib().orc_set_search(self._h, int(mode), float(cell_factor))

    def step(self, nsteps: int = 1):
        if lib().orc_step(self._h, int(nsteps)) != 0:
            raise RuntimeError("oracle step failed")
        self.n = int(lib().orc_num_particles(self._h))

    def set_mesh_motion(self, motions, groups=None):
        """Motion groups (an extension generalising the rotating mesh): a list
        of dicts with the keywords of make_motion, and the group of each
        element (None: all in group 0)."""
        arr = (Motion * len(motions))(*[make_motion(**m) for m in motions])
        g = None if groups is None else np.ascontiguousarray(groups, np.int32)
        if lib().orc_set_mesh_motion(self._h, len(motions), arr,
                                     g.ctypes.data_as(_I32) if g is not None else None) != 0:
            raise ValueError("bad mesh motion")

    def wall_velocity(self, m, p):
        """(velocity, spin) of element m's wall at point p, at the current time."""
        vw, ww = np.zeros(3), np.zeros(3)
        lib().orc_wall_velocity(self._h, int(m), _p(_vec(p)), _p(vw), _p(ww))
        return vw, ww

    def set_spawn(self, spawn=None, **kw):
        """Particle spawning (Section 3.1): a Spawn structure or the keyword
        arguments of make_spawn; None turns it off."""
        if spawn is None and kw:
            spawn = make_spawn(**kw)
        if lib().orc_set_spawn(self._h, C.byref(spawn) if spawn is not None else None) != 0:
            raise ValueError("bad spawn parameters")

    def set_spawn_status(self, attempts, carried):
        lib().orc_set_spawn_status(self._h, int(attempts), float(carried))

    def spawn_status(self):
        a, r = C.c_uint64(), C.c_double()
        lib().orc_spawn_status(self._h, C.byref(a), C.byref(r))
        return int(a.value), float(r.value)

    @property
    def radii(self):
        n = self.n
        out = np.zeros(n)
        if n:
            lib().orc_get_radii(self._h, _p(out))
        return out

    def state(self):
        n = self.n
        x, v, w = (np.zeros((n, 3)) for _ in range(3))
        q = np.zeros((n, 4))
        lib().orc_get_state(self._h, _p(x), _p(v), _p(w), _p(q))
        return {"x": x, "v": v, "w": w, "q": q}

    def forces(self):
        n = self.n
        F, T = np.zeros((n, 3)), np.zeros((n, 3))
        Fs, Ts = np.zeros(n), np.zeros(n)
        lib().orc_get_forces(self._h, _p(F), _p(T), _p(Fs), _p(Ts))
        return {"F": F, "T": T, "Fscale": Fs, "Tscale": Ts}

    def contacts(self):
        nc = lib().orc_num_contacts(self._h)
        ki = np.zeros(nc, np.int32)
        kj = np.zeros(nc, np.int32)
        us, ur, f, ti, tj = (np.zeros((nc, 3)) for _ in range(5))
        ut = np.zeros(nc)
        lib().orc_get_contacts(self._h, ki.ctypes.data_as(_I32), kj.ctypes.data_as(_I32), _p(us),
                               _p(ur), _p(ut), _p(f), _p(ti), _p(tj))
        return {"ki": ki, "kj": kj, "us": us, "ur": ur, "ut": ut, "f": f, "ti": ti, "tj": tj}

    def mesh(self):
        """Current vertices [m][4][3] (slots past an element's own vertices
        repeat its last one)."""
        v = np.zeros((self.ntri, 4, 3))
        if self.ntri:
            lib().orc_get_mesh(self._h, _p(v))
        return v

    def contact_keys(self):
        """Contact set of the current state (no forces, no advance)."""
        n = lib().orc_contact_keys(self._h, 0, None, None)
        ki = np.zeros(max(n, 1), np.int32)
        kj = np.zeros(max(n, 1), np.int32)
        lib().orc_contact_keys(self._h, n, ki.ctypes.data_as(_I32), kj.ctypes.data_as(_I32))
        return ki[:n], kj[:n]

    def sample_keys(self, idx):
        """Keys of every contact each listed particle takes part in, at the
        current state: (ki, kj, counts), one particle after another, each in
        key order."""
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        cnt = np.zeros(len(idx), np.int64)
        tot = lib().orc_sample_keys(self._h, len(idx), idx.ctypes.data_as(_I64), 0,
                                    cnt.ctypes.data_as(_I64), None, None)
        if tot < 0:
            raise IndexError("sample index out of range")
        ki = np.zeros(max(tot, 1), np.int32)
        kj = np.zeros(max(tot, 1), np.int32)
        lib().orc_sample_keys(self._h, len(idx), idx.ctypes.data_as(_I64), tot,
                              cnt.ctypes.data_as(_I64), ki.ctypes.data_as(_I32),
                              kj.ctypes.data_as(_I32))
        return ki[:tot], kj[:tot], cnt

    def sample_step(self, idx):
        """Net force/torque on each listed particle at the current state and
        its state one step later, without advancing the simulation."""
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        ns = len(idx)
        F, T, x1, v1, w1 = (np.zeros((ns, 3)) for _ in range(5))
        q1 = np.zeros((ns, 4))
        Fs, Ts = np.zeros(ns), np.zeros(ns)
        nc = np.zeros(ns, np.int64)
        rc = lib().orc_sample_step(self._h, ns, idx.ctypes.data_as(_I64), _p(F), _p(T), _p(Fs),
                                   _p(Ts), nc.ctypes.data_as(_I64), _p(x1), _p(v1), _p(w1), _p(q1))
        if rc != 0:
            raise IndexError("sample index out of range")
        return {"F": F, "T": T, "Fscale": Fs, "Tscale": Ts, "ncont": nc, "x": x1, "v": v1,
                "w": w1, "q": q1}
