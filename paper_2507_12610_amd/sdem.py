"""Thin Python binding of the sdem C ABI (``include/sdem.h``).

Argument marshalling only: every step of the DEM hot path runs in the HIP
kernels of ``libsdem.so``.  PyTorch provides device memory (state upload and
the workspace) and the HIP stream.  There is no CPU fallback: if the library
is missing or no GPU is present the constructor raises.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsdem.so")

SDEM_OK, SDEM_EINVAL, SDEM_ECAPACITY, SDEM_ENONFINITE, SDEM_EHIP, SDEM_ESTATE = 0, -1, -2, -3, -4, -5
SDEM_FP64, SDEM_MIXED = 0, 1
_NAMES = {SDEM_EINVAL: "EINVAL", SDEM_ECAPACITY: "ECAPACITY", SDEM_ENONFINITE: "ENONFINITE",
          SDEM_EHIP: "EHIP", SDEM_ESTATE: "ESTATE"}

EXPORTS = ("sdem_workspace_bytes", "sdem_init", "sdem_init_static", "sdem_init_batch",
           "sdem_add_mesh",
           "sdem_add_mesh_elements", "sdem_set_spawn", "sdem_spawn_status", "sdem_read_radii",
           "sdem_set_spawn_status", "sdem_set_clock", "sdem_read_off", "sdem_write_csv",
           "sdem_set_mesh_motion",
           "sdem_read_csv", "sdem_write_contacts_csv", "sdem_read_contacts_csv",
           "sdem_set_history", "sdem_step", "sdem_read_state", "sdem_read_contacts", "sdem_stats",
           "sdem_destroy", "sdem_last_error", "sdem_selftest_rounding", "sdem_step_profiled",
           "sdem_copy_probe", "sdem_graph_stats")
PHASES = ("grid", "sort", "begin", "step", "empty", "step_kernel")


class SdemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sdem {_NAMES.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("rho", C.c_double), ("E", C.c_double), ("nu", C.c_double),
                ("e_n", C.c_double), ("mu_s", C.c_double), ("mu_r", C.c_double),
                ("mu_t", C.c_double), ("eta", C.c_double), ("g", C.c_double * 3),
                ("dt", C.c_double), ("mesh_omega", C.c_double * 3),
                ("mesh_center", C.c_double * 3)]


class MeshMotion(C.Structure):
    _fields_ = [("omega", C.c_double * 3), ("center", C.c_double * 3), ("amp", C.c_double * 3),
                ("freq", C.c_double), ("phase", C.c_double)]


def make_motion(omega=(0.0, 0.0, 0.0), center=(0.0, 0.0, 0.0), amp=(0.0, 0.0, 0.0), freq=0.0,
                phase=0.0) -> MeshMotion:
    """Rigid motion of a group of mesh elements: turning with omega about the
    axis through center, displaced by amp (sin(2 pi freq t + phase) -
    sin(phase))."""
    return MeshMotion((C.c_double * 3)(*omega), (C.c_double * 3)(*center),
                      (C.c_double * 3)(*amp), float(freq), float(phase))


class SpawnParams(C.Structure):
    _fields_ = [("smin", C.c_double * 3), ("smax", C.c_double * 3), ("R_min", C.c_double),
                ("R_max", C.c_double), ("v0", C.c_double * 3), ("w0", C.c_double * 3),
                ("n_spawn", C.c_int64), ("n_max", C.c_int64), ("seed", C.c_uint64)]


def make_spawn(smin, smax, Rmin, Rmax, v0=(0.0, 0.0, 0.0), w0=(0.0, 0.0, 0.0), n_spawn=100,
               n_max=1000, seed=0) -> SpawnParams:
    """Spawn settings (Section 3.1): box of the centres, radius range,
    initial velocity and spin, attempts per step, cap, generator seed."""
    return SpawnParams((C.c_double * 3)(*smin), (C.c_double * 3)(*smax), float(Rmin),
                       float(Rmax), (C.c_double * 3)(*v0), (C.c_double * 3)(*w0), int(n_spawn),
                       int(n_max), int(seed))


class Config(C.Structure):
    _fields_ = [("n_max", C.c_int64), ("contacts_max", C.c_int64), ("cells_max", C.c_int64),
                ("tri_max", C.c_int64), ("nsims_max", C.c_int32), ("precision", C.c_int32),
                ("block", C.c_int32), ("detect_lanes", C.c_int32), ("cell_factor", C.c_double),
                ("skin", C.c_double), ("rebuild_every", C.c_int32),
                ("contacts_per_particle", C.c_int32)]


_lib = None
_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)
_I64 = C.POINTER(C.c_int64)
_VP = C.c_void_p


def lib():
    """Loads libsdem.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2507_12610_amd/build.py")
        L = C.CDLL(LIB_PATH)
        L.sdem_workspace_bytes.restype = C.c_size_t
        L.sdem_workspace_bytes.argtypes = [C.POINTER(Config)]
        L.sdem_init.argtypes = [C.POINTER(_VP), C.POINTER(Config), C.POINTER(Params), C.c_int64,
                                _VP, _VP, _VP, _VP, _VP, _VP, C.c_size_t, _VP]
        L.sdem_init_static.argtypes = [C.POINTER(_VP), C.POINTER(Config), C.POINTER(Params),
                                       C.c_int64, _VP, _VP, _VP, _VP, _VP, _VP]
        L.sdem_init_batch.argtypes = [C.POINTER(_VP), C.POINTER(Config), C.c_int32,
                                      C.POINTER(Params), _I64, _VP, _VP, _VP, _VP, _VP, _VP,
                                      C.c_size_t, _VP]
        L.sdem_add_mesh.argtypes = [_VP, C.c_int32, C.c_int64, _D, _D]
        L.sdem_add_mesh_elements.argtypes = [_VP, C.c_int32, C.c_int64, _I32, _D, _D]
        L.sdem_set_spawn.argtypes = [_VP, C.c_int32, C.POINTER(SpawnParams)]
        L.sdem_read_radii.argtypes = [_VP, _VP]
        L.sdem_set_spawn_status.argtypes = [_VP, C.c_uint64, C.c_double]
        L.sdem_set_clock.argtypes = [_VP, C.c_int64]
        L.sdem_set_mesh_motion.argtypes = [_VP, C.c_int32, C.c_int32, C.POINTER(MeshMotion), _I32]
        L.sdem_read_off.argtypes = [C.c_char_p, C.c_int32, _D, C.c_int64, C.POINTER(C.c_int64),
                                    _I32, _D, _D]
        L.sdem_write_csv.argtypes = [_VP, C.c_char_p]
        L.sdem_read_csv.argtypes = [C.c_char_p, C.c_int64, C.POINTER(C.c_int64), _D, _D, _D, _D,
                                    _D]
        L.sdem_write_contacts_csv.argtypes = [_VP, C.c_char_p]
        L.sdem_read_contacts_csv.argtypes = [C.c_char_p, C.c_int64, C.POINTER(C.c_int64), _I32,
                                             _I32, _D, _D, _D]
        L.sdem_spawn_status.argtypes = [_VP, C.POINTER(C.c_int64), C.POINTER(C.c_uint64),
                                        C.POINTER(C.c_double)]
        L.sdem_set_history.argtypes = [_VP, C.c_int64, _I32, _I32, _D, _D, _D]
        L.sdem_step.argtypes = [_VP, C.c_int64]
        L.sdem_step_profiled.argtypes = [_VP, C.c_int64, _D]
        L.sdem_read_state.argtypes = [_VP, _VP, _VP, _VP, _VP, _VP, _VP]
        L.sdem_read_contacts.argtypes = [_VP, C.c_int64, _I64, _VP, _VP, _VP, _VP, _VP]
        L.sdem_stats.argtypes = [_VP, _I64, _I64, _I64, _I64]
        L.sdem_destroy.argtypes = [_VP]
        L.sdem_last_error.restype = C.c_char_p
        L.sdem_last_error.argtypes = []
        L.sdem_selftest_rounding.argtypes = [C.c_int64, _VP, _VP, _VP, _VP]
        L.sdem_copy_probe.argtypes = [_VP, _VP, C.c_int64, C.c_int32, _VP, C.POINTER(C.c_double)]
        L.sdem_graph_stats.argtypes = [_VP, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
        _lib = L
    return _lib


def _check(rc):
    if rc != SDEM_OK:
        raise SdemError(rc, lib().sdem_last_error().decode())


def make_params(d: dict) -> Params:
    g = d.get("g", (0.0, 0.0, -9.81))
    om = d.get("mesh_omega", (0.0, 0.0, 0.0))
    ce = d.get("mesh_center", (0.0, 0.0, 0.0))
    mu_s = d.get("mu_s", 0.3)
    return Params(d.get("rho", 1e3), d.get("E", 1e6), d.get("nu", 0.3), d.get("e_n", 0.5), mu_s,
                  d.get("mu_r", 0.3), d.get("mu_t", 2.0 * mu_s / 3.0), d.get("eta", 0.0),
                  (C.c_double * 3)(*g), d["dt"], (C.c_double * 3)(*om), (C.c_double * 3)(*ce))


def selftest_rounding(a, b, device="cuda:0"):
    """Device sqrt(a) and a/b (float64 arrays) through the C ABI."""
    import torch
    ta = torch.as_tensor(np.ascontiguousarray(a, np.float64), device=device)
    tb = torch.as_tensor(np.ascontiguousarray(b, np.float64), device=device)
    out = torch.empty(2 * len(a), dtype=torch.float64, device=device)
    stream = torch.cuda.current_stream(device)
    _check(lib().sdem_selftest_rounding(len(a), ta.data_ptr(), tb.data_ptr(), out.data_ptr(),
                                        stream.cuda_stream))
    o = out.cpu().numpy()
    return o[: len(a)], o[len(a):]


def copy_probe(src, dst, reps=10):
    """Mean milliseconds per copy of the library's streaming copy kernel from
    device tensor src to dst (same size, a multiple of 16 bytes), through the
    C ABI, on the current stream."""
    import torch
    if src.device != dst.device or src.nbytes != dst.nbytes:
        raise ValueError("src and dst must be device tensors of equal size")
    ms = C.c_double()
    stream = torch.cuda.current_stream(src.device)
    _check(lib().sdem_copy_probe(src.data_ptr(), dst.data_ptr(), src.nbytes, int(reps),
                                 stream.cuda_stream, C.byref(ms)))
    return ms.value


def _grid_cells(x, h):
    if len(x) == 0 or not np.all(np.isfinite(x)):
        return max(1, len(x))
    ext = x.max(0) - x.min(0)
    return int(np.prod(np.floor(ext / h) + 1))


def autotune(sims, candidates=None, steps=20, warmup=6, precision="fp64", device="cuda:0",
             **kw):
    """Picks the cell edge factor, the number of lanes per particle in the
    contact search, the skin and the longest rebuild period by timing a few
    steps of each candidate (cell_factor, detect_lanes[, skin[,
    rebuild_every]]) on the given workload (each trial runs on its own copy of
    the state; a trial should span several rebuild periods).  Returns (best,
    timings) with best = {"cell_factor", "detect_lanes", "skin",
    "rebuild_every", "ms_per_step"}."""
    import time

    import torch
    if candidates is None:
        candidates = [(1.0, 1), (1.0, 2), (0.7, 1), (0.5, 1), (0.5, 2), (0.4, 1), (0.33, 1)]
    timings = []
    for cand in candidates:
        cf, lanes = cand[0], cand[1]
        skin = cand[2] if len(cand) > 2 else kw.get("skin", 0.0)
        every = cand[3] if len(cand) > 3 else kw.get("rebuild_every", 0)
        opts = dict(kw)
        opts["skin"] = skin
        opts["rebuild_every"] = every
        s = Solver(sims, precision=precision, device=device, cell_factor=cf, detect_lanes=lanes,
                   **opts)
        s.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        s.close()
        del s
        timings.append({"cell_factor": cf, "detect_lanes": lanes, "skin": skin,
                        "rebuild_every": every, "ms_per_step": ms})
    best = min(timings, key=lambda r: r["ms_per_step"])
    return dict(best), timings


def pack_elements(elements):
    """(nverts [m] int32, verts [m][4][3] float64) for sdem_add_mesh_elements
    from a list of mesh elements, each an array of 1..4 vertices (point,
    segment, triangle, rectangle with corners in cyclic order)."""
    m = len(elements)
    nv = np.zeros(m, np.int32)
    verts = np.zeros((m, 4, 3))
    for k, e in enumerate(elements):
        e = np.asarray(e, np.float64).reshape(-1, 3)
        nv[k] = len(e)
        verts[k, :len(e)] = e
    return nv, verts


def read_off(path, radii=(0.0,)):
    """Mesh elements from an OFF file (faces of 1..4 vertices, a trailing
    index into ``radii`` per face): (list of vertex arrays, radii [m])."""
    L = lib()
    r = np.ascontiguousarray(radii, np.float64).reshape(-1)
    m = C.c_int64()
    _check(L.sdem_read_off(os.fsencode(path), len(r), r.ctypes.data_as(_D), 0, C.byref(m), None,
                           None, None))
    nv = np.zeros(max(m.value, 1), np.int32)
    verts = np.zeros((max(m.value, 1), 4, 3))
    rm = np.zeros(max(m.value, 1))
    _check(L.sdem_read_off(os.fsencode(path), len(r), r.ctypes.data_as(_D), m.value, C.byref(m),
                           nv.ctypes.data_as(_I32), verts.ctypes.data_as(_D),
                           rm.ctypes.data_as(_D)))
    return [verts[k, :nv[k]].copy() for k in range(m.value)], rm[:m.value].copy()


def read_csv(path):
    """Particle state from a CSV file (header row, columns by name): dict of
    x, v, w (n, 3), q (n, 4), R (n)."""
    L = lib()
    n = C.c_int64()
    _check(L.sdem_read_csv(os.fsencode(path), 0, C.byref(n), None, None, None, None, None))
    k = n.value
    a = {key: np.zeros((w, max(k, 1))) for key, w in (("x", 3), ("v", 3), ("w", 3), ("q", 4))}
    R = np.zeros(max(k, 1))
    _check(L.sdem_read_csv(os.fsencode(path), k, C.byref(n), *[a[key].ctypes.data_as(_D)
                                                                for key in ("x", "v", "w", "q")],
                           R.ctypes.data_as(_D)))
    out = {key: np.ascontiguousarray(val[:, :k].T) for key, val in a.items()}
    out["R"] = R[:k].copy()
    return out


def read_contacts_csv(path):
    """Contact keys and springs from a CSV file written by
    Solver.write_contacts_csv: dict of ki, kj, us, ur, ut."""
    L = lib()
    n = C.c_int64()
    _check(L.sdem_read_contacts_csv(os.fsencode(path), 0, C.byref(n), None, None, None, None,
                                    None))
    k = max(n.value, 1)
    ki, kj = np.zeros(k, np.int32), np.zeros(k, np.int32)
    us, ur, ut = np.zeros((k, 3)), np.zeros((k, 3)), np.zeros(k)
    _check(L.sdem_read_contacts_csv(os.fsencode(path), n.value, C.byref(n),
                                    ki.ctypes.data_as(_I32), kj.ctypes.data_as(_I32),
                                    us.ctypes.data_as(_D), ur.ctypes.data_as(_D),
                                    ut.ctypes.data_as(_D)))
    m = n.value
    return {"ki": ki[:m], "kj": kj[:m], "us": us[:m], "ur": ur[:m], "ut": ut[:m]}


def _mesh_count(s):
    return len(s["elements"]) if s.get("elements") is not None else len(s.get("tri", ()))


class Solver:
    """One context of the HIP solver holding one or several simulations.

    ``sims`` is one workload dict or a list of them (see ``workloads``).  The
    state lives on ``device`` for the lifetime of the object.
    """

    def __init__(self, sims, precision="fp64", device="cuda:0", contacts_max=None,
                 cells_max=None, cell_factor=1.0, block=0, cell_slack=8.0, detect_lanes=0,
                 skin=0.0, rebuild_every=0, spawn=None, contacts_per_particle=0,
                 static_scratch=False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("sdem needs a GPU: torch.cuda.is_available() is False")
        L = lib()
        if isinstance(sims, dict):
            sims = [sims]
        self.sims = sims
        self.device = torch.device(device)
        self.nsims = len(sims)
        counts = [len(s["R"]) for s in sims]
        self.offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
        n = int(self.offsets[-1])
        self.n = n
        ntri = sum(_mesh_count(s) for s in sims)
        x = np.concatenate([s["x"] for s in sims]) if n else np.zeros((0, 3))
        self._spawn = spawn
        n_cap = n
        if spawn is not None:
            if self.nsims != 1:
                raise ValueError("spawning needs one simulation per solver")
            n_cap = max(n, int(spawn.get("n_max", 1000)))
        if cells_max is None:
            est = 0
            for s in sims:
                pts, rmax = [s["x"]], float(np.max(s["R"])) if len(s["R"]) else 0.0
                if spawn is not None:
                    # particles will fill the spawn box and whatever the mesh holds
                    pts.append(np.array([spawn["smin"], spawn["smax"]], float))
                    rmax = max(rmax, float(spawn["Rmax"]))
                    if s.get("elements") is not None:
                        pts.append(np.concatenate([np.asarray(e, float).reshape(-1, 3)
                                                   for e in s["elements"]]))
                    elif len(s.get("tri", ())):
                        pts.append(np.asarray(s["tri"], float).reshape(-1, 3))
                h = cell_factor * 2.0 * rmax if rmax > 0 else 1.0
                est += _grid_cells(np.concatenate(pts), h)
            cells_max = int(max(1024, cell_slack * est, 2 * n_cap))
        if contacts_max is None:
            contacts_max = int(max(4096, 8 * n_cap))
        self.cfg = Config(max(n_cap, 1), contacts_max, cells_max, max(ntri, 1), self.nsims,
                          SDEM_MIXED if precision == "mixed" else SDEM_FP64, block,
                          int(detect_lanes), float(cell_factor), float(skin),
                          int(rebuild_every), int(contacts_per_particle))
        nbytes = L.sdem_workspace_bytes(C.byref(self.cfg))
        if nbytes == 0:
            _check(SDEM_EINVAL)
        if static_scratch:
            # the library's own device scratch (sdem_init_static): no workspace
            if self.nsims != 1:
                raise ValueError("the static scratch holds one simulation")
            self.workspace = None
        else:
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.Stream(device=self.device)

        def soa(key, k):
            a = np.concatenate([s[key] for s in sims]) if n else np.zeros((0, k))
            return torch.as_tensor(np.ascontiguousarray(a.T), device=self.device)

        tx, tv, tw, tq = soa("x", 3), soa("v", 3), soa("w", 3), soa("q", 4)
        tR = torch.as_tensor(np.concatenate([s["R"] for s in sims]) if n else np.zeros(0),
                             device=self.device)
        params = (Params * self.nsims)(*[make_params(s["params"]) for s in sims])
        torch.cuda.synchronize(self.device)
        h = _VP()
        if static_scratch:
            _check(L.sdem_init_static(C.byref(h), C.byref(self.cfg), params, n, tx.data_ptr(),
                                      tv.data_ptr(), tw.data_ptr(), tq.data_ptr(), tR.data_ptr(),
                                      self.stream.cuda_stream))
        else:
            _check(L.sdem_init_batch(C.byref(h), C.byref(self.cfg), self.nsims, params,
                                     self.offsets.ctypes.data_as(_I64), tx.data_ptr(),
                                     tv.data_ptr(), tw.data_ptr(), tq.data_ptr(), tR.data_ptr(),
                                     self.workspace.data_ptr(), nbytes, self.stream.cuda_stream))
        self._h = h
        for k, s in enumerate(sims):
            if s.get("elements") is not None:
                if len(s.get("tri", ())):
                    raise ValueError("a simulation gives either 'tri' or 'elements'")
                nv, verts = pack_elements(s["elements"])
                rm = np.ascontiguousarray(s.get("rmesh", np.zeros(len(nv))), np.float64)
                _check(L.sdem_add_mesh_elements(h, k, len(nv), nv.ctypes.data_as(_I32),
                                                verts.ctypes.data_as(_D), rm.ctypes.data_as(_D)))
            elif len(s.get("tri", ())):
                tri = np.ascontiguousarray(s["tri"], np.float64).reshape(-1, 9)
                rm = np.ascontiguousarray(s.get("rmesh", np.zeros(len(tri))), np.float64)
                _check(L.sdem_add_mesh(h, k, len(tri), tri.ctypes.data_as(_D),
                                       rm.ctypes.data_as(_D)))
        for k, s in enumerate(sims):
            if s.get("motion") is not None:
                self.set_mesh_motion(k, s["motion"], s.get("motion_groups"))
        if spawn is not None:
            self.set_spawn(**spawn)

    # ---------------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().sdem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, nsteps=1):
        _check(lib().sdem_step(self._h, int(nsteps)))
        if self._spawn is not None:
            self._refresh_n()

    def _refresh_n(self):
        m = C.c_int64()
        _check(lib().sdem_spawn_status(self._h, C.byref(m), None, None))
        self.n = int(m.value)
        self.offsets = np.array([0, self.n], np.int64)

    def set_spawn(self, **kw):
        """Particle spawning (Section 3.1) with the keyword arguments of
        make_spawn; no arguments turn it off."""
        if kw:
            sp = make_spawn(**kw)
            _check(lib().sdem_set_spawn(self._h, 0, C.byref(sp)))
            self._spawn = dict(kw)
        else:
            _check(lib().sdem_set_spawn(self._h, 0, None))

    def set_mesh_motion(self, sim, motions, groups=None):
        """Motion groups of simulation sim's mesh: a list of dicts with the
        keywords of make_motion and the group of each element (None: all in
        group 0)."""
        arr = (MeshMotion * len(motions))(*[make_motion(**m) for m in motions])
        g = None if groups is None else np.ascontiguousarray(groups, np.int32)
        _check(lib().sdem_set_mesh_motion(self._h, int(sim), len(motions), arr,
                                          g.ctypes.data_as(_I32) if g is not None else None))

    def set_spawn_status(self, attempts, carried):
        _check(lib().sdem_set_spawn_status(self._h, int(attempts), float(carried)))

    def set_clock(self, steps):
        """Step counter (and moving-mesh clock t = steps dt), for a resume."""
        _check(lib().sdem_set_clock(self._h, int(steps)))

    def write_csv(self, path):
        _check(lib().sdem_write_csv(self._h, os.fsencode(path)))

    def write_contacts_csv(self, path):
        _check(lib().sdem_write_contacts_csv(self._h, os.fsencode(path)))

    def spawn_status(self):
        """(particle count, attempts made, radius carried over)."""
        m, a, r = C.c_int64(), C.c_uint64(), C.c_double()
        _check(lib().sdem_spawn_status(self._h, C.byref(m), C.byref(a), C.byref(r)))
        return int(m.value), int(a.value), float(r.value)

    def step_profiled(self, nsteps=1):
        """Steps without a graph, timing each phase with HIP events; returns
        the mean milliseconds per step of each phase."""
        ms = (C.c_double * len(PHASES))()
        _check(lib().sdem_step_profiled(self._h, int(nsteps), ms))
        if self._spawn is not None:
            self._refresh_n()
        return dict(zip(PHASES, list(ms)))

    def set_history(self, ki, kj, us, ur, ut):
        ki = np.ascontiguousarray(ki, np.int32)
        kj = np.ascontiguousarray(kj, np.int32)
        us = np.ascontiguousarray(us, np.float64).reshape(-1, 3)
        ur = np.ascontiguousarray(ur, np.float64).reshape(-1, 3)
        ut = np.ascontiguousarray(ut, np.float64)
        _check(lib().sdem_set_history(self._h, len(ki), ki.ctypes.data_as(_I32),
                                      kj.ctypes.data_as(_I32), us.ctypes.data_as(_D),
                                      ur.ctypes.data_as(_D), ut.ctypes.data_as(_D)))

    def state(self, forces=True):
        """State by persistent id as numpy: x, v, w (n,3), q (n,4), F, T."""
        n = self.n
        out = {k: np.empty((3, n)) for k in ("x", "v", "w", "F", "T")}
        out["q"] = np.empty((4, n))
        ptr = lambda k: out[k].ctypes.data if n else None
        _check(lib().sdem_read_state(self._h, ptr("x"), ptr("v"), ptr("w"), ptr("q"),
                                     ptr("F") if forces else None, ptr("T") if forces else None))
        return {k: np.ascontiguousarray(a.T) for k, a in out.items()}

    def radii(self):
        """Radii by persistent id (spawned particles included)."""
        out = np.empty(self.n)
        _check(lib().sdem_read_radii(self._h, out.ctypes.data if self.n else None))
        return out

    def contacts(self):
        """Contacts of the last step in key order, with their springs."""
        nout = C.c_int64(0)
        lib().sdem_read_contacts(self._h, 0, C.byref(nout), None, None, None, None, None)
        m = nout.value
        ki = np.zeros(max(m, 1), np.int32)
        kj = np.zeros(max(m, 1), np.int32)
        us = np.zeros((max(m, 1), 3))
        ur = np.zeros((max(m, 1), 3))
        ut = np.zeros(max(m, 1))
        _check(lib().sdem_read_contacts(self._h, m, C.byref(nout), ki.ctypes.data,
                                        kj.ctypes.data, us.ctypes.data, ur.ctypes.data,
                                        ut.ctypes.data))
        return {"ki": ki[:m], "kj": kj[:m], "us": us[:m], "ur": ur[:m], "ut": ut[:m]}

    def stats(self):
        s, pp, pw, rb = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().sdem_stats(self._h, C.byref(s), C.byref(pp), C.byref(pw), C.byref(rb)))
        return {"steps": s.value, "pp": pp.value, "pw": pw.value, "rebuilds": rb.value}

    def graph_stats(self):
        """HIP graphs instantiated so far, and whether capturing one failed."""
        made, failed = C.c_int64(), C.c_int32()
        _check(lib().sdem_graph_stats(self._h, C.byref(made), C.byref(failed)))
        return {"instantiated": made.value, "failed": bool(failed.value)}
