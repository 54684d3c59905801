"""Shared comparison helpers for the GPU parity tests (not collected)."""
import numpy as np

import oracle


def rel(a, b):
    """Normwise-max relative difference max|a-b| / max|b|."""
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.abs(b).max() if b.size else 0.0
    if den == 0.0:
        return float(np.abs(a).max()) if a.size else 0.0
    return float(np.abs(a - b).max() / den)


def rel_w(wg, wo, R, vo):
    """Angular velocity error: the larger of (a) the error as a surface speed,
    max|dw| R_max over max(max|v|, max|w| R_max), so rounding-level spins of
    particles that should not rotate are not compared against themselves,
    and (b) the plain normwise relative error over the particles whose
    surface speed |w| R_i is above 1e-6 of that scale (far above rounding)."""
    wg, wo = np.asarray(wg), np.asarray(wo)
    R = np.asarray(R, dtype=float)
    rmax = float(np.max(R)) if len(R) else 1.0
    den = max(float(np.abs(vo).max()) if np.size(vo) else 0.0,
              float(np.abs(wo).max()) * rmax if np.size(wo) else 0.0)
    if den == 0.0:
        return float(np.abs(wg).max()) * rmax if np.size(wg) else 0.0
    surface = float(np.abs(wg - wo).max() * rmax / den)
    spinning = np.linalg.norm(wo, axis=1) * R > 1e-6 * den
    plain = rel(wg[spinning], wo[spinning]) if spinning.any() else 0.0
    return max(surface, plain)


def force_err(Fg, Fo, scale):
    """Per-particle force error scaled by sum_c |contribution| + m|g|."""
    d = np.linalg.norm(np.asarray(Fg) - np.asarray(Fo), axis=1)
    s = np.maximum(np.asarray(scale), 1e-300)
    return float((d / s).max()) if len(d) else 0.0


def torque_err(Tg, To, Tscale, Fscale, R):
    """Per-particle torque error scaled by sum_c |torque| + (sum_c |force| +
    m|g|) R_i: a rounding error in a force direction shows up as a torque
    of that size even where the reference torques vanish."""
    d = np.linalg.norm(np.asarray(Tg) - np.asarray(To), axis=1)
    s = np.maximum(np.asarray(Tscale) + np.asarray(Fscale) * np.asarray(R), 1e-300)
    return float((d / s).max()) if len(d) else 0.0


def keys(c):
    return np.stack([c["ki"], c["kj"]], 1) if len(c["ki"]) else np.zeros((0, 2), np.int32)


def mesh_args(w):
    """Oracle mesh arguments of a workload: triangles, or mesh elements of
    one to four vertices."""
    if w.get("elements") is not None:
        return dict(elements=w["elements"], rmesh=w["rmesh"])
    if len(w["tri"]):
        return dict(tri=w["tri"], rmesh=w["rmesh"])
    return {}


def with_motion(o, w):
    """Applies a workload's mesh motion groups, if any, to an oracle run."""
    if w.get("motion") is not None:
        o.set_mesh_motion(w["motion"], w.get("motion_groups"))
    return o


def oracle_from(w):
    return with_motion(oracle.Sim(w["params"], w["x"], v=w["v"], w=w["w"], q=w["q"], R=w["R"],
                                  **mesh_args(w)), w)


def oracle_resync(w, st, c, t):
    """Oracle started from a GPU state and GPU springs at time t."""
    o = with_motion(oracle.Sim(w["params"], st["x"], v=st["v"], w=st["w"], q=st["q"], R=w["R"],
                               **mesh_args(w)), w)
    o.set_time(t)
    if len(c["ki"]):
        o.set_history(c["ki"], c["kj"], c["us"], c["ur"], c["ut"])
    return o


def spring_err(cg, co):
    """Springs matched by key (keys must already be equal)."""
    out = {}
    for k in ("us", "ur"):
        out[k] = rel(cg[k], co[k])
    out["ut"] = rel(cg["ut"], co["ut"])
    return out


def keys_per_particle(c, idx):
    """Keys of the contacts (ki, kj arrays in key order) that each listed
    particle takes part in, one particle after another: (ki, kj, counts)."""
    ki, kj = np.asarray(c["ki"]), np.asarray(c["kj"])
    idx = np.asarray(idx)
    sel = np.isin(ki, idx) | ((kj > 0) & np.isin(kj, idx))
    ks, js = ki[sel], kj[sel]
    oi, oj, cnt = [], [], []
    for p in idx:
        m = (ks == p) | ((js > 0) & (js == p))
        oi.append(ks[m])
        oj.append(js[m])
        cnt.append(int(m.sum()))
    cat = (lambda a: np.concatenate(a) if a else np.zeros(0, np.int32))
    return cat(oi), cat(oj), np.array(cnt, np.int64)


def sampled_errors(g, w, st, hist, t, idx):
    """Steps the GPU context g once from the state st / springs hist it holds
    at time t, and checks the listed particles against the oracle's sampled
    step from the same point: returns (keys equal, contacts of the sample,
    dict of per-quantity errors)."""
    o = oracle_resync(w, st, hist, t)
    oki, okj, ocnt = o.sample_keys(idx)
    smp = o.sample_step(idx)
    g.step(1)
    sg, cg = g.state(), g.contacts()
    gki, gkj, gcnt = keys_per_particle(cg, idx)
    same = (np.array_equal(ocnt, gcnt) and np.array_equal(oki, gki) and np.array_equal(okj, gkj))
    R = w["R"][idx]
    err = {
        "F": force_err(sg["F"][idx], smp["F"], smp["Fscale"]),
        "T": torque_err(sg["T"][idx], smp["T"], smp["Tscale"], smp["Fscale"], R),
        "x": rel(sg["x"][idx], smp["x"]),
        "v": rel(sg["v"][idx], smp["v"]),
        "q": rel(sg["q"][idx], smp["q"]),
        "w": rel_w(sg["w"][idx], smp["w"], R, smp["v"]),
    }
    return same, int(ocnt.sum()), err
