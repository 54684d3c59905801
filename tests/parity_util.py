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
    """Angular velocity error as a surface speed: max|dw| R_max over
    max(max|v|, max|w| R_max), so rounding-level spins of particles that
    should not rotate are not compared against themselves."""
    rmax = float(np.max(R)) if len(R) else 1.0
    den = max(float(np.abs(vo).max()) if np.size(vo) else 0.0,
              float(np.abs(wo).max()) * rmax if np.size(wo) else 0.0)
    if den == 0.0:
        return float(np.abs(wg).max()) * rmax if np.size(wg) else 0.0
    return float(np.abs(np.asarray(wg) - np.asarray(wo)).max() * rmax / den)


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


def oracle_from(w):
    return oracle.Sim(w["params"], w["x"], v=w["v"], w=w["w"], q=w["q"], R=w["R"],
                      tri=w["tri"] if len(w["tri"]) else None,
                      rmesh=w["rmesh"] if len(w["tri"]) else None)


def oracle_resync(w, st, c, t):
    """Oracle started from a GPU state and GPU springs at time t."""
    o = oracle.Sim(w["params"], st["x"], v=st["v"], w=st["w"], q=st["q"], R=w["R"],
                   tri=w["tri"] if len(w["tri"]) else None,
                   rmesh=w["rmesh"] if len(w["tri"]) else None)
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
