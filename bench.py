#!/usr/bin/env python3
"""Throughput of the DEM hot path on one MI355X.

Workload (default): the dense static packing of 8,000,000 spheres (half of
radius 1.4 mm, half 1.0 mm, body-centred, pre-compressed, eleven contacts
per sphere, about 44M contacts per step) in force balance in a closed
12-triangle box, full friction, dt from Eq. dt at 1.0 mm, plain FP64: the
largest single-GPU configuration, whose state is far larger than the 256 MB
Infinity Cache.  A step is one full time step of the hot path: bounding box
and grid, cell sort and state reorder (on the steps that rebuild the
cells), narrow phase, contact forces with spring carry-over, integration.
The state is resident in HBM before timing starts.

Timing: after --warmup steps, exactly --steps consecutive steps (default:
the workload's whole run, 10,000 relaxation steps for the packing) in one
window bracketed by device synchronisations, rebuilds of the cells
included at their real rate; value = particles x steps / seconds.

Prints one JSON line: particle-steps/s (value) and contacts/s; the roofline
of the step kernel (narrow phase, contact law, integration: 264 N + 120 C
algorithmic bytes per launch, 264 N + 68 C in mixed precision) over its mean duration from HIP events on its
own dispatch; other forms
(mixed precision, cells rebuilt every step, the 200,000-sphere column, the
2,000,000-sphere rotating drum, 256 batched box drops) with their speedups
over plain FP64 on the same GPU; and the CPU oracle timed on the same 8M
workload.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s & contacts/s: FP32/batched vs plain FP64 at stated tolerance"
HBM_PEAK_GBS = 8000.0


def step_bytes(n, c, mixed=False):
    """Algorithmic HBM bytes of one launch of the step kernel on a step that
    keeps the cells (narrow phase, contact law with spring carry-over, sums
    and integration in one kernel): the contact-force kernel's 128 N + 120 C
    (x, v, w, R read, F and T written; per contact the pair and the seven
    spring doubles read and written) plus the integration's 264 N (state and
    F, T read, state written), less what one kernel does not move twice:
    F and T read back (48 N) and x, v, w, R read again (80 N).  That is
    264 N + 120 C: the state read (112 B) and written (104 B), F and T
    written (48 B) per particle, 120 B per contact.  The mixed path keeps the
    springs as floats between steps: 8 + 28 B read and 8 + 24 B written per
    contact, 264 N + 68 C."""
    return 264.0 * n + (68.0 if mixed else 120.0) * c


def step_bytes_formula(mixed=False):
    return "264 N + 68 C" if mixed else "264 N + 120 C"


# bench workloads, each with its counter summary and its settings when none
# are given (None: autotuned)
WORKLOADS = {
    "packing_8M": {"make": "cfg5",
                   "radii": "half 1.4 mm, half 1.0 mm (body-centred arrangement)",
                   "traffic": "k_step_cfg5_packing_8M_hbm_traffic.md",
                   "traffic_mixed": "k_step_cfg5_packing_8M_mixed_hbm_traffic.md",
                   "settings": (1.0, 1, 0.2, 256)},
    "column_200k": {"make": "cfg2", "radii": "lognormal, median 1 mm, sigma 0.2",
                    "traffic": "k_step_cfg2_column_200k_hbm_traffic.md", "settings": None},
}


def host_info():
    """The host the CPU oracle runs on: logical CPUs visible to this process,
    the CPU model and the OpenMP thread setting."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"nproc": avail, "cpu_count": os.cpu_count(), "model": model,
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}


def measured_traffic(workload, precision="fp64"):
    """HBM bytes per step-kernel launch from the committed counter summary of
    that workload and precision (FETCH_SIZE and WRITE_SIZE scaled by a copy of
    known size), or None when there is none or the kernel source changed
    since those counters were taken."""
    import hashlib
    name = WORKLOADS[workload].get("traffic" if precision == "fp64" else "traffic_mixed")
    if name is None:
        return None
    try:
        text = open(os.path.join(ROOT, "profiles", name)).read()
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in text.splitlines() if ": " in line and
                  line.split(": ", 1)[0] in ("traffic_bytes_per_launch", "kernel_source_sha256_16"))
    src = b"".join(open(os.path.join(ROOT, "paper_2507_12610_amd", "csrc", f), "rb").read()
                   for f in ("kernels.hip", "sdem_internal.h"))
    if hashlib.sha256(src).hexdigest()[:16] != fields.get("kernel_source_sha256_16", "").strip():
        return None
    return float(fields["traffic_bytes_per_launch"])


def cpu_baseline(w, steps=4, what="the same workload"):
    """The serial FP64 oracle (one host thread) on workload w: `steps` steps
    from its start, wall time per step; the value is the median rate of the
    steps after the first (which also builds the oracle's tables)."""
    import oracle
    o = oracle.Sim(w["params"], w["x"], v=w["v"], w=w["w"], q=w["q"], R=w["R"],
                   tri=w["tri"], rmesh=w["rmesh"])
    per = []
    for _ in range(steps):
        t0 = time.perf_counter()
        o.step(1)
        per.append(time.perf_counter() - t0)
    n = len(w["R"])
    timed = per[1:] if len(per) > 1 else per
    return {"value": n / statistics.median(timed), "unit": "particle-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{what} (N={n}): {steps} steps from its start, serial FP64 oracle in one "
                      f"thread; median of the steps after the first; "
                      + ", ".join(f"{t:.2f}" for t in per) + " s per step",
            "host": host_info()}


def timed_run(s, n, K, chunk=1000):
    """Times K consecutive steps of solver s as one window on the host clock
    between device synchronisations (the host schedule runs in calls of at
    most `chunk` steps, each printing a progress line): ms per step,
    contacts, rebuilds, and ms per step of each call."""
    import torch
    a = s.stats()
    per = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < K:
        k = min(chunk, K - done)
        t1 = time.perf_counter()
        s.step(k)  # returns after the stream has drained
        per.append(round(1e3 * (time.perf_counter() - t1) / k, 5))
        done += k
        if K > chunk:
            print(f"[bench]   {done}/{K} steps, {per[-1]:.3f} ms/step", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    b = s.stats()
    c = (b["pp"] - a["pp"]) + (b["pw"] - a["pw"])
    return {"s": sec, "ms_per_step": round(1e3 * sec / K, 5),
            "particle_steps_per_s": round(n * K / sec, 1),
            "contacts_per_s": round(c / sec, 1), "contacts_per_step": round(c / K, 1),
            "cell_rebuilds": f"{b['rebuilds'] - a['rebuilds']} of {K} steps",
            "chunk_steps": chunk, "chunks_ms_per_step": per}


def timed_blocks(s, n, K, blocks=3, min_block_steps=128):
    """Times `blocks` blocks of consecutive steps of solver s.  A block is a
    run of windows of exactly K steps, each window bracketed by device
    synchronisations and timed on the host clock; a block spans at least
    min_block_steps steps so that it holds whole rebuild periods.  Returns
    the median block (by rate) and all blocks: steps, seconds, rebuilds,
    contacts."""
    import torch
    out = []
    per_block = max(1, -(-min_block_steps // K))
    for _ in range(blocks):
        a = s.stats()
        sec = 0.0
        for _ in range(per_block):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.step(K)  # returns after the stream has drained
            torch.cuda.synchronize()
            sec += time.perf_counter() - t0
        b = s.stats()
        out.append({"steps": per_block * K, "s": sec, "rebuilds": b["rebuilds"] - a["rebuilds"],
                    "pp": b["pp"] - a["pp"], "pw": b["pw"] - a["pw"]})
    med = sorted(out, key=lambda r: r["steps"] / r["s"])[len(out) // 2]
    return med, out


def block_summary(med, blocks, n):
    return {"ms_per_step": round(1e3 * med["s"] / med["steps"], 5),
            "particle_steps_per_s": round(n * med["steps"] / med["s"], 1),
            "contacts_per_s": round((med["pp"] + med["pw"]) / med["s"], 1),
            "contacts_per_step": round((med["pp"] + med["pw"]) / med["steps"], 1),
            "cell_rebuilds": f"{med['rebuilds']} of {med['steps']} steps",
            "blocks_ms_per_step": [round(1e3 * b["s"] / b["steps"], 5) for b in blocks]}


def profiled_step_kernel(s, n, steps):
    """Phase times over `steps` profiled steps (one at a time) and the mean
    duration of the step kernel on the steps that keep the cells, from
    start/stop events attached to its dispatch; with the algorithmic bytes
    per launch over that duration against the HBM peak."""
    prof = []
    for _ in range(steps):
        a = s.stats()
        ph = s.step_profiled(1)
        b = s.stats()
        prof.append((b["rebuilds"] > a["rebuilds"], ph, (b["pp"] - a["pp"]) + (b["pw"] - a["pw"])))
    keep = [p for p in prof if not p[0]] or prof
    phases = {k: sum(p[1][k] for p in prof) / len(prof) for k in prof[0][1]}
    fms = sum(p[1]["step_kernel"] for p in keep) / len(keep)
    c_prof = sum(p[2] for p in keep) / len(keep)
    from paper_2507_12610_amd.sdem import SDEM_MIXED
    mixed = s.cfg.precision == SDEM_MIXED
    alg = step_bytes(n, c_prof, mixed)
    achieved = alg / (fms * 1e-3) / 1e9
    dominant = max((k for k in phases if k != "step_kernel"), key=phases.get)
    return {"kernel": "k_step (narrow phase, contact law with spring carry-over, integration)",
            "bound": "hbm", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "mean_ms": round(fms, 5), "algorithmic_bytes": alg,
            "algorithmic_bytes_formula": step_bytes_formula(mixed),
            "contacts_per_launch": round(c_prof, 1), "launches_timed": len(keep),
            "phase_ms": {k: round(v, 5) for k, v in phases.items() if k != "step_kernel"},
            "dominant_phase": dominant}


def rel(a, b):
    import numpy as np
    den = float(np.abs(b).max()) if np.size(b) else 0.0
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a).max())


def sim_slice(w, st, c, lo, hi):
    """Workload dict of particles [lo, hi) of a batched state, with its contacts
    (keys made local) for sdem_set_history."""
    d = dict(w)
    d.update(x=st["x"][lo:hi].copy(), v=st["v"][lo:hi].copy(), w=st["w"][lo:hi].copy(),
             q=st["q"][lo:hi].copy())
    m = (c["ki"] >= lo) & (c["ki"] < hi)
    kj = c["kj"][m]
    hist = (c["ki"][m] - lo, kj.copy(), c["us"][m], c["ur"][m], c["ut"][m])
    hist[1][kj > 0] -= lo
    return d, hist


def mixed_vs_fp64(w, opts, steps_before=200):
    """One step of the mixed path and of the FP64 path from the same state
    and springs (taken after steps_before FP64 steps): per quantity, the
    largest difference relative to the largest FP64 value (for x, relative
    to the largest displacement of the step)."""
    from paper_2507_12610_amd import Solver
    a = Solver(w, precision="fp64", **opts)
    a.step(steps_before)
    st, c = a.state(forces=False), a.contacts()
    d = dict(w)
    d.update({k: st[k] for k in ("x", "v", "w", "q")})
    b = Solver(d, precision="mixed", **opts)
    b.set_history(c["ki"], c["kj"], c["us"], c["ur"], c["ut"])
    b.set_clock(steps_before)
    a.step(1)
    b.step(1)
    sa, sb = a.state(), b.state()
    a.close()
    b.close()
    out = {k: rel(sb[k], sa[k]) for k in ("F", "T", "v", "w", "q")}
    out["x"] = rel(sb["x"] - st["x"], sa["x"] - st["x"])
    return {"after_fp64_steps": steps_before, "contacts": int(len(c["ki"])),
            "max_rel_diff": {k: float(f"{v:.3e}") for k, v in out.items()}}


# (cell_factor, detect_lanes, skin, longest rebuild period) tried by the
# autotuner on the column (0: the library's 64 steps)
TUNE_CANDIDATES = [(0.4, 1, 0.05, 0), (0.33, 1, 0.05, 0), (0.5, 1, 0.05, 0), (1.0, 1, 0.1, 128),
                   (0.4, 1, 0.1, 128), (0.4, 1, 0.1, 256), (0.33, 1, 0.1, 256), (0.5, 1, 0.1, 256),
                   (0.4, 1, 0.2, 256), (0.4, 1, 0.0, 0)]


# (cell_factor, detect_lanes, skin) tried for the 256 box drops (bouncier than the column)
BATCH_CANDIDATES = [(1.0, 1, 1.0), (0.7, 1, 1.0), (1.0, 1, 0.6), (0.7, 1, 0.6), (1.0, 1, 0.3),
                    (1.0, 1, 0.0)]


def column_forms(K):
    """The 200,000-sphere column (configuration 2): FP64 and mixed precision
    with autotuned settings."""
    import workloads as W
    from paper_2507_12610_amd import Solver, autotune
    w = W.cfg2()
    n = len(w["R"])
    print(f"[bench] column: {n} particles", file=sys.stderr, flush=True)
    best, _ = autotune(w, candidates=TUNE_CANDIDATES, steps=512, warmup=10)
    cf, lanes, skin, every = (best["cell_factor"], best["detect_lanes"], best["skin"],
                              best["rebuild_every"])
    out = {"workload": w["name"], "particles": n, "settings": {
        "cell_factor": cf, "detect_lanes": lanes, "skin": skin,
        "rebuild_every": every if every > 0 else 64}}
    for prec in ("fp64", "mixed"):
        s = Solver(w, precision=prec, cell_factor=cf, detect_lanes=lanes, skin=skin,
                   rebuild_every=every)
        s.step(50)
        med, blocks = timed_blocks(s, n, K, min_block_steps=2 * max(every, 64))
        out[prec] = block_summary(med, blocks, n)
        s.close()
    out["mixed_speedup_vs_fp64"] = round(out["fp64"]["ms_per_step"] / out["mixed"]["ms_per_step"], 4)
    return out


def drum_forms(K, sample=3000):
    """The 2,000,000-sphere rotating drum (configuration 3, 8,192 triangles,
    1 rad/s), FP64 and mixed precision after the bed has landed: ms/step,
    contacts/s and the contact-force kernel's roofline; the mixed path's
    difference per quantity from the FP64 path after 1 and 20 steps from the
    same state, and the error of each path against the FP64 oracle re-synced
    to its own state (one step of `sample` sampled particles, half of them in
    contact) at the first and the twentieth of those steps."""
    import numpy as np

    import oracle
    import workloads as W
    from paper_2507_12610_amd import Solver
    w = W.cfg3()
    n = len(w["R"])
    print(f"[bench] drum: {n} particles, {len(w['tri'])} triangles", file=sys.stderr, flush=True)
    # skin 0.6 R_max: fewer rebuilds of the turning bed (0.2: 0.45 ms/step,
    # 0.4: 0.41, 0.6: 0.40, 1.0: 0.52 over 400 steps after landing)
    opts = dict(cell_factor=1.0, detect_lanes=1, skin=0.6)
    land = Solver(w, precision="fp64", **opts)
    land.step(300)
    st0, c0 = land.state(forces=False), land.contacts()
    t_land = 300 * w["params"]["dt"]
    land.close()
    d = dict(w)
    d.update({k: st0[k] for k in ("x", "v", "w", "q")})
    out = {"workload": w["name"], "particles": n, "triangles": len(w["tri"]),
           "landing_steps": 300, "settings": opts}
    for prec in ("fp64", "mixed"):
        s = Solver(d, precision=prec, **opts)
        s.set_history(c0["ki"], c0["kj"], c0["us"], c0["ur"], c0["ut"])
        s.set_clock(300)
        s.step(20)
        med, blocks = timed_blocks(s, n, K, min_block_steps=128)
        out[prec] = block_summary(med, blocks, n)
        out[prec]["roofline"] = profiled_step_kernel(s, n, 12)
        s.close()
    out["mixed_speedup_vs_fp64"] = round(out["fp64"]["ms_per_step"] / out["mixed"]["ms_per_step"], 4)

    # per-quantity differences, mixed against FP64, from the landed state
    runs = {}
    for prec in ("fp64", "mixed"):
        s = Solver(d, precision=prec, **opts)
        s.set_history(c0["ki"], c0["kj"], c0["us"], c0["ur"], c0["ut"])
        s.set_clock(300)
        snaps = {}
        s.step(1)
        snaps[1] = (s.state(), s.contacts())
        s.step(18)
        snaps[19] = (s.state(forces=False), s.contacts())
        s.step(1)
        snaps[20] = (s.state(), s.contacts())
        runs[prec] = snaps
        s.close()
    diff = {}
    for h in (1, 20):
        a, b = runs["fp64"][h][0], runs["mixed"][h][0]
        dd = {k: rel(b[k], a[k]) for k in ("F", "T", "v", "w", "q")}
        dd["x"] = rel(b["x"] - st0["x"], a["x"] - st0["x"])
        ca, cb = runs["fp64"][h][1], runs["mixed"][h][1]
        same = (len(ca["ki"]) == len(cb["ki"]) and np.array_equal(ca["ki"], cb["ki"]) and
                np.array_equal(ca["kj"], cb["kj"]))
        if same:
            dd["us"] = rel(cb["us"], ca["us"])
            dd["ur"] = rel(cb["ur"], ca["ur"])
            dd["ut"] = rel(cb["ut"], ca["ut"])
        diff[f"after_{h}_steps"] = {"same_contact_keys": bool(same),
                                    "max_rel_diff": {k: float(f"{v:.3e}") for k, v in dd.items()}}
    out["mixed_vs_fp64"] = diff

    # against the oracle: one sampled step from the GPU path's own state
    rng = np.random.Generator(np.random.PCG64(3030))
    touching = np.unique(np.concatenate([c0["ki"], c0["kj"][c0["kj"] > 0]]))
    idx = np.sort(np.concatenate([rng.choice(touching, sample // 2, replace=False),
                                  rng.choice(n, sample // 2, replace=False)]))
    idx = np.unique(idx)
    vs_oracle = {}
    for prec in ("fp64", "mixed"):
        for h in (1, 20):
            if h == 1:
                start, hist, t = st0, c0, t_land
            else:
                start, hist = runs[prec][19]
                t = t_land + 19 * w["params"]["dt"]
            o = oracle.Sim(w["params"], start["x"], v=start["v"], w=start["w"], q=start["q"],
                           R=w["R"], tri=w["tri"], rmesh=w["rmesh"])
            o.set_time(t)
            o.set_history(hist["ki"], hist["kj"], hist["us"], hist["ur"], hist["ut"])
            smp = o.sample_step(idx)
            g = runs[prec][h][0]
            scale_F = np.maximum(smp["Fscale"], 1e-300)
            errF = float((np.linalg.norm(g["F"][idx] - smp["F"], axis=1) / scale_F).max())
            errT = float((np.linalg.norm(g["T"][idx] - smp["T"], axis=1) /
                          np.maximum(smp["Tscale"] + smp["Fscale"] * w["R"][idx], 1e-300)).max())
            e = {"F": errF, "T": errT, "v": rel(g["v"][idx], smp["v"]),
                 "q": rel(g["q"][idx], smp["q"]),
                 "x": rel(g["x"][idx] - start["x"][idx], smp["x"] - start["x"][idx])}
            vs_oracle[f"{prec}_step_{h}"] = {k: float(f"{v:.3e}") for k, v in e.items()}
            del o
    out["vs_oracle_resynced_sampled"] = {"particles": int(len(idx)), "errors": vs_oracle,
                                        "tolerance": {"fp64": 1e-12, "mixed": 1e-5}}
    return out


def copy_ceiling(achieved_gbs, mib=1024, reps=20):
    """The HBM bandwidth of a plain streaming copy (the library's copy probe,
    `mib` MiB each way, mean of `reps` copies after one untimed): the
    practical ceiling, reported beside the published peak, with the step
    kernel's algorithmic bandwidth as a fraction of it."""
    import torch

    from paper_2507_12610_amd import copy_probe
    nb = mib << 20
    src = torch.ones(nb // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    ms = copy_probe(src, dst, reps)
    del src, dst
    gbs = 2.0 * nb / (ms * 1e-3) / 1e9
    return {"copy_ceiling": {"GB/s": round(gbs, 1), "bytes_moved_per_copy": 2 * nb,
                             "ms_per_copy": round(ms, 5), "kernel": "sdem_copy_probe"},
            "frac_of_copy_ceiling": round(achieved_gbs / gbs, 4)}


def kept_step_ms(s, windows=24):
    """Median wall time per step of `windows` calls of eight steps each on
    solver s, over the calls in which no step rebuilt the cells (None if
    every call rebuilt)."""
    import torch
    per = []
    for _ in range(windows):
        r0 = s.stats()["rebuilds"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(8)  # returns after the stream has drained
        dt = time.perf_counter() - t0
        if s.stats()["rebuilds"] == r0:
            per.append(1e3 * dt / 8)
    return round(statistics.median(per), 5) if per else None


def batched_forms(K, landing_steps, precision_list=("fp64", "mixed")):
    """Configuration 4: 256 box drops of uneven size in one context, timed after
    the sims have landed, against the same 256 states stepped one simulation
    after another (separate contexts, plain FP64), all on the GPU.  Every
    context has stepped (and so instantiated its step graphs) before timing;
    each form is the median of three blocks."""
    import torch

    import workloads as W
    from paper_2507_12610_amd import Solver, autotune
    sims = W.cfg4()
    total = sum(len(s["R"]) for s in sims)
    print(f"[bench] batched: {len(sims)} sims, {total} particles", file=sys.stderr, flush=True)
    b = Solver(sims, cell_factor=1.0, detect_lanes=1, skin=1.0)
    b.step(landing_steps)
    st, c = b.state(forces=False), b.contacts()
    b.close()
    landed = [sim_slice(sims[k], st, c, b.offsets[k], b.offsets[k + 1]) for k in range(len(sims))]
    # tuned on the landed state (the regime that is timed)
    best, _ = autotune([p[0] for p in landed], candidates=BATCH_CANDIDATES, steps=96, warmup=4)
    cf, skin = best["cell_factor"], best["skin"]
    out = {"workload": "cfg4_256_box_drops", "sims": len(sims), "particles": total,
           "landing_steps": landing_steps, "cell_factor": cf, "skin": skin}
    for prec in precision_list:
        g = Solver([p[0] for p in landed], precision=prec, cell_factor=cf, detect_lanes=1,
                   skin=skin)
        g.set_history(c["ki"], c["kj"], c["us"], c["ur"], c["ut"])
        g.step(4)
        med, blocks = timed_blocks(g, total, K, min_block_steps=96)
        out[prec] = block_summary(med, blocks, total)
        # wall time of windows of eight steps that all kept the cells (one
        # graph replay each), against the step kernel's own duration on such
        # steps: the difference is the launch and host time per step that a
        # persistent kernel could remove; the rest of a block's time per step
        # is its rebuilds
        out[prec]["kept_step_ms"] = kept_step_ms(g)
        rl = profiled_step_kernel(g, total, 12)
        out[prec]["step_kernel_ms"] = rl["mean_ms"]
        out[prec]["roofline"] = rl
        g.close()
    # the same 256 states, one simulation after another (plain FP64)
    seq = []
    for k in range(len(sims)):
        d, h = sim_slice(sims[k], st, c, b.offsets[k], b.offsets[k + 1])
        g = Solver(d, cell_factor=cf, detect_lanes=1, skin=skin)
        g.set_history(*h)
        seq.append(g)
    for g in seq:
        g.step(4)
    torch.cuda.synchronize()
    reps = []
    for _ in range(3):
        t0 = time.perf_counter()
        for g in seq:
            g.step(K)
        torch.cuda.synchronize()
        reps.append(time.perf_counter() - t0)
    for g in seq:
        g.close()
    dt = statistics.median(reps)
    out["sequential_fp64"] = {"ms_per_step": round(1e3 * dt / K, 5),
                              "particle_steps_per_s": round(total * K / dt, 1),
                              "repeats_ms_per_step": [round(1e3 * r / K, 5) for r in reps]}
    for prec in precision_list:
        out[prec]["speedup_vs_sequential_fp64"] = round(
            out["sequential_fp64"]["ms_per_step"] / out[prec]["ms_per_step"], 3)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: the workload's run, 10,000 steps for the packing)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--form-window", type=int, default=20,
                    help="steps per timed window of the other forms")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--cell-factor", type=float, default=None,
                    help="cell edge / (2 R_max); default: the workload's setting or autotuned")
    ap.add_argument("--detect-lanes", type=int, default=None,
                    help="lanes per particle in the contact search")
    ap.add_argument("--skin", type=float, default=None,
                    help="cell skin in units of R_max (0: rebuild every step)")
    ap.add_argument("--rebuild-every", type=int, default=None,
                    help="longest rebuild period with a skin (0: 64; default: the workload's)")
    ap.add_argument("--no-forms", action="store_true", help="skip the other forms")
    ap.add_argument("--forms", default="mixed,rebuilt,column,drum,batched",
                    help="comma-separated forms to run besides the headline")
    ap.add_argument("--batch-landing-steps", type=int, default=1500)
    ap.add_argument("--workload", choices=list(WORKLOADS), default="packing_8M")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run a plain device copy of this size (for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the library has "
              "no multi-GPU path (batched simulations would shard by simulation, one large "
              "system by slabs with halo exchange)", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W
    from paper_2507_12610_amd import Solver, autotune

    if args.copy_calibration_mib:
        # a plain copy of known size: FETCH_SIZE / WRITE_SIZE of this kernel
        # calibrate the counters read on the solver's kernels
        nb = args.copy_calibration_mib << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: 3 copies of {nb} bytes", file=sys.stderr, flush=True)
        del src, dst

    spec = WORKLOADS[args.workload]
    w = getattr(W, spec["make"])()
    n = len(w["R"])
    print(f"[bench] workload {w['name']}: N={n}, {len(w['tri'])} triangles", file=sys.stderr,
          flush=True)
    tuned = None
    if spec["settings"] is not None:
        fixed = spec["settings"]
        cf, lanes, skin = (fixed[0] if args.cell_factor is None else args.cell_factor,
                           fixed[1] if args.detect_lanes is None else args.detect_lanes,
                           fixed[2] if args.skin is None else args.skin)
        every = fixed[3] if args.rebuild_every is None else args.rebuild_every
    elif args.cell_factor is None or args.detect_lanes is None or args.skin is None:
        best, timings = autotune(w, candidates=TUNE_CANDIDATES, steps=512, warmup=10,
                                 precision=args.precision)
        tuned = {"chosen": best, "trials": timings}
        print(f"[bench] autotuned: {best}", file=sys.stderr, flush=True)
        cf, lanes, skin = best["cell_factor"], best["detect_lanes"], best["skin"]
        every = best["rebuild_every"]
    else:
        cf, lanes, skin = args.cell_factor, args.detect_lanes, args.skin
        every = args.rebuild_every or 0
    period = every if every > 0 else 64
    opts = dict(device="cuda:0", cell_factor=cf, detect_lanes=lanes, skin=skin,
                rebuild_every=every)
    K = w["steps"] if args.steps is None else args.steps
    s = Solver(w, precision=args.precision, **opts)
    s.step(args.warmup)
    graphs0 = s.graph_stats()
    if K >= 1000:
        run = timed_run(s, n, K)
        window = (f"steps {args.warmup + 1}-{args.warmup + K} of the run, one window on the host "
                  f"clock between device synchronisations")
    else:
        # a short window: the median of three consecutive ones
        med, blocks = timed_blocks(s, n, K, blocks=3, min_block_steps=K)
        run = dict(block_summary(med, blocks, n), s=med["s"], chunk_steps=K,
                   chunks_ms_per_step=[round(1e3 * b["s"] / b["steps"], 5) for b in blocks])
        window = (f"the median of three consecutive windows of {K} steps after step "
                  f"{args.warmup}, each on the host clock between device synchronisations")
    print(f"[bench] {K} steps in {run['s']:.3f} s, {run['contacts_per_step']:.0f} contacts/step",
          file=sys.stderr, flush=True)
    graphs1 = s.graph_stats()
    value = n * K / run["s"]
    # the state after exactly warmup + K steps, for the other precision's run
    end_state = s.state() if (K >= 1000 and not args.no_forms and "mixed" in args.forms) else None
    roofline = profiled_step_kernel(s, n, args.profile_steps)
    roofline["traffic"] = measured_traffic(args.workload, args.precision)
    s.close()
    del s
    roofline.update(copy_ceiling(roofline["achieved"]))

    out = {"metric": METRIC, "value": round(value, 1), "unit": "particle-steps/s", "n_gpus": 1,
           "steps": K, "warmup": args.warmup, "ms_per_step": run["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if args.precision == "fp64" else "f32+f64",
           "data": "synthetic",
           "config": {"workload": w["name"], "particles": n, "triangles": len(w["tri"]),
                      "dt": w["params"]["dt"], "precision": args.precision,
                      "radii": spec["radii"],
                      "friction": [w["params"]["mu_s"], w["params"]["mu_r"], w["params"]["mu_t"]],
                      "cell_factor": cf, "detect_lanes": lanes, "skin": skin,
                      "rebuild_every": period, "cell_rebuilds": run["cell_rebuilds"],
                      "run_steps": w["steps"]},
           "contacts_per_s": run["contacts_per_s"],
           "contacts_per_step": run["contacts_per_step"],
           "timing": {"window": window, "chunk_steps": run["chunk_steps"],
                      "chunks_ms_per_step": run["chunks_ms_per_step"],
                      "graphs_instantiated_before_window": graphs0["instantiated"],
                      "graphs_instantiated_in_window":
                          graphs1["instantiated"] - graphs0["instantiated"],
                      "graph_capture_failed": graphs1["failed"]},
           "roofline": roofline}
    if tuned is not None:
        out["autotune"] = tuned
    forms_wanted = set() if args.no_forms else set(f for f in args.forms.split(",") if f)
    forms = {}
    F = args.form_window
    if "mixed" in forms_wanted:
        # the other precision over the same run
        other = "mixed" if args.precision == "fp64" else "fp64"
        print(f"[bench] {other}: the same {K} steps", file=sys.stderr, flush=True)
        g = Solver(w, precision=other, **opts)
        g.step(args.warmup)
        end_diff = None
        if K >= 1000:
            r2 = timed_run(g, n, K)
            if end_state is not None:
                # the two precisions after the same whole run, free-running
                st2 = g.state()
                end_diff = {"after_steps": args.warmup + K, "max_rel_diff": {
                    k: round(rel(st2[k], end_state[k]), 10) for k in ("F", "T", "v", "w", "q")}}
                end_diff["max_rel_diff"]["x"] = round(
                    rel(st2["x"] - w["x"], end_state["x"] - w["x"]), 10)
                end_diff["note"] = ("free-running beyond the horizon of agreement: two FP64 runs "
                                    "one ulp apart differ by as much after this run; the "
                                    "tolerance applies to one step and short horizons")
                del st2
        else:
            m2, b2 = timed_blocks(g, n, K, blocks=3, min_block_steps=K)
            r2 = dict(block_summary(m2, b2, n), s=m2["s"])
        g.close()
        r2.pop("chunk_steps", None)
        forms[other] = dict(workload=w["name"], **r2,
                            tolerance=1e-5 if other == "mixed" else 1e-12)
        forms[other]["speedup_vs_" + args.precision] = round(
            run["ms_per_step"] / forms[other]["ms_per_step"], 4)
        forms["mixed_vs_fp64_one_step"] = mixed_vs_fp64(w, opts)
        if end_diff is not None:
            forms["mixed_vs_fp64_after_run"] = end_diff
    end_state = None
    if "rebuilt" in forms_wanted and skin > 0:
        # the paper's scheme, cells rebuilt every step, same workload
        print("[bench] cells rebuilt every step", file=sys.stderr, flush=True)
        g = Solver(w, precision=args.precision, **dict(opts, skin=0.0))
        g.step(5)
        m3, b3 = timed_blocks(g, n, F, min_block_steps=F)
        g.close()
        forms["cells_rebuilt_every_step"] = dict(workload=w["name"], **block_summary(m3, b3, n))
    if "column" in forms_wanted and args.workload != "column_200k":
        forms["column_200k"] = column_forms(F)
    if "drum" in forms_wanted:
        forms["drum_2M"] = drum_forms(F)
    if "batched" in forms_wanted:
        forms["batched"] = batched_forms(F, args.batch_landing_steps)
    if forms:
        out["forms"] = forms
    if not args.no_cpu:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        if args.workload == "packing_8M":
            # a bounded sample: the same packing in a box of 100^3 + 99^3 spheres
            ws = W.cfg5(dims=(100, 100, 100), n=None)
            out["cpu_baseline"] = cpu_baseline(
                ws, steps=args.cpu_steps,
                what="the same body-centred packing in a smaller box (100^3 large, 99^3 small)")
        else:
            out["cpu_baseline"] = cpu_baseline(w, steps=args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
