#!/usr/bin/env python3
"""Throughput of the DEM hot path on one MI355X.

Workload (default): 200,000 polydisperse spheres (R = 1 mm exp(0.2 Z)),
granular column on a 600 x 600 mm two-triangle floor, full friction,
dt = 5e-7 s, plain FP64 (the configuration the headline metric is quoted on).
A step is one full time step of the hot path: bounding box and grid, cell
sort and state reorder, narrow phase, contact forces with spring carry-over,
integration.  The state is resident in HBM before timing starts.

Prints one JSON line: particle-steps/s (value) and contacts/s, the roofline
of the kernel that computes the contact law on steps that keep the cells
(the fused narrow phase and contact law on grids of at most 1,024 slot groups,
128 N + 128 C algorithmic bytes per launch; else the contact-force kernel,
128 N + 120 C) over its mean duration, timed with HIP events on its own
dispatch, and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s & contacts/s: FP32/batched vs plain FP64 at stated tolerance"
HBM_PEAK_GBS = 8000.0


def force_bytes(n, c):
    """Algorithmic HBM bytes of one contact-force launch: per particle x, v, w,
    R read (80 B) and F, T written (48 B); per contact the pair (8 B) and the
    seven spring doubles read and written (112 B)."""
    return 128.0 * n + 120.0 * c


def fused_bytes(n, c):
    """Algorithmic HBM bytes of one launch of the fused narrow phase and
    contact law: those of the contact-force kernel, with the pair record and
    the partner-list entry written per contact (16 B) in place of the pair
    read."""
    return 128.0 * n + 128.0 * c


# grids of at most this many slot groups of 256 run the narrow phase and the
# contact law in one kernel on steps that keep the cells (one search lane)
ONE_ROUND_GROUPS = 1024


# bench workloads: the headline column, and the 8M packing whose state is
# far larger than the 256 MB Infinity Cache; each with its counter summary
# and its settings when none are given (None: autotuned)
WORKLOADS = {
    "column_200k": {"make": "cfg2", "radii": "lognormal, median 1 mm, sigma 0.2",
                    "traffic": "k_detect_force_cfg2_column_200k_hbm_traffic.md", "settings": None},
    "packing_8M": {"make": "cfg5", "radii": "half 1.0 mm, half 1.4 mm (rock-salt lattice)",
                   "traffic": "k_force_cfg5_packing_8M_hbm_traffic.md",
                   "settings": (1.0, 1, 0.2)},
}


def measured_traffic(workload):
    """HBM bytes per contact-force launch from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a copy of known size), or None when
    the kernel source changed since those counters were taken."""
    import hashlib
    try:
        text = open(os.path.join(ROOT, "profiles", WORKLOADS[workload]["traffic"])).read()
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in text.splitlines() if ": " in line and
                  line.split(": ", 1)[0] in ("traffic_bytes_per_launch", "kernel_source_sha256_16"))
    src = b"".join(open(os.path.join(ROOT, "paper_2507_12610_amd", "csrc", f), "rb").read()
                   for f in ("kernels.hip", "sdem_internal.h"))
    if hashlib.sha256(src).hexdigest()[:16] != fields.get("kernel_source_sha256_16", "").strip():
        return None
    return float(fields["traffic_bytes_per_launch"])


def cpu_baseline(w, budget_s=12.0, max_steps=40):
    import oracle
    o = oracle.Sim(w["params"], w["x"], v=w["v"], w=w["w"], q=w["q"], R=w["R"],
                   tri=w["tri"], rmesh=w["rmesh"])
    t0 = time.perf_counter()
    o.step(1)
    one = time.perf_counter() - t0
    k = int(max(1, min(max_steps - 1, budget_s / max(one, 1e-9) - 1)))
    t1 = time.perf_counter()
    o.step(k)
    dt = time.perf_counter() - t1
    steps = k + 1
    total = one + dt
    n = len(w["R"])
    return {"value": n * steps / total, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"first {steps} steps of the same workload (N={n}), serial FP64 oracle, "
                      f"{total:.1f} s"}


CPU_CHILD = r"""
import json, sys, time
sys.path.insert(0, sys.argv[1])
import oracle
import workloads as W
w = W.cfg2()
o = oracle.Sim(w["params"], w["x"], v=w["v"], w=w["w"], q=w["q"], R=w["R"], tri=w["tri"],
               rmesh=w["rmesh"])
steps = int(sys.argv[2])
t0 = time.perf_counter()
o.step(steps)
print(json.dumps({"n": len(w["R"]), "steps": steps, "s": time.perf_counter() - t0}))
"""


def cpu_all_cores(steps=3, max_procs=16):
    """The same serial oracle in one process per host core (at most 16, the
    host share of one GPU), each stepping its own copy of the workload:
    whole-host throughput = all their particle-steps over the slowest one's
    time.  Child processes, started fresh (never forked from this one)."""
    import subprocess
    k = max(1, min(max_procs, os.cpu_count() or 1))
    procs = [subprocess.Popen([sys.executable, "-c", CPU_CHILD, ROOT, str(steps)],
                              stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, text=True)
             for _ in range(k)]
    res = []
    for p in procs:
        out, _ = p.communicate(timeout=900)
        if p.returncode == 0:
            res.append(json.loads(out.strip().splitlines()[-1]))
    if not res:
        return None
    n, slowest = res[0]["n"], max(r["s"] for r in res)
    return {"value": len(res) * n * steps / slowest, "unit": "particle-steps/s", "cores": len(res),
            "kind": "oracle",
            "sample": f"first {steps} steps of the same workload (N={n}) in {len(res)} serial "
                      f"FP64 oracle processes at once, slowest {slowest:.1f} s"}


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


def mixed_vs_fp64(w, cf, lanes, skin, steps_before=200):
    """One step of the mixed path and of the FP64 path from the same state
    and springs (taken after steps_before FP64 steps): per quantity, the
    largest difference relative to the largest FP64 value (for x, relative
    to the largest displacement of the step)."""
    import numpy as np
    from paper_2507_12610_amd import Solver
    a = Solver(w, precision="fp64", cell_factor=cf, detect_lanes=lanes, skin=skin)
    a.step(steps_before)
    st, c = a.state(forces=False), a.contacts()
    d = dict(w)
    d.update({k: st[k] for k in ("x", "v", "w", "q")})
    b = Solver(d, precision="mixed", cell_factor=cf, detect_lanes=lanes, skin=skin)
    b.set_history(c["ki"], c["kj"], c["us"], c["ur"], c["ut"])
    a.step(1)
    b.step(1)
    sa, sb = a.state(), b.state()
    a.close()
    b.close()

    def rel(x, y):
        den = float(np.abs(y).max())
        return float(np.abs(x - y).max() / den) if den > 0 else float(np.abs(x).max())

    out = {k: rel(sb[k], sa[k]) for k in ("F", "T", "v", "w", "q")}
    out["x"] = rel(sb["x"] - st["x"], sa["x"] - st["x"])
    return {"after_fp64_steps": steps_before, "contacts": int(len(c["ki"])),
            "max_rel_diff": {k: float(f"{v:.3e}") for k, v in out.items()}}


# (cell_factor, detect_lanes, skin, longest rebuild period) tried by the
# autotuner on the bench workload (0: the library's 64 steps)
TUNE_CANDIDATES = [(0.4, 1, 0.05, 0), (0.33, 1, 0.05, 0), (0.5, 1, 0.05, 0), (0.4, 2, 0.05, 0),
                   (0.4, 1, 0.1, 128), (0.4, 1, 0.1, 256), (0.33, 1, 0.1, 256), (0.5, 1, 0.1, 256),
                   (0.4, 1, 0.2, 256), (0.4, 1, 0.0, 0)]


# (cell_factor, detect_lanes, skin) tried for the 256 box drops (bouncier than the column)
BATCH_CANDIDATES = [(1.0, 1, 1.0), (0.7, 1, 1.0), (1.0, 1, 0.6), (0.7, 1, 0.6), (1.0, 1, 0.3),
                    (1.0, 1, 0.0)]


def packing_forms(warmup=10, steps=40):
    """The 8,000,000-sphere pre-compressed packing (six contacts per sphere
    at the start), FP64 and mixed precision with the same settings: where the
    contact law's arithmetic weighs more than at 200,000 spheres."""
    import torch

    import workloads as W
    from paper_2507_12610_amd import Solver
    w = W.cfg5()
    n = len(w["R"])
    print(f"[bench] packing: {n} particles", file=sys.stderr, flush=True)
    out = {"workload": w["name"], "particles": n, "cell_factor": 1.0, "skin": 0.2,
           "steps": steps}
    for prec in ("fp64", "mixed"):
        g = Solver(w, precision=prec, device="cuda:0", cell_factor=1.0, detect_lanes=1, skin=0.2)
        g.step(warmup)
        torch.cuda.synchronize()
        s0 = g.stats()
        t0 = time.perf_counter()
        g.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s1 = g.stats()
        g.close()
        del g
        out[prec] = {"ms_per_step": round(1e3 * dt / steps, 4),
                     "particle_steps_per_s": round(n * steps / dt, 1),
                     "contacts_per_step": round((s1["pp"] + s1["pw"] - s0["pp"] - s0["pw"]) / steps, 1)}
    out["mixed_speedup_vs_fp64"] = round(out["fp64"]["ms_per_step"] / out["mixed"]["ms_per_step"], 4)
    return out


def batched_forms(landing_steps, steps, precision_list=("fp64", "mixed")):
    """Configuration 4: 256 box drops of uneven size in one context, timed after
    the sims have landed, against the same 256 states stepped one simulation
    after another (separate contexts, plain FP64), all on the GPU."""
    import numpy as np
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
           "landing_steps": landing_steps, "steps": steps, "cell_factor": cf, "skin": skin}
    res = {}
    for prec in precision_list:
        g = Solver([p[0] for p in landed], precision=prec, cell_factor=cf, detect_lanes=1,
                   skin=skin)
        g.set_history(c["ki"], c["kj"], c["us"], c["ur"], c["ut"])
        g.step(2)
        torch.cuda.synchronize()
        s0 = g.stats()
        t0 = time.perf_counter()
        g.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s1 = g.stats()
        cont = (s1["pp"] - s0["pp"]) + (s1["pw"] - s0["pw"])
        res[prec] = {"ms_per_step": 1e3 * dt / steps, "particle_steps_per_s": total * steps / dt,
                     "contacts_per_s": cont / dt, "contacts_per_step": cont / steps}
        g.close()
    # the same 256 states, one simulation after another (plain FP64)
    seq = []
    for k in range(len(sims)):
        d, h = sim_slice(sims[k], st, c, b.offsets[k], b.offsets[k + 1])
        g = Solver(d, cell_factor=cf, detect_lanes=1, skin=skin)
        g.set_history(*h)
        seq.append(g)
    for g in seq:
        g.step(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g in seq:
        g.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for g in seq:
        g.close()
    res["sequential_fp64"] = {"ms_per_step": 1e3 * dt / steps,
                              "particle_steps_per_s": total * steps / dt}
    for prec in precision_list:
        res[prec]["speedup_vs_sequential_fp64"] = (res["sequential_fp64"]["ms_per_step"] /
                                                   res[prec]["ms_per_step"])
    out.update(res)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cell-factor", type=float, default=None,
                    help="cell edge / (2 R_max); default: autotuned")
    ap.add_argument("--detect-lanes", type=int, default=None,
                    help="lanes per particle in the contact search; default: autotuned")
    ap.add_argument("--skin", type=float, default=None,
                    help="cell skin in units of R_max (0: rebuild every step); default: autotuned")
    ap.add_argument("--rebuild-every", type=int, default=0,
                    help="longest rebuild period with a skin (0: 64); autotuned with the rest")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the mixed-precision and batched forms")
    ap.add_argument("--batch-landing-steps", type=int, default=1500)
    ap.add_argument("--batch-steps", type=int, default=100)
    ap.add_argument("--workload", choices=list(WORKLOADS), default="column_200k",
                    help="column_200k (the headline configuration) or packing_8M")
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
        every = args.rebuild_every
    elif args.cell_factor is None or args.detect_lanes is None or args.skin is None:
        # trials of 512 steps, two of the longest periods tried: a thin skin
        # or a long period looks fast over a few steps and loses once
        # particles drift past the skin
        best, timings = autotune(w, candidates=TUNE_CANDIDATES, steps=512, warmup=10,
                                 precision=args.precision)
        tuned = {"chosen": best, "trials": timings}
        print(f"[bench] autotuned: {best}", file=sys.stderr, flush=True)
        cf, lanes, skin = best["cell_factor"], best["detect_lanes"], best["skin"]
        every = best["rebuild_every"]
    else:
        cf, lanes, skin = args.cell_factor, args.detect_lanes, args.skin
        every = args.rebuild_every
    s = Solver(w, precision=args.precision, device="cuda:0", cell_factor=cf, detect_lanes=lanes,
               skin=skin, rebuild_every=every)
    s.step(args.warmup)
    torch.cuda.synchronize()
    st0 = s.stats()
    t0 = time.perf_counter()
    s.step(args.steps)  # returns after the stream has drained
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st1 = s.stats()
    wall = t1 - t0
    ms_per_step = 1e3 * wall / args.steps
    contacts = (st1["pp"] - st0["pp"]) + (st1["pw"] - st0["pw"])
    value = n * args.steps / wall
    print(f"[bench] {args.steps} steps in {wall:.3f} s, {contacts / args.steps:.0f} contacts/step",
          file=sys.stderr, flush=True)

    # per-phase times with HIP events (no graph) on the solver's stream, one
    # step at a time so that the steps that rebuild the cells are told apart
    prof = []
    for _ in range(args.profile_steps):
        a = s.stats()
        ph = s.step_profiled(1)
        b = s.stats()
        prof.append((b["rebuilds"] > a["rebuilds"], ph, (b["pp"] - a["pp"]) + (b["pw"] - a["pw"])))
    keep = [p for p in prof if not p[0]] or prof
    phases = {k: sum(p[1][k] for p in prof) / len(prof) for k in prof[0][1]}
    # start/stop events attached to the dispatch of the kernel in the force
    # phase, over the steps that keep the cells (the timed steps are such
    # steps but for a few rebuilds)
    fms = sum(p[1]["force_kernel"] for p in keep) / len(keep)
    c_prof = sum(p[2] for p in keep) / len(keep)
    fused = skin > 0 and lanes == 1 and -(-n // 256) <= ONE_ROUND_GROUPS
    if fused:
        # the library counts the narrow phase as 0 on the steps where it
        # runs inside the force phase's kernel
        assert all(p[1]["detect"] == 0.0 for p in keep), "narrow phase not fused"
        kname = "k_detect_force (narrow phase, contact law, spring carry-over)"
        alg = fused_bytes(n, c_prof)
    else:
        kname = "k_force (contact forces, torques, spring carry-over)"
        alg = force_bytes(n, c_prof)
    achieved = alg / (fms * 1e-3) / 1e9
    dominant = max((k for k in phases if k != "force_kernel"), key=phases.get)
    roofline = {"kernel": kname, "bound": "hbm",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(args.workload),
                "mean_ms": round(fms, 5), "algorithmic_bytes": alg,
                "contacts_per_launch": round(c_prof, 1),
                "launches_timed": len(keep),
                "phase_ms": {k: round(v, 5) for k, v in phases.items() if k != "force_kernel"},
                "dominant_phase": dominant}

    out = {"metric": METRIC, "value": round(value, 1), "unit": "particle-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if args.precision == "fp64" else "f32+f64",
           "data": "synthetic",
           "config": {"workload": w["name"], "particles": n, "triangles": len(w["tri"]),
                      "dt": w["params"]["dt"], "precision": args.precision,
                      "radii": spec["radii"],
                      "friction": [w["params"]["mu_s"], w["params"]["mu_r"], w["params"]["mu_t"]],
                      "cell_factor": cf, "detect_lanes": lanes, "skin": skin,
                      "rebuild_every": every if every > 0 else 64,
                      "cell_rebuilds": f"{st1['rebuilds'] - st0['rebuilds']} of {args.steps} steps"},
           "contacts_per_s": round(contacts / wall, 1),
           "contacts_per_step": round(contacts / args.steps, 1),
           "pair_contacts_per_step": round((st1["pp"] - st0["pp"]) / args.steps, 1),
           "wall_contacts_per_step": round((st1["pw"] - st0["pw"]) / args.steps, 1),
           "roofline": roofline}
    if tuned is not None:
        out["autotune"] = tuned
    if not args.no_forms:
        forms = {}
        other = "mixed" if args.precision == "fp64" else "fp64"
        g = Solver(w, precision=other, device="cuda:0", cell_factor=cf, detect_lanes=lanes,
                   skin=skin, rebuild_every=every)
        g.step(args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(args.steps)
        torch.cuda.synchronize()
        ms_other = 1e3 * (time.perf_counter() - t0) / args.steps
        g.close()
        forms[other] = {"workload": w["name"], "ms_per_step": round(ms_other, 5),
                        "particle_steps_per_s": round(n * 1e3 / ms_other, 1),
                        "speedup_vs_" + args.precision: round(ms_per_step / ms_other, 4),
                        "tolerance": 1e-5 if other == "mixed" else 1e-12}
        forms["mixed_vs_fp64_one_step"] = mixed_vs_fp64(w, cf, lanes, skin)
        if skin > 0:
            # the paper's scheme, cells rebuilt every step, same workload
            g = Solver(w, precision=args.precision, device="cuda:0", cell_factor=cf,
                       detect_lanes=lanes, skin=0.0)
            g.step(args.warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.step(args.steps)
            torch.cuda.synchronize()
            ms_rb = 1e3 * (time.perf_counter() - t0) / args.steps
            g.close()
            forms["cells_rebuilt_every_step"] = {
                "workload": w["name"], "ms_per_step": round(ms_rb, 5),
                "particle_steps_per_s": round(n * 1e3 / ms_rb, 1)}
        forms["batched"] = batched_forms(args.batch_landing_steps, args.batch_steps)
        if args.workload != "packing_8M":
            forms["packing_8M"] = packing_forms()
        out["forms"] = forms
    if not args.no_cpu:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w)
        print("[bench] timing the CPU oracle on every host core", file=sys.stderr, flush=True)
        out["cpu_all_cores"] = cpu_all_cores()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
