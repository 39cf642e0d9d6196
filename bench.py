"""Throughput of the fracture hot path on one MI355X.

One step = one full time step of the whole hot path (three SSP-RK3 stage
launches: reconstruction, HLLC with the void-opening modifier, conservative
update; the source step -- plastic return, damage, phi0 gather -- and the
CFL reduction fused into the third) over one batch of synthetic input.
Inputs are resident in HBM when a timed region starts.

The headline is the largest single-GPU workload: the 3D plate impact on
512^3 cells (copper-like flyer at 400 m/s on a target with 1000 spherical
inclusions), FP32-bulk timed, the plain FP64 form timed after it on the same
input, and the per-field L1 error of the FP32-bulk run against the FP64 run.
The same JSON line carries the 2D expanding ring at 1024^2 (both forms, plus
a window timed after fracture: the run restarts from its state at 20 us),
the batched ensemble of 64 rings of uneven sizes in one context (FP32-bulk,
beside a loop of the same members run one context at a time) and the 400^2
expanding disk in void with Lagrangian seeding (both forms).

Prints one JSON line: cell-updates/s, the roofline of the dominant (stage)
kernel and the CPU oracle timed on a bounded window of the headline
workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("cell-updates/s (FP32-bulk vs FP64, 1 GPU) at stated L1 error; "
          "% HBM roofline")
HBM_PEAK_GBS = 8000.0
SCHEDULES = {0: "by-instance", 1: "largest-first", 2: "interleaved"}  # fv_options.tile[2]
PROFILE_DIR = os.path.join(ROOT, "profiles")
# committed counter summaries per workload (HBM bytes per stage launch)
TRAFFIC_FILES = {
    "ring": os.path.join(PROFILE_DIR, "stage_kernel_ring1024.txt"),
    "impact3d": os.path.join(PROFILE_DIR, "stage_kernel_impact512.txt"),
    "shell3d": os.path.join(PROFILE_DIR, "stage_kernel_shell256.txt"),
    "ensemble": os.path.join(PROFILE_DIR, "stage_kernel_ensemble64.txt"),
    "disk": os.path.join(PROFILE_DIR, "stage_kernel_disk400.txt"),
}
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2210_04037_amd", "csrc", f)
                  for f in ("fv_core.hpp", "fv_stage.hpp", "fv_kernels.hpp",
                            "fv_fp64.hip", "fv_fp32.hip")]
BARS = {"rho": 1e-4, "u": 1e-3, "eps_p": 1e-3, "D": 1e-2}
DRIFT_BARS = {"mass": 1e-6, "energy": 1e-5}


def kernel_source_hash(paths=None):
    """Hash of the stage-kernel sources the counter summaries belong to."""
    h = hashlib.sha256()
    for p in (KERNEL_SOURCES if paths is None else paths):
        if os.path.exists(p):
            with open(p, "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


def profile_fields(path):
    """key: value lines of a committed rocprofv3 summary, if it was taken on
    the current kernel source; else None."""
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_hash") != kernel_source_hash():
        return None
    return vals


def profile_value(workload, key, precision=None, tile=None):
    """A figure from the committed summary of a workload (taken on the
    current kernel source, and in the given tile shape where one is
    named); else None."""
    vals = profile_fields(TRAFFIC_FILES.get(workload, ""))
    if vals is None or key not in vals:
        return None
    if precision is not None and tile is not None and f"tile_{precision}" in vals:
        if vals[f"tile_{precision}"] != "%dx%d" % (tile[0], tile[1]):
            return None
    try:
        return float(vals[key])
    except ValueError:
        return None


# VALU issue rate without packed FP32: 256 CUs x 4 SIMDs, one wave64
# instruction per SIMD every 4 cycles at 2.4 GHz
VALU_WAVE_INSTR_PER_S = 256 * 4 * 2.4e9 / 4


def host_cpu():
    """Model name and logical CPU count of the host the oracle ran on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count()}


def _window(case, lo_idx, w):
    """A sub-box of w cells per active direction starting at lo_idx (x, y,
    z), with the case's fields, phi0 and transmissive sides."""
    import fvinputs as F
    d = case.dim
    n = tuple(w if k < d else 1 for k in range(3))
    sl = tuple(slice(lo_idx[k], lo_idx[k] + n[k]) for k in (2, 1, 0))
    lo = tuple(case.lo[k] + lo_idx[k] * case.dx[k] if k < d else case.lo[k]
               for k in range(3))
    hi = tuple(lo[k] + n[k] * case.dx[k] if k < d else case.hi[k]
               for k in range(3))
    bc = tuple(("transmissive",) * 2 for _ in range(3))
    return F.Case(case.name + "_window", d, n, lo, hi, bc, case.mats,
                  case.prim[(slice(None),) + sl].copy(),
                  case.phi0[sl].copy(), case.t_end)


def cpu_baseline(case, lo_idx, w, seconds=15.0, max_steps=200):
    """The oracle, single-threaded, on a w^d window of the same workload,
    stepped until about `seconds` of CPU time."""
    from threadpoolctl import threadpool_limits
    from oracle import Solver
    sub = _window(case, lo_idx, w)
    with threadpool_limits(limits=1):
        s = Solver(sub)
        t0 = time.process_time()
        w0 = time.perf_counter()
        steps = 0
        while time.process_time() - t0 < seconds and steps < max_steps:
            s.step()
            steps += 1
        wall = time.perf_counter() - w0
    cells = sub.n_cells
    shape = "x".join(str(v) for v in sub.n[:case.dim])
    return {"value": cells * steps / wall, "unit": "cell-updates/s",
            "cores": 1, "kind": "oracle",
            "sample": f"{shape} window of the {case.name} workload, {steps} "
                      f"steps, single thread",
            "host": host_cpu()}


def _step_chunked(g, n, chunk):
    """n steps as replays of captured chunk-step graphs (plus one call for
    the remainder), or one eager call when chunk is 0."""
    if chunk <= 0:
        g.step(n)
        return
    for _ in range(n // chunk):
        g.step(chunk)
    if n % chunk:
        g.step(n % chunk)


def _timed(g, steps, chunk):
    import torch
    torch.cuda.synchronize()
    s = g.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    _step_chunked(g, steps, chunk)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def run_gpu(cases, precision, steps, warmup, autotune=True, chunk=10,
            keep_state=True, tile=None, advance_to=None):
    """Time `steps` steps after `warmup` untimed ones (the autotuner runs
    before the warm-up).  advance_to: first step every instance to this
    time (untimed), then time from there.  Returns the timing, the chosen
    tile, and the primitive states and conservation totals at the end."""
    from paper_2210_04037_amd.solver import GpuSolver
    import numpy as np
    g = GpuSolver(cases, precision=precision, device="cuda:0",
                  use_graph=chunk > 0, tile=tile)
    tot0, _ = g.totals()
    table = None
    if autotune and tile is None:
        tile, table = g.autotune(reps=3 if cases[0].dim == 3 else 10)
    start = None
    if advance_to is not None:
        t_end = np.array([c.t_end for c in cases])
        g.step(0, t_end=np.full(len(cases), advance_to))
        while np.any(g.time() < advance_to):
            _step_chunked(g, 200, chunk)
        g.cfl_dt()                       # raises on the device flag
        g.step(0, t_end=t_end)
        start = float(np.min(g.time()))
    _step_chunked(g, warmup, chunk)
    ms = _timed(g, steps, chunk)
    t = g.time()
    g.cfl_dt()          # raises if the device flagged a non-physical state
    tot1, out1 = g.totals()
    W = [g.primitive(i) for i in range(len(g.cases))] if keep_state else None
    crit = None
    if start is not None:
        from paper_2210_04037_amd.abi import state_rows
        c0 = cases[0]
        rows = state_rows(c0.dim, len(c0.mats), [m["kind"] == "solid" for m in c0.mats])
        # critical cells in the band of the form's storage precision
        band = 1e-9 if precision == "fp64" else 1e-6
        crit = 0
        for i in range(len(cases)):
            Wi = W[i] if W is not None else g.primitive(i)
            crit += int(np.sum(Wi[rows["dmg"][0]] >= c0.mats[0]["D_crit"] * (1 - band)))
    S = g.S
    elem = 8 if precision == "fp64" else 4
    g.close()
    del g
    import torch
    torch.cuda.empty_cache()
    return dict(ms=ms, S=S, elem=elem, t=t, W=W, tot0=tot0, tot1=tot1 + out1,
                tile=tile, tiles_ms=table, t_start=start, critical_cells=crit)


def precision_report(cases, r32, r64):
    """Per-field L1 of the FP32-bulk run against the FP64 run after the same
    steps (relative to the FP64 field's L1, summed over every instance; eps_p
    and D over solid cells; null where the FP64 field is zero everywhere),
    and the worst relative conservation drift of the FP32-bulk run over the
    instances (interior total plus cumulative outflow against the start)."""
    import numpy as np
    from paper_2210_04037_amd.abi import state_rows
    c0 = cases[0]
    rows = state_rows(c0.dim, len(c0.mats),
                      [m["kind"] == "solid" for m in c0.mats])
    num = dict(rho=0.0, u=0.0, eps_p=0.0, D=0.0)
    den = dict(rho=0.0, u=0.0, eps_p=0.0, D=0.0)

    def rho(W):
        return np.sum(W[rows["phi"]] * W[rows["mass"]], axis=0)

    def spd(W):
        return np.sqrt(np.sum(W[rows["mom"]] ** 2, axis=0))

    for W32, W64 in zip(r32["W"], r64["W"]):
        solid = W64[rows["phi"][0]] > 0.5
        pairs = dict(rho=(rho(W32), rho(W64)), u=(spd(W32), spd(W64)),
                     eps_p=(W32[rows["eps"][0]][solid], W64[rows["eps"][0]][solid]),
                     D=(W32[rows["dmg"][0]][solid], W64[rows["dmg"][0]][solid]))
        for k, (a, b) in pairs.items():
            num[k] += float(np.sum(np.abs(a - b)))
            den[k] += float(np.sum(np.abs(b)))
    nm = len(c0.mats)
    a0, a1 = r32["tot0"], r32["tot1"]
    l1 = {k: (num[k] / den[k] if den[k] > 0 else None) for k in num}
    drift = {
        "mass": max(abs(a1[i][l] - a0[i][l]) / abs(a0[i][l])
                    for i in range(len(cases)) for l in range(nm)),
        "energy": max(abs(a1[i][-1] - a0[i][-1]) / abs(a0[i][-1])
                      for i in range(len(cases))),
    }
    within = all(v is None or v <= BARS[k] for k, v in l1.items())
    within = within and all(drift[k] <= DRIFT_BARS[k] for k in drift)
    return {
        "l1_rel_vs_fp64": l1,
        "bars": BARS,
        "mass_drift": drift["mass"],
        "energy_drift": drift["energy"],
        "drift_bars": DRIFT_BARS,
        "within_bars": within,
        "sim_time_fp32_fp64": [float(r32["t"][0]), float(r64["t"][0])],
    }


def loop_single_runs(cases, precision, steps, warmup, chunk):
    """The same members one context at a time (each autotuned, warmed up
    and timed alone); returns the summed timed milliseconds."""
    total = 0.0
    for c in cases:
        r = run_gpu([c], precision, steps, warmup, chunk=chunk,
                    keep_state=False)
        total += r["ms"]
    return total


def fragment_report(cases, chunk):
    """Members run to their end time in one ensemble, FP64 and FP32-bulk;
    per member: fragment count of each form, the cumulative fragment-mass
    histogram of each (fragments of mass >= edge, fv_fragment_histogram),
    and the number of borderline cells (solid fraction within 0.05 of the
    0.5 cut in the FP64 state).  A form that raises the non-physical flag is
    reported at its last checkpoint before the flag, with the time reached."""
    import numpy as np
    import fvinputs as F
    from paper_2210_04037_amd import abi
    from paper_2210_04037_amd.solver import GpuSolver
    edges = F.mass_edges()
    t_end = np.array([c.t_end for c in cases])
    rep = {"edges_kg_per_m": edges, "members": [
        {"member": c.meta.get("member", i), "n": c.n[0]} for i, c in enumerate(cases)]}
    for prec in ("fp64", "fp32"):
        g = GpuSolver(cases, precision=prec, use_graph=chunk > 0)
        g.step(0, t_end=t_end)
        n = max(chunk, 1) * 10
        steps, flag = 0, None
        while np.any(g.time() < t_end) and steps < 200000:
            ck = g.checkpoint()
            try:
                g.step(n)
                g.cfl_dt()
            except abi.FvError as e:
                flag = str(e)
                g.restore(ck)
                break
            steps += n
            if steps % 1000 == 0:
                print(f"[fragments] {prec} step {steps} t/t_end "
                      f"{float(np.min(g.time() / t_end)):.3f}",
                      file=sys.stderr, flush=True)
        t = g.time()
        for i, c in enumerate(cases):
            _, frags = g.fragments(i, 0.5)
            m = rep["members"][i]
            if prec == "fp64":
                U = g.state(i)
                m["borderline_cells"] = int(np.sum(np.abs(U[0] - 0.5) < 0.05))
            m[f"t_reached_{prec}"] = float(t[i])
            m[f"fragments_{prec}"] = len(frags)
            m[f"cumulative_{prec}"] = g.mass_histogram(frags, edges)
        rep[f"steps_{prec}"] = steps
        rep[f"nonphysical_flag_{prec}"] = flag
        g.close()
    return rep


def calibrate_copy(nbytes=1 << 30, reps=5):
    """A plain device copy of known size, for scaling the FETCH_SIZE and
    WRITE_SIZE counters of rocprofv3 to bytes."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "copy", "bytes_read_per_copy": nbytes,
                      "bytes_written_per_copy": nbytes, "copies": reps}))


# ---------------------------------------------------------------------------
# rocprofv3 summaries (written on the GPU host from the csv output of
# --kernel-trace and --pmc runs of this script; read back by profile_value)
# ---------------------------------------------------------------------------
def _prof_rows(d, suffix):
    import csv
    import glob
    rows = []
    for f in sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)):
        with open(f, newline="") as fh:
            rows += list(csv.DictReader(fh))
    return rows


def _kernel_key(name):
    """Short kernel name: the template-id between the namespace and the
    argument list ('stage_kernel<2, 2, 1, float, float, 16, 14, 256>')."""
    n = name.split("(")[0]
    n = n.split("fvk::")[-1] if "fvk::" in n else n.replace("void ", "")
    return n.strip()


STAGE_PASSES = ("stage_kernel", "prim3_kernel", "xface3_kernel", "march3_kernel", "finish3_kernel")


def _median(v):
    v = sorted(v)
    n = len(v)
    return 0.0 if n == 0 else (v[n // 2] if n % 2 else 0.5 * (v[n // 2 - 1] + v[n // 2]))


def _counter_by_kernel(d, counter):
    """{kernel key: [value per dispatch]} for one counter of a --pmc run."""
    out = {}
    for r in _prof_rows(d, "counter_collection.csv"):
        if r.get("Counter_Name") != counter:
            continue
        out.setdefault(_kernel_key(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return out


def profile_summary(args):
    """Write a committed-style summary of one workload's rocprofv3 runs:
    per-pass dispatch durations, HBM bytes per stage from FETCH_SIZE and
    WRITE_SIZE scaled by a plain 1 GiB copy, and instruction counters."""
    prec = args.precision
    lines = [f"# stage passes, workload {args.workload} ({prec}): rocprofv3 summaries",
             "# kernel_source_hash: hash of the stage-kernel sources the counters belong to",
             f"kernel_source_hash: {kernel_source_hash()}"]
    if args.prof_notes and os.path.exists(args.prof_notes):
        lines.append("## commands (R = repository root; run from /tmp with TMPDIR=/tmp)")
        lines += ["# " + l.rstrip() for l in open(args.prof_notes) if l.strip()]
    if args.tile:
        lines.append(f"tile_{prec}: " + "x".join(args.tile.split(",")[:2]))
    # durations
    dur = {}
    for r in _prof_rows(args.prof_kt, "kernel_trace.csv"):
        k = _kernel_key(r["Kernel_Name"])
        dur.setdefault(k, []).append(
            (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
    passes = [k for k in dur if k.startswith(STAGE_PASSES)]
    lines.append("## kernel trace: dispatches and median duration (us)")
    for k in sorted(dur, key=lambda k: -sum(dur[k])):
        lines.append(f"#   {k:64s} calls {len(dur[k]):5d}  median_us {_median(dur[k]):10.1f}"
                     f"  mean_us {sum(dur[k]) / len(dur[k]):10.1f}")
    two_d = any(k.startswith("stage_kernel") for k in passes)
    if two_d:
        k = [k for k in passes if k.startswith("stage_kernel")][0]
        v = dur[k]
        by = [[v[i] for i in range(j, len(v), 3)] for j in range(3)]
        lines.append("# stage kernel by stage (median us): " + "  ".join(
            f"stage{j + 1} {_median(by[j]):.1f}" for j in range(3)))
        stage_us = sum(v) / len(v)
    else:
        stage_us = sum(sum(dur[k]) / len(dur[k]) for k in passes)
    lines.append(f"stage_mean_us_{prec}: {stage_us:.2f}")
    # counter scaling from the copy
    fc = max((max(v) for v in _counter_by_kernel(args.prof_copy_fetch, "FETCH_SIZE").values()),
             default=0.0)
    wc = max((max(v) for v in _counter_by_kernel(args.prof_copy_write, "WRITE_SIZE").values()),
             default=0.0)
    copy_kib = (1 << 30) / 1024.0
    fscale = copy_kib / fc if fc > 0 else float("nan")
    wscale = copy_kib / wc if wc > 0 else float("nan")
    lines.append("## counter scaling from a plain 1 GiB device copy")
    lines.append(f"# copy FETCH_SIZE KiB per copy {fc:.1f} -> fetch_scale {fscale:.4f}; "
                 f"WRITE_SIZE KiB per copy {wc:.1f} -> write_scale {wscale:.4f}")
    fetch = _counter_by_kernel(args.prof_fetch, "FETCH_SIZE")
    write = _counter_by_kernel(args.prof_write, "WRITE_SIZE")
    total = 0.0
    lines.append("## HBM traffic per dispatch (median; KiB as counted, GB scaled)")
    for k in sorted(passes):
        f = _median(fetch.get(k, [])) * 1024 * fscale
        w = _median(write.get(k, [])) * 1024 * wscale
        total += f + w
        lines.append(f"#   {k:64s} read_GB {f / 1e9:8.3f} write_GB {w / 1e9:8.3f}"
                     f"  GB/s {(f + w) / (_median(dur[k]) * 1e-6) / 1e9:8.0f}")
    lines.append(f"bytes_per_launch_{prec}: {total:.6e}")
    if args.prof_sq:
        lines.append("## instruction counters of the stage passes (median per dispatch)")
        rows = _prof_rows(args.prof_sq, "counter_collection.csv")
        names = sorted({r["Counter_Name"] for r in rows})
        for c in names:
            by = _counter_by_kernel(args.prof_sq, c)
            tot = sum(_median(by.get(k, [])) for k in passes)
            lines.append(f"{c}: {tot:.0f}")
    with open(args.profile_summary, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
def make_workload(name, n=None, members=64):
    """(cases, description, cpu window (lo index, width) or None)."""
    import fvinputs as F
    if name == "ring":
        ne = n or 1024
        cases = [F.make_case(2, n=ne)]
        desc = (f"2D expanding ring {ne}x{ne} over a 60 mm square: copper-like "
                "annulus 25-26.5 mm in gas, 150 m/s r/R, Gaussian phi0 "
                "(0.2 mm, 5%)")
        x0 = int(ne * (0.5 + 0.4292 * 0.7071)) - 48     # on the ring, 45 deg
        return cases, desc, ((x0, x0, 0), 96)
    if name == "disk":
        ne = n or 400
        cases = [F.expanding_disk(ne)]
        desc = (f"2D expanding disk {ne}x{ne} over a 26 cm square: 304L disk of "
                "radius 10 cm in void at u = 2000 r, Gaussian phi0 (std 0.1), "
                "Lagrangian seeding of void cells, CFL 0.4")
        return cases, desc, None
    if name == "ensemble":
        cases = [F.make_case(4, member=m) for m in range(members)]
        desc = (f"ensemble of {members} seeded 2D expanding rings, edges drawn "
                "from {256,384,512,768}, ring speeds U(100, 250) m/s, one "
                "context (every member in each launch)")
        return cases, desc, None
    if name == "shell3d":
        ne = n or 256
        cases = [F.make_case(3, n=ne)]
        desc = (f"3D expanding cylindrical shell {ne}^3 over a 40 mm cube: "
                "copper-like shell r 15-16 mm, |z| <= 15 mm, 200 m/s radial, "
                "in gas; log-normal phi0 (0.3 mm, sigma 0.05)")
        return cases, desc, None
    ne = n or 512
    cases = [F.make_case(5, n=ne)]
    desc = (f"3D plate impact {ne}^3 over a 20 mm cube: 4 mm copper-like flyer "
            "at 400 m/s on a 16 mm target with 1000 spherical inclusions "
            "(phi0 0.7, r 0.1-0.3 mm), free x-ends")
    # a window across the impact plane (x = 4 mm) through the inclusions
    w = 20
    x0 = max(0, int(ne * 0.2) - w // 2)
    y0 = ne // 2 - w // 2
    return cases, desc, ((x0, y0, y0), w)


def measure(name, cases, desc, args, compare=True, post_fracture=None):
    """Timed FP32-bulk (or --precision) run of a workload, the other form
    beside it, the precision report and the roofline of the stage kernel."""
    chunk = args.graph_chunk
    tile = tuple(int(v) for v in args.tile.split(",")) if args.tile else None
    ncell = sum(c.n_cells for c in cases)
    print(f"[bench] {name}: {ncell} cells, {args.precision}", file=sys.stderr,
          flush=True)
    r = run_gpu(cases, args.precision, args.steps, args.warmup,
                autotune=not args.no_autotune, chunk=chunk, tile=tile)
    ms, S, elem = r["ms"], r["S"], r["elem"]
    cu_s = ncell * args.steps / (ms * 1e-3)
    launches = 3 * args.steps
    avg_launch_s = ms * 1e-3 / launches
    # algorithmic bytes per cell-update: SSP-RK3 moves 2S + 3S + 3S fields
    # plus one phi0 read; per stage launch that is a third of it
    bytes_per_launch = (8 * S + 1) * elem * ncell / 3.0
    achieved = bytes_per_launch / avg_launch_s / 1e9
    traffic = profile_value(name, f"bytes_per_launch_{args.precision}",
                            args.precision, r["tile"])
    out = {
        "value": cu_s,
        "ms_per_step": ms / args.steps,
        "config": {
            "workload": desc, "cells": ncell, "instances": len(cases),
            "state_fields": S,
            "precision": ("fp32-bulk (FP64 EOS island, FP64 plastic return "
                          "and damage, exact totals)"
                          if args.precision == "fp32" else "fp64"),
            "tile": r["tile"], "graph_chunk_steps": chunk,
            "simulated_time_s": float(r["t"][0]),
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "stage kernel (3 launches per step)",
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "avg_launch_ms": avg_launch_s * 1e3,
        },
    }
    n_valu = profile_value(name, "SQ_INSTS_VALU", args.precision, r["tile"])
    if n_valu is not None:
        floor = n_valu / VALU_WAVE_INSTR_PER_S
        out["valu"] = {"wave_instructions_per_launch": n_valu,
                       "issue_floor_ms": floor * 1e3,
                       "measured_launch_ms": avg_launch_s * 1e3,
                       "frac": floor / avg_launch_s}
    if r["tiles_ms"]:
        out["autotune_ms_per_stage1_launch"] = {
            "%dx%d/%s" % (k[0], k[1], SCHEDULES.get(k[2], k[2])): v
            for k, v in r["tiles_ms"].items()}
    other = "fp64" if args.precision == "fp32" else "fp32"
    if compare:
        r2 = run_gpu(cases, other, args.steps, args.warmup,
                     autotune=not args.no_autotune, chunk=chunk)
        out[f"{other}_form"] = {
            "value": ncell * args.steps / (r2["ms"] * 1e-3),
            "ms_per_step": r2["ms"] / args.steps, "tile": r2["tile"]}
        r32, r64 = (r, r2) if args.precision == "fp32" else (r2, r)
        out["precision"] = precision_report(cases, r32, r64)
        del r2
    del r
    if post_fracture is not None:
        pf = {"start_time_s": post_fracture}
        for prec in ((args.precision, other) if compare else (args.precision,)):
            rp = run_gpu(cases, prec, args.steps, args.warmup, autotune=False,
                         chunk=chunk, keep_state=False, tile=None,
                         advance_to=post_fracture)
            pf[prec] = {"value": ncell * args.steps / (rp["ms"] * 1e-3),
                        "ms_per_step": rp["ms"] / args.steps,
                        "window_start_s": rp["t_start"],
                        "critical_cells_at_end": rp["critical_cells"]}
        out["post_fracture"] = pf
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32"],
                    help="timed form: fp32 = FP32-bulk (default), fp64 = plain")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the run of the other form (throughput and "
                         "per-field L1 error of FP32-bulk against FP64)")
    ap.add_argument("--n", type=int, default=None,
                    help="grid edge of the headline workload (default: its "
                         "full size)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", default="impact3d",
                    choices=["impact3d", "ring", "ensemble", "shell3d", "disk"],
                    help="headline workload: impact3d, the 512^3 plate impact "
                         "(default, the largest single-GPU workload); ring: "
                         "the 1024^2 expanding ring; ensemble: 64 seeded "
                         "rings of uneven sizes in one context; shell3d: the "
                         "256^3 expanding shell")
    ap.add_argument("--only", action="store_true",
                    help="measure the headline workload alone (no ring and "
                         "ensemble sections)")
    ap.add_argument("--members", type=int, default=64)
    ap.add_argument("--no-loop", action="store_true",
                    help="ensemble: skip timing the members one at a time")
    ap.add_argument("--fragments", action="store_true",
                    help="ensemble: also run members 0-7 at full size to "
                         "their end time in both forms and report fragment "
                         "counts and cumulative mass histograms")
    ap.add_argument("--post-fracture", type=float, default=20e-6,
                    help="ring: start time of the window timed after "
                         "fracture (0: skip)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tile", default=None,
                    help="fixed tile 'TX,TY' or 'TX,TY,SCHEDULE' (0: by "
                         "instance, 1: largest first, 2: interleaved); skips "
                         "the autotuner")
    ap.add_argument("--graph-chunk", type=int, default=10,
                    help="steps per captured graph (0: eager launches)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a 1 GiB device copy (counter scaling)")
    ap.add_argument("--profile-summary", default=None, metavar="OUT",
                    help="write the summary of rocprofv3 csv runs of this "
                         "script (--prof-* directories) to OUT and exit")
    for k in ("kt", "fetch", "write", "sq", "copy-fetch", "copy-write", "notes"):
        ap.add_argument(f"--prof-{k}", default=None)
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.profile_summary:
        profile_summary(args)
        return
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU; --gpus {args.gpus} is not "
              "supported (sharding over several GPUs is not implemented)",
              file=sys.stderr)
        sys.exit(2)
    head = args.workload
    cases, desc, window = make_workload(head, args.n, args.members)
    pf = args.post_fracture if (head == "ring" and args.post_fracture > 0) else None
    hm = measure(head, cases, desc, args, compare=not args.no_compare,
                 post_fracture=pf)
    out = {
        "metric": METRIC,
        "value": hm.pop("value"),
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hm.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": hm.pop("config"),
        "roofline": hm.pop("roofline"),
    }
    out.update(hm)
    if head == "ensemble" and not args.no_loop:
        ncell = sum(c.n_cells for c in cases)
        loop_ms = loop_single_runs(cases, args.precision, args.steps,
                                   args.warmup, args.graph_chunk)
        out["loop_of_single_runs"] = {
            "value": ncell * args.steps / (loop_ms * 1e-3),
            "ms_per_step": loop_ms / args.steps,
            "ensemble_speedup": loop_ms / out["ms_per_step"] / args.steps}
    if head == "ensemble" and args.fragments:
        out["fragments_members_0_7"] = fragment_report(cases[:8], args.graph_chunk)
    if not args.no_cpu and window is not None:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cases[0], window[0], window[1])
    del cases
    if not args.only and head == "impact3d":
        others = {}
        for name in ("ring", "ensemble", "disk", "shell3d"):
            c2, d2, _ = make_workload(name, None, args.members)
            m = measure(name, c2, d2, args, compare=name in ("ring", "disk", "shell3d")
                        and not args.no_compare,
                        post_fracture=(args.post_fracture if name == "ring"
                                       and args.post_fracture > 0 else None))
            if name == "ensemble" and not args.no_loop:
                ncell = sum(c.n_cells for c in c2)
                loop_ms = loop_single_runs(c2, args.precision, args.steps,
                                           args.warmup, args.graph_chunk)
                m["loop_of_single_runs"] = {
                    "value": ncell * args.steps / (loop_ms * 1e-3),
                    "ms_per_step": loop_ms / args.steps,
                    "ensemble_speedup": loop_ms / (m["ms_per_step"] * args.steps)}
            others[name] = m
            del c2
        out["other_workloads"] = others
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
