"""Throughput of the fracture hot path on one MI355X.

The timed form is the FP32-bulk one by default; the plain FP64 form runs
after it on the same workload for the comparison (its throughput and the
per-field L1 error of FP32-bulk against it).

One step = one full time step of the whole hot path over the 1024^2
expanding-ring workload (or, with --workload ensemble, over every member of
the seeded ensemble of uneven rings in one context): three SSP-RK3 stage launches (reconstruction, HLLC
with the void-opening modifier, conservative update) with the source step
(plastic return, damage, phi0 gather) and the CFL reduction fused into the
third.  Inputs are resident in HBM when the timed region starts.

Prints one JSON line: cell-updates/s, the roofline of the dominant (stage)
kernel and the CPU oracle timed on a bounded window of the same workload.
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

HBM_PEAK_GBS = 8000.0
SCHEDULES = {0: "by-instance", 1: "largest-first", 2: "interleaved"}  # fv_options.tile[2]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stage_kernel_traffic.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2210_04037_amd", "csrc", f)
                  for f in ("fv_core.hpp", "fv_stage.hpp", "fv_kernels.hpp",
                            "fv_fp64.hip", "fv_fp32.hip")]


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _profile_fields():
    """Fields of the committed rocprofv3 summary, if it was taken on the
    current kernel source; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_hash") != kernel_source_hash():
        return None
    return vals


def profile_value(key, precision=None, tile=None):
    """A figure from the committed rocprofv3 summary, if it was taken on the
    current kernel source (and, given a precision and tile, in that tile
    shape); else None."""
    vals = _profile_fields()
    if vals is None or key not in vals:
        return None
    if precision is not None:
        want = vals.get(f"tile_{precision}")
        if tile is None or want != "%dx%d" % (tile[0], tile[1]):
            return None
    try:
        return float(vals[key])
    except ValueError:
        return None


# VALU issue rate without packed FP32: 256 CUs x 4 SIMDs, one wave64
# instruction per SIMD every 4 cycles at 2.4 GHz
VALU_WAVE_INSTR_PER_S = 256 * 4 * 2.4e9 / 4


def measured_traffic(precision, tile):
    """HBM bytes per stage launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source in this tile
    shape; else None."""
    return profile_value(f"bytes_per_launch_{precision}", precision, tile)


def cpu_baseline(case, seconds=15.0):
    """The oracle on a bounded window of the same workload: a 96 x 96
    window through the ring, stepped until ~`seconds` of CPU time."""
    from threadpoolctl import threadpool_limits
    import fvinputs as F
    from oracle import Solver
    nx = case.n[0]
    w = 96
    x0 = int(nx * (0.5 + 0.4292 * 0.7071)) - w // 2     # on the ring, 45 deg
    y0 = x0
    dx, dy = case.dx[0], case.dx[1]
    sub = F.Case(case.name + "_window", 2, (w, w, 1),
                 (case.lo[0] + x0 * dx, case.lo[1] + y0 * dy, case.lo[2]),
                 (case.lo[0] + (x0 + w) * dx, case.lo[1] + (y0 + w) * dy,
                  case.hi[2]), case.bc, case.mats,
                 case.prim[:, :, y0:y0 + w, x0:x0 + w].copy(),
                 case.phi0[:, y0:y0 + w, x0:x0 + w].copy(), case.t_end)
    with threadpool_limits(limits=1):
        s = Solver(sub)
        t0 = time.process_time()
        w0 = time.perf_counter()
        steps = 0
        while time.process_time() - t0 < seconds and steps < 200:
            s.step()
            steps += 1
        wall = time.perf_counter() - w0
    return {"value": w * w * steps / wall, "unit": "cell-updates/s",
            "cores": 1, "kind": "oracle",
            "sample": f"{w}x{w} window of the 1024^2 ring workload through "
                      f"the annulus, {steps} steps, single thread",
            "host": host_cpu()}


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


def run_gpu(cases, precision, steps, warmup, autotune=True, chunk=10,
            keep_state=True, tile=None):
    """Time `steps` steps after `warmup` untimed ones (the autotuner runs
    before the warm-up); return the timing, the chosen tile, and the
    primitive states and conservation totals at the end."""
    import torch
    from paper_2210_04037_amd.solver import GpuSolver
    g = GpuSolver(cases, precision=precision, device="cuda:0",
                  use_graph=chunk > 0, tile=tile)
    tot0, _ = g.totals()
    table = None
    if autotune and tile is None:
        tile, table = g.autotune(reps=10)
    _step_chunked(g, warmup, chunk)
    torch.cuda.synchronize()
    s = g.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    _step_chunked(g, steps, chunk)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    t = g.time()
    g.cfl_dt()          # raises if the device flagged a non-physical state
    tot1, out1 = g.totals()
    W = [g.primitive(i) for i in range(len(g.cases))] if keep_state else None
    S = g.S
    elem = 8 if precision == "fp64" else 4
    g.close()
    return dict(ms=ms, S=S, elem=elem, t=t, W=W, tot0=tot0, tot1=tot1 + out1,
                tile=tile, tiles_ms=table)


def valu_report(args, r, avg_launch_s):
    """Instruction-issue bound of the stage kernel (1024^2 ring, FP32-bulk,
    in the tile shape the counters were taken in): the VALU
    wave-instructions one launch executes (rocprofv3 SQ_INSTS_VALU) at the
    chip's issue rate, against the measured launch time."""
    if args.workload != "ring" or args.precision != "fp32":
        return None
    n = profile_value("SQ_INSTS_VALU", "fp32", r["tile"])
    if n is None:
        return None
    floor = n / VALU_WAVE_INSTR_PER_S
    return {"wave_instructions_per_launch": n, "issue_floor_ms": floor * 1e3,
            "measured_launch_ms": avg_launch_s * 1e3,
            "frac": floor / avg_launch_s}


def precision_report(cases, r32, r64):
    """Per-field L1 of the FP32-bulk run against the FP64 run after the same
    steps (relative to the FP64 field's L1, summed over every instance; eps_p
    and D over solid cells), and the worst relative conservation drift of
    the FP32-bulk run over the instances."""
    import numpy as np
    from paper_2210_04037_amd.abi import state_rows
    c0 = cases[0]
    rows = state_rows(c0.dim, len(c0.mats),
                      [m["kind"] == "solid" for m in c0.mats])
    num = dict(rho=0.0, u=0.0, eps_p=0.0, D=0.0)
    den = dict(rho=0.0, u=0.0, eps_p=0.0, D=0.0)
    rho = lambda W: np.sum(W[rows["phi"]] * W[rows["mass"]], axis=0)
    spd = lambda W: np.sqrt(np.sum(W[rows["mom"]] ** 2, axis=0))
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
    return {
        "l1_rel_vs_fp64": {k: (num[k] / den[k] if den[k] > 0 else 0.0)
                           for k in num},
        "bars": {"rho": 1e-4, "u": 1e-3, "eps_p": 1e-3, "D": 1e-2},
        "mass_drift": max(abs(a1[i][l] - a0[i][l]) / abs(a0[i][l])
                          for i in range(len(cases)) for l in range(nm)),
        "energy_drift": max(abs(a1[i][-1] - a0[i][-1]) / abs(a0[i][-1])
                            for i in range(len(cases))),
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32"],
                    help="timed form: fp32 = FP32-bulk (default), fp64 = plain")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the run of the other form (throughput and "
                         "per-field L1 error of FP32-bulk against FP64)")
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", default="ring",
                    choices=["ring", "ensemble", "shell3d", "impact3d"],
                    help="ring: the 1024^2 expanding ring (default); "
                         "ensemble: seeded rings of uneven sizes in one "
                         "context; shell3d: the 256^3 expanding shell; "
                         "impact3d: the 512^3 plate impact")
    ap.add_argument("--members", type=int, default=64)
    ap.add_argument("--no-loop", action="store_true",
                    help="ensemble: skip timing the members one at a time")
    ap.add_argument("--fragments", action="store_true",
                    help="ensemble: also run members 0-7 at full size to "
                         "their end time in both forms and report fragment "
                         "counts and cumulative mass histograms")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tile", default=None,
                    help="fixed tile 'TX,TY' or 'TX,TY,SCHEDULE' (0: by "
                         "instance, 1: largest first, 2: interleaved); skips "
                         "the autotuner")
    ap.add_argument("--graph-chunk", type=int, default=10,
                    help="steps per captured graph (0: eager launches)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a 1 GiB device copy (counter scaling)")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU; --gpus {args.gpus} is not "
              "supported (sharding over several GPUs is not implemented)",
              file=sys.stderr)
        sys.exit(2)
    import fvinputs as F
    chunk = args.graph_chunk
    if args.workload == "ring":
        cases = [F.make_case(2, n=args.n)]
        workload = (f"2D expanding ring {args.n}x{args.n} over a 60 mm "
                    "square: copper-like annulus 25-26.5 mm in gas, "
                    "150 m/s r/R, Gaussian phi0 (0.2 mm, 5%)")
    elif args.workload == "ensemble":
        cases = [F.make_case(4, member=m) for m in range(args.members)]
        workload = (f"ensemble of {args.members} seeded 2D expanding rings, "
                    "edges drawn from {256,384,512,768}, ring speeds "
                    "U(100, 250) m/s, one context (every member in each "
                    "launch)")
    elif args.workload == "shell3d":
        ne = args.n if args.n != 1024 else 256
        cases = [F.make_case(3, n=ne)]
        workload = (f"3D expanding cylindrical shell {ne}^3 over a 40 mm cube: "
                    "copper-like shell r 15-16 mm, |z| <= 15 mm, 200 m/s "
                    "radial, in gas; log-normal phi0 (0.3 mm, sigma 0.05)")
    else:
        ne = args.n if args.n != 1024 else 512
        cases = [F.make_case(5, n=ne)]
        workload = (f"3D plate impact {ne}^3 over a 20 mm cube: 4 mm "
                    "copper-like flyer at 400 m/s on a 16 mm target with "
                    "1000 spherical inclusions (phi0 0.7, r 0.1-0.3 mm)")
    ncell = sum(c.n_cells for c in cases)
    other = "fp64" if args.precision == "fp32" else "fp32"
    tile = tuple(int(v) for v in args.tile.split(",")) if args.tile else None
    r = run_gpu(cases, args.precision, args.steps, args.warmup,
                autotune=not args.no_autotune, chunk=chunk, tile=tile)
    ms, S, elem = r["ms"], r["S"], r["elem"]
    cu_s = ncell * args.steps / (ms * 1e-3)
    launches = 3 * args.steps
    avg_launch_s = ms * 1e-3 / launches
    # algorithmic bytes per cell-update: SSP-RK3 moves 2S + 3S + 3S fields
    # plus one phi0 read; per launch that is a third of it
    bytes_per_launch = (8 * S + 1) * elem * ncell / 3.0
    achieved = bytes_per_launch / avg_launch_s / 1e9
    traffic = (measured_traffic(args.precision, r["tile"])
               if args.workload == "ring" else None)
    out = {
        "metric": "cell-updates/s",
        "value": cu_s,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {
            "workload": workload,
            "cells": ncell, "instances": len(cases), "state_fields": S,
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
            "kernel": ("stage_kernel (3 launches per step)" if cases[0].dim < 3
                       else "3D stage: prim3 + 3 x face3 + finish3 per stage"),
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "avg_launch_ms": avg_launch_s * 1e3,
        },
        "valu": valu_report(args, r, avg_launch_s),
        "autotune_ms_per_stage1_launch": (
            {"%dx%d/%s" % (k[0], k[1], SCHEDULES.get(k[2], k[2])): v
             for k, v in r["tiles_ms"].items()}
            if r["tiles_ms"] else None),
    }
    if not args.no_compare:
        r2 = run_gpu(cases, other, args.steps, args.warmup,
                     autotune=not args.no_autotune, chunk=chunk)
        out[f"{other}_form"] = {
            "value": ncell * args.steps / (r2["ms"] * 1e-3),
            "ms_per_step": r2["ms"] / args.steps, "tile": r2["tile"]}
        r32, r64 = (r, r2) if args.precision == "fp32" else (r2, r)
        out["precision"] = precision_report(cases, r32, r64)
    if args.workload == "ensemble" and not args.no_loop:
        loop_ms = loop_single_runs(cases, args.precision, args.steps,
                                   args.warmup, chunk)
        out["loop_of_single_runs"] = {
            "value": ncell * args.steps / (loop_ms * 1e-3),
            "ms_per_step": loop_ms / args.steps,
            "ensemble_speedup": loop_ms / ms}
    if args.workload == "ensemble" and args.fragments:
        out["fragments_members_0_7"] = fragment_report(cases[:8], chunk)
    if not args.no_cpu and args.workload == "ring":
        out["cpu_baseline"] = cpu_baseline(cases[0])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
