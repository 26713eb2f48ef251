"""Throughput of the BB minimiser hot path on one MI355X.

Workload: the 400 x 200 x 4 film of 5 nm cells (2000 x 1000 x 20 nm, the
Standard Problem #1 stand-in), Ms = 8e5 A/m, A = 1.3e-11 J/m, Ku = 500 J/m^3
along x, field +50 mT along x tilted 1 degree toward y, start +x with 1e-3
noise (seeded).  One step = one minimiser iteration: the effective field
(FFT demag convolution, exchange, anisotropy, Zeeman), g, the torque, the
energy and BB reductions, the step size and the midpoint update.  The timed
region runs K iterations through the library's run-to-tolerance loop with a
zero tolerance, so the device-side stop flag and the host polling are
exercised as in a hysteresis sweep.  Inputs are resident in HBM before the
clock starts.

With --workload cube the same measurement runs on the 128^3 cube of 2 nm
cells (full 3-D demag path, random start, 60 mT at 2 degrees from z); the
default film line carries a shorter run of it as "cube" (FP64 and mixed
iterations/s, the FP64 iteration's algorithmic bytes and rate).

The line also carries "batched": 64 uneven thin platelets (64..256 x
32..128 x 1..2 cells) swept through every 10th field of their +-40 mT loop,
once with all samples sharing launches (one persistent launch per pass,
covering every transform length; captured graph) and once sample by sample,
both in FP64: summed minimiser iterations per second, the speed-up and the
HBM fraction of the samples' algorithmic bytes.  --workload batched runs that alone on the whole loop (81 fields);
--workload adjoint times the implicit gradient of the 200 x 100 x 2 film
with a per-cell Ku map (conjugate gradients + parameter gradients);
--workload loop runs whole hysteresis loops (one device-driven sweep each):
the film in FP64 and mixed (201 fields), and the Standard Problem 1 film
along its long and short edge at 10 nm cells (200 x 100 x 2) with 1 and
0.5 mT steps and at 5 nm cells (short edge), reporting H_eff evaluations
per loop and per field step (the paper's Tab. 1 unit).  The mixed form runs
with its defect correction.  The timed iterations use the tile the library's
autotuner picks at set-up; --quick --graph also times captured HIP graphs.

Prints one JSON line.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


# name -> (synthetic workload id, field index, description, padded grid)
WORKLOADS = {
    "film": (1, 0, "film 400x200x4 cells of 5 nm (Standard Problem 1 stand-in), "
                   "BB midpoint minimiser, +50 mT at 1 deg", [896, 448, 4]),
    "cube": (2, 3, "cube 128^3 cells of 2 nm, full 3-D demag, BB midpoint minimiser, "
                   "random start, 60 mT at 2 deg from z", [256, 256, 256]),
}
EXTRA_WORKLOADS = ("batched", "adjoint", "loop", "cube-sweep")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=2000)
    p.add_argument("--warmup", type=int, default=100)
    p.add_argument("--prec", choices=["fp64", "mixed"], default="fp64")
    p.add_argument("--workload", choices=sorted(WORKLOADS) + list(EXTRA_WORKLOADS),
                   default="film")
    p.add_argument("--no-batched", action="store_true", help="skip the batched comparison")
    p.add_argument("--no-cube", action="store_true",
                   help="skip the 128^3 cube leg of the default film line")
    p.add_argument("--cube-steps", type=int, default=300)
    p.add_argument("--graph", action="store_true",
                   help="with --quick: also time the run with captured HIP graphs")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--cpu-iters", type=int, default=40)
    p.add_argument("--bb-switch", type=float, default=0.0, metavar="KAPPA",
                   help="with --workload loop: step choice (0 alternation of eq. (12); "
                        "kappa > 0 the ratio switch tau2 if tau2 < kappa tau1)")
    p.add_argument("--line-search", action="store_true",
                   help="with --workload loop: the non-monotone line search on every step")
    p.add_argument("--quick", action="store_true",
                   help="only the timed run (for profilers): no profiled pass, no other "
                        "precision, no CPU baseline")
    p.add_argument("--rows-per-block", type=int, default=0, metavar="R",
                   help="with --quick: x-pass tile R instead of the autotuner's choice (for "
                        "profiler runs, whose counters distort the tuner's timings)")
    p.add_argument("--yz-variant", type=int, default=-1, metavar="V",
                   help="with --quick: yz occupancy variant V instead of the autotuner's choice")
    p.add_argument("--copy-probe", type=float, default=0.0, metavar="MB",
                   help="run a plain device copy of MB megabytes 5 times and exit "
                        "(calibration of the memory-traffic counters)")
    return p.parse_args()


def run_gpu(prec, steps, warmup, w, profile, field=0, graph=False, rows=0, yz=-1):
    """Warm up, then time `steps` iterations.  With `profile` ("all" or a
    list of kernel names), the library records HIP events around those
    kernels' launches in the timed region (on the library's stream) and the
    per-kernel averages are returned.  The x-pass tile comes from the
    library's autotuner (timed at set-up, outside the timed region).  With
    `graph`, batches of poll_every iterations replay a captured HIP graph
    (on a stream of its own)."""
    import contextlib
    import torch
    from paper_1405_2728_amd import Context
    nx, ny, nz = w["n"]
    stream = torch.cuda.Stream() if graph else None
    ctx = Context(prec, stream=stream)
    ctx.set_option("use_graph", 1 if graph else 0)
    ctx.set_option("autotune", 1)
    if rows:
        ctx.set_option("rows_per_block", rows)
    ctx.set_option("yz_variant", yz)
    ctx.set_geometry(0, nx, ny, nz, *w["d"])
    rows = ctx.rows_per_block(0)
    yz_var = ctx.yz_variant(0)
    ctx.set_material(0, w["Ms"], w["A"], w["Ku"], w["u"])
    ctx.set_field(0, w["fields"][field])
    m = torch.tensor(w["m0"], dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    on = torch.cuda.stream(stream) if graph else contextlib.nullcontext()
    with on:
        ctx.minimize_to_tol(0, m, tol=0.0, max_iter=warmup)
        torch.cuda.synchronize()
        if profile:
            ctx.profile(profile)
        t0 = time.perf_counter()
        r = ctx.minimize_to_tol(0, m, tol=0.0, max_iter=steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    prof = ctx.profile_read() if profile else None
    if profile:
        ctx.profile(None)
    kb = ctx.kernel_bytes(0)
    ctx.close()
    return {"iters": r["iters"], "evals": r["heff_evals"], "seconds": dt, "prof": prof,
            "bytes": kb, "torque": r["torque"], "rows_per_block": rows, "yz_variant": yz_var}


def cube_leg(steps):
    """The 128^3 cube (3-D demag path) timed beside the film: FP64 and mixed
    iterations/s, and the FP64 iteration's algorithmic bytes and rate from a
    second run with events around every kernel."""
    import synth
    wid, field, desc, padded = WORKLOADS["cube"]
    w = synth.workload(wid)
    warm = max(10, steps // 10)
    r64 = run_gpu("fp64", steps, warm, w, profile=None, field=field)
    rp = run_gpu("fp64", steps, warm, w, profile="all", field=field)
    rmx = run_gpu("mixed", steps, warm, w, profile=None, field=field)
    prof = rp["prof"]
    per_iter = sum(r64["bytes"][k] * v[1] / rp["iters"] for k, v in prof.items() if v[1] > 0)
    ips = r64["iters"] / r64["seconds"]
    mips = rmx["iters"] / rmx["seconds"]
    return {"workload": desc, "padded_grid": padded, "value": ips, "unit": "iters/s",
            "steps": steps, "ms_per_step": 1e3 * r64["seconds"] / r64["iters"],
            "model_bytes": per_iter, "model_GBps": per_iter * ips / 1e9,
            "model_frac_of_8TBps": per_iter * ips / 8e12,
            "kernel_avg_us_all_timed": {k: 1e3 * v[0] / max(v[1], 1)
                                        for k, v in prof.items() if v[1] > 0},
            "mixed": {"value": mips, "unit": "iters/s", "speedup_vs_fp64": mips / ips}}


def stored_traffic(prec, kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/traffic_<prec>.json for the film, traffic_<prec>_<workload>.json
    otherwise), or None if absent or stale."""
    suffix = "" if workload == "film" else "_" + workload
    p = os.path.join(ROOT, "profiles", "traffic_%s%s.json" % (prec, suffix))
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        t = json.load(fh)
    from paper_1405_2728_amd.profiling import source_hash
    if t.get("source_hash") != source_hash():
        return None
    return t.get("kernels", {}).get(kernel, {}).get("bytes_per_launch")


def run_batched(torch, batched, field_step=10, prec="fp64", mixed_radix=1, concurrent=1,
                persistent=1, rebuild=None):
    """Sweep the 64 platelets through every field_step-th field of their
    loop; returns (summed iterations, seconds, status)."""
    import synth
    from paper_1405_2728_amd import Context
    plats = synth.batched_platelets()
    stream = torch.cuda.Stream()
    ctx = Context(prec, n_samples=len(plats), stream=stream)
    ctx.set_option("batched", 1 if batched else 0)
    ctx.set_option("use_graph", 1 if batched else 0)
    ctx.set_option("autotune", 1)   # tiles per shape, cached: both runs use the same
    ctx.set_option("mixed_radix", mixed_radix)
    ctx.set_option("concurrent_groups", concurrent)
    ctx.set_option("persistent", persistent)
    if rebuild is not None:
        ctx.set_option("batch_rebuild", rebuild)
    ms, H = [], []
    for k, p in enumerate(plats):
        ctx.set_geometry(k, *p["n"], *p["d"])
        ctx.set_material(k, p["Ms"], p["A"], p["Ku"], p["u"])
        ms.append(torch.tensor(p["m0"], device="cuda"))
        H.append(p["fields"][::field_step])
    H = np.array(H)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        t0 = time.perf_counter()
        mavg, iters, rc = ctx.hysteresis_sweep(ms, H, tol=plats[0]["tol"])
        stream.synchronize()
        dt = time.perf_counter() - t0
    # algorithmic bytes of the run: each sample's iterations times its bytes
    # per iteration (the x, yz and finish passes; the reference pass of the
    # mixed form once per poll_every iterations, 32 by default)
    per_sample = iters.sum(axis=1)
    nbytes = 0.0
    for k in range(len(plats)):
        kb = ctx.kernel_bytes(k)
        b = kb["xf"] + kb["yz_thin"] + kb["xil"] + kb["finish"] + kb["reference"] / 32.0
        nbytes += float(per_sample[k]) * b
    ctx.close()
    stats = {"bytes": nbytes, "max_sample_iters": int(per_sample.max()),
             "mean_sample_iters": float(per_sample.mean())}
    return int(iters.sum()), dt, rc, H.shape[1], stats


def run_adjoint(torch):
    """200x100x2 film with a Ku map: sweep 0..-5 mT (tol 1e-10), then the
    gradient of <m_x> by the adjoint (timed)."""
    import synth
    from paper_1405_2728_amd import Context
    w = synth.workload(4)
    ctx = Context("fp64")
    ctx.set_geometry(0, *w["n"], *w["d"])
    ctx.set_material(0, w["Ms"], w["A"], 0.0, w["u"],
                     torch.tensor(w["Ku"], dtype=torch.float64, device="cuda"))
    m = torch.tensor(w["m0"], device="cuda")
    t0 = time.perf_counter()
    _, iters, rc = ctx.hysteresis_sweep([m], w["fields"], tol=1e-10)
    torch.cuda.synchronize()
    t_sweep = time.perf_counter() - t0
    dJ = torch.zeros_like(m)
    dJ[0] = 1.0 / m[0].numel()
    ctx.adjoint_solve(0, m, dJ, tol=1e-10)           # warm-up (workspace allocation)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lam, it, res, rc2 = ctx.adjoint_solve(0, m, dJ, tol=1e-10)
    g = ctx.param_grads(0, m, lam)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    ctx.close()
    return {"sweep_iters": int(iters.sum()), "sweep_s": t_sweep, "cg_iterations": it,
            "cg_residual": res, "adjoint_s": t_adj, "cg_iters_per_s": it / t_adj,
            "dJ_dA": g["A"], "dJ_dMs": g["Ms"], "status": [int(rc), int(rc2)]}


def run_loop(torch, prec, n, d, m0, fields, tol=1e-6, bb_switch=0.0, line_search=False):
    """One device-driven sweep over the whole loop; (evaluations, seconds,
    <m> per field, status).  bb_switch, line_search: the library's
    step-choice options."""
    import synth
    from paper_1405_2728_amd import Context
    ctx = Context(prec)
    ctx.set_option("bb_switch", bb_switch)
    ctx.set_option("line_search", 1 if line_search else 0)
    ctx.set_geometry(0, *n, *d)
    ctx.set_material(0, synth.PERMALLOY["Ms"], synth.PERMALLOY["A"], synth.PERMALLOY["Ku"],
                     synth.PERMALLOY["u"])
    m = torch.tensor(m0, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mavg, iters, rc = ctx.hysteresis_sweep([m], fields[None], tol=tol)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    evals, _ = ctx.counters(0)          # every evaluation, rejected trials included
    ctx.close()
    return int(evals), dt, mavg[0], int(rc)


def coercive_fields_mT(mavg, fields, h):
    """Field (mT, along h) of the first sign change of <m>.h on each branch."""
    import synth
    proj = mavg @ h
    amp = fields @ h / synth.MT
    nd = (len(fields) + 1) // 2
    down = next((amp[f] for f in range(nd) if proj[f] < 0), None)
    up = next((amp[f] for f in range(nd, len(proj)) if proj[f] > 0), None)
    return [None if v is None else float(v) for v in (down, up)]


def loops(torch, bb_switch=0.0, line_search=False):
    import synth
    out = {}
    w = synth.workload(1)
    h = synth.tilted(1.0)
    for prec in ("fp64", "mixed"):
        ev, dt, mavg, rc = run_loop(torch, prec, w["n"], w["d"], w["m0"], w["fields"],
                                    bb_switch=bb_switch, line_search=line_search)
        out["film400x200x4_" + prec] = {"evals_per_loop": ev, "seconds": dt, "evals_per_s": ev / dt,
                                        "coercive_mT": coercive_fields_mT(mavg, w["fields"], h),
                                        "status": rc}
    out["film400x200x4_fp64"]["evals_per_field"] = out["film400x200x4_fp64"]["evals_per_loop"] / len(
        w["fields"])
    # Standard Problem 1 stand-in (2 um x 1 um x 20 nm permalloy) along its long
    # and short edge: 10 nm cells (200 x 100 x 2) at 1 and 0.5 mT steps, and the
    # short edge at 5 nm cells (400 x 200 x 4; the long edge at 5 nm is the film
    # above).  Paper Tab. 1 counts for 10 nm, 1 mT: 64814 and 81454 evaluations
    # per loop on other hardware and code (context only).
    cases = [("sp1_10nm_long_edge", "long", 10e-9, 1.0),
             ("sp1_10nm_short_edge", "short", 10e-9, 1.0),
             ("sp1_10nm_long_edge_0.5mT", "long", 10e-9, 0.5),
             ("sp1_10nm_short_edge_0.5mT", "short", 10e-9, 0.5),
             ("sp1_5nm_short_edge", "short", 5e-9, 1.0)]
    for name, edge, cell, step in cases:
        w = synth.sp1_loop(edge, cell, step)
        f = w["fields"]
        ev, dt, mavg, rc = run_loop(torch, "fp64", w["n"], w["d"], w["m0"], f,
                                    bb_switch=bb_switch, line_search=line_search)
        hh = w["h"]
        out[name] = {"fields": len(f), "evals_per_loop": ev, "evals_per_field": ev / len(f),
                     "seconds": dt, "coercive_mT": coercive_fields_mT(mavg, f, hh), "status": rc}
        print(name, out[name], file=sys.stderr, flush=True)
    return out


def copy_ceiling(torch, mb=1024, reps=10):
    """Bandwidth of a plain device copy of `mb` megabytes (read + write bytes
    over the time, HIP events on torch's stream): the attainable HBM
    ceiling next to the 8 TB/s peak."""
    n = int(mb * 1e6 / 8)
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    s = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst
    return 2 * 8 * n / s / 1e9


def host_cores():
    """Threads the CPU baseline may use: the CPUs this process may run on,
    capped by OMP_NUM_THREADS where it is set (the box's share)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cap = os.environ.get("OMP_NUM_THREADS")
    if cap and cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, n)


def cube_sweep(torch, fields_idx=None, max_iter=100000, oracle_check=True):
    """The 128^3 cube (2 nm cells, random start) relaxed at H = 0, then at
    20, 40, ..., 200 mT along z + 2 degrees, in FP64 and in the mixed form
    side by side, field by field.  Per field: <m> of both, iterations, the
    mixed state's distance to the FP64 state (|dm|_inf), the torque of the
    mixed state under the FP64 effective field (cross-stationarity), and the
    first field at which every cell points along the field (m.h > 0) in
    each form.  With oracle_check, the oracle's torque at the first and
    last FP64 states (its own FFT convolution at 256^3)."""
    import synth
    from paper_1405_2728_amd import Context
    w = synth.workload(2)
    F = w["fields"] if fields_idx is None else w["fields"][list(fields_idx)]
    h = F[-1] / np.linalg.norm(F[-1])
    ctx, m = {}, {}
    for prec in ("fp64", "mixed"):
        c = Context(prec)
        c.set_geometry(0, *w["n"], *w["d"])
        c.set_material(0, w["Ms"], w["A"], w["Ku"], w["u"])
        ctx[prec], m[prec] = c, torch.tensor(w["m0"], device="cuda")
    rows, states = [], []
    for f, H in enumerate(F):
        r = {"field_mT": float(np.linalg.norm(H) / synth.MT)}
        for prec in ("fp64", "mixed"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            a, it, rc = ctx[prec].hysteresis_sweep([m[prec]], H[None, None], tol=w["tol"],
                                                   max_iter=max_iter)
            torch.cuda.synchronize()
            mh = (m[prec] * torch.tensor(h, device="cuda")[:, None, None, None]).sum(0)
            r[prec] = {"mavg": [float(v) for v in a[0, 0]], "iters": int(it[0, 0]),
                       "status": int(rc), "seconds": time.perf_counter() - t0,
                       "all_along_field": bool((mh > 0).all())}
        ctx["fp64"].set_field(0, H)
        Hm = ctx["fp64"].heff(0, m["mixed"])
        g = torch.linalg.cross(m["mixed"], torch.linalg.cross(m["mixed"], Hm, dim=0), dim=0)
        r["mixed_torque_fp64_field"] = float(g.norm(dim=0).max()) / w["Ms"]
        r["dm_inf"] = float((m["mixed"] - m["fp64"]).abs().max())
        rows.append(r)
        print("cube field %d %s" % (f, json.dumps(r)), file=sys.stderr, flush=True)
        if oracle_check and f in (0, len(F) - 1):
            states.append((H.copy(), m["fp64"].cpu().numpy()))
    for c in ctx.values():
        c.close()
    out = {"fields": rows}
    for prec in ("fp64", "mixed"):
        out["first_saturated_index_" + prec] = next(
            (i for i, r in enumerate(rows) if r[prec]["all_along_field"]), None)
    out["max_dm_inf"] = max(r["dm_inf"] for r in rows)
    out["max_mixed_torque_fp64_field"] = max(r["mixed_torque_fp64_field"] for r in rows)
    if oracle_check:
        from oracle import fields as of, minimizer as om
        P = of.Problem(*w["n"], *w["d"], Ms=w["Ms"], A=w["A"], Ku=w["Ku"], u=w["u"],
                       fft_workers=host_cores())
        out["oracle_torque_at_fp64_states"] = []
        for H, mg in states:
            P.H_ext = H
            out["oracle_torque_at_fp64_states"].append(om.torque(mg, P.heff(mg), P.Ms))
    return out


def cpu_baseline(w, iters, field, label, workers=1):
    """The oracle (as it stands) on `iters` minimiser iterations of the same
    workload; its FFT convolution on `workers` threads (scipy.fft), the rest
    of it (stencil, per-cell solves of eq. (7), sums) in NumPy on one."""
    from oracle import fields as of, minimizer as om
    P = of.Problem(*w["n"], *w["d"], Ms=w["Ms"], A=w["A"], Ku=w["Ku"], u=w["u"],
                   H_ext=w["fields"][field], fft_workers=workers)
    P.heff(w["m0"])                      # tensor and its transform: set-up, not timed
    t0 = time.perf_counter()
    om.minimize(P, w["m0"], tol=0.0, max_iter=iters)
    dt = time.perf_counter() - t0
    how = ("numpy FFT, one thread" if workers == 1 else
           "scipy.fft on %d threads, stencil and update in NumPy" % workers)
    return {"value": iters / dt, "unit": "iters/s", "cores": workers, "kind": "oracle",
            "sample": "%d minimiser iterations of the same %s workload (%s); tensor set-up "
                      "excluded" % (iters, label, how)}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    if a.copy_probe > 0:
        n = int(a.copy_probe * 1e6 / 8)
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 8 * n, "launches": 5}))
        return
    if a.workload == "batched":
        ib, tb, rcb, nf, _ = run_batched(torch, True, field_step=1)
        iseq, tseq, rcs, _, _ = run_batched(torch, False, field_step=1)
        print(json.dumps({"metric": "summed minimiser iterations/s, 64 uneven platelets, "
                                    "81-field loop", "value": ib / tb, "unit": "iters/s",
                          "n_gpus": 1, "higher_is_better": True, "dtype": "f64",
                          "data": "synthetic", "batched_s": tb, "iterations": ib,
                          "per_sample": {"value": iseq / tseq, "seconds": tseq,
                                         "iterations": iseq},
                          "speedup": (ib / tb) / (iseq / tseq), "status": [rcb, rcs]}))
        return
    if a.workload == "loop":
        r = loops(torch, a.bb_switch, a.line_search)
        print(json.dumps({"metric": "H_eff evaluations and seconds per hysteresis loop "
                                    "(201 fields)", "n_gpus": 1, "data": "synthetic",
                          "bb_switch": a.bb_switch, "line_search": a.line_search,
                          "loops": r}))
        return
    if a.workload == "cube-sweep":
        r = cube_sweep(torch)
        r.update({"metric": "128^3 cube sweep 0..200 mT, FP64 vs mixed per field",
                  "n_gpus": 1, "data": "synthetic"})
        print(json.dumps(r))
        return
    if a.workload == "adjoint":
        r = run_adjoint(torch)
        r.update({"metric": "implicit gradient of <m_x>, 200x100x2 film with Ku map",
                  "n_gpus": 1, "dtype": "f64", "data": "synthetic"})
        print(json.dumps(r))
        return
    wid, field, wdesc, padded = WORKLOADS[a.workload]
    w = synth.workload(wid)
    label = "x".join(str(v) for v in w["n"])
    if a.quick:
        q = run_gpu(a.prec, a.steps, a.warmup, w, profile=False, field=field,
                    rows=a.rows_per_block, yz=a.yz_variant)
        r = {"value": q["iters"] / q["seconds"], "unit": "iters/s", "precision": a.prec,
             "steps": a.steps}
        if a.graph:
            g = run_gpu(a.prec, a.steps, a.warmup, w, profile=False, field=field, graph=True,
                        rows=a.rows_per_block, yz=a.yz_variant)
            r["graph_value"] = g["iters"] / g["seconds"]
        print(json.dumps(r))
        return
    # timed region (no events)
    main_run = run_gpu(a.prec, a.steps, a.warmup, w, profile=None, field=field)
    # same region with events around every kernel: the per-kernel breakdown
    all_run = run_gpu(a.prec, a.steps, a.warmup, w, profile="all", field=field)
    prof = all_run["prof"]
    dom = max(prof, key=lambda k: prof[k][0])
    # same region with events around the dominant kernel only: its duration
    dom_run = run_gpu(a.prec, a.steps, a.warmup, w, profile=[dom], field=field)
    other = "mixed" if a.prec == "fp64" else "fp64"
    other_run = run_gpu(other, a.steps, a.warmup, w, profile=None, field=field)
    other_prof = run_gpu(other, a.steps, a.warmup, w, profile="all", field=field)["prof"]

    ips = main_run["iters"] / main_run["seconds"]
    ms, n = dom_run["prof"][dom]
    avg_s = ms / 1e3 / max(n, 1)
    achieved = main_run["bytes"][dom] / avg_s / 1e9
    traffic = stored_traffic(a.prec, dom, a.workload)
    copy_gbps = copy_ceiling(torch)
    # launches per iteration weight each kernel (the mixed form's reference
    # pass runs once per poll_every iterations)
    per_iter_bytes = sum(main_run["bytes"][k] * v[1] / all_run["iters"]
                         for k, v in prof.items() if v[1] > 0)
    kernel_us = {k: 1e3 * v[0] / max(v[1], 1) for k, v in prof.items() if v[1] > 0}
    oips = other_run["iters"] / other_run["seconds"]
    out = {
        "metric": "minimiser iterations/s (= H_eff evals/s) at %s" % label,
        "value": ips,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * main_run["seconds"] / main_run["iters"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": wdesc, "precision": a.prec, "padded_grid": padded},
        "tile": {"rows_per_block": main_run["rows_per_block"],
                 "yz_variant": main_run["yz_variant"], "chosen_by": "autotuner"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": 8000.0,
                     "unit": "GB/s", "frac": achieved / 8000.0,
                     "traffic": traffic, "avg_kernel_us": avg_s * 1e6,
                     "algorithmic_bytes": main_run["bytes"][dom],
                     "traffic_GBps": traffic / avg_s / 1e9 if traffic else None,
                     "copy_ceiling_GBps": copy_gbps},
        "iteration": {"model_bytes": per_iter_bytes,
                      "model_GBps": per_iter_bytes * ips / 1e9,
                      "model_frac_of_8TBps": per_iter_bytes * ips / 8e12,
                      "kernel_avg_us_all_timed": kernel_us},
        other: {"value": oips, "unit": "iters/s",
                "speedup_vs_" + a.prec: oips / ips,
                "kernel_avg_us_all_timed": {k: 1e3 * v[0] / max(v[1], 1)
                                            for k, v in other_prof.items() if v[1] > 0}},
    }
    if a.workload == "film" and not a.no_cube:
        out["cube"] = cube_leg(a.cube_steps)
    if not a.no_batched:
        ib, tb, rcb, nf, bst = run_batched(torch, True)
        iseq, tseq, rcs, _, _ = run_batched(torch, False)
        out["batched"] = {"workload": "64 uneven platelets (64..256 x 32..128 x 1..2 cells), "
                                      "%d fields of the +-40 mT loop, FP64" % nf,
                          "value": ib / tb, "unit": "iters/s (summed over samples)",
                          "iterations": ib, "seconds": tb,
                          "model_GBps": bst["bytes"] / tb / 1e9,
                          "model_frac_of_8TBps": bst["bytes"] / tb / 8e12,
                          "sample_iters_max_over_mean": bst["max_sample_iters"] /
                                                        bst["mean_sample_iters"],
                          "per_sample_value": iseq / tseq, "per_sample_seconds": tseq,
                          "speedup_vs_per_sample": (ib / tb) / (iseq / tseq),
                          "status": [int(rcb), int(rcs)]}
    if not a.no_cpu:
        iters = a.cpu_iters if a.workload == "film" else max(1, a.cpu_iters // 10)
        out["cpu_baseline"] = cpu_baseline(w, iters, field, label, workers=host_cores())
        out["cpu_baseline_1core"] = cpu_baseline(w, iters, field, label, workers=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
