"""Summaries of rocprofv3 result databases (profiling support; not on the
hot path).

  python -m paper_1405_2728_amd.profiling stats DB [--title T] [--cmd C]
      per-kernel dispatch count, average and total duration (markdown)
  python -m paper_1405_2728_amd.profiling traffic --prec P --fetch DB --write DB
          --copy-fetch DB --copy-write DB --copy-bytes B [--cmd-... C] --out JSON
      HBM bytes per launch of every kernel from FETCH_SIZE / WRITE_SIZE
      (KiB per dispatch), each scaled by the ratio of the known size of a
      plain device copy to what the same counter reports for that copy.
      The result records a hash of the HIP sources; bench.py uses it only
      while the kernels are unchanged.
  python -m paper_1405_2728_amd.profiling sq --pmc DB --trace DB [--title T] [--cmd C]
      occupancy and issue figures per kernel (markdown) from a run with
      SQ_WAVES SQ_WAVE_CYCLES SQ_ACTIVE_INST_VALU SQ_INSTS_VALU SQ_INSTS_LDS
      SQ_LDS_BANK_CONFLICT SQ_WAIT_INST_ANY, with the kernel durations of a
      kernel-trace run of the same command.
"""

import argparse
import hashlib
import json
import os
import re
import sqlite3
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def source_hash():
    """Hash of the device-kernel sources (host-side capi.hip excluded)."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1405_2728_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f == "capi.hip":
            continue
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def short_name(full):
    """mmk::k_yz_wave<double, 8, 4, true>(...) -> k_yz_wave<double,8,4,true>."""
    m = re.search(r"mmk::(k_\w+)(<[^(]*>)?", full)
    if m:
        return m.group(1) + (m.group(2) or "").replace(" ", "")
    return full.split("(")[0][:60]


def kernel_stats(db):
    """Per (kernel, launch shape): calls, average and total duration.  Launches
    of one kernel with other shapes (the tile autotuner's timing runs, set-up)
    get rows of their own."""
    con = sqlite3.connect(db)
    rows = con.execute("select name, duration, grid_x, workgroup_x from kernels").fetchall()
    agg = defaultdict(list)
    for name, dur, gx, wx in rows:
        agg[(short_name(name), int(gx) // max(int(wx), 1), int(wx))].append(dur)
    return {k: {"calls": len(v), "avg_us": sum(v) / len(v) / 1e3, "total_ms": sum(v) / 1e6}
            for k, v in agg.items()}


def counter_means(db, counter, counts=None):
    """Mean of `counter` per kernel over the dispatches of its most frequent
    launch shape (so that the tile autotuner's timing launches of other
    shapes do not enter the figure); `counts` (a dict), if given, receives
    the number of those dispatches per kernel."""
    con = sqlite3.connect(db)
    agg = defaultdict(lambda: defaultdict(list))
    for name, gx, wx, cn, val in con.execute(
            "select kernel_name, grid_size_x, workgroup_size_x, counter_name, value "
            "from counters_collection"):
        if cn == counter:
            agg[short_name(name)][int(gx) // max(int(wx), 1)].append(val)
    out = {}
    for k, shapes in agg.items():
        v = max(shapes.values(), key=len)
        out[k] = sum(v) / len(v)
        if counts is not None:
            counts[k] = len(v)
    return out


def cmd_stats(a):
    st = kernel_stats(a.db)
    lines = ["# %s" % (a.title or os.path.basename(a.db)), ""]
    if a.cmd:
        lines += ["Command: `%s`" % a.cmd, ""]
    lines += ["| kernel | blocks | threads/block | calls | avg us | total ms |",
              "|---|---:|---:|---:|---:|---:|"]
    for k, v in sorted(st.items(), key=lambda kv: -kv[1]["total_ms"]):
        lines.append("| %s | %d | %d | %d | %.2f | %.3f |" % (k[0], k[1], k[2], v["calls"],
                                                          v["avg_us"], v["total_ms"]))
    print("\n".join(lines))


N_CU = 256             # compute units of the device (4 SIMDs each)
CLOCK_HZ = 2.4e9       # peak engine clock


def cmd_sq(a):
    """Per kernel (its most frequent launch shape): waves, mean resident waves
    per CU and per SIMD over the kernel's duration, VALU issue fraction per
    SIMD, share of wave time spent waiting on memory or LDS counters, LDS
    bank-conflict cycles per LDS instruction.  SQ_WAVE_CYCLES,
    SQ_ACTIVE_INST_VALU and SQ_WAIT_INST_ANY count in units of 4 cycles."""
    names = ("SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_ACTIVE_INST_VALU", "SQ_INSTS_VALU",
             "SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_WAIT_INST_ANY")
    vals = {n: counter_means(a.pmc, n) for n in names}
    dur = {k[0]: v["avg_us"] for k, v in sorted(kernel_stats(a.trace).items(),
                                                   key=lambda kv: kv[1]["calls"])}
    lines = ["# %s" % (a.title or os.path.basename(a.pmc)), ""]
    if a.cmd:
        lines += ["Commands: %s" % a.cmd, ""]
    lines += ["Kernel time from the kernel-trace run; SQ_WAVE_CYCLES, SQ_ACTIVE_INST_VALU "
              "and SQ_WAIT_INST_ANY in units of 4 cycles at %.1f GHz; %d CUs of 4 SIMDs." %
              (CLOCK_HZ / 1e9, N_CU), "",
              "| kernel | us | waves | VALU instr / wave | resident waves / CU | "
              "per SIMD | VALU busy / SIMD | waiting share | LDS conflict cycles / LDS instr |",
              "|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for k in sorted(vals["SQ_WAVES"], key=lambda k: -dur.get(k, 0.0)):
        if k not in dur or dur[k] <= 0:
            continue
        cyc = dur[k] * 1e-6 * CLOCK_HZ
        w = vals["SQ_WAVES"][k]
        wc = 4 * vals["SQ_WAVE_CYCLES"].get(k, 0.0)
        res = wc / (cyc * N_CU)
        busy = 4 * vals["SQ_ACTIVE_INST_VALU"].get(k, 0.0) / (cyc * N_CU * 4)
        wait = 4 * vals["SQ_WAIT_INST_ANY"].get(k, 0.0) / wc if wc else 0.0
        lds = vals["SQ_INSTS_LDS"].get(k, 0.0)
        conf = vals["SQ_LDS_BANK_CONFLICT"].get(k, 0.0) / lds if lds else 0.0
        lines.append("| %s | %.2f | %d | %.0f | %.2f | %.2f | %.2f | %.2f | %.2f |" % (
            k, dur[k], w, vals["SQ_INSTS_VALU"].get(k, 0.0) / max(w, 1), res, res / 4, busy,
            wait, conf))
    print("\n".join(lines))


def cmd_traffic(a):
    cf = counter_means(a.copy_fetch, "FETCH_SIZE")
    cw = counter_means(a.copy_write, "WRITE_SIZE")
    # the copy kernel is the one that both reads and writes the most (the
    # probe's fill of the source only writes)
    ckey = max((k for k in cf if k in cw), key=lambda k: min(cf[k], cw[k]))
    f_fetch = a.copy_bytes / (cf[ckey] * 1024.0)
    f_write = a.copy_bytes / (cw[ckey] * 1024.0)
    launches = {}
    fe = counter_means(a.fetch, "FETCH_SIZE", launches)
    wr = counter_means(a.write, "WRITE_SIZE")
    kernels = {}
    for k in set(fe) | set(wr):
        fb = fe.get(k, 0.0) * 1024.0 * f_fetch
        wb = wr.get(k, 0.0) * 1024.0 * f_write
        kernels[k] = {"fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb}
    # bench.py looks kernels up by the library's timing names
    alias = {"k_xf_w": "xf", "k_xf": "xf", "k_yz_wave": "yz_thin", "k_yz_thin": "yz_thin",
             "k_xil_w": "xil", "k_xil": "xil", "k_update": "update", "k_y3_fwd": "y3_fwd",
             "k_z3": "z3", "k_y3_inv": "y3_inv"}
    # several instantiations of one pass (the mixed form's double-precision
    # reference pass, for one): the timing name takes the most launched one
    for k in sorted(kernels, key=lambda k: -launches.get(k, 0)):
        base = k.split("<")[0]
        if base in alias:
            kernels.setdefault(alias[base], dict(kernels[k], instance=k))
    out = {"precision": a.prec, "source_hash": source_hash(),
           "calibration": {"copy_kernel": ckey, "copy_bytes": a.copy_bytes,
                           "fetch_factor": f_fetch, "write_factor": f_write},
           "commands": {"fetch": a.cmd_fetch, "write": a.cmd_write,
                        "copy_fetch": a.cmd_copy_fetch, "copy_write": a.cmd_copy_write},
           "kernels": kernels}
    with open(a.out, "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
    print(json.dumps(out, indent=1, sort_keys=True))


def main(argv=None):
    p = argparse.ArgumentParser()
    sub = p.add_subparsers(dest="cmd_name", required=True)
    s = sub.add_parser("stats")
    s.add_argument("db")
    s.add_argument("--title", default="")
    s.add_argument("--cmd", default="")
    t = sub.add_parser("traffic")
    t.add_argument("--prec", required=True)
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        t.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
        t.add_argument("--cmd-" + k.replace("_", "-"), dest="cmd_" + k, default="")
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--out", required=True)
    q = sub.add_parser("sq")
    q.add_argument("--pmc", required=True)
    q.add_argument("--trace", required=True)
    q.add_argument("--title", default="")
    q.add_argument("--cmd", default="")
    a = p.parse_args(argv)
    if a.cmd_name == "stats":
        cmd_stats(a)
    elif a.cmd_name == "sq":
        cmd_sq(a)
    else:
        cmd_traffic(a)


if __name__ == "__main__":
    main(sys.argv[1:])
