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
    """Mean of `counter` per kernel; `counts` (a dict), if given, receives
    the number of dispatches per kernel."""
    con = sqlite3.connect(db)
    agg = defaultdict(list)
    for name, cn, val in con.execute(
            "select kernel_name, counter_name, value from counters_collection"):
        if cn == counter:
            agg[short_name(name)].append(val)
    if counts is not None:
        counts.update({k: len(v) for k, v in agg.items()})
    return {k: sum(v) / len(v) for k, v in agg.items()}


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
    a = p.parse_args(argv)
    if a.cmd_name == "stats":
        cmd_stats(a)
    else:
        cmd_traffic(a)


if __name__ == "__main__":
    main(sys.argv[1:])
