"""Writes the oracle's Standard Problem 1 stand-in hysteresis loops.

Calls only the CPU oracle (`oracle/`) and the seeded inputs (`synth/`): the
2000 x 1000 x 20 nm permalloy film at 10 nm cells (200 x 100 x 2), field
along the long (or short) edge tilted by 1 degree, +-50 mT in 1 mT steps,
relaxed to max|m x (m x H_eff)|/Ms < 1e-6 at every field, warm-started
from the previous field (paper Sec. 4: loop of Fig. 1 / Fig. 3(c), mesh of
the Tab. 1 comparison).  Stores, per field, the mean magnetisation, the
number of updates, the energy and whether the stop rule was met, plus the
coercive field indices (first field of each branch at which <m>.h changes
sign).

Usage:  python tests/golden/make_sp1_loop.py long|short   (about 1-2 hours)
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import fields as of, minimizer as om  # noqa: E402


def coercive_indices(mavg, h):
    """First index of the descending branch with <m>.h < 0 and of the
    ascending branch with <m>.h > 0 (None where the sign never changes)."""
    proj = mavg @ h
    nd = (len(proj) + 1) // 2
    down = next((f for f in range(nd) if proj[f] < 0), None)
    up = next((f for f in range(nd, len(proj)) if proj[f] > 0), None)
    return down, up


def main(edge):
    w = synth.sp1_loop(edge, 10e-9, 1.0)
    P = of.Problem(*w["n"], *w["d"], Ms=w["Ms"], A=w["A"], Ku=w["Ku"], u=w["u"])
    m = om.normalise(np.array(w["m0"]))
    fields = w["fields"]
    out = os.path.join(HERE, "sp1_10nm_%s_edge.json" % edge)
    rec = {"source": "oracle sweep (Sec. 2 minimiser, Sec. 4 loop); written by "
                     "tests/golden/make_sp1_loop.py from synth.sp1_loop(%r, 10e-9, 1.0)" % edge,
           "n": list(w["n"]), "cell": w["d"][0], "tol": w["tol"], "h": list(w["h"]),
           "mavg": [], "iters": [], "energy": [], "converged": []}
    t0 = time.time()
    for f, H in enumerate(fields):
        P.H_ext = H.copy()
        r = om.minimize(P, m, tol=w["tol"], max_iter=100000)
        m = r["m"]
        rec["mavg"].append([float(v) for v in m.reshape(3, -1).mean(axis=1)])
        rec["iters"].append(int(r["iters"]))
        rec["energy"].append(float(r["energy"]))
        rec["converged"].append(bool(r["converged"]))
        print("field %3d  iters %6d  <m> %s  %.0f s" % (f, r["iters"],
              np.round(rec["mavg"][-1], 4), time.time() - t0), flush=True)
    down, up = coercive_indices(np.array(rec["mavg"]), np.array(w["h"]))
    rec["coercive_index"] = [down, up]
    rec["evals_per_loop"] = int(sum(rec["iters"]) + len(fields))
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=0)
    print("wrote", out, "coercive indices", down, up, flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "long")
