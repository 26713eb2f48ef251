"""Whole hysteresis loop of the 400x200x4 film (201 fields, +50 -> -50 ->
+50 mT at 1 deg): the single-precision form (FP32 convolution with its
defect correction, the default) against FP64, field by field.

The oracle cannot run this loop in reasonable time; FP64 GPU is the
reference here, validated against the oracle on the same grid (H_eff to
1e-10 in test_gpu_parity).

* At torque tolerance 1e-8 of Ms the mixed form runs from the plain start
  and from two starts perturbed by 1e-7: every field converges, every
  converged mixed state is stationary for the FP64 effective field (torque
  below 2 tol: cross-stationarity), where a run shares FP64's basin the
  states agree to |dm|_inf <= 1e-3, and on each branch at least two of the
  three runs switch within one field step of FP64 while none switches later
  than that or more than five steps earlier.  A single run's switching
  field is not determined even at this tolerance: near the coercive field
  the barrier is low and BB's non-monotone step can carry a run across it.
  Measured: with one reduction order the plain mixed run switched four
  fields early on the ascending branch (and one early on the descending
  one), while four FP64 runs and four mixed runs from 1e-7-perturbed starts
  all switched at FP64's fields; with another order the mixed run once
  stayed in another basin for fields 64-98 (then rejoined).
* At the loop's own tolerance (1e-6) the converged states are not
  determined to 1e-3 near switching: an FP64 run from a start perturbed by
  1e-7 (the scale of FP32 rounding) leaves the unperturbed run's basin after
  the first switch, as the mixed run does.  There the bound is that the
  mixed run departs from FP64 no more than that perturbed FP64 run does
  (same coercive step within one field, other-basin fields only where the
  perturbed run's are or next to a switch, same-basin |dm|_inf within twice
  the perturbed run's)."""

import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1405_2728_amd import _build
    _build.ensure_built()
    return torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def coercive_index(mavg, h, n_down):
    """First field of the descending branch with <m>.h < 0, and of the
    ascending branch with <m>.h > 0 (indices into the loop)."""
    proj = mavg @ h
    down = next((f for f in range(n_down) if proj[f] < 0), None)
    up = next((f for f in range(n_down, len(proj)) if proj[f] > 0), None)
    return down, up


def run_loops(torch, runs, tol):
    """runs: name -> (precision, perturbation of m0).  Field by field, every
    run advances one field; returns <m>, updates, statuses, |dm|_inf of
    each run against the first one after every field, and the torque of
    each run's converged state under the FP64 effective field."""
    from paper_1405_2728_amd import Context
    w = synth.workload(1)
    F = w["fields"]
    rng = np.random.default_rng(5)
    ctxs, ms = {}, {}
    for name, (prec, pert) in runs.items():
        c = Context(prec)
        c.set_geometry(0, *w["n"], *w["d"])
        c.set_material(0, w["Ms"], w["A"], w["Ku"], w["u"])
        m0 = w["m0"].copy()
        if pert:
            m0 = m0 + pert * rng.standard_normal(m0.shape)
            m0 /= np.linalg.norm(m0, axis=0, keepdims=True)
        ctxs[name] = c
        ms[name] = torch.tensor(m0, device="cuda")
    chk = Context("fp64")          # FP64 effective field of every converged state
    chk.set_geometry(0, *w["n"], *w["d"])
    chk.set_material(0, w["Ms"], w["A"], w["Ku"], w["u"])
    first = next(iter(runs))
    t64 = {k: np.zeros(len(F)) for k in runs}
    mavg = {k: np.zeros((len(F), 3)) for k in runs}
    iters = {k: np.zeros(len(F), dtype=np.int64) for k in runs}
    status = {k: [] for k in runs}
    dm = {k: np.zeros(len(F)) for k in runs}
    for f in range(len(F)):
        for k, c in ctxs.items():
            a, it, rc = c.hysteresis_sweep([ms[k]], F[f:f + 1][None], tol=tol, max_iter=400000)
            mavg[k][f] = a[0, 0]
            iters[k][f] = it[0, 0]
            status[k].append(rc)
        chk.set_field(0, F[f])
        for k in runs:
            dm[k][f] = float((ms[k] - ms[first]).abs().max())
            Hm = chk.heff(0, ms[k])
            g = torch.linalg.cross(ms[k], torch.linalg.cross(ms[k], Hm, dim=0), dim=0)
            t64[k][f] = float(g.norm(dim=0).max()) / w["Ms"]
        if f % 40 == 0:
            say("  field", f, {k: (int(iters[k][f]), "%.1e" % dm[k][f]) for k in runs})
    for c in ctxs.values():
        c.close()
    chk.close()
    h = synth.tilted(1.0)
    n_down = (len(F) + 1) // 2
    out = {}
    for k in runs:
        other = np.max(np.abs(mavg[k] - mavg[first]), axis=1) > 1e-2
        out[k] = {"coercive": coercive_index(mavg[k], h, n_down), "other": other, "dm": dm[k],
                  "status": status[k], "evals": int(iters[k].sum()) + len(F),
                  "torque64": t64[k]}
        say("  ", k, "coercive", out[k]["coercive"], "evaluations", out[k]["evals"],
            "other-basin", np.flatnonzero(other).tolist(),
            "max |dm| same basin %.2e" % (dm[k][~other].max() if (~other).any() else 0.0),
            "max FP64 torque %.2e" % t64[k].max())
    return out


def test_film_loop_mixed_matches_fp64_at_tight_tolerance(torch_cuda):
    say("case film loop, tol 1e-8")
    names = ("mixed", "mixed_p1", "mixed_p2")
    r = run_loops(torch_cuda, {"fp64": ("fp64", 0.0), "mixed": ("mixed", 0.0),
                               "mixed_p1": ("mixed", 1e-7), "mixed_p2": ("mixed", 1e-7)}, 1e-8)
    a = r["fp64"]
    assert all(s == 0 for k in r for s in r[k]["status"])
    assert a["coercive"][0] is not None and a["coercive"][1] is not None
    assert a["torque64"].max() < 1e-8
    for branch in (0, 1):
        c64 = a["coercive"][branch]
        cs = [r[k]["coercive"][branch] for k in names]
        assert all(c is not None and c64 - 5 <= c <= c64 + 1 for c in cs), (branch, c64, cs)
        assert sum(abs(c - c64) <= 1 for c in cs) >= 2, (branch, c64, cs)
    for k in names:
        b = r[k]
        assert b["torque64"].max() < 2e-8
        same = ~b["other"]
        assert b["dm"][same].max() <= 1e-3


def test_film_loop_mixed_within_fp64_sensitivity(torch_cuda):
    say("case film loop, tol 1e-6")
    r = run_loops(torch_cuda, {"fp64": ("fp64", 0.0), "mixed": ("mixed", 0.0),
                               "fp64_perturbed": ("fp64", 1e-7)}, 1e-6)
    a, b, p = r["fp64"], r["mixed"], r["fp64_perturbed"]
    assert all(s == 0 for s in a["status"] + b["status"] + p["status"])
    c64 = a["coercive"]
    assert c64[0] is not None and c64[1] is not None
    assert abs(c64[0] - b["coercive"][0]) <= 1 and abs(c64[1] - b["coercive"][1]) <= 1
    near = np.zeros(len(a["dm"]), dtype=bool)
    for cidx in c64:
        near[max(cidx - 1, 0):cidx + 2] = True
    assert not np.any(b["other"] & ~p["other"] & ~near)
    same = ~b["other"] & ~p["other"]
    assert b["dm"][same].max() <= max(2.0 * p["dm"][same].max(), 1e-3)
