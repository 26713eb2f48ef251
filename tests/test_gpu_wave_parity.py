"""Step-by-step parity of the benchmarked kernels with the CPU oracle.

Every grid here pads to transform lengths that take the wave-FFT kernels
(x: M = Px/2 in 64..512, a multiple of 64; y: Py in 64..512, a multiple of
64; at most 4 layers), so the runs go through the fused forward x pass with
the pending midpoint update of eq. (7), the wave yz pass with the tensor
product and the fused inverse x pass with the local terms and the BB sums,
then the one-block finish (stop rule and step of eq. (12)) -- the kernels
`bench.py` times.  The iterates come from runs to tolerance 0 with
max_iter = k (the device-driven loop), not from single steps.

Bounds (the first 10 tau_k and m_k agree to 1e-8 relative):
* near-uniform starts: m_k (max abs over cells and components), tau_k,
  torque_k and U(m_k) within 1e-8 relative;
* random start: the first BB steps rotate cells by up to ~pi and amplify
  rounding by a factor of several million in 10 iterations.  The oracle
  started from m0 perturbed by 1e-15 (relative) moves away from its own
  unperturbed run by ~4e-9 on the 64 x 32 x 2 grid; the library differs from
  the oracle's arithmetic by rounding in every evaluation (effective field
  ~1e-15 relative, another FFT, another tensor evaluation, the closed-form
  update), which is several such perturbations.  Bound on m_k: 10x the
  largest departure of the oracle from five perturbed starts, measured in
  the test (the library measured 5x); tau_k, torque_k and U(m_k): 1e-8.
"""

import sys

import numpy as np
import pytest

import synth
from oracle import fields as of, minimizer as om

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def wave_lengths(nx, ny, nz):
    """Padded lengths of the thin-film path with mixed-radix padding (as the
    library documents them): x 2nx-1 up to the smaller of the power of two and
    the multiple of 128; y 2ny-1 up to the smaller of the power of two and the
    multiple of 64."""
    def pad(n, unit, cap):
        p = 1
        while p < n:
            p *= 2
        q = -(-n // unit) * unit
        return q if (q < p and q <= cap) else p
    Px = pad(2 * nx - 1, 128, 1024)
    Py = pad(2 * ny - 1, 64, 512)
    return Px // 2, Py


def on_wave_path(nx, ny, nz):
    M, Py = wave_lengths(nx, ny, nz)
    return nz <= 4 and M % 64 == 0 and 64 <= M <= 512 and Py % 64 == 0 and 64 <= Py <= 512


def context(torch_cuda, n, d, Ms, A, Ku, u, H, rows=0, prec="fp64"):
    from paper_1405_2728_amd import Context
    ctx = Context(prec)
    if rows:
        ctx.set_option("rows_per_block", rows)
    ctx.set_geometry(0, *n, *d)
    ctx.set_material(0, Ms, A, Ku, u)
    ctx.set_field(0, H)
    return ctx


def fused_iterates(torch, ctx, m0, kmax):
    """m_k, tau_{k-1}, torque_k, U(m_k) for k = 0..kmax from runs to
    tolerance 0 with max_iter = k, each from m0."""
    ms, taus, torques, energies = [], [], [], []
    for k in range(kmax + 1):
        m = torch.tensor(m0, device="cuda")
        r = ctx.minimize_to_tol(0, m, tol=0.0, max_iter=k)
        st = ctx.last_step(0)
        assert r["iters"] == k and r["heff_evals"] == k + 1 and st["k"] == k
        ms.append(m.cpu().numpy())
        taus.append(st["tau"])
        torques.append(r["torque"])
        energies.append(r["energy"])
    return ms, taus[1:], torques, energies


def compare(ref, ms, taus, torques, energies):
    em = max(float(np.max(np.abs(a - b))) for a, b in zip(ms, ref["states"]))
    et = float(np.max(np.abs(np.array(taus) / np.array(ref["taus"]) - 1)))
    eT = float(np.max(np.abs(np.array(torques) / np.array(ref["torques"]) - 1)))
    eU = float(np.max(np.abs(np.array(energies) / np.array(ref["energies"]) - 1)))
    return em, et, eT, eU


# (name, grid, cell sizes, start, field in A/m, rows per block: 0 = automatic)
CASES = [
    # the benchmark's grid, start, field and tile (896-point x and 448-point y
    # transforms, 4 layers, one row per x block: 800 per-block sums)
    ("film400x200x4", (400, 200, 4), (5e-9,) * 3, "bench", None, 1),
    # one shape per transform-length class
    ("64x32x2", (64, 32, 2), (5e-9,) * 3, "noise", (2e4, 3e3, 0.0), 0),
    ("200x100x2", (200, 100, 2), (5e-9,) * 3, "noise", (-1.5e4, 2e3, 500.0), 0),
    ("385x193x1", (385, 193, 1), (5e-9,) * 3, "noise", (3e4, -4e3, 0.0), 0),
    ("448x224x2", (448, 224, 2), (4e-9, 5e-9, 3e-9), "noise", (1e4, 1e4, 2e3), 0),
    # the 200x100x2 grid with four rows per x block and two (other tiles)
    ("200x100x2_R2", (200, 100, 2), (5e-9,) * 3, "noise", (-1.5e4, 2e3, 500.0), 2),
]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1405_2728_amd import _build
    _build.ensure_built()
    return torch


@pytest.mark.parametrize("name,n,d,start,H,rows", CASES, ids=[c[0] for c in CASES])
def test_fused_iterates_match_oracle(torch_cuda, name, n, d, start, H, rows):
    torch = torch_cuda
    assert on_wave_path(*n)
    say("case fused iterates", name, n, "rows", rows)
    if start == "bench":
        w = synth.workload(1)
        m0, H = w["m0"], w["fields"][0]
        mat = (w["Ms"], w["A"], w["Ku"], w["u"])
    else:
        rng = np.random.default_rng(sum(n) + 7)
        m0 = synth.uniform_with_noise((1, 0.3, 0.1), *n, 0.05, rng)
        mat = (8e5, 1.3e-11, 800.0, (1, 0, 0))
    P = of.Problem(*n, *d, Ms=mat[0], A=mat[1], Ku=mat[2], u=mat[3], H_ext=H)
    ref = om.minimize(P, m0, tol=0.0, max_iter=10, record=True, keep_states=True)
    ctx = context(torch, n, d, *mat, H, rows)
    if rows:
        assert ctx.rows_per_block(0) == rows
    ms, taus, torques, energies = fused_iterates(torch, ctx, m0, 10)
    ctx.close()
    em, et, eT, eU = compare(ref, ms, taus, torques, energies)
    say("  m %.2e  tau %.2e  torque %.2e  energy %.2e" % (em, et, eT, eU))
    assert em < 1e-8 and et < 1e-8 and eT < 1e-8 and eU < 1e-8


def test_fused_iterates_random_start(torch_cuda):
    """Random start on the 64-point wave path: bounded by the oracle's own
    sensitivity to a rounding-level perturbation of m0."""
    torch = torch_cuda
    n, d = (64, 32, 2), (5e-9,) * 3
    H = (2e4, 3e3, 0.0)
    rng = np.random.default_rng(11)
    m0 = synth.random_unit(*n, rng)
    P = of.Problem(*n, *d, Ms=8e5, A=1.3e-11, Ku=500.0, H_ext=H)
    ref = om.minimize(P, m0, tol=0.0, max_iter=10, record=True, keep_states=True)
    self_dev = 0.0
    for seed in range(5):
        p = np.random.default_rng(100 + seed).standard_normal(m0.shape)
        alt = om.minimize(P, om.normalise(m0 + 1e-15 * p), tol=0.0, max_iter=10)
        self_dev = max(self_dev, float(np.max(np.abs(alt["m"] - ref["m"]))))
    ctx = context(torch, n, d, 8e5, 1.3e-11, 500.0, (1, 0, 0), H)
    ms, taus, torques, energies = fused_iterates(torch, ctx, m0, 10)
    ctx.close()
    em, et, eT, eU = compare(ref, ms, taus, torques, energies)
    bound = max(1e-8, 10 * self_dev)
    say("  random start: m %.2e tau %.2e torque %.2e energy %.2e; oracle self-departure %.2e"
        % (em, et, eT, eU, self_dev))
    assert em < bound and et < 1e-8 and eT < 1e-8 and eU < 1e-8


def test_bb_switch_on_wave_path(torch_cuda):
    """The ratio switch between the two steps of eq. (12) (option bb_switch)
    on the fused kernels: iterates and a run to tolerance follow the
    oracle's rule."""
    torch = torch_cuda
    n, d = (64, 32, 2), (5e-9,) * 3
    kappa = 0.5
    H = (2e4, 3e3, 0.0)
    rng = np.random.default_rng(13)
    m0 = synth.uniform_with_noise((1, 0.2, 0), *n, 0.05, rng)
    P = of.Problem(*n, *d, Ms=8e5, A=1.3e-11, Ku=500.0, H_ext=H)
    ref = om.minimize(P, m0, tol=0.0, max_iter=12, record=True, bb_switch=kappa,
                      keep_states=True)
    alt = om.minimize(P, m0, tol=0.0, max_iter=12, record=True)
    assert not np.array_equal(ref["taus"], alt["taus"])
    from paper_1405_2728_amd import Context
    ctx = Context("fp64")
    ctx.set_option("bb_switch", kappa)
    ctx.set_geometry(0, *n, *d)
    ctx.set_material(0, 8e5, 1.3e-11, 500.0, (1, 0, 0))
    ctx.set_field(0, H)
    ms, taus, torques, energies = fused_iterates(torch, ctx, m0, 12)
    em, et, eT, eU = compare(ref, ms, taus, torques, energies)
    say("  bb_switch: m %.2e tau %.2e torque %.2e energy %.2e" % (em, et, eT, eU))
    assert em < 1e-8 and et < 1e-8 and eT < 1e-8 and eU < 1e-8
    m = torch.tensor(m0, device="cuda")
    r = ctx.minimize_to_tol(0, m, tol=1e-7, max_iter=100000)
    full = om.minimize(P, m0, tol=1e-7, bb_switch=kappa)
    say("  iters gpu", r["iters"], "oracle", full["iters"])
    assert r["converged"] and full["converged"]
    mg = m.cpu().numpy()
    assert om.torque(mg, P.heff(mg), P.Ms) < 1e-7 * 1.0001
    assert np.max(np.abs(mg - full["m"])) < 1e-4
    assert abs(r["energy"] - full["energy"]) < 1e-9 * abs(full["energy"])
    ctx.close()


def test_random_start_sweep_on_wave_path(torch_cuda):
    """Workload 0's recipe (random start, H = 0, 4, ..., 20 mT at 1 degree,
    tol 1e-6) on a 64 x 32 x 1 film, whose transforms take the wave kernels:
    the device-driven sweep against the oracle's sweep."""
    torch = torch_cuda
    n, d = (64, 32, 1), (5e-9,) * 3
    rng = synth.rng_for(0)
    m0 = synth.random_unit(*n, rng)
    fields = synth.workload(0)["fields"]
    mat = synth.PERMALLOY
    from paper_1405_2728_amd import Context
    ctx = Context("fp64")
    ctx.set_geometry(0, *n, *d)
    ctx.set_material(0, mat["Ms"], mat["A"], mat["Ku"], mat["u"])
    m = torch.tensor(m0, device="cuda")
    mavg, iters, rc = ctx.hysteresis_sweep([m], fields, tol=1e-6)
    ctx.close()
    P = of.Problem(*n, *d, **mat)
    ref = om.sweep(P, m0, fields, tol=1e-6)
    say("  gpu iters", iters[0].tolist(), "oracle", ref["iters"].tolist())
    assert rc == 0 and ref["converged"].all()
    mg = m.cpu().numpy()
    P.H_ext = fields[-1]
    assert om.torque(mg, P.heff(mg), P.Ms) < 1e-6 * 1.0001
    # a random start may relax into another metastable state; where the
    # final states share a basin the loop agrees field by field
    if np.max(np.abs(mg - ref["m"])) < 1e-3:
        assert np.max(np.abs(mavg[0] - ref["mavg"])) < 1e-3
    else:
        say("  final states in different basins (allowed from a random start)")


def test_converged_start_costs_one_evaluation(torch_cuda):
    """A start that already meets the stop rule: no update, one evaluation
    (the stop test comes before every update), on the benchmark's kernels."""
    torch = torch_cuda
    n, d = (200, 100, 2), (5e-9,) * 3
    rng = np.random.default_rng(3)
    m0 = synth.uniform_with_noise((1, 0, 0), *n, 1e-3, rng)
    H = (2e4, 300.0, 0.0)
    ctx = context(torch, n, d, 8e5, 1.3e-11, 500.0, (1, 0, 0), H)
    m = torch.tensor(m0, device="cuda")
    r = ctx.minimize_to_tol(0, m, tol=1e-7)
    assert r["converged"]
    before = m.clone()
    r2 = ctx.minimize_to_tol(0, m, tol=1e-7)
    ctx.close()
    assert r2["converged"] and r2["iters"] == 0 and r2["heff_evals"] == 1
    assert torch.equal(m, before)
    P = of.Problem(*n, *d, Ms=8e5, A=1.3e-11, Ku=500.0, H_ext=H)
    mg = m.cpu().numpy()
    assert om.torque(mg, P.heff(mg), P.Ms) < 1e-7 * 1.0001


def test_zero_denominator_keeps_previous_step(torch_cuda):
    """Guard of eq. (12) on the device: with tau0 = 1e-300 every update moves
    m = +x by ~1e-296, so s.s, s.y and y.y underflow to exactly 0, both
    quotients are 0/0 and each step keeps the previous tau (tau0); the oracle
    does the same.  Wave-path grid, run to tolerance 0."""
    torch = torch_cuda
    n, d = (64, 32, 1), (5e-9,) * 3
    H = (1e4, 2e3, 0.0)
    tau0 = 1e-300
    m0 = np.zeros((3,) + n[::-1])
    m0[0] = 1.0
    from paper_1405_2728_amd import Context
    ctx = Context("fp64")
    ctx.set_option("tau0", tau0)
    ctx.set_geometry(0, *n, *d)
    ctx.set_material(0, 8e5, 1.3e-11, 500.0, (1, 0, 0))
    ctx.set_field(0, H)
    P = of.Problem(*n, *d, Ms=8e5, A=1.3e-11, Ku=500.0, H_ext=H)
    ref = om.minimize(P, m0, tol=0.0, max_iter=6, tau0=tau0, record=True, keep_states=True)
    assert all(t == tau0 for t in ref["taus"]) and ref["torques"][0] > 1e-3
    ms, taus, torques, energies = fused_iterates(torch, ctx, m0, 6)
    ctx.close()
    assert all(t == tau0 for t in taus)
    em, et, eT, eU = compare(ref, ms, taus, torques, energies)
    say("  guard: m %.2e tau %.2e torque %.2e energy %.2e" % (em, et, eT, eU))
    assert em < 1e-12 and eT < 1e-8 and eU < 1e-8


# ---- non-monotone line search (option line_search; oracle minimize_ls) ----------
def ls_context(torch, n, d, H, tau0, mat=(8e5, 1.3e-11, 500.0, (1, 0, 0)), n_samples=1):
    from paper_1405_2728_amd import Context
    ctx = Context("fp64", n_samples=n_samples)
    ctx.set_option("line_search", 1)
    ctx.set_option("tau0", tau0)
    for k in range(n_samples):
        ctx.set_geometry(k, *n, *d)
        ctx.set_material(k, *mat)
        ctx.set_field(k, H)
    return ctx


def test_line_search_iterates_match_oracle(torch_cuda):
    """A first step far too long (tau0 = 3 / Ms): the device rejects and
    shortens trials exactly as the oracle's line search does; accepted
    states m_k, their steps, torques, energies and the evaluation counts
    (rejected trials included) agree for k = 0..10 on the fused kernels."""
    torch = torch_cuda
    n, d = (64, 32, 2), (5e-9,) * 3
    H = (2e4, 3e3, 0.0)
    tau0 = 3.0 / 8e5
    rng = np.random.default_rng(17)
    m0 = synth.uniform_with_noise((1, 0.3, 0.1), *n, 0.2, rng)
    P = of.Problem(*n, *d, Ms=8e5, A=1.3e-11, Ku=500.0, H_ext=H)
    ctx = ls_context(torch, n, d, H, tau0)
    back = 0
    for k in range(11):
        ref = om.minimize_ls(P, m0, tol=0.0, max_iter=k, tau0=tau0, record=True)
        m = torch.tensor(m0, device="cuda")
        r = ctx.minimize_to_tol(0, m, tol=0.0, max_iter=k)
        st = ctx.last_step(0)
        em = float(np.max(np.abs(m.cpu().numpy() - ref["m"])))
        say("  k %d evals gpu %d oracle %d backtracks %d |dm| %.2e" % (
            k, r["heff_evals"], ref["heff_evals"], ref["backtracks"], em))
        assert r["iters"] == k and r["heff_evals"] == ref["heff_evals"]
        assert em < 1e-8
        assert abs(r["torque"] / ref["torque"] - 1) < 1e-8
        assert abs(r["energy"] / ref["energy"] - 1) < 1e-8
        if k > 0:
            assert abs(st["tau"] / ref["taus"][-1] - 1) < 1e-8
        back = ref["backtracks"]
    ctx.close()
    assert back >= 1            # the case exercises rejections


def test_line_search_run_and_sweep(torch_cuda):
    """Runs to tolerance with the line search: the device reaches the
    oracle's state (same basin, energy 1e-9) with an evaluation count within
    10% of the oracle's; a two-sample sweep (per-sample launches: the batched
    form excludes the line search) equals two one-sample sweeps bit for bit
    and follows the oracle's sweep."""
    torch = torch_cuda
    n, d = (64, 32, 2), (5e-9,) * 3
    H = (2e4, 3e3, 0.0)
    rng = np.random.default_rng(19)
    m0 = synth.uniform_with_noise((1, 0.3, 0.1), *n, 0.2, rng)
    P = of.Problem(*n, *d, Ms=8e5, A=1.3e-11, Ku=500.0, H_ext=H)
    ref = om.minimize_ls(P, m0, tol=1e-7)
    ctx = ls_context(torch, n, d, H, 1e-3 / 8e5)
    m = torch.tensor(m0, device="cuda")
    r = ctx.minimize_to_tol(0, m, tol=1e-7)
    ctx.close()
    say("  run: evals gpu %d oracle %d" % (r["heff_evals"], ref["heff_evals"]))
    assert r["converged"] and ref["converged"]
    mg = m.cpu().numpy()
    assert om.torque(mg, P.heff(mg), P.Ms) < 1e-7 * 1.0001
    assert np.max(np.abs(mg - ref["m"])) < 1e-4
    assert abs(r["energy"] - ref["energy"]) < 1e-9 * abs(ref["energy"])
    assert abs(r["heff_evals"] / ref["heff_evals"] - 1) < 0.1
    # sweeps
    F = synth.loop_fields(20.0, 5.0, synth.tilted(10.0))
    two = ls_context(torch, n, d, H, 1e-3 / 8e5, n_samples=2)
    ms = [torch.tensor(m0, device="cuda"), torch.tensor(m0, device="cuda")]
    mavg2, it2, rc2 = two.hysteresis_sweep(ms, np.stack([F, F]), tol=1e-6)
    two.close()
    one = ls_context(torch, n, d, H, 1e-3 / 8e5)
    m1 = torch.tensor(m0, device="cuda")
    mavg1, it1, rc1 = one.hysteresis_sweep([m1], F, tol=1e-6)
    one.close()
    assert rc1 == 0 and rc2 == 0
    assert np.array_equal(mavg2[0], mavg1[0]) and np.array_equal(mavg2[1], mavg1[0])
    assert torch.equal(ms[0], m1) and torch.equal(ms[1], m1)
    Q = of.Problem(*n, *d, Ms=8e5, A=1.3e-11, Ku=500.0)
    osw = om.sweep(Q, m0, F, tol=1e-6, line_search=True)
    say("  sweep <m> max diff %.2e" % np.max(np.abs(mavg1[0] - osw["mavg"])))
    assert np.max(np.abs(mavg1[0] - osw["mavg"])) < 1e-3
