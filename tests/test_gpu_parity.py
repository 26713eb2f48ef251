"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances (max-norm over all cells and components, relative to the
reference's max-norm):
* FP64 effective field 1e-10: FFT rounding is ~1e-15 log2(N); the near-field
  Newell closed form in double loses up to ~3e-11 relative to cancellation
  (the oracle evaluates it in 64-bit-mantissa precision), which enters H
  scaled by the small tensor entries near the 6-cell switch.
* mixed (FP32 convolution) effective field 1e-5 (single-precision FFTs of
  length ~1e3 give ~1e-6).
* iterates (10 steps): near-uniform start 1e-11 on m, 1e-9 on tau; random
  start (chaotic amplification of rounding) 10x the oracle's own departure
  from a start perturbed by 1e-15, tau 1e-8.  The benchmarked kernels'
  iterates are compared in test_gpu_wave_parity.py.
"""

import sys

import numpy as np
import pytest

import synth
from oracle import fields as of, minimizer as om

pytestmark = pytest.mark.gpu

MU0 = 4e-7 * np.pi


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


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def make(torch, prec, nx, ny, nz, d, Ms=8e5, A=1.3e-11, Ku=500.0, u=(1, 0, 0), H=(0, 0, 0),
         ku_map=None):
    from paper_1405_2728_amd import Context
    ctx = Context(prec)
    ctx.set_geometry(0, nx, ny, nz, *d)
    km = None if ku_map is None else torch.tensor(ku_map, dtype=torch.float64, device="cuda")
    ctx.set_material(0, Ms, A, Ku, u, km)
    ctx.set_field(0, H)
    P = of.Problem(nx, ny, nz, *d, Ms=Ms, A=A, Ku=Ku if ku_map is None else ku_map, u=u, H_ext=H)
    return ctx, P


SHAPES = [
    ((5, 4, 1), (5e-9, 5e-9, 5e-9)),
    ((6, 3, 2), (5e-9, 4e-9, 3e-9)),
    ((7, 5, 3), (2e-9, 3e-9, 2.5e-9)),
    ((1, 4, 2), (5e-9, 5e-9, 5e-9)),
    ((4, 1, 2), (5e-9, 5e-9, 5e-9)),
    ((1, 1, 1), (5e-9, 5e-9, 5e-9)),
    ((2, 2, 4), (5e-9, 5e-9, 5e-9)),
    ((33, 17, 4), (5e-9, 5e-9, 5e-9)),
    ((32, 16, 1), (5e-9, 5e-9, 5e-9)),
    ((64, 9, 1), (3e-9, 5e-9, 4e-9)),
    ((13, 40, 2), (5e-9, 5e-9, 5e-9)),
    # every wave x-pass length with 4 rows per block (M = 64 .. 256) and 2 (M = 512)
    ((200, 100, 2), (5e-9, 5e-9, 5e-9)),
    ((150, 37, 1), (4e-9, 5e-9, 6e-9)),
    ((90, 7, 3), (5e-9, 5e-9, 5e-9)),
    ((300, 5, 1), (5e-9, 5e-9, 5e-9)),
    # mixed-radix transform lengths 64 VL: VL = 7 at both ends of its range
    # (x 896, y 448; 2n - 1 just above 768 / 384, and exactly 896 / 448), then
    # VL = 3 (x 384, y 192), 5 (640, 320) and 6 (768, 384)
    ((385, 193, 1), (5e-9, 5e-9, 5e-9)),
    ((448, 224, 2), (4e-9, 5e-9, 3e-9)),
    ((150, 80, 2), (5e-9, 5e-9, 5e-9)),
    ((290, 140, 1), (4e-9, 5e-9, 6e-9)),
    ((350, 180, 3), (5e-9, 5e-9, 5e-9)),
    # LDS-FFT x passes beyond the wave lengths, up to the longest rows (Px 4096)
    ((1100, 4, 2), (5e-9, 5e-9, 5e-9)),
    ((2048, 3, 1), (5e-9, 5e-9, 5e-9)),
]


@pytest.mark.parametrize("shape,d", SHAPES)
def test_heff_terms_fp64(torch_cuda, shape, d):
    torch = torch_cuda
    nx, ny, nz = shape
    say("case heff fp64", shape, d)
    rng = np.random.default_rng(nx * 100 + ny * 10 + nz)
    m0 = synth.random_unit(nx, ny, nz, rng)
    H = (2.3e4, -4e3, 1.1e4)
    ctx, P = make(torch, "fp64", nx, ny, nz, d, Ku=3e4, u=(0.6, 0.0, 0.8), H=H)
    m = torch.tensor(m0, device="cuda")
    Hg = ctx.heff(0, m).cpu().numpy()
    Ho = P.heff(m0)
    e = rel(Hg, Ho)
    say("  H_eff rel err", e)
    assert e < 1e-10
    hd, hex_, han = (t.cpu().numpy() for t in ctx.field_terms(0, m))
    t = P.field_terms(m0)
    scale = np.max(np.abs(Ho))
    assert np.max(np.abs(hd - t["demag"])) < 1e-10 * scale
    assert np.max(np.abs(hex_ - t["exchange"])) < 1e-12 * scale
    assert np.max(np.abs(han - t["anisotropy"])) < 1e-12 * scale
    E, terms = ctx.energy(0, m)
    Eo = P.energy_terms(m0)
    assert abs(E - sum(Eo)) < 1e-10 * sum(abs(x) for x in Eo)
    for a, b in zip(terms, Eo):
        assert abs(a - b) < 1e-10 * sum(abs(x) for x in Eo)
    ctx.close()


def test_heff_ku_map_and_determinism(torch_cuda):
    torch = torch_cuda
    nx, ny, nz = 24, 10, 2
    d = (5e-9,) * 3
    say("case ku map", (nx, ny, nz))
    rng = np.random.default_rng(5)
    m0 = synth.random_unit(nx, ny, nz, rng)
    ku = 500.0 * (1 + 0.1 * rng.standard_normal((nz, ny, nx)))
    ctx, P = make(torch, "fp64", nx, ny, nz, d, ku_map=ku, H=(1e3, 2e3, 3e3))
    m = torch.tensor(m0, device="cuda")
    a = ctx.heff(0, m).cpu().numpy()
    b = ctx.heff(0, m).cpu().numpy()
    assert np.array_equal(a, b)
    assert rel(a, P.heff(m0)) < 1e-10
    ctx.close()


@pytest.mark.parametrize("shape", [(32, 16, 1), (33, 17, 4), (100, 50, 2), (260, 129, 2),
                                   (150, 80, 2), (290, 140, 1), (2048, 3, 1)])
def test_heff_mixed_precision(torch_cuda, shape):
    torch = torch_cuda
    nx, ny, nz = shape
    d = (5e-9,) * 3
    say("case heff mixed", shape)
    rng = np.random.default_rng(7)
    m0 = synth.random_unit(nx, ny, nz, rng)
    ctx, P = make(torch, "mixed", nx, ny, nz, d, H=(1e4, 0, 0))
    m = torch.tensor(m0, device="cuda")
    e = rel(ctx.heff(0, m).cpu().numpy(), P.heff(m0))
    say("  mixed H_eff rel err", e)
    assert e < 1e-5
    ctx.close()


@pytest.mark.parametrize("start", ["noise", "random"])
def test_iterates_match_oracle(torch_cuda, start):
    """Ten single steps (mm_minimize_step: evaluation kernels of this small
    grid, stand-alone update) against the oracle's iterates.  Near-uniform
    start: m within 1e-11, tau 1e-9 relative.  Random start: the first BB
    steps rotate cells by up to ~pi and amplify rounding chaotically; m is
    bounded by 10x the departure of the oracle from its own run started at
    m0 perturbed by 1e-15 (largest of five draws, ~6e-9 here), tau by 1e-8."""
    torch = torch_cuda
    nx, ny, nz = 20, 12, 2
    d = (5e-9,) * 3
    say("case iterates", start, (nx, ny, nz))
    rng = np.random.default_rng(11)
    if start == "random":
        m0 = synth.random_unit(nx, ny, nz, rng)
    else:
        m0 = synth.uniform_with_noise((1, 0.2, 0), nx, ny, nz, 0.05, rng)
    H = (2e4, 3e3, 0.0)
    ctx, P = make(torch, "fp64", nx, ny, nz, d, H=H)
    m = torch.tensor(m0, device="cuda")
    ref = om.minimize(P, m0, tol=0.0, max_iter=10, record=True)
    if start == "random":
        self_dev = 0.0
        for seed in range(5):
            p = np.random.default_rng(100 + seed).standard_normal(m0.shape)
            alt = om.minimize(P, om.normalise(m0 + 1e-15 * p), tol=0.0, max_iter=10)
            self_dev = max(self_dev, float(np.max(np.abs(alt["m"] - ref["m"]))))
        tol_m, tol_tau = max(1e-8, 10 * self_dev), 1e-8
    else:
        tol_m, tol_tau = 1e-11, 1e-9
    taus = []
    for k in range(10):
        info = ctx.minimize_step(0, m)
        taus.append(info["tau"])
        assert info["k"] == k
        assert abs(info["torque"] - ref["torques"][k]) < 1e-9 * ref["torques"][k]
    err = np.max(np.abs(m.cpu().numpy() - ref["m"]))
    tau_err = np.max(np.abs(np.array(taus) / np.array(ref["taus"]) - 1))
    say("  10-iterate max diff", err, "tau rel", tau_err, "bound", tol_m)
    assert err < tol_m
    assert tau_err < tol_tau
    ctx.close()


def test_bb_switch_matches_oracle(torch_cuda):
    """Option bb_switch (the ratio switch between the two steps of eq. (12)):
    the first iterates and a run to tolerance follow the oracle's rule."""
    from paper_1405_2728_amd import Context
    torch = torch_cuda
    nx, ny, nz = 20, 12, 2
    d = (5e-9,) * 3
    kappa = 0.5
    say("case bb_switch", (nx, ny, nz), kappa)
    rng = np.random.default_rng(11)
    m0 = synth.uniform_with_noise((1, 0.2, 0), nx, ny, nz, 0.05, rng)
    H = (2e4, 3e3, 0.0)
    P = of.Problem(nx, ny, nz, *d, Ms=8e5, A=1.3e-11, Ku=500.0, u=(1, 0, 0), H_ext=H)
    ctx = Context("fp64")
    ctx.set_option("bb_switch", kappa)
    ctx.set_geometry(0, nx, ny, nz, *d)
    ctx.set_material(0, 8e5, 1.3e-11, 500.0, (1, 0, 0))
    ctx.set_field(0, H)
    m = torch.tensor(m0, device="cuda")
    ref = om.minimize(P, m0, tol=0.0, max_iter=15, record=True, bb_switch=kappa)
    alt = om.minimize(P, m0, tol=0.0, max_iter=15, record=True)
    assert not np.array_equal(ref["taus"], alt["taus"])     # the switch is in effect
    taus = []
    for k in range(15):
        info = ctx.minimize_step(0, m)
        taus.append(info["tau"])
        assert abs(info["torque"] - ref["torques"][k]) < 1e-9 * ref["torques"][k]
    err = np.max(np.abs(m.cpu().numpy() - ref["m"]))
    tau_err = np.max(np.abs(np.array(taus) / np.array(ref["taus"]) - 1))
    say("  15-iterate max diff", err, "tau rel", tau_err)
    assert err < 1e-11 and tau_err < 1e-9
    m = torch.tensor(m0, device="cuda")
    r = ctx.minimize_to_tol(0, m, tol=1e-7, max_iter=100000)
    full = om.minimize(P, m0, tol=1e-7, bb_switch=kappa)
    say("  iters gpu", r["iters"], "oracle", full["iters"], "alternation",
        om.minimize(P, m0, tol=1e-7)["iters"])
    assert r["converged"] and full["converged"]
    assert np.max(np.abs(m.cpu().numpy() - full["m"])) < 1e-4
    assert abs(r["energy"] - full["energy"]) < 1e-9 * abs(full["energy"])
    ctx.close()


def test_minimize_to_tol_cross_stationary(torch_cuda):
    torch = torch_cuda
    nx, ny, nz = 16, 8, 1
    d = (5e-9,) * 3
    say("case minimize_to_tol", (nx, ny, nz))
    rng = np.random.default_rng(12)
    m0 = synth.random_unit(nx, ny, nz, rng)
    ctx, P = make(torch, "fp64", nx, ny, nz, d)
    m = torch.tensor(m0, device="cuda")
    r = ctx.minimize_to_tol(0, m, tol=1e-6, max_iter=100000)
    ref = om.minimize(P, m0, tol=1e-6)
    say("  gpu iters", r["iters"], "oracle iters", ref["iters"])
    assert r["converged"] and r["heff_evals"] == r["iters"] + 1
    mg = m.cpu().numpy()
    assert om.torque(mg, P.heff(mg), P.Ms) < 1e-6 * 1.0001
    assert om.torque(ref["m"], P.heff(ref["m"]), P.Ms) < 1e-6
    # same basin: same state and energy
    assert np.max(np.abs(mg - ref["m"])) < 1e-3
    assert abs(r["energy"] - ref["energy"]) < 1e-8 * abs(ref["energy"])
    ctx.close()


@pytest.mark.parametrize("shape", [(64, 32, 2), (20, 10, 1), (12, 10, 6)])
def test_mixed_defect_correction_reaches_fp64_tolerance(torch_cuda, shape):
    """The single-precision form with its defect correction converges to a
    tolerance far below the plain FP32 convolution's error (1e-9 of Ms) on
    the thin wave path, the LDS x path and the 3-D path: the oracle's FP64
    torque at the final state confirms it, and the state is the FP64 run's."""
    torch = torch_cuda
    nx, ny, nz = shape
    d = (5e-9,) * 3
    say("case mixed defect correction", shape)
    rng = np.random.default_rng(41)
    m0 = synth.uniform_with_noise(synth.tilted(30.0), nx, ny, nz, 0.3, rng)
    out = {}
    for prec in ("mixed", "fp64"):
        ctx, P = make(torch, prec, nx, ny, nz, d, H=(-2e3, 1e3, 0))
        m = torch.tensor(m0, device="cuda")
        r = ctx.minimize_to_tol(0, m, tol=1e-9, max_iter=200000)
        out[prec] = (r, m.cpu().numpy())
        ctx.close()
    r, mg = out["mixed"]
    T = om.torque(mg, P.heff(mg), P.Ms)
    say("  mixed iters", r["iters"], "fp64 iters", out["fp64"][0]["iters"], "oracle torque", T)
    assert r["converged"] and out["fp64"][0]["converged"]
    assert T < 1e-9 * 1.01
    assert np.max(np.abs(mg - out["fp64"][1])) < 1e-5


def test_workload0_sweep_matches_oracle(torch_cuda):
    """32x16x1 film, random start, H = 0, 4, ..., 20 mT at 1 degree."""
    torch = torch_cuda
    w = synth.workload(0)
    nx, ny, nz = w["n"]
    say("case workload 0 sweep")
    from paper_1405_2728_amd import Context
    ctx = Context("fp64")
    ctx.set_geometry(0, nx, ny, nz, *w["d"])
    ctx.set_material(0, w["Ms"], w["A"], w["Ku"], w["u"])
    m = torch.tensor(w["m0"], device="cuda")
    mavg, iters, rc = ctx.hysteresis_sweep([m], w["fields"], tol=w["tol"])
    P = of.Problem(nx, ny, nz, *w["d"], Ms=w["Ms"], A=w["A"], Ku=w["Ku"], u=w["u"])
    ref = om.sweep(P, w["m0"], w["fields"], tol=w["tol"])
    say("  gpu iters", iters[0].tolist(), "oracle", ref["iters"].tolist())
    assert rc == 0 and ref["converged"].all()
    assert np.max(np.abs(mavg[0] - ref["mavg"])) < 1e-3
    mg = m.cpu().numpy()
    P.H_ext = w["fields"][-1]
    assert om.torque(mg, P.heff(mg), P.Ms) < 1e-6 * 1.0001
    ctx.close()


def test_sp1_size_heff_fp64_and_mixed(torch_cuda):
    """The benchmarked 400x200x4 film: full comparison with the oracle's
    FFT convolution."""
    torch = torch_cuda
    w = synth.workload(1)
    nx, ny, nz = w["n"]
    say("case 400x200x4 heff")
    H = w["fields"][0]
    P = of.Problem(nx, ny, nz, *w["d"], Ms=w["Ms"], A=w["A"], Ku=w["Ku"], u=w["u"], H_ext=H)
    rng = np.random.default_rng(3)
    m0 = synth.random_unit(nx, ny, nz, rng)
    Ho = P.heff(m0)
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-5)):
        ctx, _ = make(torch, prec, nx, ny, nz, w["d"], H=H)
        m = torch.tensor(m0, device="cuda")
        e = rel(ctx.heff(0, m).cpu().numpy(), Ho)
        say("  ", prec, "rel err", e)
        assert e < tol
        ctx.close()


# full 3-D path (more than 4 layers, or forced): several tiles of the wave
# FFTs along y and z, ragged tails, degenerate axes, anisotropic cells
SHAPES_3D = [
    ((6, 5, 8), (5e-9, 5e-9, 5e-9)),
    ((10, 7, 12), (3e-9, 4e-9, 2e-9)),
    ((17, 3, 33), (2e-9, 2e-9, 3e-9)),
    ((1, 1, 7), (5e-9, 5e-9, 5e-9)),
    ((3, 1, 5), (4e-9, 5e-9, 3e-9)),
    ((1, 40, 6), (5e-9, 5e-9, 5e-9)),
    ((70, 33, 5), (5e-9, 5e-9, 5e-9)),
    ((9, 130, 10), (5e-9, 5e-9, 5e-9)),
    ((300, 12, 6), (5e-9, 5e-9, 5e-9)),     # x padded to 896 on the 3-D path
]


@pytest.mark.parametrize("shape,d", SHAPES_3D)
def test_heff_terms_fp64_3d(torch_cuda, shape, d):
    torch = torch_cuda
    nx, ny, nz = shape
    say("case heff fp64 3-D", shape, d)
    rng = np.random.default_rng(nx * 1000 + ny * 10 + nz)
    m0 = synth.random_unit(nx, ny, nz, rng)
    ctx, P = make(torch, "fp64", nx, ny, nz, d, Ku=3e4, u=(0.0, 0.6, 0.8), H=(1e4, 2e3, -5e3))
    m = torch.tensor(m0, device="cuda")
    Ho = P.heff(m0)
    e = rel(ctx.heff(0, m).cpu().numpy(), Ho)
    say("  H_eff rel err", e)
    assert e < 1e-10
    hd = ctx.field_terms(0, m)[0].cpu().numpy()
    assert np.max(np.abs(hd - P.field_terms(m0)["demag"])) < 1e-10 * np.max(np.abs(Ho))
    E, terms = ctx.energy(0, m)
    Eo = P.energy_terms(m0)
    for a, b in zip(terms, Eo):
        assert abs(a - b) < 1e-10 * sum(abs(x) for x in Eo)
    ctx.close()


@pytest.mark.parametrize("shape", [(32, 16, 1), (33, 17, 4), (7, 5, 3)])
def test_forced_3d_path_matches_thin_path(torch_cuda, shape):
    """The two demag paths on the same film: both against the oracle and
    against each other."""
    torch = torch_cuda
    from paper_1405_2728_amd import Context
    nx, ny, nz = shape
    d = (5e-9, 4e-9, 3e-9)
    say("case forced 3-D path", shape)
    m0 = synth.random_unit(nx, ny, nz, np.random.default_rng(21))
    Ho = of.Problem(nx, ny, nz, *d, Ms=8e5, A=1.3e-11, Ku=0.0).heff(m0)
    out = []
    for path in (1, 2):
        ctx = Context("fp64")
        ctx.set_option("demag_path", path)
        ctx.set_geometry(0, nx, ny, nz, *d)
        ctx.set_material(0, 8e5, 1.3e-11, 0.0)
        m = torch.tensor(m0, device="cuda")
        out.append(ctx.heff(0, m).cpu().numpy())
        ctx.close()
    say("  thin", rel(out[0], Ho), "3-D", rel(out[1], Ho), "between", rel(out[1], out[0]))
    assert rel(out[0], Ho) < 1e-10 and rel(out[1], Ho) < 1e-10
    assert rel(out[1], out[0]) < 1e-10


@pytest.mark.parametrize("shape", [(33, 17, 9), (20, 64, 40)])
def test_heff_mixed_precision_3d(torch_cuda, shape):
    torch = torch_cuda
    nx, ny, nz = shape
    d = (3e-9,) * 3
    say("case heff mixed 3-D", shape)
    m0 = synth.random_unit(nx, ny, nz, np.random.default_rng(8))
    ctx, P = make(torch, "mixed", nx, ny, nz, d, H=(1e4, 0, 0))
    m = torch.tensor(m0, device="cuda")
    e = rel(ctx.heff(0, m).cpu().numpy(), P.heff(m0))
    say("  mixed H_eff rel err", e)
    assert e < 1e-5
    ctx.close()


# (6, 64, 40) with one row per block: 2560 per-block sums, more than the
# one-block finish takes directly, so they go through the two-stage reduction
@pytest.mark.parametrize("shape,rows", [((10, 7, 12), 0), ((6, 64, 40), 1)])
def test_iterates_match_oracle_3d(torch_cuda, shape, rows):
    from paper_1405_2728_amd import Context
    torch = torch_cuda
    nx, ny, nz = shape
    d = (3e-9,) * 3
    say("case iterates 3-D", (nx, ny, nz), "rows per block", rows)
    rng = np.random.default_rng(13)
    m0 = synth.uniform_with_noise((0.3, 0.2, 1.0), nx, ny, nz, 0.05, rng)
    Ku, u, H = 5e4, (0, 0, 1), (2e4, 0.0, 3e4)
    ctx = Context("fp64")
    if rows:
        ctx.set_option("rows_per_block", rows)
    ctx.set_geometry(0, nx, ny, nz, *d)
    ctx.set_material(0, 8e5, 1.3e-11, Ku, u)
    ctx.set_field(0, H)
    if rows:
        assert ctx.rows_per_block(0) == rows
    P = of.Problem(nx, ny, nz, *d, Ms=8e5, A=1.3e-11, Ku=Ku, u=u, H_ext=H)
    m = torch.tensor(m0, device="cuda")
    ref = om.minimize(P, m0, tol=0.0, max_iter=10, record=True)
    for k in range(10):
        info = ctx.minimize_step(0, m)
        assert info["k"] == k
        assert abs(info["torque"] - ref["torques"][k]) < 1e-9 * ref["torques"][k]
        assert abs(info["tau"] / ref["taus"][k] - 1) < 1e-9
    err = np.max(np.abs(m.cpu().numpy() - ref["m"]))
    say("  10-iterate max diff", err)
    assert err < 1e-11
    ctx.close()


def test_cube128_heff_fp64_and_mixed(torch_cuda):
    """The 128^3 cube of 2 nm cells: full comparison with the oracle's FFT
    convolution, and the field of the uniform state (mean demag factor 1/3
    for a cube, by the trace identity and symmetry)."""
    torch = torch_cuda
    w = synth.workload(2)
    nx, ny, nz = w["n"]
    say("case 128^3 heff")
    H = w["fields"][3]
    P = of.Problem(nx, ny, nz, *w["d"], Ms=w["Ms"], A=w["A"], Ku=w["Ku"], u=w["u"], H_ext=H)
    Ho = P.heff(w["m0"])
    uni = np.zeros((3, nz, ny, nx))
    uni[2] = 1.0
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-5)):
        ctx, _ = make(torch, prec, nx, ny, nz, w["d"], Ms=w["Ms"], A=w["A"], Ku=w["Ku"],
                      u=w["u"], H=H)
        m = torch.tensor(w["m0"], device="cuda")
        e = rel(ctx.heff(0, m).cpu().numpy(), Ho)
        say("  ", prec, "rel err", e)
        assert e < tol
        hd = ctx.field_terms(0, torch.tensor(uni, device="cuda"))[0].cpu().numpy()
        nzz = -hd[2].mean() / w["Ms"]
        say("   mean N_zz of the uniform cube", nzz)
        assert abs(nzz - 1.0 / 3.0) < (1e-12 if prec == "fp64" else 1e-6)
        # transverse mean vanishes by symmetry; FP32 convolution leaves ~1e-8 Ms
        assert np.max(np.abs(hd[:2].mean(axis=(1, 2, 3)))) < (1e-9 if prec == "fp64" else 1e-6) * w["Ms"]
        ctx.close()


def test_error_paths(torch_cuda):
    torch = torch_cuda
    from paper_1405_2728_amd import Context, MMError
    ctx = Context("fp64")
    with pytest.raises(MMError) as ei:
        ctx.set_geometry(0, 8, 300, 8, 1e-9, 1e-9, 1e-9)      # y padding 1024 in 3-D
    assert ei.value.code == -6
    with pytest.raises(MMError) as ei:
        ctx.set_geometry(0, 2049, 2, 1, 1e-9, 1e-9, 1e-9)     # x rows beyond Px 4096
    assert ei.value.code == -6
    for bad in ((0, 4, 1, 1e-9, 1e-9, 1e-9), (4, 4, 1, -1e-9, 1e-9, 1e-9),
                (4, 4, 1, 1e-9, float("nan"), 1e-9)):
        with pytest.raises(MMError) as ei:
            ctx.set_geometry(0, *bad)                          # empty grid, bad cell
        assert ei.value.code == -1
    ctx.set_option("demag_path", 1)
    with pytest.raises(MMError) as ei:
        ctx.set_geometry(0, 8, 8, 8, 1e-9, 1e-9, 1e-9)        # thin path: at most 4 layers
    assert ei.value.code == -6
    ctx.set_option("demag_path", 0)
    ctx.set_geometry(0, 8, 4, 1, 5e-9, 5e-9, 5e-9)
    with pytest.raises(MMError) as ei:
        ctx.heff(0, torch.zeros(3 * 32, dtype=torch.float64, device="cuda"))
    assert ei.value.code == -5                     # no material yet
    ctx.set_material(0, 8e5, 1.3e-11, 500.0)
    m = torch.tensor(synth.random_unit(8, 4, 1, np.random.default_rng(0)), device="cuda")
    m[0, 0, 1, 1] = float("nan")
    with pytest.raises(MMError) as ei:
        ctx.minimize_to_tol(0, m, tol=1e-6, max_iter=100)
    assert ei.value.code == -4
    m = torch.tensor(synth.random_unit(8, 4, 1, np.random.default_rng(0)), device="cuda")
    r = ctx.minimize_to_tol(0, m, tol=0.0, max_iter=7)
    assert r["status"] == 1 and r["iters"] == 7
    with pytest.raises(ValueError):
        ctx.heff(0, torch.zeros(5, dtype=torch.float64, device="cuda"))
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("shape", [(100, 40, 2), (20, 10, 1), (12, 10, 6), (300, 150, 1)])
def test_row_tiles_agree(torch_cuda, prec, shape):
    """Every valid rows-per-block tile of the x passes (the autotuner's
    search space) gives the oracle's field and the same first iterates:
    tiles change only the grouping of the per-block sums (last-bit changes
    of the BB step, which BB amplifies over later iterations)."""
    from paper_1405_2728_amd import Context, MMError
    torch = torch_cuda
    nx, ny, nz = shape
    d = (5e-9,) * 3
    say("case row tiles", prec, shape)
    rng = np.random.default_rng(8)
    m0 = synth.random_unit(nx, ny, nz, rng)
    P = of.Problem(nx, ny, nz, *d, Ms=8e5, A=1.3e-11, Ku=500.0, u=(1, 0, 0), H_ext=(1e4, 0, 0))
    Ho = P.heff(m0)
    tol = 1e-10 if prec == "fp64" else 1e-5
    runs = {}
    for R in range(1, 9):
        ctx = Context(prec)
        ctx.set_option("rows_per_block", R)
        try:
            ctx.set_geometry(0, nx, ny, nz, *d)
        except MMError as e:
            assert e.code == -1
            ctx.close()
            continue
        assert ctx.rows_per_block(0) == R
        ctx.set_material(0, 8e5, 1.3e-11, 500.0, (1, 0, 0))
        ctx.set_field(0, (1e4, 0, 0))
        m = torch.tensor(m0, device="cuda")
        H = ctx.heff(0, m).cpu().numpy()
        assert rel(H, Ho) < tol
        # FP64: the first 10 iterates; mixed: the first two (tau0, then the
        # first BB step), since a last-bit change of tau changes the FP32
        # roundings of m - mref, which a random start amplifies
        ctx.minimize_to_tol(0, m, tol=0.0, max_iter=10 if prec == "fp64" else 2)
        runs[R] = (H, m.cpu().numpy())
        ctx.close()
    say("  valid tiles", sorted(runs))
    assert 1 in runs and len(runs) >= 2
    H1, m1 = runs[1]
    for R, (H, m) in runs.items():
        assert rel(H, H1) < 1e-13
        assert np.max(np.abs(m - m1)) < 1e-8
    # the autotuner picks one of them
    ctx = Context(prec)
    ctx.set_option("autotune", 1)
    ctx.set_geometry(0, nx, ny, nz, *d)
    say("  autotuned tile", ctx.rows_per_block(0))
    assert ctx.rows_per_block(0) in runs
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("shape", [(100, 40, 2), (64, 32, 1), (400, 200, 4)])
def test_yz_variants_agree(torch_cuda, prec, shape):
    """The thin yz pass's occupancy variants (the autotuner's yz search
    space) run the same code under another register bound: the same field
    and the same iterates bit for bit.  Double precision has the second
    variant only for nz <= 2 (a block's 3 nz waves must fit 2 per SIMD)."""
    from paper_1405_2728_amd import Context, MMError
    torch = torch_cuda
    nx, ny, nz = shape
    d = (5e-9,) * 3
    say("case yz variants", prec, shape)
    rng = np.random.default_rng(9)
    m0 = synth.random_unit(nx, ny, nz, rng)
    runs = {}
    for var in (0, 1):
        ctx = Context(prec)
        ctx.set_option("yz_variant", var)
        try:
            ctx.set_geometry(0, nx, ny, nz, *d)
        except MMError as e:
            assert e.code == -1 and var == 1 and prec == "fp64" and nz > 2
            ctx.close()
            continue
        assert ctx.yz_variant(0) == var
        ctx.set_material(0, 8e5, 1.3e-11, 500.0, (1, 0, 0))
        ctx.set_field(0, (1e4, 0, 0))
        m = torch.tensor(m0, device="cuda")
        H = ctx.heff(0, m).cpu().numpy()
        ctx.minimize_to_tol(0, m, tol=0.0, max_iter=10)
        runs[var] = (H, m.cpu().numpy())
        ctx.close()
    say("  variants", sorted(runs))
    if len(runs) == 2:
        assert np.array_equal(runs[0][0], runs[1][0])
        assert np.array_equal(runs[0][1], runs[1][1])
    ctx = Context(prec)
    ctx.set_option("autotune", 1)
    ctx.set_geometry(0, nx, ny, nz, *d)
    say("  autotuned yz variant", ctx.yz_variant(0))
    assert ctx.yz_variant(0) in runs
    ctx.close()


def test_mixed_without_fp64_reference(torch_cuda):
    """32x300x4: the single-precision thin-film block (3 nz Py = 12288
    values, Py = 1024) fits, the double-precision one does not, so the mixed
    form runs without its defect correction: field within the mixed bound,
    and the minimiser either converges or reports its torque floor
    (MM_STALLED = 2) at a state the oracle finds near-stationary."""
    torch = torch_cuda
    from paper_1405_2728_amd.api import supported
    nx, ny, nz = 32, 300, 4
    d = (5e-9,) * 3
    assert supported("mixed", nx, ny, nz) and not supported("fp64", nx, ny, nz)
    say("case mixed without reference", (nx, ny, nz))
    rng = np.random.default_rng(19)
    m0 = synth.uniform_with_noise(synth.tilted(80.0), nx, ny, nz, 0.2, rng)
    ctx, P = make(torch, "mixed", nx, ny, nz, d, H=(0.0, 2e4, 0.0))
    m = torch.tensor(m0, device="cuda")
    e = rel(ctx.heff(0, m).cpu().numpy(), P.heff(m0))
    r = ctx.minimize_to_tol(0, m, tol=1e-6, max_iter=20000)
    mg = m.cpu().numpy()
    T = om.torque(mg, P.heff(mg), P.Ms)
    say("  H_eff rel err", e, "status", r["status"], "iters", r["iters"], "torque", r["torque"],
        "oracle torque", T)
    assert e < 1e-5
    assert r["status"] in (0, 2)
    assert T < 1e-5
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("shape", [(300, 150, 2), (150, 80, 1), (400, 200, 1), (350, 180, 1)])
def test_mixed_radix_padding_matches_powers_of_two(torch_cuda, prec, shape):
    """Mixed-radix lengths (64 VL with VL = 7, 3, 5, 6) and power-of-two
    padding compute the same convolution: fields agree to rounding, and so
    do the first iterates."""
    torch = torch_cuda
    from paper_1405_2728_amd import Context
    nx, ny, nz = shape
    d = (5e-9,) * 3
    say("case mixed-radix padding", prec, (nx, ny, nz))
    rng = np.random.default_rng(23)
    m0 = synth.uniform_with_noise(synth.tilted(20.0), nx, ny, nz, 0.3, rng)
    out = {}
    for r7 in (1, 0):
        ctx = Context(prec)
        ctx.set_option("mixed_radix", r7)
        ctx.set_geometry(0, nx, ny, nz, *d)
        ctx.set_material(0, 8e5, 1.3e-11, 500.0, (1, 0, 0))
        ctx.set_field(0, (-1e4, 2e3, 0))
        m = torch.tensor(m0, device="cuda")
        H = ctx.heff(0, m).cpu().numpy()
        ctx.minimize_to_tol(0, m, tol=0.0, max_iter=5)
        out[r7] = (H, m.cpu().numpy())
        ctx.close()
    e = rel(out[1][0], out[0][0])
    dm = float(np.max(np.abs(out[1][1] - out[0][1])))
    say("  field rel diff", e, "5-iterate max diff", dm)
    assert e < (1e-13 if prec == "fp64" else 1e-5)
    assert dm < (1e-10 if prec == "fp64" else 1e-4)
