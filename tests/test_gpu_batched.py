"""Batched sweeps: several samples of different shapes share launches and
run their field lists on the device.  By default each pass is one
persistent launch covering every sample whatever its transform length (the
yz pass one launch per layer count); the "persistent" option 0 gives one
launch per group of equal lengths instead.  The batched kernels run the
same per-block code with the same reduction order as the per-sample path,
so the results must be bitwise identical to it; replays of a captured graph
likewise.  "mixed" is the
single-precision form with its defect correction (a double-precision
reference pass every poll_every iterations, batched like the iteration);
"mixed_plain" is the form without it."""

import sys

import numpy as np
import pytest

import synth
from oracle import fields as of, minimizer as om

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


# thin wave-eligible shapes of several groups (some with mixed-radix lengths),
# one Stockham-path shape and one 3-D shape on the Stockham x pass (those two
# run per sample inside the same sweep), one 3-D shape on the wave x pass
# (batched: the persistent 3-D stages; per sample with the grouped launches)
SHAPES = [(64, 32, 1), (100, 40, 2), (70, 33, 1), (130, 64, 2), (256, 128, 1), (20, 10, 1),
          (10, 8, 6), (260, 130, 1),   # 640-point x and 320-point y transforms
          (48, 20, 5)]


def run(torch, prec, batched, graph=False, shapes=SHAPES, n_fields=4, concurrent=True,
        bb_switch=0.0, persistent=True, rebuild=None):
    from paper_1405_2728_amd import Context
    stream = torch.cuda.Stream() if graph else None
    ctx = Context("mixed" if prec == "mixed_plain" else prec, n_samples=len(shapes), stream=stream)
    ctx.set_option("concurrent_groups", 1 if concurrent else 0)
    ctx.set_option("persistent", 1 if persistent else 0)
    if rebuild is not None:
        ctx.set_option("batch_rebuild", rebuild)
    if prec == "mixed_plain":
        ctx.set_option("refine", 0)
    ctx.set_option("batched", 1 if batched else 0)
    ctx.set_option("use_graph", 1 if graph else 0)
    ctx.set_option("poll_every", 8)
    ctx.set_option("bb_switch", bb_switch)
    rng = np.random.default_rng(31)
    ms, H = [], []
    for k, n in enumerate(shapes):
        ctx.set_geometry(k, *n, 5e-9, 5e-9, 5e-9)
        ctx.set_material(k, 8e5, 1.3e-11, float(rng.uniform(0, 2e3)), (1.0, 0.0, 0.0))
        h = synth.tilted(float(rng.uniform(0, 90)))
        ms.append(torch.tensor(synth.uniform_with_noise(h, *n, 1e-3, rng), device="cuda"))
        H.append(np.linspace(40, -40, n_fields)[:, None] * synth.MT * h[None, :])
    if stream is not None:
        with torch.cuda.stream(stream):
            mavg, iters, rc = ctx.hysteresis_sweep(ms, np.array(H), tol=1e-6)
        stream.synchronize()
    else:
        mavg, iters, rc = ctx.hysteresis_sweep(ms, np.array(H), tol=1e-6)
    out = [m.cpu().numpy() for m in ms]
    ctx.close()
    return mavg, iters, rc, out, H


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_plain"])
def test_batched_equals_per_sample(torch_cuda, prec):
    torch = torch_cuda
    say("case batched vs per-sample", prec)
    a = run(torch, prec, batched=False)
    b = run(torch, prec, batched=True)
    say("  iterations", b[1].tolist(), "status", a[2], b[2])
    # FP64 and the corrected mixed form converge; the plain mixed form may
    # instead report its torque floor (MM_STALLED = 2) when FP32 rounding
    # keeps max|g|/Ms above tol
    assert a[2] == b[2]
    assert a[2] in ((0, 2) if prec == "mixed_plain" else (0,))
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[0], b[0])
    for x, y in zip(a[3], b[3]):
        assert np.array_equal(x, y)


def test_batched_equals_per_sample_with_bb_switch(torch_cuda):
    """The step switch lives in the shared finish step: the batched sweep
    (one finish launch for all samples) matches the per-sample one bitwise."""
    torch = torch_cuda
    say("case batched vs per-sample, bb_switch 0.5")
    a = run(torch, "fp64", batched=False, shapes=SHAPES[:5], bb_switch=0.5)
    b = run(torch, "fp64", batched=True, shapes=SHAPES[:5], bb_switch=0.5)
    c = run(torch, "fp64", batched=True, shapes=SHAPES[:5])
    say("  iterations", b[1].tolist(), "alternation", c[1].tolist(), "status", a[2], b[2])
    assert a[2] == b[2]
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[0], b[0])
    for x, y in zip(a[3], b[3]):
        assert np.array_equal(x, y)
    assert not np.array_equal(b[1], c[1])        # the switch is in effect


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_graph_replays_equal_eager(torch_cuda, prec):
    torch = torch_cuda
    say("case graph replay", prec)
    a = run(torch, prec, batched=True, graph=False)
    b = run(torch, prec, batched=True, graph=True)
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[0], b[0])
    for x, y in zip(a[3], b[3]):
        assert np.array_equal(x, y)


def test_batched_sweep_stationary(torch_cuda):
    """Each sample's final state is stationary for the oracle at its last
    field (cross-stationarity, tol 1e-6)."""
    torch = torch_cuda
    say("case batched stationarity")
    shapes = [(64, 32, 1), (70, 33, 2), (20, 10, 1)]
    mavg, iters, rc, out, H = run(torch, "fp64", batched=True, shapes=shapes, n_fields=3)
    assert rc == 0
    rng = np.random.default_rng(31)
    for k, n in enumerate(shapes):
        ku = float(rng.uniform(0, 2e3))
        rng.uniform(0, 90)
        synth.uniform_with_noise((1, 0, 0), *n, 1e-3, rng)   # keep the draw order of run()
        P = of.Problem(*n, 5e-9, 5e-9, 5e-9, Ms=8e5, A=1.3e-11, Ku=ku, u=(1, 0, 0),
                       H_ext=H[k][-1])
        T = om.torque(out[k], P.heff(out[k]), P.Ms)
        say("  sample", k, "oracle torque", T)
        assert T < 1e-6 * 1.001
        assert np.allclose(mavg[k, -1], out[k].reshape(3, -1).mean(axis=1), atol=1e-12)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_minimize_graph_replays_equal_eager(torch_cuda, prec):
    """mm_minimize_to_tol with use_graph replays one captured batch of
    poll_every iterations (host polls, synchronisations and eager work in
    between): every run equals the eager run bitwise, also with the cached
    graph on a second start and after a material change (recapture)."""
    torch = torch_cuda
    from paper_1405_2728_amd import Context
    say("case minimize graph replay", prec)
    n = (100, 40, 2)
    rng = np.random.default_rng(77)
    starts = [synth.uniform_with_noise(synth.tilted(a), *n, 0.2, rng) for a in (20.0, 160.0)]
    out = {}
    for graph in (False, True):
        stream = torch.cuda.Stream()
        ctx = Context(prec, stream=stream)
        ctx.set_option("use_graph", 1 if graph else 0)
        ctx.set_option("poll_every", 16)
        ctx.set_geometry(0, *n, 5e-9, 5e-9, 5e-9)
        res = []
        m = torch.zeros((3,) + n[::-1], dtype=torch.float64, device="cuda")
        for k, (Ku, m0) in enumerate([(500.0, starts[0]), (500.0, starts[1]), (1500.0, starts[1])]):
            ctx.set_material(0, 8e5, 1.3e-11, Ku, (1.0, 0.0, 0.0))
            ctx.set_field(0, (-3e3, 1e3, 0.0))
            m.copy_(torch.tensor(m0, device="cuda"))
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                r = ctx.minimize_to_tol(0, m, tol=1e-7, max_iter=3000)
                stream.synchronize()
            res.append((r["iters"], r["status"], m.cpu().numpy()))
            say("  graph", graph, "run", k, "iters", r["iters"], "status", r["status"])
        ctx.close()
        out[graph] = res
    for a, b in zip(out[False], out[True]):
        assert a[0] == b[0] and a[1] == b[1]
        assert np.array_equal(a[2], b[2])
    assert all(r[0] > 3 * 16 for r in out[True])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_concurrent_groups_equal_serial(torch_cuda, prec):
    """Launch groups forked onto auxiliary streams (parallel graph branches)
    give the same sweep, bit for bit, as groups launched one after another."""
    torch = torch_cuda
    say("case concurrent groups", prec)
    a = run(torch, prec, batched=True, graph=True, concurrent=False)
    b = run(torch, prec, batched=True, graph=True, concurrent=True)
    assert a[2] == b[2]
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[0], b[0])
    for x, y in zip(a[3], b[3]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_persistent_equals_grouped(torch_cuda, prec):
    """One persistent launch per pass gives the same bits as one launch per
    group of equal transform lengths (same blocks, same reductions)."""
    torch = torch_cuda
    say("case persistent vs grouped", prec)
    a = run(torch, prec, batched=True, graph=True, persistent=False)
    b = run(torch, prec, batched=True, graph=True, persistent=True)
    assert a[2] == b[2]
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[0], b[0])
    for x, y in zip(a[3], b[3]):
        assert np.array_equal(x, y)


def test_rebuilt_tables_give_the_same_sweep(torch_cuda):
    """Rebuilding the batch tables as samples finish (the default at 3/4 of
    the batch, and at every finished sample) gives the same bits as never
    rebuilding: each sample's blocks and reductions are its own."""
    torch = torch_cuda
    say("case batch rebuild")
    a = run(torch, "fp64", batched=True, graph=True, rebuild=0.0)
    b = run(torch, "fp64", batched=True, graph=True, rebuild=0.75)
    c = run(torch, "fp64", batched=True, graph=True, rebuild=0.99)
    for r in (b, c):
        assert r[2] == a[2]
        assert np.array_equal(a[1], r[1])
        assert np.array_equal(a[0], r[0])
        for x, y in zip(a[3], r[3]):
            assert np.array_equal(x, y)
