"""The finish taken over by the forward x pass ("fused_finish", on by
default): in mm_minimize_to_tol and in sweeps, block 0 of each forward x
pass reduces the previous iteration's per-block sums in the finish kernel's
order and takes the decision (stop rule, step of eq. (12), sweep field
changes), while the other blocks wait for the published step.  The
arithmetic is the finish kernel's, so runs with the option on and off must
agree bitwise: fixed iteration counts, runs that stop inside a poll
interval, device-driven sweeps (field changes leave no update pending),
several rows per block (idle threads in the reduction) and replays of a
captured graph.  The waiting blocks' poll is bounded; with the bound set to
zero from the host ("fin_spin") they give up at once, and the run must fail
with MM_ESTATE instead of returning a result."""

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


def relax(torch, prec, n, fused, tol, max_iter, rows=0, graph=False, seed=5):
    from paper_1405_2728_amd import Context
    stream = torch.cuda.Stream() if graph else None
    ctx = Context(prec, stream=stream)
    ctx.set_option("fused_finish", 1 if fused else 0)
    ctx.set_option("use_graph", 1 if graph else 0)
    ctx.set_option("poll_every", 16)
    if rows:
        ctx.set_option("rows_per_block", rows)
    ctx.set_geometry(0, *n, 5e-9, 5e-9, 5e-9)
    ctx.set_material(0, 8e5, 1.3e-11, 500.0, (1.0, 0.0, 0.0))
    ctx.set_field(0, (-4e3, 1.5e3, 0.0))
    rng = np.random.default_rng(seed)
    m = torch.tensor(synth.uniform_with_noise(synth.tilted(30.0), *n, 0.3, rng), device="cuda")
    torch.cuda.synchronize()
    if graph:
        with torch.cuda.stream(stream):
            r = ctx.minimize_to_tol(0, m, tol=tol, max_iter=max_iter)
            stream.synchronize()
    else:
        r = ctx.minimize_to_tol(0, m, tol=tol, max_iter=max_iter)
    out = m.cpu().numpy()
    ctx.close()
    return r, out


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("n,rows", [((200, 100, 2), 0), ((100, 40, 2), 4), ((100, 40, 2), 1),
                                    ((64, 32, 1), 0)])
def test_fixed_iterations_equal(torch_cuda, prec, n, rows):
    torch = torch_cuda
    say("case fixed iterations", prec, n, "rows", rows)
    a = relax(torch, prec, n, False, 0.0, 75, rows)
    b = relax(torch, prec, n, True, 0.0, 75, rows)
    say("  iters", a[0]["iters"], b[0]["iters"], "torque", a[0]["torque"], b[0]["torque"])
    assert a[0]["iters"] == b[0]["iters"] == 75
    assert a[0]["torque"] == b[0]["torque"] and a[0]["energy"] == b[0]["energy"]
    assert np.array_equal(a[1], b[1])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_run_to_tolerance_equal(torch_cuda, prec):
    """The stop decision falls inside a poll interval: the passes after it
    see the published stop and write nothing."""
    torch = torch_cuda
    say("case run to tolerance", prec)
    n = (120, 60, 2)
    a = relax(torch, prec, n, False, 1e-6, 5000)
    b = relax(torch, prec, n, True, 1e-6, 5000)
    say("  iters", a[0]["iters"], b[0]["iters"], "status", a[0]["status"], b[0]["status"])
    assert a[0]["status"] == b[0]["status"] == 0
    assert a[0]["iters"] == b[0]["iters"]
    assert np.array_equal(a[1], b[1])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_graph_replay_equal(torch_cuda, prec):
    torch = torch_cuda
    say("case graph replay", prec)
    n = (100, 40, 2)
    a = relax(torch, prec, n, False, 1e-7, 3000)
    b = relax(torch, prec, n, True, 1e-7, 3000, graph=True)
    say("  iters", a[0]["iters"], b[0]["iters"])
    assert a[0]["iters"] == b[0]["iters"] and a[0]["iters"] > 3 * 16
    assert np.array_equal(a[1], b[1])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_sweep_equal(torch_cuda, prec):
    """A device-driven sweep: at each field change the decision leaves no
    update pending and the next field starts from the same m."""
    torch = torch_cuda
    from paper_1405_2728_amd import Context
    say("case sweep", prec)
    n = (128, 64, 2)
    h = synth.tilted(1.0)
    H = (np.array([20.0, 5.0, -5.0, -12.0])[:, None] * synth.MT * h[None, :])[None]
    res = []
    for fused in (False, True):
        ctx = Context(prec)
        ctx.set_option("fused_finish", 1 if fused else 0)
        ctx.set_option("poll_every", 16)
        ctx.set_geometry(0, *n, 5e-9, 5e-9, 5e-9)
        ctx.set_material(0, 8e5, 1.3e-11, 500.0, (1.0, 0.0, 0.0))
        rng = np.random.default_rng(9)
        m = torch.tensor(synth.uniform_with_noise(h, *n, 1e-3, rng), device="cuda")
        mavg, iters, rc = ctx.hysteresis_sweep([m], H, tol=1e-6)
        res.append((mavg, iters, rc, m.cpu().numpy()))
        say("  fused", fused, "iters", iters.tolist(), "status", rc)
        ctx.close()
    (a, b) = res
    assert a[2] == b[2] == 0
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[3], b[3])


def test_give_up_is_reported(torch_cuda):
    """Every waiting block gives up at once (no poll): the run reports
    MM_ESTATE; after a reset the context runs normally again."""
    torch = torch_cuda
    from paper_1405_2728_amd import Context
    from paper_1405_2728_amd.api import MMError
    say("case give-up path")
    n = (200, 100, 2)
    rng = np.random.default_rng(5)
    m0 = synth.uniform_with_noise(synth.tilted(30.0), *n, 0.3, rng)
    ctx = Context("fp64")
    ctx.set_option("poll_every", 16)
    ctx.set_geometry(0, *n, 5e-9, 5e-9, 5e-9)
    ctx.set_material(0, 8e5, 1.3e-11, 500.0, (1.0, 0.0, 0.0))
    ctx.set_field(0, (-4e3, 1.5e3, 0.0))
    m = torch.tensor(m0, device="cuda")
    ctx.set_option("fin_spin", 0)
    with pytest.raises(MMError) as e:
        ctx.minimize_to_tol(0, m, tol=0.0, max_iter=40)
    say("  error", e.value)
    assert e.value.code == -5 and "gave up" in str(e.value)
    ctx.set_option("fin_spin", 1 << 22)
    m.copy_(torch.tensor(m0, device="cuda"))
    r = ctx.minimize_to_tol(0, m, tol=0.0, max_iter=40)
    ctx.close()
    ref = relax(torch, "fp64", n, False, 0.0, 40)
    assert r["iters"] == 40
    assert np.array_equal(m.cpu().numpy(), ref[1])
