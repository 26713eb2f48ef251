"""Parity of the derivative entry points (mm_energy_grads, mm_hessvec,
mm_adjoint_solve, mm_param_grads) and of the autograd layer with the CPU
oracle, through the C ABI.

Tolerances: the derivatives are linear in fields that match the oracle to
1e-10 (max-norm relative, see test_gpu_parity), so 1e-9 relative for the
energy derivatives and the Hessian-vector product.  The adjoint field is the
CG solution to a relative residual of 1e-12 on both sides; the two CG runs
take different rounding paths, so their solutions agree to about the
residual times the condition number (1e-7 relative allowed)."""

import sys

import numpy as np
import pytest

import synth
from oracle import adjoint as oa, fields as of, minimizer as om

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
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(b)))


def setup(torch, n, d, Ms=8e5, A=1.3e-11, ku=None, u=(0.6, 0.8, 0.0), H=(0.0, 0.0, 0.0),
          path=0):
    from paper_1405_2728_amd import Context
    ctx = Context("fp64")
    ctx.set_option("demag_path", path)
    ctx.set_geometry(0, *n, *d)
    km = None if ku is None else torch.tensor(ku, dtype=torch.float64, device="cuda")
    ctx.set_material(0, Ms, A, 0.0, u, km)
    ctx.set_field(0, H)
    P = of.Problem(*n, *d, Ms=Ms, A=A, Ku=ku if ku is not None else 0.0, u=u, H_ext=H)
    return ctx, P


def ku_map(n, seed):
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    return 2e4 * (1.0 + 0.3 * rng.standard_normal((nz, ny, nx)))


@pytest.mark.parametrize("n,A,path", [((7, 5, 2), 1.3e-11, 0), ((6, 4, 7), 1.3e-11, 0),
                                      ((9, 3, 3), 0.0, 2)])
def test_energy_grads(torch_cuda, n, A, path):
    torch = torch_cuda
    say("case energy grads", n, A, path)
    d = (4e-9, 5e-9, 3e-9)
    ctx, P = setup(torch, n, d, A=A, ku=ku_map(n, 1), H=(1e4, -3e3, 2e3), path=path)
    m0 = synth.random_unit(*n, np.random.default_rng(2))
    g = ctx.energy_grads(0, torch.tensor(m0, device="cuda"))
    ref = oa.energy_grads(P, m0)
    assert rel(g["m"].cpu().numpy(), ref["m"]) < 1e-9
    assert rel(g["Ku"].cpu().numpy(), ref["Ku"]) < 1e-12
    assert abs(g["Ms"] - ref["Ms"]) < 1e-9 * abs(ref["Ms"])
    assert abs(g["A"] - ref["A"]) < 1e-12 * abs(ref["A"])
    assert rel(g["H_ext"], ref["H_ext"]) < 1e-12
    ctx.close()


@pytest.mark.parametrize("n,path", [((8, 6, 2), 0), ((5, 4, 6), 0), ((33, 17, 3), 0),
                                    ((8, 6, 2), 2)])
def test_hessvec(torch_cuda, n, path):
    torch = torch_cuda
    say("case hessvec", n, path)
    d = (5e-9, 5e-9, 4e-9)
    ctx, P = setup(torch, n, d, ku=ku_map(n, 3), H=(2e4, 1e4, -5e3), path=path)
    rng = np.random.default_rng(4)
    m0 = synth.random_unit(*n, rng)
    v = oa.project(m0, rng.standard_normal(m0.shape))
    out = ctx.hessvec(0, torch.tensor(m0, device="cuda"), torch.tensor(v, device="cuda"))
    ref = oa.hessvec(P, m0, v)
    e = rel(out.cpu().numpy(), ref)
    say("  rel err", e)
    assert e < 1e-9
    ctx.close()


def relaxed_gpu(ctx, m, tol):
    r = ctx.minimize_to_tol(0, m, tol=tol, max_iter=500000)
    assert r["converged"], r
    return m


def test_adjoint_matches_oracle_and_re_relaxation(torch_cuda):
    """Small platelet: adjoint field and implicit gradients against the
    oracle's CG at the same relaxed state, and dJ/dA, dJ/dMs against central
    differences of GPU re-relaxations (error budget as in the oracle pins)."""
    torch = torch_cuda
    n, d = (4, 3, 1), (4e-9, 5e-9, 3e-9)
    h = 5e3 * np.array([np.cos(np.deg2rad(20)), np.sin(np.deg2rad(20)), 0.0])
    ku = ku_map(n, 1)
    ctx, P = setup(torch, n, d, ku=ku, H=h)
    say("case adjoint small")
    m0 = synth.uniform_with_noise((1, 0, 0), *n, 1e-2, np.random.default_rng(5))
    m = relaxed_gpu(ctx, torch.tensor(m0, device="cuda"), 1e-12)
    mh = m.cpu().numpy()
    N = mh[0].size
    dJ = np.zeros_like(mh)
    dJ[0] = 1.0 / N
    lam, it, res, rc = ctx.adjoint_solve(0, m, torch.tensor(dJ, device="cuda"), tol=1e-12)
    assert rc == 0 and res <= 1e-12
    lam_ref, it_ref, _ = oa.cg_solve(P, mh, dJ, tol=1e-12)
    say("  CG iterations gpu", it, "oracle", it_ref, "lam rel", rel(lam.cpu().numpy(), lam_ref))
    assert rel(lam.cpu().numpy(), lam_ref) < 1e-7
    g = ctx.param_grads(0, m, lam)
    ref = oa.param_grads(P, mh, lam_ref)
    for k in ("A", "Ms"):
        assert abs(g[k] - ref[k]) < 1e-7 * abs(ref[k]), k
    assert rel(g["Ku"].cpu().numpy(), ref["Ku"]) < 1e-7
    assert rel(g["H_ext"], ref["H_ext"]) < 1e-7

    def J_at(**kw):
        from paper_1405_2728_amd import Context
        c2 = Context("fp64")
        c2.set_geometry(0, *n, *d)
        c2.set_material(0, kw.get("Ms", 8e5), kw.get("A", 1.3e-11), 0.0, (0.6, 0.8, 0.0),
                        torch.tensor(ku, dtype=torch.float64, device="cuda"))
        c2.set_field(0, h)
        mm = relaxed_gpu(c2, m.clone(), 1e-12)
        c2.close()
        return float(mm[0].mean())

    for k, base, re in (("A", 1.3e-11, 3e-3), ("Ms", 8e5, 1e-3)):
        eps = re * base
        fd = (J_at(**{k: base + eps}) - J_at(**{k: base - eps})) / (2 * eps)
        say("  FD", k, fd, "adjoint", g[k])
        assert abs(fd - g[k]) < 1e-4 * abs(g[k])
    ctx.close()


def test_workload4_gradients(torch_cuda):
    """200x100x2 film with a per-cell Ku map: sweep 0..-5 mT, then the
    gradients of J = <m_x> at -5 mT through the adjoint, against the oracle's
    CG and parameter gradients at the same relaxed state."""
    torch = torch_cuda
    from paper_1405_2728_amd import Context
    w = synth.workload(4)
    n = w["n"]
    say("case workload 4 gradients")
    ctx = Context("fp64")
    ctx.set_geometry(0, *n, *w["d"])
    ctx.set_material(0, w["Ms"], w["A"], 0.0, w["u"],
                     torch.tensor(w["Ku"], dtype=torch.float64, device="cuda"))
    m = torch.tensor(w["m0"], device="cuda")
    mavg, iters, rc = ctx.hysteresis_sweep([m], w["fields"], tol=1e-10)
    say("  sweep iterations", iters[0].tolist(), "rc", rc)
    assert rc == 0
    mh = m.cpu().numpy()
    N = mh[0].size
    dJ = np.zeros_like(mh)
    dJ[0] = 1.0 / N
    lam, it, res, rc = ctx.adjoint_solve(0, m, torch.tensor(dJ, device="cuda"), tol=1e-10)
    say("  CG iterations", it, "residual", res)
    assert rc == 0
    g = ctx.param_grads(0, m, lam)
    P = of.Problem(*n, *w["d"], Ms=w["Ms"], A=w["A"], Ku=w["Ku"], u=w["u"], H_ext=w["fields"][-1])
    assert om.torque(mh, P.heff(mh), P.Ms) < 1e-9
    lam_ref, it_ref, _ = oa.cg_solve(P, mh, dJ, tol=1e-10)
    ref = oa.param_grads(P, mh, lam_ref)
    say("  oracle CG iterations", it_ref, "lam rel", rel(lam.cpu().numpy(), lam_ref))
    assert rel(lam.cpu().numpy(), lam_ref) < 1e-6
    for k in ("A", "Ms"):
        assert abs(g[k] - ref[k]) < 1e-6 * abs(ref[k]), (k, g[k], ref[k])
    assert rel(g["Ku"].cpu().numpy(), ref["Ku"]) < 1e-6
    ctx.close()


def test_autograd_energy_gradcheck(torch_cuda):
    """torch.autograd.gradcheck of the energy in m and in relative
    perturbations of Ms, A, the Ku map and H (FP64, central differences)."""
    torch = torch_cuda
    from paper_1405_2728_amd import Context
    from paper_1405_2728_amd.autograd import energy
    n, d = (4, 3, 2), (4e-9, 5e-9, 3e-9)
    say("case autograd gradcheck")
    ctx = Context("fp64")
    ctx.set_geometry(0, *n, *d)
    ku0 = torch.tensor(ku_map(n, 7), dtype=torch.float64, device="cuda")
    H0 = torch.tensor([1e4, -3e3, 2e3], dtype=torch.float64)
    m0 = torch.tensor(synth.random_unit(*n, np.random.default_rng(8)), device="cuda",
                      requires_grad=True)
    xs = [torch.zeros((), dtype=torch.float64, requires_grad=True) for _ in range(2)]
    xk = torch.zeros(ku0.shape, dtype=torch.float64, device="cuda", requires_grad=True)
    xh = torch.zeros(3, dtype=torch.float64, requires_grad=True)
    scale = 1e19     # U is ~1e-19 J for these cells

    def f(m, a, b, k, h):
        return scale * energy(ctx, 0, m, 8e5 * (1 + a), 1.3e-11 * (1 + b), ku0 * (1 + k),
                              H0 * (1 + h), u=(0.6, 0.8, 0.0))

    assert torch.autograd.gradcheck(f, (m0, xs[0], xs[1], xk, xh), eps=1e-6, atol=1e-7,
                                    rtol=1e-6)
    ctx.close()


def test_autograd_relax_backward(torch_cuda):
    """relax(): implicit gradients of J = <m_x> for A and the field against
    the oracle at the same relaxed state."""
    torch = torch_cuda
    from paper_1405_2728_amd import Context
    from paper_1405_2728_amd.autograd import relax
    n, d = (5, 4, 1), (4e-9, 5e-9, 3e-9)
    say("case autograd relax")
    ctx = Context("fp64")
    ctx.set_geometry(0, *n, *d)
    ku = ku_map(n, 9)
    h = 5e3 * np.array([np.cos(np.deg2rad(30)), np.sin(np.deg2rad(30)), 0.0])
    A = torch.tensor(1.3e-11, dtype=torch.float64, requires_grad=True)
    H = torch.tensor(h, dtype=torch.float64, requires_grad=True)
    Ku = torch.tensor(ku, dtype=torch.float64, requires_grad=True)
    m0 = torch.tensor(synth.uniform_with_noise((1, 0, 0), *n, 1e-2, np.random.default_rng(1)),
                      device="cuda")
    m = relax(ctx, 0, m0, 8e5, A, Ku, H, u=(0.6, 0.8, 0.0), tol=1e-12, adj_tol=1e-12)
    J = m[0].mean()
    J.backward()
    P = of.Problem(*n, *d, Ms=8e5, A=1.3e-11, Ku=ku, u=(0.6, 0.8, 0.0), H_ext=h)
    mh = m.detach().cpu().numpy()
    dJ = np.zeros_like(mh)
    dJ[0] = 1.0 / mh[0].size
    lam, _, _ = oa.cg_solve(P, mh, dJ, tol=1e-12)
    ref = oa.param_grads(P, mh, lam)
    assert abs(A.grad.item() - ref["A"]) < 1e-7 * abs(ref["A"])
    assert rel(H.grad.numpy(), ref["H_ext"]) < 1e-7
    assert rel(Ku.grad.numpy(), ref["Ku"]) < 1e-7
    ctx.close()


def test_autograd_interleaved_forward_calls(torch_cuda):
    """Two energy() calls on one context and sample with different materials
    and fields, then one backward of their sum: each call's gradients are
    those of its own parameters (equal to separate backward passes)."""
    torch = torch_cuda
    from paper_1405_2728_amd import Context
    from paper_1405_2728_amd.autograd import energy
    n, d = (6, 5, 2), (5e-9, 5e-9, 4e-9)
    say("case autograd interleaved")
    ctx = Context("fp64")
    ctx.set_geometry(0, *n, *d)
    m_np = synth.random_unit(*n, np.random.default_rng(21))
    pars = [(8e5, 1.3e-11, 500.0, [1e4, -3e3, 2e3]), (6e5, 2.0e-11, 3e4, [-2e3, 5e3, 1e3])]

    def leaves(p):
        Ms, A, Ku, H = p
        return [torch.tensor(Ms, dtype=torch.float64, requires_grad=True),
                torch.tensor(A, dtype=torch.float64, requires_grad=True),
                torch.tensor(Ku, dtype=torch.float64, requires_grad=True),
                torch.tensor(H, dtype=torch.float64, requires_grad=True)]

    sep = []
    for p in pars:
        m = torch.tensor(m_np, device="cuda", requires_grad=True)
        x = leaves(p)
        energy(ctx, 0, m, *x, u=(0.6, 0.8, 0.0)).backward()
        sep.append([m.grad.clone()] + [t.grad.clone() for t in x])
    ms = [torch.tensor(m_np, device="cuda", requires_grad=True) for _ in pars]
    xs = [leaves(p) for p in pars]
    E = sum(energy(ctx, 0, m, *x, u=(0.6, 0.8, 0.0)) for m, x in zip(ms, xs))
    E.backward()
    for k in range(2):
        got = [ms[k].grad] + [t.grad for t in xs[k]]
        for a, b in zip(got, sep[k]):
            assert torch.allclose(a.cpu(), b.cpu(), rtol=1e-12, atol=0.0)
    # the two parameter sets give different gradients in m, Ms and H (the
    # check has teeth; dU/dA and dU/dKu depend on m and u only)
    for i in (0, 1, 4):
        assert not torch.allclose(sep[0][i], sep[1][i], rtol=1e-3, atol=0.0)
    ctx.close()
