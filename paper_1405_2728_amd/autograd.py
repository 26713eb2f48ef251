"""torch.autograd hooks for the energy and for relaxed states (argument
marshalling and the chain rule only; every derivative is computed by the
library: mm_energy_grads, mm_adjoint_solve, mm_param_grads).

energy(ctx, sample, m, Ms, A, Ku, H, u)
    U(m; Ms, A, Ku, H_ext) of Sec. 2 with gradients for m, Ms, A, Ku (scalar
    tensor or per-cell map [nz, ny, nx]) and H_ext (3-vector).
relax(ctx, sample, m0, Ms, A, Ku, H, u, tol, ...)
    the state m* the minimiser reaches from m0 (a local minimum of U); its
    backward is the implicit (adjoint) gradient: Hess(m*) lam = P grad_m*,
    solved by conjugate gradients, then dJ/dtheta = -lam . d(dU/dm)/dtheta.
    m* does not depend differentiably on m0 (it is locally constant within
    a basin), so m0 receives no gradient.

Both keep the material and field their forward pass used and set them on
the context again before the backward pass computes derivatives, so that
several forward calls on one context and sample (with different
parameters) before a single backward give each call its own gradients.
Setting them resets that sample's minimiser state.
"""

import torch

from .api import MMError


def _saved(Ms, A, Ku, H, u):
    """Detached copies of the parameters of one forward call."""
    return tuple(t.detach().clone() for t in (Ms, A, Ku, H)) + (u,)


def _material(ctx, sample, Ms, A, Ku, H, u):
    if Ku.dim() == 0:
        ctx.set_material(sample, float(Ms), float(A), float(Ku), u)
    else:
        ctx.set_material(sample, float(Ms), float(A), 0.0, u,
                         ku_map=Ku.detach().to("cuda", torch.float64).contiguous())
    ctx.set_field(sample, H.detach().cpu().double().numpy())


class _Energy(torch.autograd.Function):
    @staticmethod
    def forward(fctx, m, Ms, A, Ku, H, lib, sample, u):
        _material(lib, sample, Ms, A, Ku, H, u)
        E, _ = lib.energy(sample, m)
        fctx.lib, fctx.sample = lib, sample
        fctx.mat = _saved(Ms, A, Ku, H, u)
        fctx.ku_map = Ku.dim() > 0
        fctx.devs = [t.device for t in (Ms, A, Ku, H)]
        fctx.save_for_backward(m)
        return torch.tensor(E, dtype=torch.float64, device=m.device)

    @staticmethod
    def backward(fctx, go):
        (m,) = fctx.saved_tensors
        _material(fctx.lib, fctx.sample, *fctx.mat)
        g = fctx.lib.energy_grads(fctx.sample, m)
        s = go.to(m.device)
        dKu = g["Ku"] if fctx.ku_map else g["Ku"].sum()
        d = fctx.devs
        t = lambda x, dev: torch.as_tensor(x, dtype=torch.float64).to(dev)
        return (s * g["m"], t(s.cpu() * g["Ms"], d[0]), t(s.cpu() * g["A"], d[1]),
                (s * dKu).to(d[2]), t(s.cpu() * torch.as_tensor(g["H_ext"]), d[3]),
                None, None, None)


def energy(ctx, sample, m, Ms, A, Ku, H, u=(1.0, 0.0, 0.0)):
    """Differentiable U; the context's material and field are set from the
    arguments (Ms, A: 0-d tensors; Ku: 0-d tensor or map; H: 3-vector)."""
    as_t = lambda x: x if torch.is_tensor(x) else torch.tensor(x, dtype=torch.float64)
    return _Energy.apply(m, as_t(Ms), as_t(A), as_t(Ku), as_t(H), ctx, sample, tuple(u))


class _Relax(torch.autograd.Function):
    @staticmethod
    def forward(fctx, m0, Ms, A, Ku, H, lib, sample, u, tol, max_iter, adj_tol, adj_max_iter):
        _material(lib, sample, Ms, A, Ku, H, u)
        m = m0.detach().clone().contiguous()
        r = lib.minimize_to_tol(sample, m, tol=tol, max_iter=max_iter)
        if not r["converged"]:
            raise MMError(r["status"], "relaxation did not reach the tolerance")
        fctx.lib, fctx.sample = lib, sample
        fctx.mat = _saved(Ms, A, Ku, H, u)
        fctx.ku_map = Ku.dim() > 0
        fctx.devs = [t.device for t in (Ms, A, Ku, H)]
        fctx.adj = (adj_tol, adj_max_iter)
        fctx.save_for_backward(m)
        return m

    @staticmethod
    def backward(fctx, gm):
        (m,) = fctx.saved_tensors
        lib, sample = fctx.lib, fctx.sample
        _material(lib, sample, *fctx.mat)
        lam, _, _, rc = lib.adjoint_solve(sample, m, gm.contiguous(), tol=fctx.adj[0],
                                          max_iter=fctx.adj[1])
        if rc != 0:
            raise MMError(rc, "adjoint solve did not converge")
        g = lib.param_grads(sample, m, lam, ku=True)
        dKu = g["Ku"] if fctx.ku_map else g["Ku"].sum()
        d = fctx.devs
        t = lambda x, dev: torch.as_tensor(x, dtype=torch.float64).to(dev)
        return (None, t(g["Ms"], d[0]), t(g["A"], d[1]), dKu.to(d[2]), t(g["H_ext"], d[3]),
                None, None, None, None, None, None, None)


def relax(ctx, sample, m0, Ms, A, Ku, H, u=(1.0, 0.0, 0.0), tol=1e-10, max_iter=200000,
          adj_tol=1e-10, adj_max_iter=20000):
    """Relaxed state m* with implicit gradients for Ms, A, Ku and H."""
    as_t = lambda x: x if torch.is_tensor(x) else torch.tensor(x, dtype=torch.float64)
    return _Relax.apply(m0, as_t(Ms), as_t(A), as_t(Ku), as_t(H), ctx, sample, tuple(u), tol,
                        max_iter, adj_tol, adj_max_iter)
