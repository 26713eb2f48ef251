"""Pins of the oracle's energy derivatives, Riemannian Hessian and implicit
(adjoint) gradients.  Each is checked against finite differences of the
oracle's energy or of re-relaxed states, which share no code with the
formulas under test."""

import copy

import numpy as np
import pytest

import synth
from oracle import adjoint as oa, fields as of, minimizer as om

MU0 = 4e-7 * np.pi


def small_problem(H=(0.0, 0.0, 0.0), seed=1, n=(5, 4, 2)):
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    ku = 2e4 * (1.0 + 0.3 * rng.standard_normal((nz, ny, nx)))
    return of.Problem(nx, ny, nz, 4e-9, 5e-9, 3e-9, Ms=8e5, A=1.3e-11, Ku=ku,
                      u=(0.6, 0.8, 0.0), H_ext=H)


def tangent(m, rng):
    return oa.project(m, rng.standard_normal(m.shape))


def test_energy_grads_match_central_differences():
    P = small_problem(H=(1e4, -3e3, 2e3))
    rng = np.random.default_rng(2)
    m = synth.random_unit(*P.n, rng)
    g = oa.energy_grads(P, m)
    U0 = abs(P.energy(m))

    def fd(setter, eps):
        Q = copy.deepcopy(P)
        setter(Q, +eps)
        up = Q.energy(m)
        Q = copy.deepcopy(P)
        setter(Q, -eps)
        return (up - Q.energy(m)) / (2 * eps)

    # U is quadratic in m, Ms and H: central differences are exact up to rounding
    dm = rng.standard_normal(m.shape)
    e = 1e-3
    dU = (P.energy(m + e * dm) - P.energy(m - e * dm)) / (2 * e)
    assert abs(dU - np.sum(g["m"] * dm)) < 1e-9 * U0
    assert abs(fd(lambda Q, s: setattr(Q, "Ms", P.Ms + s), 10.0) - g["Ms"]) < 1e-8 * abs(g["Ms"])
    assert abs(fd(lambda Q, s: setattr(Q, "A", P.A + s), 1e-14) - g["A"]) < 1e-8 * abs(g["A"])
    for q in range(3):
        def setH(Q, s, q=q):
            Q.H_ext = P.H_ext.copy()
            Q.H_ext[q] += s
        assert abs(fd(setH, 10.0) - g["H_ext"][q]) < 1e-8 * np.max(np.abs(g["H_ext"]))
    for idx in [(0, 0, 0), (1, 3, 4), (0, 2, 1)]:
        def setK(Q, s, idx=idx):
            Q.Ku = P.Ku.copy()
            Q.Ku[idx] += s
        assert abs(fd(setK, 1.0) - g["Ku"][idx]) < 1e-8 * np.max(np.abs(g["Ku"]))


def test_hessian_is_the_second_derivative_along_the_retraction():
    """<v, Hess v> = d^2/dt^2 U(normalise(m + t v)) at t = 0 (any m)."""
    P = small_problem(H=(2e4, 1e4, -5e3))
    rng = np.random.default_rng(3)
    m = synth.random_unit(*P.n, rng)
    for _ in range(3):
        v = tangent(m, rng)
        v /= np.max(np.abs(v))
        q = np.sum(v * oa.hessvec(P, m, v))
        h = 1e-4
        U = lambda t: P.energy(om.normalise(m + t * v))
        fd = (U(h) - 2 * U(0.0) + U(-h)) / (h * h)
        assert abs(fd - q) < 1e-5 * abs(q)


def test_hessian_symmetric_and_tangent():
    P = small_problem(H=(0.0, 3e4, 0.0))
    rng = np.random.default_rng(4)
    m = synth.random_unit(*P.n, rng)
    v, w = tangent(m, rng), tangent(m, rng)
    Hv, Hw = oa.hessvec(P, m, v), oa.hessvec(P, m, w)
    assert abs(np.sum(w * Hv) - np.sum(v * Hw)) < 1e-12 * np.sqrt(np.sum(Hv ** 2) * np.sum(w ** 2))
    assert np.max(np.abs(np.sum(m * Hv, axis=0))) < 1e-12 * np.max(np.abs(Hv))


def relaxed(P, m0, tol=1e-11):
    r = om.minimize(P, m0, tol=tol, max_iter=200000)
    assert r["converged"]
    return r["m"]


def test_cg_converges_where_self_demag_dominates():
    """24x12x1 film after a 0..-5 mT sweep: m . H_eff < 0 in most cells (the
    self-demag field), so the curvature along m is negative; CG on the
    tangent space must still converge, and the gradient must match
    re-relaxation."""
    n = (24, 12, 1)
    rng = np.random.default_rng(1)
    ku = 500 * (1 + 0.1 * rng.standard_normal(n[::-1]))
    P = of.Problem(*n, 5e-9, 5e-9, 5e-9, Ms=8e5, A=1.3e-11, Ku=ku, u=(1, 0, 0))
    m0 = synth.uniform_with_noise((1, 0, 0), *n, 1e-3, rng)
    fields = -np.arange(0, 6, 1.0)[:, None] * synth.MT * synth.tilted(1.0)[None, :]
    m = om.sweep(P, m0, fields, tol=1e-11)["m"]
    P.H_ext = fields[-1]
    assert np.mean(np.sum(m * P.heff(m), axis=0) < 0) > 0.5
    dJ = np.zeros_like(m)
    dJ[0] = 1.0 / m[0].size
    lam, it, res = oa.cg_solve(P, m, dJ, tol=1e-11, max_iter=2000)
    assert res < 1e-11, (it, res)
    g = oa.param_grads(P, m, lam)

    def J(A):
        Q = copy.deepcopy(P)
        Q.A = A
        return float(relaxed(Q, m, tol=1e-12)[0].mean())

    eps = 3e-3 * P.A
    fd = (J(P.A + eps) - J(P.A - eps)) / (2 * eps)
    assert abs(fd - g["A"]) < 1e-4 * abs(g["A"]), (fd, g["A"])


@pytest.mark.parametrize("param,rel_eps", [("Ku", 3e-2), ("A", 3e-3), ("Ms", 1e-3), ("Hy", 3e-2)])
def test_adjoint_gradient_matches_re_relaxation(param, rel_eps):
    """J = mean m_x of the relaxed state; dJ/dtheta from the adjoint against
    central differences of states re-relaxed to torque 1e-12.  Error budget:
    the relaxation leaves |dm| ~ tol Ms / H_stiff ~ 1e-11, divided by 2 eps;
    the central difference adds O(eps^2) relative; 1e-4 relative covers both."""
    h = 5e3 * np.array([np.cos(np.deg2rad(20)), np.sin(np.deg2rad(20)), 0.0])
    P = small_problem(H=h, n=(4, 3, 1))
    rng = np.random.default_rng(5)
    m0 = synth.uniform_with_noise((1, 0, 0), *P.n, 1e-2, rng)
    m = relaxed(P, m0, tol=1e-12)
    N = m[0].size
    dJdm = np.zeros_like(m)
    dJdm[0] = 1.0 / N
    lam, it, res = oa.cg_solve(P, m, dJdm, tol=1e-12)
    assert res < 1e-12
    g = oa.param_grads(P, m, lam)
    J = lambda mm: float(mm[0].mean())

    def perturbed(s):
        Q = copy.deepcopy(P)
        if param == "Ku":
            Q.Ku = P.Ku.copy()
            Q.Ku[0, 1, 2] += s
        elif param == "Hy":
            Q.H_ext = P.H_ext.copy()
            Q.H_ext[1] += s
        else:
            setattr(Q, param, getattr(P, param) + s)
        return J(relaxed(Q, m, tol=1e-12))

    if param == "Ku":
        eps, ref = rel_eps * float(P.Ku[0, 1, 2]), g["Ku"][0, 1, 2]
    elif param == "Hy":
        eps, ref = rel_eps * float(np.linalg.norm(P.H_ext)), g["H_ext"][1]
    else:
        eps, ref = rel_eps * getattr(P, param), g[param]
    fd = (perturbed(eps) - perturbed(-eps)) / (2 * eps)
    assert abs(fd - ref) < 1e-4 * abs(ref), (param, fd, ref)
