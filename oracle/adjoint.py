"""Derivatives of the energy and of relaxed states (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

The paper gives the energy U(m) and its link to the effective field
(Sec. 2, eq. (5): H_eff = -(1/(mu0 Ms)) dU/dm per unit volume, i.e.
dU/dm_i = -mu0 Ms V H_eff,i for a cell of volume V) and minimises U over
unit vectors.  Everything below is plain calculus on that energy; none of it
is in the paper.

* Energy derivatives (for automatic differentiation of U):
    dU/dm_i   = -mu0 Ms V H_eff,i
    dU/dMs    = (2 U_demag + U_zeeman) / Ms   (H_d is proportional to Ms,
                H_ex and H_an to 1/Ms, so Ms H_ex, Ms H_an do not depend on Ms)
    dU/dA     = U_exchange at A = 1           (U_exchange is linear in A)
    dU/dKu_i  = -V (m_i . u)^2                (anisotropy reading R11)
    dU/dH_ext = -mu0 Ms V sum_i m_i
* Riemannian Hessian of U on the product of unit spheres, applied to a
  tangent field v (v_i . m_i = 0):
    Hess v = P (d2U v) - (m . dU/dm) v,  P_i = I - m_i m_i^T,
  with d2U v = -mu0 Ms V H_lin[v] and H_lin the linear part of H_eff
  (demag + exchange + anisotropy, no Zeeman), so
    Hess v = mu0 Ms V [ -P(H_lin[v]) + (m . H_eff(m)) v ].
  For the retraction R(t) = normalise(m + t v) the second derivative of
  U(R(t)) at t = 0 is exactly <v, Hess v> (at any m, not only at a
  stationary point), which is what the tests pin it against.
  Along the normal direction m_i itself the same expression has curvature
  m_i . H_eff,i, which is negative where the self-demag field dominates;
  the operator is therefore applied to P v (identity for tangent v) and the
  CG directions are projected every step, so that rounding components along
  m cannot be amplified by the Krylov iteration.
* Implicit (adjoint) gradient of an objective J(m*) of a relaxed state m*
  (P dU/dm = 0): with Hess lam = P dJ/dm (solved by conjugate gradients on
  the tangent space), dJ/dtheta = -lam . d(dU/dm)/dtheta, i.e.
    dJ/dKu_i = 2 V (m_i . u)(lam_i . u)
    dJ/dA    = mu0 Ms V sum_i lam_i . H_ex,i(A = 1)
    dJ/dMs   = mu0 V sum_i lam_i . (2 H_d,i + H_ext)
    dJ/dH    = mu0 Ms V sum_i lam_i
"""

import copy

import numpy as np

from .fields import MU0


def project(m, v):
    """P_i v_i = v_i - (m_i . v_i) m_i."""
    return v - np.sum(m * v, axis=0, keepdims=True) * m


def energy_grads(P, m):
    """Derivatives of U(m; Ms, A, Ku, H_ext) at m (dict)."""
    t = P.field_terms(m)
    Ud, Uex, Uan, Uz = P.energy_terms(m, t)
    H = t["demag"] + t["exchange"] + t["anisotropy"] + t["zeeman"]
    Q = copy.copy(P)
    Q.A = 1.0
    dA = Q.energy_terms(m, {"demag": np.zeros_like(m), "exchange": Q.h_exchange(m),
                            "anisotropy": np.zeros_like(m), "zeeman": np.zeros_like(m)})[1]
    mu = np.einsum("c...,c->...", m, P.u)
    return {"m": -MU0 * P.Ms * P.V * H,
            "Ms": (2.0 * Ud + Uz) / P.Ms,
            "A": dA,
            "Ku": -P.V * mu * mu,
            "H_ext": -MU0 * P.Ms * P.V * m.reshape(3, -1).sum(axis=1)}


def h_linear(P, v):
    """Linear part of H_eff applied to v: demag + exchange + anisotropy."""
    return P.h_demag(v) + P.h_exchange(v) + P.h_anisotropy(v)


def hessvec(P, m, v, H_m=None):
    """Riemannian Hessian of U at m applied to P v (v tangent: v itself)."""
    if H_m is None:
        H_m = P.heff(m)
    v = project(m, v)
    mH = np.sum(m * H_m, axis=0, keepdims=True)
    return MU0 * P.Ms * P.V * (-project(m, h_linear(P, v)) + mH * v)


def cg_solve(P, m, rhs, tol=1e-10, max_iter=10000):
    """Conjugate gradients for Hess lam = P rhs on the tangent space at m.
    Returns (lam, iterations, relative residual)."""
    H_m = P.heff(m)
    b = project(m, rhs)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = float(np.sum(r * r))
    bb = rr
    if bb == 0.0:
        return x, 0, 0.0
    it = 0
    while it < max_iter and rr > tol * tol * bb:
        Ap = hessvec(P, m, p, H_m)
        alpha = rr / float(np.sum(p * Ap))
        x += alpha * p
        r -= alpha * Ap
        rr_new = float(np.sum(r * r))
        p = project(m, r + (rr_new / rr) * p)
        rr = rr_new
        it += 1
    return x, it, float(np.sqrt(rr / bb))


def param_grads(P, m, lam):
    """dJ/dA, dJ/dMs, dJ/dKu_i and dJ/dH_ext from the adjoint field lam at m."""
    Q = copy.copy(P)
    Q.A = 1.0
    hex1 = Q.h_exchange(m)
    hd = P.h_demag(m)
    hz = P.h_zeeman(m)
    mu = np.einsum("c...,c->...", m, P.u)
    lu = np.einsum("c...,c->...", lam, P.u)
    return {"A": MU0 * P.Ms * P.V * float(np.sum(lam * hex1)),
            "Ms": MU0 * P.V * float(np.sum(lam * (2.0 * hd + hz))),
            "Ku": 2.0 * P.V * mu * lu,
            "H_ext": MU0 * P.Ms * P.V * lam.reshape(3, -1).sum(axis=1)}
