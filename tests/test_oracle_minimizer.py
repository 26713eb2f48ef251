"""Pins of the oracle's minimiser: the midpoint step of eq. (7), the BB
iteration of eqs. (8)-(12), the stop rule and the sweep.

Independent facts used: geometry of the Cayley rotation, an in-plane
angle-only re-derivation of the whole iteration for one cell, the
Stoner-Wohlfarth switching astroid, a 1-D root find of the equilibrium angle
and a general-purpose optimiser on a few cells.
"""

import numpy as np
import pytest
from scipy.optimize import brentq, minimize as sp_minimize

from oracle import fields, minimizer as mz

MU0 = 4e-7 * np.pi


def random_unit(shape, seed):
    rng = np.random.default_rng(seed)
    m = rng.standard_normal((3,) + shape)
    return m / np.linalg.norm(m, axis=0)


def small_problem(**kw):
    args = dict(Ms=8e5, A=1.3e-11, Ku=500.0, u=(1, 0, 0), H_ext=(2e4, 5e3, -1e3))
    args.update(kw)
    return fields.Problem(6, 4, 2, 5e-9, 5e-9, 5e-9, **args)


# ---------------------------------------------------------------- midpoint step
def test_midpoint_step_preserves_norm_exactly():
    P = small_problem()
    m = random_unit((2, 4, 6), 1)
    H = P.heff(m)
    mp = mz.midpoint_step(m, H, 3e-5)           # large step on purpose
    assert np.max(np.abs(np.linalg.norm(mp, axis=0) - 1.0)) < 1e-14


def test_midpoint_step_is_a_rotation_about_m_cross_h():
    """The Cayley map of b x . rotates m about b = (tau/2) m x H by the
    angle 2 atan(|b| ...) -- here checked as: m+ - m is orthogonal to b, and
    the angle between m and m+ is 2 atan(tau |m x H| / 2) (m is orthogonal
    to b, so the full rotation angle shows)."""
    P = small_problem()
    m = random_unit((2, 4, 6), 2)
    H = P.heff(m)
    tau = 2e-5
    mp = mz.midpoint_step(m, H, tau)
    a = mz.cross(m, H)
    ahat = a / np.linalg.norm(a, axis=0)
    assert np.max(np.abs(np.sum((mp - m) * ahat, axis=0))) < 1e-14
    ang = np.arctan2(np.linalg.norm(mz.cross(m, mp), axis=0), np.sum(m * mp, axis=0))
    expect = 2 * np.arctan(tau * np.linalg.norm(a, axis=0) / 2)
    assert np.max(np.abs(ang - expect)) < 1e-12
    # the rotation moves m toward the tangential field (descent)
    Hperp = H - np.sum(H * m, axis=0) * m
    assert np.all(np.sum((mp - m) * Hperp, axis=0) > 0)


def test_midpoint_step_first_order_is_projected_gradient():
    """For small tau, (m+ - m)/tau -> -g = -m x (m x H) (eq. (6), descent)."""
    P = small_problem()
    m = random_unit((2, 4, 6), 3)
    H = P.heff(m)
    g = mz.projected_direction(m, H)
    gmax = np.max(np.linalg.norm(g, axis=0))
    errs = []
    for tau in (1e-9, 1e-10):
        d = (mz.midpoint_step(m, H, tau) - m) / tau
        errs.append(np.max(np.abs(d + g)))
        assert errs[-1] < tau * gmax * gmax          # second-order remainder
    assert 8 < errs[0] / errs[1] < 12                # and it shrinks like tau


def test_step_length_over_tau_formula():
    """|m+ - m| / tau = |g| / sqrt(1 + (tau |g| / 2)^2) cell by cell."""
    P = small_problem()
    m = random_unit((2, 4, 6), 4)
    H = P.heff(m)
    tau = 5e-5
    g = mz.projected_direction(m, H)
    gn = np.linalg.norm(g, axis=0)
    lhs = np.linalg.norm(mz.midpoint_step(m, H, tau) - m, axis=0) / tau
    assert np.allclose(lhs, gn / np.sqrt(1 + (tau * gn / 2) ** 2), rtol=1e-12)


def test_printed_plus_sign_climbs_and_descent_reading_falls():
    """Reading R1: with the printed '+' the midpoint step raises U."""
    P = small_problem()
    m = random_unit((2, 4, 6), 5)
    H = P.heff(m)
    tau = 1e-7
    E0 = P.energy(m)
    down = P.energy(mz.normalise(mz.midpoint_step(m, H, tau)))
    up = P.energy(mz.normalise(mz.midpoint_step(m, H, -tau)))   # the printed sign
    assert down < E0 < up


def test_fixed_small_tau_is_monotone():
    P = small_problem()
    m = random_unit((2, 4, 6), 6)
    E = [P.energy(m)]
    for _ in range(60):
        m = mz.normalise(mz.midpoint_step(m, P.heff(m), mz.default_tau0(P.Ms)))
        E.append(P.energy(m))
    assert np.all(np.diff(E) < 0)


# ---------------------------------------------------------------- BB iteration
def sw_angle_iteration(theta0, HK, h, psiH, Ms, tau0, n_iter):
    """Independent in-plane re-derivation for one cell with uniaxial
    anisotropy along x and an in-plane field: the midpoint step is the
    rotation theta -> theta + 2 atan(tau h_t / 2), with h_t the tangential
    effective field; s and y are built from angles."""
    def ht(t):
        return -HK * np.sin(t) * np.cos(t) + h * np.sin(psiH - t)

    def vec_m(t):
        return np.array([np.cos(t), np.sin(t)])

    def vec_g(t):
        return -ht(t) * np.array([-np.sin(t), np.cos(t)])

    th, tau = theta0, tau0
    thetas = [th]
    prev = None
    for k in range(n_iter):
        if k > 0:
            s = vec_m(th) - vec_m(prev)
            y = vec_g(th) - vec_g(prev)
            ss, sy, yy = s @ s, s @ y, y @ y
            cand = ss / abs(sy) if k % 2 == 1 else abs(sy) / yy
            if np.isfinite(cand) and cand > 0:
                tau = cand
        prev = th
        th = th + 2 * np.arctan(tau * ht(th) / 2)
        thetas.append(th)
    return np.array(thetas)


def test_bb_iteration_matches_angle_rederivation():
    """Whole trajectory, step by step, before the 1-D problem converges
    (BB overshoots in steps 3 and 5 here, so the alternation and the
    |s.y| guard are exercised)."""
    Ms, K = 8e5, 500.0
    HK = 2 * K / (MU0 * Ms)
    h, psiH = 0.2 * HK, np.deg2rad(170.0)
    th0 = 2.5
    m0 = np.array([np.cos(th0), np.sin(th0), 0.0]).reshape(3, 1, 1, 1)
    ref = sw_angle_iteration(th0, HK, h, psiH, Ms, mz.default_tau0(Ms), 7)
    assert np.any(np.diff(ref) < 0) and np.any(np.diff(ref) > 0)
    for n in range(1, 8):
        # the self-demag of one cube is parallel to m (no torque); it is left
        # out so that its rounding (~Ms eps) does not enter the tiny first s, y
        P = fields.Problem(1, 1, 1, 5e-9, 5e-9, 5e-9, Ms=Ms, A=0.0, Ku=K, u=(1, 0, 0),
                           H_ext=(h * np.cos(psiH), h * np.sin(psiH), 0.0),
                           include_demag=False)
        res = mz.minimize(P, m0, tol=0.0, max_iter=n, record=True)
        th_n = np.arctan2(res["m"][1].item(), res["m"][0].item())
        # the first step is ~1e-6 rad, so s and y carry a relative rounding of
        # ~eps/1e-6; the 1-rad BB step that follows inherits ~1e-10 rad
        assert abs(np.angle(np.exp(1j * (th_n - ref[n])))) < 2e-9, (n, th_n, ref[n])
    assert res["taus"][0] == mz.default_tau0(Ms) and res["taus"][1] != res["taus"][0]


def sw_switching_field(psi):
    return 1.0 / (np.cos(psi) ** (2 / 3) + np.sin(psi) ** (2 / 3)) ** 1.5


@pytest.mark.parametrize("psi_deg", [0.0, 45.0, 20.0])
def test_stoner_wohlfarth_switching(psi_deg):
    """One cubic cell (isotropic self-demag, no exchange): the metastable
    state survives just below the astroid field and switches just above."""
    Ms, K = 8e5, 500.0
    HK = 2 * K / (MU0 * Ms)
    psi = np.deg2rad(psi_deg)
    hsw = sw_switching_field(psi)
    m0 = np.array([np.cos(1e-3), np.sin(1e-3), 0.0]).reshape(3, 1, 1, 1)
    for factor, survives in ((0.98, True), (1.02, False)):
        h = factor * hsw * HK
        P = fields.Problem(1, 1, 1, 5e-9, 5e-9, 5e-9, Ms=Ms, A=0.0, Ku=K, u=(1, 0, 0),
                           H_ext=(-h * np.cos(psi), -h * np.sin(psi), 0.0))
        r = mz.minimize(P, m0, tol=1e-10, max_iter=200000)
        assert r["converged"]
        assert (r["m"][0].item() > 0) == survives, (psi_deg, factor, r["m"].ravel())


def test_stoner_wohlfarth_half_field_at_45():
    assert abs(sw_switching_field(np.pi / 4) - 0.5) < 1e-15
    assert sw_switching_field(0.0) == 1.0


def test_equilibrium_angle_matches_root_find():
    Ms, K = 8e5, 500.0
    HK = 2 * K / (MU0 * Ms)
    h, psiH = 0.3 * HK, np.deg2rad(30.0)
    P = fields.Problem(1, 1, 1, 5e-9, 5e-9, 5e-9, Ms=Ms, A=0.0, Ku=K, u=(1, 0, 0),
                       H_ext=(h * np.cos(psiH), h * np.sin(psiH), 0.0))
    m0 = np.array([1.0, 0.0, 0.0]).reshape(3, 1, 1, 1)
    r = mz.minimize(P, m0, tol=1e-12)
    th = np.arctan2(r["m"][1].item(), r["m"][0].item())
    root = brentq(lambda t: -HK * np.sin(t) * np.cos(t) + h * np.sin(psiH - t), 0.0, psiH,
                  xtol=1e-15)
    assert abs(th - root) < 1e-10
    assert abs(r["m"][2].item()) < 1e-12


def test_few_cells_against_general_optimiser():
    """Four cells with demag, exchange, anisotropy and field: the BB result
    is a stationary point and coincides with a quasi-Newton minimum over
    spherical angles started from the same state."""
    P = fields.Problem(2, 2, 1, 5e-9, 5e-9, 5e-9, Ms=8e5, A=1.3e-11, Ku=5e4,
                       u=(0.0, 0.6, 0.8), H_ext=(3e4, -1e4, 2e4), demag="direct")
    m0 = random_unit((1, 2, 2), 8)
    r = mz.minimize(P, m0, tol=1e-11)
    assert r["converged"]

    th0 = np.arccos(np.clip(m0[2].ravel(), -1, 1))
    ph0 = np.arctan2(m0[1].ravel(), m0[0].ravel())

    def unpack(x):
        th, ph = x[:4], x[4:]
        return np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph),
                         np.cos(th)]).reshape(3, 1, 2, 2)

    scale = 1.0 / abs(P.energy(m0))
    sol = sp_minimize(lambda x: P.energy(unpack(x)) * scale, np.concatenate([th0, ph0]),
                      method="BFGS", options={"gtol": 1e-13, "maxiter": 10000})
    mb = unpack(sol.x)
    assert np.max(np.abs(mb - r["m"])) < 1e-5
    assert abs(P.energy(mb) - r["energy"]) < 1e-9 * abs(r["energy"])


def test_bb_guard_rejects_degenerate_candidates():
    assert mz.bb_candidate(1, 1.0, 0.0, 1.0) is None
    assert mz.bb_candidate(2, 1.0, 1.0, 0.0) is None
    assert mz.bb_candidate(2, 1.0, 0.0, 1.0) is None        # tau = 0 rejected
    assert mz.bb_candidate(1, 2.0, -4.0, 1.0) == 0.5        # |s.y| used
    assert mz.bb_candidate(2, 2.0, -4.0, 8.0) == 0.5


def test_bb_switch_picks_by_ratio():
    """Reading R10: tau1 = s.s/|s.y| = 2, tau2 = |s.y|/y.y = 1 (ratio 1/2);
    the switch ignores the parity of k."""
    for k in (1, 2):
        assert mz.bb_candidate(k, 4.0, -2.0, 2.0, bb_switch=0.4) == 2.0
        assert mz.bb_candidate(k, 4.0, -2.0, 2.0, bb_switch=0.6) == 1.0
        assert mz.bb_candidate(k, 1.0, 0.0, 1.0, bb_switch=0.5) is None   # tau2 = 0
        assert mz.bb_candidate(k, 0.0, 0.0, 0.0, bb_switch=0.5) is None
    # without the switch, the parity decides
    assert mz.bb_candidate(1, 4.0, -2.0, 2.0) == 2.0
    assert mz.bb_candidate(2, 4.0, -2.0, 2.0) == 1.0


def test_bb_switch_extremes_on_random_sums():
    """kappa > 1 always takes the short step and a tiny kappa the long one:
    tau2 <= tau1 by Cauchy-Schwarz, and tau1 tau2 = s.s / y.y."""
    rng = np.random.default_rng(3)
    for _ in range(200):
        s_, y_ = rng.standard_normal(12), rng.standard_normal(12)
        ss, sy, yy = float(s_ @ s_), float(s_ @ y_), float(y_ @ y_)
        short = mz.bb_candidate(1, ss, sy, yy, bb_switch=2.0)
        long_ = mz.bb_candidate(2, ss, sy, yy, bb_switch=1e-300)
        assert short <= long_
        assert abs(short * long_ - ss / yy) <= 1e-14 * ss / yy
        assert mz.bb_candidate(2, ss, sy, yy) == short       # alternation, even k
        assert mz.bb_candidate(1, ss, sy, yy) == long_       # odd k


def test_bb_switch_reaches_the_same_minimum():
    """The ratio switch (and its short-step extreme) is a descent to the
    same stationary point as the alternation from the same start (four
    cells, the general-optimiser case above).  Long steps alone (tiny
    kappa) need not converge without a safeguard and are not run here."""
    P = fields.Problem(2, 2, 1, 5e-9, 5e-9, 5e-9, Ms=8e5, A=1.3e-11, Ku=5e4,
                       u=(0.0, 0.6, 0.8), H_ext=(3e4, -1e4, 2e4), demag="direct")
    m0 = random_unit((1, 2, 2), 8)
    ref = mz.minimize(P, m0, tol=1e-11, record=True)
    assert ref["converged"]
    for kappa in (0.5, 2.0):
        r = mz.minimize(P, m0, tol=1e-11, record=True, bb_switch=kappa)
        assert r["converged"], kappa
        assert np.max(np.abs(r["m"] - ref["m"])) < 1e-8, kappa
        assert abs(r["energy"] - ref["energy"]) < 1e-12 * abs(ref["energy"]), kappa
        n = min(len(r["taus"]), len(ref["taus"]))
        assert not np.array_equal(r["taus"][:n], ref["taus"][:n]), kappa


def test_converged_start_takes_no_step_and_max_iter_caps():
    P = fields.Problem(1, 1, 1, 5e-9, 5e-9, 5e-9, Ms=8e5, A=0.0, Ku=500.0,
                       H_ext=(1e4, 0.0, 0.0))
    m0 = np.array([1.0, 0.0, 0.0]).reshape(3, 1, 1, 1)
    r = mz.minimize(P, m0, tol=1e-6)
    assert r["iters"] == 0 and r["heff_evals"] == 1 and r["converged"]
    P2 = small_problem()
    r2 = mz.minimize(P2, random_unit((2, 4, 6), 9), tol=0.0, max_iter=3)
    assert r2["iters"] == 3 and not r2["converged"]


def test_sweep_warm_start_repeated_field_costs_nothing():
    P = small_problem()
    H = np.array([[2e4, 0.0, 0.0], [2e4, 0.0, 0.0]])
    out = mz.sweep(P, random_unit((2, 4, 6), 10), H, tol=1e-7)
    assert out["converged"].all()
    assert out["iters"][0] > 0 and out["iters"][1] == 0
    assert np.allclose(out["mavg"][0], out["mavg"][1])


def test_sweep_records_each_fields_state_and_restarts_bb():
    """The sweep's per-field records: <m> is the cell mean of that field's
    final state (summed here with math.fsum per component, not by the
    sweep's own reduction); every field's run is a fresh BB run from the
    previous field's state (the step restarts at tau0), so it equals
    minimize() started there, iterate count and state."""
    import math
    P = small_problem()
    H = np.array([[2e4, 0.0, 0.0], [-1e4, 2e3, 0.0], [-3e4, 0.0, 1e3]])
    m0 = random_unit((2, 4, 6), 14)
    out = mz.sweep(P, m0, H, tol=1e-7)
    assert out["converged"].all()
    for f in range(len(H)):
        mf = out["states"][f]
        for c in range(3):
            ref = math.fsum(mf[c].ravel().tolist()) / mf[c].size
            assert abs(out["mavg"][f][c] - ref) < 1e-15
    prev = m0 / np.linalg.norm(m0, axis=0)
    for f in range(len(H)):
        Q = small_problem(H_ext=tuple(H[f]))
        r = mz.minimize(Q, prev, tol=1e-7, record=True)
        assert r["taus"][0] == mz.default_tau0(Q.Ms)
        assert r["iters"] == out["iters"][f]
        assert np.array_equal(r["m"], out["states"][f])
        prev = r["m"]


@pytest.mark.parametrize("psi_deg", [30.0, 60.0])
def test_sweep_switches_at_the_stoner_wohlfarth_field(psi_deg):
    """One cubic cell (isotropic self-demag, no exchange) swept from +1.2 to
    -1.2 H_K in steps of 0.02 H_K along psi from the easy axis: the sweep's
    <m> along the easy axis changes sign at the first field beyond the
    astroid's switching field (closed form), and the branch before it stays
    on the metastable side."""
    Ms, K = 8e5, 500.0
    HK = 2 * K / (MU0 * Ms)
    psi = np.deg2rad(psi_deg)
    hsw = sw_switching_field(psi)
    hs = np.round(np.arange(1.2, -1.2 - 1e-9, -0.02), 10)
    H = np.stack([hs * HK * np.cos(psi), hs * HK * np.sin(psi), 0.0 * hs], axis=1)
    P = fields.Problem(1, 1, 1, 5e-9, 5e-9, 5e-9, Ms=Ms, A=0.0, Ku=K, u=(1, 0, 0))
    m0 = np.array([1.0, 0.0, 0.0]).reshape(3, 1, 1, 1)
    out = mz.sweep(P, m0, H, tol=1e-10, max_iter=200000)
    assert out["converged"].all()
    first = next(f for f in range(len(hs)) if out["mavg"][f][0] < 0)
    expect = next(f for f in range(len(hs)) if hs[f] < -hsw)
    assert first == expect, (psi_deg, first, expect, hs[first], -hsw)


def test_relaxation_lowers_energy_c0_like():
    P = fields.Problem(16, 8, 1, 5e-9, 5e-9, 5e-9, Ms=8e5, A=1.3e-11, Ku=500.0)
    m0 = random_unit((1, 8, 16), 12)
    r = mz.minimize(P, m0, tol=1e-6, record=True)
    assert r["converged"]
    assert r["energy"] < P.energy(m0)
    assert r["torques"][-1] < 1e-6


# ------------------------------------------------- non-monotone line search (R22)
def test_energy_slope_along_the_midpoint_curve():
    """dU/dtau at tau = 0 along tau -> m(tau) of eq. (7) is -mu0 Ms V sum |g|^2
    (the slope the line search's sufficient-decrease test uses), checked by a
    central difference of the energy."""
    P = small_problem()
    m = random_unit((2, 4, 6), 31)
    H = P.heff(m)
    g = mz.projected_direction(m, H)
    slope = -MU0 * P.Ms * P.V * float(np.sum(g * g))
    h = 1e-9 / P.Ms
    up = P.energy(mz.normalise(mz.midpoint_step(m, H, h)))
    dn = P.energy(mz.normalise(mz.midpoint_step(m, H, -h)))
    fd = (up - dn) / (2 * h)
    assert abs(fd - slope) < 1e-6 * abs(slope)


def test_line_search_accepts_plain_bb_steps_on_a_benign_case():
    """Near-uniform start in a strong field: every BB step already decreases
    the reference value enough, nothing is rejected and the iterates are the
    plain alternation's, bit for bit."""
    P = small_problem(H_ext=(8e4, 0.0, 0.0))
    m0 = mz.normalise(np.stack([np.ones((2, 4, 6)), 0.01 * np.ones((2, 4, 6)),
                                0.005 * np.ones((2, 4, 6))]))
    a = mz.minimize(P, m0, tol=1e-8, keep_states=True)
    b = mz.minimize_ls(P, m0, tol=1e-8, keep_states=True)
    assert b["backtracks"] == 0
    assert b["iters"] == a["iters"] and b["heff_evals"] == a["heff_evals"]
    for x, y in zip(a["states"], b["states"]):
        assert np.array_equal(x, y)


def test_line_search_rejects_an_energy_rise():
    """A first step far too long (tau0 = 1e-3 / Ms * 3e3) raises the energy in
    the plain method; the line search rejects it, shrinks tau until the
    sufficient-decrease test holds, and every accepted energy respects its
    reference value (checked with the recorded C and an independent slope)."""
    P = small_problem()
    m0 = random_unit((2, 4, 6), 32)
    tau0 = 3.0 / P.Ms
    E0 = P.energy(m0)
    plain = mz.minimize(P, m0, tol=0.0, max_iter=1, tau0=tau0)
    assert plain["energy"] > E0                      # the plain first step climbs
    r = mz.minimize_ls(P, m0, tol=1e-6, tau0=tau0, record=True, keep_states=True)
    assert r["converged"] and r["backtracks"] >= 1
    assert r["energies"][1] < E0
    c = MU0 * P.Ms * P.V
    for k in range(1, len(r["energies"])):
        m = r["states"][k - 1]
        g = mz.projected_direction(m, P.heff(m))
        bound = r["refs"][k - 1] - 1e-4 * r["taus"][k - 1] * c * float(np.sum(g * g))
        assert r["energies"][k] <= bound * (1 + 1e-14) + 1e-30
    assert max(r["energies"]) <= r["energies"][0]


def test_line_search_reaches_a_stationary_minimum():
    """From a random start the safeguarded iteration converges to a state the
    plain torque test accepts, with no more evaluations than the plain
    alternation here, and to the same energy on the 4-cell problem that a
    general optimiser solves."""
    P = small_problem()
    m0 = random_unit((2, 4, 6), 33)
    r = mz.minimize_ls(P, m0, tol=1e-8)
    assert r["converged"]
    assert mz.torque(r["m"], P.heff(r["m"]), P.Ms) < 1e-8
    q = fields.Problem(2, 2, 1, 5e-9, 5e-9, 5e-9, Ms=8e5, A=1.3e-11, Ku=2e4, u=(1, 0, 0),
                       H_ext=(1e4, 8e3, 0.0))
    m1 = random_unit((1, 2, 2), 34)
    a = mz.minimize(q, m1, tol=1e-10)
    b = mz.minimize_ls(q, m1, tol=1e-10)
    assert a["converged"] and b["converged"]
    assert abs(a["energy"] - b["energy"]) < 1e-9 * abs(a["energy"])
