"""Projected-gradient energy minimiser with Barzilai-Borwein steps (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Follows Sec. 2 of the paper step by step:

* auxiliary fields (eqs. (8)-(10)):  g_k = m_k x (m_k x H_eff(m_k)),
  s_{k-1} = m_k - m_{k-1},  y_{k-1} = g_k - g_{k-1};
* step sizes (eq. (12)), sums over all cells and components:
  tau1 = sum s.s / sum s.y,   tau2 = sum s.y / sum y.y,
  used alternately; the first step uses a small guess tau0;
* update: the midpoint scheme of eq. (7), linear in m_{k+1} and local to each
  cell, solved cell by cell as a 3x3 linear system;
* stop rule: the torque max_i |g_k^i| / Ms below a tolerance.

Readings (the paper is garbled or silent; each reading is listed in the
design notes as well, under the same number):

R1  Sign.  Eq. (4) equates v - (v.m)m with m x (m x v), but the identity is
    m x (m x v) = -(v - (v.m)m).  Carried into eqs. (6)/(7) the printed "+"
    moves uphill for tau > 0.  The descent reading is used:
        m_{k+1} = m_k - tau (m_k + m_{k+1})/2 x (m_k x H_eff(m_k)),  tau > 0.
R2  Secant equation.  The printed "H s_{k-1} = m_{k-1}" is read as
    H s_{k-1} = y_{k-1}; eq. (12) is the pair of projections of that.
R3  H_eff(m) in eq. (8) is H_eff(m_k).
R4  Alternation: tau1 on odd k, tau2 on even k (k = 1 is the first BB step).
R5  Guard: the magnitude |s.y| is used; a candidate that is not finite or
    not positive keeps the previous tau.  No clamp and no line search.
R6  First step: tau0 = 1e-3 / Ms (in m/A), so the first rotation is at most
    about 1e-3 |g|/Ms rad.
R7  Stop rule: max_i |g_k^i| / Ms < tol, checked before every update.  The
    paper's "angular change over tau" equals |g|/sqrt(1 + (tau|g|/2)^2)
    cell by cell, the same quantity to first order.
R8  Renormalisation after every update (eq. (7) preserves |m| exactly; this
    only removes rounding drift).
R9  Each field of a sweep restarts the BB state (k = 0, tau = tau0) from the
    previous field's magnetisation (Sec. 4: the previous configuration is
    the starting point).
R21 Step switch (optional, bb_switch = kappa > 0).  Sec. 2 contrasts its
    plain alternation with a more elaborate switch between the two steps
    used by Exl et al., without stating it.  The switch offered here is the
    ratio rule of adaptive BB methods: tau2 where tau2 < kappa tau1, else
    tau1, each formed with |s.y| and guarded as in R5.  Since
    (s.y)^2 <= (s.s)(y.y), tau2 <= tau1: kappa > 1 always takes tau2, a
    tiny kappa always tau1.  Parity unpinned against Exl et al.'s own rule.
R22 Non-monotone line search (optional safeguard of the step choice; the
    paper uses none).  Along the curve tau -> m(tau) of eq. (7) the energy
    falls at rate dU/dtau = -mu0 Ms V sum_i |g_i|^2 at tau = 0 (first order
    m(tau) = m - tau g, and dU/dm_i = -mu0 Ms V H_eff,i).  A trial step tau
    is accepted when U(m(tau)) <= C - rho tau mu0 Ms V sum |g|^2, with the
    reference value C the Zhang-Hager weighted average of the accepted
    energies (C_0 = U_0, Q_0 = 1; after an accepted step
    Q' = eta Q + 1, C' = (eta Q C + U_new) / Q'); otherwise tau is
    multiplied by sigma and the trial repeated from the same m (at most
    ls_max times, after which the last trial is taken).  Every trial is an
    effective-field evaluation; the BB quotients use the accepted s and y,
    and a rejected candidate's "previous tau" is the accepted one.
    Defaults eta = 0.85, rho = 1e-4, sigma = 0.5, ls_max = 30.
"""

import numpy as np

MU0 = 4e-7 * np.pi


def cross(a, b):
    """Cell-wise cross product of [3, ...] arrays."""
    return np.stack([a[1] * b[2] - a[2] * b[1],
                     a[2] * b[0] - a[0] * b[2],
                     a[0] * b[1] - a[1] * b[0]])


def projected_direction(m, H):
    """g = m x (m x H), eq. (8)."""
    return cross(m, cross(m, H))


def torque(m, H, Ms):
    """Stop-rule quantity max_i |m_i x (m_i x H_i)| / Ms (reading R7)."""
    g = projected_direction(m, H)
    return float(np.sqrt(np.max(np.sum(g * g, axis=0)))) / Ms


def midpoint_step(m, H, tau):
    """Solve eq. (7), descent sign (reading R1), for m_{k+1}.

    With a = m x H and b = (tau/2) a, eq. (7) reads
        m_{k+1} - b x m_{k+1} = m_k + b x m_k,
    a 3x3 linear system per cell, solved with numpy.linalg.solve.
    """
    a = cross(m, H)
    b = 0.5 * tau * a
    flat_m = m.reshape(3, -1).T                     # [ncell, 3]
    flat_b = b.reshape(3, -1).T
    ncell = flat_m.shape[0]
    Bx = np.zeros((ncell, 3, 3))                    # [b]_x v = b x v
    Bx[:, 0, 1] = -flat_b[:, 2]
    Bx[:, 0, 2] = flat_b[:, 1]
    Bx[:, 1, 0] = flat_b[:, 2]
    Bx[:, 1, 2] = -flat_b[:, 0]
    Bx[:, 2, 0] = -flat_b[:, 1]
    Bx[:, 2, 1] = flat_b[:, 0]
    eye = np.eye(3)[None]
    rhs = np.einsum("nij,nj->ni", eye + Bx, flat_m)
    out = np.linalg.solve(eye - Bx, rhs[..., None])[..., 0]
    return out.T.reshape(m.shape)


def normalise(m):
    return m / np.sqrt(np.sum(m * m, axis=0))[None]


def bb_candidate(k, ss, sy, yy, bb_switch=0.0):
    """Step size of eq. (12) for iteration k >= 1 (readings R4, R5; with
    bb_switch > 0 the ratio switch of reading R21); returns None when the
    guard rejects the candidate."""
    with np.errstate(divide="ignore", invalid="ignore"):
        ss, sy, yy = np.float64(ss), np.float64(abs(sy)), np.float64(yy)
        tau1 = ss / sy
        tau2 = sy / yy
        if bb_switch > 0:
            cand = tau2 if tau2 < bb_switch * tau1 else tau1
        else:
            cand = tau1 if k % 2 == 1 else tau2
    if not np.isfinite(cand) or cand <= 0:
        return None
    return float(cand)


def default_tau0(Ms):
    """Reading R6."""
    return 1e-3 / Ms


def minimize(problem, m0, tol=1e-6, max_iter=100000, tau0=None, record=False, bb_switch=0.0,
             keep_states=False):
    """Relax m0 with the BB midpoint scheme until the torque is below tol.

    Returns a dict with the final m, the number of updates ``iters``, the
    number of effective-field evaluations ``heff_evals`` (= iters + 1, the
    unit counted in the paper's Tab. 1), ``converged``, the final torque and
    energy, and when ``record`` is set the per-iteration tau, torque and
    energy traces; with ``keep_states`` also every iterate m_0, m_1, ... in
    ``states``.
    """
    Ms = problem.Ms
    tau = default_tau0(Ms) if tau0 is None else float(tau0)
    m = normalise(np.array(m0, dtype=np.float64))
    m_prev = g_prev = None
    taus, torques, energies = [], [], []
    states = [m.copy()] if keep_states else None
    k = 0
    while True:
        terms = problem.field_terms(m)
        H = terms["demag"] + terms["exchange"] + terms["anisotropy"] + terms["zeeman"]
        g = projected_direction(m, H)
        T = float(np.sqrt(np.max(np.sum(g * g, axis=0)))) / Ms
        if record:
            torques.append(T)
            energies.append(float(sum(problem.energy_terms(m, terms))))
        if T < tol or k >= max_iter:
            return {"m": m, "iters": k, "heff_evals": k + 1, "converged": T < tol,
                    "torque": T, "energy": float(sum(problem.energy_terms(m, terms))),
                    "taus": taus, "torques": torques, "energies": energies, "states": states}
        if k > 0:
            s = m - m_prev
            y = g - g_prev
            cand = bb_candidate(k, float(np.sum(s * s)), float(np.sum(s * y)),
                                float(np.sum(y * y)), bb_switch)
            if cand is not None:
                tau = cand
        if record:
            taus.append(tau)
        m_prev, g_prev = m, g
        m = normalise(midpoint_step(m, H, tau))
        if keep_states:
            states.append(m.copy())
        k += 1


def minimize_ls(problem, m0, tol=1e-6, max_iter=100000, tau0=None, bb_switch=0.0,
                eta=0.85, rho=1e-4, sigma=0.5, ls_max=30, record=False, keep_states=False):
    """The minimiser with the non-monotone line search of reading R22.

    Same return dict as minimize (``iters`` = accepted updates,
    ``heff_evals`` = evaluations including rejected trials), plus
    ``backtracks`` (rejected trials) and, with ``record``, the accepted
    taus, torques, energies and the reference values C per accepted state.
    """
    Ms, V = problem.Ms, problem.V
    c = MU0 * Ms * V

    def evaluate(m):
        terms = problem.field_terms(m)
        H = terms["demag"] + terms["exchange"] + terms["anisotropy"] + terms["zeeman"]
        g = projected_direction(m, H)
        gg = np.sum(g * g, axis=0)
        return (H, g, float(np.sqrt(np.max(gg))) / Ms, float(np.sum(gg)),
                float(sum(problem.energy_terms(m, terms))))

    tau = default_tau0(Ms) if tau0 is None else float(tau0)
    m = normalise(np.array(m0, dtype=np.float64))
    H, g, T, G, E = evaluate(m)
    evals, k, back = 1, 0, 0
    C, Q = E, 1.0
    taus, torques, energies, refs = [], [T], [E], [C]
    states = [m.copy()] if keep_states else None
    while True:
        if T < tol or k >= max_iter:
            return {"m": m, "iters": k, "heff_evals": evals, "converged": T < tol, "torque": T,
                    "energy": E, "backtracks": back, "taus": taus, "torques": torques,
                    "energies": energies, "refs": refs, "states": states}
        nb = 0
        while True:
            mt = normalise(midpoint_step(m, H, tau))
            Ht, gt, Tt, Gt, Et = evaluate(mt)
            evals += 1
            if Et <= C - rho * tau * c * G or nb >= ls_max:
                break
            tau *= sigma
            nb += 1
            back += 1
        s, y = mt - m, gt - g
        m, H, g, T, G, E = mt, Ht, gt, Tt, Gt, Et
        Qn = eta * Q + 1.0
        C = (eta * Q * C + E) / Qn
        Q = Qn
        k += 1
        if record:
            taus.append(tau)
            torques.append(T)
            energies.append(E)
            refs.append(C)
        if keep_states:
            states.append(m.copy())
        cand = bb_candidate(k, float(np.sum(s * s)), float(np.sum(s * y)), float(np.sum(y * y)),
                            bb_switch)
        if cand is not None:
            tau = cand


def sweep(problem, m0, fields, tol=1e-6, max_iter=100000, tau0=None, bb_switch=0.0,
          line_search=False):
    """Warm-started hysteresis sweep (Sec. 4, reading R9).

    ``fields`` is [n_fields, 3] in A/m.  For each field the minimiser runs
    once from the previous field's result (with ``line_search`` the
    safeguarded form of reading R22, its reference value restarting at every
    field).  Returns per-field mean
    magnetisation <m> [n_fields, 3], iteration counts, energies and the final
    magnetisation.
    """
    m = normalise(np.array(m0, dtype=np.float64))
    fields = np.asarray(fields, dtype=np.float64).reshape(-1, 3)
    mavg = np.zeros((len(fields), 3))
    iters = np.zeros(len(fields), dtype=np.int64)
    evals = np.zeros(len(fields), dtype=np.int64)
    energy = np.zeros(len(fields))
    conv = np.zeros(len(fields), dtype=bool)
    states = []
    for f, H in enumerate(fields):
        problem.H_ext = H.copy()
        run = minimize_ls if line_search else minimize
        res = run(problem, m, tol=tol, max_iter=max_iter, tau0=tau0, bb_switch=bb_switch)
        m = res["m"]
        mavg[f] = m.reshape(3, -1).mean(axis=1)
        iters[f] = res["iters"]
        evals[f] = res["heff_evals"]
        energy[f] = res["energy"]
        conv[f] = res["converged"]
        states.append(m.copy())
    return {"m": m, "mavg": mavg, "iters": iters, "heff_evals": evals, "energy": energy,
            "converged": conv, "states": states}
