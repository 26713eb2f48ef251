// Per-cell and per-iteration device logic shared by the stand-alone and the
// fused kernels: local field terms and g (eqs. (5), (8)), the BB sums
// (eqs. (9), (10), (12)), the stop rule and step choice, and the midpoint
// update of eq. (7) (descent sign).
#pragma once

#include "mm_device.h"
#include "mm_kernels.h"

namespace mmk {

// Inputs of the local terms of one cell.  A missing neighbour (free
// boundary) is replaced by the cell itself, which contributes zero; the
// exchange field is formed as soon as the neighbours arrive, so that only
// it (not the six neighbours) stays live.
struct CellIn {
  double m[3];
  double hex[3];     // exchange field
  double g[3], s[3];
  double ku;
};

// G: the type of the g and s streams (the transform type of the kernel).
template <typename G>
__device__ __forceinline__ void fetch_cell(const LocalArgs& a, int i, bool bb, CellIn& d) {
  const int N = a.nx * a.ny * a.nz;
  const int x = i % a.nx;
  const int y = (i / a.nx) % a.ny;
  const int z = i / (a.nx * a.ny);
  const int sy = a.nx, sz = a.nx * a.ny;
  const int j[6] = {x > 0 ? i - 1 : i,        x < a.nx - 1 ? i + 1 : i,
                    y > 0 ? i - sy : i,       y < a.ny - 1 ? i + sy : i,
                    z > 0 ? i - sz : i,       z < a.nz - 1 ? i + sz : i};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double* mc = a.m + (size_t)c * N;
    const double m0 = mc[i];
    double nb[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) nb[q] = mc[j[q]];
    d.m[c] = m0;
    d.hex[c] = a.cx * ((nb[0] - m0) + (nb[1] - m0)) + a.cy * ((nb[2] - m0) + (nb[3] - m0)) +
               a.cz * ((nb[4] - m0) + (nb[5] - m0));
  }
  if (a.g != nullptr) {
    const G* gp = static_cast<const G*>(a.g);
    const G* sp = static_cast<const G*>(a.s);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      d.g[c] = bb ? (double)gp[(size_t)c * N + i] : 0.0;
      d.s[c] = bb ? (double)sp[(size_t)c * N + i] : 0.0;
    }
  }
  d.ku = a.ku_map != nullptr ? a.ku_map[i] : a.ku;
}

// Local terms of one cell i given its demag field hd: H_eff, g = m x (m x H)
// (written to a.g_out, or back to a.g, when a.g is set) and the partial sums
// [s.s, s.y, y.y, m.H_d, m.H_ex, Ku (m.u)^2, m.H_ext, max |g|^2, sum m,
// sum |g|^2].  The sums and the stop test take g_k in double precision; it
// is rounded to G only where it is stored.
template <typename G>
__device__ __forceinline__ void compute_cell(const LocalArgs& a, int i, const double hd[3],
                                             bool bb, const CellIn& d, double part[kNPartial]) {
  const int N = a.nx * a.ny * a.nz;
  const double* hex = d.hex;
  const double* mi = d.m;
  const double mu = mi[0] * a.u[0] + mi[1] * a.u[1] + mi[2] * a.u[2];
  const double pan = a.kan * d.ku * mu;
  double h[3], han[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    han[c] = pan * a.u[c];
    h[c] = hd[c] + hex[c] + han[c] + a.H[c];
  }
  if (a.Hout != nullptr) {
#pragma unroll
    for (int c = 0; c < 3; ++c) a.Hout[(size_t)c * N + i] = h[c];
  }
  if (a.Hex_out != nullptr) {
#pragma unroll
    for (int c = 0; c < 3; ++c) a.Hex_out[(size_t)c * N + i] = hex[c];
  }
  if (a.Han_out != nullptr) {
#pragma unroll
    for (int c = 0; c < 3; ++c) a.Han_out[(size_t)c * N + i] = han[c];
  }
  part[3] += mi[0] * hd[0] + mi[1] * hd[1] + mi[2] * hd[2];
  part[4] += mi[0] * hex[0] + mi[1] * hex[1] + mi[2] * hex[2];
  part[5] += d.ku * mu * mu;
  part[6] += mi[0] * a.H[0] + mi[1] * a.H[1] + mi[2] * a.H[2];
  part[8] += mi[0];
  part[9] += mi[1];
  part[10] += mi[2];
  const double ax = mi[1] * h[2] - mi[2] * h[1];
  const double ay = mi[2] * h[0] - mi[0] * h[2];
  const double az = mi[0] * h[1] - mi[1] * h[0];
  const double g0 = mi[1] * az - mi[2] * ay;
  const double g1 = mi[2] * ax - mi[0] * az;
  const double g2 = mi[0] * ay - mi[1] * ax;
  const double gg = g0 * g0 + g1 * g1 + g2 * g2;
  part[7] = fmax(part[7], gg);
  part[11] += gg;
  if (a.g != nullptr) {
    if (bb) {
      const double y0 = g0 - d.g[0], y1 = g1 - d.g[1], y2 = g2 - d.g[2];
      part[0] += d.s[0] * d.s[0] + d.s[1] * d.s[1] + d.s[2] * d.s[2];
      part[1] += d.s[0] * y0 + d.s[1] * y1 + d.s[2] * y2;
      part[2] += y0 * y0 + y1 * y1 + y2 * y2;
    }
    G* go = static_cast<G*>(a.g_out != nullptr ? a.g_out : a.g);
    go[i] = (G)g0;
    go[(size_t)N + i] = (G)g1;
    go[2 * (size_t)N + i] = (G)g2;
  }
}

template <typename G>
__device__ __forceinline__ void local_cell(const LocalArgs& a, int i, const double hd[3],
                                           bool bb, double part[kNPartial]) {
  CellIn d;
  fetch_cell<G>(a, i, bb, d);
  compute_cell<G>(a, i, hd, bb, d, part);
}

// State fields the stop rule and step choice read, loaded together with the
// per-block sums (one memory round trip before the decision instead of two).
struct FinishIn {
  double tau, tol, best_torque;
  long long k, best_k, max_iter, stall_iters, evals;
  int mode, sweep;
  double bb_switch;
  LineSearch ls;
  int ls_trial, ls_nb;
  double ls_C, ls_Q, ls_G;
};

__device__ __forceinline__ FinishIn load_finish_in(const MinState* st) {
  FinishIn f;
  f.tau = st->tau;
  f.tol = st->tol;
  f.best_torque = st->best_torque;
  f.k = st->k;
  f.best_k = st->best_k;
  f.max_iter = st->max_iter;
  f.stall_iters = st->stall_iters;
  f.evals = st->evals;
  f.mode = st->mode;
  f.sweep = st->sweep;
  f.bb_switch = st->bb_switch;
  f.ls = st->ls;
  f.ls_trial = st->ls_trial;
  f.ls_nb = st->ls_nb;
  f.ls_C = st->ls_C;
  f.ls_Q = st->ls_Q;
  f.ls_G = st->ls_G;
  return f;
}

// BB candidate of eq. (12) for the step after update k (k >= 1): tau1 =
// s.s / |s.y|, tau2 = |s.y| / y.y alternately by the parity of k, or
// (bb_switch = kappa > 0) tau2 where tau2 < kappa tau1; a candidate that is
// not finite and positive keeps tau.
__device__ __forceinline__ double bb_step(long long k, double bb_switch, const double v[kNPartial],
                                          double tau) {
  const double ss = v[0], sy = fabs(v[1]), yy = v[2];
  const double t1 = ss / sy, t2 = sy / yy;
  const double cand = bb_switch > 0.0 ? (t2 < bb_switch * t1 ? t2 : t1) : ((k & 1) ? t1 : t2);
  return (isfinite(cand) && cand > 0.0) ? cand : tau;
}

// End of a run after k updates with status end (1 converged, 2 max_iter,
// 3 stalled): outside a sweep the run stops; in a sweep this field's mean
// magnetisation and update count are recorded and the next field starts
// from the same m (BB state, line-search state and stall tracking reset).
__device__ __forceinline__ void end_run(MinState* st, int end, long long k,
                                        const double v[kNPartial]) {
  if (st->sweep == 0) {
    st->done = end;
    return;
  }
  const int fi = st->field;
  for (int q = 0; q < 3; ++q) st->mavg_out[3 * fi + q] = v[8 + q] * st->inv_N;
  st->iters_out[fi] = k;
  if (end > st->worst) st->worst = end;
  st->field = fi + 1;
  if (fi + 1 >= st->n_fields) {
    st->done = st->worst;
  } else {
    for (int q = 0; q < 3; ++q) st->H[q] = st->fields[3 * (fi + 1) + q];
    st->k = 0;
    st->tau = st->tau0;
    st->last_tau = st->tau0;
    st->best_torque = __builtin_huge_val();
    st->best_k = 0;
    st->ls_trial = 0;
    st->ls_retry = 0;
    st->ls_nb = 0;
  }
}

// Stop rule and step size from the reduced sums v (one thread); f holds the
// state as it was when the sums were taken.  Sets done / tau / k / pending;
// records torque and energy.
__device__ __forceinline__ void finish_decision(MinState* st, const FinishIn& f,
                                                const double v[kNPartial], double Ms, double V) {
  const double c = -kMu0 * Ms * V;
  const double Ed = 0.5 * c * v[3], Eex = 0.5 * c * v[4], Ean = -V * v[5], Ez = c * v[6];
  const double E = Ed + Eex + Ean + Ez;
  const double T = sqrt(v[7]) / Ms;
  const long long k = f.k;
  st->torque = T;
  st->energy = E;
  st->eterm[0] = Ed;
  st->eterm[1] = Eex;
  st->eterm[2] = Ean;
  st->eterm[3] = Ez;
  st->ss = v[0];
  st->sy = v[1];
  st->yy = v[2];
  st->last_k = k;
  st->pending = 0;
  if (f.mode == 2) return;  // evaluation only
  st->evals = f.evals + 1;
  if (!isfinite(T) || !isfinite(E)) {
    st->done = -1;
    return;
  }
  if (f.mode == 0 && f.ls.on) {
    // Non-monotone line search: this evaluation is either the first of the
    // run (the base) or a trial m(tau) from the base
    long long k = f.k;
    if (f.ls_trial) {
      const double thr = f.ls_C - f.ls.rho * f.tau * (kMu0 * Ms * V) * f.ls_G;
      if (!(E <= thr) && f.ls_nb < f.ls.max_back) {
        // rejected: the same base, a shorter step
        const double tau = f.tau * f.ls.sigma;
        st->tau = tau;
        st->last_tau = tau;
        st->ls_nb = f.ls_nb + 1;
        st->ls_retry = 1;
        st->pending = 1;
        return;
      }
      // accepted: the trial is the new state
      const double Qn = f.ls.eta * f.ls_Q + 1.0;
      st->ls_C = (f.ls.eta * f.ls_Q * f.ls_C + E) / Qn;
      st->ls_Q = Qn;
      k += 1;
      st->k = k;
      st->last_k = k;
    } else {
      st->ls_C = E;
      st->ls_Q = 1.0;
    }
    st->ls_G = v[11];
    st->ls_nb = 0;
    st->ls_retry = 0;
    int end = 0;
    if (T < f.tol) end = 1;
    else if (k >= f.max_iter) end = 2;
    if (end != 0) {
      end_run(st, end, k, v);
      return;
    }
    const double tau = k > 0 ? bb_step(k, f.bb_switch, v, f.tau) : f.tau;
    st->tau = tau;
    st->last_tau = tau;
    st->ls_trial = 1;
    st->pending = 1;
    return;
  }
  if (f.mode == 0) {
    int end = 0;
    if (T < f.tol) end = 1;
    else if (k >= f.max_iter) end = 2;
    else if (f.stall_iters > 0) {
      if (T < f.best_torque) {
        st->best_torque = T;
        st->best_k = k;
      } else if (k - f.best_k >= f.stall_iters) {
        end = 3;
      }
    }
    if (end != 0) {
      end_run(st, end, k, v);
      return;
    }
  }
  // eq. (12) for k >= 1; the first step keeps tau0
  const double tau = k > 0 ? bb_step(k, f.bb_switch, v, f.tau) : f.tau;
  st->tau = tau;
  st->last_tau = tau;
  st->k = k + 1;
  st->pending = 1;
}

// One block reduces the per-block sums partials[nb][kNPartial] in a fixed
// order (thread t < kFinishThreads sums rows t, t + T, ... in row order,
// kFinishRows rows in flight; then block_reduce), and thread 0 takes the
// decision: the stop rule, the step size of eq. (12) and the iteration
// counters.  Threads t >= kFinishThreads of a larger block (the forward x
// pass that takes the finish over) add nothing: their waves' zeros come last
// in block_reduce's wave order, so the result is the finish kernel's.
constexpr int kFinishThreads = 192;
constexpr int kFinishRows = 4;

// rows b0, b0 + T, ..., b0 + (ROWS - 1) T, those past the end clamped to the
// last row (dropped again by finish_add)
template <int ROWS>
__device__ __forceinline__ void finish_load(const double* __restrict__ partials, int nb, int b0,
                                            double (&x)[ROWS][kNPartial]) {
#pragma unroll
  for (int u = 0; u < ROWS; ++u) {
    const int b = min(b0 + u * kFinishThreads, nb - 1);
#pragma unroll
    for (int q = 0; q < kNPartial; ++q) x[u][q] = partials[(size_t)b * kNPartial + q];
  }
}

// add the loaded rows in row order; rows past the end are dropped by a
// select, not a branch, so that all the loads stay in flight together
template <int ROWS>
__device__ __forceinline__ void finish_add(int nb, int b0, const double (&x)[ROWS][kNPartial],
                                           double (&v)[kNPartial]) {
#pragma unroll
  for (int u = 0; u < ROWS; ++u) {
    const bool ok = b0 + u * kFinishThreads < nb;
#pragma unroll
    for (int q = 0; q < kNPartial; ++q) {
      const double t = q == kPartMax ? fmax(v[q], x[u][q]) : v[q] + x[u][q];
      v[q] = ok ? t : v[q];
    }
  }
}

// ROWS: rows in flight per thread (registers against latency); the sums do
// not depend on it, each thread adding its rows in row order.
template <int MAXT, int ROWS, int NS>
__device__ __forceinline__ void finish_in_block(const double* __restrict__ partials, int nb,
                                                MinState* st, double Ms, double V,
                                                double (&scratch)[NS]) {
  const int t = threadIdx.x;
  const bool act = t < kFinishThreads;
  double x[ROWS][kNPartial];
  if (act) finish_load<ROWS>(partials, nb, t, x);
  // the state is read while the first rows' loads are in flight
  const int dn = st->done;
  const FinishIn f = load_finish_in(st);
  double v[kNPartial] = {};
  if (act) {
    finish_add<ROWS>(nb, t, x, v);
    for (int b0 = t + ROWS * kFinishThreads; b0 < nb; b0 += ROWS * kFinishThreads) {
      finish_load<ROWS>(partials, nb, b0, x);
      finish_add<ROWS>(nb, b0, x, v);
    }
  }
  if (dn != 0) return;
  bool is_max[kNPartial];
  for (int q = 0; q < kNPartial; ++q) is_max[q] = q == kPartMax;
  block_reduce<MAXT>(v, is_max, scratch);
  if (t != 0) return;
  finish_decision(st, f, v, Ms, V);
}

// Midpoint step: m+ = (I - [b]x)^-1 (I + [b]x) m with b = (tau/2) m x H
// = -(tau/2) m x g for |m| = 1, i.e. m+ = m + 2 (b x m + b x (b x m)) /
// (1 + |b|^2), followed by renormalisation.
__device__ __forceinline__ void cayley_step(const double m[3], const double g[3], double tau,
                                            double out[3]) {
  const double h = -0.5 * tau;
  const double b0 = h * (m[1] * g[2] - m[2] * g[1]);
  const double b1 = h * (m[2] * g[0] - m[0] * g[2]);
  const double b2 = h * (m[0] * g[1] - m[1] * g[0]);
  const double c0 = b1 * m[2] - b2 * m[1];
  const double c1 = b2 * m[0] - b0 * m[2];
  const double c2 = b0 * m[1] - b1 * m[0];
  const double d0 = b1 * c2 - b2 * c1;
  const double d1 = b2 * c0 - b0 * c2;
  const double d2 = b0 * c1 - b1 * c0;
  const double f = 2.0 / (1.0 + b0 * b0 + b1 * b1 + b2 * b2);
  double n0 = m[0] + f * (c0 + d0);
  double n1 = m[1] + f * (c1 + d1);
  double n2 = m[2] + f * (c2 + d2);
  const double inv = 1.0 / sqrt(n0 * n0 + n1 * n1 + n2 * n2);
  out[0] = n0 * inv;
  out[1] = n1 * inv;
  out[2] = n2 * inv;
}

// Block index -> logical work index so that the blocks a given XCD runs
// (hardware dispatches block b to XCD b mod 8) cover a contiguous range.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int full = (nb / 8) * 8;
  if (b >= full) return b;
  return (b & 7) * (nb / 8) + (b >> 3);
}

}  // namespace mmk
