// Local field terms, the projected direction g, the Barzilai-Borwein sums,
// the step-size / stop-rule kernel and the midpoint (Cayley) update.
//
// Paper references (Sec. 2):
//   g_k = m_k x (m_k x H_eff(m_k))                           eq. (8)
//   s_{k-1} = m_k - m_{k-1},  y_{k-1} = g_k - g_{k-1}         eqs. (9), (10)
//   tau1 = sum s.s / sum s.y,  tau2 = sum s.y / sum y.y      eq. (12), alternated
//   m_{k+1} = m_k - tau (m_k + m_{k+1})/2 x (m_k x H_eff)    eq. (7), descent sign
//   stop: max_i |g_i| / Ms < tol; first step: a small tau0
// Readings: |s.y| in both quotients; a candidate that is not finite and
// positive keeps the previous tau; tau1 on odd k, tau2 on even k.
#include "mm_device.h"
#include "mm_kernels.h"

namespace mmk {

// One thread per cell: H_eff = H_d + H_ex + H_an + H_ext, g = m x (m x H),
// per-block partial sums [s.s, s.y, y.y, m.H_d, m.H_ex, Ku (m.u)^2, m.H_ext,
// max |g|^2].
__global__ void __launch_bounds__(kLocalThreads) k_local(LocalArgs a) {
  __shared__ double scratch[kNPartial * (kLocalThreads / 64)];
  if (a.done != nullptr && *a.done != 0) return;
  const int N = a.nx * a.ny * a.nz;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool bb = a.g != nullptr && a.s != nullptr && a.st != nullptr && a.st->k > 0;
  double part[kNPartial] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (i < N) {
    const int x = i % a.nx;
    const int y = (i / a.nx) % a.ny;
    const int z = i / (a.nx * a.ny);
    const double* m = a.m;
    double mi[3], hex[3] = {0, 0, 0};
#pragma unroll
    for (int c = 0; c < 3; ++c) mi[c] = m[(size_t)c * N + i];
    // six face neighbours; a missing one contributes nothing
    const int sx = 1, sy = a.nx, sz = a.nx * a.ny;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double* mc = m + (size_t)c * N;
      double acc = 0.0;
      double t = 0.0;
      if (x > 0) t += mc[i - sx] - mi[c];
      if (x < a.nx - 1) t += mc[i + sx] - mi[c];
      acc += a.cx * t;
      t = 0.0;
      if (y > 0) t += mc[i - sy] - mi[c];
      if (y < a.ny - 1) t += mc[i + sy] - mi[c];
      acc += a.cy * t;
      t = 0.0;
      if (z > 0) t += mc[i - sz] - mi[c];
      if (z < a.nz - 1) t += mc[i + sz] - mi[c];
      acc += a.cz * t;
      hex[c] = acc;
    }
    const double ku = a.ku_map != nullptr ? a.ku_map[i] : a.ku;
    const double mu = mi[0] * a.u[0] + mi[1] * a.u[1] + mi[2] * a.u[2];
    const double pan = a.kan * ku * mu;
    double hd[3], h[3], han[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      hd[c] = a.Hd[(size_t)c * N + i];
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
    // energy densities (without prefactors)
    part[3] = mi[0] * hd[0] + mi[1] * hd[1] + mi[2] * hd[2];
    part[4] = mi[0] * hex[0] + mi[1] * hex[1] + mi[2] * hex[2];
    part[5] = ku * mu * mu;
    part[6] = mi[0] * a.H[0] + mi[1] * a.H[1] + mi[2] * a.H[2];
    // g = m x (m x H)
    const double ax = mi[1] * h[2] - mi[2] * h[1];
    const double ay = mi[2] * h[0] - mi[0] * h[2];
    const double az = mi[0] * h[1] - mi[1] * h[0];
    const double g0 = mi[1] * az - mi[2] * ay;
    const double g1 = mi[2] * ax - mi[0] * az;
    const double g2 = mi[0] * ay - mi[1] * ax;
    part[7] = g0 * g0 + g1 * g1 + g2 * g2;
    if (a.g != nullptr) {
      if (bb) {
        const double s0 = a.s[i], s1 = a.s[(size_t)N + i], s2 = a.s[2 * (size_t)N + i];
        const double y0 = g0 - a.g[i], y1 = g1 - a.g[(size_t)N + i], y2 = g2 - a.g[2 * (size_t)N + i];
        part[0] = s0 * s0 + s1 * s1 + s2 * s2;
        part[1] = s0 * y0 + s1 * y1 + s2 * y2;
        part[2] = y0 * y0 + y1 * y1 + y2 * y2;
      }
      a.g[i] = g0;
      a.g[(size_t)N + i] = g1;
      a.g[2 * (size_t)N + i] = g2;
    }
  }
  const bool is_max[kNPartial] = {false, false, false, false, false, false, false, true};
  block_reduce<kNPartial>(part, is_max, scratch);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int v = 0; v < kNPartial; ++v) a.partials[(size_t)blockIdx.x * kNPartial + v] = part[v];
  }
}

// Single block: finish the reductions in a fixed order, then (thread 0) the
// stop rule, the step size of eq. (12) and the iteration counters.
__global__ void __launch_bounds__(256) k_finish(const double* __restrict__ partials, int nblocks,
                                                MinState* __restrict__ st, double Ms, double V) {
  __shared__ double scratch[kNPartial * 4];
  if (st->done != 0) return;
  double v[kNPartial] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
#pragma unroll
    for (int q = 0; q < kNPartial - 1; ++q) v[q] += partials[(size_t)b * kNPartial + q];
    v[7] = fmax(v[7], partials[(size_t)b * kNPartial + 7]);
  }
  const bool is_max[kNPartial] = {false, false, false, false, false, false, false, true};
  block_reduce<kNPartial>(v, is_max, scratch);
  if (threadIdx.x != 0) return;
  const double c = -kMu0 * Ms * V;
  const double Ed = 0.5 * c * v[3], Eex = 0.5 * c * v[4], Ean = -V * v[5], Ez = c * v[6];
  const double E = Ed + Eex + Ean + Ez;
  const double T = sqrt(v[7]) / Ms;
  st->torque = T;
  st->energy = E;
  st->eterm[0] = Ed;
  st->eterm[1] = Eex;
  st->eterm[2] = Ean;
  st->eterm[3] = Ez;
  st->ss = v[0];
  st->sy = v[1];
  st->yy = v[2];
  st->last_k = st->k;
  if (st->mode == 2) return;            // evaluation only
  st->evals += 1;
  if (!isfinite(T) || !isfinite(E)) {
    st->done = -1;
    return;
  }
  const long long k = st->k;
  if (st->mode == 0) {
    if (T < st->tol) { st->done = 1; return; }
    if (k >= st->max_iter) { st->done = 2; return; }
    if (st->stall_iters > 0) {
      if (T < st->best_torque) {
        st->best_torque = T;
        st->best_k = k;
      } else if (k - st->best_k >= st->stall_iters) {
        st->done = 3;
        return;
      }
    }
  }
  if (k > 0) {
    const double ss = v[0], sy = fabs(v[1]), yy = v[2];
    const double cand = (k & 1) ? ss / sy : sy / yy;
    if (isfinite(cand) && cand > 0.0) st->tau = cand;
  }
  st->last_tau = st->tau;
  st->k = k + 1;
}

// m+ = (I - [b]x)^-1 (I + [b]x) m with b = (tau/2) m x H = -(tau/2) m x g
// (|m| = 1), i.e. m+ = m + 2 (b x m + b x (b x m)) / (1 + |b|^2); then
// renormalise and store s = m+ - m.
__global__ void __launch_bounds__(256) k_update(double* __restrict__ m, const double* __restrict__ g,
                                                double* __restrict__ sb, int N,
                                                const MinState* __restrict__ st) {
  if (st->done != 0) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double tau = st->last_tau;
  const double m0 = m[i], m1 = m[(size_t)N + i], m2 = m[2 * (size_t)N + i];
  const double g0 = g[i], g1 = g[(size_t)N + i], g2 = g[2 * (size_t)N + i];
  const double h = -0.5 * tau;
  const double b0 = h * (m1 * g2 - m2 * g1);
  const double b1 = h * (m2 * g0 - m0 * g2);
  const double b2 = h * (m0 * g1 - m1 * g0);
  const double c0 = b1 * m2 - b2 * m1;
  const double c1 = b2 * m0 - b0 * m2;
  const double c2 = b0 * m1 - b1 * m0;
  const double d0 = b1 * c2 - b2 * c1;
  const double d1 = b2 * c0 - b0 * c2;
  const double d2 = b0 * c1 - b1 * c0;
  const double f = 2.0 / (1.0 + b0 * b0 + b1 * b1 + b2 * b2);
  double n0 = m0 + f * (c0 + d0);
  double n1 = m1 + f * (c1 + d1);
  double n2 = m2 + f * (c2 + d2);
  const double inv = 1.0 / sqrt(n0 * n0 + n1 * n1 + n2 * n2);
  n0 *= inv;
  n1 *= inv;
  n2 *= inv;
  m[i] = n0;
  m[(size_t)N + i] = n1;
  m[2 * (size_t)N + i] = n2;
  sb[i] = n0 - m0;
  sb[(size_t)N + i] = n1 - m1;
  sb[2 * (size_t)N + i] = n2 - m2;
}

__global__ void __launch_bounds__(256) k_mean_partial(const double* __restrict__ m, int N,
                                                      double* __restrict__ partials) {
  __shared__ double scratch[3 * 4];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double v[3] = {0, 0, 0};
  if (i < N) {
    v[0] = m[i];
    v[1] = m[(size_t)N + i];
    v[2] = m[2 * (size_t)N + i];
  }
  const bool is_max[3] = {false, false, false};
  block_reduce<3>(v, is_max, scratch);
  if (threadIdx.x == 0)
    for (int c = 0; c < 3; ++c) partials[(size_t)blockIdx.x * 3 + c] = v[c];
}

__global__ void __launch_bounds__(256) k_mean_finish(const double* __restrict__ partials, int nb,
                                                     int N, double* __restrict__ out) {
  __shared__ double scratch[3 * 4];
  double v[3] = {0, 0, 0};
  for (int b = threadIdx.x; b < nb; b += blockDim.x)
    for (int c = 0; c < 3; ++c) v[c] += partials[(size_t)b * 3 + c];
  const bool is_max[3] = {false, false, false};
  block_reduce<3>(v, is_max, scratch);
  if (threadIdx.x == 0)
    for (int c = 0; c < 3; ++c) out[c] = v[c] / (double)N;
}

__global__ void k_reset_state(MinState* st, double tau0, double tol, long long max_iter,
                              long long stall_iters, int mode) {
  MinState z;
  z.tau = tau0;
  z.torque = 0.0;
  z.energy = 0.0;
  for (int q = 0; q < 4; ++q) z.eterm[q] = 0.0;
  z.ss = z.sy = z.yy = 0.0;
  z.best_torque = __builtin_huge_val();
  z.tol = tol;
  z.tau0 = tau0;
  z.k = 0;
  z.best_k = 0;
  z.evals = 0;
  z.max_iter = max_iter;
  z.stall_iters = stall_iters;
  z.done = 0;
  z.mode = mode;
  z.last_tau = tau0;
  z.last_k = 0;
  *st = z;
}

// Switch the mode of a run without touching its BB history (clears done).
__global__ void k_set_mode(MinState* st, int mode) {
  st->mode = mode;
  st->done = 0;
}

void launch_reset_state(hipStream_t s, MinState* st, double tau0, double tol, long long max_iter,
                        long long stall_iters, int mode) {
  hipLaunchKernelGGL(k_reset_state, dim3(1), dim3(1), 0, s, st, tau0, tol, max_iter, stall_iters,
                     mode);
}

void launch_set_mode(hipStream_t s, MinState* st, int mode) {
  hipLaunchKernelGGL(k_set_mode, dim3(1), dim3(1), 0, s, st, mode);
}

int local_blocks(int N) { return (N + kLocalThreads - 1) / kLocalThreads; }

void launch_local(hipStream_t s, const LocalArgs& a) {
  const int N = a.nx * a.ny * a.nz;
  hipLaunchKernelGGL(k_local, dim3(local_blocks(N)), dim3(kLocalThreads), 0, s, a);
}

void launch_finish(hipStream_t s, const double* partials, int nblocks, MinState* st, double Ms,
                   double V) {
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, partials, nblocks, st, Ms, V);
}

void launch_update(hipStream_t s, double* m, const double* g, double* sbuf, int N,
                   const MinState* st) {
  hipLaunchKernelGGL(k_update, dim3((N + 255) / 256), dim3(256), 0, s, m, g, sbuf, N, st);
}

void launch_mean(hipStream_t s, const double* m, int N, double* partials, double* out3) {
  const int nb = (N + 255) / 256;
  hipLaunchKernelGGL(k_mean_partial, dim3(nb), dim3(256), 0, s, m, N, partials);
  hipLaunchKernelGGL(k_mean_finish, dim3(1), dim3(256), 0, s, partials, nb, N, out3);
}

}  // namespace mmk
