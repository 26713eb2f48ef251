// The step-size / stop-rule kernel, the midpoint (Cayley) update and the
// state kernels of the minimiser.  The local field terms, the projected
// direction g and the Barzilai-Borwein sums (mm_iter.h) run inside the
// inverse x pass.
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
#include "mm_iter.h"
#include "mm_kernels.h"

namespace mmk {

__global__ void __launch_bounds__(kFinishThreads) k_finish(const double* __restrict__ partials,
                                                           int nblocks, MinState* __restrict__ st,
                                                           double Ms, double V) {
  __shared__ double scratch[kNPartial * kFinishThreads / 64];
  finish_in_block<kFinishThreads, kFinishRows>(partials, nblocks, st, Ms, V, scratch);
}

// Batched: block b finishes sample b of the table.
__global__ void __launch_bounds__(kFinishThreads) k_finish_b(const BatchDesc* __restrict__ descs) {
  __shared__ double scratch[kNPartial * kFinishThreads / 64];
  const BatchDesc& d = descs[blockIdx.x];
  finish_in_block<kFinishThreads, kFinishRows>(d.partials, d.nb3, d.st, d.Ms, d.V, scratch);
}

// Apply a pending midpoint update (eq. (7)) to m and store s = m+ - m.
template <typename G>
__global__ void __launch_bounds__(256) k_update(double* __restrict__ m, const G* __restrict__ g,
                                                G* __restrict__ sb, int N,
                                                const MinState* __restrict__ st) {
  if (st->done != 0 || st->pending == 0) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double tau = st->last_tau;
  double mi[3], gi[3], mo[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    mi[c] = m[(size_t)c * N + i];
    gi[c] = (double)g[(size_t)c * N + i];
  }
  cayley_step(mi, gi, tau, mo);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    m[(size_t)c * N + i] = mo[c];
    sb[(size_t)c * N + i] = (G)(mo[c] - mi[c]);
  }
}

__global__ void k_clear_pending(MinState* st) { st->pending = 0; }

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
  block_reduce<256>(v, is_max, scratch);
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
  block_reduce<256>(v, is_max, scratch);
  if (threadIdx.x == 0)
    for (int c = 0; c < 3; ++c) out[c] = v[c] / (double)N;
}

__global__ void k_reset_state(MinState* st, double tau0, double tol, long long max_iter,
                              long long stall_iters, int mode, double hx, double hy, double hz,
                              double bb_switch, LineSearch ls, double* ls_mbase, void* ls_g2) {
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
  z.pending = 0;
  z.H[0] = hx;
  z.H[1] = hy;
  z.H[2] = hz;
  z.sweep = 0;
  z.field = 0;
  z.n_fields = 0;
  z.fields = nullptr;
  z.mavg_out = nullptr;
  z.iters_out = nullptr;
  z.worst = 1;
  z.inv_N = 0.0;
  z.bb_switch = bb_switch;
  z.ls = ls;
  z.ls_trial = 0;
  z.ls_retry = 0;
  z.ls_nb = 0;
  z.ls_C = z.ls_Q = z.ls_G = 0.0;
  z.ls_mbase = ls_mbase;
  z.ls_g2 = ls_g2;
  z.fin_slot[0] = z.fin_slot[1] = kFinSent;
  z.fin_err = 0;
  *st = z;
}

// Turn a freshly reset state into a sweep over fields[0 .. n_fields).
__global__ void k_sweep_start(MinState* st, const double* fields, int n_fields, double* mavg_out,
                              long long* iters_out, double inv_N) {
  st->sweep = 1;
  st->field = 0;
  st->n_fields = n_fields;
  st->fields = fields;
  st->mavg_out = mavg_out;
  st->iters_out = iters_out;
  st->worst = 1;
  st->inv_N = inv_N;
  for (int c = 0; c < 3; ++c) st->H[c] = fields[c];
  if (n_fields <= 0) st->done = 1;
}

// Continue a run with new stop limits.  A state whose next action is already
// set (an update pending, an update applied since the last evaluation, or
// nothing evaluated yet) only takes the limits; a run that ended at its last
// evaluation takes that evaluation's decision again under the new limits,
// as the finish would have taken it: stop at T < tol or k >= max_iter, else
// the step of eq. (12) from the recorded sums (tau0 at k = 0) becomes the
// pending update.
__global__ void k_continue_state(MinState* st, double tol, long long max_iter,
                                 long long stall_iters) {
  st->tol = tol;
  st->max_iter = max_iter;
  st->stall_iters = stall_iters;
  st->mode = 0;
  st->sweep = 0;
  st->ls_trial = 0;
  st->ls_retry = 0;
  st->ls_nb = 0;
  st->fin_err = 0;
  if (st->done == -1) return;
  st->done = 0;
  const long long k = st->k;
  if (st->pending != 0 || k != st->last_k || st->evals == 0) return;
  if (st->torque < tol) {
    st->done = 1;
    return;
  }
  if (k >= max_iter) {
    st->done = 2;
    return;
  }
  double v[kNPartial] = {};
  v[0] = st->ss;
  v[1] = st->sy;
  v[2] = st->yy;
  const double tau = k > 0 ? bb_step(k, st->bb_switch, v, st->tau) : st->tau;
  st->tau = tau;
  st->last_tau = tau;
  st->k = k + 1;
  st->pending = 1;
}

void launch_continue_state(hipStream_t s, MinState* st, double tol, long long max_iter,
                           long long stall_iters) {
  hipLaunchKernelGGL(k_continue_state, dim3(1), dim3(1), 0, s, st, tol, max_iter, stall_iters);
}

// Switch the mode of a run without touching its BB history (clears done).
__global__ void k_set_mode(MinState* st, int mode) {
  st->mode = mode;
  st->done = 0;
}

void launch_reset_state(hipStream_t s, MinState* st, double tau0, double tol, long long max_iter,
                        long long stall_iters, int mode, const double H[3], double bb_switch,
                        const LineSearch* ls, double* ls_mbase, void* ls_g2) {
  LineSearch off;
  off.on = 0;
  off.eta = off.rho = off.sigma = 0.0;
  off.max_back = 0;
  hipLaunchKernelGGL(k_reset_state, dim3(1), dim3(1), 0, s, st, tau0, tol, max_iter, stall_iters,
                     mode, H[0], H[1], H[2], bb_switch, ls != nullptr ? *ls : off, ls_mbase,
                     ls_g2);
}

void launch_sweep_start(hipStream_t s, MinState* st, const double* fields, int n_fields,
                        double* mavg_out, long long* iters_out, double inv_N) {
  hipLaunchKernelGGL(k_sweep_start, dim3(1), dim3(1), 0, s, st, fields, n_fields, mavg_out,
                     iters_out, inv_N);
}

void launch_clear_pending(hipStream_t s, MinState* st) {
  hipLaunchKernelGGL(k_clear_pending, dim3(1), dim3(1), 0, s, st);
}

void launch_set_mode(hipStream_t s, MinState* st, int mode) {
  hipLaunchKernelGGL(k_set_mode, dim3(1), dim3(1), 0, s, st, mode);
}

int local_blocks(int N) { return (N + kLocalThreads - 1) / kLocalThreads; }

// Many per-block sums (large grids): a first stage in which block b sums
// rows kFinishThreads b .. kFinishThreads (b + 1) - 1 in the fixed order of
// block_reduce, writing one row per block to out; the one-block finish then
// sums those.  Few rows are summed by the finish block directly.
constexpr int kFinishDirect = 2048;

__global__ void __launch_bounds__(kFinishThreads)
k_finish_stage1(const double* __restrict__ partials, int nb, double* __restrict__ out,
                const MinState* __restrict__ st) {
  __shared__ double scratch[kNPartial * kFinishThreads / 64];
  const int dn = st->done;   // read while the sums' loads are in flight
  double v[kNPartial] = {};
  const int r = blockIdx.x * kFinishThreads + threadIdx.x;
  if (r < nb) {
#pragma unroll
    for (int q = 0; q < kNPartial; ++q) v[q] = partials[(size_t)r * kNPartial + q];
  }
  if (dn != 0) return;
  bool is_max[kNPartial];
  for (int q = 0; q < kNPartial; ++q) is_max[q] = q == kPartMax;
  block_reduce<kFinishThreads>(v, is_max, scratch);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < kNPartial; ++q) out[(size_t)blockIdx.x * kNPartial + q] = v[q];
  }
}

int finish_single_stage_max() { return kFinishDirect; }

int finish_extra_rows(int nblocks) {
  return nblocks > kFinishDirect ? (nblocks + kFinishThreads - 1) / kFinishThreads : 0;
}

// partials: nblocks rows, followed by room for finish_extra_rows(nblocks) more
void launch_finish(hipStream_t s, double* partials, int nblocks, MinState* st, double Ms,
                   double V) {
  if (nblocks > kFinishDirect) {
    const int nb2 = finish_extra_rows(nblocks);
    double* out = partials + (size_t)nblocks * kNPartial;
    hipLaunchKernelGGL(k_finish_stage1, dim3(nb2), dim3(kFinishThreads), 0, s, partials, nblocks,
                       out, st);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kFinishThreads), 0, s, out, nb2, st, Ms, V);
    return;
  }
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kFinishThreads), 0, s, partials, nblocks, st, Ms, V);
}

void launch_finish_batched(hipStream_t s, const BatchDesc* descs, int n_samples) {
  hipLaunchKernelGGL(k_finish_b, dim3(n_samples), dim3(kFinishThreads), 0, s, descs);
}

template <typename G>
void launch_update(hipStream_t s, double* m, const G* g, G* sbuf, int N, const MinState* st) {
  hipLaunchKernelGGL(k_update<G>, dim3((N + 255) / 256), dim3(256), 0, s, m, g, sbuf, N, st);
}
template void launch_update<double>(hipStream_t, double*, const double*, double*, int,
                                    const MinState*);
template void launch_update<float>(hipStream_t, double*, const float*, float*, int,
                                   const MinState*);

void launch_mean(hipStream_t s, const double* m, int N, double* partials, double* out3) {
  const int nb = (N + 255) / 256;
  hipLaunchKernelGGL(k_mean_partial, dim3(nb), dim3(256), 0, s, m, N, partials);
  hipLaunchKernelGGL(k_mean_finish, dim3(1), dim3(256), 0, s, partials, nb, N, out3);
}

}  // namespace mmk
