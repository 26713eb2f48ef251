// Derivatives of the energy U of Sec. 2 and of relaxed states: the
// Riemannian Hessian on the product of unit spheres, conjugate gradients for
// the adjoint field, the implicit parameter gradients and the energy
// derivatives used for automatic differentiation.  (Calculus on the paper's
// energy; the paper itself has no adjoint.)
//
//   Hess v   = mu0 Ms V [ -P(H_lin[v]) + (m . H_eff(m)) v ],  P_i = I - m_i m_i^T,
//              H_lin = demag + exchange + anisotropy (no Zeeman)
//   CG       Hess lam = P dJ/dm on the tangent space, x0 = 0
//   dJ/dKu_i = 2 V (m_i . u)(lam_i . u)
//   dJ/dA    = mu0 Ms V sum lam . H_ex(A = 1)
//   dJ/dMs   = mu0 V sum lam . (2 H_d + H_ext)
//   dJ/dH    = mu0 Ms V sum lam
//   dU/dm_i  = -mu0 Ms V H_eff,i,   dU/dKu_i = -V (m_i . u)^2
// Along the normal m_i the same expression has curvature m_i . H_eff,i, which
// is negative where the self-demag field dominates, so the operator is only
// ever applied to tangent fields: CG directions are projected every step
// (the identity in exact arithmetic) and mm_hessvec projects its input.
// Vectors are [3][N] double.  Sums are per-block partials reduced by one
// block in a fixed order, so results are deterministic.
#include "mm_device.h"
#include "mm_kernels.h"

namespace mmk {

constexpr int kAdjThreads = 256;

__device__ __forceinline__ void load3(const double* __restrict__ a, int N, int i, double v[3]) {
  v[0] = a[i];
  v[1] = a[(size_t)N + i];
  v[2] = a[2 * (size_t)N + i];
}
__device__ __forceinline__ void store3(double* __restrict__ a, int N, int i, const double v[3]) {
  a[i] = v[0];
  a[(size_t)N + i] = v[1];
  a[2 * (size_t)N + i] = v[2];
}
__device__ __forceinline__ double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

template <int NV>
__device__ __forceinline__ void write_partials(double (&v)[NV], double* __restrict__ partials) {
  __shared__ double scratch[NV * kAdjThreads / 64];
  const bool is_max[NV] = {};
  block_reduce<kAdjThreads>(v, is_max, scratch);
  if (threadIdx.x == 0)
    for (int q = 0; q < NV; ++q) partials[(size_t)blockIdx.x * NV + q] = v[q];
}

template <int NV>
__device__ __forceinline__ void sum_partials(const double* __restrict__ partials, int nb,
                                             double (&v)[NV]) {
  __shared__ double scratch[NV * kAdjThreads / 64];
  for (int q = 0; q < NV; ++q) v[q] = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x)
    for (int q = 0; q < NV; ++q) v[q] += partials[(size_t)b * NV + q];
  const bool is_max[NV] = {};
  block_reduce<kAdjThreads>(v, is_max, scratch);
}

// b = P rhs; x = 0; r = p = b; partial b.b
__global__ void __launch_bounds__(kAdjThreads)
k_cg_init(const double* __restrict__ m, const double* __restrict__ rhs, double* __restrict__ x,
          double* __restrict__ r, double* __restrict__ p, int N, double* __restrict__ partials) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double part[1] = {0.0};
  if (i < N) {
    double mi[3], b[3];
    load3(m, N, i, mi);
    load3(rhs, N, i, b);
    const double mb = dot3(mi, b);
    for (int c = 0; c < 3; ++c) b[c] -= mb * mi[c];
    const double z[3] = {0.0, 0.0, 0.0};
    store3(x, N, i, z);
    store3(r, N, i, b);
    store3(p, N, i, b);
    part[0] = dot3(b, b);
  }
  write_partials<1>(part, partials);
}

__global__ void __launch_bounds__(kAdjThreads)
k_cg_start(const double* __restrict__ partials, int nb, CGState* __restrict__ cg, double tol,
           long long max_iter) {
  double v[1];
  sum_partials<1>(partials, nb, v);
  if (threadIdx.x != 0) return;
  cg->bb = v[0];
  cg->rr = v[0];
  cg->tol2 = tol * tol;
  cg->k = 0;
  cg->max_iter = max_iter;
  cg->alpha = cg->beta = cg->pAp = 0.0;
  cg->done = !isfinite(v[0]) ? -1 : (v[0] == 0.0 ? 1 : (max_iter <= 0 ? 2 : 0));
}

// out = c [ -P(Hlin) + (m . Hm) v ]; optional partial v.out
__global__ void __launch_bounds__(kAdjThreads)
k_hess_apply(const double* __restrict__ m, const double* __restrict__ Hm,
             const double* __restrict__ Hlin, const double* __restrict__ v, double* __restrict__ out,
             int N, double c, double* __restrict__ partials, const int* __restrict__ done) {
  if (done != nullptr && *done != 0) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double part[1] = {0.0};
  if (i < N) {
    double mi[3], h[3], hl[3], vi[3], o[3];
    load3(m, N, i, mi);
    load3(Hm, N, i, h);
    load3(Hlin, N, i, hl);
    load3(v, N, i, vi);
    const double mh = dot3(mi, h), ml = dot3(mi, hl);
    for (int q = 0; q < 3; ++q) o[q] = c * (-(hl[q] - ml * mi[q]) + mh * vi[q]);
    store3(out, N, i, o);
    part[0] = dot3(vi, o);
  }
  if (partials != nullptr) write_partials<1>(part, partials);
}

__global__ void __launch_bounds__(kAdjThreads)
k_cg_alpha(const double* __restrict__ partials, int nb, CGState* __restrict__ cg) {
  if (cg->done != 0) return;
  double v[1];
  sum_partials<1>(partials, nb, v);
  if (threadIdx.x != 0) return;
  cg->pAp = v[0];
  // a non-positive curvature means m is not a strict local minimum
  if (!(v[0] > 0.0) || !isfinite(v[0])) cg->done = -1;
  else cg->alpha = cg->rr / v[0];
}

// x += alpha p; r -= alpha Ap; partial r.r
__global__ void __launch_bounds__(kAdjThreads)
k_cg_update(double* __restrict__ x, double* __restrict__ r, const double* __restrict__ p,
            const double* __restrict__ Ap, int N, const CGState* __restrict__ cg,
            double* __restrict__ partials) {
  if (cg->done != 0) return;
  const double alpha = cg->alpha;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double part[1] = {0.0};
  if (i < N) {
    for (int c = 0; c < 3; ++c) {
      const size_t j = (size_t)c * N + i;
      x[j] += alpha * p[j];
      const double rn = r[j] - alpha * Ap[j];
      r[j] = rn;
      part[0] += rn * rn;
    }
  }
  write_partials<1>(part, partials);
}

__global__ void __launch_bounds__(kAdjThreads)
k_cg_beta(const double* __restrict__ partials, int nb, CGState* __restrict__ cg) {
  if (cg->done != 0) return;
  double v[1];
  sum_partials<1>(partials, nb, v);
  if (threadIdx.x != 0) return;
  const double rr_new = v[0];
  cg->k += 1;
  cg->beta = rr_new / cg->rr;
  cg->rr = rr_new;
  if (!isfinite(rr_new)) cg->done = -1;
  else if (rr_new <= cg->tol2 * cg->bb) cg->done = 1;
  else if (cg->k >= cg->max_iter) cg->done = 2;
}

// p = P(r + beta p) (runs while the solve continues)
__global__ void __launch_bounds__(kAdjThreads)
k_cg_direction(const double* __restrict__ m, const double* __restrict__ r,
               double* __restrict__ p, int N, const CGState* __restrict__ cg) {
  if (cg->done != 0) return;
  const double beta = cg->beta;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double mi[3], ri[3], pi[3];
  load3(m, N, i, mi);
  load3(r, N, i, ri);
  load3(p, N, i, pi);
  for (int c = 0; c < 3; ++c) pi[c] = ri[c] + beta * pi[c];
  const double mp = dot3(mi, pi);
  for (int c = 0; c < 3; ++c) pi[c] -= mp * mi[c];
  store3(p, N, i, pi);
}

// out = P v
__global__ void __launch_bounds__(kAdjThreads)
k_project(const double* __restrict__ m, const double* __restrict__ v, double* __restrict__ out,
          int N) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double mi[3], vi[3];
  load3(m, N, i, mi);
  load3(v, N, i, vi);
  const double mv = dot3(mi, vi);
  for (int c = 0; c < 3; ++c) vi[c] -= mv * mi[c];
  store3(out, N, i, vi);
}

// dKu_i = 2 V (m.u)(lam.u); partials [lam . Hex1, lam . (2 Hd + Hext), sum lam]
__global__ void __launch_bounds__(kAdjThreads)
k_param_grads(const double* __restrict__ m, const double* __restrict__ lam,
              const double* __restrict__ Hd, const double* __restrict__ Hex1, double hx, double hy,
              double hz, double ux, double uy, double uz, double V, double* __restrict__ dKu, int N,
              double* __restrict__ partials) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double part[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (i < N) {
    double mi[3], li[3], hd[3], he[3];
    load3(m, N, i, mi);
    load3(lam, N, i, li);
    load3(Hd, N, i, hd);
    load3(Hex1, N, i, he);
    const double u[3] = {ux, uy, uz}, h[3] = {hx, hy, hz};
    part[0] = dot3(li, he);
    for (int q = 0; q < 3; ++q) part[1] += li[q] * (2.0 * hd[q] + h[q]);
    for (int q = 0; q < 3; ++q) part[2 + q] = li[q];
    if (dKu != nullptr) dKu[i] = 2.0 * V * dot3(mi, u) * dot3(li, u);
  }
  write_partials<5>(part, partials);
}

// out = c H (3N values); dKu_i = -V (m.u)^2 (may be NULL); partial sums of m
__global__ void __launch_bounds__(kAdjThreads)
k_energy_grads(const double* __restrict__ m, const double* __restrict__ H, double c,
               double* __restrict__ dm, double ux, double uy, double uz, double V,
               double* __restrict__ dKu, int N, double* __restrict__ partials) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double part[3] = {0.0, 0.0, 0.0};
  if (i < N) {
    double mi[3];
    load3(m, N, i, mi);
    if (dm != nullptr) {
      double h[3];
      load3(H, N, i, h);
      for (int q = 0; q < 3; ++q) h[q] *= c;
      store3(dm, N, i, h);
    }
    const double u[3] = {ux, uy, uz};
    const double mu = dot3(mi, u);
    if (dKu != nullptr) dKu[i] = -V * mu * mu;
    for (int q = 0; q < 3; ++q) part[q] = mi[q];
  }
  write_partials<3>(part, partials);
}

template <int NV>
__global__ void __launch_bounds__(kAdjThreads)
k_sums_finish(const double* __restrict__ partials, int nb, double* __restrict__ out) {
  double v[NV];
  sum_partials<NV>(partials, nb, v);
  if (threadIdx.x == 0)
    for (int q = 0; q < NV; ++q) out[q] = v[q];
}

// ---------------------------------------------------------------------------
int adj_blocks(int N) { return (N + kAdjThreads - 1) / kAdjThreads; }

void launch_cg_init(hipStream_t s, const double* m, const double* rhs, double* x, double* r,
                    double* p, int N, double* partials, CGState* cg, double tol,
                    long long max_iter) {
  const int nb = adj_blocks(N);
  hipLaunchKernelGGL(k_cg_init, dim3(nb), dim3(kAdjThreads), 0, s, m, rhs, x, r, p, N, partials);
  hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(kAdjThreads), 0, s, partials, nb, cg, tol, max_iter);
}

void launch_hess_apply(hipStream_t s, const double* m, const double* Hm, const double* Hlin,
                       const double* v, double* out, int N, double c, double* partials,
                       const int* done) {
  hipLaunchKernelGGL(k_hess_apply, dim3(adj_blocks(N)), dim3(kAdjThreads), 0, s, m, Hm, Hlin, v,
                     out, N, c, partials, done);
}

void launch_project(hipStream_t s, const double* m, const double* v, double* out, int N) {
  hipLaunchKernelGGL(k_project, dim3(adj_blocks(N)), dim3(kAdjThreads), 0, s, m, v, out, N);
}

void launch_cg_step(hipStream_t s, const double* m, double* x, double* r, double* p,
                    const double* Ap, int N, double* partials, CGState* cg) {
  const int nb = adj_blocks(N);
  hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(kAdjThreads), 0, s, partials, nb, cg);
  hipLaunchKernelGGL(k_cg_update, dim3(nb), dim3(kAdjThreads), 0, s, x, r, p, Ap, N, cg, partials);
  hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(kAdjThreads), 0, s, partials, nb, cg);
  hipLaunchKernelGGL(k_cg_direction, dim3(nb), dim3(kAdjThreads), 0, s, m, r, p, N, cg);
}

void launch_param_grads(hipStream_t s, const double* m, const double* lam, const double* Hd,
                        const double* Hex1, const double H[3], const double u[3], double V,
                        double* dKu, int N, double* partials, double* out5) {
  const int nb = adj_blocks(N);
  hipLaunchKernelGGL(k_param_grads, dim3(nb), dim3(kAdjThreads), 0, s, m, lam, Hd, Hex1, H[0],
                     H[1], H[2], u[0], u[1], u[2], V, dKu, N, partials);
  hipLaunchKernelGGL(k_sums_finish<5>, dim3(1), dim3(kAdjThreads), 0, s, partials, nb, out5);
}

void launch_energy_grads(hipStream_t s, const double* m, const double* H, double c, double* dm,
                         const double u[3], double V, double* dKu, int N, double* partials,
                         double* out3) {
  const int nb = adj_blocks(N);
  hipLaunchKernelGGL(k_energy_grads, dim3(nb), dim3(kAdjThreads), 0, s, m, H, c, dm, u[0], u[1],
                     u[2], V, dKu, N, partials);
  hipLaunchKernelGGL(k_sums_finish<3>, dim3(1), dim3(kAdjThreads), 0, s, partials, nb, out3);
}

}  // namespace mmk
