// Fused x passes of one minimiser iteration (thin-film path).
//
//   k_xf   pending midpoint update of eq. (7) on R rows (all three
//          components), s = m+ - m, then the forward half-length real FFT
//          along x of the updated rows into the spectrum A[kx][z][y][c].
//   k_xil  inverse x transform of R rows (all three components) -> H_d, then
//          the local terms, g = m x (m x H) (eq. (8)), the BB sums and the
//          energy sums of the rows (eq. (12), Sec. 2), one set per block;
//          a one-block kernel that follows reduces them in a fixed order and
//          applies the stop rule and the alternating step choice.  (A fused
//          "last block finishes" variant needs a device-scope release per
//          block, which writes back the XCD's L2 and cost more than the
//          extra launch.)
// Block b works on rows (z, y0 .. y0+R-1) with the XCD-contiguous mapping
// of xcd_remap so that neighbouring row groups share L2.
// Defect correction (single-precision form): k_xf may transform m - mref
// instead of m, and k_xil then adds the double-precision field of mref; a
// reference pass (double precision) copies m to mref without updating it.
#include "mm_iter.h"
#include "mm_wfft.h"

namespace mmk {

constexpr int kXsThreads = 512;   // launch bound of the LDS-Stockham x passes
constexpr int kXwThreads = 768;   // launch bound of the wave-FFT x passes (R <= 4)

template <typename T, int VPT>
__global__ void __launch_bounds__(kXsThreads)
k_xf(double* __restrict__ m, const T* __restrict__ g, T* __restrict__ sbuf,
     const MinState* __restrict__ st, int nx, int ny, int nz, int Px, int R,
     cx<T>* __restrict__ out, const cx<T>* __restrict__ twx, const double* __restrict__ msub,
     double* __restrict__ mcopy) {
  bool upd = false, ls_upd = false, retry = false;
  double tau = 0.0;
  double* mbase = nullptr;
  const T* g2 = nullptr;
  if (st != nullptr) {
    if (st->done != 0) return;
    upd = st->pending != 0 && mcopy == nullptr;
    tau = st->last_tau;
    ls_upd = upd && st->ls.on != 0;
    retry = st->ls_retry != 0;
    mbase = st->ls_mbase;
    g2 = static_cast<const T*>(st->ls_g2);
  }
  extern __shared__ __align__(16) unsigned char smem[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
  const int M = Px >> 1;
  const int nyb = (ny + R - 1) / R;
  const int nb = nz * nyb;
  const int L = xcd_remap(blockIdx.x, nb);
  const int z = L / nyb;
  const int y0 = (L - z * nyb) * R;
  const int N = nx * ny * nz;
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int idx = tid; idx < R * M; idx += nthr) {
    const int r = idx / M, j = idx - r * M;
    const int y = y0 + r;
    T v0[3] = {T(0), T(0), T(0)}, v1[3] = {T(0), T(0), T(0)};
    if (y < ny) {
      const size_t row = ((size_t)z * ny + y) * nx;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int x = 2 * j + h;
        if (x >= nx) break;
        const size_t i = row + x;
        double mi[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) mi[c] = m[(size_t)c * N + i];
        if (upd) {
          double gi[3], mo[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) gi[c] = (double)g[(size_t)c * N + i];
          if (ls_upd) {
            // line search: see the wave-FFT pass below
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              if (retry) {
                mi[c] = mbase[(size_t)c * N + i];
              } else {
                gi[c] = (double)g2[(size_t)c * N + i];
                mbase[(size_t)c * N + i] = mi[c];
                const_cast<T*>(g)[(size_t)c * N + i] = g2[(size_t)c * N + i];
              }
            }
          }
          cayley_step(mi, gi, tau, mo);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            m[(size_t)c * N + i] = mo[c];
            sbuf[(size_t)c * N + i] = (T)(mo[c] - mi[c]);
            mi[c] = mo[c];
          }
        }
        if (mcopy != nullptr) {
#pragma unroll
          for (int c = 0; c < 3; ++c) mcopy[(size_t)c * N + i] = mi[c];
        }
        if (msub != nullptr) {
#pragma unroll
          for (int c = 0; c < 3; ++c) mi[c] -= msub[(size_t)c * N + i];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if (h == 0) v0[c] = (T)mi[c];
          else v1[c] = (T)mi[c];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) buf[(c * R + r) * M + j] = mk(v0[c], v1[c]);
  }
  __syncthreads();
  fft_lds<-1, VPT>(buf, M, 3 * R, M, twx, Px, tid, nthr);
  const size_t slab = (size_t)3 * nz * ny;
  const int q3 = 3 * R;
  for (int idx = tid; idx < (M + 1) * q3; idx += nthr) {
    const int k = idx / q3, q = idx - k * q3;
    const int r = q / 3, c = q - r * 3;       // [z][y][c] order: contiguous in q
    const int y = y0 + r;
    if (y >= ny) continue;
    const cx<T>* row = buf + (c * R + r) * M;
    const cx<T> zk = row[k == M ? 0 : k];
    const cx<T> zc = conj(row[k == 0 ? 0 : M - k]);
    const cx<T> w = twx[k];
    out[(size_t)k * slab + ((size_t)z * ny + y) * 3 + c] =
        scl(add(add(zk, zc), rot90<-1>(mul(w, sub(zk, zc)))), T(0.5));
  }
}

template <typename T, int VPT>
__global__ void __launch_bounds__(kXsThreads)
k_xil(const cx<T>* __restrict__ in, LocalArgs a, int Px, int R, double* __restrict__ Hd_out,
      double* __restrict__ partials, const cx<T>* __restrict__ twx) {
  if (a.done != nullptr && *a.done != 0) return;
  if (a.Hdyn != nullptr)
    for (int c = 0; c < 3; ++c) a.H[c] = a.Hdyn[c];
  extern __shared__ __align__(16) unsigned char smem[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
  __shared__ double scratch[kNPartial * kXsThreads / 64];
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int M = Px >> 1;
  const int nyb = (ny + R - 1) / R;
  const int nb = nz * nyb;
  const int L = xcd_remap(blockIdx.x, nb);
  const int z = L / nyb;
  const int y0 = (L - z * nyb) * R;
  const int N = nx * ny * nz;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const size_t slab = (size_t)3 * nz * ny;
  const int q3 = 3 * R;
  for (int idx = tid; idx < M * q3; idx += nthr) {
    const int k = idx / q3, q = idx - k * q3;
    const int r = q / 3, c = q - r * 3;
    const int y = y0 + r;
    cx<T> Zv = mk(T(0), T(0));
    if (y < ny) {
      const size_t col = ((size_t)z * ny + y) * 3 + c;
      const cx<T> Xk = in[(size_t)k * slab + col];
      const cx<T> Xc = conj(in[(size_t)(M - k) * slab + col]);
      const cx<T> wi = conj(twx[k]);
      Zv = scl(add(add(Xk, Xc), rot90<1>(mul(wi, sub(Xk, Xc)))), T(0.5));
    }
    buf[(c * R + r) * M + k] = Zv;
  }
  __syncthreads();
  fft_lds<1, VPT>(buf, M, q3, M, twx, Px, tid, nthr);
  const bool bb = a.g != nullptr && a.s != nullptr && a.st != nullptr &&
                  (a.st->k > 0 || a.st->ls_trial != 0);
  double part[kNPartial] = {};
  for (int idx = tid; idx < R * nx; idx += nthr) {
    const int r = idx / nx, x = idx - r * nx;
    const int y = y0 + r;
    if (y >= ny) continue;
    const int i = (z * ny + y) * nx + x;
    double hd[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const cx<T> v = buf[(c * R + r) * M + (x >> 1)];
      hd[c] = (double)((x & 1) ? v.y : v.x);
      if (a.Hd_add != nullptr) hd[c] += a.Hd_add[(size_t)c * N + i];
    }
    if (Hd_out != nullptr) {
#pragma unroll
      for (int c = 0; c < 3; ++c) Hd_out[(size_t)c * N + i] = hd[c];
    }
    local_cell<T>(a, i, hd, bb, part);
  }
  bool is_max[kNPartial];
  for (int q = 0; q < kNPartial; ++q) is_max[q] = q == kPartMax;
  block_reduce<kXsThreads>(part, is_max, scratch);
  if (partials != nullptr && tid == 0) {
#pragma unroll
    for (int v = 0; v < kNPartial; ++v) partials[(size_t)L * kNPartial + v] = part[v];
  }
}

// ---------------------------------------------------------------------------
// Wave-FFT variants (M = Px/2 = 64 VL, VL in 1..8).  A block holds R
// rows; wave w = 3 r + c transforms component c of row r.  Each (row,
// component) owns an LDS region of wx_region<VL>() elements, used in turn
// for the natural-order sequence, the transposes of the wave FFT and the
// spectrum X[0..M]; natural index k is stored at wx_pad(k) = k + k/8 so that
// the permuted writes of the wave FFT (lanes 8 apart) avoid bank conflicts.
// Global traffic goes through LDS so that every block moves contiguous
// chunks of 3 R values per kx.  The region length is 3 mod 8 elements, so
// that the 3 R regions read or written at one kx (one per lane of a chunk)
// start on different LDS banks.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int wx_region_of(int VL) { return VL * 72 + 11; }
template <int VL>
__host__ __device__ constexpr int wx_region() { return wx_region_of(VL); }
__device__ __forceinline__ int wx_pad(int k) { return k + (k >> 3); }

// The previous iteration's finish taken over by a forward x pass (FinFuse,
// partials set).  Block 0 reduces the sums and decides (the finish kernel's
// order and arithmetic), then publishes the word the pass needs; every
// other block's thread 0 polls for it.  Both return the word in every
// thread of the block (block-uniform; they contain block barriers).
__device__ __forceinline__ double fin_decide(const FinFuse& fz) {
  __shared__ double s_w;
  __shared__ double scratch[kNPartial * kXwThreads / 64];
  finish_in_block<kXwThreads, 1>(fz.partials, fz.nb, fz.st, fz.Ms, fz.V, scratch);
  if (threadIdx.x == 0) {
    const MinState* st = fz.st;   // this thread's own writes of the decision
    const double w = st->done != 0 ? kFinStop : (st->pending != 0 ? st->last_tau : kFinNoUpdate);
    __hip_atomic_store(&fz.st->fin_slot[fz.par], (unsigned long long)__double_as_longlong(w),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_w = w;
  }
  __syncthreads();
  return s_w;
}

__device__ __forceinline__ double fin_wait(const FinFuse& fz) {
  __shared__ double s_w;
  if (threadIdx.x == 0) {
    unsigned long long* slot = &fz.st->fin_slot[fz.par];
    unsigned long long b = kFinSent;
    for (int n = 0; n < fz.spin; ++n) {
      b = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (b != kFinSent) break;
      __builtin_amdgcn_s_sleep(2);
    }
    if (b == kFinSent) {   // gave up: this block writes nothing; the host reports it
      __hip_atomic_store(&fz.st->fin_err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      b = (unsigned long long)__double_as_longlong(kFinStop);
    }
    s_w = __longlong_as_double((long long)b);
  }
  __syncthreads();
  return s_w;
}

// Body of the forward x pass for logical block L (rows z, y0 .. y0+R-1).
// FUSE: the pass takes the previous iteration's finish over (fz.st set).
template <typename T, int VL, bool FUSE>
__device__ __forceinline__ void xf_w_body(double* __restrict__ m, const T* __restrict__ g,
                                          T* __restrict__ sbuf, const MinState* st, int nx,
                                          int ny, int nz, int R, cx<T>* __restrict__ out,
                                          const cx<T>* __restrict__ twx, int L,
                                          const double* __restrict__ msub,
                                          double* __restrict__ mcopy, const FinFuse& fz) {
  constexpr int M = 64 * VL;
  constexpr int NG = 8 * VL;
  constexpr int RG = wx_region<VL>();
  // The state is read while the first cells' loads are in flight: nothing
  // branches on it before they are issued, and a finished run (done) writes
  // nothing and leaves after phase 1 (the flag is the same for the block).
  int done = 0, pend = 0, ls = 0, retry = 0;
  double tau = 0.0;
  double* mbase = nullptr;
  const T* g2 = nullptr;
  if (st != nullptr) {
    done = st->done;
    pend = st->pending;
    tau = st->last_tau;
    ls = st->ls.on;
    retry = st->ls_retry;
    mbase = st->ls_mbase;
    g2 = static_cast<const T*>(st->ls_g2);
  }
  extern __shared__ __align__(16) unsigned char smem[];
  cx<T>* sm = reinterpret_cast<cx<T>*>(smem);
  T* smr = reinterpret_cast<T*>(smem);
  const int nyb = (ny + R - 1) / R;
  const int z = L / nyb;
  const int y0 = (L - z * nyb) * R;
  const int rows = min(R, ny - y0);
  const int N = nx * ny * nz;
  const int tid = thread_index(), nthr = 192 * R;
  // the row-parallel loops take 192 R threads (a persistent launch may have
  // more: they only join the barriers), so that every cell is summed by the
  // same thread as in a launch of exactly 192 R threads
  const int first = tid < nthr ? tid : (1 << 30);
  // phase 1: pending update of the rows, sequences into LDS (x = 2j + h -> re/im of j)
  {
    constexpr int U = 4;                       // cells in flight per thread
    const int total = rows * nx;
    const size_t row0 = ((size_t)z * ny + y0) * nx;   // rows of the block are contiguous
    // one cell of phase 1: line-search base handling, the pending update
    // (eq. (7)) with s = m+ - m, the copy / subtraction of the reference,
    // and the sequence value into LDS
    auto cell = [&](int idx, double (&mi)[3], double (&gi)[3], bool upd, bool ls_upd) {
      const int r = idx / nx, x = idx - r * nx;
      const size_t i = row0 + idx;
      if (ls_upd) {
        // line search: the trial starts from the saved base (retry) or from
        // the accepted state in m with the gradient of its evaluation in
        // g2, which then become the saved base (mbase, g)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if (retry) {
            mi[c] = mbase[(size_t)c * N + i];
          } else {
            const T gt = g2[(size_t)c * N + i];
            gi[c] = (double)gt;
            mbase[(size_t)c * N + i] = mi[c];
            const_cast<T*>(g)[(size_t)c * N + i] = gt;
          }
        }
      }
      if (upd) {
        double mo[3];
        cayley_step(mi, gi, tau, mo);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          m[(size_t)c * N + i] = mo[c];
          sbuf[(size_t)c * N + i] = (T)(mo[c] - mi[c]);
          mi[c] = mo[c];
        }
      }
      if (mcopy != nullptr && done == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) mcopy[(size_t)c * N + i] = mi[c];
      }
      if (msub != nullptr) {
#pragma unroll
        for (int c = 0; c < 3; ++c) mi[c] -= msub[(size_t)c * N + i];
      }
#pragma unroll
      for (int c = 0; c < 3; ++c)
        smr[2 * ((size_t)(r * 3 + c) * RG + (x >> 1)) + (x & 1)] = (T)mi[c];
    };
    if constexpr (!FUSE) {
      // the cell code written out in the loop: through the lambda the
      // compiler holds this pass at 134 VGPRs instead of 128 (3 waves per
      // SIMD instead of 4)
      const bool upd = pend != 0 && done == 0 && mcopy == nullptr;
      const bool ls_upd = upd && ls != 0;
      for (int base = first; base < total; base += U * nthr) {
        double mi[U][3], gi[U][3];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int idx = base + u * nthr;
          if (idx < total) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              mi[u][c] = m[(size_t)c * N + row0 + idx];
              gi[u][c] = g != nullptr ? (double)g[(size_t)c * N + row0 + idx] : 0.0;
            }
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int idx = base + u * nthr;
          if (idx >= total) continue;
          const int r = idx / nx, x = idx - r * nx;
          const size_t i = row0 + idx;
          if (ls_upd) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              if (retry) {
                mi[u][c] = mbase[(size_t)c * N + i];
              } else {
                const T gt = g2[(size_t)c * N + i];
                gi[u][c] = (double)gt;
                mbase[(size_t)c * N + i] = mi[u][c];
                const_cast<T*>(g)[(size_t)c * N + i] = gt;
              }
            }
          }
          if (upd) {
            double mo[3];
            cayley_step(mi[u], gi[u], tau, mo);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              m[(size_t)c * N + i] = mo[c];
              sbuf[(size_t)c * N + i] = (T)(mo[c] - mi[u][c]);
              mi[u][c] = mo[c];
            }
          }
          if (mcopy != nullptr && done == 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) mcopy[(size_t)c * N + i] = mi[u][c];
          }
          if (msub != nullptr) {
#pragma unroll
            for (int c = 0; c < 3; ++c) mi[u][c] -= msub[(size_t)c * N + i];
          }
#pragma unroll
          for (int c = 0; c < 3; ++c)
            smr[2 * ((size_t)(r * 3 + c) * RG + (x >> 1)) + (x & 1)] = (T)mi[u][c];
        }
      }
    } else {
      double mi[U][3], gi[U][3];
      auto load = [&](int base) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int idx = base + u * nthr;
          if (idx < total) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              mi[u][c] = m[(size_t)c * N + row0 + idx];
              gi[u][c] = g != nullptr ? (double)g[(size_t)c * N + row0 + idx] : 0.0;
            }
          }
        }
      };
      // block 0 clears the slot of the next pass; with a finish to take
      // over, its decision replaces the state read above (blocks other than
      // 0 issue their first cells' loads before they wait for it)
      bool prefetched = false;
      if (blockIdx.x == 0 && threadIdx.x == 0) fz.st->fin_slot[fz.par ^ 1] = kFinSent;
      if (fz.partials != nullptr) {
        double w;
        if (blockIdx.x == 0) {
          w = fin_decide(fz);
        } else {
          load(first);
          prefetched = true;
          w = fin_wait(fz);
        }
        // block-uniform: taken into scalar registers, so that the update's
        // branches stay uniform as with the state read above
        const long long wb = __double_as_longlong(w);
        const int lo = __builtin_amdgcn_readfirstlane((int)(wb & 0xffffffffll));
        const int hi = __builtin_amdgcn_readfirstlane((int)(wb >> 32));
        w = __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
        done = w == kFinStop ? 1 : 0;
        pend = w > 0.0 ? 1 : 0;
        tau = w;
      }
      const bool upd = pend != 0 && done == 0 && mcopy == nullptr;
      const bool ls_upd = upd && ls != 0;
      for (int base = first; base < total; base += U * nthr) {
        if (!(prefetched && base == first)) load(base);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int idx = base + u * nthr;
          if (idx < total) cell(idx, mi[u], gi[u], upd, ls_upd);
        }
      }
    }
  }
  if (done != 0) return;
  // zero padding x in [nx, 2M)
  const int jz = nx >> 1;   // first complex slot holding padding (its .y if nx is odd)
  for (int idx = first; idx < rows * 3 * (M - jz); idx += nthr) {
    const int q = idx / (M - jz), j = jz + idx - q * (M - jz);
    if (2 * j >= nx) sm[(size_t)q * RG + j] = mk(T(0), T(0));
    else smr[2 * ((size_t)q * RG + j) + 1] = T(0);          // x = nx - 1 even: .y is padding
  }
  __syncthreads();
  // phase 2: wave FFT of one (row, component)
  const int lane = tid & 63, w = tid >> 6;
  const int r = w / 3, c = w - r * 3;
  cx<T>* reg = sm + (size_t)w * RG;
  if (r < rows) {
    cx<T> v[VL], u[8];
    // element by element: as one aggregate copy the single element of the
    // 64-point transform stayed in scratch memory across the barrier
#pragma unroll
    for (int q = 0; q < VL; ++q) {
      const cx<T>& e = reg[lane + 64 * q];
      v[q] = mk(e.x, e.y);
    }
    __builtin_amdgcn_wave_barrier();
    wfft_forward<T, VL, false, 2>(v, u, reg, twx, lane);   // table of length Px = 2M
    __builtin_amdgcn_wave_barrier();
    if (lane < NG) {
#pragma unroll
      for (int d = 0; d < 8; ++d) reg[wx_pad(wfft_freq<VL>(lane, d))] = u[d];
    }
    __builtin_amdgcn_wave_barrier();
    // split into the spectrum of the real row: X[k] = (Zk + Zc)/2 - i W^k (Zk - Zc)/2
    cx<T> X[VL + 1];
#pragma unroll
    for (int q = 0; q <= VL; ++q) {
      const int k = lane + 64 * q;
      const int kk = k < M ? k : 0;
      const int km = k == 0 ? 0 : (k >= M ? 0 : M - k);
      const cx<T> zk = reg[wx_pad(kk)];
      const cx<T> zc = conj(reg[wx_pad(km)]);
      const cx<T> wk = twx[k < M ? k : M];
      X[q] = scl(add(add(zk, zc), rot90<-1>(mul(wk, sub(zk, zc)))), T(0.5));
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int q = 0; q <= VL; ++q) {
      const int k = lane + 64 * q;
      if (k <= M) reg[wx_pad(k)] = X[q];
    }
  }
  __syncthreads();
  // phase 3: contiguous chunks of 3 R values per kx
  const size_t slab = (size_t)3 * nz * ny;
  const int q3 = 3 * rows;
  cx<T>* dst = out + ((size_t)z * ny + y0) * 3;
  for (int idx = first; idx < (M + 1) * q3; idx += nthr) {
    const int k = idx / q3, q = idx - k * q3;
    dst[(size_t)k * slab + q] = sm[(size_t)q * RG + wx_pad(k)];
  }
}

template <typename T, int VL, bool FUSE>
__global__ void __launch_bounds__(kXwThreads)
k_xf_w(double* __restrict__ m, const T* __restrict__ g, T* __restrict__ sbuf,
       const MinState* st, int nx, int ny, int nz, int R, cx<T>* __restrict__ out,
       const cx<T>* __restrict__ twx, const double* __restrict__ msub,
       double* __restrict__ mcopy, FinFuse fz) {
  xf_w_body<T, VL, FUSE>(m, g, sbuf, st, nx, ny, nz, R, out, twx,
                         xcd_remap(blockIdx.x, gridDim.x), msub, mcopy, fz);
}

// Body of the inverse x pass with the local terms for logical block L.
template <typename T, int VL>
__device__ __forceinline__ void xil_w_body(const cx<T>* __restrict__ in, LocalArgs a, int R,
                                           double* __restrict__ Hd_out,
                                           double* __restrict__ partials,
                                           const cx<T>* __restrict__ twx, int L) {
  constexpr int M = 64 * VL;
  constexpr int NG = 8 * VL;
  constexpr int RG = wx_region<VL>();
  // state read while the spectrum loads are in flight; a finished run leaves
  // after phase 1 (LDS writes only)
  const int done = a.done != nullptr ? *a.done : 0;
  const long long kst = a.st != nullptr ? a.st->k : 0;
  const int lst = a.st != nullptr ? a.st->ls_trial : 0;
  if (a.Hdyn != nullptr)
    for (int c = 0; c < 3; ++c) a.H[c] = a.Hdyn[c];
  extern __shared__ __align__(16) unsigned char smem[];
  cx<T>* sm = reinterpret_cast<cx<T>*>(smem);
  __shared__ double scratch[kNPartial * kXwThreads / 64];
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int nyb = (ny + R - 1) / R;
  const int z = L / nyb;
  const int y0 = (L - z * nyb) * R;
  const int rows = min(R, ny - y0);
  const int N = nx * ny * nz;
  const int tid = thread_index(), nthr = 192 * R;
  // the row-parallel loops take 192 R threads (a persistent launch may have
  // more: they only join the barriers), so that every cell is summed by the
  // same thread as in a launch of exactly 192 R threads
  const int first = tid < nthr ? tid : (1 << 30);
  // phase 1: spectrum chunks into LDS
  const size_t slab = (size_t)3 * nz * ny;
  const int q3 = 3 * rows;
  const cx<T>* src = in + ((size_t)z * ny + y0) * 3;
  {
    constexpr int U = 8;                       // loads in flight per thread
    const int total = (M + 1) * q3;
    for (int base = first; base < total; base += U * nthr) {
      T re[U], im[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int idx = min(base + u * nthr, total - 1);
        const int k = idx / q3, q = idx - k * q3;
        const cx<T> v = src[(size_t)k * slab + q];
        re[u] = v.x;
        im[u] = v.y;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int idx = base + u * nthr;
        if (idx < total) {
          const int k = idx / q3, q = idx - k * q3;
          sm[(size_t)q * RG + wx_pad(k)] = mk(re[u], im[u]);
        }
      }
    }
  }
  if (done != 0) return;
  __syncthreads();
  // phase 2: inverse real transform of one (row, component):
  // Z[k] = (X[k] + conj X[M-k])/2 + i W^-k (X[k] - conj X[M-k])/2, then
  // z = conj(FFT(conj Z)) and the row samples are x[2j] = Re z[j], x[2j+1] = Im z[j]
  const int lane = tid & 63, w = tid >> 6;
  const int r = w / 3, c = w - r * 3;
  cx<T>* reg = sm + (size_t)w * RG;
  if (r < rows) {
    cx<T> v[VL], u[8];
#pragma unroll
    for (int q = 0; q < VL; ++q) {
      const int k = lane + 64 * q;
      const cx<T> Xk = reg[wx_pad(k)];
      const cx<T> Xc = conj(reg[wx_pad(M - k)]);
      const cx<T> wi = conj(twx[k]);
      v[q] = conj(scl(add(add(Xk, Xc), rot90<1>(mul(wi, sub(Xk, Xc)))), T(0.5)));
    }
    __builtin_amdgcn_wave_barrier();
    wfft_forward<T, VL, false, 2>(v, u, reg, twx, lane);   // table of length Px = 2M
    __builtin_amdgcn_wave_barrier();
    if (lane < NG) {
#pragma unroll
      for (int d = 0; d < 8; ++d) reg[wx_pad(wfft_freq<VL>(lane, d))] = conj(u[d]);
    }
  }
  __syncthreads();
  // phase 3: local terms of the rows
  const bool bb = a.g != nullptr && a.s != nullptr && a.st != nullptr && (kst > 0 || lst != 0);
  double part[kNPartial] = {};
  {
    constexpr int U = 1;                       // cells per thread per round
    const int total = rows * nx;
    const int row0 = (z * ny + y0) * nx;
    for (int base = first; base < total; base += U * nthr) {
      CellIn cin[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int idx = base + u * nthr;
        if (idx < total) fetch_cell<T>(a, row0 + idx, bb, cin[u]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int idx = base + u * nthr;
        if (idx >= total) continue;
        const int rr = idx / nx, x = idx - rr * nx;
        const int i = row0 + idx;
        double hd[3];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
          const cx<T> v = sm[(size_t)(rr * 3 + cc) * RG + wx_pad(x >> 1)];
          hd[cc] = (double)((x & 1) ? v.y : v.x);
          if (a.Hd_add != nullptr) hd[cc] += a.Hd_add[(size_t)cc * N + i];
        }
        if (Hd_out != nullptr) {
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) Hd_out[(size_t)cc * N + i] = hd[cc];
        }
        compute_cell<T>(a, i, hd, bb, cin[u], part);
      }
    }
  }
  bool is_max[kNPartial];
  for (int q = 0; q < kNPartial; ++q) is_max[q] = q == kPartMax;
  if (partials != nullptr)
    block_reduce_store<kXwThreads>(part, is_max, scratch, partials + (size_t)L * kNPartial);
}

template <typename T, int VL>
__global__ void __launch_bounds__(kXwThreads)
k_xil_w(const cx<T>* __restrict__ in, LocalArgs a, int R, double* __restrict__ Hd_out,
        double* __restrict__ partials, const cx<T>* __restrict__ twx) {
  xil_w_body<T, VL>(in, a, R, Hd_out, partials, twx, xcd_remap(blockIdx.x, gridDim.x));
}

// ---- batched passes: one launch covers the blocks of several samples ---------
// items[b] names the sample and its logical block; every sample of a launch
// has the same transform length and rows per block.
// Logical block `block` of sample d's forward x pass.
template <typename T, int VL>
__device__ __forceinline__ void xf_desc(const BatchDesc& d, int block) {
  const FinFuse none{nullptr, nullptr, 0.0, 0.0, 0, 0, 0};
  xf_w_body<T, VL, false>(d.m, static_cast<const T*>(d.g), static_cast<T*>(d.s), d.st, d.nx, d.ny,
                   d.nz, d.R, (cx<T>*)d.spec, (const cx<T>*)d.twx, block,
                   d.pass == 1 ? d.mref : nullptr, d.pass == 2 ? d.mref : nullptr, none);
}

template <typename T, int VL>
__global__ void __launch_bounds__(kXwThreads)
k_xf_wb(const BatchDesc* __restrict__ descs, const WorkItem* __restrict__ items) {
  const WorkItem it = items[blockIdx.x];
  xf_desc<T, VL>(descs[it.sample], it.block);
}

// Logical block `block` of sample d's inverse x pass with its local terms.
template <typename T, int VL>
__device__ __forceinline__ void xil_desc(const BatchDesc& d, int block) {
  LocalArgs a;
  a.m = d.m;
  a.Hd = nullptr;
  a.g = d.g;
  a.g_out = nullptr;
  a.s = d.s;
  a.Hout = nullptr;
  a.Hex_out = nullptr;
  a.Han_out = nullptr;
  a.ku_map = d.ku_map;
  a.nx = d.nx;
  a.ny = d.ny;
  a.nz = d.nz;
  a.cx = d.cx;
  a.cy = d.cy;
  a.cz = d.cz;
  a.ku = d.ku;
  a.kan = d.kan;
  for (int c = 0; c < 3; ++c) {
    a.u[c] = d.u[c];
    a.H[c] = 0.0;
  }
  a.Hdyn = d.st->H;
  a.Hd_add = d.pass == 1 ? d.hdref : nullptr;
  a.partials = d.partials;
  a.st = d.st;
  a.done = &d.st->done;
  if (d.pass == 2) {
    // reference pass: the demag field of mref only
    a.g = nullptr;
    a.s = nullptr;
    a.st = nullptr;
    xil_w_body<T, VL>((const cx<T>*)d.spec, a, d.R, d.hdref, nullptr, (const cx<T>*)d.twx,
                      block);
    return;
  }
  xil_w_body<T, VL>((const cx<T>*)d.spec, a, d.R, nullptr, d.partials, (const cx<T>*)d.twx,
                    block);
}

template <typename T, int VL>
__global__ void __launch_bounds__(kXwThreads)
k_xil_wb(const BatchDesc* __restrict__ descs, const WorkItem* __restrict__ items) {
  const WorkItem it = items[blockIdx.x];
  xil_desc<T, VL>(descs[it.sample], it.block);
}

// ---- persistent batched x passes ------------------------------------------------
// One launch covers the blocks of every sample, whatever its transform length
// M = 64 VL: the grid holds the blocks that stay resident together and each
// block takes its static share of the table (persist_loop) and branches on
// the item's sample length.  A sample's rows per block R may be
// below the launch's blockDim.x / 192 (the surplus waves then skip the
// transform).
template <typename T, bool INV>
__device__ __forceinline__ void x_item(const BatchDesc& d, int block) {
  switch (d.M >> 6) {
#define MMK_X_CASE(V)                          \
  case V:                                      \
    if (INV) xil_desc<T, V>(d, block);         \
    else xf_desc<T, V>(d, block);              \
    break;
    MMK_X_CASE(1)
    MMK_X_CASE(2)
    MMK_X_CASE(3)
    MMK_X_CASE(4)
    MMK_X_CASE(5)
    MMK_X_CASE(6)
    MMK_X_CASE(7)
    MMK_X_CASE(8)
#undef MMK_X_CASE
    default: break;
  }
}

template <typename T, bool INV>
__global__ void __launch_bounds__(kXwThreads)
k_x_wp(const BatchDesc* __restrict__ descs, const WorkItem* __restrict__ items, int n_items) {
  persist_loop(n_items, [&](int v) {
    const WorkItem it = items[v];
    x_item<T, INV>(descs[it.sample], it.block);
  });
}

// ---------------------------------------------------------------------------
static int threads_for(long long values, int vpt) {
  long long t = (values + vpt - 1) / vpt;
  t = (t + 63) / 64 * 64;
  if (t < 64) t = 64;
  if (t > 512) t = 512;
  return (int)t;
}

template <typename K>
static void set_lds(K kernel, size_t bytes) {
  if (bytes > 48 * 1024)
    (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)bytes);
}

static bool wave_x(int M) { return M % 64 == 0 && M >= 64 && M <= 512; }

int rows_per_block(int M, int ny, bool single) {
  if (wave_x(M)) {
    // short rows: 4 per block (12 waves), fewer and larger blocks; the
    // longest (M >= 384): one row per block (3 waves), more blocks per CU
    if (M <= 256 && ny >= 4) return 4;
    if (M >= 384) return 1;
    return ny >= 2 ? 2 : 1;
  }
  // 3 R M complex values per block: at most 4096 (VPT 8, 512 threads) and
  // at most 48 KiB of LDS
  const int bytes = single ? 8 : 16;
  int R = 4096 / (3 * M);
  const int Rl = (48 * 1024) / (3 * M * bytes);
  if (Rl < R) R = Rl;
  if (R < 1) R = 1;
  if (R > ny) R = ny;
  return R;
}

template <typename T, int VL>
static void xf_wave(hipStream_t s, double* m, const T* g, T* sbuf, const MinState* st,
                    int nx, int ny, int nz, int R, void* out, const void* twx, const double* msub,
                    double* mcopy, const FinFuse& fz) {
  const size_t lds = (size_t)3 * R * wx_region<VL>() * sizeof(cx<T>);
  const int nb = nz * ((ny + R - 1) / R);
  auto k = fz.st != nullptr ? k_xf_w<T, VL, true> : k_xf_w<T, VL, false>;
  set_lds(k, lds);
  hipLaunchKernelGGL(k, dim3(nb), dim3(192 * R), lds, s, m, g, sbuf, st, nx, ny, nz, R,
                     (cx<T>*)out, (const cx<T>*)twx, msub, mcopy, fz);
}

template <typename T, int VL>
static void xil_wave(hipStream_t s, const void* in, const LocalArgs& a, int R, double* Hd_out,
                     double* partials, const void* twx) {
  const size_t lds = (size_t)3 * R * wx_region<VL>() * sizeof(cx<T>);
  const int nb = a.nz * ((a.ny + R - 1) / R);
  auto k = k_xil_w<T, VL>;
  set_lds(k, lds);
  hipLaunchKernelGGL(k, dim3(nb), dim3(192 * R), lds, s, (const cx<T>*)in, a, R, Hd_out, partials,
                     (const cx<T>*)twx);
}

// the wave-FFT forward pass (half lengths 64 VL, VL = 1..8) takes the finish over
bool xf_fuses_finish(int Px) {
  const int M = Px / 2;
  return Px % 2 == 0 && M % 64 == 0 && M >= 64 && M <= 512;
}

template <typename T>
void launch_xf(hipStream_t s, double* m, const T* g, T* sbuf, const MinState* st, int nx, int ny,
               int nz, int Px, int R, void* out, const void* twx, const double* msub,
               double* mcopy, const FinFuse* fzp) {
  const FinFuse fz = fzp != nullptr ? *fzp : FinFuse{nullptr, nullptr, 0.0, 0.0, 0, 0, 0};
  const int M = Px / 2;
  switch (M) {
    case 64: xf_wave<T, 1>(s, m, g, sbuf, st, nx, ny, nz, R, out, twx, msub, mcopy, fz); return;
    case 128: xf_wave<T, 2>(s, m, g, sbuf, st, nx, ny, nz, R, out, twx, msub, mcopy, fz); return;
    case 192: xf_wave<T, 3>(s, m, g, sbuf, st, nx, ny, nz, R, out, twx, msub, mcopy, fz); return;
    case 256: xf_wave<T, 4>(s, m, g, sbuf, st, nx, ny, nz, R, out, twx, msub, mcopy, fz); return;
    case 320: xf_wave<T, 5>(s, m, g, sbuf, st, nx, ny, nz, R, out, twx, msub, mcopy, fz); return;
    case 384: xf_wave<T, 6>(s, m, g, sbuf, st, nx, ny, nz, R, out, twx, msub, mcopy, fz); return;
    case 448: xf_wave<T, 7>(s, m, g, sbuf, st, nx, ny, nz, R, out, twx, msub, mcopy, fz); return;
    case 512: xf_wave<T, 8>(s, m, g, sbuf, st, nx, ny, nz, R, out, twx, msub, mcopy, fz); return;
    default: break;
  }
  const long long vals = 3LL * R * M;
  const size_t lds = (size_t)vals * sizeof(cx<T>);
  const int nb = nz * ((ny + R - 1) / R);
  if (vals <= 4096) {
    auto k = k_xf<T, 8>;
    set_lds(k, lds);
    hipLaunchKernelGGL(k, dim3(nb), dim3(threads_for(vals, 8)), lds, s, m, g, sbuf, st, nx, ny, nz,
                       Px, R, (cx<T>*)out, (const cx<T>*)twx, msub, mcopy);
  } else {
    auto k = k_xf<T, 16>;
    set_lds(k, lds);
    hipLaunchKernelGGL(k, dim3(nb), dim3(threads_for(vals, 16)), lds, s, m, g, sbuf, st, nx, ny,
                       nz, Px, R, (cx<T>*)out, (const cx<T>*)twx, msub, mcopy);
  }
}

template <typename T>
void launch_xil(hipStream_t s, const void* in, const LocalArgs& a, int Px, int R, double* Hd_out,
                double* partials, const void* twx) {
  const int M = Px / 2;
  switch (M) {
    case 64: xil_wave<T, 1>(s, in, a, R, Hd_out, partials, twx); return;
    case 128: xil_wave<T, 2>(s, in, a, R, Hd_out, partials, twx); return;
    case 192: xil_wave<T, 3>(s, in, a, R, Hd_out, partials, twx); return;
    case 256: xil_wave<T, 4>(s, in, a, R, Hd_out, partials, twx); return;
    case 320: xil_wave<T, 5>(s, in, a, R, Hd_out, partials, twx); return;
    case 384: xil_wave<T, 6>(s, in, a, R, Hd_out, partials, twx); return;
    case 448: xil_wave<T, 7>(s, in, a, R, Hd_out, partials, twx); return;
    case 512: xil_wave<T, 8>(s, in, a, R, Hd_out, partials, twx); return;
    default: break;
  }
  const long long vals = 3LL * R * M;
  const size_t lds = (size_t)vals * sizeof(cx<T>);
  const int nb = a.nz * ((a.ny + R - 1) / R);
  if (vals <= 4096) {
    auto k = k_xil<T, 8>;
    set_lds(k, lds);
    hipLaunchKernelGGL(k, dim3(nb), dim3(threads_for(vals, 8)), lds, s, (const cx<T>*)in, a, Px, R,
                       Hd_out, partials, (const cx<T>*)twx);
  } else {
    auto k = k_xil<T, 16>;
    set_lds(k, lds);
    hipLaunchKernelGGL(k, dim3(nb), dim3(threads_for(vals, 16)), lds, s, (const cx<T>*)in, a, Px,
                       R, Hd_out, partials, (const cx<T>*)twx);
  }
}

template <typename T, int VL>
static void xb_launch(hipStream_t s, bool inverse, const BatchDesc* descs, const WorkItem* items,
                      int n_items, int R) {
  const size_t lds = (size_t)3 * R * wx_region<VL>() * sizeof(cx<T>);
  if (inverse) {
    auto k = k_xil_wb<T, VL>;
    set_lds(k, lds);
    hipLaunchKernelGGL(k, dim3(n_items), dim3(192 * R), lds, s, descs, items);
  } else {
    auto k = k_xf_wb<T, VL>;
    set_lds(k, lds);
    hipLaunchKernelGGL(k, dim3(n_items), dim3(192 * R), lds, s, descs, items);
  }
}

// Blocks of a persistent x launch that stay resident together (a multiple
// of 8, at least 8).
int x_persistent_grid(bool single, bool inverse, int threads, size_t lds) {
  const void* k = single ? (inverse ? (const void*)k_x_wp<float, true> : (const void*)k_x_wp<float, false>)
                         : (inverse ? (const void*)k_x_wp<double, true> : (const void*)k_x_wp<double, false>);
  if (lds > 48 * 1024) (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, threads, lds) != hipSuccess ||
      hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    return 8;
  }
  const int g = per_cu * cus / 8 * 8;
  return g < 8 ? 8 : g;
}

template <typename T>
void launch_x_persistent(hipStream_t s, bool inverse, const BatchDesc* descs,
                         const WorkItem* items, int n_items, int threads, size_t lds, int grid) {
  const int g = n_items < grid ? n_items : grid;
  if (g <= 0) return;
  if (inverse) {
    auto k = k_x_wp<T, true>;
    set_lds(k, lds);
    hipLaunchKernelGGL(k, dim3(g), dim3(threads), lds, s, descs, items, n_items);
  } else {
    auto k = k_x_wp<T, false>;
    set_lds(k, lds);
    hipLaunchKernelGGL(k, dim3(g), dim3(threads), lds, s, descs, items, n_items);
  }
}

size_t x_block_lds(bool single, int M, int R) {
  return (size_t)3 * R * wx_region_of(M / 64) * (single ? 8 : 16);
}

template <typename T>
void launch_x_batched(hipStream_t s, bool inverse, const BatchDesc* descs, const WorkItem* items,
                      int n_items, int M, int R) {
  switch (M) {
    case 64: xb_launch<T, 1>(s, inverse, descs, items, n_items, R); break;
    case 128: xb_launch<T, 2>(s, inverse, descs, items, n_items, R); break;
    case 192: xb_launch<T, 3>(s, inverse, descs, items, n_items, R); break;
    case 256: xb_launch<T, 4>(s, inverse, descs, items, n_items, R); break;
    case 320: xb_launch<T, 5>(s, inverse, descs, items, n_items, R); break;
    case 384: xb_launch<T, 6>(s, inverse, descs, items, n_items, R); break;
    case 448: xb_launch<T, 7>(s, inverse, descs, items, n_items, R); break;
    default: xb_launch<T, 8>(s, inverse, descs, items, n_items, R); break;
  }
}

template void launch_x_batched<double>(hipStream_t, bool, const BatchDesc*, const WorkItem*, int,
                                       int, int);
template void launch_x_persistent<double>(hipStream_t, bool, const BatchDesc*, const WorkItem*, int,
                                          int, size_t, int);
template void launch_x_persistent<float>(hipStream_t, bool, const BatchDesc*, const WorkItem*, int,
                                         int, size_t, int);
template void launch_x_batched<float>(hipStream_t, bool, const BatchDesc*, const WorkItem*, int,
                                      int, int);
template void launch_xf<double>(hipStream_t, double*, const double*, double*, const MinState*, int,
                                int, int, int, int, void*, const void*, const double*, double*,
                                const FinFuse*);
template void launch_xf<float>(hipStream_t, double*, const float*, float*, const MinState*, int,
                               int, int, int, int, void*, const void*, const double*, double*,
                               const FinFuse*);
template void launch_xil<double>(hipStream_t, const void*, const LocalArgs&, int, int, double*,
                                 double*, const void*);
template void launch_xil<float>(hipStream_t, const void*, const LocalArgs&, int, int, double*,
                                double*, const void*);

}  // namespace mmk
