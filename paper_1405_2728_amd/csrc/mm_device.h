// Device-side building blocks shared by the HIP kernels of the minimiser:
// complex arithmetic, radix-2/4/8 butterflies, an in-place LDS Stockham FFT
// stage, and deterministic block reductions.  gfx950 only (wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mmk {

constexpr double kMu0 = 4.0e-7 * 3.14159265358979323846;

// Work loop of a persistent kernel over the items 0 .. n-1 of an XCD-ordered
// table: block b runs the items b, b + G, b + 2G, ... (G = gridDim.x, a
// multiple of 8 when below n, so that every item runs on the XCD its table
// position gives it).  A static share: a shared work counter costs each item
// an atomic round trip on its critical path.
template <typename F>
__device__ __forceinline__ void persist_loop(int n, F&& item) {
  for (int v = (int)blockIdx.x; v < n; v += (int)gridDim.x) {
    item(v);
    __syncthreads();   // the next item may reuse the LDS
  }
}

// threadIdx.x through an empty asm statement that the compiler must assume
// changes it: the persistent batched kernels run a pass body once per work
// item in a loop, and without this the compiler hoists every body's
// thread-index arithmetic (for all transform lengths at once) out of the
// loop and runs out of registers.
__device__ __forceinline__ int thread_index() {
  int t = (int)threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T a, T b) { cx<T> r; r.x = a; r.y = b; return r; }
template <typename T>
__device__ __forceinline__ cx<T> add(cx<T> a, cx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cx<T> sub(cx<T> a, cx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cx<T> mul(cx<T> a, cx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ cx<T> scl(cx<T> a, T s) { return mk(a.x * s, a.y * s); }
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return mk(a.x, -a.y); }
// multiply by -i (DIR = -1) or +i (DIR = +1)
template <int DIR, typename T>
__device__ __forceinline__ cx<T> rot90(cx<T> a) {
  return DIR < 0 ? mk(a.y, -a.x) : mk(-a.y, a.x);
}

// ---------------------------------------------------------------------------
// DFT of length R on registers, X[k] = sum_n v[n] exp(DIR 2 pi i n k / R).
// ---------------------------------------------------------------------------
template <int DIR, typename T>
__device__ __forceinline__ void dft2(cx<T>* v) {
  cx<T> a = v[0], b = v[1];
  v[0] = add(a, b);
  v[1] = sub(a, b);
}

template <int DIR, typename T>
__device__ __forceinline__ void dft4(cx<T>* v) {
  cx<T> a0 = add(v[0], v[2]), a1 = sub(v[0], v[2]);
  cx<T> a2 = add(v[1], v[3]), a3 = rot90<DIR>(sub(v[1], v[3]));
  v[0] = add(a0, a2);
  v[2] = sub(a0, a2);
  v[1] = add(a1, a3);
  v[3] = sub(a1, a3);
}

template <int DIR, typename T>
__device__ __forceinline__ void dft8(cx<T>* v) {
  cx<T> e[4] = {v[0], v[2], v[4], v[6]};
  cx<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4<DIR>(e);
  dft4<DIR>(o);
  const T h = T(0.70710678118654752440084436210485);
  // o[k] *= exp(DIR i pi k / 4)
  o[1] = mk(h * (o[1].x - DIR * o[1].y), h * (o[1].y + DIR * o[1].x));
  o[2] = rot90<DIR>(o[2]);
  o[3] = mk(h * (-o[3].x - DIR * o[3].y), h * (-o[3].y + DIR * o[3].x));
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = add(e[k], o[k]);
    v[k + 4] = sub(e[k], o[k]);
  }
}

// cos and sin of 2 pi m / P for the odd radices P = 3, 5, 7 (m = 0..P-1)
__host__ __device__ constexpr double odd_cos(int P, int m) {
  const double c3[3] = {1.0, -0.5, -0.5};
  const double c5[5] = {1.0, 0.30901699437494745, -0.8090169943749475, -0.8090169943749475,
                        0.30901699437494745};
  const double c7[7] = {1.0, 0.6234898018587336, -0.22252093395631434, -0.900968867902419,
                        -0.900968867902419, -0.22252093395631434, 0.6234898018587336};
  return P == 3 ? c3[m] : P == 5 ? c5[m] : c7[m];
}
__host__ __device__ constexpr double odd_sin(int P, int m) {
  const double s3[3] = {0.0, 0.8660254037844386, -0.8660254037844386};
  const double s5[5] = {0.0, 0.9510565162951535, 0.5877852522924731, -0.5877852522924731,
                        -0.9510565162951535};
  const double s7[7] = {0.0, 0.7818314824680298, 0.9749279121818236, 0.43388373911755823,
                        -0.43388373911755823, -0.9749279121818236, -0.7818314824680298};
  return P == 3 ? s3[m] : P == 5 ? s5[m] : s7[m];
}

// Odd prime length P: with a_j = v_j + v_{P-j}, b_j = v_j - v_{P-j}
// (j = 1..P/2), X[k] = v_0 + sum_j a_j cos(2 pi jk/P) + DIR i sum_j b_j
// sin(2 pi jk/P) and X[P-k] the same with the sine sum negated.
template <int P, int DIR, typename T>
__device__ __forceinline__ void dft_odd(cx<T>* v) {
  constexpr int H = P / 2;
  cx<T> a[H + 1], b[H + 1];
#pragma unroll
  for (int j = 1; j <= H; ++j) {
    a[j] = add(v[j], v[P - j]);
    b[j] = sub(v[j], v[P - j]);
  }
  const cx<T> x0 = v[0];
  cx<T> sum = x0;
#pragma unroll
  for (int j = 1; j <= H; ++j) sum = add(sum, a[j]);
  v[0] = sum;
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    cx<T> t = x0, u = mk(T(0), T(0));
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      const int m = (j * k) % P;
      t = add(t, scl(a[j], T(odd_cos(P, m))));
      u = add(u, scl(b[j], T(odd_sin(P, m))));
    }
    const cx<T> ru = rot90<DIR>(u);
    v[k] = add(t, ru);
    v[P - k] = sub(t, ru);
  }
}

// Length 6 = 2 x 3: the 3-point transforms of the even and odd samples,
// combined with the twiddles exp(DIR 2 pi i k / 6).
template <int DIR, typename T>
__device__ __forceinline__ void dft6(cx<T>* v) {
  cx<T> e[3] = {v[0], v[2], v[4]};
  cx<T> o[3] = {v[1], v[3], v[5]};
  dft_odd<3, DIR>(e);
  dft_odd<3, DIR>(o);
  const T h = T(0.8660254037844386);   // sin(pi / 3)
  const cx<T> o1 = mul(o[1], mk(T(0.5), T(DIR) * h));
  const cx<T> o2 = mul(o[2], mk(T(-0.5), T(DIR) * h));
  v[0] = add(e[0], o[0]);
  v[3] = sub(e[0], o[0]);
  v[1] = add(e[1], o1);
  v[4] = sub(e[1], o1);
  v[2] = add(e[2], o2);
  v[5] = sub(e[2], o2);
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dftR(cx<T>* v) {
  if constexpr (R == 2) dft2<DIR>(v);
  else if constexpr (R == 4) dft4<DIR>(v);
  else if constexpr (R == 3 || R == 5 || R == 7) dft_odd<R, DIR>(v);
  else dft8<DIR>(v);
}

// Twiddle exp(DIR 2 pi i m / twn) from a table tw[m] = exp(-2 pi i m / twn).
template <int DIR, typename T>
__device__ __forceinline__ cx<T> twiddle(const cx<T>* __restrict__ tw, int m) {
  cx<T> w = tw[m];
  return DIR < 0 ? w : conj(w);
}

// Odd factor of a length n = r * 2^p (r = 1, 3, 5 or 7).
__host__ __device__ inline int fft_odd_factor(int n) {
  return n % 7 == 0 ? 7 : n % 5 == 0 ? 5 : n % 3 == 0 ? 3 : 1;
}

// Radix plan of a length n = r * 2^p: a leading radix-r stage (r = 3, 5, 7),
// then for the power of two 8s, with one 4 (p % 3 == 2) or two 4s
// (p % 3 == 1); 2 uses a single radix-2 stage.  Encoded as the odd radix
// (1: none) and the numbers of radix-2, radix-4 and radix-8 stages.
struct FftPlan {
  int n, n4, n8, n2, r;
};

__host__ __device__ inline FftPlan make_plan(int n) {
  FftPlan p{n, 0, 0, 0, fft_odd_factor(n)};
  n /= p.r;
  int lg = 0;
  while ((1 << lg) < n) ++lg;
  if (lg == 0) return p;
  if (lg == 1) { p.n2 = 1; return p; }
  if (lg == 2) { p.n4 = 1; return p; }
  int a = lg / 3, b = lg % 3;
  if (b == 0) { p.n8 = a; }
  else if (b == 1) { p.n4 = 2; p.n8 = a - 1; }
  else { p.n4 = 1; p.n8 = a; }
  return p;
}

// Values per thread that the stages of a length-n plan hold at VPT: a
// radix-r stage (r odd) keeps r (VPT/r) values per thread.  Launchers size
// their blocks with it.
__host__ __device__ inline int fft_vpt_cap(int n, int vpt) {
  const int r = fft_odd_factor(n);
  return r > 1 ? r * (vpt / r) : vpt;
}

// One in-place Stockham stage of radix R over nseq sequences of length n
// stored at buf + s*stride.  Every thread first loads, twiddles and
// transforms up to VPT/R butterflies into registers, then (after a barrier)
// stores them: the in-place form needs all loads of a stage to precede its
// stores, so the caller guarantees nseq*n <= fft_vpt_cap(n, VPT)*nthr.
//   butterfly j of a sequence (0 <= j < n/R), k = j mod Ns:
//     v[r] = x[j + r n/R] * w^(r k),  w = exp(DIR 2 pi i / (Ns R))
//     v    = DFT_R(v)
//     y[(j div Ns) Ns R + k + r Ns] = v[r]
template <int R, int DIR, int VPT, typename T>
__device__ __forceinline__ void stockham_stage(cx<T>* buf, int n, int Ns, int nseq, int stride,
                                               const cx<T>* __restrict__ tw, int twn, int tid,
                                               int nthr) {
  constexpr int BPT = VPT / R;
  const int nbs = n / R;
  const int nb = nbs * nseq;
  const int twstep = twn / (Ns * R);
  cx<T> v[BPT][R];
  int dst[BPT];
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int t = tid + q * nthr;
    dst[q] = -1;
    if (t < nb) {
      const int s = t / nbs;
      const int j = t - s * nbs;
      const int k = (Ns & (Ns - 1)) == 0 ? j & (Ns - 1) : j % Ns;
      cx<T>* p = buf + s * stride;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = p[j + r * nbs];
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[q][r] = mul(v[q][r], twiddle<DIR>(tw, r * k * twstep));
      }
      dftR<R, DIR>(v[q]);
      dst[q] = s * stride + (j - k) * R + k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    if (dst[q] >= 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) buf[dst[q] + r * Ns] = v[q][r];
    }
  }
  __syncthreads();
}

// Full in-place FFT of nseq sequences of length n = r * 2^p in LDS; r = 3,
// 5 or 7 needs ODD (only the set-up transforms see such lengths; without
// ODD n must be a power of two and no odd-radix stage is compiled in).
// tw: table of exp(-2 pi i m / twn) with twn a multiple of n.
template <int DIR, int VPT, bool ODD = false, typename T>
__device__ void fft_lds(cx<T>* buf, int n, int nseq, int stride, const cx<T>* __restrict__ tw,
                        int twn, int tid, int nthr) {
  const FftPlan p = make_plan(n);
  int Ns = 1;
  if constexpr (ODD) {
    if (p.r == 3) stockham_stage<3, DIR, VPT>(buf, n, Ns, nseq, stride, tw, twn, tid, nthr);
    if (p.r == 5) stockham_stage<5, DIR, VPT>(buf, n, Ns, nseq, stride, tw, twn, tid, nthr);
    if (p.r == 7) stockham_stage<7, DIR, VPT>(buf, n, Ns, nseq, stride, tw, twn, tid, nthr);
    Ns *= p.r;
  }
  if (p.n2) {
    stockham_stage<2, DIR, VPT>(buf, n, Ns, nseq, stride, tw, twn, tid, nthr);
    Ns *= 2;
  }
  for (int i = 0; i < p.n4; ++i) {
    stockham_stage<4, DIR, VPT>(buf, n, Ns, nseq, stride, tw, twn, tid, nthr);
    Ns *= 4;
  }
  for (int i = 0; i < p.n8; ++i) {
    stockham_stage<8, DIR, VPT>(buf, n, Ns, nseq, stride, tw, twn, tid, nthr);
    Ns *= 8;
  }
}

// ---------------------------------------------------------------------------
// Deterministic block reductions (fixed order: a fixed cross-lane pattern
// within each wave, then the waves' partials in index order).
// ---------------------------------------------------------------------------
// The other lane's value of v through a DPP move (both 32-bit halves); lanes
// whose source is outside their row, or rows outside ROWS, get `old`.
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ double dpp_f64(double old, double v) {
  const long long o = __double_as_longlong(old), x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp((int)o, (int)x, CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(x >> 32), CTRL, ROWS, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Wave total in lane 63: an inclusive scan within each row of 16 lanes
// (row_shr 1, 2, 4, 8: lane 15 of a row holds the row's total), then row 0's
// total into row 1 and row 2's into row 3 (row_bcast 15), then lane 31's
// into rows 2 and 3 (row_bcast 31).  No LDS traffic.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0x111>(0.0, v);
  v += dpp_f64<0x112>(0.0, v);
  v += dpp_f64<0x114>(0.0, v);
  v += dpp_f64<0x118>(0.0, v);
  v += dpp_f64<0x142, 0xa>(0.0, v);
  v += dpp_f64<0x143, 0xc>(0.0, v);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_f64<0x111>(v, v));
  v = fmax(v, dpp_f64<0x112>(v, v));
  v = fmax(v, dpp_f64<0x114>(v, v));
  v = fmax(v, dpp_f64<0x118>(v, v));
  v = fmax(v, dpp_f64<0x142, 0xa>(v, v));
  v = fmax(v, dpp_f64<0x143, 0xc>(v, v));
  return v;
}

// Reduce NV values per thread across the block.  MAXT is the kernel's
// launch bound (blockDim.x <= MAXT, whole waves); scratch holds
// NV * MAXT / 64 doubles of LDS.  is_max[i] selects max vs sum.  Each wave
// reduces in registers (total in lane 63); then lane i of the first wave
// combines value i over the waves (in wave order, so the result does not
// depend on timing) and returns it (threads i < NV; others return 0).
template <int MAXT, int NV, int NS>
__device__ __forceinline__ double block_combine(double (&v)[NV], const bool (&is_max)[NV],
                                                double (&scratch)[NS]) {
  static_assert(NS >= NV * (MAXT / 64), "reduction scratch smaller than one slot per wave");
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = is_max[i] ? wave_max(v[i]) : wave_sum(v[i]);
  if (lane == 63) {
#pragma unroll
    for (int i = 0; i < NV; ++i) scratch[i * nw + wid] = v[i];
  }
  __syncthreads();
  double a = 0.0;
  if (threadIdx.x < NV) {
    const int i = threadIdx.x;
    bool mx = false;
#pragma unroll
    for (int q = 0; q < NV; ++q) mx = q == i ? is_max[q] : mx;
    a = scratch[i * nw];
    for (int w = 1; w < nw; ++w) a = mx ? fmax(a, scratch[i * nw + w]) : a + scratch[i * nw + w];
  }
  return a;
}

// The block's results in v[] of thread 0.
template <int MAXT, int NV, int NS>
__device__ __forceinline__ void block_reduce(double (&v)[NV], const bool (&is_max)[NV],
                                             double (&scratch)[NS]) {
  const double a = block_combine<MAXT>(v, is_max, scratch);
  const int nw = (blockDim.x + 63) >> 6;
  if (threadIdx.x < NV) scratch[threadIdx.x * nw] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = scratch[i * nw];
  }
}

// The block's results stored to out[0 .. NV) by threads 0 .. NV-1 (one
// barrier fewer than block_reduce; scratch is reused only after another).
template <int MAXT, int NV, int NS>
__device__ __forceinline__ void block_reduce_store(double (&v)[NV], const bool (&is_max)[NV],
                                                   double (&scratch)[NS], double* out) {
  const double a = block_combine<MAXT>(v, is_max, scratch);
  if (threadIdx.x < NV) out[threadIdx.x] = a;
}

}  // namespace mmk
