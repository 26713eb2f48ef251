// Register-resident FFT of one sequence per wavefront (64 lanes), length
// n = 64 VL with VL in 1..8.
//
// Forward, natural input: lane l holds x[l + 64 r] in v[r] (r < VL).
//   S1  DFT_VL over r, twiddle by W_n^(l k1)            (k1 < VL)
//   T1  LDS transpose: lane g = 8 k1 + a gathers the 8 values l = a + 8 b
//   S2  DFT_8 over b, twiddle by W_64^(a c)
//   T2  LDS transpose: lane g = 8 k1 + c gathers the 8 values over a
//   S3  DFT_8 over a
// Output, permuted: lane g = 8 k1 + c (g < 8 VL) holds X[k1 + VL (c + 8 d)]
// in u[d] (d < 8); lanes g >= 8 VL hold nothing.
// The inverse is the exact adjoint (stages reversed, conjugate twiddles):
// permuted input as above, natural output l + 64 r, unnormalised.
//
// Transposes use a wave-private LDS buffer of wfft_buf<VL, HALF>()
// elements; the index maps are padded (one slot per 8) so that lanes 8
// apart fall on different banks.  With HALF the buffer holds the groups
// k1 < VL/2 and k1 >= VL/2 in turn (half the LDS, twice the exchanges; even
// VL only, odd VL always uses the whole buffer).
// LDS instructions of one wavefront execute in order, so the exchange within
// a wave needs no block barrier.
#pragma once

#include "mm_device.h"

namespace mmk {

__device__ __forceinline__ int wf_f1(int k1, int q) { return k1 * 72 + q + (q >> 3); }
__device__ __forceinline__ int wf_f2(int k1, int c, int a) { return k1 * 72 + c * 9 + a; }

// passes over the k1 groups of a transpose
template <int VL, bool HALF>
__host__ __device__ constexpr int wfft_passes() {
  return (HALF && VL >= 2 && VL % 2 == 0) ? 2 : 1;
}

template <int VL, bool HALF>
__host__ __device__ constexpr int wfft_buf() {
  return VL / wfft_passes<VL, HALF>() * 72;
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dft_small(cx<T>* v) {
  if constexpr (R == 2) dft2<DIR>(v);
  else if constexpr (R == 4) dft4<DIR>(v);
  else if constexpr (R == 3 || R == 5 || R == 7) dft_odd<R, DIR>(v);
  else if constexpr (R == 6) dft6<DIR>(v);
  else if constexpr (R == 8) dft8<DIR>(v);
}

// tw: table exp(-2 pi i m / (n TS)), read with stride TS (a table of a
// multiple of the length serves as well).
template <typename T, int VL, bool HALF, int TS = 1>
__device__ __forceinline__ void wfft_forward(cx<T> (&v)[VL], cx<T> (&u)[8], cx<T>* lds,
                                             const cx<T>* __restrict__ tw, int lane) {
  constexpr int NG = 8 * VL;
  constexpr int NP = wfft_passes<VL, HALF>();       // passes over the k1 groups
  constexpr int KP = VL / NP;                       // k1 groups per pass
  dft_small<VL, -1>(v);
#pragma unroll
  for (int k1 = 1; k1 < VL; ++k1) v[k1] = mul(v[k1], tw[TS * lane * k1]);
  const int k1 = lane >> 3, a = lane & 7;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
#pragma unroll
    for (int kk = 0; kk < KP; ++kk) lds[wf_f1(kk, lane)] = v[p * KP + kk];
    __builtin_amdgcn_wave_barrier();
    if (lane < NG && k1 / KP == p) {
#pragma unroll
      for (int b = 0; b < 8; ++b) u[b] = lds[wf_f1(k1 - p * KP, a + 8 * b)];
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (lane < NG) {
    dft8<-1>(u);
#pragma unroll
    for (int c = 1; c < 8; ++c) u[c] = mul(u[c], tw[TS * a * c * VL]);
  }
  const int c = lane & 7;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const bool mine = lane < NG && k1 / KP == p;
    if (mine) {
#pragma unroll
      for (int cc = 0; cc < 8; ++cc) lds[wf_f2(k1 - p * KP, cc, a)] = u[cc];
    }
    __builtin_amdgcn_wave_barrier();
    if (mine) {
#pragma unroll
      for (int aa = 0; aa < 8; ++aa) u[aa] = lds[wf_f2(k1 - p * KP, c, aa)];
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (lane < NG) dft8<-1>(u);
}

template <typename T, int VL, bool HALF, int TS = 1>
__device__ __forceinline__ void wfft_inverse(cx<T> (&u)[8], cx<T> (&v)[VL], cx<T>* lds,
                                             const cx<T>* __restrict__ tw, int lane) {
  constexpr int NG = 8 * VL;
  constexpr int NP = wfft_passes<VL, HALF>();
  constexpr int KP = VL / NP;
  const int k1 = lane >> 3, a = lane & 7, c = lane & 7;
  if (lane < NG) dft8<1>(u);
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const bool mine = lane < NG && k1 / KP == p;
    if (mine) {
#pragma unroll
      for (int aa = 0; aa < 8; ++aa) lds[wf_f2(k1 - p * KP, c, aa)] = u[aa];
    }
    __builtin_amdgcn_wave_barrier();
    if (mine) {
#pragma unroll
      for (int cc = 0; cc < 8; ++cc) u[cc] = lds[wf_f2(k1 - p * KP, cc, a)];
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (lane < NG) {
#pragma unroll
    for (int cc = 1; cc < 8; ++cc) u[cc] = mul(u[cc], conj(tw[TS * a * cc * VL]));
    dft8<1>(u);
  }
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    if (lane < NG && k1 / KP == p) {
#pragma unroll
      for (int b = 0; b < 8; ++b) lds[wf_f1(k1 - p * KP, a + 8 * b)] = u[b];
    }
    __builtin_amdgcn_wave_barrier();
    // element by element: as one aggregate copy the single element of the
    // 64-point transform stayed in scratch memory across the barrier
#pragma unroll
    for (int kk = 0; kk < KP; ++kk) {
      const cx<T>& e = lds[wf_f1(kk, lane)];
      v[p * KP + kk] = mk(e.x, e.y);
    }
    __builtin_amdgcn_wave_barrier();
  }
#pragma unroll
  for (int kk = 1; kk < VL; ++kk) v[kk] = mul(v[kk], conj(tw[TS * lane * kk]));
  dft_small<VL, 1>(v);
}

// Frequency index held in slot d by lane g of the permuted distribution.
template <int VL>
__device__ __forceinline__ int wfft_freq(int lane, int d) {
  return (lane >> 3) + VL * ((lane & 7) + 8 * d);
}

}  // namespace mmk
