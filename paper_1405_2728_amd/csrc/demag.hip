// Demagnetisation field as a zero-padded FFT convolution on the regular
// cuboid grid (Sec. 3 of the paper), thin-film path.
//
// Padded sizes: Px = max(2, 2^ceil(log2(2nx-1))), Py = 2^ceil(log2(2ny-1)).
// The z direction (nz <= 4 here) is not transformed: the tensor product is a
// direct convolution over the nz layers in the mixed (kx, ky, z) domain.
//
// Passes per evaluation:
//   fwd_x   rows of m (real, nx values, zero padded to Px) -> half-length
//           complex FFT (M = Px/2 points, even/odd samples packed as re/im)
//           -> spectrum X[0..M] written as A[kx][z][y][c]
//   yz_thin one block per kx: y-FFT of the 3*nz columns (zero padded to Py),
//           symmetric 3x3 tensor times vector with the z convolution,
//           inverse y-FFT, keep ny rows.  The block of kx = 0 also carries
//           kx = M: both columns are spectra of real data, packed as
//           re + i*im and separated by Hermitian symmetry in ky.
//   inv_x   A[kx][z][y][c] -> half-length inverse -> H_d rows (double)
//   yz_wave as yz_thin, with register wave FFTs (one wave per layer and
//           component, Py = 64..512) and one block per column kx = 0..M
// The factor -Ms/(M Py) of the inverse transforms is applied in yz_thin.
#include <algorithm>

#include "mm_device.h"
#include "mm_kernels.h"
#include "mm_wfft.h"

namespace mmk {

// ---------------------------------------------------------------------------
// x-forward: real rows -> X[0..M] (DC and Nyquist real).
// ---------------------------------------------------------------------------
template <typename T, int VPT>
__global__ void __launch_bounds__(512)
k_fwd_x(const double* __restrict__ in, int in_row_stride, int nx_in, int rows, int ncomp, int Px,
        int R, cx<T>* __restrict__ out, const cx<T>* __restrict__ twx, const int* __restrict__ done) {
  if (done != nullptr && *done != 0) return;
  extern __shared__ __align__(16) unsigned char smem[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
  const int M = Px >> 1;
  const int nrb = (rows + R - 1) / R;
  const int c = blockIdx.x / nrb;
  const int r0 = (blockIdx.x - c * nrb) * R;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const double* src = in + (size_t)c * rows * in_row_stride;
  for (int idx = tid; idx < R * M; idx += nthr) {
    const int r = idx / M, j = idx - r * M;
    const int row = r0 + r;
    T a = T(0), b = T(0);
    if (row < rows) {
      const double* p = src + (size_t)row * in_row_stride;
      const int x0 = 2 * j;
      if (x0 < nx_in) a = (T)p[x0];
      if (x0 + 1 < nx_in) b = (T)p[x0 + 1];
    }
    buf[r * M + j] = mk(a, b);
  }
  __syncthreads();
  fft_lds<-1, VPT, true>(buf, M, R, M, twx, Px, tid, nthr);
  const size_t slab = (size_t)ncomp * rows;
  for (int idx = tid; idx < (M + 1) * R; idx += nthr) {
    const int k = idx / R, r = idx - k * R;
    const int row = r0 + r;
    if (row >= rows) continue;
    const cx<T> zk = buf[r * M + (k == M ? 0 : k)];
    const cx<T> zc = conj(buf[r * M + (k == 0 ? 0 : M - k)]);
    const cx<T> w = twx[k];
    const cx<T> X = scl(add(add(zk, zc), rot90<-1>(mul(w, sub(zk, zc)))), T(0.5));
    out[(size_t)k * slab + (size_t)c * rows + row] = X;
  }
}

// ---------------------------------------------------------------------------
// x-inverse: X[0..M] -> real rows (first nx_out values), unnormalised:
// the result is M times the normalised inverse of the length-Px spectrum.
// ---------------------------------------------------------------------------
template <typename T, int VPT>
__global__ void __launch_bounds__(512)
k_inv_x(const cx<T>* __restrict__ in, int rows, int ncomp, int nx_out, int Px, int R,
        double* __restrict__ out, const cx<T>* __restrict__ twx, const int* __restrict__ done) {
  if (done != nullptr && *done != 0) return;
  extern __shared__ __align__(16) unsigned char smem[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
  const int M = Px >> 1;
  const int nrb = (rows + R - 1) / R;
  const int c = blockIdx.x / nrb;
  const int r0 = (blockIdx.x - c * nrb) * R;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const size_t slab = (size_t)ncomp * rows;
  const cx<T>* src = in + (size_t)c * rows;
  for (int idx = tid; idx < M * R; idx += nthr) {
    const int k = idx / R, r = idx - k * R;
    const int row = r0 + r;
    cx<T> Z = mk(T(0), T(0));
    if (row < rows) {
      const cx<T> Xk = src[(size_t)k * slab + row];
      const cx<T> Xc = conj(src[(size_t)(M - k) * slab + row]);
      const cx<T> wi = conj(twx[k]);
      Z = scl(add(add(Xk, Xc), rot90<1>(mul(wi, sub(Xk, Xc)))), T(0.5));
    }
    buf[r * M + k] = Z;
  }
  __syncthreads();
  fft_lds<1, VPT, true>(buf, M, R, M, twx, Px, tid, nthr);
  for (int idx = tid; idx < R * M; idx += nthr) {
    const int r = idx / M, j = idx - r * M;
    const int row = r0 + r;
    if (row >= rows) continue;
    const cx<T> z = buf[r * M + j];
    double* p = out + ((size_t)c * rows + row) * nx_out;
    const int x0 = 2 * j;
    if (x0 < nx_out) p[x0] = (double)z.x;
    if (x0 + 1 < nx_out) p[x0 + 1] = (double)z.y;
  }
}

// ---------------------------------------------------------------------------
// Batched forward FFT of contiguous sequences (tensor set-up only).
// ---------------------------------------------------------------------------
template <typename T, int VPT>
__global__ void __launch_bounds__(512)
k_fft_cols(cx<T>* __restrict__ data, int n, int nseq, int per_block, const cx<T>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
  const int s0 = blockIdx.x * per_block;
  const int ns = min(per_block, nseq - s0);
  const int tid = threadIdx.x, nthr = blockDim.x;
  cx<T>* base = data + (size_t)s0 * n;
  for (int idx = tid; idx < ns * n; idx += nthr) buf[idx] = base[idx];
  __syncthreads();
  fft_lds<-1, VPT, true>(buf, n, ns, n, tw, n, tid, nthr);
  for (int idx = tid; idx < ns * n; idx += nthr) base[idx] = buf[idx];
}

// ---------------------------------------------------------------------------
// Symmetric 3x3 tensor times vector with the z convolution, at one (kx, ky)
// and one target layer z:  H(z) = sum_z' T(kx, ky, z - z') F(z').
// Tensor slab layout [dz][ky'][6] with ky' = min(ky, Py - ky); components
// (xx, yy, zz, xy, xz, yz); xz and yz hold the coefficient of i.  Parities:
// xy odd in ky; xz odd in dz; yz odd in ky and dz.
// ---------------------------------------------------------------------------
template <typename T, int NZ>
__device__ __forceinline__ void tensor_apply_z(const T* __restrict__ Tk, int nk, int Py, int ky,
                                               const cx<T> (&F)[3][NZ], int z, cx<T> (&H)[3]) {
  const bool neg_y = ky > (Py >> 1);
  const int kyp = neg_y ? Py - ky : ky;
  const T sy = neg_y ? T(-1) : T(1);
  H[0] = mk(T(0), T(0));
  H[1] = mk(T(0), T(0));
  H[2] = mk(T(0), T(0));
#pragma unroll
  for (int zp = 0; zp < NZ; ++zp) {
    const int dz = z - zp;
    const int dzp = dz < 0 ? -dz : dz;
    const T sz = dz < 0 ? T(-1) : T(1);
    const T* t = Tk + ((size_t)dzp * nk + kyp) * 6;
    const T xx = t[0], yy = t[1], zz = t[2];
    const T xy = t[3] * sy, xz = t[4] * sz, yz = t[5] * sy * sz;
    const cx<T> fx = F[0][zp], fy = F[1][zp], fz = F[2][zp];
    const cx<T> ifx = rot90<1>(fx), ify = rot90<1>(fy), ifz = rot90<1>(fz);
    H[0] = add(H[0], add(add(scl(fx, xx), scl(fy, xy)), scl(ifz, xz)));
    H[1] = add(H[1], add(add(scl(fx, xy), scl(fy, yy)), scl(ifz, yz)));
    H[2] = add(H[2], add(add(scl(ifx, xz), scl(ify, yz)), scl(fz, zz)));
  }
}

template <typename T, int VPT, int NZ>
__global__ void __launch_bounds__(512)
k_yz_thin(cx<T>* __restrict__ A, int ny, int Py, int M, const T* __restrict__ Tt, int tstride,
          T scale, const cx<T>* __restrict__ twy, const int* __restrict__ done) {
  if (done != nullptr && *done != 0) return;
  extern __shared__ __align__(16) unsigned char smem[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
  constexpr int nseq = 3 * NZ;
  const int S = Py;
  const int kx = blockIdx.x;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const size_t slab = (size_t)nseq * ny;
  for (int idx = tid; idx < nseq * Py; idx += nthr) {
    const int col = idx / Py, y = idx - col * Py;
    cx<T> v = mk(T(0), T(0));
    if (y < ny) {
      const size_t e = ((size_t)(col % NZ) * ny + y) * 3 + col / NZ;   // [z][y][c]
      if (kx == 0) v = mk(A[e].x, A[(size_t)M * slab + e].x);
      else v = A[(size_t)kx * slab + e];
    }
    buf[col * S + y] = v;
  }
  __syncthreads();
  fft_lds<-1, VPT>(buf, Py, nseq, S, twy, Py, tid, nthr);
  const int nk = (Py >> 1) + 1;
  const size_t tslab = (size_t)tstride;
  if (kx != 0) {
    const T* Tk = Tt + (size_t)kx * tslab;
    for (int ky = tid; ky < Py; ky += nthr) {
      cx<T> F[3][NZ];
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int z = 0; z < NZ; ++z) F[c][z] = buf[(c * NZ + z) * S + ky];
#pragma unroll
      for (int z = 0; z < NZ; ++z) {
        cx<T> H[3];
        tensor_apply_z<T, NZ>(Tk, nk, Py, ky, F, z, H);
#pragma unroll
        for (int c = 0; c < 3; ++c) buf[(c * NZ + z) * S + ky] = scl(H[c], scale);
      }
    }
  } else {
    // Column 0 carries Z = F0 + i Fn, F0 / Fn the spectra of the real kx = 0
    // and kx = M planes (Hermitian in ky).  With P = (Z(ky) + conj Z(-ky))/2
    // = F0(ky) and Q = (Z(ky) - conj Z(-ky))/2 = i Fn(ky):
    //   H(ky)  = T0 P + TM Q,   H(-ky) = conj(T0 P - TM Q)
    // because T0, TM are Hermitian in ky as well.
    const T* T0 = Tt;
    const T* Tn = Tt + (size_t)M * tslab;
    for (int ky = tid; ky < nk; ky += nthr) {
      const int km = (Py - ky) & (Py - 1);
      cx<T> P[3][NZ], Q[3][NZ];
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int z = 0; z < NZ; ++z) {
          const cx<T> fa = buf[(c * NZ + z) * S + ky];
          const cx<T> fb = conj(buf[(c * NZ + z) * S + km]);
          P[c][z] = scl(add(fa, fb), T(0.5));
          Q[c][z] = scl(sub(fa, fb), T(0.5));
        }
#pragma unroll
      for (int z = 0; z < NZ; ++z) {
        cx<T> H0[3], H1[3];
        tensor_apply_z<T, NZ>(T0, nk, Py, ky, P, z, H0);
        tensor_apply_z<T, NZ>(Tn, nk, Py, ky, Q, z, H1);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          buf[(c * NZ + z) * S + ky] = scl(add(H0[c], H1[c]), scale);
          if (km != ky) buf[(c * NZ + z) * S + km] = scl(conj(sub(H0[c], H1[c])), scale);
        }
      }
    }
  }
  __syncthreads();
  fft_lds<1, VPT>(buf, Py, nseq, S, twy, Py, tid, nthr);
  for (int idx = tid; idx < nseq * ny; idx += nthr) {
    const int col = idx / ny, y = idx - col * ny;
    const cx<T> v = buf[col * S + y];
    const size_t e = ((size_t)(col % NZ) * ny + y) * 3 + col / NZ;
    if (kx == 0) {
      A[e] = mk(v.x, T(0));
      A[(size_t)M * slab + e] = mk(v.y, T(0));
    } else {
      A[(size_t)kx * slab + e] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// y-FFT, tensor product with the z convolution, inverse y-FFT; wave FFT
// version.  One block per column kx = 0..M; 3 NZ wavefronts, wave w = 3 z + c
// transforms component c of layer z (64 VL points, zero padded beyond ny)
// with the register wave FFT, using its own LDS slice for the transposes and
// then to hold its 8 output slots (slot d of lane g: frequency
// wfft_freq(g, d)).  After a barrier the product runs per position: wave d
// (d < 8) takes slot d of every lane, reads the 3 NZ spectra of that
// position, forms every output layer and component (symmetric 3x3 tensor,
// direct convolution over the layers) and writes them back in place; after a
// second barrier each wave transforms its slice back and stores the ny kept
// rows.  The tensor slab of the column is copied to LDS by direct
// global-to-LDS loads while the forward transforms run.  Columns 0 and M are
// spectra of real rows: their results are real (the imaginary part, rounding
// only, is dropped).
// LDS: [3 NZ slices of yz_slice<VL>() elements][tensor slab, 1 KiB multiple].
// ---------------------------------------------------------------------------
// h += T f for one tensor entry set t = (xx, yy, zz, xy, xz, yz) of the
// mixed (kx, ky, dz) domain: xz and yz are coefficients of i; sy, sz are the
// parity signs of ky < 0 and dz < 0.
template <typename T>
__device__ __forceinline__ void tensor_term(const T* __restrict__ t, T sy, T sz,
                                            const cx<T> (&f)[3], cx<T> (&h)[3]) {
  const T xx = t[0], yy = t[1], zz = t[2];
  const T xy = t[3] * sy, xz = t[4] * sz, yz = t[5] * sy * sz;
  const cx<T> ifx = rot90<1>(f[0]), ify = rot90<1>(f[1]), ifz = rot90<1>(f[2]);
  h[0] = add(h[0], add(add(scl(f[0], xx), scl(f[1], xy)), scl(ifz, xz)));
  h[1] = add(h[1], add(add(scl(f[0], xy), scl(f[1], yy)), scl(ifz, yz)));
  h[2] = add(h[2], add(add(scl(ifx, xz), scl(ify, yz)), scl(f[2], zz)));
}

// complex elements of one wave's slice: the transposes of the wave FFT
// (72 VL) and the 8 slots of 64 lanes
__host__ __device__ constexpr int yz_slice_of(int VL) { return VL * 72 > 512 ? VL * 72 : 512; }
template <int VL>
__host__ __device__ constexpr int yz_slice() { return yz_slice_of(VL); }

// bytes of LDS of one yz block (real type of `real` bytes)
__host__ __device__ constexpr size_t yz_lds_of(int real, int VL, int NZ, int tstride) {
  return (size_t)3 * NZ * yz_slice_of(VL) * 2 * real + ((size_t)tstride * real + 1023) / 1024 * 1024;
}
template <typename T, int VL, int NZ>
__host__ __device__ constexpr size_t yz_lds_bytes(int tstride) {
  return yz_lds_of((int)sizeof(T), VL, NZ, tstride);
}

// Every output layer of one position: dst[(zo 3 + c) SL] = scale
// sum_zp T(zo - zp) f[zp], tensor rows at tl + (|dz| nk + kyp) 6 in LDS.
// PAIRS: two output layers per round (more independent chains; double
// precision), else one.
template <typename T, int NZ, bool PAIRS>
__device__ __forceinline__ void yz_position(const T* tl, int nk, int kyp, T sy, T scale,
                                            const cx<T> (&f)[NZ][3], cx<T>* dst, int SL) {
  if constexpr (PAIRS && NZ > 1) {
#pragma unroll 1
    for (int z0 = 0; z0 < NZ; z0 += 2) {
      const int z1 = z0 + 1 < NZ ? z0 + 1 : z0;
      cx<T> h0[3] = {mk(T(0), T(0)), mk(T(0), T(0)), mk(T(0), T(0))};
      cx<T> h1[3] = {mk(T(0), T(0)), mk(T(0), T(0)), mk(T(0), T(0))};
#pragma unroll
      for (int zp = 0; zp < NZ; ++zp) {
        const int da = z0 - zp, db = z1 - zp;
        tensor_term<T>(tl + ((da < 0 ? -da : da) * nk + kyp) * 6, sy, da < 0 ? T(-1) : T(1),
                       f[zp], h0);
        tensor_term<T>(tl + ((db < 0 ? -db : db) * nk + kyp) * 6, sy, db < 0 ? T(-1) : T(1),
                       f[zp], h1);
      }
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        dst[(z0 * 3 + cc) * SL] = scl(h0[cc], scale);
        if (z1 != z0) dst[(z1 * 3 + cc) * SL] = scl(h1[cc], scale);
      }
    }
  } else {
#pragma unroll 1
    for (int zo = 0; zo < NZ; ++zo) {
      cx<T> h[3] = {mk(T(0), T(0)), mk(T(0), T(0)), mk(T(0), T(0))};
#pragma unroll
      for (int zp = 0; zp < NZ; ++zp) {
        const int dz = zo - zp;
        tensor_term<T>(tl + ((dz < 0 ? -dz : dz) * nk + kyp) * 6, sy, dz < 0 ? T(-1) : T(1),
                       f[zp], h);
      }
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) dst[(zo * 3 + cc) * SL] = scl(h[cc], scale);
    }
  }
}

// TWL: the twiddle table (n elements) is copied to LDS after the tensor slab
// and both transforms read it there (launches whose LDS has room for it).
template <typename T, int VL, int NZ, bool TWL = false>
__device__ __forceinline__ void yz_wave_body(cx<T>* __restrict__ A, int ny, int M,
                                             const T* __restrict__ Tt, int tstride, T scale,
                                             const cx<T>* __restrict__ twy,
                                             const int* __restrict__ done, int kx) {
  constexpr int n = 64 * VL;
  constexpr int NG = 8 * VL;                 // lanes holding output slots
  constexpr int NW = 3 * NZ;
  constexpr int nk = n / 2 + 1;
  constexpr int SL = yz_slice<VL>();
  extern __shared__ __align__(16) unsigned char smem[];
  cx<T>* sm = reinterpret_cast<cx<T>*>(smem);
  T* tl = reinterpret_cast<T*>(smem + (size_t)NW * SL * sizeof(cx<T>));
  const int tid = thread_index();
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int z = w / 3, c = w - 3 * (w / 3);
  cx<T>* slice = sm + w * SL;
  cx<T>* Ak = A + (size_t)kx * 3 * NZ * ny;
  cx<T> v[VL];
#pragma unroll
  for (int r = 0; r < VL; ++r) {
    const int y = lane + 64 * r;
    v[r] = y < ny ? Ak[((size_t)z * ny + y) * 3 + c] : mk(T(0), T(0));
  }
  // the stop flag is read while the column loads are in flight
  if (done != nullptr && *done != 0) return;
  const cx<T>* tw = twy;
  if constexpr (TWL) {
    cx<T>* twl = reinterpret_cast<cx<T>*>(smem + yz_lds_of((int)sizeof(T), VL, NZ, tstride));
    for (int i = tid; i < n; i += NW * 64) twl[i] = twy[i];
    __syncthreads();
    tw = twl;
  }
  {
    // tensor slab -> LDS, 16 bytes per lane, no registers involved
    const int nchunk = tstride * (int)sizeof(T) / 16;
    const unsigned char* src = reinterpret_cast<const unsigned char*>(Tt + (size_t)kx * tstride);
    for (int base = w * 64; base < nchunk; base += NW * 64) {
      const int ch = min(base + lane, nchunk - 1);
      __builtin_amdgcn_global_load_lds(
          (const void*)(src + (size_t)ch * 16),
          (__attribute__((address_space(3))) void*)((unsigned char*)tl + (size_t)base * 16), 16,
          0, 0);
    }
  }
  // Both transforms read their twiddles through an offset the compiler
  // cannot see to be zero (kx, ny < 2^30): it then reloads them for the
  // inverse instead of holding the forward pass's in registers across the
  // product, and does not hoist them above the column loads.
  const int zoff = (kx >> 30) + (ny >> 30);
  cx<T> u[8];
  wfft_forward<T, VL, false>(v, u, slice, tw + (kx >> 30), lane);
  __builtin_amdgcn_wave_barrier();
  if (lane < NG) {
#pragma unroll
    for (int d = 0; d < 8; ++d) slice[d * 64 + lane] = u[d];
  }
  __builtin_amdgcn_s_waitcnt(0);   // this wave's tensor copies have landed
  __syncthreads();                 // ... and every wave's, and every slice is written
  // wave w forms slot w (and, with fewer than 8 waves, slots w + NW, ...)
  auto product = [&](int d) {
    const int q = wfft_freq<VL>(lane, d);
    const bool neg = q > n / 2;
    cx<T> f[NZ][3];
#pragma unroll
    for (int zp = 0; zp < NZ; ++zp)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) f[zp][cc] = sm[(zp * 3 + cc) * SL + d * 64 + lane];
    yz_position<T, NZ, sizeof(T) == 8>(tl, nk, neg ? n - q : q, neg ? T(-1) : T(1), scale, f,
                                       sm + d * 64 + lane, SL);
  };
  if (w < 8 && lane < NG) product(w);
  if constexpr (NW < 8) {
    for (int d = w + NW; d < 8; d += NW)
      if (lane < NG) product(d);
  }
  __syncthreads();
  if (lane < NG) {
#pragma unroll
    for (int d = 0; d < 8; ++d) u[d] = slice[d * 64 + lane];
  }
  __builtin_amdgcn_wave_barrier();
  cx<T> xo[VL];
  // the lane index read again for the inverse: otherwise the compiler keeps
  // the forward transform's twiddle offsets (lane multiples) across the
  // product and spills them to scratch memory (single precision at six
  // waves per SIMD, the persistent double-precision kernels for 3 and 4
  // layers), with scratch reloads in the inverse transform's chain
  const int lane_i = thread_index() & 63;
  wfft_inverse<T, VL, false>(u, xo, slice, tw + zoff, lane_i);
  const bool real_col = kx == 0 || kx == M;
#pragma unroll
  for (int r = 0; r < VL; ++r) {
    const int y = lane + 64 * r;
    if (y < ny) Ak[((size_t)z * ny + y) * 3 + c] = real_col ? mk(xo[r].x, T(0)) : xo[r];
  }
}

// waves per SIMD the yz kernels are compiled for: double precision holds
// one 4-layer block per CU (LDS), single precision two.  The tile tuner may
// pick the alternative bound yz_alt_waves_per_eu (fewer resident waves, more
// registers per wave) where a block's 3 nz waves still fit it.
template <typename T>
__host__ __device__ constexpr int yz_waves_per_eu() { return sizeof(T) == 8 ? 3 : 6; }
template <typename T>
__host__ __device__ constexpr int yz_alt_waves_per_eu() { return sizeof(T) == 8 ? 2 : 4; }
template <typename T, int NZ>
__host__ __device__ constexpr bool yz_has_alt() { return 4 * yz_alt_waves_per_eu<T>() >= 3 * NZ; }

template <typename T, int VL, int NZ, int WPE, bool TWL>
__global__ void __launch_bounds__(192 * NZ, WPE)
k_yz_wave(cx<T>* __restrict__ A, int ny, int M, const T* __restrict__ Tt, int tstride, T scale,
          const cx<T>* __restrict__ twy, const int* __restrict__ done) {
  yz_wave_body<T, VL, NZ, TWL>(A, ny, M, Tt, tstride, scale, twy, done, blockIdx.x);
}

// Column kx of sample d.
template <typename T, int VL, int NZ>
__device__ __forceinline__ void yz_desc(const BatchDesc& d, int kx) {
  yz_wave_body<T, VL, NZ>((cx<T>*)d.spec, d.ny, d.M, (const T*)d.Tt, d.tstride, (T)d.scale,
                          (const cx<T>*)d.twy, &d.st->done, kx);
}

// Batched: items[b] = (sample, kx), kx <= M; all samples share Py and nz.
template <typename T, int VL, int NZ>
__global__ void __launch_bounds__(192 * NZ, yz_waves_per_eu<T>())
k_yz_wave_b(const BatchDesc* __restrict__ descs, const WorkItem* __restrict__ items) {
  const WorkItem it = items[blockIdx.x];
  yz_desc<T, VL, NZ>(descs[it.sample], it.block);
}

// Persistent batched: one launch covers the columns of every sample with nz
// layers, whatever its y length Py = 64 VL; each block takes its static
// share of the table (persist_loop) and branches on the item's sample
// length.
template <typename T, int NZ>
__global__ void __launch_bounds__(192 * NZ, yz_waves_per_eu<T>())
k_yz_wave_p(const BatchDesc* __restrict__ descs, const WorkItem* __restrict__ items,
            int n_items) {
  persist_loop(n_items, [&](int v) {
    const WorkItem it = items[v];
    const BatchDesc& d = descs[it.sample];
    switch (d.Py >> 6) {
      case 1: yz_desc<T, 1, NZ>(d, it.block); break;
      case 2: yz_desc<T, 2, NZ>(d, it.block); break;
      case 3: yz_desc<T, 3, NZ>(d, it.block); break;
      case 4: yz_desc<T, 4, NZ>(d, it.block); break;
      case 5: yz_desc<T, 5, NZ>(d, it.block); break;
      case 6: yz_desc<T, 6, NZ>(d, it.block); break;
      case 7: yz_desc<T, 7, NZ>(d, it.block); break;
      case 8: yz_desc<T, 8, NZ>(d, it.block); break;
      default: break;
    }
  });
}

// ---------------------------------------------------------------------------
// Twiddle tables tw[m] = exp(-2 pi i m / P), m < P, from sincospi.
// ---------------------------------------------------------------------------
__global__ void k_twiddles(void* tw, int P, int single) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= P) return;
  double s, c;
  sincospi(-2.0 * (double)m / (double)P, &s, &c);
  if (single) reinterpret_cast<cx<float>*>(tw)[m] = mk((float)c, (float)s);
  else reinterpret_cast<cx<double>*>(tw)[m] = mk(c, s);
}

// ---------------------------------------------------------------------------
// launchers
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

template <typename T>
void launch_fwd_x(hipStream_t s, const double* in, int in_row_stride, int nx_in, int rows, int ncomp,
                  int Px, int R, void* out, const void* twx, const int* done) {
  const int M = Px / 2;
  const long long vals = (long long)R * M;
  const size_t lds = (size_t)vals * sizeof(cx<T>);
  const int nrb = (rows + R - 1) / R;
  dim3 grid(ncomp * nrb);
  if (vals <= 512LL * fft_vpt_cap(M, 8)) {
    auto k = k_fwd_x<T, 8>;
    set_lds(k, lds);
    hipLaunchKernelGGL(k, grid, dim3(threads_for(vals, fft_vpt_cap(M, 8))), lds, s, in,
                       in_row_stride, nx_in, rows, ncomp, Px, R, (cx<T>*)out, (const cx<T>*)twx,
                       done);
  } else {
    auto k = k_fwd_x<T, 16>;
    set_lds(k, lds);
    hipLaunchKernelGGL(k, grid, dim3(threads_for(vals, fft_vpt_cap(M, 16))), lds, s, in,
                       in_row_stride, nx_in, rows, ncomp, Px, R, (cx<T>*)out, (const cx<T>*)twx,
                       done);
  }
}

template <typename T>
void launch_inv_x(hipStream_t s, const void* in, int rows, int ncomp, int nx_out, int Px, int R,
                  double* out, const void* twx, const int* done) {
  const int M = Px / 2;
  const long long vals = (long long)R * M;
  const size_t lds = (size_t)vals * sizeof(cx<T>);
  const int nrb = (rows + R - 1) / R;
  dim3 grid(ncomp * nrb);
  if (vals <= 512LL * fft_vpt_cap(M, 8)) {
    auto k = k_inv_x<T, 8>;
    set_lds(k, lds);
    hipLaunchKernelGGL(k, grid, dim3(threads_for(vals, fft_vpt_cap(M, 8))), lds, s,
                       (const cx<T>*)in, rows, ncomp, nx_out, Px, R, out, (const cx<T>*)twx, done);
  } else {
    auto k = k_inv_x<T, 16>;
    set_lds(k, lds);
    hipLaunchKernelGGL(k, grid, dim3(threads_for(vals, fft_vpt_cap(M, 16))), lds, s,
                       (const cx<T>*)in, rows, ncomp, nx_out, Px, R, out, (const cx<T>*)twx, done);
  }
}

template <typename T>
void launch_fft_cols(hipStream_t s, void* data, int n, int nseq, const void* tw) {
  const int cap = fft_vpt_cap(n, 8);   // values per thread (7 with a radix-7 stage)
  int per = 512 * cap / n;
  if (per < 1) per = 1;   // n <= 512 cap: at most 512 threads
  const long long vals = (long long)per * n;
  const size_t lds = (size_t)vals * sizeof(cx<T>);
  dim3 grid((nseq + per - 1) / per);
  auto k = k_fft_cols<T, 8>;
  set_lds(k, lds);
  hipLaunchKernelGGL(k, grid, dim3(threads_for(vals, cap)), lds, s, (cx<T>*)data, n, nseq, per,
                     (const cx<T>*)tw);
}

bool yz_thin_fits(int nz, int Py, bool single) {
  if (nz < 1 || nz > 4) return false;
  const long long vals = 3LL * nz * Py;
  const size_t lds = (size_t)vals * (single ? 8 : 16);
  return vals <= 16LL * 1024 && lds <= 160 * 1024;
}

template <typename T, int NZ>
static void yz_dispatch(hipStream_t s, void* A, int ny, int Py, int M, const T* Tt, int tstride,
                        T scale, const void* twy, const int* done) {
  const long long vals = 3LL * NZ * Py;
  const size_t lds = (size_t)vals * sizeof(cx<T>);
  dim3 grid(M);
  if (vals <= 8LL * 1024) {
    auto k = k_yz_thin<T, 16, NZ>;
    set_lds(k, lds);
    hipLaunchKernelGGL(k, grid, dim3(threads_for(vals, 16)), lds, s, (cx<T>*)A, ny, Py, M, Tt,
                       tstride, scale, (const cx<T>*)twy, done);
  } else {
    auto k = k_yz_thin<T, 32, NZ>;
    set_lds(k, lds);
    hipLaunchKernelGGL(k, grid, dim3(threads_for(vals, 32)), lds, s, (cx<T>*)A, ny, Py, M, Tt,
                       tstride, scale, (const cx<T>*)twy, done);
  }
}

template <typename T, int VL, int NZ, int WPE>
static void yz_wave_launch(hipStream_t s, void* A, int ny, int M, const T* Tt, int tstride,
                           T scale, const void* twy, const int* done) {
  // single precision: the twiddle table joins the block's LDS where the
  // blocks resident per CU (160 KiB of LDS, WPE waves per SIMD) stay as
  // many (measured on the film: 17.6 -> 17.1 us; in double precision the
  // pass was 1% slower with it)
  const size_t lds = yz_lds_bytes<T, VL, NZ>(tstride);
  if constexpr (sizeof(T) == 4) {
    const size_t ldt = lds + (size_t)64 * VL * sizeof(cx<T>);
    constexpr size_t kCuLds = (size_t)160 * 1024;
    constexpr size_t by_waves = (size_t)(4 * WPE) / (3 * NZ);
    auto resident = [&](size_t b) { return std::min(kCuLds / b, by_waves); };
    if (ldt <= kCuLds && resident(ldt) == resident(lds)) {
      auto k = k_yz_wave<T, VL, NZ, WPE, true>;
      set_lds(k, ldt);
      hipLaunchKernelGGL(k, dim3(M + 1), dim3(192 * NZ), ldt, s, (cx<T>*)A, ny, M, Tt, tstride,
                         scale, (const cx<T>*)twy, done);
      return;
    }
  }
  auto k = k_yz_wave<T, VL, NZ, WPE, false>;
  set_lds(k, lds);
  hipLaunchKernelGGL(k, dim3(M + 1), dim3(192 * NZ), lds, s, (cx<T>*)A, ny, M, Tt, tstride, scale,
                     (const cx<T>*)twy, done);
}

template <typename T, int VL, int NZ>
static void yz_wave_dispatch(hipStream_t s, void* A, int ny, int M, const T* Tt, int tstride,
                             T scale, const void* twy, const int* done, int var) {
  if constexpr (yz_has_alt<T, NZ>()) {
    if (var == 1) {
      yz_wave_launch<T, VL, NZ, yz_alt_waves_per_eu<T>()>(s, A, ny, M, Tt, tstride, scale, twy,
                                                          done);
      return;
    }
  }
  yz_wave_launch<T, VL, NZ, yz_waves_per_eu<T>()>(s, A, ny, M, Tt, tstride, scale, twy, done);
}

template <typename T, int VL>
static void yz_wave_nz(hipStream_t s, void* A, int nz, int ny, int M, const T* Tt, int tstride,
                       T scale, const void* twy, const int* done, int var) {
  switch (nz) {
    case 1: yz_wave_dispatch<T, VL, 1>(s, A, ny, M, Tt, tstride, scale, twy, done, var); break;
    case 2: yz_wave_dispatch<T, VL, 2>(s, A, ny, M, Tt, tstride, scale, twy, done, var); break;
    case 3: yz_wave_dispatch<T, VL, 3>(s, A, ny, M, Tt, tstride, scale, twy, done, var); break;
    default: yz_wave_dispatch<T, VL, 4>(s, A, ny, M, Tt, tstride, scale, twy, done, var); break;
  }
}

bool yz_wave_ok(int nz, int Py) {
  return nz >= 1 && nz <= 4 && Py % 64 == 0 && Py >= 64 && Py <= 512;
}

int yz_variants(bool single, int nz, int Py) {
  if (!yz_wave_ok(nz, Py)) return 1;
  const int alt = single ? yz_alt_waves_per_eu<float>() : yz_alt_waves_per_eu<double>();
  return 4 * alt >= 3 * nz ? 2 : 1;
}

template <typename T>
void launch_yz_thin(hipStream_t s, void* A, int nz, int ny, int Py, int M, const T* Tt,
                    int tstride, T scale, const void* twy, const int* done, int var) {
  if (yz_wave_ok(nz, Py)) {
    switch (Py) {
      case 64: yz_wave_nz<T, 1>(s, A, nz, ny, M, Tt, tstride, scale, twy, done, var); return;
      case 128: yz_wave_nz<T, 2>(s, A, nz, ny, M, Tt, tstride, scale, twy, done, var); return;
      case 192: yz_wave_nz<T, 3>(s, A, nz, ny, M, Tt, tstride, scale, twy, done, var); return;
      case 256: yz_wave_nz<T, 4>(s, A, nz, ny, M, Tt, tstride, scale, twy, done, var); return;
      case 320: yz_wave_nz<T, 5>(s, A, nz, ny, M, Tt, tstride, scale, twy, done, var); return;
      case 384: yz_wave_nz<T, 6>(s, A, nz, ny, M, Tt, tstride, scale, twy, done, var); return;
      case 448: yz_wave_nz<T, 7>(s, A, nz, ny, M, Tt, tstride, scale, twy, done, var); return;
      default: yz_wave_nz<T, 8>(s, A, nz, ny, M, Tt, tstride, scale, twy, done, var); return;
    }
  }
  switch (nz) {
    case 1: yz_dispatch<T, 1>(s, A, ny, Py, M, Tt, tstride, scale, twy, done); break;
    case 2: yz_dispatch<T, 2>(s, A, ny, Py, M, Tt, tstride, scale, twy, done); break;
    case 3: yz_dispatch<T, 3>(s, A, ny, Py, M, Tt, tstride, scale, twy, done); break;
    default: yz_dispatch<T, 4>(s, A, ny, Py, M, Tt, tstride, scale, twy, done); break;
  }
}

template <typename T, int VL, int NZ>
static void yzb_dispatch(hipStream_t s, const BatchDesc* descs, const WorkItem* items, int n_items,
                         int tstride) {
  const size_t lds = yz_lds_bytes<T, VL, NZ>(tstride);
  auto k = k_yz_wave_b<T, VL, NZ>;
  set_lds(k, lds);
  hipLaunchKernelGGL(k, dim3(n_items), dim3(192 * NZ), lds, s, descs, items);
}

template <typename T, int VL>
static void yzb_nz(hipStream_t s, const BatchDesc* descs, const WorkItem* items, int n_items,
                   int nz, int tstride) {
  switch (nz) {
    case 1: yzb_dispatch<T, VL, 1>(s, descs, items, n_items, tstride); break;
    case 2: yzb_dispatch<T, VL, 2>(s, descs, items, n_items, tstride); break;
    case 3: yzb_dispatch<T, VL, 3>(s, descs, items, n_items, tstride); break;
    default: yzb_dispatch<T, VL, 4>(s, descs, items, n_items, tstride); break;
  }
}

template <typename T>
void launch_yz_batched(hipStream_t s, const BatchDesc* descs, const WorkItem* items, int n_items,
                       int Py, int nz, int tstride) {
  switch (Py) {
    case 64: yzb_nz<T, 1>(s, descs, items, n_items, nz, tstride); break;
    case 128: yzb_nz<T, 2>(s, descs, items, n_items, nz, tstride); break;
    case 192: yzb_nz<T, 3>(s, descs, items, n_items, nz, tstride); break;
    case 256: yzb_nz<T, 4>(s, descs, items, n_items, nz, tstride); break;
    case 320: yzb_nz<T, 5>(s, descs, items, n_items, nz, tstride); break;
    case 384: yzb_nz<T, 6>(s, descs, items, n_items, nz, tstride); break;
    case 448: yzb_nz<T, 7>(s, descs, items, n_items, nz, tstride); break;
    default: yzb_nz<T, 8>(s, descs, items, n_items, nz, tstride); break;
  }
}

template <typename T, int NZ>
static const void* yzp_kernel() {
  return (const void*)k_yz_wave_p<T, NZ>;
}

template <typename T>
static const void* yzp_kernel_nz(int nz) {
  switch (nz) {
    case 1: return yzp_kernel<T, 1>();
    case 2: return yzp_kernel<T, 2>();
    case 3: return yzp_kernel<T, 3>();
    default: return yzp_kernel<T, 4>();
  }
}

size_t yz_block_lds(bool single, int Py, int nz, int tstride) {
  return yz_lds_of(single ? 4 : 8, Py / 64, nz, tstride);
}

int yz_persistent_grid(bool single, int nz, size_t lds) {
  const void* k = single ? yzp_kernel_nz<float>(nz) : yzp_kernel_nz<double>(nz);
  if (lds > 48 * 1024) (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 192 * nz, lds) != hipSuccess ||
      hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    return 8;
  }
  const int g = per_cu * cus / 8 * 8;
  return g < 8 ? 8 : g;
}

template <typename T>
void launch_yz_persistent(hipStream_t s, const BatchDesc* descs, const WorkItem* items,
                          int n_items, int nz, size_t lds, int grid) {
  const int g = n_items < grid ? n_items : grid;
  if (g <= 0) return;
  const void* k = yzp_kernel_nz<T>(nz);
  if (lds > 48 * 1024) (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  void* args[] = {(void*)&descs, (void*)&items, (void*)&n_items};
  (void)hipLaunchKernel(k, dim3(g), dim3(192 * nz), args, lds, s);
}

template void launch_yz_persistent<double>(hipStream_t, const BatchDesc*, const WorkItem*, int,
                                           int, size_t, int);
template void launch_yz_persistent<float>(hipStream_t, const BatchDesc*, const WorkItem*, int, int,
                                          size_t, int);
template void launch_yz_batched<double>(hipStream_t, const BatchDesc*, const WorkItem*, int, int,
                                        int, int);
template void launch_yz_batched<float>(hipStream_t, const BatchDesc*, const WorkItem*, int, int,
                                       int, int);

void launch_twiddles(hipStream_t s, void* tw, int P, bool single) {
  hipLaunchKernelGGL(k_twiddles, dim3((P + 255) / 256), dim3(256), 0, s, tw, P, single ? 1 : 0);
}

template void launch_fwd_x<double>(hipStream_t, const double*, int, int, int, int, int, int, void*,
                                   const void*, const int*);
template void launch_fwd_x<float>(hipStream_t, const double*, int, int, int, int, int, int, void*,
                                  const void*, const int*);
template void launch_inv_x<double>(hipStream_t, const void*, int, int, int, int, int, double*,
                                   const void*, const int*);
template void launch_inv_x<float>(hipStream_t, const void*, int, int, int, int, int, double*,
                                  const void*, const int*);
template void launch_fft_cols<double>(hipStream_t, void*, int, int, const void*);
template void launch_yz_thin<double>(hipStream_t, void*, int, int, int, int, const double*, int,
                                     double, const void*, const int*, int);
template void launch_yz_thin<float>(hipStream_t, void*, int, int, int, int, const float*, int, float,
                                    const void*, const int*, int);

}  // namespace mmk
