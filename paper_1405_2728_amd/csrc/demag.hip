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
//   yz_wave as yz_thin, with register-resident wave FFTs (one wave per z
//           layer, Py = 64..512) and one block per column kx = 0..M
// The factor -Ms/(M Py) of the inverse transforms is applied in yz_thin.
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
// y-FFT, tensor product with z convolution, inverse y-FFT; wave FFT version.
// Block = NZ wavefronts, wave z owns layer z (three components); block kx
// handles column kx in 1..M-1, and block 0 the two real-input columns kx = 0
// and kx = M packed as re + i im (so that M blocks, not M + 1, fill the
// machine).  Lane g holds the frequencies ky = wfft_freq(g, d), d < 8.  The
// tensor slab of the column is copied to LDS with direct global-to-LDS loads
// while the forward transforms run; the z convolution exchanges two slots d
// at a time through LDS.
// Block 0: with U = F0 + i FM the transform of the packed column (F0, FM the
// Hermitian spectra of the two real columns), P = (U(k) + conj U(-k))/2 = F0
// and Q = (U(k) - conj U(-k))/2 = i FM, and T0 P + TM Q = H0 + i HM is the
// transform of the packed result.  Frequency -k lies in slot 7 - d of lane
// g' (k1 = g/8, c = g%8: g' = 8 (VL - k1) + 7 - c for k1 >= 1, g' = 8 - c
// for k1 = 0), except on lane 0, whose slots pair as (d, 8 - d).  In
// registers, slots 0..3 are turned into P(k) and slots 4..7 into Q(-q) (one
// shuffle per slot pair); pass 1 applies T0 to slots 0..3, the kx = M tensor
// then replaces T0 in LDS and pass 2 applies it to slots 4..7 (at -q); a
// second shuffle forms V(k) = V1(k) + V2(k) with V1(-k) = conj V1(k) and
// V2(-k) = -conj V2(k).  Frequencies 0 and n/2 (lane 0, slots 0 and 4) see a
// real diagonal tensor: real part with T0, imaginary part with TM.
// LDS: [tensor slab, padded to 1 KiB] [transposes | exchange buffer] [4 diagonal
// tensor entries per layer for block 0].
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ cx<T> shfl_cx(cx<T> v, int src) {
  return mk(__shfl(v.x, src, 64), __shfl(v.y, src, 64));
}

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

// Offset (complex elements) of block 0's diagonal tensor entries after the
// transposes and the exchange buffer; they take 3 NZ elements (6 NZ reals),
// followed by lane 0's saved values (24 per layer).
template <int VL, int NZ, bool HALF>
__host__ __device__ constexpr int yz_pt_offset() {
  return NZ * wfft_buf<VL, HALF>() > NZ * 3 * 2 * 64 ? NZ * wfft_buf<VL, HALF>() : NZ * 3 * 2 * 64;
}

template <typename T, int VL, int NZ, bool HALF>
__device__ __forceinline__ void yz_wave_body(cx<T>* __restrict__ A, int ny, int M,
                                             const T* __restrict__ Tt, int tstride, T scale,
                                             const cx<T>* __restrict__ twy,
                                             const int* __restrict__ done, int kx) {
  // the stop flag is read while the first column loads are in flight
  const int dn = done != nullptr ? *done : 0;
  constexpr int n = 64 * VL;
  constexpr int NG = 8 * VL;
  constexpr int DC = 2;                       // slots exchanged per round
  constexpr int nk = n / 2 + 1;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tl_bytes = ((tstride * (int)sizeof(T) + 1023) / 1024) * 1024;
  T* tl = reinterpret_cast<T*>(smem);
  cx<T>* sm = reinterpret_cast<cx<T>*>(smem + tl_bytes);
  const int lane = threadIdx.x & 63;
  const int z = threadIdx.x >> 6;
  cx<T>* tbuf = sm + z * wfft_buf<VL, HALF>();   // wave-private transpose buffer
  cx<T>* xbuf = sm;                              // exchange buffer [z][c][DC][64]
  const size_t slab = (size_t)3 * NZ * ny;
  const bool pair = kx == 0;                     // columns 0 and M, packed
  cx<T>* Ak = A + (size_t)kx * slab;
  cx<T>* AM = A + (size_t)M * slab;
  auto load = [&](int c, int y) -> cx<T> {
    if (y >= ny) return mk(T(0), T(0));
    const size_t e = ((size_t)z * ny + y) * 3 + c;
    return pair ? mk(Ak[e].x, AM[e].x) : Ak[e];
  };
  // column loads (three components of layer z), one component ahead
  cx<T> F[3][8];
  cx<T> xin[2][VL];
#pragma unroll
  for (int r = 0; r < VL; ++r) xin[0][r] = load(0, lane + 64 * r);
  if (dn != 0) return;             // before any LDS copy is started
  // tensor slab -> LDS, 16 bytes per lane, no registers involved
  auto stage_tensor = [&](const T* slab_src) {
    const int nchunk = tstride * (int)sizeof(T) / 16;
    const unsigned char* src = reinterpret_cast<const unsigned char*>(slab_src);
    for (int base = z * 64; base < nchunk; base += NZ * 64) {
      const int ch = min(base + lane, nchunk - 1);
      __builtin_amdgcn_global_load_lds(
          (const void*)(src + (size_t)ch * 16),
          (__attribute__((address_space(3))) void*)(smem + (size_t)base * 16), 16, 0, 0);
    }
  };
  stage_tensor(Tt + (size_t)kx * tstride);
  // block 0: diagonal entries T0(dz, n/2) and TM(dz, 0), [2][NZ][3]
  constexpr int pt_off = yz_pt_offset<VL, NZ, HALF>();
  T* pt = reinterpret_cast<T*>(sm + pt_off);
  if (pair && threadIdx.x < 6 * NZ) {
    const int t = threadIdx.x, which = t / (3 * NZ), dz = (t % (3 * NZ)) / 3, c = t % 3;
    pt[t] = Tt[(size_t)(which ? M : 0) * tstride + (dz * nk + (which ? 0 : n / 2)) * 6 + c];
  }
  // forward transforms
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (c < 2) {
#pragma unroll
      for (int r = 0; r < VL; ++r) xin[(c + 1) & 1][r] = load(c + 1, lane + 64 * r);
    }
    wfft_forward<T, VL, HALF>(xin[c & 1], F[c], tbuf, twy, lane);
    __builtin_amdgcn_sched_barrier(0);
  }
  __builtin_amdgcn_s_waitcnt(0);   // tensor copy complete (this wave's part)
  __syncthreads();                 // ... and every wave's; transposes done
  // block 0: lane 0 pairs its own slots (d, 8 - d); its values are kept in
  // LDS [z][c][8] around the two register transforms
  const int k1 = lane >> 3, cl = lane & 7;
  const int gp = lane >= NG ? lane : (k1 >= 1 ? 8 * (VL - k1) + 7 - cl : 8 - cl);
  cx<T>* l0 = sm + pt_off + 3 * NZ + z * 24;
  auto keep_lane0 = [&]() {
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int d = 0; d < 8; ++d) l0[c * 8 + d] = F[c][d];
    }
    __builtin_amdgcn_wave_barrier();
  };
  if (pair) {
    // slots 0..3 -> P(k), slots 4..7 -> Q(-q)
    keep_lane0();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const cx<T> uj = F[c][j], u7 = F[c][7 - j];
        const cx<T> pa = shfl_cx(u7, gp), pb = shfl_cx(uj, gp);
        cx<T> wj = scl(add(uj, conj(pa)), T(0.5));
        cx<T> w7 = scl(sub(pb, conj(u7)), T(0.5));
        if (lane == 0) {
          wj = j == 0 ? uj : scl(add(uj, conj(l0[c * 8 + ((8 - j) & 7)])), T(0.5));
          w7 = j <= 2 ? scl(sub(l0[c * 8 + j + 1], conj(u7)), T(0.5)) : u7;
        }
        F[c][j] = wj;
        F[c][7 - j] = w7;
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  // Tensor product.  Block 0: slots 0..3 with the kx = 0 tensor, slots 4..7
  // (at -q) with the kx = M tensor staged in between; lane 0's slots 0 and 4
  // (ky = 0, n/2) see real diagonal tensors, real part T0, imaginary part TM.
  const T* p0 = pt;              // T0(dz, n/2) diagonal
  const T* pM = pt + 3 * NZ;     // TM(dz, 0) diagonal
  constexpr int DCP = NZ == 1 ? 1 : DC;   // one layer: no exchange needed
#pragma unroll
  for (int d0 = 0; d0 < 8; d0 += DCP) {
    if (pair && d0 == 4) {
      // every wave has finished with T0 (barrier at the end of the round)
      stage_tensor(Tt + (size_t)M * tstride);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
    if constexpr (NZ > 1) {
      if (lane < NG) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int dl = 0; dl < DCP; ++dl) xbuf[((z * 3 + c) * DCP + dl) * 64 + lane] = F[c][d0 + dl];
      }
      __syncthreads();
    }
    if (lane < NG) {
#pragma unroll
      for (int dl = 0; dl < DCP; ++dl) {
        const int d = d0 + dl;
        const int q = wfft_freq<VL>(lane, d);
        const bool neg = q > n / 2;
        const bool at_minus = pair && d >= 4;
        const int kyp = (neg || at_minus) ? n - q : q;
        const T sy = (neg && !at_minus) ? T(-1) : T(1);
        const bool diag = pair && lane == 0 && (d == 0 || d == 4);
        cx<T> h[3] = {mk(T(0), T(0)), mk(T(0), T(0)), mk(T(0), T(0))};
#pragma unroll 1
        for (int zp = 0; zp < NZ; ++zp) {
          const int dz = z - zp;
          const int dzp = dz < 0 ? -dz : dz;
          const T sz = dz < 0 ? T(-1) : T(1);
          cx<T> f[3];
          if constexpr (NZ > 1) {
#pragma unroll
            for (int c = 0; c < 3; ++c) f[c] = xbuf[((zp * 3 + c) * DCP + dl) * 64 + lane];
          } else {
#pragma unroll
            for (int c = 0; c < 3; ++c) f[c] = F[c][d];
          }
          if (!diag) {
            tensor_term<T>(tl + (dzp * nk + kyp) * 6, sy, sz, f, h);
          } else {
            const T* tre = d == 0 ? tl + (dzp * nk) * 6 : p0 + dzp * 3;
            const T* tim = d == 0 ? pM + dzp * 3 : tl + (dzp * nk + n / 2) * 6;
#pragma unroll
            for (int c = 0; c < 3; ++c) h[c] = add(h[c], mk(tre[c] * f[c].x, tim[c] * f[c].y));
          }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) F[c][d] = scl(h[c], scale);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    if constexpr (NZ > 1) __syncthreads();
  }
  if (pair) {
    // V(k) = V1(k) + V2(k) on slots 0..3, conj V1(-q) - conj V2(-q) on 4..7
    keep_lane0();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const cx<T> vj = F[c][j], v7 = F[c][7 - j];
        const cx<T> a = shfl_cx(v7, gp), b = shfl_cx(vj, gp);
        cx<T> rj = add(vj, a);
        cx<T> r7 = sub(conj(b), conj(v7));
        if (lane == 0) {
          rj = j == 0 ? vj : add(vj, l0[c * 8 + ((8 - j) & 7)]);
          r7 = j <= 2 ? sub(conj(l0[c * 8 + j + 1]), conj(v7)) : v7;
        }
        F[c][j] = rj;
        F[c][7 - j] = r7;
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  // inverse transforms and store of the ny kept rows (block 0: unpacked)
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cx<T> xo[VL];
    wfft_inverse<T, VL, HALF>(F[c], xo, tbuf, twy, lane);
#pragma unroll
    for (int r = 0; r < VL; ++r) {
      const int y = lane + 64 * r;
      if (y >= ny) continue;
      const size_t e = ((size_t)z * ny + y) * 3 + c;
      if (pair) {
        Ak[e] = mk(xo[r].x, T(0));
        AM[e] = mk(xo[r].y, T(0));
      } else {
        Ak[e] = xo[r];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <typename T, int VL, int NZ, bool HALF>
__global__ void __launch_bounds__(64 * NZ, 2)
k_yz_wave(cx<T>* __restrict__ A, int ny, int M, const T* __restrict__ Tt, int tstride, T scale,
          const cx<T>* __restrict__ twy, const int* __restrict__ done) {
  yz_wave_body<T, VL, NZ, HALF>(A, ny, M, Tt, tstride, scale, twy, done, blockIdx.x);
}

// Batched: items[b] = (sample, kx), kx < M; all samples share Py and nz.
template <typename T, int VL, int NZ, bool HALF>
__global__ void __launch_bounds__(64 * NZ, 2)
k_yz_wave_b(const BatchDesc* __restrict__ descs, const WorkItem* __restrict__ items) {
  const WorkItem it = items[blockIdx.x];
  const BatchDesc& d = descs[it.sample];
  yz_wave_body<T, VL, NZ, HALF>((cx<T>*)d.spec, d.ny, d.M, (const T*)d.Tt, d.tstride, (T)d.scale,
                                (const cx<T>*)d.twy, &d.st->done, it.block);
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

template <typename T, int VL, int NZ>
static void yz_wave_dispatch(hipStream_t s, void* A, int ny, int M, const T* Tt, int tstride,
                             T scale, const void* twy, const int* done) {
  constexpr bool HALF = sizeof(T) == 8 && VL >= 4;     // keep two blocks per CU in FP64
  // transposes | exchange buffer, then block 0's diagonal tensor entries
  const size_t un = (size_t)yz_pt_offset<VL, NZ, HALF>() + 3 * NZ + 24 * NZ;
  const size_t tl = ((tstride * sizeof(T) + 1023) / 1024) * 1024;
  const size_t lds = tl + un * sizeof(cx<T>);
  auto k = k_yz_wave<T, VL, NZ, HALF>;
  set_lds(k, lds);
  hipLaunchKernelGGL(k, dim3(M), dim3(64 * NZ), lds, s, (cx<T>*)A, ny, M, Tt, tstride, scale,
                     (const cx<T>*)twy, done);
}

template <typename T, int VL>
static void yz_wave_nz(hipStream_t s, void* A, int nz, int ny, int M, const T* Tt, int tstride,
                       T scale, const void* twy, const int* done) {
  switch (nz) {
    case 1: yz_wave_dispatch<T, VL, 1>(s, A, ny, M, Tt, tstride, scale, twy, done); break;
    case 2: yz_wave_dispatch<T, VL, 2>(s, A, ny, M, Tt, tstride, scale, twy, done); break;
    case 3: yz_wave_dispatch<T, VL, 3>(s, A, ny, M, Tt, tstride, scale, twy, done); break;
    default: yz_wave_dispatch<T, VL, 4>(s, A, ny, M, Tt, tstride, scale, twy, done); break;
  }
}

bool yz_wave_ok(int nz, int Py) {
  return nz >= 1 && nz <= 4 && Py % 64 == 0 && Py >= 64 && Py <= 512;
}

template <typename T>
void launch_yz_thin(hipStream_t s, void* A, int nz, int ny, int Py, int M, const T* Tt,
                    int tstride, T scale, const void* twy, const int* done) {
  if (yz_wave_ok(nz, Py)) {
    switch (Py) {
      case 64: yz_wave_nz<T, 1>(s, A, nz, ny, M, Tt, tstride, scale, twy, done); return;
      case 128: yz_wave_nz<T, 2>(s, A, nz, ny, M, Tt, tstride, scale, twy, done); return;
      case 192: yz_wave_nz<T, 3>(s, A, nz, ny, M, Tt, tstride, scale, twy, done); return;
      case 256: yz_wave_nz<T, 4>(s, A, nz, ny, M, Tt, tstride, scale, twy, done); return;
      case 320: yz_wave_nz<T, 5>(s, A, nz, ny, M, Tt, tstride, scale, twy, done); return;
      case 384: yz_wave_nz<T, 6>(s, A, nz, ny, M, Tt, tstride, scale, twy, done); return;
      case 448: yz_wave_nz<T, 7>(s, A, nz, ny, M, Tt, tstride, scale, twy, done); return;
      default: yz_wave_nz<T, 8>(s, A, nz, ny, M, Tt, tstride, scale, twy, done); return;
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
  constexpr bool HALF = sizeof(T) == 8 && VL >= 4;
  const size_t un = (size_t)yz_pt_offset<VL, NZ, HALF>() + 3 * NZ + 24 * NZ;
  const size_t tl = ((tstride * sizeof(T) + 1023) / 1024) * 1024;
  const size_t lds = tl + un * sizeof(cx<T>);
  auto k = k_yz_wave_b<T, VL, NZ, HALF>;
  set_lds(k, lds);
  hipLaunchKernelGGL(k, dim3(n_items), dim3(64 * NZ), lds, s, descs, items);
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
                                     double, const void*, const int*);
template void launch_yz_thin<float>(hipStream_t, void*, int, int, int, int, const float*, int, float,
                                    const void*, const int*);

}  // namespace mmk
