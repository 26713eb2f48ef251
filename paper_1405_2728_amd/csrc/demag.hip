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
//           -> spectrum X[0..M] written as A[kx][c][z][y]
//   yz_thin one block per kx: y-FFT of the 3*nz columns (zero padded to Py),
//           symmetric 3x3 tensor times vector with the z convolution,
//           inverse y-FFT, keep ny rows.  The block of kx = 0 also carries
//           kx = M: both columns are spectra of real data, packed as
//           re + i*im and separated by Hermitian symmetry in ky.
//   inv_x   A[kx][c][z][y] -> half-length inverse -> H_d rows (double)
// The factor -Ms/(M Py) of the inverse transforms is applied in yz_thin.
#include "mm_device.h"
#include "mm_kernels.h"

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
  fft_lds<-1, VPT>(buf, M, R, M, twx, Px, tid, nthr);
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
  fft_lds<1, VPT>(buf, M, R, M, twx, Px, tid, nthr);
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
  fft_lds<-1, VPT>(buf, n, ns, n, tw, n, tid, nthr);
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
k_yz_thin(cx<T>* __restrict__ A, int ny, int Py, int M, const T* __restrict__ Tt, T scale,
          const cx<T>* __restrict__ twy, const int* __restrict__ done) {
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
      if (kx == 0) v = mk(A[(size_t)col * ny + y].x, A[(size_t)M * slab + (size_t)col * ny + y].x);
      else v = A[(size_t)kx * slab + (size_t)col * ny + y];
    }
    buf[col * S + y] = v;
  }
  __syncthreads();
  fft_lds<-1, VPT>(buf, Py, nseq, S, twy, Py, tid, nthr);
  const int nk = (Py >> 1) + 1;
  const size_t tslab = (size_t)NZ * nk * 6;
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
    if (kx == 0) {
      A[(size_t)col * ny + y] = mk(v.x, T(0));
      A[(size_t)M * slab + (size_t)col * ny + y] = mk(v.y, T(0));
    } else {
      A[(size_t)kx * slab + (size_t)col * ny + y] = v;
    }
  }
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
  if (vals <= 4LL * 1024) {
    auto k = k_fwd_x<T, 8>;
    set_lds(k, lds);
    hipLaunchKernelGGL(k, grid, dim3(threads_for(vals, 8)), lds, s, in, in_row_stride, nx_in, rows,
                       ncomp, Px, R, (cx<T>*)out, (const cx<T>*)twx, done);
  } else {
    auto k = k_fwd_x<T, 16>;
    set_lds(k, lds);
    hipLaunchKernelGGL(k, grid, dim3(threads_for(vals, 16)), lds, s, in, in_row_stride, nx_in,
                       rows, ncomp, Px, R, (cx<T>*)out, (const cx<T>*)twx, done);
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
  if (vals <= 4LL * 1024) {
    auto k = k_inv_x<T, 8>;
    set_lds(k, lds);
    hipLaunchKernelGGL(k, grid, dim3(threads_for(vals, 8)), lds, s, (const cx<T>*)in, rows, ncomp,
                       nx_out, Px, R, out, (const cx<T>*)twx, done);
  } else {
    auto k = k_inv_x<T, 16>;
    set_lds(k, lds);
    hipLaunchKernelGGL(k, grid, dim3(threads_for(vals, 16)), lds, s, (const cx<T>*)in, rows, ncomp,
                       nx_out, Px, R, out, (const cx<T>*)twx, done);
  }
}

template <typename T>
void launch_fft_cols(hipStream_t s, void* data, int n, int nseq, const void* tw) {
  int per = 4096 / n;
  if (per < 1) per = 1;   // n <= 4096: at most 512 threads of 8 values
  const long long vals = (long long)per * n;
  const size_t lds = (size_t)vals * sizeof(cx<T>);
  dim3 grid((nseq + per - 1) / per);
  auto k = k_fft_cols<T, 8>;
  set_lds(k, lds);
  hipLaunchKernelGGL(k, grid, dim3(threads_for(vals, 8)), lds, s, (cx<T>*)data, n, nseq, per,
                     (const cx<T>*)tw);
}

bool yz_thin_fits(int nz, int Py, bool single) {
  if (nz < 1 || nz > 4) return false;
  const long long vals = 3LL * nz * Py;
  const size_t lds = (size_t)vals * (single ? 8 : 16);
  return vals <= 16LL * 1024 && lds <= 160 * 1024;
}

template <typename T, int NZ>
static void yz_dispatch(hipStream_t s, void* A, int ny, int Py, int M, const T* Tt, T scale,
                        const void* twy, const int* done) {
  const long long vals = 3LL * NZ * Py;
  const size_t lds = (size_t)vals * sizeof(cx<T>);
  dim3 grid(M);
  if (vals <= 8LL * 1024) {
    auto k = k_yz_thin<T, 16, NZ>;
    set_lds(k, lds);
    hipLaunchKernelGGL(k, grid, dim3(threads_for(vals, 16)), lds, s, (cx<T>*)A, ny, Py, M, Tt,
                       scale, (const cx<T>*)twy, done);
  } else {
    auto k = k_yz_thin<T, 32, NZ>;
    set_lds(k, lds);
    hipLaunchKernelGGL(k, grid, dim3(threads_for(vals, 32)), lds, s, (cx<T>*)A, ny, Py, M, Tt,
                       scale, (const cx<T>*)twy, done);
  }
}

template <typename T>
void launch_yz_thin(hipStream_t s, void* A, int nz, int ny, int Py, int M, const T* Tt, T scale,
                    const void* twy, const int* done) {
  switch (nz) {
    case 1: yz_dispatch<T, 1>(s, A, ny, Py, M, Tt, scale, twy, done); break;
    case 2: yz_dispatch<T, 2>(s, A, ny, Py, M, Tt, scale, twy, done); break;
    case 3: yz_dispatch<T, 3>(s, A, ny, Py, M, Tt, scale, twy, done); break;
    default: yz_dispatch<T, 4>(s, A, ny, Py, M, Tt, scale, twy, done); break;
  }
}

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
template void launch_yz_thin<double>(hipStream_t, void*, int, int, int, int, const double*, double,
                                     const void*, const int*);
template void launch_yz_thin<float>(hipStream_t, void*, int, int, int, int, const float*, float,
                                    const void*, const int*);

}  // namespace mmk
