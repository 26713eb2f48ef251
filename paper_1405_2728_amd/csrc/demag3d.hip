// Demagnetisation field as a zero-padded FFT convolution on the regular
// cuboid grid (Sec. 3 of the paper), full 3-D path for grids with more than
// four layers.
//
// Padded sizes: Py = max(64, 2^ceil(log2(2ny-1))), Pz likewise for nz; both
// at most 512 (one wave-level register FFT per sequence).  The x passes
// (half-length real transform along x) are the ones of the thin-film path
// and leave the spectrum A[kx][z][y][c] (kx = 0..M, c = component).
//
//   y3 forward  one wave per (kx, z) plane: y-FFT of the three columns
//               (ny values, zero padded to Py) -> B[kx][ky][z][c]
//   z3          one wave per (kx, ky) pencil: z-FFT of the three components
//               (nz values, zero padded to Pz), product with the real
//               symmetric 3x3 Fourier tensor, inverse z-FFT, nz values kept
//               in place; the factor -Ms/(M Py Pz) of the inverse transforms
//               is applied here
//   y3 inverse  B -> A, rows y < ny kept; the real-input columns kx = 0 and
//               kx = M store imaginary part 0
//
// Tensor T3[kx][ky'][kz'][6] (xx, yy, zz, xy, xz, yz), ky' <= Py/2,
// kz' <= Pz/2: the cell tensor is even in every axis for the diagonal
// entries and odd in the two axes an off-diagonal entry names, so its
// transform is real, and the entries at ky > Py/2 or kz > Pz/2 follow from
// the stored octant with a sign flip per odd axis.
#include "mm_iter.h"
#include "mm_kernels.h"
#include "mm_wfft.h"

namespace mmk {

// The stages transpose through a full wave buffer of the wave FFT (one
// exchange per pass), not the half buffer (half the LDS, twice the
// exchanges): LDS does not limit these kernels, registers do, and the full
// buffer also takes fewer of those (FP64, 256 points: y3_fwd 132 against
// 160 VGPRs, z3 170 against 172).
constexpr bool k3dHalf = false;

constexpr int kY3Waves = 4;   // (kx, z) planes per block of the y passes
constexpr int kZ3Waves = 4;   // (kx, ky) pencils per block of the z pass

// Logical block L of the forward y pass (planes (kx, z) .. z + 3).
template <typename T, int VL, bool HALF>
__device__ __forceinline__ void y3_fwd_body(const cx<T>* __restrict__ A, cx<T>* __restrict__ B,
                                            int nz, int ny, int nzb,
                                            const cx<T>* __restrict__ twy,
                                            const int* __restrict__ done, int L) {
  if (done != nullptr && *done != 0) return;
  constexpr int n = 64 * VL;
  constexpr int NG = 8 * VL;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = thread_index();
  const int lane = tid & 63, w = tid >> 6;
  const int kx = L / nzb;
  const int z = (L - kx * nzb) * kY3Waves + w;
  if (z >= nz) return;                       // no block barrier below
  cx<T>* tbuf = reinterpret_cast<cx<T>*>(smem) + w * wfft_buf<VL, HALF>();
  const cx<T>* Ap = A + ((size_t)kx * nz + z) * ny * 3;
  cx<T> F[3][8];
  cx<T> xin[2][VL];
#pragma unroll
  for (int r = 0; r < VL; ++r) {
    const int y = lane + 64 * r;
    xin[0][r] = y < ny ? Ap[(size_t)y * 3] : mk(T(0), T(0));
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (c < 2) {
#pragma unroll
      for (int r = 0; r < VL; ++r) {
        const int y = lane + 64 * r;
        xin[(c + 1) & 1][r] = y < ny ? Ap[(size_t)y * 3 + c + 1] : mk(T(0), T(0));
      }
    }
    wfft_forward<T, VL, HALF>(xin[c & 1], F[c], tbuf, twy, lane);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (lane < NG) {
    cx<T>* Bk = B + (size_t)kx * n * nz * 3;
#pragma unroll
    for (int d = 0; d < 8; ++d) {
      cx<T>* p = Bk + ((size_t)wfft_freq<VL>(lane, d) * nz + z) * 3;
      p[0] = F[0][d];
      p[1] = F[1][d];
      p[2] = F[2][d];
    }
  }
}

template <typename T, int VL, bool HALF>
__global__ void __launch_bounds__(64 * kY3Waves)
k_y3_fwd(const cx<T>* __restrict__ A, cx<T>* __restrict__ B, int nz, int ny, int nzb,
         const cx<T>* __restrict__ twy, const int* __restrict__ done) {
  y3_fwd_body<T, VL, HALF>(A, B, nz, ny, nzb, twy, done, xcd_remap(blockIdx.x, gridDim.x));
}

// Logical block L of the inverse y pass.
template <typename T, int VL, bool HALF>
__device__ __forceinline__ void y3_inv_body(cx<T>* __restrict__ A, const cx<T>* __restrict__ B,
                                            int nz, int ny, int nzb, int M,
                                            const cx<T>* __restrict__ twy,
                                            const int* __restrict__ done, int L) {
  if (done != nullptr && *done != 0) return;
  constexpr int n = 64 * VL;
  constexpr int NG = 8 * VL;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = thread_index();
  const int lane = tid & 63, w = tid >> 6;
  const int kx = L / nzb;
  const int z = (L - kx * nzb) * kY3Waves + w;
  if (z >= nz) return;
  cx<T>* tbuf = reinterpret_cast<cx<T>*>(smem) + w * wfft_buf<VL, HALF>();
  cx<T> F[3][8];
  if (lane < NG) {
    const cx<T>* Bk = B + (size_t)kx * n * nz * 3;
#pragma unroll
    for (int d = 0; d < 8; ++d) {
      const cx<T>* p = Bk + ((size_t)wfft_freq<VL>(lane, d) * nz + z) * 3;
      F[0][d] = p[0];
      F[1][d] = p[1];
      F[2][d] = p[2];
    }
  }
  const bool real_col = (kx == 0 || kx == M);
  cx<T>* Ap = A + ((size_t)kx * nz + z) * ny * 3;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cx<T> xo[VL];
    wfft_inverse<T, VL, HALF>(F[c], xo, tbuf, twy, lane);
#pragma unroll
    for (int r = 0; r < VL; ++r) {
      const int y = lane + 64 * r;
      if (y < ny) Ap[(size_t)y * 3 + c] = real_col ? mk(xo[r].x, T(0)) : xo[r];
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <typename T, int VL, bool HALF>
__global__ void __launch_bounds__(64 * kY3Waves)
k_y3_inv(cx<T>* __restrict__ A, const cx<T>* __restrict__ B, int nz, int ny, int nzb, int M,
         const cx<T>* __restrict__ twy, const int* __restrict__ done) {
  y3_inv_body<T, VL, HALF>(A, B, nz, ny, nzb, M, twy, done, xcd_remap(blockIdx.x, gridDim.x));
}

// Logical block L of the z pass with the tensor product (pencils 4 L .. 4 L + 3).
template <typename T, int VL, bool HALF>
__device__ __forceinline__ void z3_body(cx<T>* __restrict__ B, int nz, int Py,
                                        const T* __restrict__ T3, int rstride, T scale,
                                        const cx<T>* __restrict__ twz,
                                        const int* __restrict__ done, int L) {
  if (done != nullptr && *done != 0) return;
  constexpr int n = 64 * VL;
  constexpr int NG = 8 * VL;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = thread_index();
  const int lane = tid & 63, w = tid >> 6;
  const int pen = L * kZ3Waves + w;           // pencil index kx * Py + ky
  const int kx = pen / Py;
  const int ky = pen - kx * Py;
  cx<T>* tbuf = reinterpret_cast<cx<T>*>(smem) + w * wfft_buf<VL, HALF>();
  cx<T>* P = B + (size_t)pen * nz * 3;
  cx<T> F[3][8];
  cx<T> xin[2][VL];
#pragma unroll
  for (int r = 0; r < VL; ++r) {
    const int z = lane + 64 * r;
    xin[0][r] = z < nz ? P[(size_t)z * 3] : mk(T(0), T(0));
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (c < 2) {
#pragma unroll
      for (int r = 0; r < VL; ++r) {
        const int z = lane + 64 * r;
        xin[(c + 1) & 1][r] = z < nz ? P[(size_t)z * 3 + c + 1] : mk(T(0), T(0));
      }
    }
    wfft_forward<T, VL, HALF>(xin[c & 1], F[c], tbuf, twz, lane);
    __builtin_amdgcn_sched_barrier(0);
  }
  const int hy = Py >> 1;
  const bool ny_neg = ky > hy;
  const int kyp = ny_neg ? Py - ky : ky;
  const T sy = ny_neg ? T(-1) : T(1);
  const T* trow = T3 + ((size_t)kx * (hy + 1) + kyp) * rstride;
  if (lane < NG) {
#pragma unroll
    for (int d = 0; d < 8; ++d) {
      const int kz = wfft_freq<VL>(lane, d);
      const bool nz_neg = kz > n / 2;
      const int kzp = nz_neg ? n - kz : kz;
      const T sz = nz_neg ? T(-1) : T(1);
      const T* t = trow + kzp * 6;
      const T xx = t[0], yy = t[1], zz = t[2];
      const T xy = t[3] * sy, xz = t[4] * sz, yz = t[5] * (sy * sz);
      const cx<T> fx = F[0][d], fy = F[1][d], fz = F[2][d];
      F[0][d] = scl(add(add(scl(fx, xx), scl(fy, xy)), scl(fz, xz)), scale);
      F[1][d] = scl(add(add(scl(fx, xy), scl(fy, yy)), scl(fz, yz)), scale);
      F[2][d] = scl(add(add(scl(fx, xz), scl(fy, yz)), scl(fz, zz)), scale);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cx<T> xo[VL];
    wfft_inverse<T, VL, HALF>(F[c], xo, tbuf, twz, lane);
#pragma unroll
    for (int r = 0; r < VL; ++r) {
      const int z = lane + 64 * r;
      if (z < nz) P[(size_t)z * 3 + c] = xo[r];
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// FP64 up to 256 points: compiled for 3 resident waves per SIMD (168
// VGPRs, no spill; 170 and 2 waves otherwise)
template <typename T, int VL, bool HALF>
__global__ void __launch_bounds__(64 * kZ3Waves, (sizeof(T) == 8 && VL <= 4 ? 3 : 1))
k_z3(cx<T>* __restrict__ B, int nz, int Py, const T* __restrict__ T3, int rstride, T scale,
     const cx<T>* __restrict__ twz, const int* __restrict__ done) {
  z3_body<T, VL, HALF>(B, nz, Py, T3, rstride, scale, twz, done,
                       xcd_remap(blockIdx.x, gridDim.x));
}

// ---- persistent batched 3-D stages -----------------------------------------------
// One launch per stage covers the blocks of every 3-D sample of the batch,
// whatever its padded lengths (64, 128, 256 or 512): static shares of an
// XCD-ordered table (persist_loop), a branch on the item's length.
static_assert(kY3Waves == kZ3Waves, "the 3-D stages share one block size");

template <typename T, int VL>
__device__ __forceinline__ void w3_item(int stage, const BatchDesc& d, int L) {
  constexpr bool HALF = k3dHalf;
  const int nzb = (d.nz + kY3Waves - 1) / kY3Waves;
  if (stage < 0)
    y3_fwd_body<T, VL, HALF>((const cx<T>*)d.spec, (cx<T>*)d.B, d.nz, d.ny, nzb,
                             (const cx<T>*)d.twy, &d.st->done, L);
  else if (stage > 0)
    y3_inv_body<T, VL, HALF>((cx<T>*)d.spec, (const cx<T>*)d.B, d.nz, d.ny, nzb, d.M,
                             (const cx<T>*)d.twy, &d.st->done, L);
  else
    z3_body<T, VL, HALF>((cx<T>*)d.B, d.nz, d.Py, (const T*)d.Tt, d.tstride, (T)d.scale,
                         (const cx<T>*)d.twz, &d.st->done, L);
}

template <typename T, int STAGE>
__global__ void __launch_bounds__(64 * kY3Waves)
k_w3_p(const BatchDesc* __restrict__ descs, const WorkItem* __restrict__ items, int n_items) {
  persist_loop(n_items, [&](int v) {
    const WorkItem it = items[v];
    const BatchDesc& d = descs[it.sample];
    switch ((STAGE == 0 ? d.Pz : d.Py) >> 6) {
      case 1: w3_item<T, 1>(STAGE, d, it.block); break;
      case 2: w3_item<T, 2>(STAGE, d, it.block); break;
      case 4: w3_item<T, 4>(STAGE, d, it.block); break;
      case 8: w3_item<T, 8>(STAGE, d, it.block); break;
      default: break;
    }
  });
}

// ---------------------------------------------------------------------------
template <typename K>
static void set_lds(K kernel, size_t bytes) {
  if (bytes > 48 * 1024)
    (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)bytes);
}

template <typename T, int VL>
static void y3_dispatch(hipStream_t s, void* A, void* B, int nz, int ny, int M, int dir,
                        const void* twy, const int* done) {
  constexpr bool HALF = k3dHalf;
  const size_t lds = (size_t)kY3Waves * wfft_buf<VL, HALF>() * sizeof(cx<T>);
  const int nzb = (nz + kY3Waves - 1) / kY3Waves;
  const dim3 grid((unsigned)((M + 1) * nzb));
  if (dir < 0) {
    auto k = k_y3_fwd<T, VL, HALF>;
    set_lds(k, lds);
    hipLaunchKernelGGL(k, grid, dim3(64 * kY3Waves), lds, s, (const cx<T>*)A, (cx<T>*)B, nz, ny,
                       nzb, (const cx<T>*)twy, done);
  } else {
    auto k = k_y3_inv<T, VL, HALF>;
    set_lds(k, lds);
    hipLaunchKernelGGL(k, grid, dim3(64 * kY3Waves), lds, s, (cx<T>*)A, (const cx<T>*)B, nz, ny,
                       nzb, M, (const cx<T>*)twy, done);
  }
}

template <typename T>
void launch_y3(hipStream_t s, void* A, void* B, int nz, int ny, int Py, int M, int dir,
               const void* twy, const int* done) {
  switch (Py) {
    case 64: y3_dispatch<T, 1>(s, A, B, nz, ny, M, dir, twy, done); break;
    case 128: y3_dispatch<T, 2>(s, A, B, nz, ny, M, dir, twy, done); break;
    case 256: y3_dispatch<T, 4>(s, A, B, nz, ny, M, dir, twy, done); break;
    default: y3_dispatch<T, 8>(s, A, B, nz, ny, M, dir, twy, done); break;
  }
}

template <typename T, int VL>
static void z3_dispatch(hipStream_t s, void* B, int nz, int Py, int M, const T* T3, int rstride,
                        T scale, const void* twz, const int* done) {
  constexpr bool HALF = k3dHalf;
  const size_t lds = (size_t)kZ3Waves * wfft_buf<VL, HALF>() * sizeof(cx<T>);
  // Py is a multiple of kZ3Waves, so every wave of the grid owns a pencil
  const dim3 grid((unsigned)((long long)(M + 1) * Py / kZ3Waves));
  auto k = k_z3<T, VL, HALF>;
  set_lds(k, lds);
  hipLaunchKernelGGL(k, grid, dim3(64 * kZ3Waves), lds, s, (cx<T>*)B, nz, Py, T3, rstride, scale,
                     (const cx<T>*)twz, done);
}

template <typename T>
void launch_z3(hipStream_t s, void* B, int nz, int Py, int Pz, int M, const T* T3, int rstride,
               T scale, const void* twz, const int* done) {
  switch (Pz) {
    case 64: z3_dispatch<T, 1>(s, B, nz, Py, M, T3, rstride, scale, twz, done); break;
    case 128: z3_dispatch<T, 2>(s, B, nz, Py, M, T3, rstride, scale, twz, done); break;
    case 256: z3_dispatch<T, 4>(s, B, nz, Py, M, T3, rstride, scale, twz, done); break;
    default: z3_dispatch<T, 8>(s, B, nz, Py, M, T3, rstride, scale, twz, done); break;
  }
}

int y3_blocks(int nz, int M) { return (M + 1) * ((nz + kY3Waves - 1) / kY3Waves); }
int z3_blocks(int Py, int M) { return (M + 1) * (Py / kZ3Waves); }

template <typename T, int VL>
static size_t w3_lds() {
  constexpr bool HALF = k3dHalf;
  return (size_t)kY3Waves * wfft_buf<VL, HALF>() * sizeof(cx<T>);
}

size_t w3_block_lds(bool single, int P) {
  switch (P) {
    case 64: return single ? w3_lds<float, 1>() : w3_lds<double, 1>();
    case 128: return single ? w3_lds<float, 2>() : w3_lds<double, 2>();
    case 256: return single ? w3_lds<float, 4>() : w3_lds<double, 4>();
    default: return single ? w3_lds<float, 8>() : w3_lds<double, 8>();
  }
}

template <typename T>
static const void* w3_kernel(int stage) {
  return stage < 0 ? (const void*)k_w3_p<T, -1>
                   : (stage > 0 ? (const void*)k_w3_p<T, 1> : (const void*)k_w3_p<T, 0>);
}

int w3_persistent_grid(bool single, int stage, size_t lds) {
  const void* k = single ? w3_kernel<float>(stage) : w3_kernel<double>(stage);
  if (lds > 48 * 1024) (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 64 * kY3Waves, lds) != hipSuccess ||
      hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    return 8;
  }
  const int g = per_cu * cus / 8 * 8;
  return g < 8 ? 8 : g;
}

template <typename T>
void launch_3d_persistent(hipStream_t s, int stage, const BatchDesc* descs, const WorkItem* items,
                          int n_items, size_t lds, int grid) {
  const int g = n_items < grid ? n_items : grid;
  if (g <= 0) return;
  const void* k = w3_kernel<T>(stage);
  if (lds > 48 * 1024) (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  void* args[] = {(void*)&descs, (void*)&items, (void*)&n_items};
  (void)hipLaunchKernel(k, dim3(g), dim3(64 * kY3Waves), args, lds, s);
}

template void launch_3d_persistent<double>(hipStream_t, int, const BatchDesc*, const WorkItem*, int,
                                           size_t, int);
template void launch_3d_persistent<float>(hipStream_t, int, const BatchDesc*, const WorkItem*, int,
                                          size_t, int);
template void launch_y3<double>(hipStream_t, void*, void*, int, int, int, int, int, const void*,
                                const int*);
template void launch_y3<float>(hipStream_t, void*, void*, int, int, int, int, int, const void*,
                               const int*);
template void launch_z3<double>(hipStream_t, void*, int, int, int, int, const double*, int, double,
                                const void*, const int*);
template void launch_z3<float>(hipStream_t, void*, int, int, int, int, const float*, int, float,
                               const void*, const int*);

}  // namespace mmk
