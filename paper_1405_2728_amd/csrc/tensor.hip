// Demagnetisation tensor of the regular cuboid grid, computed on the device
// in double precision once per geometry.
//
// N_ab(R) is the average over target and source cell of the point-dipole
// kernel, H_d,i = -Ms sum_j N(r_i - r_j) m_j:
//   N_ab(R) = -1/(4 pi V) Int_{[-d,d]^3} (3 u_a u_b - delta_ab u^2)/u^5
//             prod_c (d_c - |t_c|) dt,   u = R + t.
// Near field (|R| < 6 h, h the largest cell edge): closed form of Newell,
// Williams and Dunlop (J. Geophys. Res. 98, 9551 (1993)), the 27-point second
// difference of their functions f (diagonal) and g (off-diagonal).
// Far field: Gauss-Legendre quadrature of the integral above with every axis
// split at t = 0 (the kink of the tent weight): 6 points per half-axis below
// 16 h, 4 below 40 h, 3 beyond.
//
// Only the octant of non-negative offsets is computed; the other octants
// follow from the parities (xy odd in X and Y, xz odd in X and Z, yz odd in
// Y and Z, diagonal even).
#include "mm_device.h"
#include "mm_kernels.h"

namespace mmk {

__device__ double newell_f(double x, double y, double z) {
  x = fabs(x);
  y = fabs(y);
  z = fabs(z);
  const double x2 = x * x, y2 = y * y, z2 = z * z;
  const double R = sqrt(x2 + y2 + z2);
  double r = (2.0 * x2 - y2 - z2) * R / 6.0;
  const double xz2 = x2 + z2, xy2 = x2 + y2;
  if (xz2 > 0.0) r += 0.5 * y * (z2 - x2) * asinh(y / sqrt(xz2));
  if (xy2 > 0.0) r += 0.5 * z * (y2 - x2) * asinh(z / sqrt(xy2));
  if (x * R > 0.0) r -= x * y * z * atan(y * z / (x * R));
  return r;
}

__device__ double newell_g(double x, double y, double z) {
  const double sgn = (x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0)) * (y > 0.0 ? 1.0 : (y < 0.0 ? -1.0 : 0.0));
  if (sgn == 0.0) return 0.0;
  x = fabs(x);
  y = fabs(y);
  z = fabs(z);
  const double x2 = x * x, y2 = y * y, z2 = z * z;
  const double R = sqrt(x2 + y2 + z2);
  double r = -x * y * R / 3.0;
  const double xy2 = x2 + y2, yz2 = y2 + z2, xz2 = x2 + z2;
  if (xy2 > 0.0) r += x * y * z * asinh(z / sqrt(xy2));
  if (yz2 > 0.0) r += y / 6.0 * (3.0 * z2 - y2) * asinh(x / sqrt(yz2));
  if (xz2 > 0.0) r += x / 6.0 * (3.0 * z2 - x2) * asinh(y / sqrt(xz2));
  if (z * R > 0.0) r -= z * z * z / 6.0 * atan(x * y / (z * R));
  if (y * R > 0.0) r -= z * y2 / 2.0 * atan(x * z / (y * R));
  if (x * R > 0.0) r -= z * x2 / 2.0 * atan(y * z / (x * R));
  return sgn * r;
}

// All six entries by the closed form: sum over the 27 shifted points with
// weights c(ex) c(ey) c(ez), c(0) = 2, c(+-1) = -1.
__device__ void newell_closed(double X, double Y, double Z, double dx, double dy, double dz,
                              double out[6]) {
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int ex = -1; ex <= 1; ++ex) {
    const double a = X + ex * dx;
    const double cxw = ex == 0 ? 2.0 : -1.0;
    for (int ey = -1; ey <= 1; ++ey) {
      const double b = Y + ey * dy;
      const double cyw = ey == 0 ? 2.0 : -1.0;
      for (int ez = -1; ez <= 1; ++ez) {
        const double c = Z + ez * dz;
        const double w = cxw * cyw * (ez == 0 ? 2.0 : -1.0);
        acc[0] += w * newell_f(a, b, c);
        acc[1] += w * newell_f(b, a, c);
        acc[2] += w * newell_f(c, b, a);
        acc[3] += w * newell_g(a, b, c);
        acc[4] += w * newell_g(a, c, b);
        acc[5] += w * newell_g(b, c, a);
      }
    }
  }
  const double k = 1.0 / (4.0 * 3.14159265358979323846 * dx * dy * dz);
  for (int i = 0; i < 6; ++i) out[i] = acc[i] * k;
}

template <int NP>
__device__ void far_quadrature(double X, double Y, double Z, double dx, double dy, double dz,
                               const double* xi, const double* wi, double out[6]) {
  // nodes and tent-weighted weights per axis, both halves
  double tx[2 * NP], wx[2 * NP], ty[2 * NP], wy[2 * NP], tz[2 * NP], wz[2 * NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const double hx = 0.5 * dx * (xi[q] + 1.0), hy = 0.5 * dy * (xi[q] + 1.0),
                 hz = 0.5 * dz * (xi[q] + 1.0);
    tx[q] = hx; tx[q + NP] = -hx;
    ty[q] = hy; ty[q + NP] = -hy;
    tz[q] = hz; tz[q + NP] = -hz;
    wx[q] = wx[q + NP] = 0.5 * dx * wi[q] * (dx - hx);
    wy[q] = wy[q + NP] = 0.5 * dy * wi[q] * (dy - hy);
    wz[q] = wz[q + NP] = 0.5 * dz * wi[q] * (dz - hz);
  }
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int a = 0; a < 2 * NP; ++a) {
    const double ux = X + tx[a];
    for (int b = 0; b < 2 * NP; ++b) {
      const double uy = Y + ty[b];
      const double wab = wx[a] * wy[b];
      for (int c = 0; c < 2 * NP; ++c) {
        const double uz = Z + tz[c];
        const double r2 = ux * ux + uy * uy + uz * uz;
        const double inv5 = 1.0 / (r2 * r2 * sqrt(r2));
        const double w = wab * wz[c] * inv5;
        acc[0] += w * (3.0 * ux * ux - r2);
        acc[1] += w * (3.0 * uy * uy - r2);
        acc[2] += w * (3.0 * uz * uz - r2);
        acc[3] += w * (3.0 * ux * uy);
        acc[4] += w * (3.0 * ux * uz);
        acc[5] += w * (3.0 * uy * uz);
      }
    }
  }
  const double k = -1.0 / (4.0 * 3.14159265358979323846 * dx * dy * dz);
  for (int i = 0; i < 6; ++i) out[i] = acc[i] * k;
}

__global__ void k_newell_octant(double* __restrict__ out, int nx, int ny, int nz, double dx,
                                double dy, double dz, GaussRules gr) {
  const long long n = (long long)nx * ny * nz;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int i = (int)(idx % nx);
  const int j = (int)((idx / nx) % ny);
  const int k = (int)(idx / ((long long)nx * ny));
  const double X = i * dx, Y = j * dy, Z = k * dz;
  const double h = fmax(dx, fmax(dy, dz));
  const double r2 = X * X + Y * Y + Z * Z;
  double v[6];
  if (r2 < 36.0 * h * h) newell_closed(X, Y, Z, dx, dy, dz, v);
  else if (r2 < 256.0 * h * h) far_quadrature<6>(X, Y, Z, dx, dy, dz, gr.x6, gr.w6, v);
  else if (r2 < 1600.0 * h * h) far_quadrature<4>(X, Y, Z, dx, dy, dz, gr.x4, gr.w4, v);
  else far_quadrature<3>(X, Y, Z, dx, dy, dz, gr.x3, gr.w3, v);
  for (int c = 0; c < 6; ++c) out[(size_t)c * n + idx] = v[c];
}

// Embed the octant with wrap-around into real planes E[6][nz][Py][Px] for
// the transforms along x and y (z stays direct: dz >= 0 planes only).
__global__ void k_embed_thin(const double* __restrict__ oct, double* __restrict__ E, int nx, int ny,
                             int nz, int Px, int Py) {
  const long long total = 6LL * nz * Py * Px;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int ii = (int)(idx % Px);
  const int jj = (int)((idx / Px) % Py);
  const int k = (int)((idx / ((long long)Px * Py)) % nz);
  const int c = (int)(idx / ((long long)Px * Py * nz));
  int i = -1, j = -1;
  bool negx = false, negy = false;
  if (ii < nx) i = ii;
  else if (ii > Px - nx) { i = Px - ii; negx = true; }
  if (jj < ny) j = jj;
  else if (jj > Py - ny) { j = Py - jj; negy = true; }
  double v = 0.0;
  if (i >= 0 && j >= 0) {
    v = oct[(size_t)c * nx * ny * nz + ((size_t)k * ny + j) * nx + i];
    const bool oddx = (c == 3 || c == 4);
    const bool oddy = (c == 3 || c == 5);
    if ((negx && oddx) != (negy && oddy)) v = -v;
  }
  E[idx] = v;
}

// EXY[kx][c][k][ky] (complex, after x and y transforms) -> Tt[kx][k][ky'][c]
// for ky' <= Py/2: real part of the even-even / odd-odd entries, imaginary
// part of xz and yz (odd in exactly one transformed axis).
template <typename T>
__global__ void k_extract_thin(const cx<double>* __restrict__ EXY, T* __restrict__ Tt, int M,
                               int nz, int Py, int tstride) {
  const int nk = Py / 2 + 1;
  const long long total = (long long)(M + 1) * nz * nk * 6;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int c = (int)(idx % 6);
  const int ky = (int)((idx / 6) % nk);
  const int k = (int)((idx / (6LL * nk)) % nz);
  const int kx = (int)(idx / (6LL * nk * nz));
  const cx<double> v = EXY[(((size_t)kx * 6 + c) * nz + k) * Py + ky];
  // xy and xz are odd in X: their transforms vanish at kx = 0 and kx = M
  const bool zero = (kx == 0 || kx == M) && (c == 3 || c == 4);
  Tt[(size_t)kx * tstride + (idx - (long long)kx * nz * nk * 6)] = zero ? T(0) : (T)(c < 4 ? v.x : v.y);
}

// ---- full 3-D transform of the tensor (grids with more than 4 layers) ------
// Embed with wrap-around in x, y and z: E[6][Pz][Py][Px].
__global__ void k_embed_3d(const double* __restrict__ oct, double* __restrict__ E, int nx, int ny,
                           int nz, int Px, int Py, int Pz) {
  const long long total = 6LL * Pz * Py * Px;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int ii = (int)(idx % Px);
  const int jj = (int)((idx / Px) % Py);
  const int kk = (int)((idx / ((long long)Px * Py)) % Pz);
  const int c = (int)(idx / ((long long)Px * Py * Pz));
  int i = -1, j = -1, k = -1;
  bool nx_ = false, ny_ = false, nz_ = false;
  if (ii < nx) i = ii;
  else if (ii > Px - nx) { i = Px - ii; nx_ = true; }
  if (jj < ny) j = jj;
  else if (jj > Py - ny) { j = Py - jj; ny_ = true; }
  if (kk < nz) k = kk;
  else if (kk > Pz - nz) { k = Pz - kk; nz_ = true; }
  double v = 0.0;
  if (i >= 0 && j >= 0 && k >= 0) {
    v = oct[(size_t)c * nx * ny * nz + ((size_t)k * ny + j) * nx + i];
    const bool ox = (c == 3 || c == 4), oy = (c == 3 || c == 5), oz = (c == 4 || c == 5);
    const int flips = (nx_ && ox) + (ny_ && oy) + (nz_ && oz);
    if (flips & 1) v = -v;
  }
  E[idx] = v;
}

// Per (kx, c) plane: [rows][cols] -> [cols][rows] (complex double), 16 x 16
// tiles, one block per tile (1-D grid: plane-major).
__global__ void k_transpose_planes(const cx<double>* __restrict__ in, cx<double>* __restrict__ out,
                                   int rows, int cols, int tiles_r, int tiles_c) {
  __shared__ cx<double> tile[16][17];
  const int tpp = tiles_r * tiles_c;
  const long long p = blockIdx.x / tpp;
  const int t = (int)(blockIdx.x - p * tpp);
  const int r0 = (t / tiles_c) * 16, c0 = (t % tiles_c) * 16;
  const cx<double>* src = in + (size_t)p * rows * cols;
  cx<double>* dst = out + (size_t)p * rows * cols;
  const int tr = threadIdx.y, tc = threadIdx.x;
  if (r0 + tr < rows && c0 + tc < cols) tile[tr][tc] = src[(size_t)(r0 + tr) * cols + c0 + tc];
  __syncthreads();
  if (c0 + tr < cols && r0 + tc < rows) dst[(size_t)(c0 + tr) * rows + r0 + tc] = tile[tc][tr];
}

// EXYZ[kx][c][ky][kz] -> T3[kx][ky'][kz'][c], ky' <= Py/2, kz' <= Pz/2; rows
// of the output are padded to rstride elements.  Entries odd in an axis
// vanish exactly where that axis' frequency is 0 or Nyquist.
template <typename T>
__global__ void k_extract_3d(const cx<double>* __restrict__ E, T* __restrict__ T3, int M, int Py,
                             int Pz, int rstride) {
  const int nky = Py / 2 + 1, nkz = Pz / 2 + 1;
  const long long total = (long long)(M + 1) * nky * nkz * 6;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int c = (int)(idx % 6);
  const int kz = (int)((idx / 6) % nkz);
  const int ky = (int)((idx / (6LL * nkz)) % nky);
  const int kx = (int)(idx / (6LL * nkz * nky));
  const cx<double> v = E[(((size_t)kx * 6 + c) * Py + ky) * Pz + kz];
  const bool ox = (c == 3 || c == 4), oy = (c == 3 || c == 5), oz = (c == 4 || c == 5);
  const bool zero = (ox && (kx == 0 || kx == M)) || (oy && (ky == 0 || ky == Py / 2)) ||
                    (oz && (kz == 0 || kz == Pz / 2));
  T3[((size_t)kx * nky + ky) * rstride + (size_t)kz * 6 + c] = zero ? T(0) : (T)v.x;
}

void launch_embed_3d(hipStream_t s, const double* oct, double* E, int nx, int ny, int nz, int Px,
                     int Py, int Pz) {
  const long long total = 6LL * Pz * Py * Px;
  hipLaunchKernelGGL(k_embed_3d, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, oct, E,
                     nx, ny, nz, Px, Py, Pz);
}

void launch_transpose_planes(hipStream_t s, const void* in, void* out, int rows, int cols,
                             int nplanes) {
  const int tr = (rows + 15) / 16, tc = (cols + 15) / 16;
  const dim3 grid((unsigned)((long long)nplanes * tr * tc));
  hipLaunchKernelGGL(k_transpose_planes, grid, dim3(16, 16), 0, s, (const cx<double>*)in,
                     (cx<double>*)out, rows, cols, tr, tc);
}

template <typename T>
void launch_extract_3d(hipStream_t s, const void* E, T* T3, int M, int Py, int Pz, int rstride) {
  const long long total = (long long)(M + 1) * (Py / 2 + 1) * (Pz / 2 + 1) * 6;
  hipLaunchKernelGGL(k_extract_3d<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     (const cx<double>*)E, T3, M, Py, Pz, rstride);
}

template void launch_extract_3d<double>(hipStream_t, const void*, double*, int, int, int, int);
template void launch_extract_3d<float>(hipStream_t, const void*, float*, int, int, int, int);

void launch_newell_octant(hipStream_t s, double* out, int nx, int ny, int nz, double dx, double dy,
                          double dz, const GaussRules& gr) {
  const long long n = (long long)nx * ny * nz;
  hipLaunchKernelGGL(k_newell_octant, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, out, nx,
                     ny, nz, dx, dy, dz, gr);
}

void launch_embed_thin(hipStream_t s, const double* oct, double* E, int nx, int ny, int nz, int Px,
                       int Py) {
  const long long total = 6LL * nz * Py * Px;
  hipLaunchKernelGGL(k_embed_thin, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, oct, E,
                     nx, ny, nz, Px, Py);
}

template <typename T>
void launch_extract_thin(hipStream_t s, const void* EXY, T* Tt, int M, int nz, int Py, int tstride) {
  const long long total = (long long)(M + 1) * nz * (Py / 2 + 1) * 6;
  hipLaunchKernelGGL(k_extract_thin<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     (const cx<double>*)EXY, Tt, M, nz, Py, tstride);
}

template void launch_extract_thin<double>(hipStream_t, const void*, double*, int, int, int, int);
template void launch_extract_thin<float>(hipStream_t, const void*, float*, int, int, int, int);

}  // namespace mmk
