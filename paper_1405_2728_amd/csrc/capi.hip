// C ABI of the minimiser library: contexts, samples, the evaluation and
// iteration sequences, polling, sweeps, timing.  See include/mm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/mm.h"
#include "mm_kernels.h"

using namespace mmk;

namespace {

constexpr int kNumKernels = 9;
// xf: pending update + forward x FFT; yz_thin: y FFT, tensor product with the
// z convolution, inverse y FFT (grids of at most 4 layers); xil: inverse x
// FFT + local terms + sums + step choice; update: stand-alone update
// (single-step calls only); y3_fwd, z3, y3_inv: y FFT, z FFT with tensor
// product and inverse, inverse y FFT (full 3-D path); finish: reduction of
// the per-block sums, stop rule and step choice; reference: the whole
// double-precision reference pass of the single-precision form
const char* const kKernelNames[kNumKernels] = {"xf",     "yz_thin", "xil",    "update",   "y3_fwd",
                                               "z3",     "y3_inv",  "finish", "reference"};
enum { KID_XF = 0, KID_YZ = 1, KID_XIL = 2, KID_UPDATE = 3, KID_Y3F = 4, KID_Z3 = 5, KID_Y3I = 6,
       KID_FINISH = 7, KID_REF = 8 };

// demag path of a geometry
enum { PATH_NONE = 0, PATH_THIN = 1, PATH_3D = 2 };

struct Sample {
  bool has_geom = false, has_mat = false;
  int dev = -1;               // device that was current at mm_set_geometry
  int nx = 0, ny = 0, nz = 0, N = 0;
  double dx = 0, dy = 0, dz = 0, V = 0;
  int path = PATH_NONE;
  int Px = 0, Py = 0, Pz = 1, M = 0, R3 = 1, nb3 = 0, tstride = 0;
  int yz_var = 0;             // occupancy variant of the thin yz wave kernel (tile tuner)
  double Ms = 0, A = 0, Ku = 0, u[3] = {1, 0, 0}, H[3] = {0, 0, 0};
  double* ku_map = nullptr;
  void* Tt = nullptr;
  void* spec = nullptr;
  void* twx = nullptr;
  void* twy = nullptr;
  void* twz = nullptr;
  void* B = nullptr;          // 3-D path: spectrum after the y transform
  double* Hd = nullptr;
  // g_k and s_k = m_{k+1} - m_k in the transform type of the context
  // (gs_bytes per value): they feed only the step direction and the BB sums
  void* g = nullptr;
  void* s = nullptr;
  double* partials = nullptr;
  int nblk = 0;
  MinState* st = nullptr;
  MinState* st_eval = nullptr;
  MinState* st_host = nullptr;
  double* dev3 = nullptr;
  double* host3 = nullptr;
  // derivative workspace (allocated on first use): H_eff(m), H_lin[v], CG vectors
  double* Hm = nullptr;
  double* Hlin = nullptr;
  double* cr = nullptr;
  double* cp = nullptr;
  double* cAp = nullptr;
  CGState* cg = nullptr;
  CGState* cg_host = nullptr;
  double* scal = nullptr;
  double* scal_host = nullptr;
  // double-precision reference of the single-precision form (defect
  // correction): the iteration transforms m - mref in single precision and
  // adds hdref = H_d(mref), computed in double precision with its own
  // tensor, spectrum and twiddles every poll_every iterations
  bool has_ref = false;
  void* rTt = nullptr;
  void* rspec = nullptr;
  void* rtwx = nullptr;
  void* rtwy = nullptr;
  void* rtwz = nullptr;
  void* rB = nullptr;
  int rtstride = 0, rR3 = 1;
  double* mref = nullptr;
  double* hdref = nullptr;
  long long ref_age = 0;      // iterations since the last reference pass
  bool fin_pending = false;   // the last inverse pass's sums await their finish
  // line search: saved base state and the trial's gradient (on first use)
  double* ls_mbase = nullptr;
  void* ls_g2 = nullptr;      // transform type, like g
  // captured batch of poll_every minimiser iterations (use_graph), valid for
  // the m buffer, batch length, correction flag and material it was made with
  hipGraphExec_t it_graph = nullptr;
  const double* it_graph_m = nullptr;
  int it_graph_n = 0, it_graph_ref = 0, it_graph_mat = -1, it_graph_ls = 0, it_graph_fuse = 0;
  int mat_version = 0;
  int64_t evals_total = 0, iters_total = 0;
};

constexpr long long kRefStale = 1LL << 60;

struct ProfRec {
  int id;
  hipEvent_t a, b;
};

}  // namespace

struct mm_ctx {
  int prec = MM_FP64;
  hipStream_t stream = nullptr;
  std::vector<Sample> smp;
  std::string err;
  double tau0 = 0.0;
  int poll_every = 32;
  long long stall_iters = 500;
  double bb_switch = 0.0;       // step choice: 0 alternation of eq. (12); kappa > 0 ratio switch
  LineSearch ls = {0, 0.85, 1e-4, 0.5, 30};   // non-monotone line search (off by default)
  int use_graph = 0;
  int batched = 1;              // sweeps of several samples share launches
  int path_pref = 0;            // 0 automatic, 1 thin-film, 2 full 3-D
  int refine = 1;               // single-precision form: defect correction on
  int autotune = 0;             // 1: time the x-pass tiles at mm_set_geometry
  int rows_forced = 0;          // > 0: rows per block of the x passes (tests)
  int yz_forced = -1;           // >= 0: occupancy variant of the thin yz pass (tests)
  int mixed_radix = 1;          // 1: wave lengths 64 VL (VL = 3, 5, 6, 7) where shorter
  int concurrent_groups = 1;    // batched passes: launch groups on forked streams
  double batch_rebuild = 0.75;  // batched sweeps: rebuild the tables once the running
                                // samples are at most this fraction of the plan's (0: never)
  int persistent = 1;           // batched passes: one persistent launch per pass (per
                                // layer count for yz); 0: one launch per group of
                                // equal transform lengths
  int fused_finish = 1;         // single-sample runs: the next forward x pass takes each
                                // iteration's finish over (0: a finish kernel each)
  int fin_spin = kFinSpin;      // polls before a block waiting for that decision gives up
  // auxiliary streams (default priority) and fork/join events of the
  // batched passes, made on first use
  std::vector<hipStream_t> aux;
  hipEvent_t fork_ev = nullptr;
  std::vector<hipEvent_t> join_ev;
  unsigned prof = 0;            // bit k: time kernel k with events
  std::vector<ProfRec> prof_pending;
  std::vector<hipEvent_t> ev_pool;
  double prof_ms[kNumKernels] = {0};
  int64_t prof_n[kNumKernels] = {0};
};

namespace {

bool single(const mm_ctx* c) { return c->prec == MM_MIXED; }
// bytes per value of the g and s streams (the transform type)
size_t gs_bytes(const mm_ctx* c) { return single(c) ? sizeof(float) : sizeof(double); }
template <typename T>
T* as(void* p) {
  return static_cast<T*>(p);
}

int fail(mm_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(ctx, expr)                                                              \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail((ctx), MM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

int next_pow2(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

// Padded lengths >= 2n - 1: powers of two, except that with mixed radix
// the wave FFT lengths 64 VL (VL = 3, 5, 6, 7) replace the power of two
// where they are shorter: x Px = 128 VL (half-length transform 64 VL) for
// 2nx - 1 up to 1024, thin-film y Py = 64 VL for 2ny - 1 up to 512.
int pad_wave(int n, int unit, bool mr) {
  const int p = next_pow2(n);
  if (!mr || n > 8 * unit) return p;
  const int w = (n + unit - 1) / unit * unit;
  return w < p ? w : p;
}
int pad_x(int nx, bool mr) { return nx < 2 ? 2 : pad_wave(2 * nx - 1, 128, mr); }
int pad_thin_y(int ny, bool mr) { return pad_wave(2 * ny - 1, 64, mr); }
int pad_3d(int n) {
  const int p = next_pow2(2 * n - 1);
  return p < 64 ? 64 : p;
}

// Demag path for a grid: the thin-film path for at most 4 layers (unless the
// full 3-D path is asked for), the full 3-D path otherwise.
int choose_path(int prec, int pref, int nx, int ny, int nz, bool mr = true) {
  if (nx < 1 || ny < 1 || nz < 1) return PATH_NONE;
  if (nx > (1 << 14) || ny > (1 << 13)) return PATH_NONE;
  // the fused x passes hold the three components of a row in one block:
  // 3 M complex values within 512 threads x 16 values and the LDS
  const long long xv = 3LL * (pad_x(nx, mr) / 2);
  if (xv > 512LL * 16 || xv * (prec == MM_MIXED ? 8 : 16) > 160LL * 1024) return PATH_NONE;
  const bool thin_ok = yz_thin_fits(nz, pad_thin_y(ny, mr), prec == MM_MIXED);
  const bool full_ok = full3d_len_ok(pad_3d(ny)) && full3d_len_ok(pad_3d(nz));
  if (pref == 1) return thin_ok ? PATH_THIN : PATH_NONE;
  if (pref == 2) return full_ok ? PATH_3D : PATH_NONE;
  if (nz <= 4) return thin_ok ? PATH_THIN : PATH_NONE;
  return full_ok ? PATH_3D : PATH_NONE;
}

template <typename P>
void dfree(P*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

void free_sample(Sample& s) {
  dfree(s.ls_mbase);
  dfree(s.ls_g2);
  dfree(s.ku_map);
  dfree(s.Tt);
  dfree(s.spec);
  dfree(s.twx);
  dfree(s.twy);
  dfree(s.twz);
  dfree(s.B);
  dfree(s.Hd);
  dfree(s.g);
  dfree(s.s);
  dfree(s.partials);
  dfree(s.st);
  dfree(s.st_eval);
  dfree(s.dev3);
  dfree(s.Hm);
  dfree(s.Hlin);
  dfree(s.cr);
  dfree(s.cp);
  dfree(s.cAp);
  dfree(s.cg);
  dfree(s.scal);
  dfree(s.rTt);
  dfree(s.rspec);
  dfree(s.rtwx);
  dfree(s.rtwy);
  dfree(s.rtwz);
  dfree(s.rB);
  dfree(s.mref);
  dfree(s.hdref);
  s.has_ref = false;
  if (s.it_graph) (void)hipGraphExecDestroy(s.it_graph);
  s.it_graph = nullptr;
  if (s.cg_host) (void)hipHostFree(s.cg_host);
  if (s.scal_host) (void)hipHostFree(s.scal_host);
  s.cg_host = nullptr;
  s.scal_host = nullptr;
  if (s.st_host) (void)hipHostFree(s.st_host);
  if (s.host3) (void)hipHostFree(s.host3);
  s.st_host = nullptr;
  s.host3 = nullptr;
  s.has_geom = false;
  s.has_mat = false;
}

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n.
void gauss_legendre(int n, double* x, double* w) {
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    double z = std::cos(pi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int j = 2; j <= n; ++j) {
        const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int j = 2; j <= n; ++j) {
      const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

int check_sample(mm_ctx* c, int sample, bool need_mat) {
  if (!c) return MM_EINVAL;
  if (sample < 0 || sample >= (int)c->smp.size())
    return fail(c, MM_EINVAL, "sample index out of range");
  const Sample& s = c->smp[sample];
  if (!s.has_geom) return fail(c, MM_ESTATE, "mm_set_geometry has not been called");
  if (need_mat && !s.has_mat) return fail(c, MM_ESTATE, "mm_set_material has not been called");
  return MM_OK;
}

// ---- timing ------------------------------------------------------------------
hipEvent_t take_event(mm_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

struct Timer {
  mm_ctx* c;
  int id;
  hipEvent_t a = nullptr;
  Timer(mm_ctx* ctx, int kid) : c(ctx), id(kid) {
    if (c->prof & (1u << kid)) {
      a = take_event(c);
      (void)hipEventRecord(a, c->stream);
    }
  }
  ~Timer() {
    if (c->prof & (1u << id)) {
      hipEvent_t b = take_event(c);
      (void)hipEventRecord(b, c->stream);
      c->prof_pending.push_back({id, a, b});
    }
  }
};

void prof_collect(mm_ctx* c) {
  if (c->prof_pending.empty()) return;
  (void)hipStreamSynchronize(c->stream);
  for (auto& r : c->prof_pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      c->prof_ms[r.id] += ms;
      c->prof_n[r.id] += 1;
    }
    c->ev_pool.push_back(r.a);
    c->ev_pool.push_back(r.b);
  }
  c->prof_pending.clear();
}

// ---- tensor set-up ---------------------------------------------------------
int build_tensor(mm_ctx* c, Sample& s) {
  hipStream_t st = c->stream;
  GaussRules gr;
  gauss_legendre(6, gr.x6, gr.w6);
  gauss_legendre(4, gr.x4, gr.w4);
  gauss_legendre(3, gr.x3, gr.w3);
  double* oct = nullptr;
  double* E = nullptr;
  void* EX = nullptr;
  void* twx64 = nullptr;
  void* twy64 = nullptr;
  const size_t n_oct = 6ull * s.N;
  const size_t n_E = 6ull * s.nz * s.Py * s.Px;
  const size_t n_EX = (size_t)(s.M + 1) * 6 * s.nz * s.Py;
  auto cleanup = [&]() {
    dfree(oct);
    dfree(E);
    dfree(EX);
    dfree(twx64);
    dfree(twy64);
  };
  if (hipMalloc((void**)&oct, n_oct * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&E, n_E * sizeof(double)) != hipSuccess ||
      hipMalloc(&EX, n_EX * 2 * sizeof(double)) != hipSuccess ||
      hipMalloc(&twx64, (size_t)s.Px * 2 * sizeof(double)) != hipSuccess ||
      hipMalloc(&twy64, (size_t)s.Py * 2 * sizeof(double)) != hipSuccess) {
    cleanup();
    return fail(c, MM_ENOMEM, "device allocation for the tensor set-up failed");
  }
  launch_twiddles(st, twx64, s.Px, false);
  launch_twiddles(st, twy64, s.Py, false);
  launch_newell_octant(st, oct, s.nx, s.ny, s.nz, s.dx, s.dy, s.dz, gr);
  launch_embed_thin(st, oct, E, s.nx, s.ny, s.nz, s.Px, s.Py);
  const int M = s.M;
  int R = 8192 / M;
  if (R > 8) R = 8;
  if (R < 1) R = 1;
  launch_fwd_x<double>(st, E, s.Px, s.Px, s.nz * s.Py, 6, s.Px, R, EX, twx64, nullptr);
  launch_fft_cols<double>(st, EX, s.Py, (M + 1) * 6 * s.nz, twy64);
  if (single(c)) launch_extract_thin<float>(st, EX, (float*)s.Tt, M, s.nz, s.Py, s.tstride);
  else launch_extract_thin<double>(st, EX, (double*)s.Tt, M, s.nz, s.Py, s.tstride);
  if (s.rTt) launch_extract_thin<double>(st, EX, (double*)s.rTt, M, s.nz, s.Py, s.rtstride);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  cleanup();
  if (e != hipSuccess) return fail(c, MM_EHIP, std::string("tensor set-up: ") + hipGetErrorString(e));
  return MM_OK;
}

// Full 3-D tensor: embed with wrap-around in x, y, z; real x transform;
// y transform; per (kx, c) plane transpose [z][ky] -> [ky][z]; z transform;
// keep the real octant ky <= Py/2, kz <= Pz/2.
int build_tensor3d(mm_ctx* c, Sample& s) {
  hipStream_t st = c->stream;
  GaussRules gr;
  gauss_legendre(6, gr.x6, gr.w6);
  gauss_legendre(4, gr.x4, gr.w4);
  gauss_legendre(3, gr.x3, gr.w3);
  double* oct = nullptr;
  double* E = nullptr;
  void* EX = nullptr;
  void* ET = nullptr;
  void* tw64[3] = {nullptr, nullptr, nullptr};
  const size_t n_oct = 6ull * s.N;
  const size_t n_E = 6ull * s.Pz * s.Py * s.Px;
  const size_t n_EX = (size_t)(s.M + 1) * 6 * s.Pz * s.Py;
  auto cleanup = [&]() {
    dfree(oct);
    dfree(E);
    dfree(EX);
    dfree(ET);
    for (auto& t : tw64) dfree(t);
  };
  if (hipMalloc((void**)&oct, n_oct * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&E, n_E * sizeof(double)) != hipSuccess ||
      hipMalloc(&EX, n_EX * 2 * sizeof(double)) != hipSuccess ||
      hipMalloc(&tw64[0], (size_t)s.Px * 2 * sizeof(double)) != hipSuccess ||
      hipMalloc(&tw64[1], (size_t)s.Py * 2 * sizeof(double)) != hipSuccess ||
      hipMalloc(&tw64[2], (size_t)s.Pz * 2 * sizeof(double)) != hipSuccess) {
    cleanup();
    (void)hipGetLastError();
    return fail(c, MM_ENOMEM, "device allocation for the tensor set-up failed");
  }
  launch_twiddles(st, tw64[0], s.Px, false);
  launch_twiddles(st, tw64[1], s.Py, false);
  launch_twiddles(st, tw64[2], s.Pz, false);
  launch_newell_octant(st, oct, s.nx, s.ny, s.nz, s.dx, s.dy, s.dz, gr);
  launch_embed_3d(st, oct, E, s.nx, s.ny, s.nz, s.Px, s.Py, s.Pz);
  const int M = s.M;
  int R = 8192 / M;
  if (R > 8) R = 8;
  if (R < 1) R = 1;
  launch_fwd_x<double>(st, E, s.Px, s.Px, s.Pz * s.Py, 6, s.Px, R, EX, tw64[0], nullptr);
  hipError_t e = hipStreamSynchronize(st);
  dfree(E);                                   // lower the peak before the transpose buffer
  dfree(oct);
  if (e == hipSuccess && hipMalloc(&ET, n_EX * 2 * sizeof(double)) != hipSuccess) {
    cleanup();
    (void)hipGetLastError();
    return fail(c, MM_ENOMEM, "device allocation for the tensor set-up failed");
  }
  if (e == hipSuccess) {
    launch_fft_cols<double>(st, EX, s.Py, (M + 1) * 6 * s.Pz, tw64[1]);       // [kx][c][z][ky]
    launch_transpose_planes(st, EX, ET, s.Pz, s.Py, (M + 1) * 6);           // [kx][c][ky][z]
    launch_fft_cols<double>(st, ET, s.Pz, (M + 1) * 6 * s.Py, tw64[2]);      // [kx][c][ky][kz]
    if (single(c)) launch_extract_3d<float>(st, ET, (float*)s.Tt, M, s.Py, s.Pz, s.tstride);
    else launch_extract_3d<double>(st, ET, (double*)s.Tt, M, s.Py, s.Pz, s.tstride);
    if (s.rTt) launch_extract_3d<double>(st, ET, (double*)s.rTt, M, s.Py, s.Pz, s.rtstride);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  cleanup();
  if (e != hipSuccess) return fail(c, MM_EHIP, std::string("tensor set-up: ") + hipGetErrorString(e));
  return MM_OK;
}

// ---- one effective-field evaluation ----------------------------------------
struct EvalOut {
  double* Hd = nullptr;       // demag output (NULL: not written)
  double* H = nullptr;        // total field
  double* Hex = nullptr;
  double* Han = nullptr;
  bool iterate = false;       // minimiser iteration: pending update, g, BB sums
  MinState* st_fin = nullptr; // state the sums are reduced into (NULL: none)
  bool zeeman = true;         // false: linear part of H_eff only (no H_ext)
  bool unit_A = false;        // exchange with A = 1 (derivative of H_ex by A)
  const int* done = nullptr;  // flag that skips the demag and local passes
  void* spec = nullptr;       // spectrum buffer in place of the sample's (NULL: its own)
  void* B = nullptr;          // 3-D path: y-transformed spectrum likewise
  int fuse_q = -1;            // >= 0: batch position of a fused-finish iteration
};

LocalArgs local_args(const Sample& s, bool unit_A = false, bool zeeman = true) {
  LocalArgs a;
  a.m = nullptr;
  a.Hd = nullptr;
  a.g = nullptr;
  a.g_out = nullptr;
  a.s = nullptr;
  a.Hout = nullptr;
  a.Hex_out = nullptr;
  a.Han_out = nullptr;
  a.ku_map = s.ku_map;
  a.nx = s.nx;
  a.ny = s.ny;
  a.nz = s.nz;
  const double pre = 2.0 * (unit_A ? 1.0 : s.A) / (kMu0Host * s.Ms);
  a.cx = pre / (s.dx * s.dx);
  a.cy = pre / (s.dy * s.dy);
  a.cz = pre / (s.dz * s.dz);
  a.ku = s.Ku;
  a.kan = 2.0 / (kMu0Host * s.Ms);
  for (int q = 0; q < 3; ++q) {
    a.u[q] = s.u[q];
    a.H[q] = zeeman ? s.H[q] : 0.0;
  }
  a.partials = s.partials;
  a.Hdyn = nullptr;
  a.Hd_add = nullptr;
  a.st = nullptr;
  a.done = nullptr;
  return a;
}

// Buffers of one convolution: the context's own precision, or the
// double-precision reference of a single-precision context.
struct Conv {
  bool sp;
  void* Tt;
  void* spec;
  void* twx;
  void* twy;
  void* twz;
  void* B;
  int tstride, R;
  int yz_var;
};

Conv conv_main(const mm_ctx* c, const Sample& s) {
  return {single(c), s.Tt, s.spec, s.twx, s.twy, s.twz, s.B, s.tstride, s.R3, s.yz_var};
}

Conv conv_ref(const Sample& s) {
  return {false, s.rTt, s.rspec, s.rtwx, s.rtwy, s.rtwz, s.rB, s.rtstride, s.rR3, 0};
}

bool use_ref(const mm_ctx* c, const Sample& s) { return single(c) && c->refine && s.has_ref; }

// Stall detection guards the plain single-precision form, whose torque has
// a floor set by the single-precision convolution; with the defect
// correction (or in double precision) there is no such floor, and BB's
// non-monotone stretches must not end a run early.
long long stall_of(const mm_ctx* c, const Sample& s) {
  return single(c) && !use_ref(c, s) ? c->stall_iters : 0;
}

// y and z stages of the convolution (between the x passes); each stage is
// timed under its own id when timed.
void enqueue_demag_mid(mm_ctx* c, const Sample& s, const Conv& v, const int* done, bool timed) {
  hipStream_t st = c->stream;
  const unsigned prof = c->prof;
  if (!timed) c->prof = 0;
  if (s.path == PATH_3D) {
    const double scale = -s.Ms / ((double)s.M * (double)s.Py * (double)s.Pz);
    {
      Timer t(c, KID_Y3F);
      if (v.sp) launch_y3<float>(st, v.spec, v.B, s.nz, s.ny, s.Py, s.M, -1, v.twy, done);
      else launch_y3<double>(st, v.spec, v.B, s.nz, s.ny, s.Py, s.M, -1, v.twy, done);
    }
    {
      Timer t(c, KID_Z3);
      if (v.sp)
        launch_z3<float>(st, v.B, s.nz, s.Py, s.Pz, s.M, (const float*)v.Tt, v.tstride,
                         (float)scale, v.twz, done);
      else
        launch_z3<double>(st, v.B, s.nz, s.Py, s.Pz, s.M, (const double*)v.Tt, v.tstride, scale,
                          v.twz, done);
    }
    {
      Timer t(c, KID_Y3I);
      if (v.sp) launch_y3<float>(st, v.spec, v.B, s.nz, s.ny, s.Py, s.M, 1, v.twy, done);
      else launch_y3<double>(st, v.spec, v.B, s.nz, s.ny, s.Py, s.M, 1, v.twy, done);
    }
  } else {
    Timer t(c, KID_YZ);
    const double scale = -s.Ms / ((double)s.M * (double)s.Py);
    if (v.sp)
      launch_yz_thin<float>(st, v.spec, s.nz, s.ny, s.Py, s.M, (const float*)v.Tt, v.tstride,
                            (float)scale, v.twy, done, v.yz_var);
    else
      launch_yz_thin<double>(st, v.spec, s.nz, s.ny, s.Py, s.M, (const double*)v.Tt, v.tstride,
                             scale, v.twy, done, v.yz_var);
  }
  c->prof = prof;
}

// The finish of the last iteration if its sums still await it (left by a
// fused-finish iteration): before anything reads the state.
void flush_finish(mm_ctx* c, Sample& s) {
  if (!s.fin_pending) return;
  s.fin_pending = false;
  Timer t(c, KID_FINISH);
  launch_finish(c->stream, s.partials, s.nb3, s.st, s.Ms, s.V);
}

// Reference pass of the defect correction: mref = m (no pending update is
// applied) and hdref = H_d(mref) in double precision.
void enqueue_reference(mm_ctx* c, Sample& s, const double* m, const MinState* mst) {
  flush_finish(c, s);
  hipStream_t st = c->stream;
  const Conv v = conv_ref(s);
  const int* done = mst ? &mst->done : nullptr;
  Timer t(c, KID_REF);
  launch_xf<double>(st, const_cast<double*>(m), (const double*)nullptr, (double*)nullptr, mst,
                    s.nx, s.ny, s.nz, s.Px, v.R, v.spec, v.twx, nullptr, s.mref);
  enqueue_demag_mid(c, s, v, done, false);
  LocalArgs a = local_args(s);
  a.m = m;
  a.done = done;
  launch_xil<double>(st, v.spec, a, s.Px, v.R, s.hdref, nullptr, v.twx);
  s.ref_age = 0;
}

// m is updated in place when o.iterate and an update is pending.  A
// minimiser iteration of a single-precision context with a reference
// transforms m - mref and adds hdref.  o.fuse_q >= 0 (an iteration at that
// position of a batch that ends with flush_finish): the forward x pass takes
// the previous iteration's finish over and this iteration's is left pending.
void enqueue_eval(mm_ctx* c, Sample& s, const double* m, const EvalOut& o) {
  if (o.fuse_q <= 0) flush_finish(c, s);
  hipStream_t st = c->stream;
  FinFuse fz{nullptr, nullptr, s.Ms, s.V, s.nb3, 0, c->fin_spin};
  if (o.fuse_q >= 0) {
    fz.st = s.st;
    fz.par = o.fuse_q & 1;
    if (o.fuse_q > 0 && s.fin_pending) fz.partials = s.partials;
    s.fin_pending = false;
  }
  MinState* mst = o.iterate ? s.st : nullptr;
  const int* done = mst ? &mst->done : o.done;
  double* mm = const_cast<double*>(m);
  Conv v = conv_main(c, s);
  if (o.spec) v.spec = o.spec;
  if (o.B) v.B = o.B;
  const bool corr = o.iterate && use_ref(c, s);
  // g and s only where the pass may apply an update (a minimiser iteration)
  void* gx = o.iterate ? s.g : nullptr;
  void* sx = o.iterate ? s.s : nullptr;
  {
    Timer t(c, KID_XF);
    if (v.sp)
      launch_xf<float>(st, mm, as<float>(gx), as<float>(sx), mst, s.nx, s.ny, s.nz, s.Px, v.R,
                       v.spec, v.twx, corr ? s.mref : nullptr, nullptr, &fz);
    else
      launch_xf<double>(st, mm, as<double>(gx), as<double>(sx), mst, s.nx, s.ny, s.nz, s.Px, v.R,
                        v.spec, v.twx, nullptr, nullptr, &fz);
  }
  enqueue_demag_mid(c, s, v, done, true);
  LocalArgs a = local_args(s, o.unit_A, o.zeeman);
  a.m = m;
  a.g = o.iterate ? s.g : nullptr;
  a.g_out = o.iterate && c->ls.on ? s.ls_g2 : nullptr;   // line search: g keeps the base's
  a.s = o.iterate ? s.s : nullptr;
  a.Hout = o.H;
  a.Hex_out = o.Hex;
  a.Han_out = o.Han;
  a.st = mst;
  a.done = done;
  a.Hdyn = mst ? mst->H : nullptr;   // the minimiser's field lives in its state
  a.Hd_add = corr ? s.hdref : nullptr;
  double* part = o.st_fin ? s.partials : nullptr;
  {
    Timer t(c, KID_XIL);
    if (v.sp)
      launch_xil<float>(st, v.spec, a, s.Px, v.R, o.Hd, part, v.twx);
    else
      launch_xil<double>(st, v.spec, a, s.Px, v.R, o.Hd, part, v.twx);
  }
  if (o.st_fin) {
    if (o.fuse_q >= 0) {
      s.fin_pending = true;
    } else {
      Timer t(c, KID_FINISH);
      launch_finish(st, s.partials, s.nb3, o.st_fin, s.Ms, s.V);
    }
  }
}

// Whether the sample's forward x pass can take the finish over: the wave
// pass, sums reduced in one stage, no line search (whose trial logic reads
// more of the state in the forward pass).
bool fuse_ok(const mm_ctx* c, const Sample& s) {
  return c->fused_finish && !c->ls.on && xf_fuses_finish(s.Px) &&
         s.nb3 <= finish_single_stage_max();
}

// One minimiser iteration; with the defect correction, a reference pass
// first whenever the reference is poll_every iterations old (or stale).
// q >= 0: position in a batch of iterations that ends with flush_finish.
void enqueue_iteration(mm_ctx* c, Sample& s, double* m, int q = -1) {
  if (use_ref(c, s) && s.ref_age >= c->poll_every) enqueue_reference(c, s, m, s.st);
  EvalOut o;
  o.iterate = true;
  o.st_fin = s.st;
  o.fuse_q = q >= 0 && fuse_ok(c, s) ? q : -1;
  enqueue_eval(c, s, m, o);
  ++s.ref_age;
}

double tau0_of(const mm_ctx* c, const Sample& s) { return c->tau0 > 0 ? c->tau0 : 1e-3 / s.Ms; }

// ---- batched sweep ---------------------------------------------------------------
// Samples whose passes have wave-FFT kernels (thin films, x and y lengths in
// 64..512) run together: one launch per group of equal transform lengths
// covers the blocks of all of them, and one finish launch covers all.
struct BatchGroup {
  int a = 0, b = 0, t = 0;    // x: (M, R); yz: (Py, nz, tstride)
  int off = 0, n = 0;         // range in the item table
};

// A persistent launch: its range in the item table, block size, dynamic
// LDS and grid, for the iteration (main) and the reference pass (ref).
struct PersistLaunch {
  int off = 0, n = 0, threads = 0, nz = 0;
  size_t lds = 0, lds_ref = 0;
  int grid = 8, grid_inv = 8, grid_ref = 8, grid_ref_inv = 8;
};

struct BatchPlan {
  std::vector<int> members;               // sample indices, in table order
  std::vector<BatchGroup> xg, yg;
  std::vector<PersistLaunch> px;          // x passes: one per rows per block R
  std::vector<PersistLaunch> pyz;         // yz pass: one per layer count
  PersistLaunch p3[3];                    // 3-D samples: y forward, z, y inverse
  BatchDesc* descs = nullptr;
  BatchDesc* descs_ref = nullptr;         // reference pass (defect correction), or NULL
  WorkItem* items = nullptr;
  hipGraphExec_t graph = nullptr;
  ~BatchPlan() {
    if (graph) (void)hipGraphExecDestroy(graph);
    if (descs) (void)hipFree(descs);
    if (descs_ref) (void)hipFree(descs_ref);
    if (items) (void)hipFree(items);
  }
};

bool batchable(const mm_ctx* c, const Sample& s) {
  if (c->ls.on || s.M % 64 != 0 || s.M < 64 || s.M > 512) return false;
  if (single(c) && c->refine && !s.has_ref) return false;
  if (s.path == PATH_THIN) return yz_wave_ok(s.nz, s.Py);
  // the 3-D stages have persistent batched launches only
  return s.path == PATH_3D && c->persistent;
}

// XCD-aware order: hardware block b takes logical item xcd_remap(b, n), so
// each XCD works through a contiguous run of logical items (whole samples).
void xcd_order(std::vector<WorkItem>& v) {
  const int n = (int)v.size();
  const int full = (n / 8) * 8;
  std::vector<WorkItem> o(v.size());
  for (int b = 0; b < n; ++b) {
    const int L = b >= full ? b : (b & 7) * (n / 8) + (b >> 3);
    o[b] = v[L];
  }
  v.swap(o);
}

// only (optional): the samples to include (running ones), by index
int build_batch(mm_ctx* c, double* const* m, BatchPlan& P, const std::vector<char>* only = nullptr) {
  std::vector<BatchDesc> d;
  for (int k = 0; k < (int)c->smp.size(); ++k) {
    Sample& s = c->smp[k];
    if (!batchable(c, s) || (only && !(*only)[k])) continue;
    BatchDesc b;
    const LocalArgs a = local_args(s);
    b.m = m[k];
    b.g = s.g;
    b.s = s.s;
    b.spec = s.spec;
    b.Tt = s.Tt;
    b.twx = s.twx;
    b.twy = s.twy;
    const bool full = s.path == PATH_3D;
    b.B = full ? s.B : nullptr;
    b.twz = full ? s.twz : nullptr;
    b.Pz = full ? s.Pz : 1;
    b.st = s.st;
    b.partials = s.partials;
    b.ku_map = s.ku_map;
    b.nx = s.nx;
    b.ny = s.ny;
    b.nz = s.nz;
    b.M = s.M;
    b.Py = s.Py;
    b.R = s.R3;
    b.tstride = s.tstride;
    b.nb3 = s.nb3;
    b.cx = a.cx;
    b.cy = a.cy;
    b.cz = a.cz;
    b.ku = a.ku;
    b.kan = a.kan;
    for (int q = 0; q < 3; ++q) b.u[q] = a.u[q];
    b.scale = -s.Ms / ((double)s.M * (double)s.Py * (double)b.Pz);
    b.Ms = s.Ms;
    b.V = s.V;
    const bool corr = use_ref(c, s);
    b.mref = corr ? s.mref : nullptr;
    b.hdref = corr ? s.hdref : nullptr;
    b.pass = corr ? 1 : 0;
    P.members.push_back(k);
    d.push_back(b);
  }
  if (d.empty()) return MM_OK;
  // the reference pass: the same blocks on the double-precision buffers
  const bool refine = single(c) && c->refine;
  std::vector<BatchDesc> dr;
  if (refine) {
    for (int i = 0; i < (int)d.size(); ++i) {
      const Sample& s = c->smp[P.members[i]];
      BatchDesc b = d[i];
      b.spec = s.rspec;
      b.Tt = s.rTt;
      b.twx = s.rtwx;
      b.twy = s.rtwy;
      b.tstride = s.rtstride;
      if (b.B) {
        b.B = s.rB;
        b.twz = s.rtwz;
      }
      b.g = nullptr;    // no update and no BB sums in the reference pass (and
      b.s = nullptr;    // these streams have the single-precision type)
      b.pass = 2;
      dr.push_back(b);
    }
  }
  std::vector<WorkItem> all;
  auto add_groups = [&](bool x, std::vector<BatchGroup>& groups) {
    std::vector<BatchGroup> keys;
    for (int i = 0; i < (int)d.size(); ++i) {
      BatchGroup g;
      if (!x && d[i].B) continue;    // 3-D samples: persistent launches only
      if (x) { g.a = d[i].M; g.b = d[i].R; }
      else { g.a = d[i].Py; g.b = d[i].nz; g.t = d[i].tstride; }
      bool seen = false;
      for (auto& q : keys) seen = seen || (q.a == g.a && q.b == g.b && q.t == g.t);
      if (!seen) keys.push_back(g);
    }
    for (auto g : keys) {
      std::vector<WorkItem> v;
      for (int i = 0; i < (int)d.size(); ++i) {
        const bool match = x ? (d[i].M == g.a && d[i].R == g.b)
                             : (!d[i].B && d[i].Py == g.a && d[i].nz == g.b &&
                                d[i].tstride == g.t);
        if (!match) continue;
        const int nb = x ? d[i].nb3 : d[i].M + 1;   // yz: one block per column kx = 0..M
        for (int blk = 0; blk < nb; ++blk) v.push_back({i, blk});
      }
      xcd_order(v);
      g.off = (int)all.size();
      g.n = (int)v.size();
      all.insert(all.end(), v.begin(), v.end());
      groups.push_back(g);
    }
  };
  add_groups(true, P.xg);
  add_groups(false, P.yg);
  // persistent launches: the x blocks of the samples with R rows per block
  // in one table per R (blocks of exactly 192 R threads); the yz columns in
  // one table per layer count
  const bool sp = single(c);
  for (int R = 1; R <= 4; ++R) {
    PersistLaunch L;
    L.threads = 192 * R;
    std::vector<WorkItem> v;
    for (int i = 0; i < (int)d.size(); ++i) {
      if (d[i].R != R) continue;
      for (int blk = 0; blk < d[i].nb3; ++blk) v.push_back({i, blk});
      L.lds = std::max(L.lds, x_block_lds(sp, d[i].M, R));
      L.lds_ref = std::max(L.lds_ref, x_block_lds(false, d[i].M, R));
    }
    if (v.empty()) continue;
    xcd_order(v);
    L.off = (int)all.size();
    L.n = (int)v.size();
    all.insert(all.end(), v.begin(), v.end());
    L.grid = x_persistent_grid(sp, false, L.threads, L.lds);
    L.grid_inv = x_persistent_grid(sp, true, L.threads, L.lds);
    if (refine) {
      L.grid_ref = x_persistent_grid(false, false, L.threads, L.lds_ref);
      L.grid_ref_inv = x_persistent_grid(false, true, L.threads, L.lds_ref);
    }
    P.px.push_back(L);
  }
  for (int nz = 1; nz <= 4; ++nz) {
    PersistLaunch L;
    L.nz = nz;
    L.threads = 192 * nz;
    std::vector<WorkItem> v;
    for (int i = 0; i < (int)d.size(); ++i) {
      if (d[i].nz != nz || d[i].B) continue;
      for (int kx = 0; kx <= d[i].M; ++kx) v.push_back({i, kx});
      L.lds = std::max(L.lds, yz_block_lds(sp, d[i].Py, nz, d[i].tstride));
      if (refine) L.lds_ref = std::max(L.lds_ref, yz_block_lds(false, d[i].Py, nz, dr[i].tstride));
    }
    if (v.empty()) continue;
    xcd_order(v);
    L.off = (int)all.size();
    L.n = (int)v.size();
    all.insert(all.end(), v.begin(), v.end());
    L.grid = yz_persistent_grid(sp, nz, L.lds);
    if (refine) L.grid_ref = yz_persistent_grid(false, nz, L.lds_ref);
    P.pyz.push_back(L);
  }
  // 3-D samples: forward y, z with the tensor product, inverse y
  for (int st = 0; st < 3; ++st) {
    PersistLaunch& L = P.p3[st];
    L.threads = 256;
    std::vector<WorkItem> v;
    for (int i = 0; i < (int)d.size(); ++i) {
      if (!d[i].B) continue;
      const int nb = st == 1 ? z3_blocks(d[i].Py, d[i].M) : y3_blocks(d[i].nz, d[i].M);
      for (int blk = 0; blk < nb; ++blk) v.push_back({i, blk});
      const int len = st == 1 ? d[i].Pz : d[i].Py;
      L.lds = std::max(L.lds, w3_block_lds(sp, len));
      L.lds_ref = std::max(L.lds_ref, w3_block_lds(false, len));
    }
    if (v.empty()) continue;
    xcd_order(v);
    L.off = (int)all.size();
    L.n = (int)v.size();
    all.insert(all.end(), v.begin(), v.end());
    L.grid = w3_persistent_grid(sp, st - 1, L.lds);
    if (refine) L.grid_ref = w3_persistent_grid(false, st - 1, L.lds_ref);
  }
  if (hipMalloc((void**)&P.descs, d.size() * sizeof(BatchDesc)) != hipSuccess ||
      (refine && hipMalloc((void**)&P.descs_ref, d.size() * sizeof(BatchDesc)) != hipSuccess) ||
      hipMalloc((void**)&P.items, all.size() * sizeof(WorkItem)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, MM_ENOMEM, "device allocation for the batch tables failed");
  }
  HIPCHK(c, hipMemcpyAsync(P.descs, d.data(), d.size() * sizeof(BatchDesc), hipMemcpyHostToDevice,
                           c->stream));
  if (refine)
    HIPCHK(c, hipMemcpyAsync(P.descs_ref, dr.data(), dr.size() * sizeof(BatchDesc),
                             hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(P.items, all.data(), all.size() * sizeof(WorkItem),
                           hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MM_OK;
}

// Auxiliary streams for the launch groups of a batched pass.
constexpr int kAuxStreams = 4;

// All or nothing: on a failure the handles made so far are destroyed and the
// batched passes keep launching their groups one after another.
int ensure_aux(mm_ctx* c) {
  if (!c->aux.empty()) return MM_OK;
  std::vector<hipStream_t> aux;
  std::vector<hipEvent_t> join;
  hipEvent_t fork = nullptr;
  hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
  for (int k = 0; k < kAuxStreams && e == hipSuccess; ++k) {
    hipStream_t a = nullptr;
    hipEvent_t j = nullptr;
    e = hipStreamCreateWithFlags(&a, hipStreamNonBlocking);
    if (e != hipSuccess) break;
    aux.push_back(a);
    e = hipEventCreateWithFlags(&j, hipEventDisableTiming);
    if (e == hipSuccess) join.push_back(j);
  }
  if (e != hipSuccess) {
    for (auto a : aux) (void)hipStreamDestroy(a);
    for (auto j : join) (void)hipEventDestroy(j);
    if (fork) (void)hipEventDestroy(fork);
    return fail(c, MM_EHIP, std::string("auxiliary streams: ") + hipGetErrorString(e));
  }
  c->aux = aux;
  c->join_ev = join;
  c->fork_ev = fork;
  return MM_OK;
}

// Launch fn(g, stream) for the n groups of one pass.  The groups touch
// disjoint samples: with concurrent groups they go round-robin to the
// auxiliary streams, forked from and joined back into the context's stream
// (under graph capture: parallel branches); otherwise one after another.
template <typename F>
void for_groups(mm_ctx* c, int n, F fn) {
  if (n <= 1 || !c->concurrent_groups || c->aux.empty()) {
    for (int g = 0; g < n; ++g) fn(g, c->stream);
    return;
  }
  const int K = n < (int)c->aux.size() ? n : (int)c->aux.size();
  (void)hipEventRecord(c->fork_ev, c->stream);
  for (int k = 0; k < K; ++k) (void)hipStreamWaitEvent(c->aux[k], c->fork_ev, 0);
  for (int g = 0; g < n; ++g) fn(g, c->aux[g % K]);
  for (int k = 0; k < K; ++k) {
    (void)hipEventRecord(c->join_ev[k], c->aux[k]);
    (void)hipStreamWaitEvent(c->stream, c->join_ev[k], 0);
  }
}

// Launches between the x passes: one per yz layer-count class, and one
// chain of the three 3-D stages when the batch holds 3-D samples.
int n_mid(const BatchPlan& P) { return (int)P.pyz.size() + (P.p3[0].n > 0 ? 1 : 0); }

// Reference pass of every batched sample (double precision, same blocks).
void enqueue_batched_reference(mm_ctx* c, const BatchPlan& P) {
  if (!P.descs_ref) return;
  Timer t(c, KID_REF);
  if (c->persistent) {
    for (int inv = 0; inv < 2; ++inv) {
      if (inv)
        for_groups(c, n_mid(P), [&](int i, hipStream_t st) {
          if (i == (int)P.pyz.size()) {
            for (int q = 0; q < 3; ++q)
              launch_3d_persistent<double>(st, q - 1, P.descs_ref, P.items + P.p3[q].off,
                                           P.p3[q].n, P.p3[q].lds_ref, P.p3[q].grid_ref);
            return;
          }
          const PersistLaunch& L = P.pyz[i];
          launch_yz_persistent<double>(st, P.descs_ref, P.items + L.off, L.n, L.nz, L.lds_ref,
                                       L.grid_ref);
        });
      for_groups(c, (int)P.px.size(), [&](int i, hipStream_t st) {
        const PersistLaunch& L = P.px[i];
        launch_x_persistent<double>(st, inv != 0, P.descs_ref, P.items + L.off, L.n, L.threads,
                                    L.lds_ref, inv ? L.grid_ref_inv : L.grid_ref);
      });
    }
    return;
  }
  for_groups(c, (int)P.xg.size(), [&](int i, hipStream_t st) {
    const auto& g = P.xg[i];
    launch_x_batched<double>(st, false, P.descs_ref, P.items + g.off, g.n, g.a, g.b);
  });
  for_groups(c, (int)P.yg.size(), [&](int i, hipStream_t st) {
    const auto& g = P.yg[i];
    launch_yz_batched<double>(st, P.descs_ref, P.items + g.off, g.n, g.a, g.b,
                              thin_tensor_stride(g.b, g.a, false));
  });
  for_groups(c, (int)P.xg.size(), [&](int i, hipStream_t st) {
    const auto& g = P.xg[i];
    launch_x_batched<double>(st, true, P.descs_ref, P.items + g.off, g.n, g.a, g.b);
  });
}

// One iteration of every batched sample.
void enqueue_batched_iteration(mm_ctx* c, const BatchPlan& P) {
  hipStream_t st = c->stream;
  const bool sp = single(c);
  if (c->persistent) {
    auto x_pass = [&](bool inv) {
      for_groups(c, (int)P.px.size(), [&](int i, hipStream_t s) {
        const PersistLaunch& L = P.px[i];
        const int g = inv ? L.grid_inv : L.grid;
        if (sp)
          launch_x_persistent<float>(s, inv, P.descs, P.items + L.off, L.n, L.threads, L.lds, g);
        else
          launch_x_persistent<double>(s, inv, P.descs, P.items + L.off, L.n, L.threads, L.lds, g);
      });
    };
    {
      Timer t(c, KID_XF);
      x_pass(false);
    }
    {
      Timer t(c, KID_YZ);
      for_groups(c, n_mid(P), [&](int i, hipStream_t s) {
        if (i == (int)P.pyz.size()) {
          for (int q = 0; q < 3; ++q) {
            const PersistLaunch& L = P.p3[q];
            if (sp) launch_3d_persistent<float>(s, q - 1, P.descs, P.items + L.off, L.n, L.lds, L.grid);
            else launch_3d_persistent<double>(s, q - 1, P.descs, P.items + L.off, L.n, L.lds, L.grid);
          }
          return;
        }
        const PersistLaunch& L = P.pyz[i];
        if (sp)
          launch_yz_persistent<float>(s, P.descs, P.items + L.off, L.n, L.nz, L.lds, L.grid);
        else
          launch_yz_persistent<double>(s, P.descs, P.items + L.off, L.n, L.nz, L.lds, L.grid);
      });
    }
    {
      Timer t(c, KID_XIL);
      x_pass(true);
    }
    Timer t(c, KID_FINISH);
    launch_finish_batched(st, P.descs, (int)P.members.size());
    return;
  }
  {
    Timer t(c, KID_XF);
    for_groups(c, (int)P.xg.size(), [&](int i, hipStream_t s) {
      const auto& g = P.xg[i];
      if (sp) launch_x_batched<float>(s, false, P.descs, P.items + g.off, g.n, g.a, g.b);
      else launch_x_batched<double>(s, false, P.descs, P.items + g.off, g.n, g.a, g.b);
    });
  }
  {
    Timer t(c, KID_YZ);
    for_groups(c, (int)P.yg.size(), [&](int i, hipStream_t s) {
      const auto& g = P.yg[i];
      if (sp) launch_yz_batched<float>(s, P.descs, P.items + g.off, g.n, g.a, g.b, g.t);
      else launch_yz_batched<double>(s, P.descs, P.items + g.off, g.n, g.a, g.b, g.t);
    });
  }
  {
    Timer t(c, KID_XIL);
    for_groups(c, (int)P.xg.size(), [&](int i, hipStream_t s) {
      const auto& g = P.xg[i];
      if (sp) launch_x_batched<float>(s, true, P.descs, P.items + g.off, g.n, g.a, g.b);
      else launch_x_batched<double>(s, true, P.descs, P.items + g.off, g.n, g.a, g.b);
    });
  }
  {
    Timer t(c, KID_FINISH);
    launch_finish_batched(st, P.descs, (int)P.members.size());
  }
}

// ---- tile autotuner: rows per block of the fused x passes -----------------
// The x passes (xf, xil) work on R rows per block.  With the autotune
// option, mm_set_geometry times every valid R on the sample's own buffers
// (both passes in their minimiser form on scratch data) and keeps the
// fastest; the
// choice is cached per (precision, grid, path, padded lengths) for the
// process.
struct TuneKey {
  int sp, nx, ny, nz, path, Px, Py;
  bool operator<(const TuneKey& o) const {
    return std::tie(sp, nx, ny, nz, path, Px, Py) <
           std::tie(o.sp, o.nx, o.ny, o.nz, o.path, o.Px, o.Py);
  }
};

std::map<TuneKey, int>& tune_cache() {
  static std::map<TuneKey, int> m;
  return m;
}

std::mutex& tune_mutex() {
  static std::mutex mu;
  return mu;
}

// Valid tiles: the wave passes take 192 R threads (R <= 4); the LDS passes
// up to the heuristic's bound (LDS and threads per block); never above ny.
std::vector<int> row_tiles(int M, int ny, bool sp) {
  const bool wave = M % 64 == 0 && M >= 64 && M <= 512;
  const int hi = wave ? 4 : rows_per_block(M, ny, sp);
  std::vector<int> v;
  for (int r = 1; r <= hi && r <= ny; ++r)
    if (wave || (r & (r - 1)) == 0 || r == hi) v.push_back(r);
  return v;
}

// Mean time of one xf + xil pair with R rows per block (microseconds), in
// the form they take in a minimiser iteration: pending update, g and s read
// and written, BB and energy sums.  Scratch data: m is the field-output
// buffer (set up by prepare_tuning), g and s the sample's own, the state
// st_eval; the caller clears g and s afterwards.
int time_rows(mm_ctx* c, Sample& s, int R, double* us) {
  hipStream_t st = c->stream;
  const bool sp = single(c);
  Sample q = s;                 // material constants, finite even before mm_set_material
  if (!(q.Ms > 0)) {
    q.Ms = 8e5;
    q.A = 1.3e-11;
  }
  LocalArgs a = local_args(q);
  a.m = s.Hd;
  a.g = s.g;
  a.s = s.s;
  a.st = s.st_eval;
  auto pass = [&]() {
    if (sp) {
      launch_xf<float>(st, s.Hd, as<float>(s.g), as<float>(s.s), s.st_eval, s.nx, s.ny, s.nz,
                       s.Px, R, s.spec, s.twx, nullptr, nullptr);
      launch_xil<float>(st, s.spec, a, s.Px, R, nullptr, s.partials, s.twx);
    } else {
      launch_xf<double>(st, s.Hd, as<double>(s.g), as<double>(s.s), s.st_eval, s.nx, s.ny,
                        s.nz, s.Px, R, s.spec, s.twx, nullptr, nullptr);
      launch_xil<double>(st, s.spec, a, s.Px, R, nullptr, s.partials, s.twx);
    }
  };
  constexpr int kReps = 5;
  hipEvent_t e0 = take_event(c), e1 = take_event(c);
  pass();
  pass();
  hipError_t e = hipEventRecord(e0, st);
  for (int q = 0; q < kReps && e == hipSuccess; ++q) pass();
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  c->ev_pool.push_back(e0);
  c->ev_pool.push_back(e1);
  if (e != hipSuccess) return fail(c, MM_EHIP, std::string("tile timing: ") + hipGetErrorString(e));
  *us = 1e3 * ms / kReps;
  return MM_OK;
}

int choose_rows(mm_ctx* c, Sample& s) {
  const bool sp = single(c);
  const std::vector<int> tiles = row_tiles(s.M, s.ny, sp);
  int R = rows_per_block(s.M, s.ny, sp);
  if (c->rows_forced > 0) {
    bool ok = false;
    for (int r : tiles) ok = ok || r == c->rows_forced;
    if (!ok) return fail(c, MM_EINVAL, "rows_per_block is not a valid tile for this grid");
    R = c->rows_forced;
  } else if (c->autotune && tiles.size() > 1) {
    const TuneKey key{sp ? 1 : 0, s.nx, s.ny, s.nz, s.path, s.Px, s.Py};
    std::lock_guard<std::mutex> lock(tune_mutex());
    auto it = tune_cache().find(key);
    if (it != tune_cache().end()) {
      R = it->second;
    } else {
      // scratch: m = 0x3f3f... in every byte (about 4.8e-4 per component,
      // finite; the update normalises it), a state with an update pending
      // and k = 1 (BB sums on)
      HIPCHK(c, hipMemsetAsync(s.Hd, 0x3f, 3ull * s.N * sizeof(double), c->stream));
      MinState& h = *s.st_host;
      std::memset(&h, 0, sizeof(MinState));
      h.tau = h.last_tau = h.tau0 = 1e-3 / 8e5;
      h.k = 1;
      h.pending = 1;
      h.max_iter = 1;
      HIPCHK(c, hipMemcpyAsync(s.st_eval, s.st_host, sizeof(MinState), hipMemcpyHostToDevice,
                               c->stream));
      // three rounds over the candidates in turn; each keeps its best window,
      // so that a transient disturbance of one window decides nothing
      std::vector<double> best(tiles.size(), 0.0);
      for (int round = 0; round < 3; ++round) {
        for (size_t q = 0; q < tiles.size(); ++q) {
          double us = 0.0;
          int rc = time_rows(c, s, tiles[q], &us);
          if (rc != MM_OK) return rc;
          if (round == 0 || us < best[q]) best[q] = us;
        }
      }
      size_t qb = 0;
      for (size_t q = 1; q < tiles.size(); ++q)
        if (best[q] < best[qb]) qb = q;
      R = tiles[qb];
      tune_cache()[key] = R;
    }
  }
  s.R3 = R;
  s.nb3 = s.nz * ((s.ny + R - 1) / R);
  return MM_OK;
}

std::map<TuneKey, int>& yz_tune_cache() {
  static std::map<TuneKey, int> m;
  return m;
}

// Mean time of one thin yz pass with occupancy variant var (microseconds)
// on the sample's tensor and spectrum buffer (scratch contents: every
// iteration's forward x pass rewrites the spectrum).
int time_yz(mm_ctx* c, Sample& s, int var, double* us) {
  hipStream_t st = c->stream;
  const bool sp = single(c);
  auto pass = [&]() {
    if (sp)
      launch_yz_thin<float>(st, s.spec, s.nz, s.ny, s.Py, s.M, (const float*)s.Tt, s.tstride,
                            -1.0f, s.twy, nullptr, var);
    else
      launch_yz_thin<double>(st, s.spec, s.nz, s.ny, s.Py, s.M, (const double*)s.Tt, s.tstride,
                             -1.0, s.twy, nullptr, var);
  };
  constexpr int kReps = 5;
  hipEvent_t e0 = take_event(c), e1 = take_event(c);
  pass();
  pass();
  hipError_t e = hipEventRecord(e0, st);
  for (int q = 0; q < kReps && e == hipSuccess; ++q) pass();
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  c->ev_pool.push_back(e0);
  c->ev_pool.push_back(e1);
  if (e != hipSuccess) return fail(c, MM_EHIP, std::string("yz timing: ") + hipGetErrorString(e));
  *us = 1e3 * ms / kReps;
  return MM_OK;
}

// The thin yz pass's occupancy variant: with the autotune option, both
// variants (where the grid has two) are timed in three interleaved rounds
// and the faster kept, cached per precision, grid and padded lengths.
int choose_yz(mm_ctx* c, Sample& s) {
  const bool sp = single(c);
  s.yz_var = 0;
  const int nvar = s.path == PATH_THIN ? yz_variants(sp, s.nz, s.Py) : 1;
  if (c->yz_forced >= 0) {
    if (c->yz_forced >= nvar)
      return fail(c, MM_EINVAL, "yz_variant: this grid's yz pass has no such variant");
    s.yz_var = c->yz_forced;
    return MM_OK;
  }
  if (!c->autotune || nvar < 2) return MM_OK;
  const TuneKey key{sp ? 1 : 0, s.nx, s.ny, s.nz, s.path, s.Px, s.Py};
  std::lock_guard<std::mutex> lock(tune_mutex());
  auto it = yz_tune_cache().find(key);
  if (it != yz_tune_cache().end()) {
    s.yz_var = it->second;
    return MM_OK;
  }
  double best[2] = {0.0, 0.0};
  for (int round = 0; round < 3; ++round) {
    for (int v = 0; v < 2; ++v) {
      double us = 0.0;
      const int rc = time_yz(c, s, v, &us);
      if (rc != MM_OK) return rc;
      if (round == 0 || us < best[v]) best[v] = us;
    }
  }
  s.yz_var = best[1] < best[0] ? 1 : 0;
  yz_tune_cache()[key] = s.yz_var;
  return MM_OK;
}

int status_of(int done) {
  switch (done) {
    case 1: return MM_OK;
    case 2: return MM_NOT_CONVERGED;
    case 3: return MM_STALLED;
    case -1: return MM_ENONFINITE;
    default: return MM_NOT_CONVERGED;
  }
}

int read_state(mm_ctx* c, Sample& s) {
  flush_finish(c, s);
  HIPCHK(c, hipMemcpyAsync(s.st_host, s.st, sizeof(MinState), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MM_OK;
}

// Captured batch of poll_every iterations of one sample (made on first use,
// kept while the m buffer, batch length, correction and material stay).
// The batch starts with the reference pass when the defect correction is on,
// as an eager batch does.
int ensure_iter_graph(mm_ctx* c, Sample& s, double* m) {
  const int ref = use_ref(c, s) ? 1 : 0;
  if (s.it_graph && s.it_graph_m == m && s.it_graph_n == c->poll_every && s.it_graph_ref == ref &&
      s.it_graph_mat == s.mat_version && s.it_graph_ls == c->ls.on &&
      s.it_graph_fuse == (fuse_ok(c, s) ? 1 : 0))
    return MM_OK;
  if (s.it_graph) (void)hipGraphExecDestroy(s.it_graph);
  s.it_graph = nullptr;
  hipGraph_t g = nullptr;
  s.ref_age = kRefStale;
  hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    for (int q = 0; q < c->poll_every; ++q) enqueue_iteration(c, s, m, q);
    flush_finish(c, s);
    e = hipStreamEndCapture(c->stream, &g);
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&s.it_graph, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    s.it_graph = nullptr;
    return fail(c, MM_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
  }
  s.it_graph_m = m;
  s.it_graph_n = c->poll_every;
  s.it_graph_ref = ref;
  s.it_graph_mat = s.mat_version;
  s.it_graph_ls = c->ls.on;
  s.it_graph_fuse = fuse_ok(c, s) ? 1 : 0;
  return MM_OK;
}

// Line-search buffers of a sample (saved base m and the trial gradient),
// allocated on the first run with the line search on.
int ensure_ls(mm_ctx* c, Sample& s) {
  if (!c->ls.on || s.ls_g2 != nullptr) return MM_OK;
  if (hipMalloc((void**)&s.ls_mbase, 3ull * s.N * sizeof(double)) != hipSuccess ||
      hipMalloc(&s.ls_g2, 3ull * s.N * gs_bytes(c)) != hipSuccess) {
    dfree(s.ls_mbase);
    dfree(s.ls_g2);
    (void)hipGetLastError();
    return fail(c, MM_ENOMEM, "device allocation for the line search failed");
  }
  return MM_OK;
}

// Minimiser state reset of a run: BB state, stop rule, step choice and
// (when on) the line search with the sample's buffers.
void reset_run(mm_ctx* c, hipStream_t st, Sample& s, double tol, long long max_iter) {
  s.fin_pending = false;   // a reset state drops any pending finish
  launch_reset_state(st, s.st, tau0_of(c, s), tol, max_iter, stall_of(c, s), 0, s.H, c->bb_switch,
                     c->ls.on ? &c->ls : nullptr, s.ls_mbase, s.ls_g2);
}

// Poll loop of a run whose device state is set: batches of poll_every
// iterations until the state ends the run.  left bounds the evaluations
// enqueued (launches beyond the end would only read the stop flag and
// return); k0 and e0 are the state's update and evaluation counts when the
// loop starts (the context's totals count what the loop adds).
int run_loop(mm_ctx* c, Sample& s, double* m, long long left, long long k0, long long e0,
             mm_min_result* out) {
  // full batches after the first replay a captured graph (use_graph on a
  // non-null stream, kernels not being timed); the first batch runs eagerly
  const bool graph = c->use_graph && c->stream != nullptr && c->prof == 0;
  // A captured batch starts with the reference pass of the defect
  // correction; with a reference younger than poll_every (a continued run)
  // the first batch ends where it falls due, so that the references come at
  // the iterations of an uninterrupted run
  long long first = c->poll_every;
  if (use_ref(c, s) && s.ref_age >= 0 && s.ref_age < c->poll_every) first = c->poll_every - s.ref_age;
  long long evals_before = e0;
  for (int nbatch = 0;; ++nbatch) {
    const long long cap = nbatch == 0 ? first : c->poll_every;
    const long long batch = left < 1 ? 1 : (left < cap ? left : cap);
    const bool replay = graph && nbatch > 0 && batch == c->poll_every;
    // reference age before the batch (a captured batch starts with the pass)
    const long long age_before = replay ? c->poll_every : s.ref_age;
    if (replay) {
      int rc = ensure_iter_graph(c, s, m);
      if (rc != MM_OK) return rc;
      HIPCHK(c, hipGraphLaunch(s.it_graph, c->stream));
      s.ref_age = c->poll_every;   // as after an eager batch
    } else {
      for (long long q = 0; q < batch; ++q) enqueue_iteration(c, s, m, (int)q);
      flush_finish(c, s);
    }
    left -= batch;
    HIPCHK(c, hipGetLastError());
    int rc = read_state(c, s);
    if (rc != MM_OK) return rc;
    prof_collect(c);
    if (s.st_host->fin_err != 0)
      return fail(c, MM_ESTATE, "a forward x pass gave up waiting for the finish decision");
    if (s.st_host->done != 0) {
      // iterations enqueued after the run ended did nothing: the reference
      // age counts the evaluations that ran (a continued run needs it)
      if (use_ref(c, s)) {
        long long age = age_before;
        for (long long q = 0; q < s.st_host->evals - evals_before; ++q) {
          if (age >= c->poll_every) age = 0;
          ++age;
        }
        s.ref_age = age;
      }
      break;
    }
    evals_before = s.st_host->evals;
    // the evaluation that reaches max_iter ends the run on the device; a
    // state that still runs well after it would keep the host polling
    if (left < -(long long)c->poll_every)
      return fail(c, MM_ESTATE, "the device state did not end the run at max_iter");
  }
  const MinState& h = *s.st_host;
  s.evals_total += h.evals - e0;
  s.iters_total += h.k - k0;
  if (out) {
    out->status = status_of(h.done);
    out->iters = h.k;
    out->heff_evals = h.evals;
    out->torque = h.torque;
    out->energy = h.energy;
  }
  if (h.done == -1) return fail(c, MM_ENONFINITE, "non-finite torque or energy");
  return status_of(h.done);
}

int run_to_tol(mm_ctx* c, Sample& s, double* m, double tol, int64_t max_iter, mm_min_result* out) {
  int lrc = ensure_ls(c, s);
  if (lrc != MM_OK) return lrc;
  reset_run(c, c->stream, s, tol, (long long)max_iter);
  s.ref_age = kRefStale;
  // a run evaluates at most max_iter + 1 times
  return run_loop(c, s, m, (long long)max_iter + 1, 0, 0, out);
}

// Allocate the derivative workspace of a sample on first use.
int ensure_adj(mm_ctx* c, Sample& s) {
  if (s.Hm) return MM_OK;
  const size_t b3 = 3ull * s.N * sizeof(double);
  bool ok = hipMalloc((void**)&s.Hm, b3) == hipSuccess && hipMalloc((void**)&s.Hlin, b3) == hipSuccess &&
            hipMalloc((void**)&s.cr, b3) == hipSuccess && hipMalloc((void**)&s.cp, b3) == hipSuccess &&
            hipMalloc((void**)&s.cAp, b3) == hipSuccess &&
            hipMalloc((void**)&s.cg, sizeof(CGState)) == hipSuccess &&
            hipMalloc((void**)&s.scal, 8 * sizeof(double)) == hipSuccess &&
            hipHostMalloc((void**)&s.cg_host, sizeof(CGState), hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void**)&s.scal_host, 8 * sizeof(double), hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    dfree(s.Hm);
    dfree(s.Hlin);
    dfree(s.cr);
    dfree(s.cp);
    dfree(s.cAp);
    dfree(s.cg);
    dfree(s.scal);
    if (s.cg_host) (void)hipHostFree(s.cg_host);
    if (s.scal_host) (void)hipHostFree(s.scal_host);
    s.cg_host = nullptr;
    s.scal_host = nullptr;
    return fail(c, MM_ENOMEM, "device allocation for the derivative workspace failed");
  }
  return MM_OK;
}

// H_eff(m) into s.Hm
void enqueue_heff_m(mm_ctx* c, Sample& s, const double* m) {
  EvalOut o;
  o.H = s.Hm;
  enqueue_eval(c, s, m, o);
}

// H_lin[v] (demag + exchange + anisotropy, no Zeeman) into s.Hlin
void enqueue_hlin(mm_ctx* c, Sample& s, const double* v, const int* done) {
  EvalOut o;
  o.H = s.Hlin;
  o.zeeman = false;
  o.done = done;
  enqueue_eval(c, s, v, o);
}

int read_scal(mm_ctx* c, Sample& s, int n) {
  HIPCHK(c, hipMemcpyAsync(s.scal_host, s.scal, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MM_OK;
}

}  // namespace

// ---- allocation-free evaluation ----------------------------------------------
// mm_heff_static keeps the spectrum of its convolution (and, on the 3-D path,
// the y-transformed spectrum) in this array instead of the sample's own
// buffers.  Every GPU the library runs on holds one copy until the process
// ends; host code reaches it only through the per-device address taken with
// hipGetSymbolAddress (the array's name is a host-side stand-in).
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev (current), resolved once per device.
int scratch_address(mm_ctx* c, int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(c, MM_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return fail(c, MM_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
  return MM_OK;
}

}  // namespace

// ============================================================================
extern "C" {

int mm_create(mm_ctx** out, int prec, int n_samples, void* hip_stream) {
  if (!out) return MM_EINVAL;
  *out = nullptr;
  if ((prec != MM_FP64 && prec != MM_MIXED) || n_samples < 1) return MM_EINVAL;
  mm_ctx* c = new mm_ctx();
  c->prec = prec;
  c->stream = (hipStream_t)hip_stream;
  c->smp.resize(n_samples);
  *out = c;
  return MM_OK;
}

void mm_destroy(mm_ctx* c) {
  if (!c) return;
  bool any = false;
  for (auto& s : c->smp) any = any || s.has_geom;
  if (any || !c->prof_pending.empty() || !c->ev_pool.empty()) (void)hipStreamSynchronize(c->stream);
  for (auto& s : c->smp) free_sample(s);
  for (auto& r : c->prof_pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);
  for (auto a : c->aux) {
    (void)hipStreamSynchronize(a);
    (void)hipStreamDestroy(a);
  }
  for (auto e : c->join_ev) (void)hipEventDestroy(e);
  if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
  delete c;
}

int mm_supported(int prec, int nx, int ny, int nz) {
  if (prec != MM_FP64 && prec != MM_MIXED) return 0;
  return choose_path(prec, 0, nx, ny, nz) != PATH_NONE ? 1 : 0;
}

int mm_set_geometry(mm_ctx* c, int sample, int nx, int ny, int nz, double dx, double dy, double dz) {
  if (!c) return MM_EINVAL;
  if (sample < 0 || sample >= (int)c->smp.size()) return fail(c, MM_EINVAL, "sample index out of range");
  if (nx < 1 || ny < 1 || nz < 1 || !(dx > 0) || !(dy > 0) || !(dz > 0) || !std::isfinite(dx) ||
      !std::isfinite(dy) || !std::isfinite(dz))
    return fail(c, MM_EINVAL, "grid sizes must be >= 1 and cell sizes positive");
  if ((long long)nx * ny * nz > (1LL << 30)) return fail(c, MM_EINVAL, "grid too large");
  const bool mr = c->mixed_radix != 0;
  const int path = choose_path(c->prec, c->path_pref, nx, ny, nz, mr);
  if (path == PATH_NONE)
    return fail(c, MM_EUNSUPPORTED, "grid shape not supported by the library's kernels");
  (void)hipStreamSynchronize(c->stream);
  Sample& s = c->smp[sample];
  const double Ms = s.Ms, A = s.A, Ku = s.Ku;
  const double u0 = s.u[0], u1 = s.u[1], u2 = s.u[2];
  const double H0 = s.H[0], H1 = s.H[1], H2 = s.H[2];
  free_sample(s);
  s.Ms = Ms; s.A = A; s.Ku = Ku;
  s.u[0] = u0; s.u[1] = u1; s.u[2] = u2;
  s.H[0] = H0; s.H[1] = H1; s.H[2] = H2;
  s.nx = nx; s.ny = ny; s.nz = nz;
  s.N = nx * ny * nz;
  s.dx = dx; s.dy = dy; s.dz = dz;
  s.V = dx * dy * dz;
  s.path = path;
  if (hipGetDevice(&s.dev) != hipSuccess) s.dev = -1;
  s.Px = pad_x(nx, mr);
  s.M = s.Px / 2;
  const bool full = path == PATH_3D;
  s.Py = full ? pad_3d(ny) : pad_thin_y(ny, mr);
  s.Pz = full ? pad_3d(nz) : 1;
  const bool sp = single(c);
  s.R3 = rows_per_block(s.M, ny, sp);
  s.nb3 = nz * ((ny + s.R3 - 1) / s.R3);
  const size_t creal = sp ? sizeof(float) : sizeof(double);
  s.tstride = full ? tensor3_row(s.Pz, sp) : thin_tensor_stride(nz, s.Py, sp);
  const size_t nT = (size_t)(s.M + 1) * (full ? (size_t)(s.Py / 2 + 1) : 1) * s.tstride;
  const size_t nspec = (size_t)(s.M + 1) * 3 * nz * ny;
  const size_t nB = full ? (size_t)(s.M + 1) * s.Py * 3 * nz : 0;
  s.nblk = local_blocks(s.N);
  // per-block sums: room for one row per block (the smallest tile), and for
  // the first stage of their reduction
  const int prow = s.nblk > nz * ny ? s.nblk : nz * ny;
  const size_t npart = (size_t)(prow + finish_extra_rows(prow)) * kNPartial;
  bool ok = hipMalloc(&s.Tt, nT * creal) == hipSuccess &&
            hipMalloc(&s.spec, nspec * 2 * creal) == hipSuccess &&
            hipMalloc(&s.twx, (size_t)s.Px * 2 * creal) == hipSuccess &&
            hipMalloc(&s.twy, (size_t)s.Py * 2 * creal) == hipSuccess &&
            (!full || hipMalloc(&s.B, nB * 2 * creal) == hipSuccess) &&
            (!full || hipMalloc(&s.twz, (size_t)s.Pz * 2 * creal) == hipSuccess) &&
            hipMalloc((void**)&s.Hd, 3ull * s.N * sizeof(double)) == hipSuccess &&
            hipMalloc(&s.g, 3ull * s.N * gs_bytes(c)) == hipSuccess &&
            hipMalloc(&s.s, 3ull * s.N * gs_bytes(c)) == hipSuccess &&
            hipMalloc((void**)&s.partials, npart * sizeof(double)) == hipSuccess &&
            hipMalloc((void**)&s.st, sizeof(MinState)) == hipSuccess &&
            hipMalloc((void**)&s.st_eval, sizeof(MinState)) == hipSuccess &&
            hipMalloc((void**)&s.dev3, 3 * sizeof(double)) == hipSuccess &&
            hipHostMalloc((void**)&s.st_host, sizeof(MinState), hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void**)&s.host3, 3 * sizeof(double), hipHostMallocDefault) == hipSuccess;
  // double-precision reference of the single-precision form, where the
  // double-precision kernels handle the same path for this grid
  if (ok && sp && choose_path(MM_FP64, c->path_pref, nx, ny, nz, mr) == path) {
    s.rR3 = rows_per_block(s.M, ny, false);
    s.rtstride = full ? tensor3_row(s.Pz, false) : thin_tensor_stride(nz, s.Py, false);
    const size_t nTr = (size_t)(s.M + 1) * (full ? (size_t)(s.Py / 2 + 1) : 1) * s.rtstride;
    ok = hipMalloc(&s.rTt, nTr * sizeof(double)) == hipSuccess &&
         hipMalloc(&s.rspec, nspec * 2 * sizeof(double)) == hipSuccess &&
         hipMalloc(&s.rtwx, (size_t)s.Px * 2 * sizeof(double)) == hipSuccess &&
         hipMalloc(&s.rtwy, (size_t)s.Py * 2 * sizeof(double)) == hipSuccess &&
         (!full || hipMalloc(&s.rB, nB * 2 * sizeof(double)) == hipSuccess) &&
         (!full || hipMalloc(&s.rtwz, (size_t)s.Pz * 2 * sizeof(double)) == hipSuccess) &&
         hipMalloc((void**)&s.mref, 3ull * s.N * sizeof(double)) == hipSuccess &&
         hipMalloc((void**)&s.hdref, 3ull * s.N * sizeof(double)) == hipSuccess;
    if (ok) {
      s.has_ref = true;
      HIPCHK(c, hipMemsetAsync(s.rTt, 0, nTr * sizeof(double), c->stream));
      launch_twiddles(c->stream, s.rtwx, s.Px, false);
      launch_twiddles(c->stream, s.rtwy, s.Py, false);
      if (full) launch_twiddles(c->stream, s.rtwz, s.Pz, false);
    }
  }
  s.ref_age = kRefStale;
  if (!ok) {
    free_sample(s);
    (void)hipGetLastError();
    return fail(c, MM_ENOMEM, "device allocation failed");
  }
  HIPCHK(c, hipMemsetAsync(s.Tt, 0, nT * creal, c->stream));
  HIPCHK(c, hipMemsetAsync(s.g, 0, 3ull * s.N * gs_bytes(c), c->stream));
  HIPCHK(c, hipMemsetAsync(s.s, 0, 3ull * s.N * gs_bytes(c), c->stream));
  launch_twiddles(c->stream, s.twx, s.Px, sp);
  launch_twiddles(c->stream, s.twy, s.Py, sp);
  if (full) launch_twiddles(c->stream, s.twz, s.Pz, sp);
  int rc = full ? build_tensor3d(c, s) : build_tensor(c, s);
  if (rc == MM_OK) rc = choose_rows(c, s);
  if (rc == MM_OK) rc = choose_yz(c, s);
  if (rc != MM_OK) {
    free_sample(s);
    return rc;
  }
  // the tile timing ran minimiser passes on g and s: start from zero again
  HIPCHK(c, hipMemsetAsync(s.g, 0, 3ull * s.N * gs_bytes(c), c->stream));
  HIPCHK(c, hipMemsetAsync(s.s, 0, 3ull * s.N * gs_bytes(c), c->stream));
  s.has_geom = true;
  s.has_mat = s.Ms > 0;
  s.evals_total = s.iters_total = 0;
  if (s.has_mat)
    launch_reset_state(c->stream, s.st, tau0_of(c, s), 0.0, 0, 0, 1, s.H, c->bb_switch);
  s.fin_pending = false;   // a reset state drops any pending finish
  HIPCHK(c, hipGetLastError());
  return MM_OK;
}

int mm_set_material(mm_ctx* c, int sample, double Ms, double A, double Ku, const double* u,
                    const double* Ku_map) {
  int rc = check_sample(c, sample, false);
  if (rc != MM_OK) return rc;
  if (!(Ms > 0) || !std::isfinite(Ms) || !(A >= 0) || !std::isfinite(A) || !std::isfinite(Ku))
    return fail(c, MM_EINVAL, "Ms must be > 0, A >= 0, Ku finite");
  Sample& s = c->smp[sample];
  double uu[3] = {1, 0, 0};
  if (u) {
    const double n = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    if (!(n > 0) || !std::isfinite(n)) return fail(c, MM_EINVAL, "easy axis must be non-zero");
    for (int q = 0; q < 3; ++q) uu[q] = u[q] / n;
  }
  s.Ms = Ms;
  s.A = A;
  s.Ku = Ku;
  for (int q = 0; q < 3; ++q) s.u[q] = uu[q];
  if (Ku_map) {
    if (!s.ku_map && hipMalloc((void**)&s.ku_map, (size_t)s.N * sizeof(double)) != hipSuccess) {
      s.ku_map = nullptr;
      return fail(c, MM_ENOMEM, "device allocation failed");
    }
    HIPCHK(c, hipMemcpyAsync(s.ku_map, Ku_map, (size_t)s.N * sizeof(double),
                             hipMemcpyDeviceToDevice, c->stream));
  } else {
    dfree(s.ku_map);
  }
  s.has_mat = true;
  s.ref_age = kRefStale;   // the reference field scales with Ms
  ++s.mat_version;         // material constants are baked into captured launches
  launch_reset_state(c->stream, s.st, tau0_of(c, s), 0.0, 0, 0, 1, s.H, c->bb_switch);
  s.fin_pending = false;   // a reset state drops any pending finish
  HIPCHK(c, hipGetLastError());
  return MM_OK;
}

int mm_set_field(mm_ctx* c, int sample, const double* H) {
  int rc = check_sample(c, sample, false);
  if (rc != MM_OK) return rc;
  if (!H || !std::isfinite(H[0]) || !std::isfinite(H[1]) || !std::isfinite(H[2]))
    return fail(c, MM_EINVAL, "field must be three finite numbers");
  Sample& s = c->smp[sample];
  for (int q = 0; q < 3; ++q) s.H[q] = H[q];
  if (s.has_mat)
    launch_reset_state(c->stream, s.st, tau0_of(c, s), 0.0, 0, 0, 1, s.H, c->bb_switch);
  s.fin_pending = false;   // a reset state drops any pending finish
  HIPCHK(c, hipGetLastError());
  return MM_OK;
}

int mm_reset(mm_ctx* c, int sample) {
  int rc = check_sample(c, sample, true);
  if (rc != MM_OK) return rc;
  Sample& s = c->smp[sample];
  launch_reset_state(c->stream, s.st, tau0_of(c, s), 0.0, 0, 0, 1, s.H, c->bb_switch);
  s.fin_pending = false;   // a reset state drops any pending finish
  HIPCHK(c, hipGetLastError());
  return MM_OK;
}

int mm_heff(mm_ctx* c, int sample, const double* m, double* H) {
  int rc = check_sample(c, sample, true);
  if (rc != MM_OK) return rc;
  if (!m || !H) return fail(c, MM_EINVAL, "null buffer");
  EvalOut o;
  o.H = H;
  enqueue_eval(c, c->smp[sample], m, o);
  HIPCHK(c, hipGetLastError());
  return MM_OK;
}

int mm_heff_static(mm_ctx* c, int sample, const double* m, double* H) {
  int rc = check_sample(c, sample, true);
  if (rc != MM_OK) return rc;
  if (!m || !H) return fail(c, MM_EINVAL, "null buffer");
  Sample& s = c->smp[sample];
  int dev = -1;
  HIPCHK(c, hipGetDevice(&dev));
  if (dev != s.dev)
    return fail(c, MM_ESTATE, "mm_heff_static: call with the device of mm_set_geometry current");
  const size_t creal = single(c) ? sizeof(float) : sizeof(double);
  const size_t spec = (size_t)(s.M + 1) * 3 * s.nz * s.ny * 2 * creal;
  const size_t spec_al = (spec + 255) / 256 * 256;
  const size_t nB = s.path == PATH_3D ? (size_t)(s.M + 1) * s.Py * 3 * s.nz * 2 * creal : 0;
  const size_t need = spec_al + nB;
  if (need > kStaticScratchBytes)
    return fail(c, MM_EINVAL, "mm_heff_static: this grid needs " + std::to_string(need) +
                                  " bytes of scratch, more than its maximum of " +
                                  std::to_string(kStaticScratchBytes));
  unsigned char* base = nullptr;
  rc = scratch_address(c, dev, &base);
  if (rc != MM_OK) return rc;
  EvalOut o;
  o.H = H;
  o.spec = base;
  o.B = nB ? base + spec_al : nullptr;
  enqueue_eval(c, s, m, o);
  HIPCHK(c, hipGetLastError());
  return MM_OK;
}

int mm_field_terms(mm_ctx* c, int sample, const double* m, double* H_demag, double* H_exchange,
                   double* H_anisotropy) {
  int rc = check_sample(c, sample, true);
  if (rc != MM_OK) return rc;
  if (!m) return fail(c, MM_EINVAL, "null buffer");
  EvalOut o;
  o.Hd = H_demag;
  o.Hex = H_exchange;
  o.Han = H_anisotropy;
  enqueue_eval(c, c->smp[sample], m, o);
  HIPCHK(c, hipGetLastError());
  return MM_OK;
}

int mm_energy(mm_ctx* c, int sample, const double* m, double* E, double* terms4) {
  int rc = check_sample(c, sample, true);
  if (rc != MM_OK) return rc;
  if (!m || !E) return fail(c, MM_EINVAL, "null buffer");
  Sample& s = c->smp[sample];
  launch_reset_state(c->stream, s.st_eval, 0.0, 0.0, 0, 0, 2, s.H);
  EvalOut o;
  o.st_fin = s.st_eval;
  enqueue_eval(c, s, m, o);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(s.st_host, s.st_eval, sizeof(MinState), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  prof_collect(c);
  *E = s.st_host->energy;
  if (terms4)
    for (int q = 0; q < 4; ++q) terms4[q] = s.st_host->eterm[q];
  if (!std::isfinite(*E)) return fail(c, MM_ENONFINITE, "non-finite energy");
  return MM_OK;
}

int mm_minimize_step(mm_ctx* c, int sample, double* m, mm_step_info* info) {
  int rc = check_sample(c, sample, true);
  if (rc != MM_OK) return rc;
  if (!m) return fail(c, MM_EINVAL, "null buffer");
  if (c->ls.on)
    return fail(c, MM_EINVAL, "the line search runs in mm_minimize_to_tol and sweeps only");
  Sample& s = c->smp[sample];
  launch_set_mode(c->stream, s.st, 1);
  enqueue_iteration(c, s, m);
  {
    Timer t(c, KID_UPDATE);
    if (single(c))
      launch_update<float>(c->stream, m, as<float>(s.g), as<float>(s.s), s.N, s.st);
    else
      launch_update<double>(c->stream, m, as<double>(s.g), as<double>(s.s), s.N, s.st);
  }
  launch_clear_pending(c->stream, s.st);
  HIPCHK(c, hipGetLastError());
  s.evals_total += 1;
  s.iters_total += 1;
  if (info) {
    rc = read_state(c, s);
    if (rc != MM_OK) return rc;
    prof_collect(c);
    info->tau = s.st_host->last_tau;
    info->torque = s.st_host->torque;
    info->energy = s.st_host->energy;
    info->k = s.st_host->last_k;
    if (s.st_host->done == -1) return fail(c, MM_ENONFINITE, "non-finite torque or energy");
  }
  return MM_OK;
}

int mm_minimize_to_tol(mm_ctx* c, int sample, double* m, double tol, int64_t max_iter,
                       mm_min_result* out) {
  int rc = check_sample(c, sample, true);
  if (rc != MM_OK) return rc;
  if (!m || !(tol >= 0) || max_iter < 0) return fail(c, MM_EINVAL, "bad argument");
  return run_to_tol(c, c->smp[sample], m, tol, max_iter, out);
}

int mm_minimize_continue(mm_ctx* c, int sample, double* m, double tol, int64_t max_iter,
                         mm_min_result* out) {
  int rc = check_sample(c, sample, true);
  if (rc != MM_OK) return rc;
  if (!m || !(tol >= 0) || max_iter < 0) return fail(c, MM_EINVAL, "bad argument");
  if (c->ls.on) return fail(c, MM_EINVAL, "a line-search run is not continued");
  Sample& s = c->smp[sample];
  rc = read_state(c, s);   // also runs a pending finish
  if (rc != MM_OK) return rc;
  if (s.st_host->done == -1) return fail(c, MM_ENONFINITE, "the run ended on a non-finite state");
  const long long k0 = s.st_host->k, e0 = s.st_host->evals;
  launch_continue_state(c->stream, s.st, tol, (long long)max_iter, stall_of(c, s));
  HIPCHK(c, hipGetLastError());
  // at most max_iter - k0 + 1 evaluations remain (k0 + 1 where a step was
  // just decided; the device state ends the run in either case)
  const long long left = (long long)max_iter - k0 + 1;
  return run_loop(c, s, m, left < 1 ? 1 : left, k0, e0, out);
}

// ---- checkpoint of a run ----------------------------------------------------
namespace {

// The run fields of MinState (no pointers, sweep or line-search bookkeeping).
struct CkptRun {
  double tau, torque, energy, eterm[4], ss, sy, yy, best_torque, tol, tau0;
  long long k, best_k, evals, max_iter, stall_iters;
  int done, mode;
  double last_tau;
  long long last_k;
  int pending, pad;
  double H[3];
  double bb_switch;
};

struct CkptHeader {
  char magic[8];
  int32_t version, prec, nx, ny, nz, gs, has_ref, pad;
  int64_t ref_age, bytes;
  CkptRun run;
};

constexpr char kCkptMagic[8] = {'M', 'M', 'B', 'B', 'C', 'K', 'P', 'T'};

int64_t ckpt_bytes(const mm_ctx* c, const Sample& s) {
  const int64_t n3 = 3LL * s.N;
  int64_t b = (int64_t)sizeof(CkptHeader) + 2 * n3 * (int64_t)gs_bytes(c);
  if (use_ref(c, s)) b += 2 * n3 * (int64_t)sizeof(double);
  return b;
}

}  // namespace

int mm_state_bytes(mm_ctx* c, int sample, int64_t* bytes) {
  int rc = check_sample(c, sample, true);
  if (rc != MM_OK) return rc;
  if (!bytes) return fail(c, MM_EINVAL, "null pointer");
  *bytes = ckpt_bytes(c, c->smp[sample]);
  return MM_OK;
}

int mm_state_save(mm_ctx* c, int sample, void* host, int64_t bytes) {
  int rc = check_sample(c, sample, true);
  if (rc != MM_OK) return rc;
  if (!host) return fail(c, MM_EINVAL, "null buffer");
  if (c->ls.on) return fail(c, MM_EINVAL, "a line-search run is not checkpointed");
  Sample& s = c->smp[sample];
  const int64_t need = ckpt_bytes(c, s);
  if (bytes < need)
    return fail(c, MM_EINVAL, "checkpoint buffer of " + std::to_string(bytes) + " bytes; " +
                                  std::to_string(need) + " needed");
  rc = read_state(c, s);   // also runs a pending finish
  if (rc != MM_OK) return rc;
  const MinState& h = *s.st_host;
  CkptHeader hd;
  std::memset(&hd, 0, sizeof(hd));
  std::memcpy(hd.magic, kCkptMagic, sizeof(kCkptMagic));
  hd.version = 1;
  hd.prec = c->prec;
  hd.nx = s.nx;
  hd.ny = s.ny;
  hd.nz = s.nz;
  hd.gs = (int32_t)gs_bytes(c);
  hd.has_ref = use_ref(c, s) ? 1 : 0;
  hd.ref_age = s.ref_age;
  hd.bytes = need;
  CkptRun& r = hd.run;
  r.tau = h.tau;
  r.torque = h.torque;
  r.energy = h.energy;
  for (int q = 0; q < 4; ++q) r.eterm[q] = h.eterm[q];
  r.ss = h.ss;
  r.sy = h.sy;
  r.yy = h.yy;
  r.best_torque = h.best_torque;
  r.tol = h.tol;
  r.tau0 = h.tau0;
  r.k = h.k;
  r.best_k = h.best_k;
  r.evals = h.evals;
  r.max_iter = h.max_iter;
  r.stall_iters = h.stall_iters;
  r.done = h.done;
  r.mode = h.mode;
  r.last_tau = h.last_tau;
  r.last_k = h.last_k;
  r.pending = h.pending;
  for (int q = 0; q < 3; ++q) r.H[q] = h.H[q];
  r.bb_switch = h.bb_switch;
  unsigned char* p = static_cast<unsigned char*>(host);
  std::memcpy(p, &hd, sizeof(hd));
  p += sizeof(hd);
  const size_t gsb = 3ull * s.N * gs_bytes(c), db = 3ull * s.N * sizeof(double);
  HIPCHK(c, hipMemcpyAsync(p, s.g, gsb, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(p + gsb, s.s, gsb, hipMemcpyDeviceToHost, c->stream));
  if (hd.has_ref) {
    HIPCHK(c, hipMemcpyAsync(p + 2 * gsb, s.mref, db, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(p + 2 * gsb + db, s.hdref, db, hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MM_OK;
}

int mm_state_load(mm_ctx* c, int sample, const void* host, int64_t bytes) {
  int rc = check_sample(c, sample, true);
  if (rc != MM_OK) return rc;
  if (!host) return fail(c, MM_EINVAL, "null buffer");
  if (c->ls.on) return fail(c, MM_EINVAL, "a line-search run is not checkpointed");
  Sample& s = c->smp[sample];
  if (bytes < (int64_t)sizeof(CkptHeader)) return fail(c, MM_EINVAL, "checkpoint too short");
  CkptHeader hd;
  std::memcpy(&hd, host, sizeof(hd));
  if (std::memcmp(hd.magic, kCkptMagic, sizeof(kCkptMagic)) != 0 || hd.version != 1)
    return fail(c, MM_EINVAL, "not a checkpoint of this library");
  if (hd.prec != c->prec || hd.nx != s.nx || hd.ny != s.ny || hd.nz != s.nz ||
      hd.gs != (int32_t)gs_bytes(c) || hd.has_ref != (use_ref(c, s) ? 1 : 0))
    return fail(c, MM_EINVAL, "checkpoint of another precision, grid or correction setting");
  const int64_t need = ckpt_bytes(c, s);
  if (hd.bytes != need || bytes < need) return fail(c, MM_EINVAL, "checkpoint size mismatch");
  {
    const CkptRun& r = hd.run;
    const bool ok = std::isfinite(r.H[0]) && std::isfinite(r.H[1]) && std::isfinite(r.H[2]) &&
                    std::isfinite(r.tau) && std::isfinite(r.last_tau) && r.k >= 0 &&
                    r.last_k >= 0 && r.evals >= 0 && r.mode >= 0 && r.mode <= 2 &&
                    r.pending >= 0 && r.pending <= 1 && r.done >= -1 && r.done <= 3 &&
                    hd.ref_age >= 0;
    if (!ok) return fail(c, MM_EINVAL, "checkpoint holds an invalid run state");
  }
  rc = read_state(c, s);   // the device state's pointers and slots are kept
  if (rc != MM_OK) return rc;
  MinState& h = *s.st_host;
  const CkptRun& r = hd.run;
  h.tau = r.tau;
  h.torque = r.torque;
  h.energy = r.energy;
  for (int q = 0; q < 4; ++q) h.eterm[q] = r.eterm[q];
  h.ss = r.ss;
  h.sy = r.sy;
  h.yy = r.yy;
  h.best_torque = r.best_torque;
  h.tol = r.tol;
  h.tau0 = r.tau0;
  h.k = r.k;
  h.best_k = r.best_k;
  h.evals = r.evals;
  h.max_iter = r.max_iter;
  h.stall_iters = r.stall_iters;
  h.done = r.done;
  h.mode = r.mode;
  h.last_tau = r.last_tau;
  h.last_k = r.last_k;
  h.pending = r.pending;
  for (int q = 0; q < 3; ++q) h.H[q] = r.H[q];
  h.bb_switch = r.bb_switch;
  h.sweep = 0;
  h.ls_trial = h.ls_retry = h.ls_nb = 0;
  h.ls_C = h.ls_Q = h.ls_G = 0.0;
  h.fin_err = 0;
  for (int q = 0; q < 3; ++q) s.H[q] = r.H[q];
  s.fin_pending = false;
  s.ref_age = hd.ref_age;
  const unsigned char* p = static_cast<const unsigned char*>(host) + sizeof(hd);
  const size_t gsb = 3ull * s.N * gs_bytes(c), db = 3ull * s.N * sizeof(double);
  HIPCHK(c, hipMemcpyAsync(s.st, s.st_host, sizeof(MinState), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(s.g, p, gsb, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(s.s, p + gsb, gsb, hipMemcpyHostToDevice, c->stream));
  if (hd.has_ref) {
    HIPCHK(c, hipMemcpyAsync(s.mref, p + 2 * gsb, db, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(s.hdref, p + 2 * gsb + db, db, hipMemcpyHostToDevice, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MM_OK;
}

int mm_mean(mm_ctx* c, int sample, const double* m, double* mavg) {
  int rc = check_sample(c, sample, false);
  if (rc != MM_OK) return rc;
  if (!m || !mavg) return fail(c, MM_EINVAL, "null buffer");
  Sample& s = c->smp[sample];
  launch_mean(c->stream, m, s.N, s.partials, s.dev3);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(s.host3, s.dev3, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int q = 0; q < 3; ++q) mavg[q] = s.host3[q];
  return MM_OK;
}

int mm_hysteresis_sweep(mm_ctx* c, double* const* m, const double* H, int n_fields, double tol,
                        int64_t max_iter, double* m_avg, int64_t* iters) {
  if (!c) return MM_EINVAL;
  if (!m || !H || !m_avg || n_fields < 0 || !(tol >= 0) || max_iter < 0)
    return fail(c, MM_EINVAL, "bad argument");
  const int S = (int)c->smp.size();
  for (int k = 0; k < S; ++k) {
    int rc = check_sample(c, k, true);
    if (rc != MM_OK) return rc;
    if (!m[k]) return fail(c, MM_EINVAL, "null magnetisation pointer");
  }
  for (size_t q = 0; q < (size_t)S * n_fields * 3; ++q)
    if (!std::isfinite(H[q])) return fail(c, MM_EINVAL, "fields must be finite");
  if (n_fields == 0) return MM_OK;
  hipStream_t st = c->stream;
  const size_t nf3 = (size_t)S * n_fields * 3;
  double* fields = nullptr;
  double* mavg = nullptr;
  long long* its = nullptr;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(st);
    dfree(fields);
    dfree(mavg);
    dfree(its);
  };
  // a failed HIP call frees the sweep's tables before it returns
#define SWEEP_CHK(expr)                                                          \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) {                                                      \
      cleanup();                                                                 \
      return fail(c, MM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    }                                                                            \
  } while (0)
  if (hipMalloc((void**)&fields, nf3 * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&mavg, nf3 * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&its, (size_t)S * n_fields * sizeof(long long)) != hipSuccess) {
    cleanup();
    (void)hipGetLastError();
    return fail(c, MM_ENOMEM, "device allocation for the sweep tables failed");
  }
  SWEEP_CHK(hipMemcpyAsync(fields, H, nf3 * sizeof(double), hipMemcpyHostToDevice, st));
  // every sample runs its whole field list on the device; the host polls
  for (int k = 0; k < S; ++k) {
    Sample& s = c->smp[k];
    for (int q = 0; q < 3; ++q) s.H[q] = H[((size_t)k * n_fields) * 3 + q];
    const int lrc = ensure_ls(c, s);
    if (lrc != MM_OK) {
      cleanup();
      return lrc;
    }
    reset_run(c, st, s, tol, (long long)max_iter);
    launch_sweep_start(st, s.st, fields + (size_t)k * n_fields * 3, n_fields,
                       mavg + (size_t)k * n_fields * 3, its + (size_t)k * n_fields, 1.0 / s.N);
    s.ref_age = kRefStale;
  }
  std::unique_ptr<BatchPlan> plan(new BatchPlan);
  std::vector<char> in_batch(S, 0);
  if (c->batched && S > 1) {
    int rc = build_batch(c, m, *plan);
    if (rc != MM_OK) {
      cleanup();
      return rc;
    }
    if (plan->members.size() < 2) plan->members.clear();
    for (int k : plan->members) in_batch[k] = 1;
    if (!plan->members.empty() && c->concurrent_groups) {
      rc = ensure_aux(c);
      if (rc != MM_OK) {
        cleanup();
        return rc;
      }
    }
  }
  // a captured batch of iterations is replayed when the stream allows it
  const bool graph = c->use_graph && c->stream != nullptr && c->prof == 0 && !plan->members.empty();
  std::vector<char> running(S, 1);
  int left = S;
  int batch_left = (int)plan->members.size();
  int polls = 0;
  bool eager = true;   // a new plan's first poll runs eagerly, later ones replay its graph
  while (left > 0) {
    if (batch_left > 0) {
      // the first batch runs eagerly (kernel attributes are set there); later
      // batches replay one captured graph of poll_every iterations
      if (graph && !eager) {
        if (!plan->graph) {
          hipGraph_t g = nullptr;
          hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
          if (e == hipSuccess) {
            enqueue_batched_reference(c, *plan);
            for (int q = 0; q < c->poll_every; ++q) enqueue_batched_iteration(c, *plan);
            e = hipStreamEndCapture(c->stream, &g);
          }
          if (e == hipSuccess) e = hipGraphInstantiate(&plan->graph, g, nullptr, nullptr, 0);
          if (g) (void)hipGraphDestroy(g);
          if (e != hipSuccess) {
            cleanup();
            return fail(c, MM_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
          }
        }
        SWEEP_CHK(hipGraphLaunch(plan->graph, c->stream));
      } else {
        enqueue_batched_reference(c, *plan);
        for (int q = 0; q < c->poll_every; ++q) enqueue_batched_iteration(c, *plan);
      }
    }
    for (int k = 0; k < S; ++k) {
      if (!running[k] || in_batch[k]) continue;
      for (int q = 0; q < c->poll_every; ++q) enqueue_iteration(c, c->smp[k], m[k], q);
      flush_finish(c, c->smp[k]);
    }
    ++polls;
    eager = false;
    hipError_t e = hipGetLastError();
    for (int k = 0; k < S && e == hipSuccess; ++k)
      if (running[k])
        e = hipMemcpyAsync(c->smp[k].st_host, c->smp[k].st, sizeof(MinState),
                           hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      cleanup();
      return fail(c, MM_EHIP, std::string("sweep: ") + hipGetErrorString(e));
    }
    prof_collect(c);
    for (int k = 0; k < S; ++k)
      if (running[k] && c->smp[k].st_host->fin_err != 0) {
        cleanup();
        return fail(c, MM_ESTATE, "a forward x pass gave up waiting for the finish decision");
      }
    for (int k = 0; k < S; ++k)
      if (running[k] && c->smp[k].st_host->done != 0) {
        running[k] = 0;
        --left;
        if (in_batch[k]) --batch_left;
      }
    // once the running samples are at most the batch_rebuild fraction of the
    // plan's, the tables are rebuilt from them (and the graph captured
    // again), so that the launches stop walking finished samples' blocks;
    // results do not change, every sample's blocks and reductions being its
    // own
    if (batch_left >= 2 && c->batch_rebuild > 0.0 &&
        batch_left <= c->batch_rebuild * (double)plan->members.size()) {
      std::unique_ptr<BatchPlan> np(new BatchPlan);
      const int rc = build_batch(c, m, *np, &running);
      if (rc != MM_OK) {
        cleanup();
        return rc;
      }
      if (np->members.size() < 2) np->members.clear();
      std::fill(in_batch.begin(), in_batch.end(), 0);
      for (int k : np->members) in_batch[k] = 1;
      batch_left = (int)np->members.size();
      plan.swap(np);
      eager = true;
    }
  }
  std::vector<long long> ih((size_t)S * n_fields);
  SWEEP_CHK(hipMemcpyAsync(m_avg, mavg, nf3 * sizeof(double), hipMemcpyDeviceToHost, st));
  SWEEP_CHK(hipMemcpyAsync(ih.data(), its, ih.size() * sizeof(long long), hipMemcpyDeviceToHost, st));
  cleanup();
  int worst = MM_OK;
  for (int k = 0; k < S; ++k) {
    Sample& s = c->smp[k];
    for (int q = 0; q < 3; ++q) s.H[q] = H[((size_t)k * n_fields + n_fields - 1) * 3 + q];
    s.evals_total += s.st_host->evals;
    for (int f = 0; f < n_fields; ++f) s.iters_total += ih[(size_t)k * n_fields + f];
    const int d = s.st_host->done;
    if (d == -1) return fail(c, MM_ENONFINITE, "non-finite torque or energy in the sweep");
    const int code = status_of(d);
    if (code > worst) worst = code;
  }
  if (iters)
    for (size_t q = 0; q < ih.size(); ++q) iters[q] = ih[q];
  return worst;
}
#undef SWEEP_CHK

int mm_set_option(mm_ctx* c, const char* key, double value) {
  if (!c || !key) return MM_EINVAL;
  if (!std::isfinite(value)) return fail(c, MM_EINVAL, "option value must be finite");
  if (!std::strcmp(key, "tau0")) {
    if (value < 0) return fail(c, MM_EINVAL, "tau0 must be >= 0");
    c->tau0 = value;
  } else if (!std::strcmp(key, "poll_every")) {
    if (value < 1 || value > 100000) return fail(c, MM_EINVAL, "poll_every out of range");
    c->poll_every = (int)value;
  } else if (!std::strcmp(key, "bb_switch")) {
    if (!(value >= 0.0) || !std::isfinite(value))
      return fail(c, MM_EINVAL, "bb_switch must be finite and >= 0");
    c->bb_switch = value;
  } else if (!std::strcmp(key, "line_search")) {
    if (value != 0.0 && value != 1.0) return fail(c, MM_EINVAL, "line_search is 0 or 1");
    c->ls.on = value != 0.0;
  } else if (!std::strcmp(key, "ls_eta")) {
    if (!(value >= 0.0 && value <= 1.0)) return fail(c, MM_EINVAL, "ls_eta must be in [0, 1]");
    c->ls.eta = value;
  } else if (!std::strcmp(key, "ls_rho")) {
    if (!(value > 0.0 && value < 1.0)) return fail(c, MM_EINVAL, "ls_rho must be in (0, 1)");
    c->ls.rho = value;
  } else if (!std::strcmp(key, "ls_sigma")) {
    if (!(value > 0.0 && value < 1.0)) return fail(c, MM_EINVAL, "ls_sigma must be in (0, 1)");
    c->ls.sigma = value;
  } else if (!std::strcmp(key, "ls_max")) {
    if (value < 0 || value > 1000 || value != std::floor(value))
      return fail(c, MM_EINVAL, "ls_max must be an integer in 0..1000");
    c->ls.max_back = (int)value;
  } else if (!std::strcmp(key, "stall_iters")) {
    if (value < 0) return fail(c, MM_EINVAL, "stall_iters must be >= 0");
    c->stall_iters = (long long)value;
  } else if (!std::strcmp(key, "use_graph")) {
    c->use_graph = value != 0.0;
  } else if (!std::strcmp(key, "batched")) {
    c->batched = value != 0.0;
  } else if (!std::strcmp(key, "refine")) {
    c->refine = value != 0.0;
  } else if (!std::strcmp(key, "mixed_radix")) {
    c->mixed_radix = value != 0.0;
  } else if (!std::strcmp(key, "concurrent_groups")) {
    c->concurrent_groups = value != 0.0;
  } else if (!std::strcmp(key, "batch_rebuild")) {
    if (!(value >= 0.0 && value < 1.0))
      return fail(c, MM_EINVAL, "batch_rebuild is a fraction in [0, 1)");
    c->batch_rebuild = value;
  } else if (!std::strcmp(key, "persistent")) {
    c->persistent = value != 0.0;
  } else if (!std::strcmp(key, "fused_finish")) {
    c->fused_finish = value != 0.0;
  } else if (!std::strcmp(key, "fin_spin")) {
    if (!(value >= 0.0 && value <= (double)(1 << 30)) || value != std::floor(value))
      return fail(c, MM_EINVAL, "fin_spin is an integer in [0, 2^30]");
    c->fin_spin = (int)value;
  } else if (!std::strcmp(key, "autotune")) {
    c->autotune = value != 0.0;
  } else if (!std::strcmp(key, "yz_variant")) {
    if (value != -1 && value != 0 && value != 1)
      return fail(c, MM_EINVAL, "yz_variant is -1 (automatic), 0 or 1");
    c->yz_forced = (int)value;
  } else if (!std::strcmp(key, "rows_per_block")) {
    if (value < 0 || value > 64 || value != std::floor(value))
      return fail(c, MM_EINVAL, "rows_per_block is 0 (automatic) or a tile size");
    c->rows_forced = (int)value;
  } else if (!std::strcmp(key, "demag_path")) {
    if (value != 0 && value != 1 && value != 2) return fail(c, MM_EINVAL, "demag_path is 0, 1 or 2");
    c->path_pref = (int)value;
  } else {
    return fail(c, MM_EINVAL, std::string("unknown option ") + key);
  }
  return MM_OK;
}

int mm_rows_per_block(mm_ctx* c, int sample, int* rows) {
  int rc = check_sample(c, sample, false);
  if (rc != MM_OK) return rc;
  if (!rows) return fail(c, MM_EINVAL, "null pointer");
  *rows = c->smp[sample].R3;
  return MM_OK;
}

int mm_yz_variant(mm_ctx* c, int sample, int* var) {
  int rc = check_sample(c, sample, false);
  if (rc != MM_OK) return rc;
  if (!var) return fail(c, MM_EINVAL, "null pointer");
  *var = c->smp[sample].yz_var;
  return MM_OK;
}

int mm_counters(mm_ctx* c, int sample, int64_t* heff_evals, int64_t* iters) {
  int rc = check_sample(c, sample, false);
  if (rc != MM_OK) return rc;
  if (heff_evals) *heff_evals = c->smp[sample].evals_total;
  if (iters) *iters = c->smp[sample].iters_total;
  return MM_OK;
}

int mm_last_step(mm_ctx* c, int sample, mm_step_info* info) {
  int rc = check_sample(c, sample, false);
  if (rc != MM_OK) return rc;
  if (!info) return fail(c, MM_EINVAL, "null pointer");
  Sample& s = c->smp[sample];
  rc = read_state(c, s);
  if (rc != MM_OK) return rc;
  info->tau = s.st_host->last_tau;
  info->torque = s.st_host->torque;
  info->energy = s.st_host->energy;
  info->k = s.st_host->last_k;
  return MM_OK;
}

int mm_profile(mm_ctx* c, int mask) {
  if (!c || mask < 0) return MM_EINVAL;
  prof_collect(c);
  c->prof = (unsigned)mask & ((1u << kNumKernels) - 1u);
  if (c->prof)
    for (int k = 0; k < kNumKernels; ++k) {
      c->prof_ms[k] = 0;
      c->prof_n[k] = 0;
    }
  return MM_OK;
}

int mm_profile_read(mm_ctx* c, int id, double* total_ms, int64_t* launches) {
  if (!c || id < 0 || id >= kNumKernels) return MM_EINVAL;
  prof_collect(c);
  if (total_ms) *total_ms = c->prof_ms[id];
  if (launches) *launches = c->prof_n[id];
  return MM_OK;
}

const char* mm_kernel_name(int id) {
  if (id < 0 || id >= kNumKernels) return nullptr;
  return kKernelNames[id];
}

int mm_kernel_bytes(mm_ctx* c, int sample, int id, double* bytes) {
  int rc = check_sample(c, sample, false);
  if (rc != MM_OK) return rc;
  if (!bytes || id < 0 || id >= kNumKernels) return fail(c, MM_EINVAL, "bad argument");
  const Sample& s = c->smp[sample];
  const double sr = single(c) ? 4.0 : 8.0;
  const double N3 = 3.0 * s.N * 8.0;                                  // one [3][N] double array
  const double G3 = 3.0 * s.N * sr;                                   // g or s (transform type)
  const double spec = (double)(s.M + 1) * 3 * s.nz * s.ny * 2 * sr;   // spectrum A
  const double trows = s.path == PATH_3D ? (double)(s.Py / 2 + 1) : 1.0;
  const double tens = (double)(s.M + 1) * trows * s.tstride * sr;
  const double bsp = s.path == PATH_3D ? (double)(s.M + 1) * s.Py * 3 * s.nz * 2 * sr : 0.0;
  const double ku = s.ku_map ? s.N * 8.0 : 0.0;
  const bool thin = s.path == PATH_THIN;
  const double corr = use_ref(c, s) ? N3 : 0.0;   // mref in (xf), hdref in (xil)
  // reference pass (double precision): xf m in, mref and spectrum out; y/z
  // stages; xil spectrum and m in, hdref out
  const double spec64 = (double)(s.M + 1) * 3 * s.nz * s.ny * 16.0;
  const double tens64 = (double)(s.M + 1) * trows * s.rtstride * 8.0;
  const double bsp64 = s.path == PATH_3D ? (double)(s.M + 1) * s.Py * 3 * s.nz * 16.0 : 0.0;
  const double mid64 = thin ? 2 * spec64 + tens64 : 2 * spec64 + 4 * bsp64 + tens64;
  double b = 0;
  switch (id) {
    case KID_XF: b = 2 * N3 + 2 * G3 + spec + corr; break;   // m, g in; m, s out; spectrum out
    case KID_YZ: b = thin ? 2 * spec + tens : 0; break;   // spectrum in/out; tensor in
    case KID_XIL: b = spec + N3 + 3 * G3 + ku + corr; break;   // spectrum, m, g, s in; g out
    case KID_REF: b = s.has_ref ? 4 * N3 + 2 * spec64 + mid64 + ku : 0; break;
    case KID_UPDATE: b = 2 * N3 + 2 * G3; break;    // m, g in; m, s out
    case KID_Y3F: b = thin ? 0 : spec + bsp; break; // spectrum in, y spectrum out
    case KID_Z3: b = thin ? 0 : 2 * bsp + tens; break;    // y spectrum in/out; tensor in
    case KID_Y3I: b = thin ? 0 : bsp + spec; break;
    case KID_FINISH: b = (double)s.nb3 * kNPartial * 8.0; break;   // per-block sums
  }
  *bytes = b;
  return MM_OK;
}

int mm_hessvec(mm_ctx* c, int sample, const double* m, const double* v, double* out) {
  int rc = check_sample(c, sample, true);
  if (rc != MM_OK) return rc;
  if (!m || !v || !out) return fail(c, MM_EINVAL, "null buffer");
  Sample& s = c->smp[sample];
  rc = ensure_adj(c, s);
  if (rc != MM_OK) return rc;
  enqueue_heff_m(c, s, m);
  launch_project(c->stream, m, v, s.cp, s.N);     // the operator acts on tangent fields
  enqueue_hlin(c, s, s.cp, nullptr);
  launch_hess_apply(c->stream, m, s.Hm, s.Hlin, s.cp, out, s.N, kMu0Host * s.Ms * s.V, nullptr,
                    nullptr);
  HIPCHK(c, hipGetLastError());
  return MM_OK;
}

int mm_adjoint_solve(mm_ctx* c, int sample, const double* m, const double* rhs, double* lam,
                     double tol, int64_t max_iter, int64_t* iters, double* resid) {
  int rc = check_sample(c, sample, true);
  if (rc != MM_OK) return rc;
  if (!m || !rhs || !lam || !(tol >= 0) || max_iter < 0) return fail(c, MM_EINVAL, "bad argument");
  Sample& s = c->smp[sample];
  rc = ensure_adj(c, s);
  if (rc != MM_OK) return rc;
  hipStream_t st = c->stream;
  enqueue_heff_m(c, s, m);
  launch_cg_init(st, m, rhs, lam, s.cr, s.cp, s.N, s.partials, s.cg, tol, (long long)max_iter);
  const double cH = kMu0Host * s.Ms * s.V;
  const int* done = &s.cg->done;
  for (;;) {
    for (int q = 0; q < c->poll_every; ++q) {
      enqueue_hlin(c, s, s.cp, done);
      launch_hess_apply(st, m, s.Hm, s.Hlin, s.cp, s.cAp, s.N, cH, s.partials, done);
      launch_cg_step(st, m, lam, s.cr, s.cp, s.cAp, s.N, s.partials, s.cg);
    }
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(s.cg_host, s.cg, sizeof(CGState), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    prof_collect(c);
    if (s.cg_host->done != 0) break;
  }
  const CGState& h = *s.cg_host;
  if (iters) *iters = h.k;
  if (resid) *resid = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
  if (h.done == -1)
    return fail(c, MM_ENONFINITE,
                "conjugate gradients broke down: the Hessian is not positive definite along a "
                "search direction (m is not a strict local minimum) or a value is not finite");
  return h.done == 1 ? MM_OK : MM_NOT_CONVERGED;
}

int mm_param_grads(mm_ctx* c, int sample, const double* m, const double* lam, double* dJ_dA,
                   double* dJ_dMs, double* dJ_dH, double* dJ_dKu) {
  int rc = check_sample(c, sample, true);
  if (rc != MM_OK) return rc;
  if (!m || !lam) return fail(c, MM_EINVAL, "null buffer");
  Sample& s = c->smp[sample];
  rc = ensure_adj(c, s);
  if (rc != MM_OK) return rc;
  EvalOut o;
  o.Hd = s.Hd;
  o.Hex = s.Hlin;
  o.unit_A = true;
  enqueue_eval(c, s, m, o);
  launch_param_grads(c->stream, m, lam, s.Hd, s.Hlin, s.H, s.u, s.V, dJ_dKu, s.N, s.partials,
                     s.scal);
  HIPCHK(c, hipGetLastError());
  rc = read_scal(c, s, 5);
  if (rc != MM_OK) return rc;
  prof_collect(c);
  if (dJ_dA) *dJ_dA = kMu0Host * s.Ms * s.V * s.scal_host[0];
  if (dJ_dMs) *dJ_dMs = kMu0Host * s.V * s.scal_host[1];
  if (dJ_dH)
    for (int q = 0; q < 3; ++q) dJ_dH[q] = kMu0Host * s.Ms * s.V * s.scal_host[2 + q];
  return MM_OK;
}

int mm_energy_grads(mm_ctx* c, int sample, const double* m, double* dU_dm, double* dU_dKu,
                    double* scal5) {
  int rc = check_sample(c, sample, true);
  if (rc != MM_OK) return rc;
  if (!m) return fail(c, MM_EINVAL, "null buffer");
  Sample& s = c->smp[sample];
  rc = ensure_adj(c, s);
  if (rc != MM_OK) return rc;
  hipStream_t st = c->stream;
  // energy terms and H_eff(m)
  launch_reset_state(st, s.st_eval, 0.0, 0.0, 0, 0, 2, s.H);
  EvalOut o;
  o.H = s.Hm;
  o.st_fin = s.st_eval;
  enqueue_eval(c, s, m, o);
  launch_energy_grads(st, m, s.Hm, -kMu0Host * s.Ms * s.V, dU_dm, s.u, s.V, dU_dKu, s.N,
                      s.partials, s.scal);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(s.st_host, s.st_eval, sizeof(MinState), hipMemcpyDeviceToHost, st));
  rc = read_scal(c, s, 3);
  if (rc != MM_OK) return rc;
  const double Ud = s.st_host->eterm[0], Uex = s.st_host->eterm[1], Uz = s.st_host->eterm[3];
  double dA = 0.0;
  if (s.A > 0) {
    dA = Uex / s.A;
  } else {
    // U_ex is linear in A: its value at A = 1
    launch_reset_state(st, s.st_eval, 0.0, 0.0, 0, 0, 2, s.H);
    EvalOut o1;
    o1.st_fin = s.st_eval;
    o1.unit_A = true;
    enqueue_eval(c, s, m, o1);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(s.st_host, s.st_eval, sizeof(MinState), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    dA = s.st_host->eterm[1];
  }
  prof_collect(c);
  if (scal5) {
    scal5[0] = (2.0 * Ud + Uz) / s.Ms;
    scal5[1] = dA;
    for (int q = 0; q < 3; ++q) scal5[2 + q] = -kMu0Host * s.Ms * s.V * s.scal_host[q];
  }
  return MM_OK;
}

const char* mm_strerror(int code) {
  switch (code) {
    case MM_OK: return "ok";
    case MM_NOT_CONVERGED: return "not converged within max_iter";
    case MM_STALLED: return "torque stopped decreasing (precision floor)";
    case MM_EINVAL: return "invalid argument";
    case MM_ENOMEM: return "device allocation failed";
    case MM_EHIP: return "HIP runtime error";
    case MM_ENONFINITE: return "non-finite value";
    case MM_ESTATE: return "call out of order";
    case MM_EUNSUPPORTED: return "grid shape not supported";
    default: return "unknown status";
  }
}

const char* mm_last_error(const mm_ctx* c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"
