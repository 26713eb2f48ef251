// Host-side sanitizer run of the library: every entry point of include/mm.h
// driven through its host logic (argument checks, buffer and table set-up,
// batch tables, graph capture, checkpoints, error paths) in a program whose
// host code is built with AddressSanitizer and UndefinedBehaviorSanitizer
// (device code unchanged).  Exits 0 only if every call returns what it
// should and no sanitizer reports; it prints each step before it runs.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "mm.h"

namespace {

int g_fail = 0;

void step(const char* what) {
  std::printf("step: %s\n", what);
  std::fflush(stdout);
}

void expect(int rc, int want, const char* what) {
  if (rc != want) {
    std::printf("FAIL %s: rc %d, expected %d\n", what, rc, want);
    ++g_fail;
  }
}

void expect_ok_or(int rc, int alt, const char* what) {
  if (rc != MM_OK && rc != alt) {
    std::printf("FAIL %s: rc %d\n", what, rc);
    ++g_fail;
  }
}

struct Dev {
  double* p = nullptr;
  size_t n = 0;
  explicit Dev(size_t count) : n(count) {
    if (hipMalloc((void**)&p, n * sizeof(double)) != hipSuccess) {
      std::printf("FAIL hipMalloc\n");
      std::exit(2);
    }
  }
  ~Dev() { (void)hipFree(p); }
  void put(const std::vector<double>& h) {
    (void)hipMemcpy(p, h.data(), n * sizeof(double), hipMemcpyHostToDevice);
  }
  std::vector<double> get() const {
    std::vector<double> h(n);
    (void)hipMemcpy(h.data(), p, n * sizeof(double), hipMemcpyDeviceToHost);
    return h;
  }
};

// Unit vectors tilted from +x with a deterministic perturbation per cell.
std::vector<double> start_state(int nx, int ny, int nz, unsigned seed) {
  const size_t N = (size_t)nx * ny * nz;
  std::vector<double> m(3 * N);
  unsigned s = seed;
  auto rnd = [&]() {
    s = s * 1664525u + 1013904223u;
    return (double)(s >> 8) / 16777216.0 - 0.5;
  };
  for (size_t i = 0; i < N; ++i) {
    double v[3] = {0.87 + 0.3 * rnd(), 0.5 + 0.3 * rnd(), 0.3 * rnd()};
    const double r = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int c = 0; c < 3; ++c) m[c * N + i] = v[c] / r;
  }
  return m;
}

struct Shape {
  int nx, ny, nz;
};

void run_context(int prec) {
  const char* pname = prec == MM_FP64 ? "fp64" : "mixed";
  std::printf("== context %s\n", pname);
  // a wave-FFT film, a short film on the LDS fallback path, a 3-D grid
  const Shape shp[3] = {{64, 32, 2}, {20, 12, 1}, {12, 10, 8}};
  mm_ctx* ctx = nullptr;
  step("create");
  expect(mm_create(&ctx, prec, 3, nullptr), MM_OK, "mm_create");
  if (!ctx) return;
  step("calls before geometry");
  {
    double H[3] = {1e3, 0, 0};
    expect(mm_set_field(ctx, 0, H), MM_ESTATE, "set_field before geometry");
    expect(mm_set_geometry(ctx, 5, 4, 4, 1, 1e-9, 1e-9, 1e-9), MM_EINVAL, "sample index");
    expect(mm_set_option(ctx, "no_such_option", 1.0), MM_EINVAL, "unknown option");
    std::printf("  last error: %s\n", mm_last_error(ctx));
  }
  step("geometry, material, field");
  for (int s = 0; s < 3; ++s) {
    expect(mm_set_geometry(ctx, s, shp[s].nx, shp[s].ny, shp[s].nz, 5e-9, 5e-9, 5e-9), MM_OK,
           "set_geometry");
    const double u[3] = {1, 0, 0};
    expect(mm_set_material(ctx, s, 8e5, 1.3e-11, 500.0, u, nullptr), MM_OK, "set_material");
    const double H[3] = {-4e3, 1.5e3, 0.0};
    expect(mm_set_field(ctx, s, H), MM_OK, "set_field");
  }
  std::vector<Dev*> m, H;
  for (int s = 0; s < 3; ++s) {
    const size_t n3 = 3ull * shp[s].nx * shp[s].ny * shp[s].nz;
    m.push_back(new Dev(n3));
    H.push_back(new Dev(n3));
    m[s]->put(start_state(shp[s].nx, shp[s].ny, shp[s].nz, 17u + s));
  }
  step("field evaluations");
  for (int s = 0; s < 3; ++s) {
    expect(mm_heff(ctx, s, m[s]->p, H[s]->p), MM_OK, "heff");
    expect(mm_heff_static(ctx, s, m[s]->p, H[s]->p), MM_OK, "heff_static");
    expect(mm_field_terms(ctx, s, m[s]->p, H[s]->p, nullptr, nullptr), MM_OK, "field_terms");
    double E = 0, terms[4];
    expect(mm_energy(ctx, s, m[s]->p, &E, terms), MM_OK, "energy");
    double mavg[3];
    expect(mm_mean(ctx, s, m[s]->p, mavg), MM_OK, "mean");
    if (!std::isfinite(E)) {
      std::printf("FAIL energy not finite\n");
      ++g_fail;
    }
  }
  expect(mm_heff(ctx, 0, nullptr, H[0]->p), MM_EINVAL, "heff null m");
  step("steps, checkpoint, continuation");
  for (int s = 0; s < 3; ++s) {
    mm_step_info info;
    for (int k = 0; k < 6; ++k) expect(mm_minimize_step(ctx, s, m[s]->p, &info), MM_OK, "step");
    int64_t bytes = 0;
    expect(mm_state_bytes(ctx, s, &bytes), MM_OK, "state_bytes");
    std::vector<unsigned char> blob((size_t)bytes);
    expect(mm_state_save(ctx, s, blob.data(), bytes), MM_OK, "state_save");
    expect(mm_state_save(ctx, s, blob.data(), bytes - 1), MM_EINVAL, "state_save short");
    expect(mm_state_load(ctx, s, blob.data(), 16), MM_EINVAL, "state_load short");
    std::vector<unsigned char> bad(blob);
    bad[0] ^= 0xff;
    expect(mm_state_load(ctx, s, bad.data(), bytes), MM_EINVAL, "state_load foreign");
    expect(mm_state_load(ctx, (s + 1) % 3, blob.data(), bytes), MM_EINVAL, "state_load other grid");
    expect(mm_state_load(ctx, s, blob.data(), bytes), MM_OK, "state_load");
    mm_min_result r;
    expect_ok_or(mm_minimize_continue(ctx, s, m[s]->p, 1e-6, 3000, &r), MM_NOT_CONVERGED,
                 "continue");
    expect_ok_or(mm_minimize_to_tol(ctx, s, m[s]->p, 1e-6, 3000, &r), MM_NOT_CONVERGED, "to_tol");
    expect(mm_last_step(ctx, s, &info), MM_OK, "last_step");
    int64_t ev = 0, it = 0;
    expect(mm_counters(ctx, s, &ev, &it), MM_OK, "counters");
  }
  step("derivatives");
  if (prec == MM_FP64) {
    for (int s = 0; s < 3; ++s) {
      const size_t n3 = m[s]->n, N = n3 / 3;
      Dev v(n3), out(n3), lam(n3), dku(N);
      v.put(std::vector<double>(n3, 0.0));
      double scal5[5];
      expect(mm_energy_grads(ctx, s, m[s]->p, out.p, dku.p, scal5), MM_OK, "energy_grads");
      expect(mm_hessvec(ctx, s, m[s]->p, out.p, v.p), MM_OK, "hessvec");
      int64_t its = 0;
      double res = 0;
      const int rc = mm_adjoint_solve(ctx, s, m[s]->p, out.p, lam.p, 1e-6, 50, &its, &res);
      if (rc != MM_OK && rc != MM_NOT_CONVERGED && rc != MM_ENONFINITE) {
        std::printf("FAIL adjoint_solve rc %d\n", rc);
        ++g_fail;
      }
      double dA, dMs, dH[3];
      expect(mm_param_grads(ctx, s, m[s]->p, lam.p, &dA, &dMs, dH, dku.p), MM_OK, "param_grads");
    }
  }
  step("sweeps: persistent batched, grouped, per sample");
  const int F = 4;
  std::vector<double> fields(3 * F * 3);
  for (int s = 0; s < 3; ++s)
    for (int f = 0; f < F; ++f) {
      fields[(s * F + f) * 3 + 0] = 2e4 - 1.2e4 * f;
      fields[(s * F + f) * 3 + 1] = 300.0;
      fields[(s * F + f) * 3 + 2] = 0.0;
    }
  std::vector<double> mavg(3 * F * 3);
  std::vector<int64_t> iters(3 * F);
  double* mp[3] = {m[0]->p, m[1]->p, m[2]->p};
  const double variants[3][2] = {{1, 1}, {1, 0}, {0, 0}};   // batched, persistent
  for (const auto& v : variants) {
    expect(mm_set_option(ctx, "batched", v[0]), MM_OK, "option batched");
    expect(mm_set_option(ctx, "persistent", v[1]), MM_OK, "option persistent");
    expect_ok_or(mm_hysteresis_sweep(ctx, mp, fields.data(), F, 1e-5, 2000, mavg.data(),
                                     iters.data()),
                 MM_NOT_CONVERGED, "sweep");
  }
  expect(mm_hysteresis_sweep(ctx, mp, fields.data(), -1, 1e-5, 10, mavg.data(), nullptr),
         MM_EINVAL, "sweep negative field count");
  step("profiling calls");
  expect(mm_profile(ctx, 0xff), MM_OK, "profile on");
  {
    mm_min_result r;
    expect_ok_or(mm_minimize_to_tol(ctx, 0, m[0]->p, 1e-9, 40, &r), MM_NOT_CONVERGED, "profiled run");
  }
  for (int id = 0; mm_kernel_name(id) != nullptr; ++id) {
    double ms = 0, bytes = 0;
    int64_t launches = 0;
    expect(mm_profile_read(ctx, id, &ms, &launches), MM_OK, "profile_read");
    (void)mm_kernel_bytes(ctx, 0, id, &bytes);
  }
  expect(mm_profile(ctx, 0), MM_OK, "profile off");
  for (int s = 0; s < 3; ++s) {
    int rows = 0;
    expect(mm_rows_per_block(ctx, s, &rows), MM_OK, "rows_per_block");
  }
  step("destroy");
  for (auto* d : m) delete d;
  for (auto* d : H) delete d;
  mm_destroy(ctx);
}

}  // namespace

#if defined(__has_feature)
#if __has_feature(address_sanitizer)
#define MM_DRIVER_ASAN 1
#endif
#endif
#ifndef MM_DRIVER_ASAN
#define MM_DRIVER_ASAN 0
#endif

int main() {
  std::printf("address sanitizer: %s\n", MM_DRIVER_ASAN ? "on" : "off");
  step("support predicate and strings");
  if (mm_supported(0, 400, 200, 4) != 1 || mm_supported(0, 0, 5, 1) != 0) {
    std::printf("FAIL mm_supported\n");
    ++g_fail;
  }
  for (int code = -6; code <= 2; ++code)
    if (mm_strerror(code) == nullptr) ++g_fail;
  mm_destroy(nullptr);
  {
    mm_ctx* bad = nullptr;
    expect(mm_create(&bad, 7, 1, nullptr), MM_EINVAL, "create bad precision");
    expect(mm_create(&bad, MM_FP64, 0, nullptr), MM_EINVAL, "create no samples");
  }
  run_context(MM_FP64);
  run_context(MM_MIXED);
  std::printf("host sanitizer driver: %d failure(s)\n", g_fail);
  return g_fail == 0 ? 0 : 1;
}
