// Host-callable launchers of the HIP kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mmk {

constexpr double kMu0Host = 4.0e-7 * 3.14159265358979323846;

// Non-monotone line search of the step (on = 0: none): Zhang-Hager weight
// eta, sufficient-decrease factor rho, backtracking factor sigma, at most
// max_back rejected trials per step.
struct LineSearch {
  int on;
  double eta, rho, sigma;
  int max_back;
};

// Minimiser state of one sample, resident in device memory.  Written only
// by the step-size kernel (one thread) and read by every kernel of the
// iteration; the host reads it when polling.
struct MinState {
  double tau;          // step applied by the update of the current iteration
  double torque;       // max_i |g_i| / Ms of the last evaluated m_k
  double energy;       // U(m_k)
  double eterm[4];     // demag, exchange, anisotropy, Zeeman parts of U(m_k)
  double ss, sy, yy;   // BB sums of the last evaluation (k >= 1)
  double best_torque;  // smallest torque of the run (stall detection)
  double tol;          // stop tolerance on max|g|/Ms
  double tau0;         // first step
  long long k;         // updates applied in this run
  long long best_k;    // k at best_torque
  long long evals;     // effective-field evaluations in this run
  long long max_iter;
  long long stall_iters;  // 0 disables
  int done;            // 0 running; 1 converged; 2 max_iter; 3 stalled; -1 non-finite
  int mode;            // 0 minimise with stop rule; 1 forced steps; 2 evaluate only
  double last_tau;     // tau used by the most recent update (for step info)
  long long last_k;    // k index of the most recent evaluation
  int pending;         // 1: an update with last_tau is due before the next evaluation
  double H[3];         // external field of the current run (A/m)
  // Hysteresis sweep on the device (sweep = 1): when a field's run ends
  // (stop rule, max_iter or stall) its mean magnetisation and update count
  // are recorded, the next field is applied and the BB state restarts from
  // the same m; after the last field done = the worst status of the fields.
  int sweep;
  int field, n_fields;
  const double* fields;    // device [n_fields][3]
  double* mavg_out;        // device [n_fields][3]
  long long* iters_out;    // device [n_fields]
  int worst;               // 1 converged, 2 max_iter, 3 stalled (worst so far)
  double inv_N;            // 1 / cells, for the mean
  // Step choice: 0 alternates the two steps of eq. (12) by the parity of k;
  // kappa > 0 takes the short step tau2 where tau2 < kappa tau1, else tau1
  // (a ratio switch between the two steps)
  double bb_switch;
  // Line search (ls.on): every evaluation after the first of a run is a
  // trial m(tau) from the accepted base (ls_trial); a rejected trial is
  // repeated from the base with a shorter step (ls_retry: the base is the
  // saved copy ls_mbase with its gradient in g, instead of the buffer m with
  // the last trial's gradient in ls_g2); ls_nb rejections of this step;
  // reference value ls_C with weight ls_Q; ls_G = sum |g|^2 of the base.
  LineSearch ls;
  int ls_trial, ls_retry, ls_nb;
  double ls_C, ls_Q, ls_G;
  double* ls_mbase;
  void* ls_g2;         // values of the transform type, like g
  // Finish taken over by the next forward x pass (FinFuse): the decision of
  // the pass is published in fin_slot[parity] (kFinSent until then);
  // fin_err is set if a block gave up waiting for it
  unsigned long long fin_slot[2];
  int fin_err;
};

// Finish of the previous iteration taken over by the next forward x pass of
// a single-sample minimiser run.  Block 0 of the pass reduces the previous
// inverse pass's per-block sums in the finish kernel's order, takes the
// decision (stop rule, step of eq. (12)) into the state and publishes what
// the pass needs (stop, no update, or the step) in st->fin_slot[par]; the
// other blocks issue their first loads, then wait for it.  partials == NULL:
// nothing to take over (the first pass after a finish kernel), block 0 only
// resets st->fin_slot[par ^ 1] for the next pass.  st == NULL: off.
struct FinFuse {
  MinState* st;
  const double* partials;
  double Ms, V;
  int nb, par;
  int spin;   // polls of the slot before a waiting block gives up
};
// published words: a signalling NaN (never an arithmetic result) until the
// decision, -1 stop, -2 no update, else the step tau > 0
constexpr unsigned long long kFinSent = 0x7FF4000000000001ull;
constexpr double kFinStop = -1.0, kFinNoUpdate = -2.0;
// default polls of the slot before a block gives up (fin_err), with a short
// sleep between them: far beyond any finish (microseconds)
constexpr int kFinSpin = 1 << 22;

// Conjugate-gradient state of an adjoint solve, resident in device memory.
struct CGState {
  double bb;           // |P rhs|^2
  double rr;           // |r_k|^2
  double pAp;          // p_k . Hess p_k
  double alpha, beta;
  double tol2;         // stop when rr <= tol2 bb
  long long k, max_iter;
  int done;            // 0 running; 1 converged; 2 max_iter; -1 breakdown or non-finite
};

// One sample of a batched launch (device table): its buffers, sizes and
// material constants.  The external field is read from st->H.
struct BatchDesc {
  double* m;
  void* g;               // g and s: values of the transform type T
  void* s;
  void* spec;            // spectrum A[kx][z][y][c] (T complex)
  const void* Tt;        // thin-film tensor, or the 3-D tensor octant (T)
  const void* twx;       // twiddles, length Px (T complex)
  const void* twy;       // twiddles, length Py (T complex)
  void* B;               // 3-D path: y-transformed spectrum B[kx][ky][z][c] (else NULL)
  const void* twz;       // 3-D path: twiddles, length Pz (T complex)
  int Pz;                // 3-D path: padded z length (else 1)
  MinState* st;
  double* partials;      // [nb3][kNPartial]
  const double* ku_map;  // NULL: scalar ku
  int nx, ny, nz, M, Py, R, tstride, nb3;
  double cx, cy, cz;     // 2A/(mu0 Ms D^2)
  double ku, kan;        // scalar Ku; 2/(mu0 Ms)
  double u[3];
  double scale;          // -Ms/(M Py), on the 3-D path -Ms/(M Py Pz)
  double Ms, V;
  // defect correction of the single-precision form: pass 0 plain; pass 1
  // transforms m - mref and adds hdref to the demag field; pass 2 (the
  // double-precision reference) copies m to mref and writes hdref = H_d(mref)
  double* mref;
  double* hdref;
  int pass;
};
// A block of a batched launch: sample index and logical block of its pass.
struct WorkItem {
  int sample;
  int block;
};

// Gauss-Legendre rules used by the far-field tensor (nodes on [-1, 1]).
struct GaussRules {
  double x6[6], w6[6];
  double x4[4], w4[4];
  double x3[3], w3[3];
};

// ---- tensor set-up (FP64) --------------------------------------------------
void launch_newell_octant(hipStream_t s, double* out, int nx, int ny, int nz, double dx,
                          double dy, double dz, const GaussRules& gr);
void launch_embed_thin(hipStream_t s, const double* oct, double* E, int nx, int ny, int nz, int Px,
                       int Py);
template <typename T>
void launch_extract_thin(hipStream_t s, const void* EXY, T* Tt, int M, int nz, int Py, int tstride);
void launch_twiddles(hipStream_t s, void* tw, int P, bool single);
void launch_embed_3d(hipStream_t s, const double* oct, double* E, int nx, int ny, int nz, int Px,
                     int Py, int Pz);
void launch_transpose_planes(hipStream_t s, const void* in, void* out, int rows, int cols,
                             int nplanes);
template <typename T>
void launch_extract_3d(hipStream_t s, const void* E, T* T3, int M, int Py, int Pz, int rstride);
// elements per (kx, ky') row of the 3-D tensor (padded to 16 bytes)
inline int tensor3_row(int Pz, bool single) {
  const int e = (Pz / 2 + 1) * 6;
  const int q = single ? 4 : 2;
  return (e + q - 1) / q * q;
}
// ---- full 3-D path (grids with more than 4 layers) --------------------------
// y transform of the (kx, z) planes: dir -1: A[kx][z][y][c] -> B[kx][ky][z][c];
// dir +1: B -> A (rows y < ny kept).
template <typename T>
void launch_y3(hipStream_t s, void* A, void* B, int nz, int ny, int Py, int M, int dir,
               const void* twy, const int* done);
// z transform of every (kx, ky) pencil of B, product with the tensor, inverse.
template <typename T>
void launch_z3(hipStream_t s, void* B, int nz, int Py, int Pz, int M, const T* T3, int rstride,
               T scale, const void* twz, const int* done);
// padded y and z lengths handled by the 3-D kernels (powers of two, 64..512)
inline bool full3d_len_ok(int P) { return P == 64 || P == 128 || P == 256 || P == 512; }

// ---- demag passes ------------------------------------------------------------
// Rows per block chosen by the host: rows_per_block.
template <typename T>
void launch_fwd_x(hipStream_t s, const double* in, int in_row_stride, int nx_in, int rows, int ncomp,
                  int Px, int rows_per_block, void* out, const void* twx, const int* done);
template <typename T>
void launch_inv_x(hipStream_t s, const void* in, int rows, int ncomp, int nx_out, int Px,
                  int rows_per_block, double* out, const void* twx, const int* done);
template <typename T>
void launch_fft_cols(hipStream_t s, void* data, int n, int nseq, const void* tw);
// var: the wave kernel's occupancy variant (0 default; 1 the alternative
// bound, where yz_variants gives 2), chosen by the tile tuner
template <typename T>
void launch_yz_thin(hipStream_t s, void* A, int nz, int ny, int Py, int M, const T* Tt,
                    int tstride, T scale, const void* twy, const int* done, int var = 0);
int yz_variants(bool single, int nz, int Py);
// elements per kx slab of the thin tensor (padded to 16 bytes)
inline int thin_tensor_stride(int nz, int Py, bool single) {
  const int e = nz * (Py / 2 + 1) * 6;
  const int q = single ? 4 : 2;
  return (e + q - 1) / q * q;
}
bool yz_thin_fits(int nz, int Py, bool single);
bool yz_wave_ok(int nz, int Py);
// batched passes (all items of a launch share M and R, resp. Py and nz)
template <typename T>
void launch_x_batched(hipStream_t s, bool inverse, const BatchDesc* descs, const WorkItem* items,
                      int n_items, int M, int R);
template <typename T>
void launch_yz_batched(hipStream_t s, const BatchDesc* descs, const WorkItem* items, int n_items,
                       int Py, int nz, int tstride);
void launch_finish_batched(hipStream_t s, const BatchDesc* descs, int n_samples);
// persistent batched passes: one launch covers the items of every sample,
// whatever its transform length (x: items of samples with R <= threads / 192;
// yz: samples with nz layers); grid: blocks resident together (a multiple of
// 8), lds: the largest block's dynamic LDS
int x_persistent_grid(bool single, bool inverse, int threads, size_t lds);
size_t x_block_lds(bool single, int M, int R);
template <typename T>
void launch_x_persistent(hipStream_t s, bool inverse, const BatchDesc* descs,
                         const WorkItem* items, int n_items, int threads, size_t lds, int grid);
// 3-D path (demag3d.hip), persistent batched: stage -1 forward y, 0 z with
// the tensor product, +1 inverse y; items = (sample, block of the stage's
// per-sample grid: (M+1) ceil(nz/4) for y, (M+1) Py/4 for z)
int w3_persistent_grid(bool single, int stage, size_t lds);
size_t w3_block_lds(bool single, int P);
int y3_blocks(int nz, int M);
int z3_blocks(int Py, int M);
template <typename T>
void launch_3d_persistent(hipStream_t s, int stage, const BatchDesc* descs, const WorkItem* items,
                          int n_items, size_t lds, int grid);
int yz_persistent_grid(bool single, int nz, size_t lds);
size_t yz_block_lds(bool single, int Py, int nz, int tstride);
template <typename T>
void launch_yz_persistent(hipStream_t s, const BatchDesc* descs, const WorkItem* items,
                          int n_items, int nz, size_t lds, int grid);

// ---- local terms, step size, update -----------------------------------------
struct LocalArgs {
  const double* m;
  const double* Hd;
  // g, g_out and s hold values of the kernel's transform type (double in
  // the double-precision form; float in the single-precision form, where
  // they feed only the step direction and the BB sums)
  void* g;              // in: g_{k-1}; out: g_k (NULL: no g / BB sums)
  void* g_out;          // NULL: g_k written to g; else written here (g only read)
  const void* s;        // s_{k-1} (NULL: no BB sums)
  double* Hout;         // total effective field (NULL: not written)
  double* Hex_out;      // exchange field (NULL: not written)
  double* Han_out;      // anisotropy field (NULL: not written)
  const double* ku_map; // per-cell Ku (NULL: scalar ku)
  int nx, ny, nz;
  double cx, cy, cz;    // 2A/(mu0 Ms D^2) per axis
  double ku, kan;       // scalar Ku; 2/(mu0 Ms)
  double u[3], H[3];
  const double* Hdyn;   // device field overriding H (NULL: use H)
  const double* Hd_add; // field added to the transformed demag field (NULL: none)
  double* partials;     // [nblocks][kNPartial]
  const MinState* st;   // NULL outside the minimiser
  const int* done;      // NULL outside the minimiser
};
constexpr int kLocalThreads = 256;
// per-block sums: [s.s, s.y, y.y, m.H_d, m.H_ex, Ku (m.u)^2, m.H_ext, max |g|^2,
// sum m_x, sum m_y, sum m_z, sum |g|^2]; entry kPartMax is a maximum, the
// others sums
constexpr int kNPartial = 12;
constexpr int kPartMax = 7;
int local_blocks(int N);
// reduction of the per-block sums, stop rule and step choice; partials has
// room for finish_extra_rows(nblocks) rows after the nblocks rows
void launch_finish(hipStream_t s, double* partials, int nblocks, MinState* st, double Ms,
                   double V);
int finish_extra_rows(int nblocks);
// G: the type of the g and s streams (the context's transform type)
template <typename G>
void launch_update(hipStream_t s, double* m, const G* g, G* sbuf, int N, const MinState* st);
void launch_reset_state(hipStream_t s, MinState* st, double tau0, double tol, long long max_iter,
                        long long stall_iters, int mode, const double H[3],
                        double bb_switch = 0.0, const LineSearch* ls = nullptr,
                        double* ls_mbase = nullptr, void* ls_g2 = nullptr);
void launch_sweep_start(hipStream_t s, MinState* st, const double* fields, int n_fields,
                        double* mavg_out, long long* iters_out, double inv_N);
void launch_set_mode(hipStream_t s, MinState* st, int mode);
void launch_clear_pending(hipStream_t s, MinState* st);
// Continue a run (mode 0 with the given stop limits) from its state: where
// the run ended at an evaluation without a step, the decision of that
// evaluation is taken anew with the new limits (stop, or the step of
// eq. (12) from the recorded BB sums, which becomes the pending update).
void launch_continue_state(hipStream_t s, MinState* st, double tol, long long max_iter,
                           long long stall_iters);
// fused x passes of the thin-film iteration
int rows_per_block(int M, int ny, bool single);
// msub (NULL: none) is subtracted from m before the transform; mcopy (NULL:
// none) receives a copy of m, and then no pending update is applied.  fz
// (NULL or fz->st NULL: none) hands the previous iteration's finish to the
// pass; only the wave-FFT lengths take it (xf_fuses_finish).
template <typename T>
void launch_xf(hipStream_t s, double* m, const T* g, T* sbuf, const MinState* st, int nx, int ny,
               int nz, int Px, int R, void* out, const void* twx, const double* msub,
               double* mcopy, const FinFuse* fz = nullptr);
bool xf_fuses_finish(int Px);
// largest per-block sum count the finish kernel reduces in one stage
int finish_single_stage_max();
template <typename T>
// partials: per-block sums out (NULL: none), reduced by launch_finish
void launch_xil(hipStream_t s, const void* in, const LocalArgs& a, int Px, int R, double* Hd_out,
                double* partials, const void* twx);
void launch_mean(hipStream_t s, const double* m, int N, double* partials, double* out3);

// ---- derivatives (adjoint.hip) ------------------------------------------------
int adj_blocks(int N);
void launch_cg_init(hipStream_t s, const double* m, const double* rhs, double* x, double* r,
                    double* p, int N, double* partials, CGState* cg, double tol,
                    long long max_iter);
void launch_hess_apply(hipStream_t s, const double* m, const double* Hm, const double* Hlin,
                       const double* v, double* out, int N, double c, double* partials,
                       const int* done);
void launch_cg_step(hipStream_t s, const double* m, double* x, double* r, double* p,
                    const double* Ap, int N, double* partials, CGState* cg);
void launch_project(hipStream_t s, const double* m, const double* v, double* out, int N);
void launch_param_grads(hipStream_t s, const double* m, const double* lam, const double* Hd,
                        const double* Hex1, const double H[3], const double u[3], double V,
                        double* dKu, int N, double* partials, double* out5);
void launch_energy_grads(hipStream_t s, const double* m, const double* H, double c, double* dm,
                         const double u[3], double V, double* dKu, int N, double* partials,
                         double* out3);

}  // namespace mmk
