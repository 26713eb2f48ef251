/*
 * mm.h -- C ABI of the MI355X (gfx950) finite-difference micromagnetic
 * energy minimiser.
 *
 * Method: Abert, Wautischer, Bruckner, Satz, Suess, "Efficient
 * Energyminimization in Finite-Difference Micromagnetics: Speeding up
 * Hysteresis Computations" (arXiv:1405.2728).
 *
 *   Sec. 2, eq. (5)  effective field H_eff = -(1/(mu0 Ms)) dU/dm
 *   Sec. 2, eq. (7)  midpoint (Cayley) projected-gradient update, read with
 *                    the descent sign:
 *                    m_{k+1} = m_k - tau (m_k + m_{k+1})/2 x (m_k x H_eff(m_k))
 *   Sec. 2, eqs. (8)-(10)  g_k = m_k x (m_k x H_eff(m_k)), s = m_k - m_{k-1},
 *                    y = g_k - g_{k-1}
 *   Sec. 2, eq. (12) Barzilai-Borwein steps tau1 = sum s.s / |sum s.y| (odd k)
 *                    and tau2 = |sum s.y| / sum y.y (even k), used
 *                    alternately; a candidate that is not finite and positive
 *                    keeps the previous tau; first step tau0 = 1e-3/Ms
 *   Sec. 2 (stop)    max_i |g_k^i| / Ms < tol, checked before every update
 *   Sec. 3           demagnetisation field as a zero-padded FFT convolution on
 *                    a regular cuboid grid.  Two paths: grids of at most 4
 *                    layers transform x and y and convolve directly over the
 *                    layers (thin-film path); thicker grids transform all
 *                    three axes (full 3-D path).
 *   Sec. 4           hysteresis loop: one minimiser run per field, started
 *                    from the previous field's magnetisation
 *
 * Field terms (the paper names them without formulas; standard FD forms):
 *   demag      H_d,i  = -Ms sum_j N(r_i - r_j) m_j, N the cell-averaged
 *              tensor (Newell closed form below 6 cell edges, Gauss-Legendre
 *              quadrature of the same integral beyond)
 *   exchange   H_ex,i = 2A/(mu0 Ms) sum_{6 face neighbours j} (m_j - m_i)/D^2,
 *              missing neighbours omitted (free boundary)
 *   anisotropy H_an,i = 2 Ku_i/(mu0 Ms) (m_i . u) u
 *   Zeeman     H_ext
 *   energy     U = -mu0 Ms V sum_i m_i . ((H_d + H_ex + H_an)_i/2 + H_ext)
 *   mu0 = 4 pi 1e-7; SI units; fields in A/m; energies in J.
 *
 * Memory layout of every magnetisation / field argument: device memory,
 * double precision, structure of arrays [3][nz][ny][nx] (x fastest), i.e.
 * component c of cell (x, y, z) at index c*N + (z*ny + y)*nx + x with
 * N = nx*ny*nz.  The caller owns these buffers; the library never frees or
 * retains them beyond the call.  Host pointers are marked "host".
 *
 * Precision: MM_FP64 computes everything in double.  MM_MIXED computes the
 * demag convolution (FFT passes and tensor product) in single precision and
 * keeps double precision for the tensor set-up, the local field terms, the
 * step-size and energy reductions, the stop test, the update and the state
 * m; the previous direction g and step s, which enter only the next update
 * and the Barzilai-Borwein sums, are stored in single precision.  Its
 * arguments are double precision as well.
 *
 * Streams: all work is ordered on the stream given to mm_create (NULL =
 * the default stream).  Calls that return host values synchronise that
 * stream.  A context is not thread-safe.
 *
 * Errors: every function returns MM_OK (0), a non-fatal status (> 0) or an
 * error (< 0).  mm_last_error() returns a message for the last error of a
 * context.  On error no caller buffer has been written unless stated.
 */
#ifndef MM_H
#define MM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mm_ctx mm_ctx;

enum mm_prec { MM_FP64 = 0, MM_MIXED = 1 };

enum mm_status {
  MM_OK = 0,
  MM_NOT_CONVERGED = 1,   /* max_iter reached before the stop rule held   */
  MM_STALLED = 2,         /* mixed form: torque stopped improving (floor)  */
  MM_EINVAL = -1,         /* invalid argument                              */
  MM_ENOMEM = -2,         /* device allocation failed                      */
  MM_EHIP = -3,           /* HIP runtime error                             */
  MM_ENONFINITE = -4,     /* non-finite torque or energy encountered       */
  MM_ESTATE = -5,         /* call out of order (e.g. no geometry yet)      */
  MM_EUNSUPPORTED = -6    /* grid shape not supported by the kernels      */
};

/* Per-iteration information (host struct). torque is max|g|/Ms before the
 * update, energy U(m_k) in J, tau the step applied, k the iteration index. */
typedef struct {
  double tau;
  double torque;
  double energy;
  int64_t k;
} mm_step_info;

/* Result of a minimiser run (host struct). iters = updates performed,
 * heff_evals = effective-field evaluations (the paper's Tab. 1 unit). */
typedef struct {
  int status;
  int64_t iters;
  int64_t heff_evals;
  double torque;
  double energy;
} mm_min_result;

/* Create a context for n_samples independent problems (n_samples >= 1).
 * prec is an mm_prec value; hip_stream is a hipStream_t or NULL.
 * *out receives the context (owned by the caller; free with mm_destroy). */
int mm_create(mm_ctx** out, int prec, int n_samples, void* hip_stream);

/* Release every device resource of ctx. NULL is accepted. */
void mm_destroy(mm_ctx* ctx);

/* Define the regular cuboid grid of one sample (Sec. 3): nx, ny, nz >= 1
 * cells of dx x dy x dz metres.  Computes the demag tensor spectrum on the
 * device (once per geometry) and allocates the sample's work buffers.
 * Resets the minimiser state.  The demag path follows the "demag_path"
 * option in force at this call.  MM_EUNSUPPORTED if the shape exceeds what
 * the library's kernels handle (see mm_supported); MM_ENOMEM if the device
 * cannot hold the set-up temporaries (full 3-D path: about
 * 192 (Px/2+1) Py Pz bytes, Px, Py, Pz the padded lengths). */
int mm_set_geometry(mm_ctx* ctx, int sample, int nx, int ny, int nz,
                    double dx, double dy, double dz);

/* Material of one sample (Sec. 4 notation): Ms > 0 (A/m), A >= 0 (J/m),
 * uniaxial Ku (J/m^3) with easy axis u (host double[3], normalised here).
 * Ku_map: NULL, or a device double[N] per-cell anisotropy constant that
 * overrides Ku; the library copies it.  Requires mm_set_geometry first.
 * Resets the minimiser state. */
int mm_set_material(mm_ctx* ctx, int sample, double Ms, double A, double Ku,
                    const double* u, const double* Ku_map);

/* Uniform external field H (host double[3], A/m).  Resets the minimiser
 * state (each field starts a new run, Sec. 4). */
int mm_set_field(mm_ctx* ctx, int sample, const double* H);

/* Reset the minimiser state: next iteration is k = 0 with tau = tau0. */
int mm_reset(mm_ctx* ctx, int sample);

/* Effective field of eq. (5) at m: H = H_d + H_ex + H_an + H_ext
 * (device in m, device out H, both [3][N] double). */
int mm_heff(mm_ctx* ctx, int sample, const double* m, double* H);

/* mm_heff without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same effective field as mm_heff, with the
 * convolution's spectrum held in a fixed array of the library (32 MiB per
 * GPU, kept until the process ends) instead of the sample's buffers.  The
 * caller still passes m and H (device [3][N] double).  Requirements: the
 * device that was current at mm_set_geometry is current (else MM_ESTATE);
 * the spectrum, 48 (Px/2+1) ny nz bytes in double precision (half that in
 * MM_MIXED), plus on the full 3-D path 48 (Px/2+1) Py nz bytes, fits the
 * 32 MiB (else MM_EINVAL with the size in mm_last_error; the 400 x 200 x 4
 * film needs 17.2 MB).  Calls and host-side code make no hipMalloc, hipFree
 * or other allocating call.  Every call on a GPU shares that GPU's array:
 * calls that overlap on one GPU (other streams, other contexts, other
 * threads) race and must be serialised by the caller.  Nothing in the array
 * needs to start at zero: each call writes the spectrum before reading it. */
int mm_heff_static(mm_ctx* ctx, int sample, const double* m, double* H);

/* Individual field terms at m; each output is a device [3][N] double or
 * NULL to skip it. */
int mm_field_terms(mm_ctx* ctx, int sample, const double* m, double* H_demag,
                   double* H_exchange, double* H_anisotropy);

/* Energy U(m) (host *E, J) and optionally its four terms (host double[4]:
 * demag, exchange, anisotropy, Zeeman; may be NULL).  Synchronises. */
int mm_energy(mm_ctx* ctx, int sample, const double* m, double* E, double* terms4);

/* One iteration of the minimiser on m (device [3][N], updated in place):
 * H_eff(m_k), g_k, the step size of eq. (12) and the update of eq. (7).
 * No stop rule is applied: the update is always performed (the caller may
 * inspect info->torque).  Continues the current run (state kept in the
 * context; call mm_reset before starting on a different m).  Returns MM_OK,
 * or MM_ENONFINITE when the torque or energy of m_k is not finite (m is
 * then left unchanged).  info (host, may be NULL) receives tau (the step
 * applied), torque and energy of m_k and k.  Synchronises when info is not
 * NULL. */
int mm_minimize_step(mm_ctx* ctx, int sample, double* m, mm_step_info* info);

/* Run the minimiser from m (device [3][N], updated in place) until
 * max|g|/Ms < tol or max_iter updates.  Starts a fresh run (k = 0,
 * tau = tau0).  out (host, may be NULL) receives the result.  Returns
 * MM_OK (converged), MM_NOT_CONVERGED, MM_STALLED or an error.
 * Synchronises. */
int mm_minimize_to_tol(mm_ctx* ctx, int sample, double* m, double tol,
                       int64_t max_iter, mm_min_result* out);

/* Continue the run held in the context (after mm_minimize_step calls, a run
 * that ended, or mm_state_load) on m (device [3][N], updated in place) until
 * max|g|/Ms < tol or the run's update count k reaches max_iter (a total over
 * the whole run, not a number of further updates).  Keeps k, tau, the BB
 * sums and the stored g and s (eq. (12)) and, in MM_MIXED, the reference of
 * the defect correction, so that the iterates are those of one
 * uninterrupted run with these limits.  Where the run ended at its last
 * evaluation (stop rule or max_iter), that evaluation's decision is taken
 * again with the new limits: stop, or the step of eq. (12) from the
 * recorded sums.  m must hold the state's m_k (the caller owns it: restore
 * it with the checkpoint).  out receives the whole run's counts.  Returns as
 * mm_minimize_to_tol; MM_EINVAL while the line search is on. */
int mm_minimize_continue(mm_ctx* ctx, int sample, double* m, double tol,
                         int64_t max_iter, mm_min_result* out);

/* Checkpoint of a relaxation in progress (the minimiser of Sec. 2 between
 * two iterations): the run's scalars (k, tau, the BB sums of eq. (12),
 * torque, energy, limits, the field), the stored g_k and s_k (the
 * context's transform type) and, in MM_MIXED with the defect correction,
 * the reference m_ref and H_d(m_ref) with its age.  m is not part of it
 * (the caller owns m).  mm_state_bytes gives the size (host *bytes);
 * mm_state_save writes it to host memory (host, at least that many bytes;
 * synchronises; runs a pending finish first); mm_state_load restores it
 * into a sample of the same precision, grid and correction setting (else
 * MM_EINVAL; also for a short or foreign buffer), replacing the sample's run
 * state and its field.  A restored state continues with mm_minimize_step or
 * mm_minimize_continue bit for bit as the saved run would have.  Both
 * return MM_EINVAL while the line search is on. */
int mm_state_bytes(mm_ctx* ctx, int sample, int64_t* bytes);
int mm_state_save(mm_ctx* ctx, int sample, void* host, int64_t bytes);
int mm_state_load(mm_ctx* ctx, int sample, const void* host, int64_t bytes);

/* Hysteresis sweep (Sec. 4) of every sample: m is a host array of
 * n_samples device pointers ([3][N_s] double each, updated in place);
 * H is host double[n_samples][n_fields][3] (A/m).  For each field the
 * sample's field is set, the state reset and the minimiser run to tol from
 * the previous field's result.  m_avg (host double[n_samples][n_fields][3])
 * receives the mean magnetisation after each field; iters (host
 * int64_t[n_samples][n_fields], may be NULL) the updates per field.
 * Returns the worst status over all runs (an error aborts the sweep). */
int mm_hysteresis_sweep(mm_ctx* ctx, double* const* m, const double* H, int n_fields,
                        double tol, int64_t max_iter, double* m_avg, int64_t* iters);

/* ---- derivatives (calculus on the energy U of Sec. 2; not in the paper) ----
 * dU/dm_i = -mu0 Ms V H_eff,i (eq. (5)); the constraint |m_i| = 1 makes the
 * relevant second derivative the Riemannian Hessian on the product of unit
 * spheres, Hess v = mu0 Ms V [ -P(H_lin[v]) + (m . H_eff(m)) v ] with
 * P_i = I - m_i m_i^T and H_lin the demag + exchange + anisotropy field of v
 * (no Zeeman term).  At a relaxed state m* (P dU/dm = 0) an objective J(m*)
 * has the implicit gradient dJ/dtheta = -lam . d(dU/dm)/dtheta with
 * Hess lam = P dJ/dm (the adjoint field). */

/* out = Hess(m) P v (for a tangent field v, v_i . m_i = 0, simply Hess v);
 * m, v, out device [3][N] double (out may alias v, not m).  The result is
 * tangent.  The normal direction is projected out first: along m_i the
 * expression has curvature m_i . H_eff,i, which is negative where the
 * self-demag field dominates. */
int mm_hessvec(mm_ctx* ctx, int sample, const double* m, const double* v, double* out);

/* Adjoint field: solve Hess(m) lam = P rhs by conjugate gradients on the
 * tangent space, starting from lam = 0, until |r| <= tol |P rhs| or max_iter
 * iterations.  m, rhs (dJ/dm), lam: device [3][N] double; lam is written.
 * iters, resid (host, may be NULL): iterations and final |r|/|P rhs|.
 * Every search direction is projected onto the tangent space.  Returns
 * MM_OK, MM_NOT_CONVERGED, or MM_ENONFINITE when a search direction has
 * non-positive curvature (m is not a strict local minimum) or a value is not
 * finite.  Synchronises. */
int mm_adjoint_solve(mm_ctx* ctx, int sample, const double* m, const double* rhs, double* lam,
                     double tol, int64_t max_iter, int64_t* iters, double* resid);

/* Implicit parameter gradients from the adjoint field lam at m:
 *   dJ/dA    = mu0 Ms V sum_i lam_i . H_ex,i(A = 1)       (host *dJ_dA)
 *   dJ/dMs   = mu0 V sum_i lam_i . (2 H_d,i + H_ext)      (host *dJ_dMs)
 *   dJ/dH    = mu0 Ms V sum_i lam_i                        (host double[3])
 *   dJ/dKu_i = 2 V (m_i . u)(lam_i . u)                   (device [N])
 * Outputs may be NULL.  Synchronises. */
int mm_param_grads(mm_ctx* ctx, int sample, const double* m, const double* lam, double* dJ_dA,
                   double* dJ_dMs, double* dJ_dH, double* dJ_dKu);

/* Derivatives of U(m; Ms, A, Ku, H_ext) at m:
 *   dU_dm  (device [3][N] or NULL) = -mu0 Ms V H_eff
 *   dU_dKu (device [N] or NULL)    = -V (m_i . u)^2
 *   scal5  (host double[5] or NULL) = { dU/dMs = (2 U_demag + U_zeeman)/Ms,
 *            dU/dA = U_exchange at A = 1, dU/dH_ext (3) = -mu0 Ms V sum_i m_i }.
 * Synchronises. */
int mm_energy_grads(mm_ctx* ctx, int sample, const double* m, double* dU_dm, double* dU_dKu,
                    double* scal5);

/* Mean magnetisation of m (device [3][N]) into host double[3]. */
int mm_mean(mm_ctx* ctx, int sample, const double* m, double* mavg);

/* Options (numeric): "tau0" (m/A; 0 = 1e-3/Ms), "poll_every" (iterations
 * between host checks of the stop flag, default 32), "stall_iters" (mixed
 * form without defect correction: iterations without a new torque minimum
 * before MM_STALLED, default 500; 0 disables), "bb_switch" (step choice,
 * taken at each reset of the minimiser state: 0, the default, alternates
 * the two steps of eq. (12) by the parity of k as Sec. 2 does; kappa > 0
 * takes tau2 = |s.y|/y.y where tau2 < kappa tau1, else tau1 = s.s/|s.y|,
 * a ratio switch between the two steps in the spirit of the more elaborate
 * switching Sec. 2 attributes to Exl et al.; must be finite and >= 0),
 * "line_search" (0 or 1, default 0, taken at each reset of the minimiser
 * state: a non-monotone safeguard of the step, which Sec. 2 does not use.
 * Every step is a trial m(tau) of eq. (7) from the accepted state, accepted
 * when U(m(tau)) <= C - ls_rho tau mu0 Ms V sum_i |g_i|^2 (the energy's
 * slope along eq. (7) at tau = 0 is -mu0 Ms V sum |g|^2) with C the
 * Zhang-Hager average of the accepted energies (C = U_0 at the start of a
 * run or field; after an accepted step Q' = ls_eta Q + 1,
 * C' = (ls_eta Q C + U) / Q'); a rejected trial is repeated from the same
 * state with tau multiplied by ls_sigma, at most ls_max times.  The stop
 * rule and the step choice of eq. (12) apply to accepted states; every
 * trial is one effective-field evaluation (mm_counters counts them).
 * mm_minimize_step returns MM_EINVAL while it is on; batched sweeps run
 * per sample), "ls_eta" (in [0, 1], default 0.85), "ls_rho" (in (0, 1),
 * default 1e-4), "ls_sigma" (in (0, 1), default 0.5), "ls_max" (integer
 * 0..1000, default 30),
 * "use_graph" (1, with a
 * non-null stream: mm_minimize_to_tol and mm_hysteresis_sweep replay each
 * batch of poll_every iterations after the first as one captured HIP graph;
 * mm_minimize_to_tol keeps its graph per sample while m, poll_every, the
 * correction and the material stay the same; not while kernels are timed), "demag_path" (0 = automatic: thin-film path for nz <= 4, full 3-D
 * path otherwise; 1 = thin-film path only; 2 = full 3-D path also for
 * nz <= 4; read by mm_set_geometry), "refine" (mixed form, default 1:
 * defect correction of the minimiser iterations.  Every poll_every
 * iterations a double-precision reference pass stores mref = m and
 * hdref = H_d(mref); each iteration then transforms only m - mref in single
 * precision and adds hdref, so the single-precision error scales with
 * |m - mref| and vanishes as the minimiser converges.  Applies where the
 * double-precision kernels handle the grid's demag path (grids whose
 * single-precision thin-film block does not fit in double precision run
 * without it); mm_heff, mm_field_terms, mm_energy and the derivative calls
 * always use the plain single-precision convolution), "autotune" (1: the
 * tile autotuner.  mm_set_geometry times the fused x passes (xf + xil) for
 * every valid number of rows per block on the sample's own buffers and
 * keeps the fastest, then, on the thin-film path, the yz pass's two
 * occupancy variants where the grid has two (the wave kernel compiled for
 * 3 or 2 resident waves per SIMD in double precision, 6 or 4 in single,
 * where a block's 3 nz waves fit); choices are cached per precision, grid
 * and demag path for the life of the process; default 0 uses a fixed
 * heuristic and the first variant, so that results do not depend on
 * timing; the variants compute the same bits),
 * "rows_per_block" (0 = automatic; otherwise that tile for every later
 * mm_set_geometry, which fails with MM_EINVAL where it is not valid: for
 * testing every tile), "yz_variant" (-1 = automatic; 0 or 1 that yz
 * occupancy variant for every later mm_set_geometry, which fails with
 * MM_EINVAL where the grid has no such variant: for testing), "mixed_radix" (default 1, read by mm_set_geometry:
 * the padded x length is the smaller of the power of two >= 2 nx - 1 and
 * the multiple of 128 >= 2 nx - 1 (up to 1024), the thin-film y length the
 * smaller of the power of two >= 2 ny - 1 and the multiple of 64 (up to
 * 512), so that transforms of 64 VL points with VL = 3, 5, 6, 7 take the
 * place of the next power of two; 0 keeps powers of two),
 * "concurrent_groups" (default 1: in batched sweeps the launches of a
 * pass, which touch disjoint samples, run on four auxiliary streams of
 * default priority forked from and joined back into the context's stream,
 * as parallel branches of the captured graph; 0 launches them one after
 * another; results are the same either way), "persistent" (default 1: in
 * batched sweeps each pass is one persistent launch covering every
 * transform length (the x passes one per rows-per-block class, the thin yz
 * pass one per layer count, the full 3-D path's three stages one each);
 * 0: one launch per group of equal lengths, and full 3-D samples run one
 * by one; results are the same either way), "batch_rebuild" (default 0.75:
 * in batched sweeps, once the running samples are at most this fraction of
 * the batch, its work tables are rebuilt from the running ones and the
 * graph captured again; 0 never; results are the same either way),
 * "fused_finish" (default 1: in mm_minimize_to_tol and in sweeps, a
 * sample's forward x pass of the wave-FFT lengths takes the previous
 * iteration's finish (the reduction of the per-block sums, the stop rule
 * and the step of eq. (12)) over instead of a one-block finish kernel: its
 * block 0 reduces and decides, the other blocks wait for the published
 * step after issuing their first loads; every poll interval still ends
 * with a finish kernel; not with the line search or a two-stage
 * reduction (more than 2048 per-block sums); 0: a finish kernel after
 * every iteration; results are the same either way), "fin_spin" (default
 * 2^22: polls of the published step before a waiting block gives up, writes
 * nothing and flags the run, which then fails with MM_ESTATE; an integer in
 * [0, 2^30], small values for testing that path).
 * Unknown keys or values give MM_EINVAL. */
int mm_set_option(mm_ctx* ctx, const char* key, double value);

/* Rows per block of the sample's fused x passes (host int output), as the
 * heuristic, the autotuner or the rows_per_block option chose it at
 * mm_set_geometry. */
int mm_rows_per_block(mm_ctx* ctx, int sample, int* rows);

/* Occupancy variant of the sample's thin-film yz pass (host int output: 0
 * or 1), as the autotuner chose it at mm_set_geometry (0 without it). */
int mm_yz_variant(mm_ctx* ctx, int sample, int* var);

/* Counters of one sample since its last mm_set_geometry: total
 * effective-field evaluations and updates (host int64_t outputs). */
int mm_counters(mm_ctx* ctx, int sample, int64_t* heff_evals, int64_t* iters);

/* Whether the library's kernels handle a grid (1) or not (0) with the
 * automatic demag path (and the default "mixed_radix" padding): nx <= 2048
 * (the fused x passes hold a row's three components, 3 Px/2 complex values,
 * in one block);
 * nz <= 4 with 2ny-1 padded (to a power of two or a multiple of 64) so that
 * 3 nz Py complex values fit one block, or nz > 4 with ny, nz <= 256 (y and
 * z padded to powers of two in 64..512). */
int mm_supported(int prec, int nx, int ny, int nz);

/* State of the sample's minimiser after its most recent call (host *info;
 * synchronises): tau = the step of the most recent update of eq. (7) (tau0
 * before the first), torque and energy of the most recent evaluation m_k
 * (Sec. 2 stop quantity max|g_k|/Ms and U(m_k)), k = that evaluation's
 * index within its run.  After mm_minimize_to_tol with max_iter = j and
 * tol = 0 these are tau_{j-1}, T(m_j), U(m_j) and j. */
int mm_last_step(mm_ctx* ctx, int sample, mm_step_info* info);

/* Per-kernel timing with HIP events on the context's stream.
 * mm_profile(ctx, mask) records an event pair around every launch of each
 * kernel whose bit is set in mask (bit k = kernel id k; 0 stops recording)
 * and clears the totals.  Events add a small gap per timed launch, so time
 * only the kernels of interest.  mm_profile_read(ctx, id, &ms, &launches)
 * reads the accumulated time of kernel id (synchronises).
 * mm_kernel_name(id) names it (NULL past the last id): 0 "xf" (pending
 * update, forward x transform), 1 "yz_thin" (thin-film y transform, tensor
 * product, inverse), 2 "xil" (inverse x transform, local terms, sums, step
 * choice), 3 "update" (mm_minimize_step only), 4 "y3_fwd", 5 "z3",
 * 6 "y3_inv" (full 3-D path: forward y, z transform with tensor product,
 * inverse y), 7 "finish" (reduction of the per-block sums, stop rule, step
 * choice), 8 "reference" (the whole double-precision reference pass of the
 * mixed form's defect correction, one record per pass).
 * mm_kernel_bytes(ctx, sample, id, &bytes) gives that kernel's algorithmic
 * bytes per launch in a minimiser iteration (compulsory reads + writes). */
int mm_profile(mm_ctx* ctx, int mask);
int mm_profile_read(mm_ctx* ctx, int kernel_id, double* total_ms, int64_t* launches);
const char* mm_kernel_name(int kernel_id);
int mm_kernel_bytes(mm_ctx* ctx, int sample, int kernel_id, double* bytes);

const char* mm_strerror(int code);
const char* mm_last_error(const mm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* MM_H */
