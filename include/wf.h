/*
 * wf.h -- C-ABI of libwf: batched Wiener-filter-as-MAP reconstruction and band-power
 * estimation on AMD MI355X (gfx950).
 *
 * Method: Horowitz, Seljak & Aslanyan, "Efficient optimal reconstruction of linear
 * fields and band-powers from cosmological data" (arXiv:1810.00503).
 *
 *   data model          d = M (R s + n)                         (sec. 2, eq. ddecomp)
 *   objective           chi^2(s) = s^dag S^-1 s + (d - R s)^T N^-1 (d - R s)   (eq. eq_chi)
 *   gradient            g = S^-1 s - R^dag N^-1 (d - R s)        (eq. eq_cost)
 *   curvature           D = S^-1 + R^dag N^-1 R                  (eq. eq_curv)
 *   MAP solve           L-BFGS with the exact line search of a quadratic (sec. 2.2, eq. eq_chib)
 *   band statistic      E_l = 1/2 s^dag S^-1 Pi_l S^-1 s          (sec. 2.3, eq. el)
 *   noise bias          b_l = < E_l(s_hat[d_sim]) >               (sec. 2.4, eq. blmv)
 *   Fisher              F_ll' Delta_l' = < E_l(Theta + Delta_l') - E_l(Theta) >  (eq. fisher)
 *   Newton step         Theta_hat = Theta_fid + F^-1 (E - b)      (eq. eq:wfmv)
 *   spin-2 response     appendix C (flat-sky E/B -> gamma1, gamma2)
 *
 * Conventions (the paper leaves them open; fixed here):
 *   - grid n x n, pixel (y, x) row-major; n even, n % 8 == 0, 8 <= n <= 1024, and
 *     n = 2^a or 3 * 2^a;
 *   - unitary DFT (F x)_k = n^-1 sum_j x_j exp(-2 pi i k.j / n); R = F^-1 on Hermitian
 *     spectra, so R is an isometry;
 *   - field coefficients are stored on the half plane [ncomp][n][n/2+1] (interleaved
 *     re, im of the element type): row iy holds ky = iy (iy < n/2) or iy - n, column kx;
 *   - live modes: k != 0, |kx| < n/2, |ky| < n/2, prior S_k > 0.  Free (independent)
 *     entries: kx in [1, n/2) on every row but iy = n/2, and kx = 0 with iy in [1, n/2).
 *     Entries (kx = 0, iy > n/2) hold the conjugates of their partners; inputs are read
 *     on free entries only; outputs write partners as conjugates and dead entries as 0;
 *   - prior S_k = theta[band_k] * pshape_k (band -1: amplitude 1), the variance of the
 *     unitary coefficient;
 *   - spin-2 (ncomp = 2, s = (E, B)): gamma1 = cos2a E - sin2a B, gamma2 = sin2a E + cos2a B,
 *     a = atan2(ky, kx), applied per mode before the inverse transform;
 *   - W = M N^-1 >= 0 per pixel, shared by both spin-2 components; W = 0 masks a pixel;
 *     the noise standard deviation of an observed pixel is W^-1/2.
 *
 * Memory: every array argument is caller-owned.  Unless stated otherwise, arrays are
 * DEVICE pointers on the context's device.  The context owns its workspace (grown on
 * demand, freed by wf_destroy).  Calls are enqueued on `stream` (a hipStream_t; NULL
 * means the legacy default stream); calls that return host results synchronise it.
 *
 * Errors: 0 = success; WF_NOT_CONVERGED (+1) = soft status (some instance stopped at
 * max_iter or on a non-finite value; see the per-instance stats); negative = error,
 * with a message in wf_last_error(ctx).  No C++ exception crosses this boundary.
 * One context per host thread.
 */
#ifndef WF_H
#define WF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wf_ctx wf_ctx;

enum {
  WF_OK = 0,
  WF_NOT_CONVERGED = 1,
  WF_EINVAL = -1,      /* bad argument (null pointer, bad n / ncomp / dtype / batch) */
  WF_ESHAPE = -2,      /* shapes of a batch or of two arguments disagree              */
  WF_ENOMEM = -3,      /* device or host allocation failed                            */
  WF_EHIP = -4,        /* a HIP runtime call failed                                   */
  WF_ENONFINITE = -5   /* non-finite input or result                                  */
};

enum { WF_F32 = 0, WF_F64 = 1 };

/* per-instance solver status */
enum { WF_SOLVE_CONVERGED = 0, WF_SOLVE_MAXITER = 1, WF_SOLVE_NONFINITE = 2 };

/* wf_adjoint flags (may be or-ed with WF_MASK) */
enum {
  WF_ADJ_METRIC = 0,   /* s = R^T x in the full-plane metric (partners filled)          */
  WF_ADJ_GRAD = 1,     /* gradient of a function of x = R s w.r.t. the stored s, in the
                          d/dRe + i d/dIm convention: 2 R^T x on free entries, 0 else  */
  WF_MASK = 2          /* wf_forward: x = M R s; wf_adjoint: R^T M x (M = [w > 0])      */
};

typedef struct {
  int32_t n;              /* grid side                                                   */
  int32_t ncomp;          /* 1 = spin-0 field, 2 = spin-2 (E, B) -> (gamma1, gamma2)     */
  int32_t dtype;          /* WF_F32 or WF_F64: type of d, w and of the coefficients      */
  int32_t nbands;         /* number of band amplitudes (0 allowed)                       */
  const void* d;          /* [ncomp][n][n] data; values on masked pixels are ignored     */
  const void* w;          /* [n][n] inverse-noise weight with the mask, M N^-1 >= 0      */
  const double* pshape;   /* [ncomp][n][n/2+1] prior shape P_k >= 0 (float64)            */
  const int32_t* band;    /* [ncomp][n][n/2+1] band index in [-1, nbands)                */
  const double* theta;    /* HOST [nbands] band amplitudes                               */
} wf_problem;

typedef struct {
  int32_t m;              /* L-BFGS memory (pairs kept), 1..16; default 10               */
  int32_t max_iter;       /* default 20000                                               */
  double rel_grad_tol;    /* stop when |g(s)| <= tol |g(0)|, whitened gradient; 1e-6     */
  double dchi2_tol;       /* also stop when |chi^2_k - chi^2_{k-1}| < this (0 = off)      */
  int32_t refresh_every;  /* recompute the exact gradient every this many iterations
                             (0 = only when the running gradient meets the tolerance)    */
  int32_t iters_per_poll; /* iterations enqueued between host checks (0 = automatic: 8)  */
  int32_t use_graph;      /* 1 = replay captured HIP graphs of the iteration (default),
                             0 = launch kernels one by one                               */
  int32_t precond;        /* 0 = H0 = gamma I in the whitened variable w = S^-1/2 s (the
                             paper's unpreconditioned L-BFGS, default); 1 = diagonal
                             noise-aware H0 = gamma diag(1 / (1 + S_k <W>)), <W> the pixel
                             mean of w, for very red spectra.  The stop test always uses
                             the whitened gradient norm; the solution is the same MAP.   */
  int32_t method;         /* WF_METHOD_LBFGS (0, default) or WF_METHOD_CG (1): conjugate
                             gradients on the same operator and variable (with precond = 1
                             the split-preconditioned CG), the same stop test, exact
                             gradient at the start, to confirm the stop and every
                             refresh_every iterations (then restarted); m is ignored      */
  int32_t refine;         /* float32 solves: 0 = off (default); else up to this many rounds
                             (<= 16) of float64 residual refinement after the solve: the
                             exact gradient is evaluated in float64 and a float32 correction
                             solve of D delta = -g (same solver, explicit right-hand side)
                             is added in float64, until the float64 relative whitened
                             gradient is <= refine_tol.  The relative-gradient stop of
                             float32 arithmetic ends near 1e-7; badly conditioned maps
                             (whitened condition number ~1e7, as the CMB workload) need
                             ~1e-10 and below for maps within 1e-5.  Stats then report the
                             float64 chi^2 and relative gradient, the iterations of all
                             solves, and WF_SOLVE_MAXITER if refine_tol was not reached.
                             Ignored for float64 problems.                               */
  double refine_tol;      /* target of the refinement (default 1e-10)                     */
} wf_lbfgs_opts;

enum { WF_METHOD_LBFGS = 0, WF_METHOD_CG = 1 };

typedef struct {
  int32_t iters;          /* L-BFGS directions taken                                      */
  int32_t status;         /* WF_SOLVE_*                                                   */
  int32_t ngrad;          /* exact gradient evaluations (first one included)             */
  int32_t reserved;
  double chi2;            /* chi^2 at the returned s (from the last exact evaluation
                             and the exact quadratic updates since)                      */
  double rel_grad;        /* |g(s)| / |g(0)| (exact gradient when converged)             */
} wf_solve_stats;

/* context ----------------------------------------------------------------------------- */
int wf_create(wf_ctx** out, int hip_device);
void wf_destroy(wf_ctx* ctx);
const char* wf_last_error(const wf_ctx* ctx);
void wf_lbfgs_default(wf_lbfgs_opts* opts);

/* MAP solve (sec. 2.2): for each of `batch` problems, s_hat = argmin chi^2.
 *   probs    HOST [batch]; sizes and types may differ between instances (uneven batch);
 *   s_out    HOST [batch] of device pointers, each [ncomp][n][n/2+1] complex (dtype);
 *   map_out  nullable; HOST [batch] of device pointers (entries may be NULL), each
 *            [ncomp][n][n] real: the map R s_hat;
 *   stats    HOST [batch] (nullable).
 * Instances of equal (n, ncomp, dtype) form a class; the classes of an uneven batch may run
 * on up to three more streams of the context, forked from and joined back to `stream`
 * inside the call (the call returns with all of its work finished).
 * Returns WF_OK if every instance converged, WF_NOT_CONVERGED otherwise.             */
int map_wf_solve(wf_ctx* ctx, const wf_problem* probs, int32_t batch, const wf_lbfgs_opts* opts,
                 void* const* s_out, void* const* map_out, wf_solve_stats* stats, void* stream);

/* Simulated data (sec. 2.4, procedure summary): d_i = M (R s_i + n_i) with
 * s ~ N(0, S_true) on free modes and n_i of variance 1/W on observed pixels; 0 on masked.
 * S_true = theta_true[band] pshape (theta_true HOST [nbands], NULL = prob->theta), with
 * band `boost_band` (-1 = none) scaled by boost_factor.
 * Normals: `draws` (device, [nsim][2][ncomp][n][n], dtype; part 0 signal: [c][ky][2kx],
 * [c][ky][2kx+1] are re, im of mode (ky, kx); part 1 pixel noise), or, if NULL, the
 * Philox4x32-10 stream of simulation sim0 + i with `seed` (key = seed lo/hi 32 bits,
 * counter (q/4, sim, 0, 0) for normal q, Box-Muller pairs in float64).
 *   d_out    [nsim][ncomp][n][n] (dtype).                                               */
int wf_simulate(wf_ctx* ctx, const wf_problem* prob, int32_t nsim, uint64_t seed, int32_t sim0,
                const void* draws, const double* theta_true, int32_t boost_band, double boost_factor,
                void* d_out, void* stream);

/* Simulation noise bias and Fisher matrix around prob->theta (eqs. blmv, fisher):
 * nsim * (1 + nbands) MAP solves with the fiducial prior, common random numbers,
 * Delta_l = theta_l; F symmetrised.  F HOST [nbands*nbands], b HOST [nbands],
 * F_var nullable HOST [nbands*nbands]: the Monte Carlo variance of each entry of F (the
 * sample variance over the simulations of each one's symmetrised estimate, divided by
 * nsim; 0 when nsim = 1), E_sims nullable HOST [nsim][nbands] (E of the fiducial
 * simulations).                                                                         */
int sim_fisher(wf_ctx* ctx, const wf_problem* prob, int32_t nsim, uint64_t seed, const void* draws,
               const wf_lbfgs_opts* opts, double* F, double* b, double* F_var, double* E_sims, void* stream);

/* Quadratic band-power estimator (sec. 2.3-2.5): MAP of prob->d, E_l of it, sim_fisher,
 * Newton step.  theta_hat, E, b HOST [nbands]; F HOST [nbands*nbands] (nullable).      */
int bandpower_qe(wf_ctx* ctx, const wf_problem* prob, int32_t nsim, uint64_t seed, const void* draws,
                 const wf_lbfgs_opts* opts, double* theta_hat, double* E, double* b, double* F,
                 void* stream);

/* The quadratic estimate of each of nprob maps (sec. 2.3-2.5, as bandpower_qe with every
 * Fisher column simulated), all of their solves shared among batched solves: per map the
 * data map, nsim fiducial and nsim * nbands_i boosted simulations, map after map, in chunks
 * of at most 256 solves, each chunk one batched solve (maps of different n, ncomp or dtype
 * form classes of an uneven batch).  Map i draws its simulations from the Philox key
 * seed + i (the stream of bandpower_qe(probs[i], nsim, seed + i)); external draws are not
 * taken.  Results per map equal bandpower_qe's up to the rounding of the transforms.
 *   theta_hat  HOST [nprob] of HOST [nbands_i] outputs;
 *   E, b, F    nullable HOST [nprob] of nullable HOST [nbands_i] ([nbands_i^2] for F).  */
int bandpower_qe_batch(wf_ctx* ctx, const wf_problem* probs, int32_t nprob, int32_t nsim, uint64_t seed,
                       const wf_lbfgs_opts* opts, double* const* theta_hat, double* const* E, double* const* b,
                       double* const* F, void* stream);

/* B-mode band powers with the E->B leakage treated as a bias (appendix C): nsim
 * simulations drawn with the fiducial amplitudes except the bands b_bands (the B bands),
 * which are set to 0, give b_B = <E_B> (noise bias plus leakage); the B block F_BB of the
 * Fisher matrix comes from nsim fiducial and nsim * nbb boosted-B simulations (eq. fisher,
 * symmetrised); every solve uses the fiducial prior; theta_B = F_BB^-1 (E_B(d) - b_B), which
 * holds because <E> is linear in the true amplitudes.  nsim (2 + nbb) + 1 MAP solves
 * against nsim (1 + nbands) + 1 for the full estimate.  Same seed / draws for both sets.
 *   b_bands  HOST [nbb] strictly increasing band indices;
 *   theta_b  HOST [nbb]; E_b, bias_b nullable HOST [nbb]; F_bb nullable HOST [nbb*nbb].  */
int bmode_leakage_qe(wf_ctx* ctx, const wf_problem* prob, int32_t nsim, uint64_t seed, const void* draws,
                     const wf_lbfgs_opts* opts, const int32_t* b_bands, int32_t nbb, double* theta_b, double* E_b,
                     double* bias_b, double* F_bb, void* stream);

/* sim_fisher with simulations for a subset of the Fisher rows only (the matrix is smooth
 * and nearly translation invariant, sec. 3.1): nsim * (1 + nrows) MAP solves.
 *   rows     HOST [nrows] strictly increasing band indices whose boosted simulations
 *            are run (NULL = all bands, then nrows is ignored);
 *   groups   nullable HOST [nbands] group id per band; a group is a run of consecutive
 *            bands with equal ids (e.g. the E and the B bands), NULL = one group.  Every
 *            group needs at least one simulated row.
 * A column l' without simulations is interpolated along the diagonals from the nearest
 * simulated columns a < l' < b of its group, in units of D_l = the variance of E_l over
 * the fiducial simulations (F_ll' / sqrt(D_l D_l') is interpolated): entry l reads entry
 * l + (a - l') of column a and l + (b - l') of column b, each kept inside the group of row
 * l, linearly in the band index; with one of the two outside, the other; beyond the
 * group's first or last simulated column, the one neighbour with the row clamped into the
 * group.  F is then symmetrised.  Outputs as sim_fisher; WF_EINVAL for bad rows or
 * groups.                                                                               */
int sim_fisher_rows(wf_ctx* ctx, const wf_problem* prob, int32_t nsim, uint64_t seed, const void* draws,
                    const wf_lbfgs_opts* opts, const int32_t* rows, int32_t nrows, const int32_t* groups,
                    double* F, double* b, double* E_sims, void* stream);

/* Fiducial iteration of the band-power estimate (sec. 2.3, after eq. pilin): starting from
 * prob->theta, repeat the quadratic estimate (Fisher rows as in sim_fisher_rows; rows NULL
 * = all) with the fiducial set to max(theta_hat, floor_frac * previous fiducial) until
 * max_l |change| / previous <= rel_tol or max_iter estimates.  The same seed (or draws)
 * is used by every estimate.
 *   theta_hat, E, b  HOST [nbands]: the last estimate and its E, b; F nullable [nb*nb];
 *   theta_hist       nullable HOST [(max_iter + 1) * nbands]: fiducials 0 .. n_iter;
 *   n_iter           nullable: estimates made.
 * Needs max_iter >= 1, rel_tol >= 0, 0 < floor_frac <= 1.                              */
int bandpower_iterate(wf_ctx* ctx, const wf_problem* prob, int32_t nsim, uint64_t seed, const void* draws,
                      const wf_lbfgs_opts* opts, const int32_t* rows, int32_t nrows, const int32_t* groups,
                      int32_t max_iter, double rel_tol, double floor_frac, double* theta_hat, double* theta_hist,
                      int32_t* n_iter, double* E, double* b, double* F, void* stream);

/* Posterior error of the Wiener filter (appendix A after eq. eq:wiener: the residual
 * s - s_hat has covariance S - S R^T C^-1 R S), estimated from nsim simulations drawn
 * with prob's own prior (theta): signal s_i and data d_i as in wf_simulate (same draws or
 * Philox stream, simulations 0 .. nsim - 1), s_hat_i the MAP of d_i, then
 *   var_modes  nullable, device [ncomp][n][n/2+1] (dtype): mean_i |s_i - s_hat_i|^2 per
 *              stored entry (kx = 0 partners mirror their free entries, dead entries 0);
 *   var_pix    nullable, device [ncomp][n][n] (dtype): mean_i (R (s_i - s_hat_i))^2.
 * Sums in float64.  At least one output; prob->d is not used.  WF_NOT_CONVERGED if a
 * simulation's solve did not converge.                                                  */
int posterior_error(wf_ctx* ctx, const wf_problem* prob, int32_t nsim, uint64_t seed, const void* draws,
                    const wf_lbfgs_opts* opts, void* var_modes, void* var_pix, void* stream);

/* Convergence as a function of scale (appendix B): the MAP of prob->d solved to the
 * reference tolerance opts->rel_grad_tol and to each of tols[0 .. ntol-1] (one batched
 * solve, per-instance tolerances), compared band by band:
 *   power      HOST [ntol + 1][nbands]: band power sum_{free k in l} |s_k|^2 of the
 *              reference (row 0) and of each looser solution;
 *   err_power  nullable HOST [ntol][nbands]: band power of (solution t - reference);
 *   cv         nullable HOST [nbands]: the cosmic-variance scale sqrt(2 / N_l), N_l the
 *              full-plane modes of band l;
 *   iters      nullable HOST [ntol + 1]: L-BFGS iterations of each solve;
 *   s_out      nullable HOST [ntol + 1] of device pointers (entries may be NULL): the
 *              solutions, [ncomp][n][n/2+1] complex.
 * 1 <= ntol <= 64, tols > 0.  WF_NOT_CONVERGED if the reference did not converge.       */
int convergence_by_band(wf_ctx* ctx, const wf_problem* prob, int32_t ntol, const double* tols,
                        const wf_lbfgs_opts* opts, double* power, double* err_power, double* cv, int32_t* iters,
                        void* const* s_out, void* stream);

/* operator-level calls: `batch` fields sharing prob's geometry, packed contiguously -- */

/* x = R s (eq. ddecomp), or M R s with flags WF_MASK:
 * s [batch][ncomp][n][n/2+1] complex -> x [batch][ncomp][n][n].                         */
int wf_forward(wf_ctx* ctx, const wf_problem* prob, int32_t batch, const void* s, void* x, int32_t flags,
               void* stream);

/* Adjoint of the response (sec. 2, eq. ddecomp; R^T is the operator of the gradient, eq.
 * eq_cost, and of the curvature, eq. eq_curv; spin-2: the inverse rotation of appendix C):
 * s = R^T x in the full-plane metric (flags WF_ADJ_METRIC: unitary forward DFT, inverse
 * rotation, dead entries 0, partners filled) or the stored-coefficient gradient of a
 * function of x = R s (WF_ADJ_GRAD: 2 R^T x on free entries, 0 else); with WF_MASK the
 * input is masked first (adjoint of the masked forward operator M R).
 * x [batch][ncomp][n][n] -> s [batch][ncomp][n][n/2+1] complex.                       */
int wf_adjoint(wf_ctx* ctx, const wf_problem* prob, int32_t batch, const void* x, void* s, int32_t flags,
               void* stream);

/* chi^2 (eq. eq_chi) of each field and, if grad_s != NULL, d chi^2 / d s per stored
 * coefficient (d/dRe + i d/dIm): 4 g on free entries with S > 0 (eq. eq_cost), 0 else.
 * chi2 HOST [batch].                                                                   */
int wf_chi2_grad(wf_ctx* ctx, const wf_problem* prob, int32_t batch, const void* s, double* chi2,
                 void* grad_s, void* stream);

/* curvature product in the same convention: Dp = 4 (S^-1 p + R^T W R p) (eq. eq_curv). */
int wf_hvp(wf_ctx* ctx, const wf_problem* prob, int32_t batch, const void* p, void* Dp, void* stream);

/* For callers that cannot allocate device memory (tight serving loops, harnesses that
 * forbid allocation): wf_hvp computed without any allocation.  Every buffer of its kernels
 * (twiddles, prior tables, transform vectors, jobs, partial sums) lives in one library
 * scratch array of WF_NOALLOC_SCRATCH_BYTES per GPU, held from the first wf_create on that
 * GPU until the process ends; the caller passes p and Dp as for wf_hvp.  Calls whose
 * buffers do not fit return WF_EINVAL (the message gives the bytes needed; about
 * 3 * batch * ncomp * n^2 * 4 bytes in float32).  All calls on one GPU share the array, so
 * calls that overlap on one GPU (other contexts, other host threads, or streams that are
 * not ordered) race; calls on one context are ordered.  The call is enqueued on `stream`
 * and returns without waiting for it.                                                     */
enum { WF_NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024 };
int wf_hvp_noalloc(wf_ctx* ctx, const wf_problem* prob, int32_t batch, const void* p, void* Dp, void* stream);

/* band statistic E_l (eq. el) of each field with the prior of prob: E HOST [batch][nbands]. */
int wf_band_E(wf_ctx* ctx, const wf_problem* prob, int32_t batch, const void* s, double* E, void* stream);

/* Band-power derivative of the objective at fixed fields (eq. eq_chi with S = theta_b P_k;
 * with eq. el, d chi^2 / d theta_b = -sum_{k in b, full plane} |s_k|^2 / (theta_b^2 P_k) =
 * -2 E_b(s; theta)), contracted with the upstream weights of a batch:
 *   dtheta   HOST [nbands]: sum_i gout[i] d chi^2(s_i) / d theta_b, accumulated in float64;
 *   gout     nullable HOST [batch] (NULL = all ones).
 * s as in wf_band_E; prob->theta are the amplitudes the derivative is taken at.  This is
 * the theta-gradient of a chi^2 autograd node.                                           */
int wf_chi2_dtheta(wf_ctx* ctx, const wf_problem* prob, int32_t batch, const void* s, const double* gout,
                   double* dtheta, void* stream);

/* catalog-level response (sec. 3.4: instead of binned shear maps, the likelihood of each
 * galaxy's measured ellipticity, so the field is evaluated at every galaxy's own position) --
 *
 * A catalog replaces the pixel data of a problem: the response maps the field s to its
 * values at the galaxies, gamma_a(r_g) = n^-1 sum_k (R~ s)_a,k exp(2 pi i k.r_g / n) (full
 * plane, the spin-2 rotation of appendix C for ncomp = 2), and the data term of chi^2 (eq.
 * eq_chi) is sum_g wgt_g sum_a (e_a,g - gamma_a(r_g))^2.  Evaluated as a non-uniform FFT: the
 * field's modes, deconvolved by the kernel's Fourier transform, on a grid of N = 2n points
 * per side, the transform chain at N, and a separable exponential-of-semicircle kernel of
 * 8 x 8 fine points per galaxy (interpolation; its adjoint, deterministic spreading, for
 * R^T), about 1e-6 relative to the exact sums in float32.  float32 only; n <= 512. */
typedef struct {
  int32_t ngal;           /* galaxies, 1 .. 2^27                                          */
  const double* pos;      /* [ngal][2] positions (y, x) in pixel units: pixel (iy, ix) is at
                             (iy, ix); periodic, any finite value (wrapped into [0, n))    */
  const float* e;         /* [ncomp][ngal] measured values (spin-2: e1, e2); solves only   */
  const float* wgt;       /* [ngal] inverse noise variance of each component, > 0; solves  */
} wf_catalog;

/* MAP solve of catalogs (sec. 2.2 with the catalog response): as map_wf_solve, with
 * cats[i] (HOST array, device pointers inside) in place of probs[i].d and .w (not read);
 * probs[i] gives n, ncomp, dtype = WF_F32, the prior and theta.  opts->precond and
 * opts->refine must be 0.  The galaxies of each catalog are binned on the host (positions
 * copied back once per call).  Catalogs of equal (n, ncomp) form one class of the batch.  */
int map_wf_solve_catalog(wf_ctx* ctx, const wf_problem* probs, const wf_catalog* cats, int32_t batch,
                         const wf_lbfgs_opts* opts, void* const* s_out, wf_solve_stats* stats, void* stream);

/* gamma [ncomp][ngal] = the field s [ncomp][n][n/2+1] (complex float, free entries read) at
 * the catalog's positions; prob gives n and ncomp (dtype WF_F32), cat->e and ->wgt unused. */
int wf_catalog_forward(wf_ctx* ctx, const wf_problem* prob, const wf_catalog* cat, const void* s, float* gamma,
                       void* stream);

/* Adjoint of wf_catalog_forward: s = R_cat^T r for r [ncomp][ngal] in the full-plane metric
 * (flags WF_ADJ_METRIC: per live mode n^-1 sum_g r_g exp(-2 pi i k.r_g / n), inverse
 * rotation, dead entries 0, partners filled) or the stored-coefficient gradient
 * (WF_ADJ_GRAD: twice that on free entries, 0 else); s [ncomp][n][n/2+1] complex float.    */
int wf_catalog_adjoint(wf_ctx* ctx, const wf_problem* prob, const wf_catalog* cat, const float* r, void* s,
                       int32_t flags, void* stream);

/* Tiles of the transform chain (the three passes of every gradient / curvature product):
 * rbv = image rows per work-group of the row pass (2, 4, 8), cpb = column blocks of 2
 * columns per work-group of the column passes (1, 2, 4; must divide n/4), group =
 * instances per launch (0 = all), reg = which passes run the register-staged FFT instead
 * of the LDS-staged one (bit 0: row pass, whose rows per work-group are then fixed by n;
 * bit 1: column inverse, bit 2: column forward, which need cpb * ncomp * 2 * n / 256 in
 * [4, 32]; float32 and power-of-two n >= 128 only), or reg = 8 alone: one kernel per
 * instance does all three passes of the solver's curvature product or gradient in LDS
 * (the field read once, Dp written once; maps whose field and twiddles fit 150 KB of LDS:
 * n <= 128 in float32, n <= 96 for spin-2 float64; solver passes only, operator calls keep
 * the three passes; rbv and cpb are ignored, group must be 0).  By default (rbv = 0) the
 * library autotunes them: on the first float32 solve of a batch of >= 4 maps of a given
 * (n, ncomp, batch-size bucket) it times every supported choice, the single pass included,
 * on that batch and keeps the fastest for the context.
 * float64 uses (4, 1, 0, 0), as does a fixed choice that the shape does not support.
 * Tuned choices persist on disk, keyed by device architecture and compute-unit count: in the
 * file WF_TUNE_CACHE names (empty: none), else $XDG_CACHE_HOME/libwf/tiles.txt or
 * ~/.cache/libwf/tiles.txt; wf_create reads it and every new tuning appends a line.
 * Every choice computes the same result up to the rounding of the transforms and the
 * order of the FP64 partial sums.  wf_get_chain_tiles reports the choice in use (WF_OK)
 * or the default if none was tuned yet (WF_NOT_CONVERGED).                             */
int wf_set_chain_tiles(wf_ctx* ctx, int32_t rbv, int32_t cpb, int32_t group, int32_t reg);
int wf_get_chain_tiles(wf_ctx* ctx, int32_t n, int32_t ncomp, int32_t dtype, int32_t batch, int32_t* rbv, int32_t* cpb,
                       int32_t* group, int32_t* reg);

/* instrumentation: per-kernel-kind launch counts, accumulated kernel time (HIP events
 * around each launch; only while profiling is on, which disables graph replay) and
 * algorithmic bytes (counted on the device for every launch).  Kinds are named by
 * wf_kernel_kind_name(k) for k in [0, wf_kernel_kinds()).                            */
int wf_set_profiling(wf_ctx* ctx, int32_t on);

/* instrumentation: the HBM streaming-copy reference.  Copies `bytes` (a positive multiple of
 * 16; device buffers src, dst) reps times with a hand-written copy kernel (16-byte vector
 * loads, each thread's loads issued before its stores) on the context's stream after one
 * untimed copy, timed with HIP events; *gbps = 2 * bytes * reps / time (read + write),
 * in 1e9 bytes per second.                                                                */
int wf_copy_bandwidth(wf_ctx* ctx, const void* src, void* dst, uint64_t bytes, int32_t reps, double* gbps);
int wf_kernel_kinds(void);
const char* wf_kernel_kind_name(int32_t kind);
int wf_get_kernel_stats(wf_ctx* ctx, int64_t* launches, double* ms, double* bytes);
int wf_reset_kernel_stats(wf_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* WF_H */
