/*
 * helic.h -- C ABI of the MI355X helical-wave Hamiltonian library.
 *
 * The library applies the discrete Hamiltonian of the helical-wave spectral
 * method (Agarwal & Banerjee, arXiv 2210.12252) to blocks of coefficient
 * vectors on one AMD Instinct MI355X (gfx950), and solves for its lowest
 * eigenpairs.  For a Bloch parameter eta and cyclic index nu the operator
 * is (Alg. 5, eqs. Simplify_2 and g_mnk)
 *
 *     (H x)_i = kappa_i x_i + [Fwd(V * Inv(x))]_i ,
 *     kappa_i = 1/2 [ (b_k^{p}/R)^2 + (2 pi/tau)^2 (m - alpha p_s - eta)^2 ],
 *     p_s = n N - nu,  p = |p_s|,
 *
 * with Inv the inverse basis transform (Alg. 1 and 2: radial sums per angular
 * mode, then a 2D inverse DFT per radius), V the real potential sampled on the
 * grid and Fwd the quadrature forward transform (Alg. 3 and 4: a 2D DFT per
 * radius, then weighted radial sums).  For cyclic order N (an N-fold
 * symmetric structure; theta2 spans the wedge [0, 1/N)) basis functions are
 * F_{m,n,k} = c_{nk} exp(i 2 pi (m theta1 + n N theta2)) J_{p_s}(b_k^{p} r/R),
 * c_{nk} = sqrt(N/(pi tau)) / (R J_{p_s+1}(b_k^{p})) (Sec. 2.3, App. B),
 * kept when kappa_i <= E_cut (Sec. 3.2).  At nu = 0 these are the paper's
 * functions.  For nu != 0 the paper keeps the order nN and adds the
 * nu^2/(2 r^2) and (i nu/(2 pi r^2)) d/dtheta2 terms of eq. Simplify_2
 * through the integrals of eq. I_nkk_prime, which diverge for n = 0; those
 * terms turn the Bessel operator of order nN into that of order nN - nu, so
 * the library uses radial functions of that order, in which the same
 * operator's kinetic part is the diagonal kappa above.
 *
 * Conventions shared by all entry points
 * - Every pointer argument documented "device" must point to memory of the
 *   current HIP device; "host" pointers are ordinary CPU memory.
 * - A coefficient block is column-major: column j (one vector) starts at
 *   element j*ld, holds L complex values as interleaved (re, im) doubles, rows
 *   in the library's compact order (helic_basis_indices); ld >= L counts
 *   complex elements.
 * - A real-space array is indexed [i1][i2][ir] with ir fastest (theta1
 *   outermost, then theta2, then r; Sec. 3.1, eq. wavefun_storage_real).
 * - `stream` is a hipStream_t (0 = the null stream).  Calls on a stream are
 *   asynchronous unless stated otherwise; the caller keeps buffers alive until
 *   the stream has passed them.
 * - Errors: every call returns a helic_status; no exception crosses the ABI.
 *   HELIC_ERR_INVALID calls write nothing.  helic_last_error() returns the
 *   calling thread's last message.
 * - A handle must not be used from two host threads, or on two streams, at
 *   the same time.
 */
#ifndef HELIC_H
#define HELIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct helic_basis_s* helic_basis;

typedef enum {
  HELIC_OK = 0,
  HELIC_ERR_INVALID = 1,      /* bad argument (null pointer, size, range)         */
  HELIC_ERR_UNSUPPORTED = 2,  /* unsupported mode (precision, group width)          */
  HELIC_ERR_GRID = 3,         /* grid too small to resolve the index set           */
  HELIC_ERR_NOMEM = 4,        /* device or host allocation failed                  */
  HELIC_ERR_HIP = 5,          /* a HIP runtime or library call failed              */
  HELIC_ERR_NOCONV = 6,       /* eigensolver stopped at maxit above tolerance      */
  HELIC_ERR_CUTOFF_TIE = 7,   /* some kinetic energy equals E_cut within 1e-10 Ha  */
  HELIC_ERR_STATE = 8         /* call out of order (e.g. apply before potential)   */
} helic_status;

/* Arithmetic of the transform stages of apply_H.  Inputs and outputs stay
 * complex double in every mode, and the kinetic term kappa x is added in
 * FP64.  FP32 runs the radial contractions (FP32 MFMA), the angular DFTs and
 * the intermediates in single precision with FP32 accumulation.  BF16 runs
 * the radial contractions on BF16 MFMA (tables and coefficients rounded to
 * bfloat16, FP32 accumulation), keeps the intermediates as bfloat16 and does
 * the angular DFTs and the potential product in FP32: unit roundoff 2^-8,
 * a first rung for eigensolvers before FP32 and FP64. */
typedef enum { HELIC_FP64 = 0, HELIC_FP32 = 1, HELIC_BF16 = 2 } helic_prec;

typedef struct {
  double R;       /* cylinder radius, Bohr (> 0); Dirichlet wall at r = R        */
  double tau;     /* axial period of the screw operation, Bohr (> 0)             */
  double alpha;   /* twist: rotation of 2*pi*alpha per period, 0 <= alpha < 1    */
  int32_t ncyc;   /* cyclic order N, 1..64; theta2 in [0, 1/N)                   */
  double ecut;    /* kinetic-energy cutoff, Ha (> 0), inclusive                  */
  double eta;     /* helical Bloch parameter, -1/2 <= eta < 1/2                  */
  int32_t nu;     /* cyclic Bloch index, 0 <= nu < ncyc                           */
  int32_t m_max;  /* clamp |m| <= m_max (-1: what the theta1 grid resolves)      */
  int32_t n_max;  /* clamp |n| <= n_max (-1: what the theta2 grid resolves)      */
  int32_t k_max;  /* clamp k <= k_max   (-1: none)                               */
  int32_t n_t1;   /* theta1 (axial) Fourier nodes; 0 with n_t2 = 0: automatic    */
  int32_t n_t2;   /* theta2 (angular) Fourier nodes                              */
  int32_t n_r;    /* radial Gauss-Jacobi nodes; 0: 4 * (largest k kept)          */
} helic_params;

/* Build the basis on the host: Bessel zeros b_k^{|n|N} (App. B), the index
 * set {(m,n,k): kappa <= E_cut} under the clamps (Sec. 3.2), the grid
 * theta1_i = i/n_t1, theta2_j = j/(N n_t2) and the n_r-point Gauss-Jacobi rule
 * for int_0^1 f(q) q dq (Sec. 3.1, App. D), and the radial tables
 * xi_{|n|,k}(r_l) and (2 pi tau / N) omega_l xi_{|n|,k}(r_l) (Alg. 1, Alg. 3).  Automatic grids
 * use the smallest 2,3,5-smooth sizes >= 2 max|m| + 2 and >= 2 max|n| + 2.
 * Synchronous; allocates no device memory (device tables are uploaded by the
 * first call that needs them).  *out receives a handle owned by the caller,
 * released with helic_basis_destroy. */
helic_status helic_basis_create(const helic_params* p, helic_basis* out);
helic_status helic_basis_destroy(helic_basis h);

/* Sizes: basis size L, grid sizes, number of angular modes (m, n) kept. Any
 * output pointer may be NULL.  Host only. */
helic_status helic_basis_info(helic_basis h, int64_t* L, int32_t* n_t1, int32_t* n_t2,
                              int32_t* n_r, int32_t* n_modes);

/* Compact row order: mnk (host, L*3 int32) receives (m, n, k) of every row;
 * kappa (host, L doubles) the kinetic diagonal.  Rows are grouped by |n|
 * (0, 1, 2, ...), then n = +|n| before -|n|, then m ascending, then k = 1..K.
 * Either pointer may be NULL. */
helic_status helic_basis_indices(helic_basis h, int32_t* mnk, double* kappa);

/* Grid (host arrays): theta1 (n_t1), theta2 (n_t2), r (n_r, Bohr) and the
 * radial weights w_r (n_r; omega_l = R^2 w_l, including the r dr Jacobian).
 * Any pointer may be NULL. */
helic_status helic_grid(helic_basis h, double* theta1, double* theta2, double* r, double* w_r);

/* Potential V (device, n_t1*n_t2*n_r doubles, real-space order).  The
 * library keeps its own re-laid-out copy; V may be freed after the stream
 * passes this call. */
helic_status helic_set_potential(helic_basis h, const double* V, void* stream);

/* Y = H X for nvec columns (device blocks, see conventions; X and Y must not
 * overlap).  Requires a potential.  The first call with a larger nvec than
 * before grows the library's intermediate buffer (hipMalloc). */
helic_status helic_apply_H(helic_basis h, const double* X, int64_t ldx, double* Y, int64_t ldy,
                           int32_t nvec, helic_prec prec, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): Y = H X
 * exactly as helic_apply_H computes it, with the intermediate slabs in a
 * fixed scratch array of HELIC_NOALLOC_SCRATCH_MIB MiB per GPU instead of
 * the handle's growable buffer.  The array is part of the library's device
 * code: each GPU the library runs on holds one copy from the first basis
 * set-up on it until the process ends.  The call allocates nothing (no
 * hipMalloc, hipFree or allocating library routine); the caller passes X and
 * Y as for helic_apply_H.  Vectors go through the stages in chunks of
 * min(64, scratch / (n_r * n_modes * 16 bytes in FP64, 8 in FP32)).
 * Requires a potential (helic_set_potential, which also completes the
 * device set-up) on the current device.  All calls on one GPU share its
 * array and leave their last chunk's slabs in it (nothing in it has to start
 * at zero: every slab element is written before it is read); calls that
 * overlap on one GPU (two streams or two host threads) race, so the caller
 * serialises them.  Errors: as helic_apply_H; HELIC_ERR_STATE without a
 * potential or on another device; HELIC_ERR_NOMEM when one vector's slabs
 * (n_r * n_modes complex values) exceed the array. */
#define HELIC_NOALLOC_SCRATCH_MIB 64
helic_status helic_apply_H_noalloc(helic_basis h, const double* X, int64_t ldx, double* Y, int64_t ldy,
                                   int32_t nvec, helic_prec prec, void* stream);

/* Inverse basis transform (Alg. 1 and 2) of nvec coefficient columns onto the
 * grid: g (device) holds nvec consecutive real-space arrays of complex
 * doubles, n_t1*n_t2*n_r each.  Forward transform (Alg. 3 and 4):
 * coefficients of nvec such arrays, by quadrature.  FP64. */
helic_status helic_transform_inverse(helic_basis h, const double* X, int64_t ldx, double* g,
                                     int32_t nvec, void* stream);
helic_status helic_transform_forward(helic_basis h, const double* g, double* X, int64_t ldx,
                                     int32_t nvec, void* stream);

/* Derivatives of the fields given by nvec coefficient columns (App. C):
 * grad (device) receives three blocks of nvec real-space arrays of complex
 * doubles (n_t1*n_t2*n_r each, the inverse transform's layout): with
 * cartesian = 0 the helical derivatives E_theta1 (transform of the
 * coefficients times i 2 pi m), E_theta2 (times i 2 pi N n) and E_r (the
 * transform with d xi_{|n|,k} / dr as radial functions, eqs. E_r and B_r);
 * with cartesian = 1 the Cartesian E_x, E_y, E_z from them by eq.
 * Cartesian_Derivatives.  FP64.  The first call uploads the derivative
 * tables and grows a coefficient workspace (hipMalloc).  Asynchronous on
 * `stream`.  Errors: HELIC_ERR_INVALID for null pointers with nvec > 0,
 * ldx < L or cartesian outside {0, 1}. */
helic_status helic_gradient(helic_basis h, const double* X, int64_t ldx, int32_t nvec, double* grad,
                            int32_t cartesian, void* stream);

/* Electron density on the grid (Sec. 4.2, the density equation, one (eta_b,
 * nu) term of its sums): rho = sum_j occ_j |phi_j|^2, phi_j the inverse
 * transform (Alg. 1 and 2) of coefficient column j of X (device block, see
 * conventions).  occ (host, nvec doubles) carries each state's whole weight,
 * (2 / N) w_b s_j, so that the caller sums several calls over (eta_b, nu)
 * with accumulate = 1.  rho (device, n_t1*n_t2*n_r doubles in the
 * potential's order: theta1 outermost, r fastest) is overwritten
 * (accumulate = 0) or added to (1); nvec = 0 with accumulate = 0 zeroes it.
 * FP64; the states are summed in column order (deterministic).  The first
 * call grows a real-space workspace of 16 grids (hipMalloc); no potential
 * is needed.  Synchronises `stream` before returning. */
helic_status helic_density(helic_basis h, const double* X, int64_t ldx, int32_t nvec,
                           const double* occ, double* rho, int32_t accumulate, void* stream);

/* Timing aid: run `nrep` applications of H to the same block exactly as
 * helic_apply_H does (nvec <= 64), each of the three stage kernels (radial
 * inverse, angular, radial forward) carrying start and end events on its own
 * dispatch (timing-only events, no system-scope fence).  ms_stage (host, 3
 * doubles) receives each kernel's mean duration in ms and *ms_total (host,
 * may be NULL) the mean span of one whole application, first kernel start to
 * last kernel end.  Synchronises `stream` before returning. */
helic_status helic_profile_apply(helic_basis h, const double* X, int64_t ldx, double* Y, int64_t ldy,
                                 int32_t nvec, helic_prec prec, int32_t nrep, void* stream,
                                 double* ms_stage, double* ms_total);

/* Teter-Payne-Allan preconditioner (Sec. 3.5) of nvec residual columns:
 * W_ij = K(kappa_i / T_j) R_ij, K(g) = (27+18g+12g^2+8g^3) /
 * (27+18g+12g^2+8g^3+16g^4), T_j = sum_i kappa_i |R_ij|^2 / sum_i |R_ij|^2
 * (zero columns stay zero).  Device blocks; W may equal R (in place). */
helic_status helic_precondition(helic_basis h, const double* Rres, int64_t ldr, double* W,
                                int64_t ldw, int32_t nvec, void* stream);

/* Lowest nev eigenpairs by block LOBPCG (Sec. 3.5) with the preconditioner
 * above, FP64 Rayleigh-Ritz, H applied in `prec` with a final FP64
 * refinement when prec != HELIC_FP64 (a precision ladder: BF16 until the
 * worst wanted residual is below 1e-2, FP32 until 1e-5, then FP64; a lower
 * rung also ends when that residual has not improved by 10 % for 10
 * iterations, or 3 filter steps in the filtered solver).  Converged when every
 * ||H x - lambda x||_2 <= tol with ||x||_2 = 1.  evals, resid (host, nev):
 * eigenvalues ascending and residual norms; evecs (device, ld >= L, nev
 * columns) may be NULL; iters (host) may be NULL.  seed fixes the random
 * start.  Synchronises `stream` before returning.  Returns HELIC_ERR_NOCONV
 * (with the best current results written) when maxit is reached. */
helic_status helic_eigensolve(helic_basis h, int32_t nev, int32_t block, double tol, int32_t maxit,
                              helic_prec prec, uint64_t seed, double* evals, double* resid,
                              double* evecs, int64_t ldv, int32_t* iters, void* stream);

/* Options and statistics of helic_eigensolve_ex. */
typedef struct {
  int32_t nev;        /* wanted eigenpairs (lowest), 1 <= nev <= L                     */
  int32_t block;      /* columns per H*X launch, 1..64                                 */
  double tol;         /* target ||H x - lambda x||_2 for ||x||_2 = 1 (Ha)              */
  int32_t maxit;      /* iteration limit                                               */
  int32_t prec;       /* helic_prec of the H*X applications (FP32: FP64 takes over)    */
  uint64_t seed;      /* random start                                                  */
  int32_t precond;    /* 0: Teter-Payne-Allan, 1: none, 2: learned (helic_lpc_*)       */
  int32_t guard;      /* extra iterated columns beyond nev (-1: automatic)             */
  double switch_tol;  /* FP32/BF16: residual below which FP64 applications take over  */
                      /* (0: 1e-5)                                                     */
  int32_t log_every;  /* > 0: one progress line on stderr every log_every iterations   */
  double switch_tol_bf16; /* BF16 mode: residual below which FP32 takes over (0: 1e-2)  */
  int32_t stop_low;   /* 1: stop at the first precision switch, by tolerance or by     */
                      /* stagnation (results of the lower precision alone, for error   */
                      /* studies); 0: refine to tol in FP64                            */
} helic_solve_opts;

typedef struct {
  int32_t iters;        /* iterations run                                             */
  int32_t iters_low;    /* of which with FP32 H*X                                     */
  int64_t n_apply;      /* H*X column applications                                    */
  int32_t n_fallback;   /* iterations where the learned preconditioner fell back      */
  double t_apply_ms;    /* time in H*X                                                */
  double t_rr_ms;       /* time in orthogonalisation and Rayleigh-Ritz                */
  double t_precond_ms;  /* time in residuals and the preconditioner                   */
  double t_total_ms;    /* wall time of the call                                      */
  int32_t iters_bf16;   /* of iters_low, iterations with BF16 H*X                     */
  int32_t n_graphs;     /* filtered solver: filter recurrences captured as HIP graphs */
} helic_solve_stats;

/* As helic_eigensolve with all options; stats (host) may be NULL. */
helic_status helic_eigensolve_ex(helic_basis h, const helic_solve_opts* opts, double* evals,
                                 double* resid, double* evecs, int64_t ldv, helic_solve_stats* stats,
                                 void* stream);

/* Lowest nev eigenpairs by Chebyshev-filtered subspace iteration, the kind
 * of eigensolver Sec. 3.5 names as the more efficient choice for later work.
 * Each outer step filters the nev + guard columns with a degree-`degree`
 * Chebyshev polynomial of H (scaled three-term recurrence; damped interval
 * from the block's largest Ritz value to an upper bound of the spectrum
 * taken from a 12-step FP64 Lanczos run), orthonormalises them (Cholesky QR,
 * SVQB fallback, random refill of collapsed directions) and rotates them by
 * FP64 Rayleigh-Ritz; degree * (nev + guard) column applications per step.
 * degree 0 picks 32; 1..200 accepted.  guard -1 picks max(8, nev / 3).  opts, outputs, convergence test,
 * FP32 ladder (prec, switch_tol), stats and errors as helic_eigensolve_ex;
 * opts->precond is not used (the filter takes the preconditioner's place);
 * stats->iters counts outer steps, t_apply_ms the filter recurrence (H*X
 * and its elementwise steps, queued without host synchronisation) and
 * t_precond_ms the residuals.  The recurrence of an outer step (m - 1
 * applications of H and m elementwise steps, coefficients read from device
 * memory) is captured into a HIP graph and replayed while the locked count
 * and the precision stay the same (stats->n_graphs counts the captures); a
 * null `stream` is replaced by a stream of the solver's own. */
helic_status helic_eigensolve_chefsi(helic_basis h, const helic_solve_opts* opts, int32_t degree,
                                     double* evals, double* resid, double* evecs, int64_t ldv,
                                     helic_solve_stats* stats, void* stream);

/* ---- batches of Bloch parameters / structures (Sec. 3.3) ----------------
 * A batch groups problems (basis handles, each with its potential set, all on
 * one device) -- e.g. the Bloch parameters eta_b of several structures.
 * Problems that share the grid (n_t1, n_t2, n_r) and the angular kernel
 * variant form a class; each H*X stage runs as one launch over the ragged
 * work of all problems of a class, the classes one after another on the
 * stream.  The batch borrows the handles (they must outlive it).  Batched
 * blocks are concatenated: problem p's nvec columns (ld = L_p, column-major,
 * complex) start at complex offset nvec * offsets[p], offsets from
 * helic_batch_info (nprob + 1 entries). */
typedef struct helic_batch_s* helic_batch;
helic_status helic_batch_create(const helic_basis* bases, int32_t nprob, helic_batch* out);
helic_status helic_batch_destroy(helic_batch b);
helic_status helic_batch_info(helic_batch b, int64_t* offsets /* host, nprob + 1 */);
/* Number of classes (host, may be NULL) and each problem's class (host,
 * nprob entries, may be NULL). */
helic_status helic_batch_classes(helic_batch b, int32_t* nclasses, int32_t* class_of);
/* Y = H X for every problem of the batch, 1 <= nvec <= 64 (device blocks). */
helic_status helic_batch_apply(helic_batch b, const double* X, double* Y, int32_t nvec, helic_prec prec,
                               void* stream);
/* Capture the batched apply on these buffers (every class) into one HIP
 * graph (replaces any previous one); helic_batch_replay launches it on
 * `stream`.  A replay reads X and writes Y as captured.  Tuning releases the
 * graph. */
helic_status helic_batch_capture(helic_batch b, const double* X, double* Y, int32_t nvec, helic_prec prec);
helic_status helic_batch_replay(helic_batch b, void* stream);
/* Choices of the tuner for one class. */
typedef struct {
  int32_t n_t1, n_t2, n_r;   /* the class's grid                                        */
  int32_t nprob;             /* problems in the class                                   */
  int32_t items_per_wg;      /* angular stage: (problem, radius, vector) items per      */
                             /* workgroup, 0 = spread over the resident workgroups      */
  int32_t inv_ksteps;        /* radial inverse: k steps (of 4) held in registers        */
  int32_t fwd_pipelined;     /* radial forward: 1 pipelined kernel, 0 plain kernel      */
  int32_t fwd_tiles;         /* radial forward: 16 x 16 output tiles per wave           */
  double ms;                 /* the class's three stages with these choices (ms)         */
} helic_batch_class_tuning;
/* Tuner: per class, times the class's three stages with each candidate of
 * one knob at a time -- the angular work split (0, 2, 4, 8, 16 items per
 * workgroup, where the specialised angular kernels serve the class), the
 * radial inverse's register k steps (the smallest that covers the class, or
 * 24) and the radial forward variant (pipelined with 8 or 4 register tiles
 * per wave where every problem fits it, plain with 4 or 8; BF16 keeps its
 * kernels) -- on these buffers, keeps the fastest and records it: out (host,
 * max_classes entries, may be NULL), *nclasses (host, may be NULL).
 * Synchronises `stream`; results are unchanged to rounding order. */
helic_status helic_batch_tune_classes(helic_batch b, const double* X, double* Y, int32_t nvec, helic_prec prec,
                                      void* stream, helic_batch_class_tuning* out, int32_t max_classes,
                                      int32_t* nclasses);
/* The same tuner; *chosen (host, may be NULL) receives the first class's
 * angular work split and *ms_best (host, may be NULL) the sum over classes
 * of the tuned stage times. */
helic_status helic_batch_tune(helic_batch b, const double* X, double* Y, int32_t nvec, helic_prec prec,
                              void* stream, int32_t* chosen, double* ms_best);
/* Lowest opts->nev eigenpairs of every problem, solved concurrently on
 * `nstreams` streams.  evals, resid: host, nprob * nev (problem-major);
 * stats, status: host, nprob entries, may be NULL.  Returns the first hard
 * error, else HELIC_ERR_NOCONV if some problem did not converge. */
helic_status helic_batch_eigensolve(helic_batch b, const helic_solve_opts* opts, int32_t nstreams,
                                    double* evals, double* resid, helic_solve_stats* stats,
                                    int32_t* status);
/* Time-reversal halving (Sec. 3.3): with enable = 1, a problem whose eta is
 * the negative of an earlier problem's (0 < |eta| < 1/2) with the same
 * geometry, cutoff, clamps, grid and potential (compared exactly) is not
 * solved by the batched eigensolvers: it takes that problem's eigenvalues and
 * residuals (lambda_j(eta) = lambda_j(-eta)), and its stats entry is zero.
 * *npairs (host, may be NULL) receives the number of such problems.
 * enable = 0 solves every problem again.  Reads the potentials back once
 * (synchronous); the pairing holds until the next call, so call again after
 * changing a potential.  Partners are (eta, nu) and (-eta, (N - nu) mod N)
 * (Sec. 3.3). */
helic_status helic_batch_time_reversal(helic_batch b, int32_t enable, int32_t* npairs);
/* As helic_batch_eigensolve, each problem by Chebyshev-filtered subspace
 * iteration (helic_eigensolve_chefsi; degree 0 picks 32). */
helic_status helic_batch_eigensolve_chefsi(helic_batch b, const helic_solve_opts* opts, int32_t degree,
                                           int32_t nstreams, double* evals, double* resid,
                                           helic_solve_stats* stats, int32_t* status);

/* ---- learned diagonal preconditioner -----------------------------------
 * Not in the paper, which only remarks (Sec. 5) that the method lends itself
 * to coupling with machine learning.  For residual column j and row i a
 * network of three layers (8 -> 64 -> 64 -> 1, SiLU) maps the features
 *   K(g), log g, log kappa_i, (V_ii - lambda_j) / T_j, lambda_j / T_j,
 *   log(|R_ij| sqrt(L) / ||R_j|| + 1e-30), 0, 0      (g = kappa_i / T_j)
 * (K, T_j as for helic_precondition; V_ii the potential's diagonal in the
 * basis; lambda_j the column's Ritz value) to z, and the correction is
 *   W_ij = s_ij R_ij,  s_ij = K(g) softplus(z) / log 2 > 0:
 * diagonal, positive and phase-equivariant, so LOBPCG stays valid; a zero
 * last layer gives the Teter-Payne-Allan preconditioner exactly.  Training
 * minimises the mean over columns of 1 - |<s R_j, T_j>|^2 / (||s R_j||^2
 * ||T_j||^2) against target corrections T_j, with Adam.  Parameters (FP32,
 * HELIC_LPC_NPARAM): W1 (64 x 8, row-major), b1 (64), W2 (64 x 64, row-major),
 * b2 (64), w3 (64), b3 (1).  A network handle lives on the device current at
 * creation; calls on one network must not overlap (they share its training
 * buffers), and it must outlive the bases it is attached to.  Device blocks
 * are column-major complex FP64 (ld >= L), lambda / lam arrays are device
 * FP64 (one per column). */
#define HELIC_LPC_NPARAM 4801
typedef struct helic_lpc_s* helic_lpc;
/* New network with He-initialised hidden layers and a zero last layer. */
helic_status helic_lpc_create(uint64_t seed, helic_lpc* out);
helic_status helic_lpc_destroy(helic_lpc net);
/* Copy the parameters out / in (host, HELIC_LPC_NPARAM floats); setting
 * them restarts Adam. */
helic_status helic_lpc_get_params(helic_lpc net, float* params);
helic_status helic_lpc_set_params(helic_lpc net, const float* params);
/* Weights file: a 16-byte header ("HELICLPC", format version 1 and the
 * parameter count as little-endian int32) followed by the HELIC_LPC_NPARAM
 * FP32 parameters, little-endian.  Loading validates the header and the
 * values (finite) and restarts Adam; a failed load leaves the network as it
 * was.  Host file I/O; errors: HELIC_ERR_INVALID (bad path or file). */
helic_status helic_lpc_save(helic_lpc net, const char* path);
helic_status helic_lpc_load(helic_lpc net, const char* path);
/* Use `net` for helic_eigensolve_ex with precond = 2 on this basis (NULL
 * detaches).  The solver falls back to the Teter-Payne-Allan preconditioner
 * for the rest of a solve once the largest residual of the wanted pairs has
 * not reached a new minimum for three iterations in a row. */
helic_status helic_lpc_attach(helic_basis h, helic_lpc net);
/* V_ii per row in the compact order (host, L doubles), computed on the
 * device by helic_set_potential; synchronises the device. */
helic_status helic_lpc_vdiag(helic_basis h, double* vdiag);
/* W = s * R for nvec columns with Ritz values lam (W may equal R). */
helic_status helic_lpc_apply(helic_basis h, helic_lpc net, const double* R, int64_t ldr, const double* lam,
                             double* W, int64_t ldw, int32_t nvec, void* stream);
/* Direction loss of nvec (R, T, lam) columns and its gradient: *loss (host)
 * the mean over columns; grad (host, HELIC_LPC_NPARAM doubles) may be NULL.
 * The gradient also stays in the network for helic_lpc_adam_step.
 * Synchronises `stream`. */
helic_status helic_lpc_loss_grad(helic_basis h, helic_lpc net, const double* R, int64_t ldr, const double* T,
                                 int64_t ldt, const double* lam, int32_t nvec, double* loss, double* grad,
                                 void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the last gradient. */
helic_status helic_lpc_adam_step(helic_lpc net, double lr, void* stream);
/* `steps` Adam steps, each on `batch` columns drawn without replacement
 * (seeded) from the ncol training columns; losses (host, steps) may be
 * NULL.  Synchronises `stream`. */
helic_status helic_lpc_train(helic_basis h, helic_lpc net, const double* R, int64_t ldr, const double* T,
                             int64_t ldt, const double* lam, int32_t ncol, int32_t batch, int32_t steps,
                             double lr, uint64_t seed, double* losses, void* stream);
/* Training pairs from one eigensolve (opts as helic_eigensolve_ex, run with
 * the preconditioner opts->precond): at up to n_snap iterations spread
 * geometrically over the run, the residuals R_j of the unconverged wanted
 * columns and their Ritz values are kept together with the Ritz block X;
 * after convergence each target is T_j = (1 - X X^H) X* X*^H x_j, the part of
 * the final eigenspace X* (nev columns) that the column still has to gain.
 * R, T: device, ld = L, max_cols columns; lam: device, max_cols; *ncol
 * (host): columns written.  stats may be NULL. */
helic_status helic_lpc_harvest(helic_basis h, const helic_solve_opts* opts, int32_t n_snap, int32_t max_cols,
                               double* R, double* T, double* lam, int32_t* ncol, helic_solve_stats* stats,
                               void* stream);

/* Host utilities used by the basis set-up, exported for testing.
 * helic_util_bessel_j: out[i] = J_p(x[i]) for integer p (any sign), x >= 0.
 * helic_util_bessel_zeros: first `count` positive zeros of J_p.
 * helic_util_gauss_jacobi: n-point rule for int_0^1 f(q) q dq (nodes q,
 * weights w, ascending). */
helic_status helic_util_bessel_j(int32_t p, int32_t n, const double* x, double* out);
helic_status helic_util_bessel_zeros(int32_t p, int32_t count, double* out);
helic_status helic_util_gauss_jacobi(int32_t n, double* q, double* w);

const char* helic_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HELIC_H */
