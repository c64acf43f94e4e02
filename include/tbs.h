/*
 * tbs.h -- C ABI of the MI355X traditional-Born-series (TBS) Helmholtz solver.
 *
 * The library evaluates the Born series of the Lippmann-Schwinger equation
 *     psi = G V psi + G S                      (paper Sec. 2.2, Eq. TBS_1)
 * term by term,
 *     u_0 = G s,  u_n = G (V u_{n-1}),  p = sum_{n<L} u_n
 *                                   (Sec. 2.2, Eqs. TBS_2, TBS_input, TBS_algorithm)
 * where G is the free-space Green's-function convolution (Sec. 2.2,
 * Eqs. soln_greens_fn and greens_fn) evaluated with zero-padded FFTs, and
 * V(x) = k(x)^2 - k0^2 carries sound speed, absorption and dispersion
 * (Sec. 2.1.2, Sec. 2.3.3 Eq. TBS_equation_inhomogeneous).
 *
 * Conventions (all entry points):
 *  - Arrays are C order with x fastest: 2D [y][x], 3D [z][y][x]; a batch of B
 *    right-hand sides is [B][...].  Complex values are interleaved (re, im):
 *    dtype TBS_C64 = 2 x float (bit-compatible with torch.complex64),
 *    TBS_C128 = 2 x double (torch.complex128).
 *  - "dev" pointers are device (HBM) pointers on the plan's device, owned by
 *    the caller, and must stay valid until the work queued on the plan's
 *    stream has finished.  "host" pointers are ordinary host memory.
 *  - Work is queued asynchronously on the plan's HIP stream; an entry point
 *    blocks only when it returns values to host memory (residual_out,
 *    exports).
 *  - Return value: TBS_OK (0) on success; a negative TBS_ERR_* code leaves the
 *    outputs unspecified; a positive TBS_WARN_* code means the outputs are
 *    written but suspicious.  tbs_last_error() describes the last failure of a
 *    plan.  No C++ exception crosses this interface.
 *  - A plan is not thread-safe; distinct plans are independent.
 */
#ifndef TBS_H
#define TBS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tbs_plan tbs_plan;
typedef struct {
  double re, im;
} tbs_c128;

enum tbs_dtype {
  TBS_C64 = 0,  /* complex FP32; partial sums Kahan-compensated */
  TBS_C128 = 1  /* complex FP64; plain summation */
};

enum tbs_status {
  TBS_OK = 0,
  TBS_ERR_INVALID = -1,     /* bad argument (NULL, size, range, dtype) */
  TBS_ERR_UNSUPPORTED = -2, /* valid request the library has no kernel for */
  TBS_ERR_OOM = -3,         /* device allocation failed; nothing leaked */
  TBS_ERR_HIP = -4,         /* a HIP runtime call failed */
  TBS_ERR_STATE = -5,       /* call out of order (e.g. solve before tabulate) */
  TBS_WARN_NONFINITE = 1,   /* a residual is NaN/Inf (non-finite input?) */
  TBS_WARN_DIVERGING = 2,   /* residuals grew over 3 consecutive terms */
  TBS_WARN_NOT_CONVERGED = 3 /* tbs_iterate reached max_iter above the tolerance */
};

/* Case II potential of the paper's periodic scheme in k-space (Sec. 2.3.2,
 * Eq. TBS_solution_absorbing-dispersive): VV(p) = eta |p|^(nu+1)
 * - i (tau omega |p|^nu + eps), tau = -2 alpha0 c^(nu-1),
 * eta = 2 alpha0 c^nu tan(pi nu / 2) (Sec. 2.1.2). */
typedef struct {
  double tau, eta, nu, omega;
} tbs_kspace_potential;

enum tbs_iterate_flags {
  TBS_ITER_PAPER = 0, /* the paper's fixed-point iteration (Algorithm 1) */
  TBS_ITER_CBS = 1    /* the convergent Born series the paper names as its extension */
};

enum tbs_adjoint_flags {
  TBS_ADJ_STORE = 0,      /* keep all L-1 forward partial sums in HBM */
  TBS_ADJ_RECOMPUTE = 1,  /* keep ~sqrt(L) checkpoints and recompute segments */
  TBS_ADJ_SERIES_ONLY = 2 /* only the adjoint field A_L^H q (no gradient pairing) */
};

/* Library version (major*10000 + minor*100 + patch). */
int tbs_version(void);

/* Human-readable name of a status code (static string). */
const char *tbs_status_string(int status);

/* ---- host-side helpers (no device needed) ------------------------------ */

/* Padded FFT length the library uses for n physical points: the smallest
 * length with compiled kernels that is >= padding*n - 1 (>= 2n - 1 makes the
 * circular convolution equal the linear one, Sec. 2.2 Eq. TBS_1).  Even.
 * TBS_ERR_UNSUPPORTED if no compiled length is large enough. */
int tbs_padded_length(int64_t n, int padding, int64_t *m_out);

/* Complex wavenumber of a power-law absorbing, dispersive medium,
 * k = omega/c + alpha0 omega^y (i + tan(pi y/2)), and k = omega/c + i alpha0
 * omega for y == 1 (first-order solution of the plane-wave relation of
 * Sec. 2.1.2, Eq. acoustic_waveequn_time_independent_absorbing_dispersion;
 * alpha0 in Np m^-1 (rad/s)^-y, Eq. power_law_absorption). */
int tbs_wavenumber(double omega, double c, double alpha0, double y, tbs_c128 *k_out);

/* Background wavenumber k0 with k0^2 = k(c0)^2 + i eps, Im k0 >= 0
 * (Sec. 2.2, Eq. acoustic_waveequn6; eps = 0 is the default reading). */
int tbs_background_k0(double omega, double c0, double alpha0, double y, double eps,
                      tbs_c128 *k0_out);

/* FP64 Hankel functions H0^(1)(z), H1^(1)(z) for Re z > 0, Im z >= 0, as used
 * by the 2D Green's function (i/4) H0(k0 r).  Exposed for testing. */
int tbs_hankel01(tbs_c128 z, tbs_c128 *h0_out, tbs_c128 *h1_out);

/* Self-cell weight W(0): the integral of the Green's function over the disk
 * (ndim 2) or ball (ndim 3) with the area/volume of one cell of side dx. */
int tbs_self_cell(int ndim, tbs_c128 k0, double dx, tbs_c128 *w0_out);

/* ---- plans ------------------------------------------------------------- */

/* Create a plan for the operator G on an ndim-dimensional grid.
 *   grid[3]   : N_x, N_y, N_z physical points (grid[2] ignored when ndim=2)
 *   dx        : cell size [m], > 0
 *   k0        : complex background wavenumber, Re k0 > 0, Im k0 >= 0
 *   padding   : >= 2; padded length per axis = tbs_padded_length(N, padding).
 *               1: a periodic plan of the paper's own scheme (no padding,
 *               M = N; 2D, N_x and N_y powers of two in [16, 4096], else
 *               TBS_ERR_UNSUPPORTED), used by tbs_green_periodic and
 *               tbs_iterate only (the padded-series calls return
 *               TBS_ERR_STATE on it; k0 is the k of g~)
 *   dtype     : TBS_C64 or TBS_C128 (precision of the series)
 *   batch     : B >= 1 right-hand sides per solve (they share V and G)
 *   hip_stream: hipStream_t to queue work on (NULL = the null stream)
 * Allocates the plan's device buffers (twiddles, intermediates, Kahan
 * compensation).  *out is NULL on failure.  TBS_ERR_OOM leaks nothing. */
int tbs_plan_create(tbs_plan **out, int ndim, const int64_t grid[3], double dx, tbs_c128 k0,
                    int padding, int dtype, int batch, void *hip_stream);

/* Padded lengths (M_x, M_y, M_z; M_z = 1 in 2D) and device bytes held. */
int tbs_plan_info(const tbs_plan *plan, int64_t padded_out[3], int64_t *device_bytes_out);

/* Queue later work on another stream. */
int tbs_plan_set_stream(tbs_plan *plan, void *hip_stream);

/* Autotuner: time the block-shape candidates of the row and column passes
 * (2D: rows per row-pass block and columns per convolution block; 3D: z lines
 * per block of the z convolution) on this plan's shapes and keep the fastest.  The choice never changes the field arithmetic
 * (p_out is bitwise identical; the FP64 residual norms are summed in another
 * grouping and may differ in the last bits); it is cached per (device model,
 * grid, padded lengths, batch, dtype) for the life of the process and, when
 * the environment variable TBS_TUNE_CACHE names a file, in that file (read on
 * first use, one line appended per new choice).  Needs the spectrum (call after tbs_green_tabulate);
 * clobbers the plan's intermediate buffers; synchronous.  Outputs (may be
 * NULL): the chosen rows and columns per block. */
int tbs_plan_autotune(tbs_plan *plan, int *row_nr_out, int *conv_nc_out);

/* Tabulate the Green spectrum in FP64 on the device: W(m) = dx^d g(k0,|m|dx)
 * on the padded grid (W(0) = tbs_self_cell), forward FFT, scale 1/prod(M),
 * fold to the [0, M_x/2] x [0, M_y/2] (x [0, M_z/2]) table, round to the plan
 * dtype.  Must precede tbs_solve/tbs_adjoint.  Blocks until done. */
int tbs_green_tabulate(tbs_plan *plan);

/* Test seam: replace the spectrum by fftn(W_pad) given on the host as a full
 * complex128 array [M_z][M_y][M_x] (unnormalised; must be even per axis). */
int tbs_green_import(tbs_plan *plan, const tbs_c128 *full_host);

/* Copy the folded, normalised table to the host as complex128
 * [M_x/2+1][M_y/2+1] (2D) or [M_x/2+1][M_y/2+1][M_z/2+1] (3D). */
int tbs_green_export(const tbs_plan *plan, tbs_c128 *folded_host);

/* Potential V = k(c)^2 - k0^2 (and optionally dV/dc = -2 k omega / c^2) of a
 * sound-speed map c (dev, float64 [P]) at angular frequency omega, with
 * k0^2 = k(c0)^2 + i eps.  V_dev / dVdc_dev: dev, plan dtype [P]; either may
 * be NULL. */
int tbs_potential(tbs_plan *plan, const double *c_dev, double omega, double c0, double alpha0,
                  double y, double eps, void *V_dev, void *dVdc_dev);

/* The L-term Born series for the plan's B right-hand sides.
 *   source      : dev [B][P] plan dtype, the source density s
 *   potential   : dev [P] plan dtype, V; NULL means V = 0 (then p = u_0)
 *   nterms      : L >= 1 summed terms, u_0 included
 *   p_out       : dev [B][P] plan dtype; receives p = sum_{n<L} u_n
 *   residual_out: host double [B][L] or NULL; receives ||u_n|| / ||sum_{m<=n} u_m||
 *                 (whole-grid L2 in FP64; Sec. 3.1 Eq. Error).  Non-NULL makes
 *                 the call synchronous and enables the TBS_WARN_* checks.
 * p_out must not alias source or potential. */
int tbs_solve(tbs_plan *plan, const void *source, const void *potential, int nterms,
              void *p_out, double *residual_out);

/* tbs_solve for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, results (bitwise) and errors as tbs_solve, but the series'
 * workspace (x-spectral intermediate, 3D y intermediate, Kahan compensation,
 * norm partials, residuals) lives in a static device array of the library,
 * 128 MiB per GPU, held from the first call on a device until the process
 * ends; no device memory is allocated or freed.  Plans whose workspace
 * exceeds it (e.g. 2048^2 FP32 with B >= 2: B (M_x N_y 8 + P 4) bytes plus
 * partials) return TBS_ERR_UNSUPPORTED, as do density-contrast plans.  The
 * array keeps the last call's contents; every region is overwritten before it
 * is read.  All calls on one GPU share that GPU's array: calls that overlap
 * in time on one device (concurrent streams, threads or processes) race and
 * give undefined results. */
int tbs_solve_noalloc(tbs_plan *plan, const void *source, const void *potential, int nterms,
                      void *p_out, double *residual_out);

/* Second-harmonic source S2 = -(1/2) xi (2 omega)^2 p1^2, xi = (1 + B/2A) /
 * (rho c^4) with the local sound speed c (Sec. 2.1.4 Eq. nonlinear_waveeqn_shi2,
 * Sec. 2.3.4 Eq. TBS_solution_shi_2, sum term only).
 *   p1_dev: dev [B][P] plan dtype (fundamental field); c_dev: dev float64 [P];
 *   S2_dev: dev [B][P] plan dtype (may alias p1_dev). */
int tbs_harmonic_source(tbs_plan *plan, const void *p1_dev, const double *c_dev, double omega,
                        double rho, double BA, void *S2_dev);

/* Source of the n-th harmonic (2 <= n <= 9) from the lower harmonics, sum-
 * frequency terms only (Sec. 2.1.4, the nonlinear wave equations with sum
 * terms; Sec. 2.3.4, Eq. TBS_solution_nonlinear_shi_n):
 *   S_n = -(1/2) xi (n omega)^2 sum_{a=1}^{n-1} psi_a psi_{n-a},
 *   xi = (1 + B/2A) / (rho c^4), local sound speed c, omega the fundamental;
 *   e.g. psi_1 psi_2 for n = 3, psi_2^2/2 + psi_1 psi_3 for n = 4.
 *   fields_dev: host array of n-1 device pointers psi_1 .. psi_{n-1}, each
 *               dev [B][P] plan dtype; c_dev: dev float64 [P];
 *   S_dev: dev [B][P] plan dtype (may alias any field).
 * Products and sums are formed in FP64 and rounded once.  n = 2 equals
 * tbs_harmonic_source.  Errors: TBS_ERR_INVALID for n out of range, a NULL
 * pointer or bad parameters. */
int tbs_harmonic_source_n(tbs_plan *plan, int n, const void *const *fields_dev, const double *c_dev,
                          double omega, double rho, double BA, void *S_dev);

/* The n-th harmonic source of tbs_harmonic_source_n on scaled fields, for
 * chains whose higher harmonics fall below the FP32 range (in the paper's
 * 4096^2 setup the 5th harmonic is about 1e-39; Sec. 3.1, Table 3).  Field a
 * (a = 1 .. n-1) holds psi_a * 2^field_exp[a-1] (host int [n-1], |e| <= 900);
 * the products and sums run in FP64 on the unscaled values, and S_out
 * receives S_n * 2^e with e (*exp_out) chosen so that the largest real or
 * imaginary part of S_n * 2^e lies in [1, 2) (e = 0 for S_n = 0).  Because
 * each solve is linear in its source, the series or iteration driven by
 * S_out returns psi_n * 2^e: the caller passes e as field n's exponent to the
 * next order.  Two passes over the fields (maximum, then the scaled values)
 * and one device-to-host copy of the maximum (synchronises the plan's stream).
 * Returns TBS_ERR_INVALID for a non-finite source. */
int tbs_harmonic_source_scaled(tbs_plan *plan, int n, const void *const *fields, const int *field_exp,
                               const double *c_dev, double omega, double rho, double BA, void *S_out,
                               int *exp_out);

/* Attach a density contrast to a padded 2D or 3D plan (NULL detaches): the term
 * div(gamma grad psi) of the inhomogeneous wave equation (Sec. 2.1.3, Eqs.
 * acoustic_waveequn_time_dependent_inhomogeneous and mismatch_parameters,
 * gamma = (rho_s - rho_f) / rho_s; the paper drops it for rho_s ~ rho_f)
 * joins the potential of every term: u_n = G(V u_{n-1} - div(gamma grad
 * u_{n-1})), in conservative second-order differences with gamma at the half
 * points the mean of the two cells and zero outside the grid.
 *   gamma_dev: dev float64 [N_y][N_x] or [N_z][N_y][N_x], owned by the caller, read by every
 *              later tbs_solve until detached (the potential of tbs_solve
 *              may then be NULL: V = 0).
 * Each term then takes one more row pass (the field is kept in space between
 * them).  TBS_ERR_UNSUPPORTED on periodic plans; tbs_adjoint and
 * tbs_batch_create refuse plans with a density contrast. */
int tbs_density_contrast(tbs_plan *plan, const double *gamma_dev);

/* ---- the paper's periodic scheme (periodic plans, padding 1) ----------- */

/* Tabulate the periodic spectrum g~(p) = 1 / (|p|^2 - k0^2 - i eps) (Sec. 2.2,
 * Eq. of g~; Algorithm 1's table), p = 2 pi m / (N dx) with m the signed
 * FFT index, in FP64, scaled 1/(N_x N_y), folded to [N_x/2+1][N_y/2+1] and
 * rounded to the plan dtype.  vv (NULL: none) adds the table g~ VV of the
 * Case II k-space potential, which tbs_iterate then applies in every
 * iteration after the first.  eps >= 0 (the paper: 0.8 k^2).
 * TBS_ERR_STATE on a padded plan.  Asynchronous on the plan's stream. */
int tbs_green_periodic(tbs_plan *plan, double eps, const tbs_kspace_potential *vv);

/* Coefficients of the Case II potential from the power law alpha0 omega^nu
 * (Sec. 2.1.2): tau = -2 alpha0 c^(nu-1), eta = 2 alpha0 c^nu tan(pi nu / 2);
 * out->nu = nu, out->omega = omega.  alpha0 in Np (rad/s)^-nu / m.  Host only.
 * (nu = 1 makes eta infinite: the paper requires nu != 1.) */
int tbs_kspace_coefficients(double alpha0, double nu, double c, double omega,
                            tbs_kspace_potential *out);

/* The paper's sigmoid absorbing layer along one axis (Sec. 3.1 Eq.
 * ABL_profile): out[i] = 1 / (1 + exp(-zeta (x_i - mu/2))) for cells whose
 * distance x_i = min(i, n-1-i) dx (in cm) from the nearer outer edge is below
 * the layer width mu = mu_cells dx, else 1.  zeta in Np/cm.  Host only;
 * out: host double [n].  The 2D layer is the product of the axis profiles. */
int tbs_abl_profile(int64_t n, double dx, double zeta, double mu_cells, double *out);

/* The paper's fixed-point iteration (Algorithm 1; Sec. 2.3 Eqs.
 * TBS_solution_lossless, _absorbing-dispersive, _inhomogeneous):
 *   psi_0 = G s,  psi_{l+1} = A (G(V psi_l) + psi_0) = A G(V psi_l + s),
 * G = F^-1 g~ F (g~ VV with a Case II table), A = mask_y[y] mask_x[x] the
 * absorbing layer (not applied to psi_0), stopping at the first l whose
 * error sum_x |psi_l - psi_{l-1}| / sum_x |psi_{l-1}| on row check_row
 * (Sec. 3.1 Eq. Error; the largest over right-hand sides) is below tol.
 *   source   : dev [B][N_y][N_x] plan dtype
 *   potential: dev [N_y][N_x] plan dtype, or NULL (V = 1: Case II, where the
 *              potential is in the spectrum)
 *   mask_x, mask_y: dev float64 [N_x], [N_y] or NULL (no layer on that axis)
 *   check_row: 0 <= check_row < N_y (the paper: the array's centre row)
 *   tol >= 0 (the paper: 1e-5); 1 <= max_iter <= 1e6 (the paper: 2000)
 *   psi_out  : dev [B][N_y][N_x] plan dtype, the last iterate (must not alias
 *              source)
 *   iters_out: host int or NULL: the iteration count l
 *   err_out  : host double [max_iter] or NULL: errors of iterations 1..l
 *   flags    : TBS_ITER_PAPER, or TBS_ITER_CBS for the convergent Born
 *              series (Osnabrugge et al., cited by the paper as its extension
 *              to strong scatterers): gamma = i V / eps (eps of
 *              tbs_green_periodic), psi_1 = gamma G s,
 *              psi_{l+1} = A (psi_l + gamma (G(V psi_l + s) - psi_l)),
 *              convergent for eps >= max |k^2 - k0^2|; needs the potential
 *              (V = k^2 - k0^2 - i eps) and no Case II table.
 * Synchronises once per 8 iterations.  Returns TBS_OK when the tolerance is
 * reached, TBS_WARN_NOT_CONVERGED (outputs valid) when max_iter is,
 * TBS_WARN_NONFINITE on a NaN/Inf error.  TBS_ERR_STATE before
 * tbs_green_periodic or on a padded plan. */
int tbs_iterate(tbs_plan *plan, const void *source, const void *potential, const double *mask_x,
                const double *mask_y, int check_row, double tol, int max_iter, void *psi_out,
                int *iters_out, double *err_out, int flags);

/* Gradient of Re<q, p_L> with respect to V for each right-hand side, i.e. the
 * adjoint of the truncated series:
 *   g_V = sum_{m=0}^{L-2} conj(w_m) * P_{L-1-m},  w_0 = G^H q,
 *   w_m = G^H (conj(V) w_{m-1}),  P_K = sum_{j<K} u_j;  G^H has spectrum conj(G^).
 *   source, potential, nterms: as tbs_solve (potential must not be NULL)
 *   adj_source : dev [B][P] plan dtype, q (e.g. R^H (R p - p_obs))
 *   grad_out   : dev [B][P] plan dtype, g_V per right-hand side
 *   residual_out: host double [B][L] or NULL: the forward residuals
 *   flags      : TBS_ADJ_STORE or TBS_ADJ_RECOMPUTE; TBS_ADJ_SERIES_ONLY
 *                writes the adjoint field instead, A_L^H q =
 *                sum_{m<L} (G^H conj(V))^m G^H q (the adjoint of p = A_L s;
 *                source may be NULL, potential may be NULL = V 0, and
 *                residual_out receives that series' residuals)
 * The forward partial sums are recomputed inside the call. */
int tbs_adjoint(tbs_plan *plan, const void *source, const void *potential, int nterms,
                const void *adj_source, void *grad_out, double *residual_out, int flags);

/* Receiver misfit.  rec_dev: dev int64 [nrec] flat spatial indices (indices
 * outside [0, P) are ignored); p_obs_dev: dev [B][nrec] plan dtype.  Writes
 * q_dev (dev [B][P]: q = R^H r, i.e. zero except q[b][rec[r]] summing
 * p[b][rec[r]] - p_obs[b][r] over receivers r on that cell; the summation
 * order of three or more receivers sharing a cell is not fixed) and J_dev
 * (dev double [1], J = 1/2 sum |p[b][rec[r]] - p_obs[b][r]|^2). */
int tbs_misfit(tbs_plan *plan, const void *p_dev, const int64_t *rec_dev, int nrec,
               const void *p_obs_dev, void *q_dev, double *J_dev);

/* grad_c_dev (dev double [P]) = (accumulate ? grad_c_dev : 0)
 *   + Re( sum_b g_V[b] * dV/dc ),  g_dev: dev [B][P], dVdc_dev: dev [P]. */
int tbs_speed_gradient(tbs_plan *plan, const void *g_dev, const void *dVdc_dev,
                       double *grad_c_dev, int accumulate);

/* ---- batches of plans (many grids, one graph launch) -------------------- */

typedef struct tbs_batch tbs_batch;

/* Group plans (e.g. one per frequency of a broadband pulse, each with its own
 * grid, k0 and B right-hand sides) for joint solves.  All plans must be 2D,
 * share the dtype and be tabulated; the batch queues its work on the first
 * plan's stream.  The plans must outlive the batch.  Schedule: each plan's
 * right-hand sides are cut into tiles of at most TBS_BATCH_TILE_RHS (default
 * 2), and consecutive tiles (in plan order) are packed into sets whose working
 * set (intermediate, sum, compensation, potential and spectrum of one term)
 * stays within TBS_BATCH_CACHE_MB megabytes (default 280, sized for the
 * 256 MB last-level cache: the estimate counts the potential and spectrum of
 * a plan once per tile although its tiles in a set share them; 0 runs all
 * plans as one set of whole plans).  The
 * sets run one after the other, each its whole series, so that a set's data
 * stays cache-resident between passes.  The tiles of a set go in turn to
 * TBS_BATCH_CHAINS launch chains (1 .. 4, default 3) on their own streams
 * (forked at the start of the set, joined at its end; with one set of whole
 * plans, the plans split into parts of equal work), so that one chain's
 * launches fill the compute units the others' leave idle at their ends.
 * Within a set and chain, passes of tiles whose padded lengths coincide run in
 * one grouped kernel launch per term.  TBS_BATCH_SHAPE="nr,nc" sets
 * the rows and columns per block of the member plans whose shapes no tuner has
 * chosen, where their lengths have those shapes.  Fields are bitwise the
 * same for every schedule and block shape; the residual norms are FP64 sums
 * of per-block partials, whose order follows the rows per row-pass block. */
int tbs_batch_create(tbs_batch **out, tbs_plan *const *plans, int nplans);

/* The L-term series of every plan in the batch (the tbs_solve contract per
 * plan): sources[i], potentials[i] (non-NULL) and p_outs[i] are dev pointers
 * for plan i.  The first call for a set of pointers and L records the whole
 * sequence as a HIP graph; later calls with the same pointers replay it.
 * residual_out: host double [sum_i B_i][L] (plan order) or NULL. */
int tbs_batch_solve(tbs_batch *batch, const void *const *sources, const void *const *potentials,
                    int nterms, void *const *p_outs, double *residual_out);

/* Choose the block shapes of the batch's grouped launches (rows per row-pass
 * block for all plans of one x length, columns per convolution block for all
 * plans of one y length) by timing each bitwise-neutral candidate as the
 * grouped launches the solves make for it (one per set of tiles, a middle
 * term) on the given buffers (same meaning as in tbs_batch_solve; the
 * contents of p_outs are undefined afterwards); then, with the cache-sized
 * schedule and unless TBS_BATCH_CHAINS is set, the number of launch chains
 * (1 .. 4) by timing a 4-term series replay per count; and regroup.  Choices are
 * kept per device model, dtype, length, member shapes and tiling for the life
 * of the process, and in the file named by the environment variable
 * TBS_TUNE_CACHE when it is set (read on first use, appended to;
 * tbs_plan_autotune shares it).  Synchronises the first plan's stream; drops
 * the recorded graph. */
int tbs_batch_autotune(tbs_batch *batch, const void *const *sources, const void *const *potentials,
                       void *const *p_outs);

/* Release the batch (not its plans; NULL-safe). */
void tbs_batch_destroy(tbs_batch *batch);

/* Message of the batch's last failure (NULL-safe). */
const char *tbs_batch_last_error(const tbs_batch *batch);

/* Per-launch device timing of batched solves (measurement only).  While
 * enabled, tbs_batch_solve does not replay its graph: it launches the same
 * grouped kernels directly on the batch stream, the two halves of the work one
 * after the other, and brackets every launch with two HIP events (results are
 * bitwise those of the graph).  Enabling (again) or disabling resets the
 * counters.  Synchronises the batch stream. */
int tbs_batch_profile_enable(tbs_batch *batch, int enable);

/* Synchronise the batch stream and return the timing since the last read, per
 * entry e < *nentries: one entry per grouped launch kind, i.e. three per row
 * group (kind[e] = 0 first row pass, 1 middle row passes, 2 last row pass) and
 * one per column group (kind[e] = 3 column convolution).  A group is one set
 * of tiles (see tbs_batch_create) and one padded length and block shape.
 * length[e]: the FFT length of the group's lines; shape[e]: lines per block
 * (rows per row-pass block, columns per column-pass block); launches[e]:
 * launches timed; ms[e]: summed event time in ms; the group's tiles are
 * members[first[e] .. first[e+1]) (the index of the tile's plan in the
 * tbs_batch_create array) with member_rhs[...] right-hand sides each
 * (member_rhs may be NULL).  cap: capacity of kind, length, shape, launches
 * and ms (first needs cap + 1; members and member_rhs the total count, at most
 * 4 x the batch's total right-hand sides); *nentries is set even when cap is
 * too small (TBS_ERR_INVALID then, nothing else written).  Resets the
 * counters. */
int tbs_batch_profile_read(tbs_batch *batch, int cap, int *nentries, int *kind, int *length, int *shape,
                           int64_t *launches, double *ms, int *first, int *members, int *member_rhs);

/* Per-pass device timing.  While enabled, every pass launch is bracketed by
 * two HIP events recorded on the plan's stream.  Pass kinds (index into the
 * output arrays): 0 first row pass (source in), 1 middle row passes,
 * 2 last row pass, 3 column convolution passes, 4 column forward-only passes
 * (3D y), 5 column inverse-only passes (3D y).  Enabling (again) resets the
 * counters. */
int tbs_profile_enable(tbs_plan *plan, int enable);

/* Synchronise the plan's stream and return, per pass kind, the summed event
 * time in ms (ms_out[6]) and the number of launches (count_out[6]); resets
 * the counters. */
int tbs_profile_read(tbs_plan *plan, double *ms_out, int64_t *count_out);

/* Release the plan and all device memory it owns (NULL-safe).  Synchronises
 * the plan's stream first. */
void tbs_plan_destroy(tbs_plan *plan);

/* Message of the last failure on this plan (NULL-safe; static string for
 * NULL plans: the last tbs_plan_create failure of this thread). */
const char *tbs_last_error(const tbs_plan *plan);

#ifdef __cplusplus
}
#endif

#endif /* TBS_H */
