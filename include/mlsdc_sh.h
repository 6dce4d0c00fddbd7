/*
 * mlsdc_sh.h -- C ABI of the MI355X (gfx950) MLSDC-SH hot path.
 *
 * Method: Hamon, Schreiber & Minion, "Multi-Level Spectral Deferred
 * Corrections Scheme for the Shallow Water Equations on the Rotating Sphere"
 * (arXiv:1805.07923).  Each entry point names the passage it implements.
 *
 * Conventions shared by every call
 *   - Truncation T_N (triangular, Sec. 3: S(r) = R, here N), zonal order m,
 *     degree n.  Spectral arrays hold m = 0..N, n = m..N, m-major:
 *     flat index idx(m, n) = m (2N + 3 - m) / 2 + (n - m), count shx_nspec(N)
 *     = (N+1)(N+2)/2.  Entries are complex FP64, interleaved (re, im), so a
 *     spectral field is `double[2 * nspec]` (a torch complex128 view).
 *     Real fields: m < 0 is implied by xi^{-m} = conj(xi^m); Im xi^0_n = 0.
 *   - Normalised associated Legendre functions: int_{-1}^{1} (P^m_n)^2 = 1,
 *     no Condon-Shortley phase (the normalisation for which the synthesis of
 *     eq. spectral_to_physical_space and the analysis of eqs.
 *     fourier_transform / legendre_transform are inverse to each other).
 *   - Grid arrays: real FP64 [field][nlat][nlon], latitude j = 0 northmost
 *     (Gaussian latitudes, roots of P_nlat), longitude lambda_i = 2 pi i / nlon.
 *   - State arrays: [3][nspec] complex in the order (Phi', zeta, delta) of
 *     Sec. 2 (U = [Phi, zeta, delta]).  Batches of states are contiguous.
 *   - Device arrays and workspaces must be 16-byte aligned (SHX_EINVAL
 *     otherwise); workspace sizes come from the *_workspace_bytes queries.
 *   - Every pointer argument named *_dev / device is device memory owned by
 *     the caller (e.g. allocated by PyTorch); the library never frees it.
 *     Plans and levels are owned by the library (create/destroy).
 *   - All compute calls only enqueue work on `stream` (hipStream_t, 0 = the
 *     null stream) and return without synchronising; argument errors are
 *     returned synchronously and nothing is enqueued then.  Calls that share
 *     a workspace must be ordered on one stream.
 *   - Return value: SHX_OK (0) or a negative shx_status.  No C++ exception
 *     crosses the ABI.
 */
#ifndef MLSDC_SH_H
#define MLSDC_SH_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct shx_plan shx_plan;   /* opaque; immutable after creation      */
typedef struct sdc_level sdc_level; /* opaque; a plan plus an SDC node set   */
typedef void* shx_stream_t;         /* a hipStream_t                          */

enum shx_status {
    SHX_OK = 0,
    SHX_EINVAL = -1,       /* null pointer, negative count, bad enum value   */
    SHX_ESHAPE = -2,       /* grid too small for the truncation (see below)  */
    SHX_EUNSUPPORTED = -3, /* nlon not of the form 2^k or 3*2^k, or a
                              precision / node kind not built               */
    SHX_EWORKSPACE = -4,   /* workspace pointer null or smaller than needed  */
    SHX_EHIP = -5          /* a HIP runtime call or launch failed            */
};

/* Precision of the Legendre contractions (everything else is FP64). */
enum shx_precision {
    SHX_FP64 = 0,
    SHX_FP32 = 1,          /* FP32 tables and FP32 accumulation               */
    SHX_SPLIT_BF16_2 = 2,  /* bf16 hi+lo splits, 3 products, FP32 accumulation */
    SHX_SPLIT_BF16_3 = 3   /* bf16 three-way splits, 6 products, FP32 accum.  */
};

/* Where the normalised P^m_n(mu_j) of the contractions (Sec. 3, the P of eq.
 * spectral_to_physical_space and eq. legendre_transform) come from. */
enum shx_table_mode {
    SHX_TABLE_HBM = 0,      /* tabulated once per plan and held in device memory
                               (FP64, or rounded / split to the working
                               precision): 2 x 8 B per (m, n, j) in FP64,
                               4 B in FP32 (1.6 GB at T1023 on 1536 latitudes) */
    SHX_TABLE_ONTHEFLY = 1  /* no table: every contraction regenerates P^m_n
                               per order m by the FP64 three-term recurrence
                               from exact restart values (at most 64 degrees
                               apart; 126 MB at T1023) and, for a reduced
                               working precision, rounds or splits it in
                               registers right before the product */
};

enum sdc_node_kind {
    SDC_GAUSS_LOBATTO = 0, /* Sec. 4.2: Gauss-Lobatto nodes on [t^n, t^n + dt] */
    SDC_RADAU_RIGHT = 1    /* t^n followed by the Radau-IIA points            */
};

/* Physical constants of Sec. 2: Earth radius a, rotation rate Omega,
 * gravity g, mean geopotential Phibar, diffusion coefficient nu. */
typedef struct { double a, omega, g, phibar, nu; } swe_params;

/* Algorithm 1 controls: iterations N_ML, sweeps per call of SweepFine /
 * SweepCoarse (the paper uses 1 and 1), and whether to compute the FP64
 * collocation residual of the final fine nodes (eq. collocation_problem). */
typedef struct { int niter, nsweep_fine, nsweep_coarse, residual_check; } mlsdc_opts;

/* ---------------------------------------------------------------- plans */

/* Number of spectral coefficients (N+1)(N+2)/2 of truncation T_N. */
size_t shx_nspec(int ntrunc);

/* Create a transform plan for T_ntrunc on nlat Gaussian latitudes and nlon
 * longitudes (Sec. 3, eqs. spectral_to_physical_space, fourier_transform,
 * legendre_transform).  Requires ntrunc >= 1, nlat even, nlon > 2 ntrunc,
 * nlat > ntrunc (else SHX_ESHAPE), nlon = 2^k or 3*2^k with
 * 16 <= nlon <= 3072 and a known precision (else SHX_EUNSUPPORTED), and
 * table_mode SHX_TABLE_HBM or SHX_TABLE_ONTHEFLY (else SHX_EINVAL).
 * Computes the Gaussian latitudes and weights on the host in quad precision,
 * the FFT twiddles in extended precision, and on the current device, with a
 * double-double recurrence built from FP64 operations, the exact restart
 * values and recurrence coefficients from which the Legendre kernels
 * regenerate P^m_n (n <= ntrunc + 1; at most 64 degrees of plain FP64
 * recurrence per restart) and, with SHX_TABLE_HBM only, the P^m_n tables
 * stored in `precision`.  Synchronises the current device.  *out receives
 * the plan (library-owned). */
int shx_plan_create(int ntrunc, int nlat, int nlon, int precision, int table_mode, shx_plan** out);
void shx_plan_destroy(shx_plan* plan);

/* Host copies of the plan's FP64 latitude data, each array [nlat]:
 * mu_j = cos(theta_j), sin(theta_j), Gauss weights w_j.  Any may be NULL. */
int shx_plan_latitudes(const shx_plan* plan, double* mu, double* sin_theta, double* w);

/* Copy P^m_n(mu_j) (FP64 table values, or the working-precision table
 * values widened to FP64) for the northern latitudes j = 0..nlat/2-1 to the
 * host array out[nlat/2].  Requires 0 <= m <= n <= ntrunc + 1, m <= ntrunc.
 * Plans without tables compute the row by the double-double recurrence (and
 * round or split it as their contractions do).  Synchronous. */
int shx_plan_legendre(const shx_plan* plan, int m, int n, double* out);

/* Number of table products P^m_n(mu_j) x (north +/- south Fourier data)
 * that the Legendre analysis (eq. legendre_transform; sh_forward,
 * sh_legendre_analysis, swe_tendency) forms per field for degrees
 * n <= nmax (nmax = ntrunc or ntrunc + 1, else SHX_EINVAL), counted per
 * latitude pair.  Plans that generate P^m_n sum every latitude pair: the
 * count is sum over (m, n) of nlat/2.  FP64 plans with tables on at most
 * 512 latitudes and FP32 plans with tables on at most 2040 latitudes apply
 * the polar truncation of the transform library the method builds on
 * (Sec. 3, Schaeffer 2013) to every field.  Per order m, parity of n - m and
 * tile of 16 such degrees, the latitude pairs are taken in groups of 4 from
 * the pole (ngrp = ceil(nlat/8) groups); c0 is the first group holding a
 * |P^m_n| >= 1e-20 for a degree of the tile (ngrp if none); the sum runs
 * over the groups from max(0, ngrp - B ceil((ngrp - c0) / B)) on, B = 8
 * from 320 latitudes up and 4 below (whole batches of table loads).  A
 * coefficient then changes by at most 1e-20 times the sum of
 * |w_j xi_m(mu_j)| over the omitted latitudes.  *terms receives the count;
 * *fourier_pairs (if not NULL) the number of (m, latitude pair) whose
 * Fourier data the analysis reads.  Synchronous. */
int shx_plan_analysis_terms(const shx_plan* plan, int nmax, long long* terms, long long* fourier_pairs);

/* ------------------------------------------------------- the SH pair */

/* Device workspace bytes for sh_inverse / sh_forward with nfield fields. */
size_t shx_workspace_bytes(const shx_plan* plan, int nfield);

/* Synthesis, eq. spectral_to_physical_space (Sec. 3):
 *   grid(lambda_i, mu_j) = Re xi_0(mu_j) + 2 Re sum_{m=1}^{N} xi_m(mu_j) e^{i m lambda_i},
 *   xi_m(mu_j) = sum_{n=m}^{N} xi^m_n P^m_n(mu_j).
 * spec_dev: [nfield][nspec] complex (read only); grid_dev: [nfield][nlat][nlon]
 * real (written).  Im xi^0_n is ignored. */
int sh_inverse(const shx_plan* plan, int nfield, const double* spec_dev, double* grid_dev,
               void* ws_dev, size_t ws_bytes, shx_stream_t stream);

/* Analysis, eqs. fourier_transform and legendre_transform (Sec. 3):
 *   xi_m(mu_j) = (1/nlon) sum_i grid(lambda_i, mu_j) e^{-i m lambda_i},
 *   xi^m_n = sum_j w_j xi_m(mu_j) P^m_n(mu_j).
 * grid_dev: [nfield][nlat][nlon] real (read only); spec_dev: [nfield][nspec]. */
int sh_forward(const shx_plan* plan, int nfield, const double* grid_dev, double* spec_dev,
               void* ws_dev, size_t ws_bytes, shx_stream_t stream);

/* The Legendre step alone, on the library's Fourier-space layouts (used by
 * swe_tendency; exposed for callers that do their own longitude transform and
 * for timing).  nmax = ntrunc or ntrunc + 1 is the highest degree.
 *   The spectral side is field-interleaved in the extended layout: [nspec_ext][nfield] complex with
 *     nspec_ext = (N+1)(N+4)/2, m-major, n = m..N+1 (entries n > nmax ignored
 *     on input, not written on output).
 *   Synthesis (eq. spectral_to_physical_space, the sum over n):
 *     fourier_out [2][nlat/2][N+1][nfield] complex: even (p = 0) and odd
 *     (p = 1) degree sums E, O at the northern latitudes; xi_m(mu_j) = E + O
 *     in the north and E - O at the mirrored southern latitude.
 *   Analysis (eq. legendre_transform): fourier_in [nlat][N+1][nfield] complex
 *     holding w_j xi_m(mu_j) (weights already applied), all latitudes.
 * Arrays are device memory, 16-byte aligned; nothing else is needed. */
int sh_legendre_synthesis(const shx_plan* plan, int nfield, int nmax, const double* spec_ext_dev,
                          double* fourier_out_dev, shx_stream_t stream);
int sh_legendre_analysis(const shx_plan* plan, int nfield, int nmax, const double* fourier_in_dev,
                         double* spec_ext_dev, shx_stream_t stream);

/* ------------------------------------------------ SWE right-hand sides */

/* Device workspace bytes for swe_tendency on nstate states. */
size_t swe_workspace_bytes(const shx_plan* plan, int nstate);

/* The split right-hand side of eq. system_of_odes (Sec. 4.1):
 * F_I = L_G (eq. linear_wave_motion_induced_by_gravitational_forces) and
 * F_E = L_F + N (eqs. linear_harmonic_oscillator_on_the_velocity_components,
 * nonlinear_operators) of the vorticity-divergence equations of Sec. 2, in
 * spectral space (eq. semidiscrete_system).  With L_n = n(n+1)/a^2:
 *   F_I = [-Phibar delta - nu L Phi', -nu L zeta, L Phi' - nu L delta],
 *   F_E = [-div(Phi' V), -div(eta V), curl(eta V) + L_n (V.V/2)^],
 * eta = zeta + 2 Omega mu; the products are formed on the Gaussian grid
 * (the grid must be alias free: nlon >= 3N+1, nlat >= (3N+1)/2, else
 * SHX_ESHAPE).  state_dev: [nstate][3][nspec] complex (read only);
 * f_impl_dev, f_expl_dev: same shape (written; may be NULL to skip). */
int swe_tendency(const shx_plan* plan, const swe_params* params, int nstate,
                 const double* state_dev, double* f_impl_dev, double* f_expl_dev,
                 void* ws_dev, size_t ws_bytes, shx_stream_t stream);

/* Solve Theta - h F_I(Theta) = b (Sec. 4.4, eq. implicit_systems) for each
 * (m, n): the geopotential from the diagonal reduced system, then delta and
 * zeta by local updates.  h = dt * qI_{m+1,m+1}.  rhs_dev, out_dev:
 * [nstate][3][nspec] complex; out may alias rhs. */
int imex_solve(const shx_plan* plan, const swe_params* params, int nstate, double h,
               const double* rhs_dev, double* out_dev, shx_stream_t stream);

/* ------------------------------------------------------ SDC and MLSDC */

/* An SDC level: the plan, the SWE constants and nnodes = M+1 nodes of
 * node_kind with the matrices of Sec. 4.2 (computed on the host in quad
 * precision, used in FP64): Q (eq. weights), forward-Euler Q_E, and the
 * LU-trick Q_Delta (Q_Delta[1:,1:] = U^T where Q[1:,1:]^T = L U, Doolittle).
 * 2 <= nnodes <= 9.  The plan must outlive the level. */
int sdc_level_create(const shx_plan* plan, const swe_params* params, int node_kind,
                     int nnodes, sdc_level** out);
void sdc_level_destroy(sdc_level* level);

/* Host copies of the level's nodes tau[M+1] on [0,1] and the row-major
 * (M+1)x(M+1) matrices Q, Q_E, Q_Delta.  Any may be NULL. */
int sdc_level_matrices(const sdc_level* level, double* tau, double* Q, double* QE, double* QD);

size_t sdc_sweep_workspace_bytes(const sdc_level* level);

/* One IMEX SDC sweep (Sec. 4.2, eq. update_equation_sdcq_discrete_form; with
 * tau, Sec. 4.3.1, eq. modified_update_equation_sdcq_discrete_form), nodes
 * m = 0..M-1 in order, in place.  theta_dev, f_impl_dev, f_expl_dev:
 * [M+1][3][nspec] complex; node 0 is the initial value (read only), F at all
 * nodes must be those of the current iterate.  tau_dev: [M+1][3][nspec] or
 * NULL. */
int sdc_sweep(const sdc_level* level, double dt, double* theta_dev, double* f_impl_dev,
              double* f_expl_dev, const double* tau_dev, void* ws_dev, size_t ws_bytes,
              shx_stream_t stream);

size_t mlsdc_workspace_bytes(const sdc_level* fine, const sdc_level* coarse, const mlsdc_opts* opts);

/* One time step of two-level MLSDC (Sec. 4.3.2, Algorithm 1; spread
 * initialisation; transfer by spectral truncation / zero padding and
 * Lagrange time interpolation, Sec. 4.3.3), or of single-level SDC when
 * coarse is NULL (step A only, niter sweeps of nsweep_fine).  The coarse plan
 * must not have a larger truncation than the fine plan, nor the coarse level
 * more nodes (equal truncations coarsen in time only, equal node counts in
 * space only).  theta_n_dev,
 * theta_np1_dev: [3][nspec_fine] complex (may alias).  status_dev: NULL or
 * device double[2]: [0] = FP64 collocation residual of the fine nodes
 * max_m ||r^m||_2 / ||Theta^0||_2 if opts->residual_check, else 0;
 * [1] = 1 if the new state holds a non-finite value, else 0. */
int mlsdc_step(const sdc_level* fine, const sdc_level* coarse, const mlsdc_opts* opts,
               double dt, const double* theta_n_dev, double* theta_np1_dev,
               double* status_dev, void* ws_dev, size_t ws_bytes, shx_stream_t stream);

/* mlsdc_step without a caller-supplied workspace and without any device
 * allocation, for callers that cannot allocate device memory: code recorded
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The workspace is a library-owned array of
 * SHX_NOALLOC_SCRATCH_BYTES on each device (a static device variable, held
 * from the first use of the library on that device until the process ends;
 * its address is looked up at sdc_level_create, or at the first call).
 * Arguments and results as for mlsdc_step; the caller still owns theta_n,
 * theta_np1 and status.  The limit covers the T255/T127 Gauss-Lobatto 5/3
 * step (about 75 MB) without the residual check; larger configurations
 * return SHX_EWORKSPACE (nothing is enqueued).  Every call on one device
 * shares that device's array and leaves its contents behind: calls that
 * overlap on one device (other streams, other threads) race and must be
 * serialised by the caller.  The step needs no zeroed workspace. */
#define SHX_NOALLOC_SCRATCH_BYTES (96u * 1024u * 1024u)
int mlsdc_step_noalloc(const sdc_level* fine, const sdc_level* coarse, const mlsdc_opts* opts, double dt,
                       const double* theta_n_dev, double* theta_np1_dev, double* status_dev,
                       shx_stream_t stream);

/* Multi-level MLSDC: the V-cycle of which Algorithm 1 is the two-level case
 * (Sec. 4.3; more than two levels are the paper's future work), over
 * levels[0] (finest) .. levels[nlevels-1], 1 <= nlevels <= SHX_MAX_LEVELS.
 * Per iteration: nsweep[0] sweeps on the finest level; going down, level l
 * takes the restriction of level l-1 at its nodes 1..M, evaluates it, forms
 * its FAS term tau_l = A_l(R Theta_{l-1}) - R A_{l-1}(Theta_{l-1}) + R tau_{l-1}
 * (eq. tau_term_level_l+1) and runs nsweep[l] sweeps; going up, the
 * corrections of Theta, F_I and F_E of level l are interpolated into level
 * l-1.  Node 0 of every coarser level is the restricted initial value,
 * evaluated once per step.  Levels: one node kind, non-increasing
 * truncations and node counts, alias-free grids.  With two levels
 * this launches what mlsdc_step launches (no residual check).
 * theta_n_dev, theta_np1_dev: [3][nspec] of levels[0]'s plan (may alias);
 * ws: device workspace of mlsdc_multi_workspace_bytes bytes (16-byte
 * aligned).  Errors: SHX_EINVAL (arguments, level order), SHX_ESHAPE (grid
 * not alias free), SHX_EWORKSPACE.  Asynchronous on `stream`. */
#define SHX_MAX_LEVELS 4
size_t mlsdc_multi_workspace_bytes(const sdc_level* const* levels, int nlevels);
int mlsdc_step_multi(const sdc_level* const* levels, int nlevels, int niter, const int* nsweep,
                     double dt, const double* theta_n_dev, double* theta_np1_dev, void* ws_dev,
                     size_t ws_bytes, shx_stream_t stream);

/* -------------------------------------------------------------- adjoints
 * Transposes of the Jacobians above (reverse mode), FP64.  Inner products:
 * spectral arrays <x, y> = sum over the stored coefficients of
 * Re x Re y + Im x Im y; grids sum_ij x_ij y_ij.  So a cotangent returned for
 * a spectral input is the gradient with respect to its real and imaginary
 * parts.  Plans of a reduced working precision are not supported here
 * (SHX_EUNSUPPORTED). */

/* spec_cot = S^T grid_cot for the synthesis S of sh_inverse:
 *   spec_cot^m_n = c_m sum_j P^m_n(mu_j) sum_i grid_cot_ij e^{-i m lambda_i}, c_0 = 1, c_m = 2.
 * Workspace: shx_workspace_bytes(plan, nfield). */
int sh_inverse_adj(const shx_plan* plan, int nfield, const double* grid_cot_dev, double* spec_cot_dev,
                   void* ws_dev, size_t ws_bytes, shx_stream_t stream);

/* grid_cot = A^T spec_cot for the analysis A of sh_forward:
 *   grid_cot_ij = (w_j / nlon) sum_{m >= 0} Re[(sum_n spec_cot^m_n P^m_n(mu_j)) e^{i m lambda_i}]. */
int sh_forward_adj(const shx_plan* plan, int nfield, const double* spec_cot_dev, double* grid_cot_dev,
                   void* ws_dev, size_t ws_bytes, shx_stream_t stream);

/* Workspace of swe_tendency_adj for nstate states.  For nlon = 2048 and 3072
 * it includes 9 nlat nlon doubles per state: those rows are too long for the
 * transposed grid products to stay in LDS, so they go through HBM. */
size_t swe_adj_workspace_bytes(const shx_plan* plan, int nstate);

/* lam_state += (dF_I/dTheta)^T lam_fi + (dF_E/dTheta)^T lam_fe, linearised at
 * state (the products of F_E are linearised on the grid; the transforms are
 * transposed as above).  lam_fi or lam_fe may be NULL.  All [nstate][3][nspec]. */
int swe_tendency_adj(const shx_plan* plan, const swe_params* params, int nstate, const double* state_dev,
                     const double* lam_fi_dev, const double* lam_fe_dev, double* lam_state_dev, void* ws_dev,
                     size_t ws_bytes, shx_stream_t stream);

/* lam_rhs = (I - h F_I)^{-T} lam_out (transpose of imex_solve). */
int imex_solve_adj(const shx_plan* plan, const swe_params* params, int nstate, double h,
                   const double* lam_out_dev, double* lam_rhs_dev, shx_stream_t stream);

size_t mlsdc_adj_workspace_bytes(const sdc_level* fine, const sdc_level* coarse, const mlsdc_opts* opts);

/* lam_n = (d Theta^{n+1} / d Theta^n)^T lam_np1 for one mlsdc_step from the
 * checkpoint theta_n: the step is recomputed, recording every state at which
 * F is evaluated, then Algorithm 1 is run backwards (step D, coarse sweeps,
 * FAS term, restriction, fine sweeps, spread) with the transposed node
 * updates, solves, transfers and tendencies.  residual_check is ignored.
 * lam_n must not alias theta_n or lam_np1. */
int mlsdc_step_adj(const sdc_level* fine, const sdc_level* coarse, const mlsdc_opts* opts, double dt,
                   const double* theta_n_dev, const double* lam_np1_dev, double* lam_n_dev, void* ws_dev,
                   size_t ws_bytes, shx_stream_t stream);

/* ------------------------------------------------------------ profiling */

/* Kernel classes for the timer below. */
enum shx_kernel_class {
    SHX_KC_LEGENDRE_SYN = 0, /* Legendre synthesis (swe_tendency, sh_inverse)   */
    SHX_KC_LEGENDRE_AN = 1,  /* Legendre analysis (swe_tendency, sh_forward)    */
    SHX_KC_GRID = 2,         /* FFTs + grid products inside swe_tendency        */
    SHX_KC_SDC_NODE = 3      /* node update (quadrature + implicit solve)       */
};

/* Start timing kernel class kclass: the next `capacity` launches of that
 * class (by any call, on its stream) are bracketed by HIP events recorded on
 * the launch stream.  Process-global and not thread safe; a new start
 * discards an unfinished timing.  Host-only bookkeeping plus event creation. */
int shx_kernel_timer_start(int kclass, int capacity);

/* Stop timing: waits for the recorded events and writes the duration of each
 * recorded launch in milliseconds to ms[0..count-1] (ms may be NULL to
 * discard); *count (may be NULL) receives the number recorded. */
int shx_kernel_timer_stop(float* ms, int* count);

/* Text for a status code. */
const char* shx_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif
