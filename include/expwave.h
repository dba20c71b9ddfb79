/*
 * expwave.h -- C ABI of the exponential wave-propagation library (gfx950).
 *
 * Method: Ravelo, Schreiber, Peixoto, "High-order exponential integration for
 * seismic wave modeling" (arXiv 2401.16322).
 *
 *   Sec. 3 (time integration methods): semi-discrete system U' = H U + f(t).
 *   Sec. 3.2, Faber approximation: u^{n+1} = sum_{j=0..m} a_j F_j(H~) [u^n; e_p],
 *       F_0 = I, F_1 = H/gamma - c0 I, F_2 = F_1^2 - 2 c1 I,
 *       F_j = F_1 F_{j-1} - c1 F_{j-2}.
 *   Sec. 3.2, Krylov subspace projection: Arnoldi (modified Gram-Schmidt)
 *       then the small Hessenberg exponential by Pade.
 *   Sec. 3.2, augmented matrix H~ = [[H, W], [0, J]]: the source and its
 *       first p-1 derivatives folded into one exponential.
 *   Sec. 3.1, low order methods: classical RK4 and leap-frog (baselines).
 *   Sec. 2: absorbing layer with the quadratic profile
 *       sigma(d) = sigma_max (1 - d/delta)^2, zero values outside the domain.
 *   Sec. 2.1: staggered first-derivative stencils (order 4 or the paper's 8).
 *
 * The operator is the first-order pressure/velocity system with a diagonal
 * damping layer and rho = 1:
 *     (H U)_p   = -c^2 sum_a D-_a v_a - (sum_a sigma_a(x_a)) p
 *     (H U)_v_a = -D+_a p - sigma_a(x_a + h/2) v_a
 * with p on nodes and v_a half a cell forward along axis a.
 *
 * Conventions
 * - State layout (canonical, unpadded, field-major): [p | v_0 | ... | v_{d-1}],
 *   each field n_0 * n_1 (* n_2) values with axis 0 (x) fastest. In 2D the
 *   axes are (x, z); in 3D (x, y, z). The velocity slots of the leap-frog
 *   state hold v at t - dt/2.
 * - Element type of every device array (state, c^2, traces) is the grid dtype.
 * - Ownership: the caller allocates and owns every device buffer (c^2, state,
 *   traces, receiver indices, workspace). The library never allocates device
 *   memory; destroy frees only the host-side handle.
 * - Streams: device work is enqueued on the handle's stream (a hipStream_t
 *   passed as void*; NULL is the legacy default stream) and is asynchronous,
 *   except where noted ("synchronizes").
 * - Errors: every entry point returns an expw_status. Arguments are validated
 *   before any launch; on a non-OK status nothing was enqueued and
 *   expw_last_error() returns a message (thread-local). Device launch
 *   failures return EXPW_EDEVICE.
 * - Host-math entry points (marked "host only") touch no GPU and may be
 *   called on a machine without one.
 */
#ifndef EXPWAVE_H
#define EXPWAVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct expw_op expw_op; /* opaque host-side handle */

typedef enum {
  EXPW_OK = 0,
  EXPW_EINVAL = -1,       /* invalid argument (message says which) */
  EXPW_ENOMEM = -2,       /* caller-supplied workspace too small */
  EXPW_EDEVICE = -3,      /* HIP runtime or launch failure */
  EXPW_ENONFINITE = -4,   /* NaN/Inf in c^2, or in a state (guard) */
  EXPW_EUNSUPPORTED = -5  /* valid but not supported combination */
} expw_status;

typedef enum { EXPW_F32 = 0, EXPW_F64 = 1 } expw_dtype;
typedef enum { EXPW_BC_ZERO = 0, EXPW_BC_PERIODIC = 1 } expw_bc;

enum {
  EXPW_MAX_KRYLOV = 64, /* largest Krylov dimension k */
  EXPW_MAX_TAYLOR = 16, /* largest source Taylor order p */
  EXPW_MAX_SOURCES = 64 /* largest number of point sources */
};

typedef struct {
  int32_t ndim;      /* 2 or 3 */
  int32_t order;     /* staggered stencil order: 4 or 8 */
  int64_t n[3];      /* (nx, nz, 1) in 2D, (nx, ny, nz) in 3D; each >= 1 */
  double h;          /* grid spacing (m), > 0 */
  int32_t dtype;     /* expw_dtype of every device array */
  int32_t bc;        /* expw_bc: zero ghost values (Sec. 2.1) or periodic */
  int32_t abc_cells; /* damping-layer thickness L in cells (delta = L h), >= 0 */
  int32_t reserved;  /* must be 0 */
  double sigma_max;  /* peak damping sigma_max (1/s), >= 0; must be 0 with periodic bc */
} expw_grid;

/* ------------------------------------------------------------------ host only */

/* Library ABI version (currently 1). */
int32_t expw_version(void);

/* Message of the last non-OK status returned on this thread ("" if none). */
const char* expw_last_error(void);

/* Bytes of device workspace expw_op_create needs for a grid, a largest Krylov
 * dimension max_krylov_k (0 = Krylov unused, <= EXPW_MAX_KRYLOV) and a largest
 * source Taylor order max_taylor_p (<= EXPW_MAX_TAYLOR). */
int32_t expw_workspace_size(const expw_grid* grid, int32_t max_krylov_k, int32_t max_taylor_p,
                            size_t* bytes);

/* Sec. 2, absorption profile: out[i] = sigma at x_i = i h (half = 0) or
 * (i + 1/2) h (half = 1); distance to the nearest outer node (0 or n-1),
 * clamped at 0; sigma_max (1 - d/delta)^2 for d < delta = cells h, else 0. */
int32_t expw_damping_profile(int64_t n, double h, int32_t cells, double sigma_max, int32_t half,
                             double* out);

/* Field-of-values rectangle [x_lo, 0] x i[-B, B] of H for a grid whose largest
 * c^2 is c2_max: B = sqrt(c2_max) sqrt(ndim) (2/h) sum |alpha_l|, x_lo = -max damping. */
int32_t expw_spectrum_rectangle(const expw_grid* grid, double c2_max, double* x_lo, double* B);

/* The rectangle for caller-given damping profiles (layout of
 * expw_op_create_profiles; NULL = the grid's quadratic layer): B as above,
 * x_lo = -max(sum_a max_i sigma_a(x_i), max_a max_i sigma_a(x_i + h/2)). */
int32_t expw_spectrum_rectangle_profiles(const expw_grid* grid, double c2_max,
                                         const double* const* sigma_host, double* x_lo,
                                         double* B);

/* Faber ellipse (gamma, c0, c1) of the minimum-area ellipse around the
 * rectangle (Sec. 3.2: the parameters of F_1 = H/gamma - c0 I). */
int32_t expw_ellipse(double x_lo, double B, double* gamma, double* c0, double* c1);

/* Faber coefficients a_0..a_m of exp(dt z) on that ellipse: the Laurent
 * coefficients of exp(dt gamma (w + c0 + c1/w)). a has m+1 entries. */
int32_t expw_faber_coefficients(double gamma, double c0, double c1, double dt, int32_t m, double* a);

/* The ellipse a Faber step on the PML operator with state dtype runs with
 * (see expw_pml_step_faber): 1/gamma, c0 and c1 rounded to that precision,
 * gamma = 1/(rounded 1/gamma); the identity for EXPW_F64. (Faber steps on the
 * pressure/velocity operator compute every term in FP64 for both dtypes and
 * run on the operator's ellipse as it is.) */
int32_t expw_step_ellipse(int32_t dtype, double gamma, double c0, double c1, double* gamma_step,
                          double* c0_step, double* c1_step);

/* Dense-output weights (Sec. 3.2, Faber approximation): the terms
 * v_j = F_j(H~) [u_n; e_p] of one step combine to the solution at any
 * t_n + tau, tau >= 0, with the Faber coefficients of exp(tau z) on the same
 * ellipse: coef[t * (m + 1) + j] = a_j(taus[t]) (a_j(0) = delta_j0). Pass the
 * step ellipse (expw_step_ellipse) to match a library step exactly. */
int32_t expw_faber_dense_coefficients(double gamma, double c0, double c1, int32_t m, int32_t n_tau,
                                      const double* taus, double* coef);

/* Ricker wavelet g(t) = (1 - 2 a tau^2) exp(-a tau^2), a = (pi f_peak)^2,
 * tau = t - t_delay, and its derivatives: out[k] = g^(k)(t), k = 0..p-1. */
int32_t expw_ricker_derivatives(double t, double f_peak, double t_delay, int32_t p, double* out);

/* Source scalars of one Faber step (Sec. 3.2, augmented matrix): with the tail
 * tau_0 = e_p run through the same three-term recurrence under J,
 * q[j-1] = (G . tau_{j-1}) / gamma for j = 1..m, where G[c] = g^(p-1-c)(t_n).
 * G has p entries; q has m entries. */
int32_t expw_faber_source_scalars(double gamma, double c0, double c1, int32_t m, int32_t p,
                                  const double* G, double* q);

/* Matrix exponential of a k x k row-major matrix (scaling and squaring with
 * the [13/13] Pade approximant; k <= EXPW_MAX_KRYLOV + 1). */
int32_t expw_expm(int32_t k, const double* A, double* E);

/* ------------------------------------------------------------------ device */

/* Create an operator from c^2 (device array, one field of the grid dtype) and
 * the damping layer in *grid: the semi-discrete operator H of U' = H U + f
 * (Sec. 3) on the staggered grid of Sec. 2.1, with the quadratic absorbing
 * profile of Sec. 2 (the paper's PML coupling terms dropped: damping on the
 * diagonal only) and zero values outside the grid. Synchronizes: computes max c^2 on the device
 * (EXPW_ENONFINITE on NaN/Inf or c^2 <= 0), then the spectrum rectangle and
 * the Faber ellipse on the host in FP64, and uploads the 1D damping profiles
 * into the workspace. c2_dev and workspace_dev must stay valid and unmodified
 * (except by the library) while the handle lives. */
int32_t expw_op_create(const expw_grid* grid, const void* c2_dev, int32_t max_krylov_k,
                       int32_t max_taylor_p, void* workspace_dev, size_t workspace_bytes,
                       void* hip_stream, expw_op** out);
/* As expw_op_create, with caller-given damping profiles (Sec. 2: the
 * absorbing term is a function of position on each axis; the reading here
 * keeps it separable and on the diagonal): sigma_host holds 2 * ndim host
 * pointers, entry 2a the values of axis a at the integer points x_i = i h and
 * entry 2a + 1 at the half points (i + 1/2) h, each n[a] finite values >= 0
 * (1/s), copied at this call. sigma_p = sum_a sigma_a(x_a) damps p and
 * axis a's half-point values damp v_a. grid->abc_cells and sigma_max are not
 * used for the profiles; sigma_host == NULL takes the quadratic layer of
 * expw_op_create. The spectrum rectangle's x_lo is minus the largest damping
 * these profiles give. Periodic ghosts require all-zero profiles
 * (EXPW_EINVAL otherwise). */
int32_t expw_op_create_profiles(const expw_grid* grid, const void* c2_dev,
                                const double* const* sigma_host, int32_t max_krylov_k,
                                int32_t max_taylor_p, void* workspace_dev, size_t workspace_bytes,
                                void* hip_stream, expw_op** out);
int32_t expw_op_destroy(expw_op* op);

/* Stream for subsequent launches (hipStream_t as void*). */
int32_t expw_set_stream(expw_op* op, void* hip_stream);

/* Host values of the spectrum rectangle and of the ellipse in use. */
int32_t expw_get_spectrum(const expw_op* op, double* x_lo, double* B);
int32_t expw_get_ellipse(const expw_op* op, double* gamma, double* c0, double* c1);
/* Override the ellipse (gamma > 0, |c1| <= 1; c1 = -1 is the segment of an
 * undamped operator); the next Faber step uses it. */
int32_t expw_set_ellipse(expw_op* op, double gamma, double c0, double c1);

/* Kernel tuning for the Faber step: fuse = recurrence terms per HBM sweep
 * (0 = automatic, 1 = one term per sweep, up to 8 accepted). 2D order 4:
 * up to 6 terms at FP32 and 4 at FP64, automatic = 6 at FP32 and 4 at FP64;
 * 2D order 8: up to 4 (3 in streamed FP64 passes), automatic = 4 in streamed
 * FP32 passes and 3 otherwise; 3D FP32 order 4: two terms unless fuse = 1;
 * 3D FP64: one term per sweep. Only zero ghosts fuse. Results do not depend
 * on it beyond rounding order. */
int32_t expw_set_tuning(expw_op* op, int32_t fuse);

/* Kernel of the fused Faber passes on 2D grids (order 4 or 8) with zero
 * ghosts:
 *   EXPW_PASS_AUTO (default): streamed when the grid gives the chip at least
 *     512 workgroups with row segments of 64 rows or more, else tiled;
 *   EXPW_PASS_TILED: each workgroup recomputes the halo of a 2D tile;
 *   EXPW_PASS_STREAMED: each workgroup walks a column band down the grid,
 *     every term two rows (order 8: four) behind the previous one (no
 *     recomputation in z); order 8 in FP64 takes at most three terms per
 *     pass.
 * Results agree to rounding (the same polynomial on the same ellipse). */
enum { EXPW_PASS_AUTO = 0, EXPW_PASS_TILED = 1, EXPW_PASS_STREAMED = 2 };
int32_t expw_set_pass_kernel(expw_op* op, int32_t kind);
/* Autotuner of the Faber step (Sec. 3.2, Faber recurrence; the pass design
 * is this library's): times expw_step_faber of degree m and step dt on
 * scratch_dev (a state vector of the op's dtype, overwritten) for every
 * terms-per-pass depth the layout admits (2D order 4 FP32: 1..6, FP64 and
 * order 8: 1..4, 3D FP32 order 4: 1..2, else 1) and, for 2D passes, both
 * pass kernels; keeps the fastest on the operator (as expw_set_tuning
 * and expw_set_pass_kernel would; batches created from the operator use
 * its depth) and returns it in fuse_out, pass_kernel_out and ms_out (one
 * step, ms; any may be NULL). cache_path (NULL = none): a text file with one
 * line per device (architecture, compute units), layout (ndim, sizes,
 * dtype, order, bc) and degree m; a line for this key applies its choice
 * without timing; otherwise the result is appended (the file is created if
 * missing; a file that cannot be opened is ignored). Synchronizes the op's
 * stream while timing. */
int32_t expw_autotune(expw_op* op, int32_t m, double dt, void* scratch_dev, const char* cache_path,
                      int32_t* fuse_out, int32_t* pass_kernel_out, double* ms_out);

/* y = H x (no source; Sec. 3, the semi-discrete operator with the staggered
 * differences of Sec. 2.1), x and y device state arrays in the state layout
 * (must not alias). */
int32_t expw_apply(expw_op* op, const void* x_dev, void* y_dev);

/* Point sources sharing one Ricker wavelet (f_peak, t_delay) entering the
 * pressure equation at flat node indices node_idx_host[s] (0 <= idx < points)
 * with strength amp_host[s] / h^ndim; taylor_p (1..max_taylor_p given at
 * create) is the Taylor order of the augmented matrix used by the Faber and
 * Krylov steps. n_src = 0 removes the sources. Synchronizes (small upload). */
int32_t expw_set_source_ricker(expw_op* op, int32_t n_src, const int64_t* node_idx_host,
                               const double* amp_host, double f_peak, double t_delay,
                               int32_t taylor_p);

/* A tabulated source time function (Sec. 3.2, augmented matrix: the source
 * over a step is its Taylor polynomial): point sources at node_idx_host with
 * amplitudes amp_host, as for expw_set_source_ricker, and gder_host
 * (nsteps x taylor_p, row-major, host) holding g^(k)(t_n), k = 0..taylor_p-1,
 * for step n = 0..nsteps-1 of each following step call (step n of a call uses
 * row n; a call with more steps than rows fails with EXPW_EINVAL; an adjoint
 * step uses row 0). Faber and Krylov use a row as the columns of W; RK4 and
 * leap-frog evaluate its Taylor polynomial at their stage times. The table is
 * copied; it stays until the next source call. Batches reject it
 * (EXPW_EUNSUPPORTED). n_src = 0 removes the sources. */
int32_t expw_set_source_taylor(expw_op* op, int32_t n_src, const int64_t* node_idx_host,
                               const double* amp_host, int32_t taylor_p, int64_t nsteps,
                               const double* gder_host);

/* Receivers (Sec. 5: seismograms recorded at points of the grid): n_rec flat
 * pressure-node indices in a caller-owned device int64 array (validated once,
 * synchronizes). After every step the pressure at the
 * receivers is written to traces[step * n_rec + r] when a step call is given
 * a non-NULL traces_dev. n_rec = 0 removes the receivers. When the indices
 * are consecutive (first, first + 1, ...: a receiver line along x) the kernel
 * that writes a step's final pressure also writes the traces (2D fused Faber
 * passes, the Krylov combination on the device, the last RK4 stage, the
 * leap-frog pressure update); otherwise one gather kernel runs per step. The
 * indices are read at this call: a later change of the array needs a new
 * call. */
int32_t expw_set_receivers(expw_op* op, int32_t n_rec, const int64_t* node_idx_dev);

/* Advance the state nsteps steps of size dt starting at time t0 (step s runs
 * from t0 + s dt). traces_dev: NULL or an array of nsteps * n_rec elements.
 * Faber steps (Sec. 3.2, Faber recurrence and sum, degree m = m products with
 * the augmented matrix): every term v_j is computed in FP64 from the stored
 * values and stored in the state dtype, the partial sum is kept in FP64 (in
 * the workspace between sweeps) and the step's result is rounded to the state
 * dtype once. With FP32 states this keeps the rounding of a step to that of
 * its stored terms: FP32 arithmetic inside a term, repeated on nearly the same
 * data every step, would round coherently and accumulate over long runs. */
int32_t expw_step_faber(expw_op* op, void* state_dev, double t0, double dt, int32_t m,
                        int64_t nsteps, void* traces_dev);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid it): expw_step_faber
 * with the step's buffers (the term vectors and the FP64 partial sum) in a
 * static device array of the library (EXPW_NOALLOC_SCRATCH_BYTES, one per
 * GPU, resolved when an operator is created on that GPU) instead of the
 * operator's workspace. It allocates nothing and calls no allocating
 * routine; results are those of expw_step_faber bit for bit. Limits: the grid
 * must need at most EXPW_NOALLOC_SCRATCH_BYTES (8 (ndim + 1) points bytes for
 * the sum + 4 state vectors of the dtype; EXPW_ENOMEM otherwise), m <=
 * EXPW_NOALLOC_MAX_M, and kernel timing off (EXPW_EINVAL). Every call on a GPU
 * uses the same array and leaves it holding its last contents (nothing in it
 * needs to start at zero): calls that overlap on one GPU (other streams,
 * other threads, other operators) race. */
enum { EXPW_NOALLOC_SCRATCH_BYTES = 64 << 20, EXPW_NOALLOC_MAX_M = 128 };
int32_t expw_step_faber_noalloc(expw_op* op, void* state_dev, double t0, double dt, int32_t m,
                                int64_t nsteps, void* traces_dev);

/* Faber steps that also record every term at the receivers: the pressure of
 * v_j = F_j(H~) [u_n; e_p], j = 0..m, at receiver r goes to
 * term_traces_dev[(s * (m + 1) + j) * n_rec + r] for step s (device array of
 * nsteps * (m + 1) * n_rec elements, state dtype; requires receivers). The
 * state and traces are those of expw_step_faber (terms are computed one per
 * sweep here). */
int32_t expw_step_faber_dense(expw_op* op, void* state_dev, double t0, double dt, int32_t m,
                              int64_t nsteps, void* traces_dev, void* term_traces_dev);
/* Receiver values between steps from recorded terms:
 * out_dev[i * n_rec + r] = sum_j coef_dev[i * (m + 1) + j] *
 * term_traces_dev[(sample_step_dev[i] * (m + 1) + j) * n_rec + r] for the
 * n_samples samples i (sample_step_dev: int64 step indices in [0, nsteps);
 * an index outside gives NaN; coef_dev: FP64 weights from
 * expw_faber_dense_coefficients). Sums in FP64; out_dev in the state dtype. */
int32_t expw_faber_dense_output(expw_op* op, int32_t m, int64_t n_samples,
                                const int64_t* sample_step_dev, const double* coef_dev,
                                const void* term_traces_dev, int64_t nsteps, void* out_dev);

/* Adjoint (gradient) support. The transpose of the step is built from the
 * same recurrence run backwards (Sec. 3.2, Faber recurrence; the adjoint
 * itself is not in the paper): with (D+)^T = -D-,
 * (H^T y)_p = sum_a D-_a y_{v_a} - sigma_p y_p and
 * (H^T y)_{v_a} = D+_a (c^2 y_p) - sigma_a y_{v_a}. */
/* y = H^T x (device state arrays, must not alias). */
int32_t expw_apply_adjoint(expw_op* op, const void* x_dev, void* y_dev);
/* Reverse of one Faber step of degree m from t with state u_dev (the state
 * at t, not modified): on entry lam_dev holds d(loss)/d(state at t + dt), on
 * return d(loss)/d(state at t) through this step; grad_c2_dev (one value per
 * point) is incremented by -(1/gamma) sum_j mu_{j,p} (sum_a D-_a v_{j-1,a}),
 * the derivative with respect to c^2 at fixed ellipse and coefficients.
 * terms_dev: caller scratch of (m - 1) state vectors (NULL when m = 1). The
 * ellipse, coefficients and source are those of expw_step_faber at t, so
 * this is the exact transpose of that step's linear part. On 2D grids with
 * zero ghosts the reverse terms run two per launch while j - 1 >= 1 (unless
 * expw_set_tuning asked for one term per sweep), with results equal to one
 * term per launch. Uses the workspace. */
int32_t expw_faber_adjoint_step(expw_op* op, const void* u_dev, void* lam_dev, double t, double dt,
                                int32_t m, void* grad_c2_dev, void* terms_dev);
/* Reverse of one Krylov step of dimension k from t (Sec. 3.2, Krylov
 * subspace projection; its adjoint is not in the paper). The Krylov step's
 * polynomial depends on its start vector, so the reverse step differentiates
 * the exponential it approximates and approximates each factor in a Krylov
 * space of dimension k: on return lam_dev holds the Krylov approximation of
 * exp(dt H^T) lam (Arnoldi with modified Gram-Schmidt on H^T from lam, the
 * forward step's breakdown rule), and grad_c2_dev (one value per point) is
 * incremented by the c^2 derivative of <lam, exp(dt H~) [u; e_p]>,
 *   dt int_0^1 <exp((1-s) dt H^T) lam, dH/dc^2[x] exp(s dt H~) [u; e_p]> ds,
 * with both exponentials taken in their Krylov spaces (the forward one is the
 * basis of the step from u_dev at t, with its source); the time integral is
 * the upper right block of one block-triangular exponential (Van Loan). Both
 * results converge to the exact exponential's derivatives as k grows.
 * k in [1, max_krylov_k at create] (the forward basis uses the workspace);
 * basis_dev: caller scratch of (k + 1) state vectors for the basis of H^T.
 * lam_dev, grad_c2_dev and basis_dev must not alias each other or u_dev.
 * Synchronizes the op's stream (two small host exponentials). */
int32_t expw_krylov_adjoint_step(expw_op* op, const void* u_dev, void* lam_dev, double t, double dt,
                                 int32_t k, void* grad_c2_dev, void* basis_dev);
/* state_dev pressure at the receivers += scale * values_dev[r] (adjoint
 * sources; device atomics, so repeated receivers add up). */
int32_t expw_inject_receivers(expw_op* op, const void* values_dev, double scale, void* state_dev);

/* Batches of independent problems (shots) stepped together (Faber
 * recurrence, Sec. 3.2): 2D order-4 zero-ghost shots run passes of S terms
 * (S = 2, 4 or 6 from the depth set on shot 0's operator by expw_set_tuning
 * or expw_autotune, rounded; default 6 in FP32, 4 in FP64; FP64 at most 4), pass p of every
 * shot still running in one launch (ceil(max m / S) + 1 launches per step,
 * or one with expw_batch_set_persistent); other shots run term j of every
 * shot with degree >= j in one launch (max m + 1 launches). The shots keep their own operators,
 * grids, ellipses, sources and receivers but must share dtype, ndim, order
 * and bc; each shot uses its operator's workspace. */
typedef struct expw_batch expw_batch;
/* Device bytes of the descriptor table of n_ops shots with grids like g. */
int32_t expw_batch_table_bytes(int32_t n_ops, const expw_grid* g, size_t* bytes);
/* Binds n_ops shots: ops[i] stepped with degree m[i] in [2, 64] and step
 * dt[i] on state states_dev[i]; traces_dev (NULL, or per shot NULL or an
 * array of steps * n_rec values) records the shot's receivers after every
 * step. The sources and receivers in effect on each operator now are the
 * ones used (recreate the batch after changing them). table_dev: caller
 * buffer of expw_batch_table_bytes bytes, 256-byte aligned, written here
 * (synchronizes). stream: HIP stream of all batch work (NULL = default). */
int32_t expw_batch_create(expw_op* const* ops, int32_t n_ops, const int32_t* m, const double* dt,
                          void* const* states_dev, void* const* traces_dev, void* table_dev,
                          size_t table_bytes, void* stream, expw_batch** out);
/* nsteps steps of every shot, numbered step0, step0 + 1, ...: shot i's step
 * n runs from t0 + n dt[i] and its traces go to row n. */
int32_t expw_batch_step_faber(expw_batch* b, double t0, int64_t nsteps, int64_t step0);
/* Captures the launches of nsteps steps into a HIP graph (stream capture on
 * the batch's stream, which must not be the default stream); later step
 * calls replay it for every whole group of nsteps steps (the step time and
 * trace row come from a clock in the table, set by a small kernel before
 * each replay). nsteps = 0 drops the graph. The graph holds no memset or
 * memcpy nodes. */
int32_t expw_batch_capture(expw_batch* b, int64_t nsteps);
/* One launch per batched step (Sec. 3.2, Faber recurrence): on = 1 runs every
 * pass of every shot, the copies of one-pass shots and the receiver
 * recording of a step in one cooperative launch whose workgroups take the
 * shots' tiles in turn and meet at a grid-wide barrier between passes; on =
 * 0 returns to one launch per pass. Needs 2D order-4 zero-ghost shots
 * (EXPW_EUNSUPPORTED otherwise, or without cooperative launches). Each
 * expw_batch_step_faber call then synchronizes the batch's stream once at
 * its end, and fails with EXPW_EDEVICE if a barrier wait timed out (bounded
 * waits: the kernel always ends). Captured sequences (expw_batch_capture)
 * keep one launch per pass. */
int32_t expw_batch_set_persistent(expw_batch* b, int32_t on);
int32_t expw_batch_destroy(expw_batch* b);

/* Krylov steps (Arnoldi with modified Gram-Schmidt on the augmented matrix,
 * then the small exponential, see expw_set_krylov_expm). Requires
 * k <= max_krylov_k. */
int32_t expw_step_krylov(expw_op* op, void* state_dev, double t0, double dt, int32_t k,
                         int64_t nsteps, void* traces_dev);
/* Classical four-stage RK4 steps (Sec. 3.1, low-order methods) of
 * U' = H U + f(t), the source sampled at the stage times t, t + dt/2 (twice)
 * and t + dt; state, traces and errors as for expw_step_faber. */
int32_t expw_step_rk4(expw_op* op, void* state_dev, double t0, double dt, int64_t nsteps,
                      void* traces_dev);
/* Leap-frog steps (Sec. 3.1; the reading for the first-order system): the
 * staggered-time update v^{n+1/2} = [(1 - sigma dt/2) v^{n-1/2} - dt D+ p^n] /
 * (1 + sigma dt/2), then p^{n+1} from D- v^{n+1/2} and the source at
 * t + dt/2, damping averaged the same way. The velocity slots of the state
 * hold v at t - dt/2 (start from zero velocities at rest). */
int32_t expw_step_leapfrog(expw_op* op, void* state_dev, double t0, double dt, int64_t nsteps,
                           void* traces_dev);

/* Synchronizes the stream and reports a pending device error (including a
 * grid barrier of the persistent Arnoldi kernel that exceeded its bounded
 * wait), then a state the non-finite guard caught (EXPW_ENONFINITE, reported
 * once). */
int32_t expw_sync_status(expw_op* op);

/* Optional non-finite guard: on != 0 checks the state for NaN and infinite
 * values after every step of every step call (one extra read of the state per
 * step); a hit surfaces as EXPW_ENONFINITE at the next expw_sync_status. */
int32_t expw_set_guard(expw_op* op, int32_t on);

/* Effective dimension and beta of the last Krylov step (host values;
 * synchronizes when the step ran its small exponential on the device).
 * k_eff is one more than the first column j <= k - 2 with h_{j+1,j} <=
 * 1e-14 beta, else k; h_{k,k-1} itself is not formed by the persistent
 * Arnoldi kernel (neither the k x k exponential nor the combination uses it)
 * and is not read. */
int32_t expw_krylov_info(const expw_op* op, int32_t* k_eff, double* beta);
/* A-posteriori error estimate of Krylov steps (Sec. 3.2, Krylov subspace
 * projection; the estimate itself is not in the paper). With on != 0, every
 * later expw_step_krylov step forms
 *   est = dt beta h_{k+1,k} |e_k^T phi_1(dt H_k) e_1|, phi_1(z) = (e^z - 1)/z,
 * the norm of the projected flow's residual integrated over the step (the
 * step's error is that residual propagated by exp((dt - s) H~)); 0 after a
 * breakdown (k_eff < k). It costs the last column's orthogonalization and
 * norm, and the small exponential then runs on the host (one synchronization
 * per step). expw_krylov_estimate returns the largest estimate over the steps
 * of the last expw_step_krylov call, or EXPW_EINVAL if that call ran without
 * the estimate. */
int32_t expw_set_krylov_estimate(expw_op* op, int32_t on);
int32_t expw_krylov_estimate(const expw_op* op, double* est);

/* Where the Krylov step evaluates y = exp(dt H_k) e_1 (Sec. 3.2: the small
 * Hessenberg exponential), both in FP64:
 *   EXPW_EXPM_DEVICE (default): one workgroup evaluates it by scaling and
 *     squaring of the degree-16 Taylor polynomial; the step stays
 *     asynchronous.
 *   EXPW_EXPM_HOST: scaling-and-squaring [13/13] Pade on the host (the same
 *     routine as expw_expm); one synchronization per step. */
enum { EXPW_EXPM_DEVICE = 0, EXPW_EXPM_HOST = 1 };
int32_t expw_set_krylov_expm(expw_op* op, int32_t mode);

/* allow = 1 (default): when the grid fits in registers across one cooperative
 * grid (every thread holding up to two grid points with all their fields,
 * three in 2D), the Arnoldi process runs as one persistent launch with one
 * grid-wide reduction per column (modified Gram-Schmidt's projections from
 * one batched reduction of the dots, the basis Gram entries and the column's
 * norm, by forward substitution) and, in place of a second barrier, waits on
 * the flags of the workgroups whose part of the new column its stencil
 * reads; otherwise, and with allow = 0, one launch per matrix-vector product
 * and four per Gram-Schmidt column. Results agree to rounding. */
int32_t expw_set_krylov_persistent(expw_op* op, int32_t allow);

/* ------------------------------------------------------------------ timing */

/* Kernel classes for expw_get_timing. */
enum {
  EXPW_KERNEL_FABER = 0,        /* Faber pass: fused multi-term sweep, or one term */
  EXPW_KERNEL_KRYLOV_MATVEC = 1, /* Arnoldi: w = H~ q with the first dot */
  EXPW_KERNEL_KRYLOV_MGS = 2,    /* Arnoldi: Gram-Schmidt axpy with the next dot */
  EXPW_KERNEL_KRYLOV_AUX = 3,    /* Arnoldi: norm, start vector, normalize, combine */
  EXPW_KERNEL_RK4 = 4,           /* RK4 stage */
  EXPW_KERNEL_LEAPFROG_V = 5,    /* leap-frog velocity update */
  EXPW_KERNEL_LEAPFROG_P = 6,    /* leap-frog pressure update */
  EXPW_KERNEL_GATHER = 7,        /* receiver gather */
  EXPW_KERNEL_KRYLOV_ARNOLDI = 8, /* Arnoldi: the whole basis in one persistent launch */
  EXPW_KERNEL_CLASSES = 9
};

/* Per-launch timing with HIP events recorded on the handle's stream around
 * every launch of the kernel classes whose bit is set in class_mask (bit k =
 * class k; 0 = off, -1 = all classes); also clears the totals. */
int32_t expw_set_timing(expw_op* op, int32_t class_mask);

/* Synchronizes and returns, per kernel class (arrays of EXPW_KERNEL_CLASSES
 * entries, any may be NULL), the summed kernel time in ms, the number of
 * launches and the algorithmic HBM bytes (each operand array counted once per
 * launch, halos not counted) since timing was enabled. */
int32_t expw_get_timing(expw_op* op, double* ms, int64_t* launches, double* bytes);

/* Bandwidth ceiling (not part of the method): times reps launches of a plain
 * stream kernel over arrays of `bytes` bytes (a positive multiple of 16;
 * device pointers, 16-byte aligned) on `stream`, after one warm-up launch,
 * with HIP events, and returns the mean time per launch in ms (synchronizes).
 * kind 0: read a (one partial sum per 4096 vectors of 16 bytes written to c,
 * which must hold bytes / 4096 floats); 1: copy c = a; 2: triad c = a + 2 b.
 * nontemporal != 0 marks loads and stores as streaming (no reuse). HBM bytes
 * per launch: bytes (read), 2 bytes (copy), 3 bytes (triad). */
int32_t expw_stream_bench(int32_t kind, int32_t nontemporal, const void* a, const void* b, void* c,
                          size_t bytes, int32_t reps, void* stream, double* ms_per_launch);

/* ---------------------------------------------- the paper's PML operator
 *
 * Sec. 2, 2.1, 2.2 and the appendix on the free surface: the 2D acoustic
 * system with perfectly matched layers in (u, v, w_x, w_y), displacement u,
 * its rate v = u_t and the auxiliaries w_x, w_y:
 *   u_t = v
 *   v_t = (-b_x b_y + c^2 (d_xx + d_yy)) u - (b_x + b_y) v + c^2 (d_x w_x + d_y w_y) + f
 *   w_x,t = (b_y - b_x) d_x u - b_x w_x,   w_y,t = (b_x - b_y) d_y u - b_y w_y
 * on nx x ny nodes, row 0 the free surface and y pointing up (y = -j h).
 * Layout of a state (dtype of the grid, device memory): four fields of
 * nx * ny values, x fastest, [u | v | w_x | w_y]; u, v and c^2 at nodes
 * (i, j), w_x at (i + 1/2, j), w_y at (i, j + 1/2). Stencils: 8th-order
 * staggered first and centred second derivatives with zero values outside
 * the sides and the bottom; at the top, the appendix's one-sided stencils for
 * d_yy u (rows 0..3) and d_y u (half rows 0..2), and Fornberg weights on the
 * surface point (w_y = 0 there) and w_y's eight nearest half rows for d_y w_y
 * (rows 0..3). The damping b_z = beta0 (1 - d/delta)^2 grows towards the two
 * sides (b_x) and the bottom (b_y); there is no layer at the top. Sources
 * enter the v equation with strength amp / h^2; receivers record u. */
typedef struct {
  int64_t nx, ny;    /* nodes along x and depth; nx >= 1, ny >= 9 */
  double h;          /* grid spacing (m), > 0 */
  int32_t dtype;     /* expw_dtype of every device array */
  int32_t abc_cells; /* layer thickness delta = abc_cells h, >= 0 */
  double beta0;      /* beta_0 of the profile (1/s), >= 0 */
} expw_pml_grid;

typedef struct expw_pml expw_pml;

/* Host only: validates a grid (EXPW_EINVAL with a message). */
int32_t expw_pml_check_grid(const expw_pml_grid* grid);

/* Host only: the rectangle [x_lo, 0] x i[-B, B] around the spectrum (the
 * paper gives no formula; the reading): B = 1.25 c_max sqrt(2 s), s the
 * largest symbol (205/72 + 2 sum |b_l|) / h^2 of the centred second derivative
 * along one axis and 1.25 a margin for the one-sided surface rows;
 * x_lo = -(max b_x + max b_y). */
int32_t expw_pml_spectrum_rectangle(const expw_pml_grid* grid, double c2_max, double* x_lo, double* B);

/* Host only: the one-sided tables the kernels use, row-major in FP64:
 * d2[4][9] (d_yy u at rows 0..3 from u_0..u_8, times 1/h^2), d1[3][8] (d_y u
 * at half rows 0..2 from u_0..u_7, times 1/h), dw[4][8] (d_y w_y at rows
 * 0..3 from w_y's half rows 0..7, times 1/h). */
int32_t expw_pml_surface_weights(double* d2, double* d1, double* dw);

/* Bytes of device workspace expw_pml_create needs for a largest Krylov
 * dimension max_krylov_k (0 = Krylov unused, <= EXPW_MAX_KRYLOV) and a largest
 * source Taylor order max_taylor_p (<= EXPW_MAX_TAYLOR). */
int32_t expw_pml_workspace_size(const expw_pml_grid* grid, int32_t max_krylov_k, int32_t max_taylor_p,
                                size_t* bytes);

/* Binds a grid, c^2 at the nodes (nx * ny values, > 0, read until destroy)
 * and a caller-owned, 256-byte aligned workspace; computes the spectrum
 * rectangle and the Faber ellipse. stream: hipStream_t (NULL = default). */
int32_t expw_pml_create(const expw_pml_grid* grid, const void* c2_dev, int32_t max_krylov_k,
                        int32_t max_taylor_p, void* workspace_dev, size_t workspace_bytes,
                        void* hip_stream, expw_pml** out);
int32_t expw_pml_destroy(expw_pml* op);
int32_t expw_pml_get_ellipse(const expw_pml* op, double* gamma, double* c0, double* c1);

/* y = H x (device arrays of 4 nx ny values; y must not alias x). */
int32_t expw_pml_apply(expw_pml* op, const void* x_dev, void* y_dev);

/* Point sources on the v equation at nodes node_idx_host[s] (j nx + i), one
 * Ricker wavelet, Taylor order taylor_p <= max_taylor_p (Sec. 3.2, augmented
 * matrix). n_src = 0 removes them. */
int32_t expw_pml_set_source_ricker(expw_pml* op, int32_t n_src, const int64_t* node_idx_host,
                                   const double* amp_host, double f_peak, double t_delay,
                                   int32_t taylor_p);

/* Receivers: u at node_idx_dev[r] (device array, kept until replaced). */
int32_t expw_pml_set_receivers(expw_pml* op, int32_t n_rec, const int64_t* node_idx_dev);

/* nsteps Faber steps of degree m (Sec. 3.2) in place on state_dev, step n
 * from t0 + n dt, one term per sweep; traces_dev (nullable) receives u at the
 * receivers after every step (nsteps x n_rec). Asynchronous on the stream. */
int32_t expw_pml_step_faber(expw_pml* op, void* state_dev, double t0, double dt, int32_t m,
                            int64_t nsteps, void* traces_dev);

/* nsteps Krylov steps of dimension k <= max_krylov_k (Sec. 3.2, Arnoldi with
 * modified Gram-Schmidt on the augmented matrix, exp(dt H_k) e_1 on the device)
 * in place; traces as for expw_pml_step_faber. */
int32_t expw_pml_step_krylov(expw_pml* op, void* state_dev, double t0, double dt, int32_t k,
                             int64_t nsteps, void* traces_dev);

/* nsteps classical RK4 steps (Sec. 3.1) in place, the source at the stage
 * times; traces as for expw_pml_step_faber. */
int32_t expw_pml_step_rk4(expw_pml* op, void* state_dev, double t0, double dt, int64_t nsteps,
                          void* traces_dev);

/* Kernel of the Faber terms: 0 = automatic (row-streamed passes where the
 * grid gives them 512 x 256 threads in row segments of 64 rows or more, else
 * at FP32 two terms per pass and at FP64 LDS tiles of 64 x 16 nodes once the
 * grid has at least 2048 of them, one thread per node below; a step of one
 * term takes the LDS tiles or one thread per node), 1 = one thread per node,
 * 2 = LDS tiles, 3 = two terms per pass on LDS tiles (temporal blocking; an
 * odd last term alone), 4 = row-streamed passes of up to 4 terms at FP32 and
 * 2 at FP64 (no recomputation along y; a last single term alone). Results
 * agree to rounding. */
int32_t expw_pml_set_path(expw_pml* op, int32_t path);

/* The path (1 to 4) a step of degree m takes under the current setting. */
int32_t expw_pml_path_for(const expw_pml* op, int32_t m, int32_t* path);

/* Synchronizes the stream and reports device errors. */
int32_t expw_pml_sync_status(expw_pml* op);

#ifdef __cplusplus
}
#endif

#endif /* EXPWAVE_H */
