// C ABI of the exponential wave-propagation library: handle, validation,
// workspace layout and the host drivers of the Faber, Krylov, RK4 and
// leap-frog steps. All device work is enqueued on the handle's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "adjoint.h"
#include "arnoldi.h"
#include "batch.h"
#include "expm_small.h"
#include "fused.h"
#include "fused3d.h"
#include "gram.h"
#include "internal.h"
#include "kernels.h"
#include "pml.h"
#include "pml_stream.h"
#include "profiler.h"
#include "stream.h"
#include "stream2d.h"
#include "term_zero.h"

struct expw_op {
  expw_grid g;
  // the Faber coefficients of the last (gamma, c0, c1, dt, m) a step used:
  // steps taken one call at a time (an inversion's forward, recomputation and
  // reverse sweeps) reuse them instead of recomputing the (m + 1) M-point
  // trapezoidal sums (about 80 us on the host at m = 20)
  double coef_key[4];
  int coef_m;  // 0: none yet
  double coef[1025];
  int K;
  double alpha[4];
  const void* c2;
  char* ws;
  size_t ws_bytes;
  hipStream_t stream;
  int kmax, pmax;
  // workspace layout (byte offsets)
  size_t off_sig[3][2];
  size_t off_src_idx, off_src_amp, off_part, off_scal, off_hess, off_kry, off_bar, off_big;
  int64_t naug_pad;  // stride of a Krylov basis vector (elements)
  // spectrum and ellipse (host FP64)
  double c2max, x_lo, B, gamma, c0, c1;
  // sources
  int n_src;
  std::vector<int64_t> src_idx;
  std::vector<double> src_amp;
  int64_t src_lo, src_hi;
  double f_peak, t_delay;
  int taylor_p;
  // a tabulated source (expw_set_source_taylor): row n holds g^(k)(t_n),
  // k = 0..taylor_p-1, for step n of the next step call
  int src_table;
  std::vector<double> src_rows;
  int64_t src_nrows;
  // receivers; rec_run_first >= 0 when they are the consecutive pressure
  // nodes rec_run_first .. rec_run_first + n_rec - 1 (then the kernel that
  // writes a step's final pressure records them, instead of a gather)
  int n_rec;
  const int64_t* rec_dev;
  int64_t rec_run_first;
  // non-finite guard after every step (expw_set_guard)
  int guard;
  // tuning
  int fuse;
  int pass_kernel;  // 2D order-4 fused passes: 0 by grid size, 1 tiled, 2 streamed
  // Krylov: small exponential on the device (0) or the host (1); last step info
  int kry_mode;
  int kry_persistent;  // 1: allow the persistent Arnoldi kernel
  int coop_blocks;     // co-resident blocks of the persistent kernel (0 = unknown)
  int arn_nvmax_clean;  // reduction area consistent for this nvmax (0: fill before the next launch)
  int last_keff;
  double last_beta;
  bool kry_estimate;    // form the a-posteriori estimate of each Krylov step
  bool last_est_valid;  // the last Krylov call formed it
  double last_est;      // the largest estimate over that call's steps
  char* noalloc_scratch;  // device address of the static scratch on the creating device
  expw::Profiler prof;
};

struct expw_batch {
  int n;
  expw_grid g;  // dtype, ndim, order, bc shared by the shots
  int K;
  hipStream_t stream;
  void* table;       // device: shots (sorted by degree), block prefix, receiver prefix
  size_t off_prefix, off_prefix_rec;
  int max_m;
  std::vector<int> count_ge;        // count_ge[j] = shots with degree >= j
  std::vector<int64_t> prefix;      // host copy of the block prefix
  int64_t rec_items;
  // fused passes (2D, order 4, zero ghosts)
  bool fused;
  size_t off_fshots, off_fprefix;
  int max_passes;
  std::vector<int> count_pass;      // count_pass[p] = shots with more than p passes
  std::vector<int64_t> fprefix;     // host copy of the tile prefix
  std::vector<void*> copy_dst, copy_src;  // one-pass shots: sum C -> state
  std::vector<int64_t> copy_elems;
  int depth;          // terms per fused pass (2, 4 or 6)
  bool persistent;    // one cooperative launch per step
  int coop_blocks;    // workgroups of that launch (0 = not known yet, < 0 = unavailable)
  size_t off_sync;    // its barrier words (BatchSync)
  size_t off_qstep;   // the step's source scalars (kBatchMaxM doubles per shot)
  size_t off_clock;
  // a captured sequence of graph_steps steps (nullptr: none)
  hipGraph_t graph;
  hipGraphExec_t gexec;
  int64_t graph_steps;
};

namespace expw {
namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
int64_t npts(const expw_grid& g) { return g.n[0] * g.n[1] * (g.ndim == 3 ? g.n[2] : 1); }
size_t elem_size(const expw_grid& g) { return g.dtype == EXPW_F32 ? 4 : 8; }
constexpr int kHessLd = EXPW_MAX_KRYLOV;  // leading dimension of the Hessenberg matrix

int32_t validate_grid(const expw_grid* g) {
  if (!g) return fail(EXPW_EINVAL, "grid is NULL");
  if (g->ndim != 2 && g->ndim != 3) return fail(EXPW_EINVAL, "ndim must be 2 or 3 (got %d)", g->ndim);
  if (g->order != 4 && g->order != 8) return fail(EXPW_EINVAL, "order must be 4 or 8 (got %d)", g->order);
  for (int a = 0; a < g->ndim; ++a)
    if (g->n[a] < 1) return fail(EXPW_EINVAL, "n[%d] must be >= 1", a);
  if (g->ndim == 2 && g->n[2] != 1) return fail(EXPW_EINVAL, "n[2] must be 1 for a 2D grid");
  if (!(g->h > 0.0) || !std::isfinite(g->h)) return fail(EXPW_EINVAL, "h must be positive and finite");
  if (g->dtype != EXPW_F32 && g->dtype != EXPW_F64) return fail(EXPW_EINVAL, "dtype must be EXPW_F32 or EXPW_F64");
  if (g->bc != EXPW_BC_ZERO && g->bc != EXPW_BC_PERIODIC) return fail(EXPW_EINVAL, "bc must be EXPW_BC_ZERO or EXPW_BC_PERIODIC");
  if (g->abc_cells < 0) return fail(EXPW_EINVAL, "abc_cells must be >= 0");
  if (!(g->sigma_max >= 0.0) || !std::isfinite(g->sigma_max)) return fail(EXPW_EINVAL, "sigma_max must be >= 0 and finite");
  if (g->bc == EXPW_BC_PERIODIC && g->sigma_max != 0.0 && g->abc_cells > 0)
    return fail(EXPW_EINVAL, "a periodic grid takes no damping layer");
  if (g->reserved != 0) return fail(EXPW_EINVAL, "reserved must be 0");
  if (npts(*g) > (int64_t(1) << 40)) return fail(EXPW_EINVAL, "grid too large");
  return EXPW_OK;
}

struct Layout {
  size_t sig[3][2];
  size_t src_idx, src_amp, part, scal, hess, kry, bar, big, total;
  int64_t naug_pad;
};

// The buffers of a Faber step (FaberBufs) in one region: the FP64 partial
// sum first, then the two (v_last, v_prev) pairs of T.
template <typename T>
FaberBufs<T> faber_bufs(char* big, int64_t ns) {
  FaberBufs<T> b;
  b.C = reinterpret_cast<double*>(big);
  b.A = reinterpret_cast<T*>(big + align_up(static_cast<size_t>(ns) * sizeof(double)));
  b.B = b.A + ns;
  b.D = b.B + ns;
  b.E = b.D + ns;
  return b;
}

size_t faber_big_bytes(int64_t ns, size_t es) {
  return align_up(static_cast<size_t>(ns) * sizeof(double)) + 4 * static_cast<size_t>(ns) * es;
}

Layout layout(const expw_grid& g, int kmax, int pmax) {
  Layout L{};
  const size_t es = elem_size(g);
  size_t off = 0;
  for (int a = 0; a < 3; ++a)
    for (int hf = 0; hf < 2; ++hf) {
      L.sig[a][hf] = off;
      if (a < g.ndim) off = align_up(off + g.n[a] * es);
    }
  L.src_idx = off; off = align_up(off + EXPW_MAX_SOURCES * sizeof(int64_t));
  L.src_amp = off; off = align_up(off + EXPW_MAX_SOURCES * es);
  L.part = off; off = align_up(off + 2 * kRedMaxBlocks * sizeof(double));  // two partial sets
  L.scal = off; off = align_up(off + 64 * sizeof(double));
  L.hess = off; off = align_up(off + (EXPW_MAX_KRYLOV + 1) * kHessLd * sizeof(double));
  L.kry = off; off = align_up(off + 64 * sizeof(double) + 72 * sizeof(double) + 64 * sizeof(int));  // y, scales, keff
  // grid reduction records and slots of the persistent Arnoldi kernel; the
  // launch-per-column Gram-Schmidt's partials and Gram table share the area
  // (below the column flags, which only the persistent kernel uses)
  static_assert(static_cast<size_t>(kGramPartials) + kGramTot + 2 * EXPW_MAX_KRYLOV <= kArnFlagWord,
                "Gram-Schmidt partials fit the reduction area");
  L.bar = off; off = align_up(off + kArnAreaWords * sizeof(unsigned long long));
  L.big = off;
  const int64_t ns = (g.ndim + 1) * npts(g);
  L.naug_pad = (ns + pmax + 63) / 64 * 64;
  size_t big = faber_big_bytes(ns, es);  // Faber: FP64 partial sum + v pairs (2 x 2)
  if (kmax > 0) big = std::max(big, static_cast<size_t>(kmax + 1) * L.naug_pad * es);
  L.total = align_up(off + big);
  return L;
}

template <typename T, int K, int BC, int DIM>
struct Cfg {
  using type = T;
  static constexpr int k = K, bc = BC, dim = DIM;
};

template <typename T, class Fn>
int32_t dispatch_t(const expw_op* op, Fn& fn) {
  const bool per = op->g.bc == EXPW_BC_PERIODIC;
  const bool d3 = op->g.ndim == 3;
  if (op->K == 2) {
    if (d3) return per ? fn(Cfg<T, 2, 1, 3>{}) : fn(Cfg<T, 2, 0, 3>{});
    return per ? fn(Cfg<T, 2, 1, 2>{}) : fn(Cfg<T, 2, 0, 2>{});
  }
  if (d3) return per ? fn(Cfg<T, 4, 1, 3>{}) : fn(Cfg<T, 4, 0, 3>{});
  return per ? fn(Cfg<T, 4, 1, 2>{}) : fn(Cfg<T, 4, 0, 2>{});
}

template <class Fn>
int32_t dispatch(const expw_op* op, Fn&& fn) {
  if (op->g.dtype == EXPW_F32) return dispatch_t<float>(op, fn);
  return dispatch_t<double>(op, fn);
}

template <typename T, int K, int DIM>
Geo<T, K, DIM> make_geo(const expw_op* op) {
  Geo<T, K, DIM> g{};
  g.n[0] = op->g.n[0];
  g.n[1] = op->g.n[1];
  g.n[2] = DIM == 3 ? op->g.n[2] : 1;
  g.st[0] = 1;
  g.st[1] = g.n[0];
  g.st[2] = g.n[0] * g.n[1];
  g.N = g.n[0] * g.n[1] * g.n[2];
  for (int l = 0; l < K; ++l) {
    g.wd[l] = op->alpha[l] / op->g.h;
    g.w[l] = static_cast<T>(g.wd[l]);
  }
  {
    double wi[4], beta = 0.0;
    int kk = 0;
    stagger_weights_int(op->g.order, wi, &beta, &kk);
    for (int l = 0; l < K; ++l) g.wi[l] = static_cast<T>(wi[l]);
    g.wscale = beta / op->g.h;
  }
  g.c2 = static_cast<const T*>(op->c2);
  for (int a = 0; a < 3; ++a) {
    g.sint[a] = reinterpret_cast<const T*>(op->ws + op->off_sig[a][0]);
    g.shalf[a] = reinterpret_cast<const T*>(op->ws + op->off_sig[a][1]);
  }
  return g;
}

template <typename T>
Src<T> make_src(const expw_op* op, double q) {
  Src<T> s{};
  s.n = op->n_src;
  s.lo = op->src_lo;
  s.hi = op->src_hi;
  s.idx = reinterpret_cast<const int64_t*>(op->ws + op->off_src_idx);
  s.amp = reinterpret_cast<const T*>(op->ws + op->off_src_amp);
  s.q = q;
  return s;
}

int32_t check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(EXPW_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  return EXPW_OK;
}

// The device kernel for y = exp(dt H_k) e_1 and its workgroup size: 16 x 16
// tiles for k <= 16, 32 x 32 tiles for 20 <= k <= 32, else the general
// kernel, whose cost grows with k (measured, 28 products: 25 us at k = 16,
// 134 us at k = 30; the 32 x 32 tiles take 43 us at any k, 16 x 16 tiles 10 us).
using ExpmKernel = void (*)(const double*, int, double, double, const double*, double*, int*);
ExpmKernel expm_kernel(int k) {
  return k <= 16 ? k_kry_expm_tile<16> : (k >= 20 && k <= kExpmSmallK) ? k_kry_expm_tile<32> : k_kry_expm;
}
unsigned expm_threads(int k) {
  return k <= 16 ? 256u : (k >= 20 && k <= kExpmSmallK) ? 1024u : static_cast<unsigned>(kBlock);
}

unsigned grid_for(int64_t n) {
  return static_cast<unsigned>(std::max<int64_t>(1, (n + kBlock - 1) / kBlock));
}
unsigned red_grid_for(int64_t n) {
  return static_cast<unsigned>(std::min<int64_t>(kRedMaxBlocks, std::max<int64_t>(1, (n + 4 * kBlock - 1) / (4 * kBlock))));
}

double src_scale(const expw_op* op) { return 1.0 / std::pow(op->g.h, op->g.ndim); }

// g^(k)(t_n), k = 0..p-1, for step st of a call (time t_n = t): the Ricker
// wavelet, or row st of the table
void source_derivs(const expw_op* op, int64_t st, double t, int p, double* der) {
  if (op->src_table) {
    const double* row = op->src_rows.data() + st * op->taylor_p;
    for (int k = 0; k < p; ++k) der[k] = row[k];
  } else {
    ricker_derivatives(t, op->f_peak, op->t_delay, p, der);
  }
}

// g(t_n + tau) for step st: the Ricker wavelet, or the table row's Taylor
// polynomial (Sec. 3.2: the source over a step is its Taylor polynomial)
double source_value(const expw_op* op, int64_t st, double t, double tau) {
  if (!op->src_table) {
    double g0;
    ricker_derivatives(t + tau, op->f_peak, op->t_delay, 1, &g0);
    return g0;
  }
  const double* row = op->src_rows.data() + st * op->taylor_p;
  double acc = 0.0, term = 1.0;
  for (int k = 0; k < op->taylor_p; ++k) {
    acc += row[k] * term;
    term *= tau / (k + 1);
  }
  return acc;
}

// a step call of nsteps steps needs as many table rows
int32_t check_source_rows(const expw_op* op, int64_t nsteps) {
  if (op->n_src > 0 && op->src_table && nsteps > op->src_nrows)
    return fail(EXPW_EINVAL, "the source table has %lld rows, the call needs %lld", (long long)op->src_nrows,
                (long long)nsteps);
  return EXPW_OK;
}


// the non-finite flag of the guard (an int of the Krylov scalar area, zeroed at create)
int* guard_flag(const expw_op* op) {
  return reinterpret_cast<int*>(op->ws + op->off_kry + 136 * sizeof(double)) + 9;
}

// the optional non-finite guard on a state of ns values, after a step
template <typename T>
int32_t guard_state(expw_op* op, const T* S, int64_t ns) {
  if (!op->guard) return EXPW_OK;
  k_guard<T><<<red_grid_for(ns), kBlock, 0, op->stream>>>(S, ns, guard_flag(op));
  return check_launch("guard");
}

template <typename T>
int32_t gather(expw_op* op, const T* S, T* traces, int64_t step) {
  if (!traces || op->n_rec == 0) return EXPW_OK;
  launch_timed(&op->prof, op->stream, EXPW_KERNEL_GATHER, op->n_rec * (2.0 * sizeof(T) + 8.0), k_gather<T>, dim3(grid_for(op->n_rec)), dim3(kBlock), S, op->rec_dev, op->n_rec, traces + step * op->n_rec);
  return check_launch("gather");
}

// The receivers of step `step` as a run recorded by the step's last kernel,
// or none (out = nullptr: no traces, no receivers, or not a run; then
// gather() records them after the step).
template <typename T>
RecRun<T> rec_run(const expw_op* op, T* traces, int64_t step) {
  if (!traces || op->n_rec == 0 || op->rec_run_first < 0) return RecRun<T>{nullptr, 0, 0};
  return RecRun<T>{traces + step * op->n_rec, op->rec_run_first, op->n_rec};
}

// ---------------------------------------------------------------- Faber step

// The ellipse of a Faber step: the operator's, in FP64 for both storage
// precisions (every term is computed in FP64).
// For FP32 states the ellipse is moved (by a relative 1e-7 at most, well
// inside the slack of the spectral bound) so that the kernels that compute a
// term entirely in FP32 apply H / gamma exactly up to rounding: kappa =
// wscale / gamma is rounded to FP32 and gamma taken back from it, and c0, c1
// are rounded to FP32. The FP64 kernels run on the same (gamma, c0, c1), and
// the coefficients and source scalars are computed in FP64 for it, so every
// kernel of a step evaluates the same polynomial. FP64 states: the
// operator's ellipse as it is.
struct WorkEllipse {
  double gamma, c0, c1;
  double kappa;   // wscale / gamma (an FP32 value for FP32 states)
  double inv_ws;  // 1 / wscale rounded like kappa (damping in units of the stencil factor)
  explicit WorkEllipse(const expw_op* op) : gamma(op->gamma), c0(op->c0), c1(op->c1) {
    double wi[4], beta = 0.0;
    int kk = 0;
    stagger_weights_int(op->g.order, wi, &beta, &kk);
    const double ws = beta / op->g.h;
    kappa = ws / gamma;
    inv_ws = 1.0 / ws;
    if (op->g.dtype == EXPW_F32) {
      kappa = static_cast<double>(static_cast<float>(kappa));
      gamma = ws / kappa;
      c0 = static_cast<double>(static_cast<float>(c0));
      c1 = static_cast<double>(static_cast<float>(c1));
      inv_ws = static_cast<double>(static_cast<float>(inv_ws));
    }
  }
};

// Stencil arithmetic of the one-term zero-ghost kernel (see k_faber_term_zero):
// difference sums in the storage precision over integer weights.
template <typename T>
using TermSC = T;

// One Faber term per sweep: the zero-ghost kernel of order 4 or 8 where it
// applies, else the generic one (same arguments and outputs).
template <typename T, int K, int BC, int DIM>
void launch_term(expw_op* op, const Geo<T, K, DIM>& g, double bytes, const T* vp, const T* vpp,
                 T* vout, const double* acc_in, double* acc_out, T* state_out, const FaberTerm& c,
                 const Src<T>& src) {
  if constexpr ((K == 2 || K == 4) && BC == 0) {
    if ((DIM + 1) * g.N < (int64_t(1) << 31)) {
      launch_timed(&op->prof, op->stream, EXPW_KERNEL_FABER, bytes, k_faber_term_zero<T, K, DIM, TermSC<T>>,
                   term_zero_grid<DIM>(g.n), dim3(kTzX * kTzY), g, vp, vpp, vout, acc_in, acc_out, state_out,
                   c, src);
      return;
    }
  }
  launch_timed(&op->prof, op->stream, EXPW_KERNEL_FABER, bytes, k_faber_term<T, K, BC, DIM>,
               dim3(grid_for(g.N)), dim3(kBlock), g, vp, vpp, vout, acc_in, acc_out, state_out, c, src);
}

// One Faber step, one term per sweep. term_out (nullable): receives the
// pressure of every term v_0..v_m at the receivers ((m + 1) * n_rec values).
template <typename T, int K, int BC, int DIM>
int32_t faber_unfused(expw_op* op, const Geo<T, K, DIM>& g, const WorkEllipse& el, T* S,
                      const FaberBufs<T>& b, const double* a, const double* q, int m,
                      T* term_out) {
  const int64_t ns = (DIM + 1) * g.N;
  const bool keep = term_out != nullptr && op->n_rec > 0;
  auto record = [&](const T* v, int j) -> int32_t {
    return keep ? gather<T>(op, v, term_out + static_cast<int64_t>(j) * op->n_rec, 0) : EXPW_OK;
  };
  if (int32_t rc = record(S, 0)) return rc;
  FaberTerm c{};
  c.inv_gamma = 1.0 / el.gamma;
  c.c0 = el.c0;
  // j = 1: v1 = F1 v0 into A; sum = a0 v0 + a1 v1 into C (m = 1: the result
  // into B and then S, which this sweep reads with its halo)
  c.cpp = 0.0;
  c.first = 1;
  c.a_first = a[0];
  c.a_j = a[1];
  const double nf = DIM + 1, pb = static_cast<double>(g.N) * sizeof(T), pd = static_cast<double>(g.N) * sizeof(double);
  // bytes: reads v_{j-1} (nf T) + c^2 [+ v_{j-2} (nf T) + sum (nf FP64)];
  // writes [v_j (nf T)] + the sum (nf FP64, or nf T for the step's result)
  T* v1 = (m == 1 && !keep) ? nullptr : b.A;
  T* out1 = m == 1 ? b.B : nullptr;
  launch_term<T, K, BC, DIM>(op, g, (nf + 1) * pb + (v1 ? nf * pb : 0.0) + (m == 1 ? nf * pb : nf * pd), S, nullptr, v1, nullptr, m == 1 ? nullptr : b.C, out1, c, make_src<T>(op, q[0]));
  if (int32_t rc = check_launch("faber j=1")) return rc;
  if (int32_t rc = record(b.A, 1)) return rc;
  if (m == 1) {
    if (hipMemcpyAsync(S, b.B, ns * sizeof(T), hipMemcpyDeviceToDevice, op->stream) != hipSuccess)
      return fail(EXPW_EDEVICE, "faber: copy failed");
    return EXPW_OK;
  }
  // j = 2: v2 = F1 v1 - 2 c1 v0 into B (v0 = S read pointwise)
  c.first = 0;
  c.a_first = 0.0;
  c.cpp = 2.0 * el.c1;
  c.a_j = a[2];
  T* v2 = (m == 2 && !keep) ? nullptr : b.B;
  launch_term<T, K, BC, DIM>(op, g, (2 * nf + 1) * pb + nf * pd + (v2 ? nf * pb : 0.0) + (m == 2 ? nf * pb : nf * pd), b.A, S, v2, b.C, m == 2 ? nullptr : b.C, m == 2 ? S : nullptr, c, make_src<T>(op, q[1]));
  if (int32_t rc = check_launch("faber j=2")) return rc;
  if (int32_t rc = record(b.B, 2)) return rc;
  T* last = b.B;   // v_{j-1}
  T* older = b.A;  // v_{j-2}
  c.cpp = el.c1;
  for (int j = 3; j <= m; ++j) {
    c.a_j = a[j];
    const bool fin = (j == m);
    T* vj = (fin && !keep) ? nullptr : older;
    launch_term<T, K, BC, DIM>(op, g, (2 * nf + 1) * pb + nf * pd + (vj ? nf * pb : 0.0) + (fin ? nf * pb : nf * pd), last, older, vj, b.C, fin ? nullptr : b.C, fin ? S : nullptr, c, make_src<T>(op, q[j - 1]));
    if (int32_t rc = check_launch("faber term")) return rc;
    if (int32_t rc = record(older, j)) return rc;
    std::swap(last, older);
  }
  return EXPW_OK;
}

// Faber steps; term_traces (nullable) records every term at the receivers
// and then runs the terms one per sweep. big: the step's buffers
// (faber_big_bytes); a, q: host scratch of m + 1 and m doubles.
// a = the Faber coefficients a_0..a_m of the step (Sec. 3.2) for the working
// ellipse, from the operator's cache when the last step had the same
// ellipse, dt and m (m <= 1024).
inline void step_coefficients(expw_op* op, double gamma, double c0, double c1, double dt, int m, double* a) {
  if (m > 1024) {
    faber_coefficients(gamma, c0, c1, dt, m, a);
    return;
  }
  if (!(op->coef_m == m && op->coef_key[0] == gamma && op->coef_key[1] == c0 && op->coef_key[2] == c1 &&
        op->coef_key[3] == dt)) {
    faber_coefficients(gamma, c0, c1, dt, m, op->coef);
    op->coef_key[0] = gamma;
    op->coef_key[1] = c0;
    op->coef_key[2] = c1;
    op->coef_key[3] = dt;
    op->coef_m = m;
  }
  std::memcpy(a, op->coef, static_cast<size_t>(m + 1) * sizeof(double));
}

template <typename T, int K, int BC, int DIM>
int32_t faber_impl(expw_op* op, T* S, double t0, double dt, int m, int64_t nsteps, T* traces,
                   T* term_traces, char* big, double* a, double* q) {
  const Geo<T, K, DIM> g = make_geo<T, K, DIM>(op);
  const int64_t ns = (DIM + 1) * g.N;
  const FaberBufs<T> b = faber_bufs<T>(big, ns);
  double der[EXPW_MAX_TAYLOR], G[EXPW_MAX_TAYLOR];
  const WorkEllipse el(op);
  step_coefficients(op, el.gamma, el.c0, el.c1, dt, m, a);
  for (int j = 0; j < m; ++j) q[j] = 0.0;
  const int p = op->taylor_p;
  int fuse = fused_depth<T, K, BC, DIM>(op->fuse, m, g.N);
  if (K == 4 && DIM == 2 && BC == 0 && fuse > 1 &&
      (op->pass_kernel == EXPW_PASS_STREAMED ||
       (op->pass_kernel == EXPW_PASS_AUTO && stream2d_fits(g.n[0], g.n[1], 4, K)))) {
    // streamed passes of order 8: automatically four terms at FP32 (8192 x
    // 4096, m = 16: 163 against 116 G grid-pt matvecs/s for three; tiles stay
    // at three), at most three in FP64 (four spill)
    if (op->fuse == 0 && sizeof(T) == 4) fuse = std::min(4, m);
    if (sizeof(T) == 8 && fuse > 3) fuse = 3;
  }
  for (int64_t st = 0; st < nsteps; ++st) {
    const double t = t0 + st * dt;
    if (op->n_src > 0) {
      source_derivs(op, st, t, p, der);
      for (int c = 0; c < p; ++c) G[c] = der[p - 1 - c];
      faber_source_scalars(el.gamma, el.c0, el.c1, m, p, G, q);
      const double sc = src_scale(op);
      for (int j = 0; j < m; ++j) q[j] *= sc;
    }
    int32_t rc = EXPW_OK;
    T* term_out = term_traces ? term_traces + st * (m + 1) * op->n_rec : nullptr;
    // a remainder of one term after the fused passes: unfused final term
    auto final_term = [&](const T* vl, const T* vpv, const double* acc, T* out, int j) -> int32_t {
      FaberTerm c{};
      c.inv_gamma = 1.0 / el.gamma;
      c.c0 = el.c0;
      c.cpp = el.c1;
      c.a_j = a[j];
      launch_term<T, K, BC, DIM>(op, g, ((3.0 * (DIM + 1) + 1) * sizeof(T) + (DIM + 1) * sizeof(double)) * g.N, vl, vpv, nullptr, acc, nullptr, out, c, make_src<T>(op, q[j - 1]));
      return check_launch("faber final term");
    };
    const Src<T> src0 = make_src<T>(op, 0.0);
    bool recorded = false;  // by the last fused pass
    if (fuse > 1 && !term_out) {
      if constexpr (BC == 0 && DIM == 2) {
        rc = faber_fused_passes<T>(op->stream, ns, S, b, m, fuse, final_term,
            [&](int n, const T* vp, const T* vpp, const double* acc_in, T* ol, T* opv, double* acc_out, T* state_out, int j, bool first) {
              // the last pass (no terms kept) writes the step's result
              const RecRun<T> rr = state_out ? rec_run(op, traces, st) : RecRun<T>{nullptr, 0, 0};
              recorded = recorded || rr.out != nullptr;
              if constexpr (K == 2 || K == 4) {
                if (op->pass_kernel == EXPW_PASS_STREAMED ||
                    (op->pass_kernel == EXPW_PASS_AUTO && stream2d_fits(g.n[0], g.n[1], n, K)))
                  return launch_stream_pass<T, K>(n, op->stream, &op->prof, g, src0, vp, vpp, acc_in, ol, opv, acc_out, state_out, j, first, a, q, el.kappa, el.inv_ws, el.c0, el.c1, rr);
                return launch_pass<T, K>(n, op->stream, &op->prof, g, src0, vp, vpp, acc_in, ol, opv, acc_out, state_out, j, first, a, q, el.kappa, el.inv_ws, el.c0, el.c1, rr);
              } else
                return launch_pass<T, K>(n, op->stream, &op->prof, g, src0, vp, vpp, acc_in, ol, opv, acc_out, state_out, j, first, a, q, el.kappa, el.inv_ws, el.c0, el.c1, rr);
            });
      } else if constexpr (K == 2 && BC == 0 && DIM == 3 && sizeof(T) == 4) {
        rc = faber_fused_passes<T>(op->stream, ns, S, b, m, 2, final_term,
            [&](int n, const T* vp, const T* vpp, const double* acc_in, T* ol, T* opv, double* acc_out, T* state_out, int j, bool first) {
              (void)n;
              return launch_fused3d<T>(op->stream, &op->prof, g, src0, vp, vpp, acc_in, ol, opv, acc_out, state_out, j, first, a, q, el.kappa, el.inv_ws, el.c0, el.c1);
            });
      } else {
        rc = faber_unfused<T, K, BC, DIM>(op, g, el, S, b, a, q, m, term_out);
      }
    } else {
      rc = faber_unfused<T, K, BC, DIM>(op, g, el, S, b, a, q, m, term_out);
    }
    if (rc != EXPW_OK) return rc;
    if (!recorded && (rc = gather<T>(op, S, traces, st)) != EXPW_OK) return rc;
    if ((rc = guard_state<T>(op, S, (DIM + 1) * g.N)) != EXPW_OK) return rc;
  }
  return EXPW_OK;
}

// ---------------------------------------------------------------- RK4 and leap-frog

template <typename T, int K, int BC, int DIM>
int32_t rk4_impl(expw_op* op, T* S, double t0, double dt, int64_t nsteps, T* traces) {
  const Geo<T, K, DIM> g = make_geo<T, K, DIM>(op);
  const int64_t ns = (DIM + 1) * g.N;
  T* Abuf = reinterpret_cast<T*>(op->ws + op->off_big);
  T* Bbuf = Abuf + ns;
  T* Cbuf = Bbuf + ns;
  const unsigned grid = grid_for(g.N);
  const double sc = src_scale(op);
  const double nf = DIM + 1, pb = static_cast<double>(g.N) * sizeof(T);
  int64_t cur = 0;  // the step being taken
  double tn = t0;
  auto srcq = [&](double t) {
    if (op->n_src == 0) return make_src<T>(op, 0.0);
    return make_src<T>(op, source_value(op, cur, tn, t - tn) * sc);
  };
  const T h2 = static_cast<T>(0.5 * dt), h1 = static_cast<T>(dt), s6 = static_cast<T>(dt / 6.0),
          s3 = static_cast<T>(dt / 3.0);
  for (int64_t st = 0; st < nsteps; ++st) {
    const double t = t0 + st * dt;
    cur = st;
    tn = t;
    // words per point: stage 1 reads u (nf) + c^2, writes y, sum (2 nf); stages 2-3 read
    // y, u, sum (3 nf) + c^2, write y, sum (2 nf); stage 4 reads y, sum + c^2, writes u
    const RecRun<T> none{nullptr, 0, 0}, rr = rec_run(op, traces, st);
    launch_timed(&op->prof, op->stream, EXPW_KERNEL_RK4, (3 * nf + 1) * pb, k_rk4_stage<T, K, BC, DIM>, dim3(grid), dim3(kBlock), g, S, S, nullptr, Abuf, Cbuf, h2, s6, srcq(t), none);
    launch_timed(&op->prof, op->stream, EXPW_KERNEL_RK4, (5 * nf + 1) * pb, k_rk4_stage<T, K, BC, DIM>, dim3(grid), dim3(kBlock), g, Abuf, S, Cbuf, Bbuf, Cbuf, h2, s3, srcq(t + 0.5 * dt), none);
    launch_timed(&op->prof, op->stream, EXPW_KERNEL_RK4, (5 * nf + 1) * pb, k_rk4_stage<T, K, BC, DIM>, dim3(grid), dim3(kBlock), g, Bbuf, S, Cbuf, Abuf, Cbuf, h1, s3, srcq(t + 0.5 * dt), none);
    launch_timed(&op->prof, op->stream, EXPW_KERNEL_RK4, (3 * nf + 1) * pb, k_rk4_stage<T, K, BC, DIM>, dim3(grid), dim3(kBlock), g, Abuf, nullptr, Cbuf, nullptr, S, T(0), s6, srcq(t + dt), rr);
    int32_t rc = check_launch("rk4 stage");
    if (rc != EXPW_OK) return rc;
    if (!rr.out && (rc = gather<T>(op, S, traces, st)) != EXPW_OK) return rc;
    if ((rc = guard_state<T>(op, S, (DIM + 1) * g.N)) != EXPW_OK) return rc;
  }
  return EXPW_OK;
}

template <typename T, int K, int BC, int DIM>
int32_t leapfrog_impl(expw_op* op, T* S, double t0, double dt, int64_t nsteps, T* traces) {
  const Geo<T, K, DIM> g = make_geo<T, K, DIM>(op);
  const unsigned grid = grid_for(g.N);
  const double sc = src_scale(op);
  const double pb = static_cast<double>(g.N) * sizeof(T);
  for (int64_t st = 0; st < nsteps; ++st) {
    const double t = t0 + st * dt;
    // velocity: reads p and v (1 + d), writes v (d); pressure: reads p, v, c^2 (d + 2), writes p
    launch_timed(&op->prof, op->stream, EXPW_KERNEL_LEAPFROG_V, (1 + 2 * DIM) * pb, k_lf_v<T, K, BC, DIM>, dim3(grid), dim3(kBlock), g, S, static_cast<T>(dt));
    double q = 0.0;
    if (op->n_src > 0) q = dt * source_value(op, st, t, 0.5 * dt) * sc;
    const RecRun<T> rr = rec_run(op, traces, st);
    launch_timed(&op->prof, op->stream, EXPW_KERNEL_LEAPFROG_P, (DIM + 3) * pb, k_lf_p<T, K, BC, DIM>, dim3(grid), dim3(kBlock), g, S, static_cast<T>(dt), make_src<T>(op, q), rr);
    int32_t rc = check_launch("leapfrog");
    if (rc != EXPW_OK) return rc;
    if (!rr.out && (rc = gather<T>(op, S, traces, st)) != EXPW_OK) return rc;
    if ((rc = guard_state<T>(op, S, (DIM + 1) * g.N)) != EXPW_OK) return rc;
  }
  return EXPW_OK;
}

// ---------------------------------------------------------------- Krylov step

// Elements per thread of the persistent Arnoldi kernel for this problem (0 =
// use the launch-per-step path): every thread holds one or two grid points
// (three in 2D) with all their fields, so the grid points and the tail of the
// augmented vector must fit in that many points per thread over all
// co-resident blocks.
template <typename T, int K, int BC, int DIM>
int persistent_un(expw_op* op, int64_t naug) {
  if (!op->kry_persistent) return 0;
  if (op->coop_blocks == 0) {
    int dev = 0, coop = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void*>(k_arnoldi_persistent<T, K, BC, DIM, 2 * (DIM + 1)>), kArnNT, 0) !=
            hipSuccess ||
        !coop || per_cu < 1) {
      op->coop_blocks = -1;
    } else {
      op->coop_blocks = std::min(kArnMaxBlocks, cus * per_cu);
    }
  }
  if (op->coop_blocks <= 0) return 0;
  // one or two grid points per thread, with all their fields; the tail of
  // the augmented vector sits in pressure slots beyond the grid
  const int64_t threads = static_cast<int64_t>(op->coop_blocks) * kArnNT;
  const int64_t npt = npts(op->g);
  const int64_t ns = (DIM + 1) * npt;
  if (naug >= (int64_t(1) << 31)) return 0;
  for (int up : {1, 2, 3})
    if ((up < 3 || DIM == 2) && npt + (naug - ns) <= up * threads) return up * (DIM + 1);
  return 0;
}

template <typename T, int K, int BC, int DIM>
int32_t arnoldi_persistent(expw_op* op, int un, const Geo<T, K, DIM>& g, const T* S, T* Q,
                           const KrySrc& ks, const T* amp, int64_t ns, int64_t naug, int64_t ld,
                           int k, double tail2, double tol, unsigned long long* slots, int* err,
                           double* hess, double* sc, double* beta_out, bool full_last) {
  ArnArgs aa{};
  aa.full_last = full_last ? 1 : 0;
  aa.ns = ns;
  aa.naug = naug;
  aa.ld = ld;
  aa.k = k;
  aa.tail2 = tail2;
  aa.tol = tol;
  aa.nvmax = 2 * k;
  aa.spin_limit = 1u << 20;  // about a second of polling
  // the kernel leaves the area consistent for the next launch with the same
  // layout (nvmax); it is filled on first use and when the layout changes
  unsigned* seq_io = reinterpret_cast<unsigned*>(err) + 2;
  if (op->arn_nvmax_clean != aa.nvmax) {
    const int nslots = static_cast<int>(kArnRecWords) + kSlotBuffers * aa.nvmax * op->coop_blocks;
    k_fill_u64<<<(nslots + 255) / 256, 256, 0, op->stream>>>(slots, nslots, kSlotEmpty);
    // column flags and the launch epoch
    k_fill_u64<<<2, 256, 0, op->stream>>>(slots + kArnFlagWord, kArnMaxBlocks + 1, 0ull);
    k_zero_u32<<<1, 64, 0, op->stream>>>(seq_io, 1);
    op->arn_nvmax_clean = aa.nvmax;
  }
  Geo<T, K, DIM> gg = g;
  const T* Sp = S;
  T* Qp = Q;
  KrySrc kk = ks;
  const T* ap = amp;
  void* args[] = {&gg, &Sp, &Qp, &kk, &ap, &aa, &slots, &err, &seq_io, &hess, &sc, &beta_out};
  const void* fn = nullptr;
  if (un == DIM + 1) fn = reinterpret_cast<const void*>(k_arnoldi_persistent<T, K, BC, DIM, DIM + 1>);
  else if (un == 2 * (DIM + 1)) fn = reinterpret_cast<const void*>(k_arnoldi_persistent<T, K, BC, DIM, 2 * (DIM + 1)>);
  else if constexpr (DIM == 2) fn = reinterpret_cast<const void*>(k_arnoldi_persistent<T, K, BC, DIM, 9>);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const int slot = op->prof.acquire(EXPW_KERNEL_KRYLOV_ARNOLDI, &e0, &e1);
  if (slot >= 0) (void)hipEventRecord(e0, op->stream);
  const hipError_t e = hipLaunchCooperativeKernel(fn, dim3(op->coop_blocks), dim3(kArnNT), args, 0,
                                                  op->stream);
  if (slot >= 0) {
    (void)hipEventRecord(e1, op->stream);
    // reads S; per column: Q_j with its stencil and c^2, Q_1..Q_j; writes
    // Q_0..Q_{k-1} (the last column's vector is not orthogonalized or stored)
    const double es = sizeof(T);
    const double words = ns + naug + k * (naug + g.N) + (k - 1.0) * naug + naug * (k * (k - 1) / 2.0);
    op->prof.commit(slot, EXPW_KERNEL_KRYLOV_ARNOLDI, words * es);
  }
  if (e != hipSuccess) return fail(EXPW_EDEVICE, "persistent Arnoldi launch: %s", hipGetErrorString(e));
  return EXPW_OK;
}

// The Arnoldi process by launches: q_0 = x / beta, then per column j one
// matvec launch (fused with the first dot) and j + 1 fused MGS launches, and
// the norm of the last column. Forward (ADJ = false): H~ on x = [S; e_p]
// (naug entries, the source tail when ks.p > 0); ADJ: H^T on x = S (naug =
// ns). Writes Q_0..Q_k (leading dimension ld), the Hessenberg entries into
// hess (leading dimension kHessLd), beta into *beta_out and the column scales
// into sc.
template <typename T, int K, int BC, int DIM, bool ADJ>
int32_t arnoldi_launches(expw_op* op, const Geo<T, K, DIM>& g, const T* S, T* Q, int64_t ld, int64_t ns,
                         int64_t naug, const KrySrc& ks, const T* amp, int k, double tol, double* part,
                         double* hess, double* beta_out, double* sc) {
  const double es = sizeof(T);
  const unsigned rg_vec = red_grid_for(naug);
  const unsigned rg_pts = red_grid_for(ADJ ? g.N : g.N + ks.p);
  const double tail2 = (!ADJ && ks.p > 0) ? 1.0 : 0.0;
  double* P[2] = {part, part + kRedMaxBlocks};
  const unsigned nb_ns = red_grid_for(ns);
  launch_timed(&op->prof, op->stream, EXPW_KERNEL_KRYLOV_AUX, ns * es, k_norm2<T>, dim3(nb_ns), dim3(kBlock), S, ns, P[0]);
  launch_timed(&op->prof, op->stream, EXPW_KERNEL_KRYLOV_AUX, (ns + naug) * es, k_kry_init<T>, dim3(rg_vec), dim3(kBlock), S, ns, Q, naug, P[0], nb_ns, tail2, beta_out, sc);
  // Gram-Schmidt in three launches per column (gram.h): the block partials
  // and the Gram table use the grid-reduction area of the persistent kernel,
  // which is filled again before its next launch; the scaled projections go
  // to the y area of the small exponential (unused until the basis is done)
  double* gpart = reinterpret_cast<double*>(op->ws + op->off_bar);
  double* gram = gpart + kGramPartials;
  double* hs = reinterpret_cast<double*>(op->ws + op->off_kry);
  op->arn_nvmax_clean = 0;
  const unsigned gu = rg_vec;  // k_gram_update: its |w|^2 partials go to a reduction set (<= kRedMaxBlocks)
  // P[0]: the partials of |w|^2 of the previous column (nin blocks); the
  // matvec's partials of w . q_0 go to P[1] and are not used here
  int nin = 0;
  for (int j = 0; j < k; ++j) {
    T* w = Q + (j + 1) * ld;
    const double* pin = j == 0 ? nullptr : P[0];
    double* hst = j == 0 ? nullptr : hess + j * kHessLd + (j - 1);
    if constexpr (ADJ) {
      // reads Q_j (with the stencil), q_0 and c^2, writes w
      launch_timed(&op->prof, op->stream, EXPW_KERNEL_KRYLOV_MATVEC, (3.0 * ns + g.N) * es, k_kry_matvec_adj<T, K, BC, DIM>, dim3(rg_pts), dim3(kBlock), g, Q + j * ld, w, Q, pin, nin, tol, beta_out, hst, sc + j, P[1]);
    } else {
      // reads Q_j (with tail), q_1 and c^2, writes w
      launch_timed(&op->prof, op->stream, EXPW_KERNEL_KRYLOV_MATVEC, (3.0 * naug + g.N) * es, k_kry_matvec<T, K, BC, DIM>, dim3(rg_pts), dim3(kBlock), g, Q + j * ld, w, Q, ks, amp, pin, nin, tol, beta_out, hst, sc + j, P[1]);
    }
    // reads w and Q_0..Q_j
    const unsigned gd = gram_dots_grid(naug, j);
    launch_timed(&op->prof, op->stream, EXPW_KERNEL_KRYLOV_MGS, (j + 2.0) * naug * es, k_gram_dots<T>, dim3(gd), dim3(kBlock), static_cast<const T*>(w), static_cast<const T*>(Q), ld, naug, j, gpart);
    launch_timed(&op->prof, op->stream, EXPW_KERNEL_KRYLOV_MGS, 0.0, k_gram_reduce, dim3(2 * j + 1), dim3(kBlock), static_cast<const double*>(gpart), static_cast<int>(gd), 2 * j + 1, gram + kGramTot);
    launch_timed(&op->prof, op->stream, EXPW_KERNEL_KRYLOV_MGS, 0.0, k_gram_subst, dim3(1), dim3(64), static_cast<const double*>(gram + kGramTot), j, static_cast<const double*>(sc), gram, hess, kHessLd, hs);
    // reads w and Q_0..Q_j, writes w (Q_{j+1})
    launch_timed(&op->prof, op->stream, EXPW_KERNEL_KRYLOV_MGS, (j + 3.0) * naug * es, k_gram_update<T>, dim3(gu), dim3(kBlock), w, static_cast<const T*>(Q), ld, naug, j, static_cast<const double*>(hs), P[0]);
    nin = static_cast<int>(gu);
  }
  launch_timed(&op->prof, op->stream, EXPW_KERNEL_KRYLOV_AUX, 0.0, k_kry_finish, dim3(1), dim3(kBlock), P[0], nin, tol, beta_out, hess + k * kHessLd + (k - 1), sc + k);
  return check_launch(ADJ ? "adjoint arnoldi" : "arnoldi");
}

template <typename T, int K, int BC, int DIM>
int32_t krylov_impl(expw_op* op, T* S, double t0, double dt, int k, int64_t nsteps, T* traces) {
  const Geo<T, K, DIM> g = make_geo<T, K, DIM>(op);
  const int64_t ns = (DIM + 1) * g.N;
  const int p = op->n_src > 0 ? op->taylor_p : 0;
  const int64_t naug = ns + p;
  const int64_t ld = op->naug_pad;
  T* Q = reinterpret_cast<T*>(op->ws + op->off_big);
  double* part = reinterpret_cast<double*>(op->ws + op->off_part);
  double* scal = reinterpret_cast<double*>(op->ws + op->off_scal);
  double* hess = reinterpret_cast<double*>(op->ws + op->off_hess);
  const T* amp = reinterpret_cast<const T*>(op->ws + op->off_src_amp);
  const double es = sizeof(T);
  double* kry_y = reinterpret_cast<double*>(op->ws + op->off_kry);
  double* kry_sc = kry_y + 64;
  int* kry_keff = reinterpret_cast<int*>(op->ws + op->off_kry + 136 * sizeof(double));
  unsigned long long* kry_slots = reinterpret_cast<unsigned long long*>(op->ws + op->off_bar);
  int* kry_err = kry_keff + 8;
  const int unp = persistent_un<T, K, BC, DIM>(op, naug);
  const double tol = 1e-14;
  // the a-posteriori estimate needs h_{k,k-1} and phi_1(dt H_k) e_1: the last
  // column is completed and the small exponential runs on the host
  const bool est_on = op->kry_estimate;
  op->last_est = 0.0;
  op->last_est_valid = est_on;
  std::vector<double> hh((EXPW_MAX_KRYLOV + 1) * kHessLd), hk(k * k), E(k * k), der(EXPW_MAX_TAYLOR);
  std::vector<double> scal_h(2);
  KrySrc ks{};
  ks.n = op->n_src;
  ks.p = p;
  ks.lo = op->src_lo;
  ks.hi = op->src_hi;
  ks.idx = reinterpret_cast<const int64_t*>(op->ws + op->off_src_idx);
  for (int64_t st = 0; st < nsteps; ++st) {
    const double t = t0 + st * dt;
    if (p > 0) {
      source_derivs(op, st, t, p, der.data());
      const double sc = src_scale(op);
      for (int c = 0; c < p; ++c) ks.G[c] = der[p - 1 - c] * sc;
    }
    if (unp > 0) {
      // the whole Arnoldi process in one cooperative launch
      int32_t rc = arnoldi_persistent<T, K, BC, DIM>(op, unp, g, S, Q, ks, amp, ns, naug, ld, k,
                                                     p > 0 ? 1.0 : 0.0, tol, kry_slots, kry_err,
                                                     hess, kry_sc, scal + 1, est_on);
      if (rc != EXPW_OK) return rc;
    } else {
      int32_t rc = arnoldi_launches<T, K, BC, DIM, false>(op, g, S, Q, ld, ns, naug, ks, amp, k, tol, part, hess, scal + 1, kry_sc);
      if (rc != EXPW_OK) return rc;
    }
    int32_t rc = check_launch("arnoldi");
    if (rc != EXPW_OK) return rc;
    RecRun<T> rr{nullptr, 0, 0};  // set when the combination records the receivers
    if (op->kry_mode == EXPW_EXPM_DEVICE && !est_on) {
      // y = exp(dt H_k) e_1 and the combination without leaving the device
      launch_timed(&op->prof, op->stream, EXPW_KERNEL_KRYLOV_AUX, 0.0, expm_kernel(k), dim3(1), dim3(expm_threads(k)), hess, k, dt, tol, scal + 1, kry_y, kry_keff);
      rr = rec_run(op, traces, st);
      launch_timed(&op->prof, op->stream, EXPW_KERNEL_KRYLOV_AUX, (k + 1.0) * ns * es, k_kry_combine_dev<T>, dim3(red_grid_for(ns)), dim3(kBlock), S, Q, ld, ns, kry_y, kry_keff, scal + 1, kry_sc, rr);
      op->last_keff = -1;  // on the device; read by expw_krylov_info
      if ((rc = check_launch("krylov exponential")) != EXPW_OK) return rc;
    } else {
      // the small Hessenberg exponential on the host (one sync per step)
      if (hipMemcpyAsync(hh.data(), hess, hh.size() * sizeof(double), hipMemcpyDeviceToHost, op->stream) != hipSuccess ||
          hipMemcpyAsync(scal_h.data(), scal, 2 * sizeof(double), hipMemcpyDeviceToHost, op->stream) != hipSuccess ||
          hipStreamSynchronize(op->stream) != hipSuccess)
        return fail(EXPW_EDEVICE, "krylov: device to host copy failed: %s", hipGetErrorString(hipGetLastError()));
      const double beta = scal_h[1];
      int keff = k;
      // columns 0..k-2: a breakdown in the last column gives keff = k anyway,
      // and the persistent Arnoldi kernel does not produce h_{k,k-1}
      for (int j = 0; j + 1 < k; ++j)
        if (!(hh[(j + 1) * kHessLd + j] > tol * beta)) {
          keff = j + 1;
          break;
        }
      op->last_beta = beta;
      if (beta == 0.0) {
        op->last_keff = 0;
        // zero state and no source: the state stays zero
      } else {
        op->last_keff = keff;
        // only the upper Hessenberg part is written by the kernels; with the
        // estimate, exp([[dt H_k, e_1], [0, 0]]) gives exp(dt H_k) e_1 (first
        // column) and phi_1(dt H_k) e_1 (last column)
        const bool est_here = est_on && keff == k;
        const int nz = est_here ? k + 1 : keff;
        hk.assign(static_cast<size_t>(nz) * nz, 0.0);
        E.resize(static_cast<size_t>(nz) * nz);
        for (int r = 0; r < keff; ++r)
          for (int c = 0; c < keff; ++c) hk[r * nz + c] = (r <= c + 1) ? dt * hh[r * kHessLd + c] : 0.0;
        if (est_here) hk[0 * nz + k] = 1.0;
        if (!expm(nz, hk.data(), E.data())) return fail(EXPW_ENONFINITE, "krylov: non-finite Hessenberg matrix");
        KryCoef y{};
        for (int r = 0; r < keff; ++r) y.y[r] = E[r * nz + 0];
        if (est_here)
          op->last_est = std::max(op->last_est, dt * beta * hh[k * kHessLd + (k - 1)] * std::fabs(E[(k - 1) * nz + k]));
        launch_timed(&op->prof, op->stream, EXPW_KERNEL_KRYLOV_AUX, (keff + 1.0) * ns * es, k_kry_combine<T>, dim3(red_grid_for(ns)), dim3(kBlock), S, Q, ld, ns, keff, y, beta, kry_sc);
        if ((rc = check_launch("krylov combine")) != EXPW_OK) return rc;
      }
    }
    if (!rr.out && (rc = gather<T>(op, S, traces, st)) != EXPW_OK) return rc;
    if ((rc = guard_state<T>(op, S, (DIM + 1) * g.N)) != EXPW_OK) return rc;
  }
  return EXPW_OK;
}

template <typename T, int K, int BC, int DIM>
int32_t apply_impl(expw_op* op, const T* x, T* y) {
  const Geo<T, K, DIM> g = make_geo<T, K, DIM>(op);
  k_apply<T, K, BC, DIM><<<grid_for(g.N), kBlock, 0, op->stream>>>(g, x, y);
  return check_launch("apply");
}

template <typename T, int K, int BC, int DIM>
int32_t apply_adjoint_impl(expw_op* op, const T* x, T* y) {
  const Geo<T, K, DIM> g = make_geo<T, K, DIM>(op);
  k_apply_adjoint<T, K, BC, DIM><<<grid_for(g.N), kBlock, 0, op->stream>>>(g, x, y);
  return check_launch("apply adjoint");
}

// Adjoint of one Faber step from t (the same ellipse, coefficients and source
// scalars as the forward step): recomputes v_1..v_{m-1} into terms, then runs
// the transposed recurrence with three rotating workspace vectors, adding the
// c^2 gradient into grad; lam becomes mu_0 in place.
template <typename T, int K, int BC, int DIM>
int32_t faber_adjoint_impl(expw_op* op, const T* U, T* lam, double t, double dt, int m, T* grad,
                           T* terms) {
  const Geo<T, K, DIM> g = make_geo<T, K, DIM>(op);
  const int64_t ns = (DIM + 1) * g.N;
  const unsigned grid = grid_for(g.N);
  const WorkEllipse el(op);
  std::vector<double> a(m + 1), q(m, 0.0), der(EXPW_MAX_TAYLOR), G(EXPW_MAX_TAYLOR);
  step_coefficients(op, el.gamma, el.c0, el.c1, dt, m, a.data());
  const int p = op->taylor_p;
  if (op->n_src > 0) {
    source_derivs(op, 0, t, p, der.data());  // a table's row 0: one step per call
    for (int c = 0; c < p; ++c) G[c] = der[p - 1 - c];
    faber_source_scalars(el.gamma, el.c0, el.c1, m, p, G.data(), q.data());
    const double sc = src_scale(op);
    for (int j = 0; j < m; ++j) q[j] *= sc;
  }
  auto v = [&](int j) -> const T* { return j == 0 ? U : terms + (j - 1) * ns; };
  // forward: v_j = F1 v_{j-1} - c_j v_{j-2} + source, j = 1..m-1; on 2D
  // zero-ghost grids in tiled passes of several terms that store every term
  // (each pass reads its v_{j-1}, v_{j-2} from the terms already stored), a
  // remaining single term one per sweep
  int done = 0;
  if constexpr (DIM == 2 && BC == 0 && (K == 2 || K == 4)) {
    const int fz = fused_depth<T, K, BC, DIM>(op->fuse, m - 1, g.N);
    if (fz > 1) {
      const Src<T> src0 = make_src<T>(op, 0.0);
      int j = 1;
      while (m - j >= 2) {
        const int n = std::min(fz, m - j);
        if (int32_t rc = launch_pass<T, K>(n, op->stream, &op->prof, g, src0, v(j - 1), j > 1 ? v(j - 2) : nullptr,
                                           nullptr, nullptr, nullptr, nullptr, nullptr, j, j == 1, a.data(),
                                           q.data(), el.kappa, el.inv_ws, el.c0, el.c1, RecRun<T>{nullptr, 0, 0},
                                           terms))
          return rc;
        if (int32_t rc = check_launch("adjoint: forward passes")) return rc;
        j += n;
      }
      done = j - 1;
    }
  }
  FaberTerm f{};
  f.inv_gamma = 1.0 / el.gamma;
  f.c0 = el.c0;
  const double nf = DIM + 1, pb = static_cast<double>(g.N) * sizeof(T);
  for (int j = done + 1; j < m; ++j) {
    f.cpp = j == 1 ? 0.0 : (j == 2 ? 2.0 * el.c1 : el.c1);
    launch_timed(&op->prof, op->stream, EXPW_KERNEL_FABER, (nf + 1 + (j > 1 ? nf : 0) + nf) * pb,
                 k_faber_term<T, K, BC, DIM>, dim3(grid), dim3(kBlock), g, v(j - 1),
                 j > 1 ? v(j - 2) : nullptr, terms + (j - 1) * ns, nullptr, nullptr, nullptr, f,
                 make_src<T>(op, q[j - 1]));
    if (int32_t rc = check_launch("adjoint: forward terms")) return rc;
  }
  // reverse: mu_j for j = m..0 (mu_j into buffer j mod 4, mu_0 into lam); on
  // 2D zero-ghost grids two terms per launch while j - 1 >= 1 (unless one
  // term per sweep is asked for), the rest one per launch
  T* mbuf[4] = {reinterpret_cast<T*>(op->ws + op->off_big), nullptr, nullptr, nullptr};
  for (int i = 1; i < 4; ++i) mbuf[i] = mbuf[i - 1] + ns;
  auto cc = [&](int j) { return j < 2 ? 0.0 : (j == 2 ? 2.0 * el.c1 : el.c1); };
  auto term_coef = [&](int j) {
    AdjointTerm c{};
    c.inv_gamma = f.inv_gamma;
    c.c0 = f.c0;
    c.a_j = a[j];
    c.cnext = cc(j + 2);
    return c;
  };
  int j = m;
  if constexpr (DIM == 2 && BC == 0) {
    if (op->fuse != 1) {
      const int tiles_x = static_cast<int>((g.n[0] + kAdjTX - 1) / kAdjTX);
      const int64_t blocks = static_cast<int64_t>(tiles_x) * ((g.n[1] + kAdjTZ - 1) / kAdjTZ);
      for (; j >= 2; j -= 2) {
        const T* mu1 = j + 1 <= m ? mbuf[(j + 1) % 4] : nullptr;
        const T* mu2 = j + 2 <= m ? mbuf[(j + 2) % 4] : nullptr;
        // reads lam, mu1 (+ c^2), mu2, v_{j-1}, v_{j-2} (velocities), grad;
        // writes mu_j, mu_{j-1}, grad
        const double words = 3 * nf + (mu1 ? nf : 0) + 1 + (mu2 ? nf : 0) + 2 * DIM + 2;
        launch_timed(&op->prof, op->stream, EXPW_KERNEL_FABER, words * pb, k_faber_adjoint_pair<T, K>,
                     dim3(static_cast<unsigned>(blocks)), dim3(kAdjNT), g, mu1, mu2, static_cast<const T*>(lam),
                     v(j - 1), v(j - 2), mbuf[j % 4], mbuf[(j - 1) % 4], grad, term_coef(j), term_coef(j - 1),
                     tiles_x);
        if (int32_t rc = check_launch("adjoint term pair")) return rc;
      }
    }
  }
  for (; j >= 0; --j) {
    const AdjointTerm c = term_coef(j);
    const T* mu1 = j + 1 <= m ? mbuf[(j + 1) % 4] : nullptr;
    const T* mu2 = j + 2 <= m ? mbuf[(j + 2) % 4] : nullptr;
    T* out = j == 0 ? lam : mbuf[j % 4];
    // reads lam, mu1 (+ c^2 with the stencil), mu2, v_{j-1}; writes mu_j, grad RMW
    const double words = nf + (mu1 ? nf + 1 : 0) + (mu2 ? nf : 0) + nf + (j > 0 ? DIM + 2 : 0);
    launch_timed(&op->prof, op->stream, EXPW_KERNEL_FABER, words * pb,
                 k_faber_adjoint_term<T, K, BC, DIM>, dim3(grid), dim3(kBlock), g, mu1, mu2,
                 static_cast<const T*>(lam), j > 0 ? v(j - 1) : nullptr, out,
                 j > 0 ? grad : nullptr, c);
    if (int32_t rc = check_launch("adjoint term")) return rc;
  }
  return EXPW_OK;
}

// Reverse of one Krylov step of dimension k from t (see adjoint.h): the
// forward basis V of the step (the op's Krylov workspace) and the basis W of
// H^T from lam (caller scratch Wb of k + 1 state vectors); on the host, one
// exponential of the block triangular matrix [[dt G_k, e_1 e_1^T], [0, dt
// H_k^T]] gives exp(dt G_k) e_1 (its first column, upper left block) and the
// coupling C (upper right block); then lam = beta' W exp(dt G_k) e_1 and the
// gradient kernel.
template <typename T, int K, int BC, int DIM>
int32_t krylov_adjoint_impl(expw_op* op, const T* U, T* lam, double t, double dt, int k, T* grad, T* Wb) {
  const Geo<T, K, DIM> g = make_geo<T, K, DIM>(op);
  const int64_t ns = (DIM + 1) * g.N;
  const int p = op->n_src > 0 ? op->taylor_p : 0;
  const int64_t naug = ns + p;
  const int64_t ld = op->naug_pad;
  T* Q = reinterpret_cast<T*>(op->ws + op->off_big);
  double* part = reinterpret_cast<double*>(op->ws + op->off_part);
  double* scal = reinterpret_cast<double*>(op->ws + op->off_scal);
  double* hess = reinterpret_cast<double*>(op->ws + op->off_hess);
  const T* amp = reinterpret_cast<const T*>(op->ws + op->off_src_amp);
  double* kry_sc = reinterpret_cast<double*>(op->ws + op->off_kry) + 64;
  const double tol = 1e-14;
  KrySrc ks{};
  ks.n = op->n_src;
  ks.p = p;
  ks.lo = op->src_lo;
  ks.hi = op->src_hi;
  ks.idx = reinterpret_cast<const int64_t*>(op->ws + op->off_src_idx);
  if (p > 0) {
    std::vector<double> der(EXPW_MAX_TAYLOR);
    source_derivs(op, 0, t, p, der.data());  // a table's row 0: one step per call
    const double sc = src_scale(op);
    for (int c = 0; c < p; ++c) ks.G[c] = der[p - 1 - c] * sc;
  }
  struct Basis {
    std::vector<double> h, s;
    double beta = 0.0;
    int keff = 0;
  };
  auto fetch = [&](Basis& b) -> int32_t {
    b.h.resize((EXPW_MAX_KRYLOV + 1) * kHessLd);
    b.s.resize(k + 1);
    if (hipMemcpyAsync(b.h.data(), hess, b.h.size() * sizeof(double), hipMemcpyDeviceToHost, op->stream) != hipSuccess ||
        hipMemcpyAsync(b.s.data(), kry_sc, (k + 1) * sizeof(double), hipMemcpyDeviceToHost, op->stream) != hipSuccess ||
        hipMemcpyAsync(&b.beta, scal + 1, sizeof(double), hipMemcpyDeviceToHost, op->stream) != hipSuccess ||
        hipStreamSynchronize(op->stream) != hipSuccess)
      return fail(EXPW_EDEVICE, "krylov adjoint: device to host copy failed: %s", hipGetErrorString(hipGetLastError()));
    // the breakdown rule of the forward step
    b.keff = b.beta == 0.0 ? 0 : k;
    for (int j = 0; b.keff > 0 && j + 1 < k; ++j)
      if (!(b.h[(j + 1) * kHessLd + j] > tol * b.beta)) {
        b.keff = j + 1;
        break;
      }
    return EXPW_OK;
  };
  Basis bv, bw;
  int32_t rc = arnoldi_launches<T, K, BC, DIM, false>(op, g, U, Q, ld, ns, naug, ks, amp, k, tol, part, hess, scal + 1, kry_sc);
  if (rc == EXPW_OK) rc = fetch(bv);
  if (rc == EXPW_OK) rc = arnoldi_launches<T, K, BC, DIM, true>(op, g, lam, Wb, ns, ns, ns, ks, amp, k, tol, part, hess, scal + 1, kry_sc);
  if (rc == EXPW_OK) rc = fetch(bw);
  if (rc != EXPW_OK) return rc;
  const int kv = bv.keff, kw = bw.keff;
  if (kw == 0) return EXPW_OK;  // lam = 0 stays 0 and adds nothing
  const int n = kw + kv;
  std::vector<double> Z(static_cast<size_t>(n) * n, 0.0), E(static_cast<size_t>(n) * n);
  for (int r = 0; r < kw; ++r)
    for (int c = 0; c < kw; ++c) Z[r * n + c] = (r <= c + 1) ? dt * bw.h[r * kHessLd + c] : 0.0;
  if (kv > 0) {
    Z[0 * n + kw] = 1.0;
    for (int r = 0; r < kv; ++r)
      for (int c = 0; c < kv; ++c) Z[(kw + r) * n + kw + c] = (c <= r + 1) ? dt * bv.h[c * kHessLd + r] : 0.0;
  }
  if (!expm(n, Z.data(), E.data())) return fail(EXPW_ENONFINITE, "krylov adjoint: non-finite Hessenberg matrix");
  const double es = sizeof(T);
  if (kv > 0) {
    // M_ab = beta beta' C_ab s^W_a s^V_b for the unnormalized columns
    std::vector<double> M(static_cast<size_t>(kw) * kv);
    for (int a = 0; a < kw; ++a)
      for (int b = 0; b < kv; ++b)
        M[a * kv + b] = bv.beta * bw.beta * E[a * n + kw + b] * bw.s[a] * bv.s[b];
    if (hipMemcpyAsync(hess, M.data(), M.size() * sizeof(double), hipMemcpyHostToDevice, op->stream) != hipSuccess)
      return fail(EXPW_EDEVICE, "krylov adjoint: host to device copy failed");
    // reads kv velocity columns (with the stencil), kw pressure columns, grad RMW
    launch_timed(&op->prof, op->stream, EXPW_KERNEL_KRYLOV_AUX, (kv * DIM + kw + 2.0) * g.N * es,
                 k_kry_grad<T, K, BC, DIM>, dim3(grid_for(g.N)), dim3(kBlock), g, static_cast<const T*>(Q), ld, kv,
                 static_cast<const T*>(Wb), ns, kw, static_cast<const double*>(hess), -dt, grad);
    if ((rc = check_launch("krylov adjoint gradient")) != EXPW_OK) return rc;
  }
  KryCoef y{};
  for (int a = 0; a < kw; ++a) y.y[a] = E[a * n + 0];
  // kry_sc holds the scales of W (the last Arnoldi process)
  launch_timed(&op->prof, op->stream, EXPW_KERNEL_KRYLOV_AUX, (kw + 1.0) * ns * es, k_kry_combine<T>,
               dim3(red_grid_for(ns)), dim3(kBlock), lam, static_cast<const T*>(Wb), ns, ns, kw, y, bw.beta,
               static_cast<const double*>(kry_sc));
  if ((rc = check_launch("krylov adjoint combine")) != EXPW_OK) return rc;
  // M lives in host memory until the copy has run
  if (hipStreamSynchronize(op->stream) != hipSuccess)
    return fail(EXPW_EDEVICE, "krylov adjoint: %s", hipGetErrorString(hipGetLastError()));
  return EXPW_OK;
}

template <typename T, int K, int DIM>
size_t batch_table_bytes(int n) {
  size_t b = align_up(n * sizeof(BatchShot<T, K, DIM>)) + 2 * align_up((n + 1) * sizeof(int64_t));
  if (K == 2 && DIM == 2)
    b += align_up(n * sizeof(FusedShot<T>)) + align_up((n + 1) * sizeof(int64_t)) + align_up(sizeof(BatchSync)) +
         align_up(static_cast<size_t>(n) * kBatchMaxM * sizeof(double));
  return b + align_up(sizeof(BatchClock));
}

template <typename T, int K, int BC, int DIM>
int32_t batch_create_impl(expw_op* const* ops, int n, const int32_t* m, const double* dt,
                          void* const* states, void* const* traces, expw_batch* b) {
  using Shot = BatchShot<T, K, DIM>;
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return m[x] > m[y]; });
  // plain bytes: the descriptors are filled field by field and copied as bytes
  std::vector<unsigned char> bytes(n * sizeof(Shot), 0);
  Shot* host = reinterpret_cast<Shot*>(bytes.data());
  std::vector<int64_t> prefix(n + 1, 0), prefix_rec(n + 1, 0);
  for (int r = 0; r < n; ++r) {
    const int i = order[r];
    expw_op* op = ops[i];
    Shot& sh = host[r];
    const Geo<T, K, DIM> geo = make_geo<T, K, DIM>(op);
    std::memcpy(static_cast<void*>(&sh.g), &geo, sizeof(geo));
    const int64_t ns = (DIM + 1) * sh.g.N;
    sh.S = static_cast<T*>(states[i]);
    const FaberBufs<T> fb = faber_bufs<T>(op->ws + op->off_big, ns);
    sh.A = fb.A;
    sh.B = fb.B;
    sh.C = fb.C;
    sh.m = m[i];
    sh.dt = dt[i];
    const WorkEllipse el(op);
    sh.inv_gamma = 1.0 / el.gamma;
    sh.c0 = el.c0;
    sh.c1 = el.c1;
    sh.kappa = el.kappa;
    sh.inv_ws = el.inv_ws;
    faber_coefficients(el.gamma, el.c0, el.c1, dt[i], m[i], sh.a);
    if (op->n_src > 0) {
      sh.n_src = op->n_src;
      sh.p = op->taylor_p;
      sh.src_lo = op->src_lo;
      sh.src_hi = op->src_hi;
      sh.src_idx = reinterpret_cast<const int64_t*>(op->ws + op->off_src_idx);
      sh.src_amp = reinterpret_cast<const T*>(op->ws + op->off_src_amp);
      sh.f_peak = op->f_peak;
      sh.t_delay = op->t_delay;
      // tail projections: the source scalar is linear in the derivative vector G
      std::vector<double> e(sh.p), qc(m[i]);
      const double sc = src_scale(op);
      for (int c = 0; c < sh.p; ++c) {
        std::fill(e.begin(), e.end(), 0.0);
        e[c] = 1.0;
        faber_source_scalars(el.gamma, el.c0, el.c1, m[i], sh.p, e.data(), qc.data());
        for (int j = 0; j < m[i]; ++j) sh.qtab[j][c] = qc[j] * sc;
      }
    }
    sh.n_rec = op->n_rec;
    sh.rec = op->rec_dev;
    sh.traces = (traces && traces[i] && op->n_rec > 0) ? static_cast<T*>(traces[i]) : nullptr;
    prefix[r + 1] = prefix[r] + (sh.g.N + kBlock - 1) / kBlock;
    prefix_rec[r + 1] = prefix_rec[r] + (sh.traces ? sh.n_rec : 0);
  }
  if (prefix[n] > INT32_MAX) return fail(EXPW_EUNSUPPORTED, "batch too large for one launch");
  char* t = static_cast<char*>(b->table);
  b->off_prefix = align_up(n * sizeof(Shot));
  b->off_prefix_rec = b->off_prefix + align_up((n + 1) * sizeof(int64_t));
  if (hipMemcpyAsync(t, bytes.data(), n * sizeof(Shot), hipMemcpyHostToDevice, b->stream) != hipSuccess ||
      hipMemcpyAsync(t + b->off_prefix, prefix.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, b->stream) != hipSuccess ||
      hipMemcpyAsync(t + b->off_prefix_rec, prefix_rec.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, b->stream) != hipSuccess ||
      hipStreamSynchronize(b->stream) != hipSuccess)
    return fail(EXPW_EDEVICE, "batch table upload failed");
  b->max_m = m[order[0]];
  b->count_ge.assign(b->max_m + 1, 0);
  for (int r = 0; r < n; ++r)
    for (int j = 1; j <= host[r].m; ++j) b->count_ge[j]++;
  b->prefix = prefix;
  b->rec_items = prefix_rec[n];
  b->fused = false;
  if constexpr (K == 2 && BC == 0 && DIM == 2) {
    bool ok = true;
    for (int r = 0; r < n; ++r) ok = ok && 3 * host[r].g.N < (int64_t(1) << 31);
    // passes of the depth set on shot 0's operator (expw_set_tuning or the
    // autotuner), rounded to 2, 4 or 6 terms (4 at most in FP64); default 6
    // in FP32 (two workgroups per CU fit the tiles' LDS), 4 in FP64
    const int req = ops[0]->fuse;
    int depth = req == 0 ? (sizeof(T) == 4 ? 6 : kBatchFuse) : (req <= 2 ? 2 : (req <= 4 ? 4 : 6));
    if (sizeof(T) == 8 && depth > 4) depth = 4;
    b->depth = depth;
    if (ok) {
      const int S = depth;
      const int TX = depth == 2 ? FusedTile<2>::TX : (depth == 4 ? FusedTile<4>::TX : FusedTile<6>::TX);
      const int TY = depth == 2 ? FusedTile<2>::TY : (depth == 4 ? FusedTile<4>::TY : FusedTile<6>::TY);
      std::vector<unsigned char> fb(n * sizeof(FusedShot<T>), 0);
      auto* fs = reinterpret_cast<FusedShot<T>*>(fb.data());
      std::vector<int64_t> fprefix(n + 1, 0);
      b->copy_dst.clear();
      b->copy_src.clear();
      b->copy_elems.clear();
      b->max_passes = 0;
      for (int r = 0; r < n; ++r) {
        const Shot& h = host[r];
        FusedShot<T>& f = fs[r];
        std::memcpy(static_cast<void*>(&f.g), &h.g, sizeof(h.g));
        const int64_t ns = 3 * h.g.N;
        f.S = h.S;
        f.A = h.A;
        f.B = h.B;
        f.C = h.C;
        f.D = h.B + ns;
        f.E = f.D + ns;
        f.m = h.m;
        f.tiles_x = static_cast<int32_t>((h.g.n[0] + TX - 1) / TX);
        f.tiles_y = static_cast<int32_t>((h.g.n[1] + TY - 1) / TY);
        f.n_src = h.n_src;
        f.p = h.p;
        f.src_lo = h.src_lo;
        f.src_hi = h.src_hi;
        f.src_idx = h.src_idx;
        f.src_amp = h.src_amp;
        f.f_peak = h.f_peak;
        f.t_delay = h.t_delay;
        f.dt = h.dt;
        f.kappa = h.kappa;
        f.inv_ws = h.inv_ws;
        f.c0 = h.c0;
        f.c1 = h.c1;
        std::memcpy(f.a, h.a, sizeof(h.a));
        for (int j = 0; j <= kBatchMaxM; ++j)
          f.cpp[j] = static_cast<T>(j <= 1 ? 0.0 : (j == 2 ? 2.0 * h.c1 : h.c1));
        std::memcpy(f.qtab, h.qtab, sizeof(h.qtab));
        fprefix[r + 1] = fprefix[r] + static_cast<int64_t>(f.tiles_x) * f.tiles_y;
        const int passes = (h.m + S - 1) / S;
        b->max_passes = std::max(b->max_passes, passes);
        if (passes == 1) {
          b->copy_dst.push_back(h.S);
          b->copy_src.push_back(h.A);
          b->copy_elems.push_back(ns);
        }
      }
      b->count_pass.assign(b->max_passes, 0);
      for (int r = 0; r < n; ++r)
        for (int p = 0; p < (host[r].m + S - 1) / S; ++p) b->count_pass[p]++;
      b->off_fshots = b->off_prefix_rec + align_up((n + 1) * sizeof(int64_t));
      b->off_fprefix = b->off_fshots + align_up(n * sizeof(FusedShot<T>));
      b->off_sync = b->off_fprefix + align_up((n + 1) * sizeof(int64_t));
      b->off_qstep = b->off_sync + align_up(sizeof(BatchSync));
      if (fprefix[n] > INT32_MAX) return fail(EXPW_EUNSUPPORTED, "batch too large for one launch");
      if (hipMemcpyAsync(t + b->off_fshots, fb.data(), fb.size(), hipMemcpyHostToDevice, b->stream) != hipSuccess ||
          hipMemcpyAsync(t + b->off_fprefix, fprefix.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, b->stream) != hipSuccess ||
          hipStreamSynchronize(b->stream) != hipSuccess)
        return fail(EXPW_EDEVICE, "batch table upload failed");
      b->fprefix = fprefix;
      b->fused = true;
    }
  }
  b->off_clock = batch_table_bytes<T, K, DIM>(n) - align_up(sizeof(BatchClock));
  return EXPW_OK;
}

// Enqueues steps st = 0..count-1 of the batch (times and trace rows from the
// clock in the table).
template <typename T, int K, int BC, int DIM>
int32_t batch_enqueue(expw_batch* b, int64_t count, bool capturing) {
  using Shot = BatchShot<T, K, DIM>;
  char* t = static_cast<char*>(b->table);
  const Shot* shots = reinterpret_cast<const Shot*>(t);
  const int64_t* prefix = reinterpret_cast<const int64_t*>(t + b->off_prefix);
  const int64_t* prefix_rec = reinterpret_cast<const int64_t*>(t + b->off_prefix_rec);
  const BatchClock* clk = reinterpret_cast<const BatchClock*>(t + b->off_clock);
  for (int64_t st = 0; st < count; ++st) {
    bool done = false;
    if constexpr (K == 2 && BC == 0 && DIM == 2) {
      if (b->fused && b->persistent && !capturing) {
        const auto* fshots = reinterpret_cast<const FusedShot<T>*>(t + b->off_fshots);
        const auto* fprefix = reinterpret_cast<const int64_t*>(t + b->off_fprefix);
        BatchSync* bs = reinterpret_cast<BatchSync*>(t + b->off_sync);
        BatchPersist pa{};
        for (int p = 0; p < b->max_passes; ++p) pa.count_pass[p] = b->count_pass[p];
        pa.max_passes = b->max_passes;
        pa.n_shots = b->n;
        pa.any_single = b->copy_dst.empty() ? 0 : 1;
        pa.spin_limit = 1u << 22;  // polls of about 0.1 us: far longer than any pass
        const Shot* shp = shots;
        const FusedShot<T>* fsp = fshots;
        const int64_t* fpp = fprefix;
        const int64_t* prp = prefix_rec;
        const BatchClock* ckp = clk;
        int64_t stv = st;
        T* qsp = reinterpret_cast<T*>(t + b->off_qstep);
        void* args[] = {&fsp, &fpp, &shp, &prp, &pa, &ckp, &stv, &bs, &qsp};
        const void* fn = b->depth == 2 ? reinterpret_cast<const void*>(k_faber_batch_persistent<T, 2>)
                         : b->depth == 4 ? reinterpret_cast<const void*>(k_faber_batch_persistent<T, 4>)
                                         : reinterpret_cast<const void*>(k_faber_batch_persistent<T, 6>);
        if (hipLaunchCooperativeKernel(fn, dim3(b->coop_blocks), dim3(kFusedNT), args, 0, b->stream) != hipSuccess)
          return fail(EXPW_EDEVICE, "batch: persistent launch failed: %s", hipGetErrorString(hipGetLastError()));
        continue;
      }
      if (b->fused) {
        const auto* fshots = reinterpret_cast<const FusedShot<T>*>(t + b->off_fshots);
        const auto* fprefix = reinterpret_cast<const int64_t*>(t + b->off_fprefix);
        T* qstep = reinterpret_cast<T*>(t + b->off_qstep);
        k_batch_source_q<T><<<(b->n + 63) / 64, 64, 0, b->stream>>>(fshots, b->n, clk, st, qstep);
        if (int32_t rc = check_launch("batch source scalars")) return rc;
        for (int p = 0; p < b->max_passes; ++p) {
          const int np = b->count_pass[p];
          const unsigned grid = static_cast<unsigned>(b->fprefix[np]);
          if (b->depth == 2)
            k_faber_fused2d_batch<T, 2><<<grid, kFusedNT, 0, b->stream>>>(fshots, fprefix, np, p, qstep);
          else if (b->depth == 4)
            k_faber_fused2d_batch<T, 4><<<grid, kFusedNT, 0, b->stream>>>(fshots, fprefix, np, p, qstep);
          else
            k_faber_fused2d_batch<T, 6><<<grid, kFusedNT, 0, b->stream>>>(fshots, fprefix, np, p, qstep);
          if (int32_t rc = check_launch("batch fused pass")) return rc;
        }
        for (size_t i = 0; i < b->copy_dst.size(); ++i) {
          const unsigned g = static_cast<unsigned>(std::min<int64_t>(4096, (b->copy_elems[i] + kBlock - 1) / kBlock));
          k_batch_copy<T><<<g, kBlock, 0, b->stream>>>(static_cast<T*>(b->copy_dst[i]), static_cast<const T*>(b->copy_src[i]), b->copy_elems[i]);
          if (int32_t rc = check_launch("batch copy")) return rc;
        }
        done = true;
      }
    }
    if (!done) {
      for (int j = 1; j <= b->max_m; ++j) {
        const int np = b->count_ge[j];
        const unsigned grid = static_cast<unsigned>(b->prefix[np]);
        k_faber_batch_term<T, K, BC, DIM><<<grid, kBlock, 0, b->stream>>>(shots, prefix, np, j, clk, st);
        if (int32_t rc = check_launch("batch term")) return rc;
      }
    }
    if (b->rec_items > 0) {
      k_batch_gather<T, K, DIM><<<grid_for(b->rec_items), kBlock, 0, b->stream>>>(shots, prefix_rec, b->n, clk, st);
      if (int32_t rc = check_launch("batch gather")) return rc;
    }
  }
  return EXPW_OK;
}

template <typename T, int K, int BC, int DIM>
int32_t batch_step_impl(expw_batch* b, double t0, int64_t nsteps, int64_t step0) {
  BatchClock* clk = reinterpret_cast<BatchClock*>(static_cast<char*>(b->table) + b->off_clock);
  const bool persistent = b->fused && b->persistent;
  BatchSync* bs = reinterpret_cast<BatchSync*>(static_cast<char*>(b->table) + b->off_sync);
  if (persistent) {
    // a clean barrier (also after a failed call) and no error
    k_zero_u32<<<1, 64, 0, b->stream>>>(reinterpret_cast<unsigned*>(bs), 4);
    if (int32_t rc = check_launch("batch barrier reset")) return rc;
  }
  int64_t done = 0;
  while (done < nsteps) {
    const bool use_graph = b->gexec && nsteps - done >= b->graph_steps;
    const int64_t count = use_graph ? b->graph_steps : nsteps - done;
    k_batch_set_clock<<<1, 1, 0, b->stream>>>(clk, t0, step0 + done, step0 + done);
    if (int32_t rc = check_launch("batch clock")) return rc;
    if (use_graph) {
      if (hipGraphLaunch(b->gexec, b->stream) != hipSuccess) return fail(EXPW_EDEVICE, "batch graph launch failed");
    } else if (int32_t rc = batch_enqueue<T, K, BC, DIM>(b, count, false)) {
      return rc;
    }
    done += count;
  }
  if (persistent) {
    int err = 0;
    if (hipMemcpyAsync(&err, &bs->err, sizeof(int), hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess)
      return fail(EXPW_EDEVICE, "batch: %s", hipGetErrorString(hipGetLastError()));
    if (err) return fail(EXPW_EDEVICE, "batch: a grid-wide barrier of the persistent step timed out");
  }
  return EXPW_OK;
}

// The Faber buffers of expw_step_faber_noalloc: one static device array per
// GPU (every code object load gets its own), shared by all calls on that GPU.
// Host code must not use the array's name as a device address; its address
// on each device is taken once with hipGetSymbolAddress while that device is
// current (noalloc_scratch_on) and used from then on.
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];
static_assert(kNoallocScratchBytes == static_cast<size_t>(EXPW_NOALLOC_SCRATCH_BYTES),
              "the header states the scratch size");

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
char* g_scratch_ptr[kMaxDevices] = {};

// The static scratch's device address on the current device (nullptr and a
// message on failure).
char* noalloc_scratch_on_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch_ptr[dev] = static_cast<char*>(p);
  }
  return g_scratch_ptr[dev];
}

// Set by an atexit handler registered at the first handle creation. Handles
// destroyed after exit() has begun (by a later atexit handler or a static
// destructor) skip their HIP calls: the runtime may already be gone, and the
// process is about to release every device resource anyway.
std::atomic<bool> g_exiting{false};

void note_exit() { g_exiting.store(true); }

void watch_exit() {
  static const bool registered = (std::atexit(note_exit), true);
  (void)registered;
}

bool runtime_usable() { return !g_exiting.load(); }

void batch_drop_graph(expw_batch* b) {
  if (!runtime_usable()) {
    b->gexec = nullptr;
    b->graph = nullptr;
    b->graph_steps = 0;
    return;
  }
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
  b->graph_steps = 0;
}

template <class Fn>
int32_t dispatch_batch(const expw_batch* b, Fn&& fn) {
  expw_op probe{};
  probe.g = b->g;
  probe.K = b->K;
  return dispatch(&probe, fn);
}

int32_t check_op(const expw_op* op) {
  if (!op) return fail(EXPW_EINVAL, "op is NULL");
  return EXPW_OK;
}

int32_t check_step_args(const expw_op* op, const void* state, double dt, int64_t nsteps) {
  if (int32_t rc = check_op(op)) return rc;
  if (!state) return fail(EXPW_EINVAL, "state is NULL");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(EXPW_EINVAL, "dt must be positive and finite");
  if (nsteps < 0) return fail(EXPW_EINVAL, "nsteps must be >= 0");
  return check_source_rows(op, nsteps);
}

}  // namespace
}  // namespace expw

using namespace expw;

extern "C" {

int32_t expw_workspace_size(const expw_grid* g, int32_t max_k, int32_t max_p, size_t* bytes) {
  if (int32_t rc = validate_grid(g)) return rc;
  if (max_k < 0 || max_k > EXPW_MAX_KRYLOV) return fail(EXPW_EINVAL, "max_krylov_k must be in [0, %d]", EXPW_MAX_KRYLOV);
  if (max_p < 0 || max_p > EXPW_MAX_TAYLOR) return fail(EXPW_EINVAL, "max_taylor_p must be in [0, %d]", EXPW_MAX_TAYLOR);
  if (!bytes) return fail(EXPW_EINVAL, "bytes is NULL");
  *bytes = layout(*g, max_k, max_p).total;
  return EXPW_OK;
}

int32_t expw_op_create(const expw_grid* g, const void* c2_dev, int32_t max_k, int32_t max_p,
                       void* ws, size_t ws_bytes, void* stream, expw_op** out) {
  return expw_op_create_profiles(g, c2_dev, nullptr, max_k, max_p, ws, ws_bytes, stream, out);
}

int32_t expw_op_create_profiles(const expw_grid* g, const void* c2_dev,
                                const double* const* sigma_host, int32_t max_k, int32_t max_p,
                                void* ws, size_t ws_bytes, void* stream, expw_op** out) {
  clear_error();
  size_t need = 0;
  if (int32_t rc = expw_workspace_size(g, max_k, max_p, &need)) return rc;
  if (!out) return fail(EXPW_EINVAL, "out is NULL");
  if (!c2_dev) return fail(EXPW_EINVAL, "c2_dev is NULL");
  if (!ws) return fail(EXPW_EINVAL, "workspace_dev is NULL");
  if (ws_bytes < need) return fail(EXPW_ENOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0) return fail(EXPW_EINVAL, "workspace must be 256-byte aligned");
  // the damping profiles: the caller's, or the quadratic layer of the grid
  std::vector<double> profiles[3][2];
  for (int a = 0; a < g->ndim; ++a)
    for (int hf = 0; hf < 2; ++hf) {
      std::vector<double>& prof = profiles[a][hf];
      prof.resize(g->n[a]);
      if (sigma_host) {
        const double* src = sigma_host[2 * a + hf];
        if (!src) return fail(EXPW_EINVAL, "sigma_host[%d] is NULL", 2 * a + hf);
        for (int64_t i = 0; i < g->n[a]; ++i) {
          if (!(src[i] >= 0.0) || !std::isfinite(src[i]))
            return fail(EXPW_EINVAL, "sigma_host[%d][%lld] must be finite and >= 0", 2 * a + hf,
                        static_cast<long long>(i));
          if (g->bc == EXPW_BC_PERIODIC && src[i] != 0.0)
            return fail(EXPW_EINVAL, "damping profiles must be zero with periodic ghosts");
          prof[i] = src[i];
        }
      } else {
        damping_profile(g->n[a], g->h, g->abc_cells, g->sigma_max, hf == 1, prof.data());
      }
    }
  watch_exit();
  expw_op* op = new expw_op();
  op->g = *g;
  stagger_weights(g->order, op->alpha, &op->K);
  op->c2 = c2_dev;
  op->ws = static_cast<char*>(ws);
  op->ws_bytes = ws_bytes;
  op->stream = static_cast<hipStream_t>(stream);
  op->kmax = max_k;
  op->pmax = max_p;
  const Layout L = layout(*g, max_k, max_p);
  std::memcpy(op->off_sig, L.sig, sizeof(L.sig));
  op->off_src_idx = L.src_idx;
  op->off_src_amp = L.src_amp;
  op->off_part = L.part;
  op->off_scal = L.scal;
  op->off_hess = L.hess;
  op->off_kry = L.kry;
  op->off_bar = L.bar;
  op->off_big = L.big;
  op->naug_pad = L.naug_pad;
  op->n_src = 0;
  op->src_table = 0;
  op->src_nrows = 0;
  op->guard = 0;
  op->n_rec = 0;
  op->rec_dev = nullptr;
  op->rec_run_first = -1;
  op->taylor_p = std::max(1, std::min(8, max_p));
  op->fuse = 0;
  op->pass_kernel = EXPW_PASS_AUTO;
  op->kry_mode = EXPW_EXPM_DEVICE;
  op->kry_persistent = 1;
  op->coop_blocks = 0;
  op->arn_nvmax_clean = 0;
  op->last_keff = 0;
  op->last_beta = 0.0;
  op->kry_estimate = false;
  op->last_est_valid = false;
  op->last_est = 0.0;
  // the allocation-free Faber entry point's buffers on this device (resolved
  // here, once per device, with the device current)
  op->noalloc_scratch = noalloc_scratch_on_current_device();

  // damping profiles (FP64 on the host, stored in the grid dtype)
  std::vector<std::vector<char>> staging;
  const size_t es = elem_size(*g);
  for (int a = 0; a < g->ndim; ++a)
    for (int hf = 0; hf < 2; ++hf) {
      const std::vector<double>& prof = profiles[a][hf];
      std::vector<char> buf(g->n[a] * es);
      for (int64_t i = 0; i < g->n[a]; ++i) {
        if (g->dtype == EXPW_F32) reinterpret_cast<float*>(buf.data())[i] = static_cast<float>(prof[i]);
        else reinterpret_cast<double*>(buf.data())[i] = prof[i];
      }
      if (hipMemcpyAsync(op->ws + L.sig[a][hf], buf.data(), buf.size(), hipMemcpyHostToDevice,
                         op->stream) != hipSuccess) {
        delete op;
        return fail(EXPW_EDEVICE, "expw_op_create: profile upload failed");
      }
      staging.push_back(std::move(buf));
    }
  k_zero_u32<<<1, 64, 0, op->stream>>>(reinterpret_cast<unsigned*>(op->ws + L.kry + 136 * sizeof(double)), 64);
  double* part = reinterpret_cast<double*>(op->ws + L.part);
  const int64_t N = npts(*g);
  const unsigned nb = red_grid_for(N);
  if (g->dtype == EXPW_F32)
    k_c2_max<float><<<nb, kBlock, 0, op->stream>>>(static_cast<const float*>(c2_dev), N, part);
  else
    k_c2_max<double><<<nb, kBlock, 0, op->stream>>>(static_cast<const double*>(c2_dev), N, part);
  std::vector<double> parts(nb);
  hipError_t e = hipMemcpyAsync(parts.data(), part, nb * sizeof(double), hipMemcpyDeviceToHost, op->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(op->stream);
  if (e != hipSuccess || hipGetLastError() != hipSuccess) {
    delete op;
    return fail(EXPW_EDEVICE, "expw_op_create: device error: %s", hipGetErrorString(e));
  }
  double c2max = -INFINITY;
  for (double v : parts) c2max = std::fmax(c2max, v);
  if (!std::isfinite(c2max)) {
    delete op;
    return fail(EXPW_ENONFINITE, "c2 holds a non-finite or non-positive value");
  }
  op->c2max = c2max;
  const double* prof_ptrs[6] = {};
  for (int a = 0; a < g->ndim; ++a)
    for (int hf = 0; hf < 2; ++hf) prof_ptrs[2 * a + hf] = profiles[a][hf].data();
  expw_spectrum_rectangle_profiles(g, c2max, prof_ptrs, &op->x_lo, &op->B);
  expw_ellipse(op->x_lo, op->B, &op->gamma, &op->c0, &op->c1);
  *out = op;
  return EXPW_OK;
}

int32_t expw_op_destroy(expw_op* op) {
  if (op && runtime_usable()) op->prof.release();
  delete op;
  return EXPW_OK;
}

int32_t expw_set_stream(expw_op* op, void* stream) {
  if (int32_t rc = check_op(op)) return rc;
  op->stream = static_cast<hipStream_t>(stream);
  return EXPW_OK;
}

int32_t expw_get_spectrum(const expw_op* op, double* x_lo, double* B) {
  if (int32_t rc = check_op(op)) return rc;
  if (!x_lo || !B) return fail(EXPW_EINVAL, "NULL output");
  *x_lo = op->x_lo;
  *B = op->B;
  return EXPW_OK;
}

int32_t expw_get_ellipse(const expw_op* op, double* gamma, double* c0, double* c1) {
  if (int32_t rc = check_op(op)) return rc;
  if (!gamma || !c0 || !c1) return fail(EXPW_EINVAL, "NULL output");
  *gamma = op->gamma;
  *c0 = op->c0;
  *c1 = op->c1;
  return EXPW_OK;
}

int32_t expw_set_ellipse(expw_op* op, double gamma, double c0, double c1) {
  if (int32_t rc = check_op(op)) return rc;
  if (!(gamma > 0.0) || !std::isfinite(gamma) || !std::isfinite(c0) || !(std::fabs(c1) <= 1.0))
    return fail(EXPW_EINVAL, "ellipse needs gamma > 0 and |c1| < 1");
  op->gamma = gamma;
  op->c0 = c0;
  op->c1 = c1;
  return EXPW_OK;
}

int32_t expw_set_tuning(expw_op* op, int32_t fuse) {
  if (int32_t rc = check_op(op)) return rc;
  if (fuse < 0 || fuse > kMaxFuse) return fail(EXPW_EINVAL, "fuse must be in [0, %d]", kMaxFuse);
  op->fuse = fuse;
  return EXPW_OK;
}

int32_t expw_set_pass_kernel(expw_op* op, int32_t kind) {
  if (int32_t rc = check_op(op)) return rc;
  if (kind < EXPW_PASS_AUTO || kind > EXPW_PASS_STREAMED)
    return fail(EXPW_EINVAL, "pass kernel must be 0 (automatic), 1 (tiled) or 2 (streamed)");
  op->pass_kernel = kind;
  return EXPW_OK;
}

int32_t expw_apply(expw_op* op, const void* x, void* y) {
  if (int32_t rc = check_op(op)) return rc;
  if (!x || !y) return fail(EXPW_EINVAL, "NULL vector");
  if (x == y) return fail(EXPW_EINVAL, "x and y must not alias");
  return dispatch(op, [&](auto cfg) {
    using C = decltype(cfg);
    using T = typename C::type;
    return apply_impl<T, C::k, C::bc, C::dim>(op, static_cast<const T*>(x), static_cast<T*>(y));
  });
}

int32_t expw_apply_adjoint(expw_op* op, const void* x, void* y) {
  if (int32_t rc = check_op(op)) return rc;
  if (!x || !y) return fail(EXPW_EINVAL, "NULL vector");
  if (x == y) return fail(EXPW_EINVAL, "x and y must not alias");
  return dispatch(op, [&](auto cfg) {
    using C = decltype(cfg);
    using T = typename C::type;
    return apply_adjoint_impl<T, C::k, C::bc, C::dim>(op, static_cast<const T*>(x), static_cast<T*>(y));
  });
}

int32_t expw_faber_adjoint_step(expw_op* op, const void* u, void* lam, double t, double dt,
                                int32_t m, void* grad, void* terms) {
  if (int32_t rc = check_step_args(op, u, dt, 1)) return rc;
  if (m < 1 || m > 1024) return fail(EXPW_EINVAL, "Faber degree m must be in [1, 1024]");
  if (!lam || !grad) return fail(EXPW_EINVAL, "NULL lam or grad");
  if (m > 1 && !terms) return fail(EXPW_EINVAL, "terms is NULL (m - 1 state vectors needed)");
  if (lam == u || lam == grad) return fail(EXPW_EINVAL, "lam must not alias u or grad");
  return dispatch(op, [&](auto cfg) {
    using C = decltype(cfg);
    using T = typename C::type;
    return faber_adjoint_impl<T, C::k, C::bc, C::dim>(op, static_cast<const T*>(u), static_cast<T*>(lam), t, dt, m, static_cast<T*>(grad), static_cast<T*>(terms));
  });
}

int32_t expw_krylov_adjoint_step(expw_op* op, const void* u, void* lam, double t, double dt,
                                 int32_t k, void* grad, void* basis) {
  if (int32_t rc = check_step_args(op, u, dt, 1)) return rc;
  if (k < 1 || k > op->kmax) return fail(EXPW_EINVAL, "Krylov dimension k must be in [1, %d] (max_krylov_k at create)", op->kmax);
  if (!lam || !grad || !basis) return fail(EXPW_EINVAL, "NULL lam, grad or basis");
  if (lam == u || lam == grad || basis == u || basis == lam || basis == grad)
    return fail(EXPW_EINVAL, "lam, grad and basis must not alias each other or u");
  return dispatch(op, [&](auto cfg) {
    using C = decltype(cfg);
    using T = typename C::type;
    return krylov_adjoint_impl<T, C::k, C::bc, C::dim>(op, static_cast<const T*>(u), static_cast<T*>(lam), t, dt, k, static_cast<T*>(grad), static_cast<T*>(basis));
  });
}

int32_t expw_inject_receivers(expw_op* op, const void* values, double scale, void* state) {
  if (int32_t rc = check_op(op)) return rc;
  if (op->n_rec == 0) return fail(EXPW_EINVAL, "no receivers set");
  if (!values || !state) return fail(EXPW_EINVAL, "NULL array");
  const unsigned grid = grid_for(op->n_rec);
  if (op->g.dtype == EXPW_F32)
    k_scatter_add<float><<<grid, kBlock, 0, op->stream>>>(static_cast<const float*>(values), op->rec_dev, op->n_rec, static_cast<float>(scale), static_cast<float*>(state));
  else
    k_scatter_add<double><<<grid, kBlock, 0, op->stream>>>(static_cast<const double*>(values), op->rec_dev, op->n_rec, scale, static_cast<double*>(state));
  return check_launch("inject receivers");
}

int32_t expw_batch_table_bytes(int32_t n_ops, const expw_grid* g, size_t* bytes) {
  if (int32_t rc = validate_grid(g)) return rc;
  if (n_ops < 1 || !bytes) return fail(EXPW_EINVAL, "n_ops must be >= 1 and bytes non-NULL");
  expw_op probe{};
  probe.g = *g;
  probe.K = g->order / 2;
  const int64_t n = n_ops;
  return dispatch(&probe, [&](auto cfg) {
    using C = decltype(cfg);
    *bytes = batch_table_bytes<typename C::type, C::k, C::dim>(static_cast<int>(n));
    return EXPW_OK;
  });
}

int32_t expw_batch_create(expw_op* const* ops, int32_t n_ops, const int32_t* m, const double* dt,
                          void* const* states_dev, void* const* traces_dev, void* table_dev,
                          size_t table_bytes, void* stream, expw_batch** out) {
  if (!out) return fail(EXPW_EINVAL, "out is NULL");
  *out = nullptr;
  if (!ops || n_ops < 1 || !m || !dt || !states_dev || !table_dev)
    return fail(EXPW_EINVAL, "NULL argument or n_ops < 1");
  for (int i = 0; i < n_ops; ++i) {
    if (!ops[i] || !states_dev[i]) return fail(EXPW_EINVAL, "shot %d: NULL operator or state", i);
    const expw_grid& g0 = ops[0]->g;
    const expw_grid& gi = ops[i]->g;
    if (gi.dtype != g0.dtype || gi.ndim != g0.ndim || gi.order != g0.order || gi.bc != g0.bc)
      return fail(EXPW_EINVAL, "shot %d: dtype, ndim, order and bc must match shot 0", i);
    if (m[i] < 2 || m[i] > kBatchMaxM) return fail(EXPW_EINVAL, "shot %d: degree must be in [2, %d]", i, kBatchMaxM);
    if (ops[i]->n_src > 0 && ops[i]->src_table)
      return fail(EXPW_EUNSUPPORTED, "shot %d: batches form the Ricker wavelet on the device; a tabulated source is not supported", i);
    if (!(dt[i] > 0.0) || !std::isfinite(dt[i])) return fail(EXPW_EINVAL, "shot %d: dt must be positive", i);
    for (int k = 0; k < i; ++k)
      if (ops[k] == ops[i] || states_dev[k] == states_dev[i])
        return fail(EXPW_EINVAL, "shots %d and %d share an operator or a state", k, i);
  }
  size_t need = 0;
  if (int32_t rc = expw_batch_table_bytes(n_ops, &ops[0]->g, &need)) return rc;
  if (table_bytes < need) return fail(EXPW_EINVAL, "batch table too small (%zu < %zu bytes)", table_bytes, need);
  if (reinterpret_cast<uintptr_t>(table_dev) % kAlign) return fail(EXPW_EINVAL, "batch table must be 256-byte aligned");
  watch_exit();
  auto* b = new (std::nothrow) expw_batch();
  if (!b) return fail(EXPW_ENOMEM, "out of host memory");
  b->n = n_ops;
  b->g = ops[0]->g;
  b->K = ops[0]->K;
  b->stream = static_cast<hipStream_t>(stream);
  b->table = table_dev;
  const int32_t rc = dispatch_batch(b, [&](auto cfg) {
    using C = decltype(cfg);
    return batch_create_impl<typename C::type, C::k, C::bc, C::dim>(ops, n_ops, m, dt, states_dev, traces_dev, b);
  });
  if (rc != EXPW_OK) {
    delete b;
    return rc;
  }
  *out = b;
  return EXPW_OK;
}

int32_t expw_batch_step_faber(expw_batch* b, double t0, int64_t nsteps, int64_t step0) {
  if (!b) return fail(EXPW_EINVAL, "batch is NULL");
  if (nsteps < 0 || step0 < 0) return fail(EXPW_EINVAL, "nsteps and step0 must be >= 0");
  return dispatch_batch(b, [&](auto cfg) {
    using C = decltype(cfg);
    return batch_step_impl<typename C::type, C::k, C::bc, C::dim>(b, t0, nsteps, step0);
  });
}

int32_t expw_batch_capture(expw_batch* b, int64_t nsteps) {
  if (!b) return fail(EXPW_EINVAL, "batch is NULL");
  if (nsteps < 0) return fail(EXPW_EINVAL, "nsteps must be >= 0");
  batch_drop_graph(b);
  if (nsteps == 0) return EXPW_OK;
  if (!b->stream) return fail(EXPW_EINVAL, "capture needs a non-default stream (expw_batch_create)");
  if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return fail(EXPW_EDEVICE, "batch: stream capture could not start");
  int32_t rc = dispatch_batch(b, [&](auto cfg) {
    using C = decltype(cfg);
    return batch_enqueue<typename C::type, C::k, C::bc, C::dim>(b, nsteps, true);
  });
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->stream, &g);
  if (rc != EXPW_OK || e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return rc != EXPW_OK ? rc : fail(EXPW_EDEVICE, "batch: stream capture failed");
  }
  hipGraphExec_t x = nullptr;
  if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(EXPW_EDEVICE, "batch: graph instantiation failed");
  }
  b->graph = g;
  b->gexec = x;
  b->graph_steps = nsteps;
  return EXPW_OK;
}

int32_t expw_batch_set_persistent(expw_batch* b, int32_t on) {
  if (!b) return fail(EXPW_EINVAL, "batch is NULL");
  if (!on) {
    b->persistent = false;
    return EXPW_OK;
  }
  if (!b->fused) return fail(EXPW_EUNSUPPORTED, "persistent batches need 2D order-4 shots with zero ghosts");
  if (b->coop_blocks == 0) {
    int dev = 0, coop = 0, cus = 0, per_cu = 0;
    const void* fn = nullptr;
    const bool f32 = b->g.dtype == EXPW_F32;
    if (b->depth == 2) fn = f32 ? reinterpret_cast<const void*>(k_faber_batch_persistent<float, 2>) : reinterpret_cast<const void*>(k_faber_batch_persistent<double, 2>);
    else if (b->depth == 4) fn = f32 ? reinterpret_cast<const void*>(k_faber_batch_persistent<float, 4>) : reinterpret_cast<const void*>(k_faber_batch_persistent<double, 4>);
    else fn = f32 ? reinterpret_cast<const void*>(k_faber_batch_persistent<float, 6>) : reinterpret_cast<const void*>(k_faber_batch_persistent<double, 6>);
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kFusedNT, 0) != hipSuccess || !coop || per_cu < 1) {
      b->coop_blocks = -1;
    } else {
      const int64_t tiles0 = b->fprefix[b->count_pass[0]];
      b->coop_blocks = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(static_cast<int64_t>(cus) * per_cu, tiles0)));
    }
  }
  if (b->coop_blocks < 0) return fail(EXPW_EUNSUPPORTED, "cooperative launches are not available");
  b->persistent = true;
  return EXPW_OK;
}

int32_t expw_batch_destroy(expw_batch* b) {
  if (b) batch_drop_graph(b);
  delete b;
  return EXPW_OK;
}

int32_t expw_set_source_ricker(expw_op* op, int32_t n_src, const int64_t* idx, const double* amp,
                               double f_peak, double t_delay, int32_t taylor_p) {
  if (int32_t rc = check_op(op)) return rc;
  if (n_src < 0 || n_src > EXPW_MAX_SOURCES) return fail(EXPW_EINVAL, "n_src must be in [0, %d]", EXPW_MAX_SOURCES);
  if (n_src == 0) {
    op->n_src = 0;
    return EXPW_OK;
  }
  if (!idx || !amp) return fail(EXPW_EINVAL, "NULL source arrays");
  if (!(f_peak > 0.0) || !std::isfinite(f_peak) || !std::isfinite(t_delay)) return fail(EXPW_EINVAL, "f_peak must be > 0");
  if (taylor_p < 1 || taylor_p > op->pmax) return fail(EXPW_EINVAL, "taylor_p must be in [1, %d] (max_taylor_p at create)", op->pmax);
  const int64_t N = npts(op->g);
  for (int s = 0; s < n_src; ++s) {
    if (idx[s] < 0 || idx[s] >= N) return fail(EXPW_EINVAL, "source %d index %lld out of range", s, (long long)idx[s]);
    if (!std::isfinite(amp[s])) return fail(EXPW_EINVAL, "source %d amplitude not finite", s);
  }
  op->src_idx.assign(idx, idx + n_src);
  op->src_amp.assign(amp, amp + n_src);
  std::vector<char> ampbuf(n_src * elem_size(op->g));
  for (int s = 0; s < n_src; ++s) {
    if (op->g.dtype == EXPW_F32) reinterpret_cast<float*>(ampbuf.data())[s] = static_cast<float>(amp[s]);
    else reinterpret_cast<double*>(ampbuf.data())[s] = amp[s];
  }
  if (hipMemcpyAsync(op->ws + op->off_src_idx, op->src_idx.data(), n_src * sizeof(int64_t),
                     hipMemcpyHostToDevice, op->stream) != hipSuccess ||
      hipMemcpyAsync(op->ws + op->off_src_amp, ampbuf.data(), ampbuf.size(), hipMemcpyHostToDevice,
                     op->stream) != hipSuccess ||
      hipStreamSynchronize(op->stream) != hipSuccess)
    return fail(EXPW_EDEVICE, "source upload failed");
  op->n_src = n_src;
  op->src_lo = *std::min_element(op->src_idx.begin(), op->src_idx.end());
  op->src_hi = *std::max_element(op->src_idx.begin(), op->src_idx.end());
  op->f_peak = f_peak;
  op->t_delay = t_delay;
  op->taylor_p = taylor_p;
  op->src_table = 0;
  return EXPW_OK;
}

int32_t expw_set_guard(expw_op* op, int32_t on) {
  if (int32_t rc = check_op(op)) return rc;
  op->guard = on != 0;
  return EXPW_OK;
}

int32_t expw_set_source_taylor(expw_op* op, int32_t n_src, const int64_t* idx, const double* amp,
                               int32_t taylor_p, int64_t nsteps, const double* gder) {
  if (int32_t rc = check_op(op)) return rc;
  if (n_src > 0) {
    if (nsteps < 1) return fail(EXPW_EINVAL, "nsteps must be >= 1");
    if (!gder) return fail(EXPW_EINVAL, "gder is NULL");
    if (taylor_p < 1 || taylor_p > op->pmax)
      return fail(EXPW_EINVAL, "taylor_p must be in [1, %d] (max_taylor_p at create)", op->pmax);
    for (int64_t i = 0; i < nsteps * taylor_p; ++i)
      if (!std::isfinite(gder[i])) return fail(EXPW_EINVAL, "gder[%lld] is not finite", (long long)i);
  }
  // the points and amplitudes as for the Ricker source (its checks and upload)
  if (int32_t rc = expw_set_source_ricker(op, n_src, idx, amp, 1.0, 0.0, n_src > 0 ? taylor_p : 1)) return rc;
  if (n_src == 0) return EXPW_OK;
  op->src_rows.assign(gder, gder + nsteps * taylor_p);
  op->src_nrows = nsteps;
  op->src_table = 1;
  return EXPW_OK;
}

int32_t expw_set_receivers(expw_op* op, int32_t n_rec, const int64_t* idx_dev) {
  if (int32_t rc = check_op(op)) return rc;
  if (n_rec < 0) return fail(EXPW_EINVAL, "n_rec must be >= 0");
  if (n_rec == 0) {
    op->n_rec = 0;
    op->rec_dev = nullptr;
    op->rec_run_first = -1;
    return EXPW_OK;
  }
  if (!idx_dev) return fail(EXPW_EINVAL, "NULL receiver array");
  std::vector<int64_t> h(n_rec);
  if (hipMemcpyAsync(h.data(), idx_dev, n_rec * sizeof(int64_t), hipMemcpyDeviceToHost, op->stream) != hipSuccess ||
      hipStreamSynchronize(op->stream) != hipSuccess)
    return fail(EXPW_EDEVICE, "receiver index read failed");
  const int64_t N = npts(op->g);
  bool run = true;
  for (int r = 0; r < n_rec; ++r) {
    if (h[r] < 0 || h[r] >= N) return fail(EXPW_EINVAL, "receiver %d index %lld out of range", r, (long long)h[r]);
    run = run && h[r] == h[0] + r;
  }
  op->n_rec = n_rec;
  op->rec_dev = idx_dev;
  op->rec_run_first = run ? h[0] : -1;
  return EXPW_OK;
}

int32_t expw_step_faber(expw_op* op, void* state, double t0, double dt, int32_t m, int64_t nsteps,
                        void* traces) {
  if (int32_t rc = check_step_args(op, state, dt, nsteps)) return rc;
  if (m < 1 || m > 1024) return fail(EXPW_EINVAL, "Faber degree m must be in [1, 1024]");
  return dispatch(op, [&](auto cfg) {
    using C = decltype(cfg);
    using T = typename C::type;
    std::vector<double> a(m + 1), q(m);
    return faber_impl<T, C::k, C::bc, C::dim>(op, static_cast<T*>(state), t0, dt, m, nsteps, static_cast<T*>(traces), nullptr, op->ws + op->off_big, a.data(), q.data());
  });
}

int32_t expw_autotune(expw_op* op, int32_t m, double dt, void* scratch, const char* cache_path,
                      int32_t* fuse_out, int32_t* pass_kernel_out, double* ms_out) {
  if (int32_t rc = check_step_args(op, scratch, dt, 1)) return rc;
  if (m < 1 || m > 1024) return fail(EXPW_EINVAL, "Faber degree m must be in [1, 1024]");
  // the key: device (architecture and compute units) and layout
  int dev = 0;
  hipDeviceProp_t prop{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return fail(EXPW_EDEVICE, "autotune: device query failed");
  const expw_grid& g = op->g;
  char key[256];
  std::snprintf(key, sizeof key, "expw-autotune-v1 %s %d %d %lldx%lldx%lld %s %d %d %d", prop.gcnArchName,
                prop.multiProcessorCount, g.ndim, static_cast<long long>(g.n[0]),
                static_cast<long long>(g.ndim > 1 ? g.n[1] : 1), static_cast<long long>(g.ndim > 2 ? g.n[2] : 1),
                g.dtype == EXPW_F32 ? "f32" : "f64", g.order, g.bc, m);
  int fuse = -1, pk = -1;
  double best = 0.0;
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "r")) {
      char line[512];
      const size_t kl = std::strlen(key);
      while (std::fgets(line, sizeof line, f))
        if (std::strncmp(line, key, kl) == 0 && line[kl] == ' ') {
          int fz = 0, pkk = 0;
          double ms = 0.0;
          if (std::sscanf(line + kl, "%d %d %lf", &fz, &pkk, &ms) == 3 && fz >= 0 && fz <= kMaxFuse &&
              pkk >= EXPW_PASS_AUTO && pkk <= EXPW_PASS_STREAMED) {
            fuse = fz;
            pk = pkk;
            best = ms;
          }
        }
      std::fclose(f);
    }
  }
  if (fuse < 0) {
    // candidates: every depth the layout admits, and both 2D pass kernels
    const bool f32 = g.dtype == EXPW_F32;
    int smax = 1;
    if (g.bc == EXPW_BC_ZERO) {
      if (g.ndim == 3) smax = (f32 && g.order == 4) ? 2 : 1;
      else smax = (g.order == 4 && f32) ? 6 : 4;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      if (e0) (void)hipEventDestroy(e0);
      return fail(EXPW_EDEVICE, "autotune: event creation failed");
    }
    const int saved_fuse = op->fuse, saved_pk = op->pass_kernel;
    int32_t rc = EXPW_OK;
    const int reps = 3;
    for (int fz = 1; fz <= std::min(smax, m) && rc == EXPW_OK; ++fz) {
      const bool two = g.ndim == 2 && g.bc == EXPW_BC_ZERO && fz >= 2;
      for (int pkk : {EXPW_PASS_TILED, EXPW_PASS_STREAMED}) {
        if (!two && pkk == EXPW_PASS_STREAMED) continue;
        op->fuse = fz;
        op->pass_kernel = two ? pkk : EXPW_PASS_AUTO;
        rc = expw_step_faber(op, scratch, 0.0, dt, m, 1, nullptr);  // warm-up
        if (rc == EXPW_OK && hipEventRecord(e0, op->stream) != hipSuccess) rc = fail(EXPW_EDEVICE, "autotune: event record failed");
        if (rc == EXPW_OK) rc = expw_step_faber(op, scratch, dt, dt, m, reps, nullptr);
        float ms = 0.f;
        if (rc == EXPW_OK && (hipEventRecord(e1, op->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                              hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
          rc = fail(EXPW_EDEVICE, "autotune: timing failed");
        if (rc != EXPW_OK) break;
        const double per = ms / reps;
        if (fuse < 0 || per < best) {
          fuse = fz;
          pk = op->pass_kernel;
          best = per;
        }
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    op->fuse = saved_fuse;
    op->pass_kernel = saved_pk;
    if (rc != EXPW_OK) return rc;
    if (cache_path) {
      if (FILE* f = std::fopen(cache_path, "a")) {
        std::fprintf(f, "%s %d %d %.9g\n", key, fuse, pk, best);
        std::fclose(f);
      }
    }
  }
  op->fuse = fuse;
  op->pass_kernel = pk;
  if (fuse_out) *fuse_out = fuse;
  if (pass_kernel_out) *pass_kernel_out = pk;
  if (ms_out) *ms_out = best;
  return EXPW_OK;
}

int32_t expw_step_faber_noalloc(expw_op* op, void* state, double t0, double dt, int32_t m,
                                int64_t nsteps, void* traces) {
  if (int32_t rc = check_step_args(op, state, dt, nsteps)) return rc;
  if (m < 1 || m > EXPW_NOALLOC_MAX_M)
    return fail(EXPW_EINVAL, "Faber degree m must be in [1, %d] here", EXPW_NOALLOC_MAX_M);
  if (op->prof.active()) return fail(EXPW_EINVAL, "expw_step_faber_noalloc: kernel timing must be off");
  if (!op->noalloc_scratch)
    return fail(EXPW_EDEVICE, "expw_step_faber_noalloc: the static scratch has no device address");
  const size_t need = faber_big_bytes((op->g.ndim + 1) * npts(op->g), elem_size(op->g));
  if (need > kNoallocScratchBytes)
    return fail(EXPW_ENOMEM, "expw_step_faber_noalloc: the grid needs %zu bytes of scratch, the static scratch holds %zu",
                need, kNoallocScratchBytes);
  double a[EXPW_NOALLOC_MAX_M + 1], q[EXPW_NOALLOC_MAX_M];
  return dispatch(op, [&](auto cfg) {
    using C = decltype(cfg);
    using T = typename C::type;
    return faber_impl<T, C::k, C::bc, C::dim>(op, static_cast<T*>(state), t0, dt, m, nsteps, static_cast<T*>(traces), nullptr, op->noalloc_scratch, a, q);
  });
}

int32_t expw_step_faber_dense(expw_op* op, void* state, double t0, double dt, int32_t m,
                              int64_t nsteps, void* traces, void* term_traces) {
  if (int32_t rc = check_step_args(op, state, dt, nsteps)) return rc;
  if (m < 1 || m > 1024) return fail(EXPW_EINVAL, "Faber degree m must be in [1, 1024]");
  if (op->n_rec == 0) return fail(EXPW_EINVAL, "dense output needs receivers (expw_set_receivers)");
  if (!term_traces) return fail(EXPW_EINVAL, "term_traces is NULL");
  return dispatch(op, [&](auto cfg) {
    using C = decltype(cfg);
    using T = typename C::type;
    std::vector<double> a(m + 1), q(m);
    return faber_impl<T, C::k, C::bc, C::dim>(op, static_cast<T*>(state), t0, dt, m, nsteps, static_cast<T*>(traces), static_cast<T*>(term_traces), op->ws + op->off_big, a.data(), q.data());
  });
}

int32_t expw_faber_dense_output(expw_op* op, int32_t m, int64_t n_samples,
                                const int64_t* sample_step, const double* coef,
                                const void* term_traces, int64_t nsteps, void* out) {
  if (int32_t rc = check_op(op)) return rc;
  if (m < 0 || m > 1024 || n_samples < 0 || nsteps < 0)
    return fail(EXPW_EINVAL, "expw_faber_dense_output: invalid sizes");
  if (op->n_rec == 0) return fail(EXPW_EINVAL, "dense output needs receivers (expw_set_receivers)");
  if (n_samples == 0) return EXPW_OK;
  if (!sample_step || !coef || !term_traces || !out)
    return fail(EXPW_EINVAL, "expw_faber_dense_output: NULL array");
  const int64_t items = n_samples * op->n_rec;
  const unsigned grid = static_cast<unsigned>(std::min<int64_t>(65536, (items + kBlock - 1) / kBlock));
  if (op->g.dtype == EXPW_F32)
    k_dense_combine<float><<<grid, kBlock, 0, op->stream>>>(m, op->n_rec, n_samples, sample_step, coef, static_cast<const float*>(term_traces), nsteps, static_cast<float*>(out));
  else
    k_dense_combine<double><<<grid, kBlock, 0, op->stream>>>(m, op->n_rec, n_samples, sample_step, coef, static_cast<const double*>(term_traces), nsteps, static_cast<double*>(out));
  return check_launch("dense output");
}

int32_t expw_step_krylov(expw_op* op, void* state, double t0, double dt, int32_t k, int64_t nsteps,
                         void* traces) {
  if (int32_t rc = check_step_args(op, state, dt, nsteps)) return rc;
  if (k < 1 || k > op->kmax) return fail(EXPW_EINVAL, "Krylov dimension k must be in [1, %d] (max_krylov_k at create)", op->kmax);
  return dispatch(op, [&](auto cfg) {
    using C = decltype(cfg);
    using T = typename C::type;
    return krylov_impl<T, C::k, C::bc, C::dim>(op, static_cast<T*>(state), t0, dt, k, nsteps, static_cast<T*>(traces));
  });
}

int32_t expw_step_rk4(expw_op* op, void* state, double t0, double dt, int64_t nsteps, void* traces) {
  if (int32_t rc = check_step_args(op, state, dt, nsteps)) return rc;
  return dispatch(op, [&](auto cfg) {
    using C = decltype(cfg);
    using T = typename C::type;
    return rk4_impl<T, C::k, C::bc, C::dim>(op, static_cast<T*>(state), t0, dt, nsteps, static_cast<T*>(traces));
  });
}

int32_t expw_step_leapfrog(expw_op* op, void* state, double t0, double dt, int64_t nsteps, void* traces) {
  if (int32_t rc = check_step_args(op, state, dt, nsteps)) return rc;
  return dispatch(op, [&](auto cfg) {
    using C = decltype(cfg);
    using T = typename C::type;
    return leapfrog_impl<T, C::k, C::bc, C::dim>(op, static_cast<T*>(state), t0, dt, nsteps, static_cast<T*>(traces));
  });
}

int32_t expw_sync_status(expw_op* op) {
  if (int32_t rc = check_op(op)) return rc;
  const hipError_t e = hipStreamSynchronize(op->stream);
  if (e != hipSuccess) return fail(EXPW_EDEVICE, "device error: %s", hipGetErrorString(e));
  const hipError_t e2 = hipGetLastError();
  if (e2 != hipSuccess) return fail(EXPW_EDEVICE, "device error: %s", hipGetErrorString(e2));
  int flags[2] = {0, 0};  // Arnoldi barrier time-out, non-finite guard
  const char* flag = op->ws + op->off_kry + 136 * sizeof(double) + 8 * sizeof(int);
  if (hipMemcpy(flags, flag, sizeof(flags), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(EXPW_EDEVICE, "status read failed");
  if (flags[0]) {
    op->arn_nvmax_clean = 0;  // the reduction area is filled again before the next launch
    return fail(EXPW_EDEVICE, "a grid barrier of the persistent Arnoldi kernel timed out");
  }
  if (flags[1]) {
    // reported once: the flag is cleared for the next steps
    k_zero_u32<<<1, 64, 0, op->stream>>>(reinterpret_cast<unsigned*>(guard_flag(op)), 1);
    if (hipStreamSynchronize(op->stream) != hipSuccess) return fail(EXPW_EDEVICE, "guard reset failed");
    return fail(EXPW_ENONFINITE, "a state held a NaN or infinite value after a step (guard)");
  }
  return EXPW_OK;
}

int32_t expw_stream_bench(int32_t kind, int32_t nontemporal, const void* a, const void* b, void* c,
                          size_t bytes, int32_t reps, void* stream, double* ms_per_launch) {
  if (kind < 0 || kind > 2) return fail(EXPW_EINVAL, "kind must be 0 (read), 1 (copy) or 2 (triad)");
  if (!a || !c || (kind == 2 && !b) || !ms_per_launch) return fail(EXPW_EINVAL, "NULL argument");
  if (bytes == 0 || bytes % 16 != 0) return fail(EXPW_EINVAL, "bytes must be a positive multiple of 16");
  if ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) | reinterpret_cast<uintptr_t>(c)) % 16)
    return fail(EXPW_EINVAL, "arrays must be 16-byte aligned");
  if (reps < 1) return fail(EXPW_EINVAL, "reps must be >= 1");
  const int64_t n4 = static_cast<int64_t>(bytes / 16);
  const unsigned blocks = stream_blocks(n4);
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto launch = [&]() {
    const float4* A = static_cast<const float4*>(a);
    const float4* B = static_cast<const float4*>(b);
    float4* C = static_cast<float4*>(c);
#define EXPW_STREAM(K_, NT_) hipLaunchKernelGGL((k_stream<K_, NT_>), dim3(blocks), dim3(kStreamNT), 0, st, A, B, C, n4, 2.0f)
    if (nontemporal) {
      if (kind == 0) EXPW_STREAM(0, true); else if (kind == 1) EXPW_STREAM(1, true); else EXPW_STREAM(2, true);
    } else {
      if (kind == 0) EXPW_STREAM(0, false); else if (kind == 1) EXPW_STREAM(1, false); else EXPW_STREAM(2, false);
    }
#undef EXPW_STREAM
  };
  launch();  // warm-up
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(EXPW_EDEVICE, "stream bench: event creation failed");
  }
  (void)hipEventRecord(e0, st);
  for (int r = 0; r < reps; ++r) launch();
  (void)hipEventRecord(e1, st);
  hipError_t e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(EXPW_EDEVICE, "stream bench: %s", hipGetErrorString(e));
  if (int32_t rc = check_launch("stream bench")) return rc;
  *ms_per_launch = static_cast<double>(ms) / reps;
  return EXPW_OK;
}

int32_t expw_set_timing(expw_op* op, int32_t class_mask) {
  if (int32_t rc = check_op(op)) return rc;
  op->prof.enable(static_cast<uint32_t>(class_mask));
  return EXPW_OK;
}

int32_t expw_get_timing(expw_op* op, double* ms, int64_t* launches, double* bytes) {
  if (int32_t rc = check_op(op)) return rc;
  if (!op->prof.collect()) return fail(EXPW_EDEVICE, "timing: event query failed");
  for (int k = 0; k < EXPW_KERNEL_CLASSES; ++k) {
    if (ms) ms[k] = op->prof.ms(k);
    if (launches) launches[k] = op->prof.launches(k);
    if (bytes) bytes[k] = op->prof.bytes(k);
  }
  return EXPW_OK;
}

int32_t expw_krylov_info(const expw_op* op, int32_t* k_eff, double* beta) {
  if (int32_t rc = check_op(op)) return rc;
  if (!k_eff || !beta) return fail(EXPW_EINVAL, "NULL output");
  if (op->last_keff >= 0) {
    *k_eff = op->last_keff;
    *beta = op->last_beta;
    return EXPW_OK;
  }
  // the last step ran its exponential on the device
  int ke = 0;
  double b = 0.0;
  if (hipMemcpyAsync(&ke, op->ws + op->off_kry + 136 * sizeof(double), sizeof(int), hipMemcpyDeviceToHost,
                     op->stream) != hipSuccess ||
      hipMemcpyAsync(&b, op->ws + op->off_scal + sizeof(double), sizeof(double), hipMemcpyDeviceToHost,
                     op->stream) != hipSuccess ||
      hipStreamSynchronize(op->stream) != hipSuccess)
    return fail(EXPW_EDEVICE, "krylov info: copy failed");
  *k_eff = ke;
  *beta = b;
  return EXPW_OK;
}

int32_t expw_set_krylov_estimate(expw_op* op, int32_t on) {
  if (int32_t rc = check_op(op)) return rc;
  op->kry_estimate = on != 0;
  return EXPW_OK;
}

int32_t expw_krylov_estimate(const expw_op* op, double* est) {
  if (int32_t rc = check_op(op)) return rc;
  if (!est) return fail(EXPW_EINVAL, "NULL output");
  if (!op->last_est_valid)
    return fail(EXPW_EINVAL, "the last Krylov call ran without the estimate (expw_set_krylov_estimate)");
  *est = op->last_est;
  return EXPW_OK;
}

int32_t expw_set_krylov_persistent(expw_op* op, int32_t allow) {
  if (int32_t rc = check_op(op)) return rc;
  op->kry_persistent = allow != 0;
  return EXPW_OK;
}

int32_t expw_set_krylov_expm(expw_op* op, int32_t mode) {
  if (int32_t rc = check_op(op)) return rc;
  if (mode != EXPW_EXPM_DEVICE && mode != EXPW_EXPM_HOST)
    return fail(EXPW_EINVAL, "mode must be EXPW_EXPM_DEVICE or EXPW_EXPM_HOST");
  op->kry_mode = mode;
  return EXPW_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- PML operator

struct expw_pml {
  expw_pml_grid g;
  const void* c2;
  char* ws;
  size_t ws_bytes;
  hipStream_t stream;
  int pmax;
  size_t off_bx, off_bxh, off_by, off_byh, off_src_idx, off_src_amp, off_big;
  double c2max, x_lo, B, gamma, c0, c1;
  double d2[4][9], d1[3][8], dw[4][8];
  int n_src;
  int64_t src_lo, src_hi;
  double f_peak, t_delay;
  int taylor_p;
  int n_rec;
  const int64_t* rec_dev;
  int path;  // 0 automatic, 1 one thread per node, 2 LDS tiles, 3 pairs of terms in LDS tiles, 4 row-streamed passes
  // Krylov (launch per step): largest dimension, workspace offsets, stride of a basis vector
  int kmax;
  size_t off_part, off_scal, off_hess, off_kry, off_gram;
  int64_t naug_pad;
};

namespace expw {
namespace {

// tiles (64 x 16 nodes) from which the LDS path is taken automatically: with
// fewer, its 256-thread blocks leave the CUs short of waves
constexpr int64_t kPmlLdsMinTiles = 2048;

// Terms per streamed PML pass (pml_stream.h): FP32 up to kPmlStreamDepth,
// FP64 two.
constexpr int kPmlStreamDepth = 4;

// The term kernel a step of degree m takes: the forced one, else the
// row-streamed passes where the grid gives them enough row segments (8192 x
// 4096, m = 16: FP32 108 against 44 G grid-pt matvecs/s for pairs, FP64 42
// against 21 for LDS tiles), below that at FP32 pairs of terms on LDS tiles
// (1001 x 501: 47 against 6 G/s for three bands of streamed passes), and at
// FP64 LDS tiles from kPmlLdsMinTiles tiles up, one thread per node below.
int pml_path_for(const expw_pml* op, int m) {
  if (op->path != 0) return op->path;
  if (op->g.dtype == EXPW_F32 && m >= 2)
    return pml_stream_fits<float>(op->g.nx, op->g.ny, kPmlStreamDepth) ? 4 : 3;
  if (m >= 2 && pml_stream_fits<double>(op->g.nx, op->g.ny, 2)) return 4;
  const int64_t tiles = ((op->g.nx + kPmlTX - 1) / kPmlTX) * ((op->g.ny + kPmlTY - 1) / kPmlTY);
  return tiles >= kPmlLdsMinTiles ? 2 : 1;
}

struct PmlLayout {
  size_t bx, bxh, by, byh, src_idx, src_amp, part, scal, hess, kry, gram, big, total;
  int64_t naug_pad;
};

PmlLayout pml_layout(const expw_pml_grid& g, int kmax, int pmax) {
  const size_t es = g.dtype == EXPW_F32 ? 4 : 8;
  PmlLayout L{};
  size_t off = 0;
  L.bx = off; off = align_up(off + g.nx * es);
  L.bxh = off; off = align_up(off + g.nx * es);
  L.by = off; off = align_up(off + g.ny * es);
  L.byh = off; off = align_up(off + g.ny * es);
  L.src_idx = off; off = align_up(off + EXPW_MAX_SOURCES * sizeof(int64_t));
  L.src_amp = off; off = align_up(off + EXPW_MAX_SOURCES * es);
  L.part = off; off = align_up(off + 2 * kRedMaxBlocks * sizeof(double));  // two partial sets
  L.scal = off; off = align_up(off + 64 * sizeof(double));
  L.hess = off; off = align_up(off + (EXPW_MAX_KRYLOV + 1) * kHessLd * sizeof(double));
  L.kry = off; off = align_up(off + 64 * sizeof(double) + 72 * sizeof(double) + 64 * sizeof(int));  // y, scales, keff
  if (kmax > 0) L.gram = off, off = align_up(off + (static_cast<size_t>(kGramPartials) + kGramTot + 2 * EXPW_MAX_KRYLOV) * sizeof(double));  // Gram-Schmidt partials, table and totals
  L.big = off;
  const int64_t ns = 4 * g.nx * g.ny;
  L.naug_pad = (ns + pmax + 63) / 64 * 64;
  // Faber: two pairs of terms and the FP64 partial sum; Krylov: kmax + 1 basis vectors
  size_t big = 4 * static_cast<size_t>(ns) * es + static_cast<size_t>(ns) * sizeof(double);
  if (kmax > 0) big = std::max(big, static_cast<size_t>(kmax + 1) * L.naug_pad * es);
  L.total = align_up(off + big);
  return L;
}

template <typename T>
PmlGeo<T> make_pml_geo(const expw_pml* op) {
  PmlGeo<T> g{};
  g.nx = static_cast<int32_t>(op->g.nx);
  g.ny = static_cast<int32_t>(op->g.ny);
  g.N = op->g.nx * op->g.ny;
  // the interior weights as integers (exact in T) with one scale each; the
  // surface tables and 1/h, 1/h^2 as hi + lo in T (lo = 0 in FP64)
  auto split = [](double w, T& hi, T& lo) {
    hi = static_cast<T>(w);
    lo = static_cast<T>(w - static_cast<double>(hi));
  };
  const double h = op->g.h;
  split(1.0 / h, g.ih, g.ih_lo);
  split(1.0 / (h * h), g.ih2, g.ih2_lo);
  double wi[4], beta = 0.0;
  int K = 0;
  stagger_weights_int(8, wi, &beta, &K);  // alpha_l = beta wi_l, beta = 1/107520
  for (int l = 0; l < 4; ++l) g.a[l] = static_cast<T>(wi[l]);
  g.sc1 = static_cast<T>(beta / h);
  // Sec. 2.1, centred second derivative (read with sums): (-205/72, 8/5,
  // -1/5, 8/315, -1/560) = (-14350, 8064, -1008, 128, -9) / 5040
  g.d2c = static_cast<T>(-14350.0);
  const double b[4] = {8064.0, -1008.0, 128.0, -9.0};
  for (int l = 0; l < 4; ++l) g.d2[l] = static_cast<T>(b[l]);
  g.sc2 = static_cast<T>(1.0 / (5040.0 * h * h));
  for (int r = 0; r < 4; ++r)
    for (int k = 0; k < 9; ++k) split(op->d2[r][k], g.s2[r][k], g.s2_lo[r][k]);
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 8; ++k) split(op->d1[r][k], g.s1[r][k], g.s1_lo[r][k]);
  for (int r = 0; r < 4; ++r)
    for (int k = 0; k < 8; ++k) split(op->dw[r][k], g.sw[r][k], g.sw_lo[r][k]);
  g.c2 = static_cast<const T*>(op->c2);
  g.bx = reinterpret_cast<const T*>(op->ws + op->off_bx);
  g.bxh = reinterpret_cast<const T*>(op->ws + op->off_bxh);
  g.by = reinterpret_cast<const T*>(op->ws + op->off_by);
  g.byh = reinterpret_cast<const T*>(op->ws + op->off_byh);
  return g;
}

template <typename T>
Src<T> make_pml_src(const expw_pml* op, double q) {
  Src<T> s{};
  s.n = op->n_src;
  s.lo = op->src_lo;
  s.hi = op->src_hi;
  s.idx = reinterpret_cast<const int64_t*>(op->ws + op->off_src_idx);
  s.amp = reinterpret_cast<const T*>(op->ws + op->off_src_amp);
  s.q = q;
  return s;
}

// One Faber step of degree m >= 2 in passes of two terms (k_pml_faber_pair_lds)
// and, for odd m, a last single term. Pass buffers: v_0 = S, then the pairs
// (A, B) and (D, E) in turn; C holds the sum. A pass reads v_{j-1} and v_{j-2}
// with halos, so it never writes them; a first pass that is also the last
// (m = 2) sums into C and copies to S.
template <typename T, typename Term>
int32_t pml_pairs(expw_pml* op, const PmlGeo<T>& g, T* S, T* A, T* B, double* C, T* D, T* E, const double* a,
                  const double* q, int m, double gs, double c0s, double c1s, int tiles_x, unsigned grid,
                  Term&& term) {
  const int64_t ns = 4 * g.N;
  const T* vp = S;
  const T* vpp = nullptr;
  T* pair_out[2][2] = {{A, B}, {D, E}};
  int which = 0;
  int j = 1;
  for (; j + 1 <= m; j += 2) {
    const bool last = (j + 1 == m);
    PmlTerm<T> t0{}, t1{};
    t0.inv_gamma = t1.inv_gamma = static_cast<T>(1.0 / gs);
    t0.c0 = t1.c0 = static_cast<T>(c0s);
    t0.first = j == 1 ? 1 : 0;
    if (j == 1) split_weight(a[0], &t0.a_first, &t0.a_first_lo);
    t0.cpp = j == 1 ? T(0) : static_cast<T>(c1s);
    t1.cpp = static_cast<T>(j + 1 == 2 ? 2.0 * c1s : c1s);
    split_weight(a[j], &t0.a_j, &t0.a_j_lo);
    split_weight(a[j + 1], &t1.a_j, &t1.a_j_lo);
    T* o0 = last ? nullptr : pair_out[which][0];
    T* o1 = last ? nullptr : pair_out[which][1];
    // the last pass rounds the sum into S, or into A when it reads S (m = 2)
    double* acc_out = last ? nullptr : C;
    T* state_out = last ? (vp != S ? S : A) : nullptr;
    // FP32: 1024-thread blocks on 64 x 32 tiles; FP64 (more registers): 256 on 64 x 16
    constexpr int NT = sizeof(T) == 4 ? 1024 : 256, TY = sizeof(T) == 4 ? 32 : 16;
    const int ptx = static_cast<int>((g.nx + kPmlTX - 1) / kPmlTX);
    const int pty = static_cast<int>((g.ny + TY - 1) / TY);
    const int pbw = (ptx + 7) / 8;
    const unsigned pgrid = 8u * static_cast<unsigned>(pbw) * static_cast<unsigned>(pty);
    k_pml_faber_pair_lds<T, NT, TY><<<pgrid, NT, 0, op->stream>>>(g, vp, vpp, o0, o1, j == 1 ? nullptr : C, acc_out,
                                                                  state_out, t0, t1, make_pml_src<T>(op, q[j - 1]),
                                                                  make_pml_src<T>(op, q[j]), ptx, pty, pbw);
    if (int32_t rc = check_launch("pml faber pair")) return rc;
    if (last && state_out == A) {
      if (hipMemcpyAsync(S, A, ns * sizeof(T), hipMemcpyDeviceToDevice, op->stream) != hipSuccess)
        return fail(EXPW_EDEVICE, "pml faber: copy failed");
    }
    vpp = pair_out[which][0];
    vp = pair_out[which][1];
    which ^= 1;
  }
  if (j == m) {
    // odd m: the last term alone (v_{m-1} = vp, v_{m-2} = vpp, neither is S)
    PmlTerm<T> c{};
    c.inv_gamma = static_cast<T>(1.0 / gs);
    c.c0 = static_cast<T>(c0s);
    c.cpp = static_cast<T>(c1s);
    split_weight(a[m], &c.a_j, &c.a_j_lo);
    term(vp, vpp, nullptr, C, nullptr, S, c, q[m - 1]);
    if (int32_t rc = check_launch("pml faber last term")) return rc;
  }
  return EXPW_OK;
}

// One Faber step of degree m >= 2 in row-streamed passes (pml_stream.h) of at
// most kPmlStreamDepth terms (FP64: 2), sized as evenly as the count of
// passes allows (the larger ones first); a last pass of one term (m odd at
// FP64) takes the one-term kernel. Buffers as in pml_pairs.
template <typename T, typename Term>
int32_t pml_stream_passes(expw_pml* op, const PmlGeo<T>& g, T* S, T* A, T* B, double* C, T* D, T* E, const double* a,
                          const double* q, int m, double gs, double c0s, double c1s, Term&& term) {
  const int64_t ns = 4 * g.N;
  constexpr int smax = sizeof(T) == 4 ? kPmlStreamDepth : 2;
  const int npass = (m + smax - 1) / smax;
  const int base = m / npass, rem = m % npass;
  const T* vp = S;
  const T* vpp = nullptr;
  T* pair_out[2][2] = {{A, B}, {D, E}};
  int which = 0;
  int j = 1;
  for (int p = 0; p < npass; ++p) {
    const int n = base + (p < rem ? 1 : 0);
    const bool last = p + 1 == npass;
    if (n == 1) {
      // the last term alone (v_{m-1} = vp, v_{m-2} = vpp, neither is S)
      PmlTerm<T> c{};
      c.inv_gamma = static_cast<T>(1.0 / gs);
      c.c0 = static_cast<T>(c0s);
      c.cpp = static_cast<T>(c1s);
      split_weight(a[m], &c.a_j, &c.a_j_lo);
      term(vp, vpp, nullptr, C, nullptr, S, c, q[m - 1]);
      if (int32_t rc = check_launch("pml faber last term")) return rc;
      break;
    }
    T* ol = last ? nullptr : pair_out[which][1];
    T* opv = last ? nullptr : pair_out[which][0];
    // the last pass rounds the sum into S, or into A when it reads S
    double* acc_out = last ? nullptr : C;
    T* state_out = last ? (vp != S ? S : A) : nullptr;
    const Src<T> src = make_pml_src<T>(op, 0.0);
    int32_t rc = EXPW_OK;
    if constexpr (sizeof(T) == 4) {
      switch (n) {
        case 2: rc = launch_pml_stream<T, 2>(op->stream, g, src, vp, vpp, C, ol, opv, acc_out, state_out, j, a, q, gs, c0s, c1s); break;
        case 3: rc = launch_pml_stream<T, 3>(op->stream, g, src, vp, vpp, C, ol, opv, acc_out, state_out, j, a, q, gs, c0s, c1s); break;
        default: rc = launch_pml_stream<T, 4>(op->stream, g, src, vp, vpp, C, ol, opv, acc_out, state_out, j, a, q, gs, c0s, c1s); break;
      }
    } else {
      rc = launch_pml_stream<T, 2>(op->stream, g, src, vp, vpp, C, ol, opv, acc_out, state_out, j, a, q, gs, c0s, c1s);
    }
    if (rc != EXPW_OK) return rc;
    if (last && state_out == A) {
      if (hipMemcpyAsync(S, A, ns * sizeof(T), hipMemcpyDeviceToDevice, op->stream) != hipSuccess)
        return fail(EXPW_EDEVICE, "pml faber: copy failed");
    }
    vpp = opv;
    vp = ol;
    which ^= 1;
    j += n;
  }
  return EXPW_OK;
}

// Faber steps (Sec. 3.2) on the PML operator, one term per sweep; the ellipse
// is the step ellipse of precision T, as for the p/v operator.
template <typename T>
int32_t pml_faber_impl(expw_pml* op, T* S, double t0, double dt, int m, int64_t nsteps, T* traces) {
  const PmlGeo<T> g = make_pml_geo<T>(op);
  const int64_t ns = 4 * g.N;
  T* A = reinterpret_cast<T*>(op->ws + op->off_big);
  T* B = A + ns;
  double* C = reinterpret_cast<double*>(B + ns);  // the FP64 partial sum
  double gs, c0s, c1s;
  step_ellipse(sizeof(T) == 4 ? EXPW_F32 : EXPW_F64, op->gamma, op->c0, op->c1, &gs, &c0s, &c1s);
  std::vector<double> a(m + 1), q(m, 0.0), der(EXPW_MAX_TAYLOR), G(EXPW_MAX_TAYLOR);
  faber_coefficients(gs, c0s, c1s, dt, m, a.data());
  const int p = op->taylor_p;
  const double sc = 1.0 / (op->g.h * op->g.h);
  const int tiles_x = static_cast<int>((op->g.nx + kPmlTX - 1) / kPmlTX);
  const int tiles_y = static_cast<int>((op->g.ny + kPmlTY - 1) / kPmlTY);
  const int band_w = (tiles_x + 7) / 8;
  const int path = pml_path_for(op, m);
  const bool pairs = path == 3;
  const bool streamed = path == 4;
  const bool lds = path >= 2;
  const unsigned grid = lds ? 8u * static_cast<unsigned>(band_w) * static_cast<unsigned>(tiles_y) : grid_for(g.N);
  T* D = reinterpret_cast<T*>(C + ns);
  T* E = D + ns;
  // one term: the LDS kernel on tiles or one thread per node; the sum to
  // acc_out, or rounded into state_out on the step's last term
  auto term = [&](const T* vp, const T* vpp, T* vout, const double* acc_in, double* acc_out, T* state_out,
                  const PmlTerm<T>& c, double qj) {
    if (lds)
      k_pml_faber_term_lds<T><<<grid, kBlock, 0, op->stream>>>(g, vp, vpp, vout, acc_in, acc_out, state_out, c,
                                                               make_pml_src<T>(op, qj), tiles_x, tiles_y, band_w);
    else
      k_pml_faber_term<T><<<grid, kBlock, 0, op->stream>>>(g, vp, vpp, vout, acc_in, acc_out, state_out, c,
                                                           make_pml_src<T>(op, qj));
  };
  for (int64_t st = 0; st < nsteps; ++st) {
    const double t = t0 + st * dt;
    if (op->n_src > 0) {
      ricker_derivatives(t, op->f_peak, op->t_delay, p, der.data());
      for (int c = 0; c < p; ++c) G[c] = der[p - 1 - c];
      faber_source_scalars(gs, c0s, c1s, m, p, G.data(), q.data());
      for (int j = 0; j < m; ++j) q[j] *= sc;
    }
    if ((pairs || streamed) && m >= 2) {
      if (streamed) {
        if (int32_t rc = pml_stream_passes<T>(op, g, S, A, B, C, D, E, a.data(), q.data(), m, gs, c0s, c1s, term))
          return rc;
      } else if (int32_t rc = pml_pairs<T>(op, g, S, A, B, C, D, E, a.data(), q.data(), m, gs, c0s, c1s, tiles_x,
                                           grid, term)) {
        return rc;
      }
      if (traces && op->n_rec > 0) {
        k_gather<T><<<grid_for(op->n_rec), kBlock, 0, op->stream>>>(S, op->rec_dev, op->n_rec, traces + st * op->n_rec);
        if (int32_t rc = check_launch("pml gather")) return rc;
      }
      continue;
    }
    PmlTerm<T> c{};
    c.inv_gamma = static_cast<T>(1.0 / gs);
    c.c0 = static_cast<T>(c0s);
    // j = 1: v1 = F1 v0 into A, sum a0 v0 + a1 v1 into C
    c.first = 1;
    split_weight(a[0], &c.a_first, &c.a_first_lo);
    split_weight(a[1], &c.a_j, &c.a_j_lo);
    // (S is read with a halo here, so a one-term step rounds its sum into A first)
    term(S, nullptr, m == 1 ? nullptr : A, nullptr, m == 1 ? nullptr : C, m == 1 ? A : nullptr, c, q[0]);
    if (int32_t rc = check_launch("pml faber j=1")) return rc;
    if (m == 1) {
      if (hipMemcpyAsync(S, A, ns * sizeof(T), hipMemcpyDeviceToDevice, op->stream) != hipSuccess)
        return fail(EXPW_EDEVICE, "pml faber: copy failed");
    } else {
      // j = 2: v2 = F1 v1 - 2 c1 v0 into B
      c.first = 0;
      c.a_first = c.a_first_lo = T(0);
      c.cpp = static_cast<T>(2.0 * c1s);
      split_weight(a[2], &c.a_j, &c.a_j_lo);
      term(A, S, m == 2 ? nullptr : B, C, m == 2 ? nullptr : C, m == 2 ? S : nullptr, c, q[1]);
      if (int32_t rc = check_launch("pml faber j=2")) return rc;
      T* last = B;
      T* older = A;
      c.cpp = static_cast<T>(c1s);
      for (int j = 3; j <= m; ++j) {
        split_weight(a[j], &c.a_j, &c.a_j_lo);
        const bool fin = j == m;
        term(last, older, fin ? nullptr : older, C, fin ? nullptr : C, fin ? S : nullptr, c, q[j - 1]);
        if (int32_t rc = check_launch("pml faber term")) return rc;
        std::swap(last, older);
      }
    }
    if (traces && op->n_rec > 0) {
      k_gather<T><<<grid_for(op->n_rec), kBlock, 0, op->stream>>>(S, op->rec_dev, op->n_rec, traces + st * op->n_rec);
      if (int32_t rc = check_launch("pml gather")) return rc;
    }
  }
  return EXPW_OK;
}

// RK4 steps (Sec. 3.1) on the PML operator; the source enters at the stage times.
template <typename T>
int32_t pml_rk4_impl(expw_pml* op, T* S, double t0, double dt, int64_t nsteps, T* traces) {
  const PmlGeo<T> g = make_pml_geo<T>(op);
  const int64_t ns = 4 * g.N;
  T* A = reinterpret_cast<T*>(op->ws + op->off_big);
  T* B = A + ns;
  T* C = B + ns;
  const unsigned grid = grid_for(g.N);
  const double sc = 1.0 / (op->g.h * op->g.h);
  auto srcq = [&](double t) {
    double gv = 0.0;
    if (op->n_src > 0) ricker_derivatives(t, op->f_peak, op->t_delay, 1, &gv);
    return make_pml_src<T>(op, gv * sc);
  };
  const T h2 = static_cast<T>(0.5 * dt), h1 = static_cast<T>(dt), s6 = static_cast<T>(dt / 6.0),
          s3 = static_cast<T>(dt / 3.0);
  for (int64_t st = 0; st < nsteps; ++st) {
    const double t = t0 + st * dt;
    k_pml_rk4_stage<T><<<grid, kBlock, 0, op->stream>>>(g, S, S, nullptr, A, C, h2, s6, srcq(t));
    k_pml_rk4_stage<T><<<grid, kBlock, 0, op->stream>>>(g, A, S, C, B, C, h2, s3, srcq(t + 0.5 * dt));
    k_pml_rk4_stage<T><<<grid, kBlock, 0, op->stream>>>(g, B, S, C, A, C, h1, s3, srcq(t + 0.5 * dt));
    k_pml_rk4_stage<T><<<grid, kBlock, 0, op->stream>>>(g, A, nullptr, C, nullptr, S, T(0), s6, srcq(t + dt));
    if (int32_t rc = check_launch("pml rk4 stage")) return rc;
    if (traces && op->n_rec > 0) {
      k_gather<T><<<grid_for(op->n_rec), kBlock, 0, op->stream>>>(S, op->rec_dev, op->n_rec, traces + st * op->n_rec);
      if (int32_t rc = check_launch("pml gather")) return rc;
    }
  }
  return EXPW_OK;
}

// Krylov steps (Sec. 3.2) on the PML operator: the launch-per-step Arnoldi
// process (modified Gram-Schmidt, one projection per reduction) and the small
// exponential on the device.
template <typename T>
int32_t pml_krylov_impl(expw_pml* op, T* S, double t0, double dt, int k, int64_t nsteps, T* traces) {
  const PmlGeo<T> g = make_pml_geo<T>(op);
  const int64_t ns = 4 * g.N;
  const int p = op->n_src > 0 ? op->taylor_p : 0;
  const int64_t naug = ns + p;
  const int64_t ld = op->naug_pad;
  T* Q = reinterpret_cast<T*>(op->ws + op->off_big);
  double* part = reinterpret_cast<double*>(op->ws + op->off_part);
  double* scal = reinterpret_cast<double*>(op->ws + op->off_scal);
  double* hess = reinterpret_cast<double*>(op->ws + op->off_hess);
  const T* amp = reinterpret_cast<const T*>(op->ws + op->off_src_amp);
  double* kry_y = reinterpret_cast<double*>(op->ws + op->off_kry);
  double* kry_sc = kry_y + 64;
  int* kry_keff = reinterpret_cast<int*>(op->ws + op->off_kry + 136 * sizeof(double));
  const unsigned rg_vec = red_grid_for(naug);
  const unsigned rg_pts = red_grid_for(g.N + p);
  const double tol = 1e-14;
  std::vector<double> der(EXPW_MAX_TAYLOR);
  KrySrc ks{};
  ks.n = op->n_src;
  ks.p = p;
  ks.lo = op->src_lo;
  ks.hi = op->src_hi;
  ks.idx = reinterpret_cast<const int64_t*>(op->ws + op->off_src_idx);
  const double sc = 1.0 / (op->g.h * op->g.h);
  for (int64_t st = 0; st < nsteps; ++st) {
    const double t = t0 + st * dt;
    if (p > 0) {
      ricker_derivatives(t, op->f_peak, op->t_delay, p, der.data());
      for (int c = 0; c < p; ++c) ks.G[c] = der[p - 1 - c] * sc;
    }
    double* P[2] = {part, part + kRedMaxBlocks};
    const unsigned nb_ns = red_grid_for(ns);
    k_norm2<T><<<nb_ns, kBlock, 0, op->stream>>>(S, ns, P[0]);
    k_kry_init<T><<<rg_vec, kBlock, 0, op->stream>>>(S, ns, Q, naug, P[0], nb_ns, p > 0 ? 1.0 : 0.0, scal + 1,
                                                     kry_sc);
    // Gram-Schmidt in three launches per column (gram.h); P[0] carries the
    // partials of |w|^2 to the next column's matvec, P[1] takes the matvec's
    // unused partials of w . q_0
    double* gpart = reinterpret_cast<double*>(op->ws + op->off_gram);
    double* gram = gpart + kGramPartials;
    int nin = 0;
    for (int j = 0; j < k; ++j) {
      T* w = Q + (j + 1) * ld;
      k_pml_kry_matvec<T><<<rg_pts, kBlock, 0, op->stream>>>(g, Q + j * ld, w, Q, ks, amp, j == 0 ? nullptr : P[0],
                                                             nin, tol, scal + 1,
                                                             j == 0 ? nullptr : hess + j * kHessLd + (j - 1),
                                                             kry_sc + j, P[1]);
      const unsigned gd = gram_dots_grid(naug, j);
      k_gram_dots<T><<<gd, kBlock, 0, op->stream>>>(w, Q, ld, naug, j, gpart);
      k_gram_reduce<<<2 * j + 1, kBlock, 0, op->stream>>>(gpart, static_cast<int>(gd), 2 * j + 1, gram + kGramTot);
      k_gram_subst<<<1, 64, 0, op->stream>>>(gram + kGramTot, j, kry_sc, gram, hess, kHessLd, kry_y);
      k_gram_update<T><<<rg_vec, kBlock, 0, op->stream>>>(w, Q, ld, naug, j, kry_y, P[0]);
      nin = static_cast<int>(rg_vec);
    }
    k_kry_finish<<<1, kBlock, 0, op->stream>>>(P[0], nin, tol, scal + 1, hess + k * kHessLd + (k - 1), kry_sc + k);
    expm_kernel(k)<<<1, expm_threads(k), 0, op->stream>>>(hess, k, dt, tol, scal + 1, kry_y, kry_keff);
    k_kry_combine_dev<T><<<red_grid_for(ns), kBlock, 0, op->stream>>>(S, Q, ld, ns, kry_y, kry_keff, scal + 1, kry_sc,
                                                                      RecRun<T>{nullptr, 0, 0});
    if (int32_t rc = check_launch("pml krylov")) return rc;
    if (traces && op->n_rec > 0) {
      k_gather<T><<<grid_for(op->n_rec), kBlock, 0, op->stream>>>(S, op->rec_dev, op->n_rec, traces + st * op->n_rec);
      if (int32_t rc = check_launch("pml gather")) return rc;
    }
  }
  return EXPW_OK;
}

int32_t check_pml(const expw_pml* op) {
  if (!op) return fail(EXPW_EINVAL, "op is NULL");
  return EXPW_OK;
}

}  // namespace
}  // namespace expw

extern "C" {

int32_t expw_pml_workspace_size(const expw_pml_grid* g, int32_t max_k, int32_t max_p, size_t* bytes) {
  clear_error();
  if (int32_t rc = expw_pml_check_grid(g)) return rc;
  if (max_k < 0 || max_k > EXPW_MAX_KRYLOV) return fail(EXPW_EINVAL, "max_krylov_k must be in [0, %d]", EXPW_MAX_KRYLOV);
  if (max_p < 0 || max_p > EXPW_MAX_TAYLOR) return fail(EXPW_EINVAL, "max_taylor_p must be in [0, %d]", EXPW_MAX_TAYLOR);
  if (!bytes) return fail(EXPW_EINVAL, "bytes is NULL");
  *bytes = pml_layout(*g, max_k, max_p).total;
  return EXPW_OK;
}

int32_t expw_pml_create(const expw_pml_grid* g, const void* c2_dev, int32_t max_k, int32_t max_p, void* ws,
                        size_t ws_bytes, void* stream, expw_pml** out) {
  clear_error();
  size_t need = 0;
  if (int32_t rc = expw_pml_workspace_size(g, max_k, max_p, &need)) return rc;
  if (!out) return fail(EXPW_EINVAL, "out is NULL");
  if (!c2_dev) return fail(EXPW_EINVAL, "c2_dev is NULL");
  if (!ws) return fail(EXPW_EINVAL, "workspace_dev is NULL");
  if (ws_bytes < need) return fail(EXPW_ENOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0) return fail(EXPW_EINVAL, "workspace must be 256-byte aligned");
  expw_pml* op = new expw_pml();
  op->g = *g;
  op->c2 = c2_dev;
  op->ws = static_cast<char*>(ws);
  op->ws_bytes = ws_bytes;
  op->stream = static_cast<hipStream_t>(stream);
  op->pmax = max_p;
  op->kmax = max_k;
  const PmlLayout L = pml_layout(*g, max_k, max_p);
  op->off_gram = L.gram;
  op->off_part = L.part;
  op->off_scal = L.scal;
  op->off_hess = L.hess;
  op->off_kry = L.kry;
  op->naug_pad = L.naug_pad;
  op->off_bx = L.bx;
  op->off_bxh = L.bxh;
  op->off_by = L.by;
  op->off_byh = L.byh;
  op->off_src_idx = L.src_idx;
  op->off_src_amp = L.src_amp;
  op->off_big = L.big;
  op->n_src = 0;
  op->n_rec = 0;
  op->rec_dev = nullptr;
  op->taylor_p = std::max(1, std::min(8, max_p));
  op->path = 0;
  pml_surface_tables(op->d2, op->d1, op->dw);
  // damping profiles (FP64 on the host, stored in the grid dtype)
  const size_t es = g->dtype == EXPW_F32 ? 4 : 8;
  std::vector<std::vector<char>> staging;
  for (int k = 0; k < 4; ++k) {
    const int64_t n = k < 2 ? g->nx : g->ny;
    std::vector<double> prof(n);
    if (k < 2) damping_profile(n, g->h, g->abc_cells, g->beta0, k == 1, prof.data());
    else bottom_profile(n, g->h, g->abc_cells, g->beta0, k == 3, prof.data());
    std::vector<char> buf(n * es);
    for (int64_t i = 0; i < n; ++i) {
      if (g->dtype == EXPW_F32) reinterpret_cast<float*>(buf.data())[i] = static_cast<float>(prof[i]);
      else reinterpret_cast<double*>(buf.data())[i] = prof[i];
    }
    const size_t off = k == 0 ? L.bx : k == 1 ? L.bxh : k == 2 ? L.by : L.byh;
    if (hipMemcpyAsync(op->ws + off, buf.data(), buf.size(), hipMemcpyHostToDevice, op->stream) != hipSuccess) {
      delete op;
      return fail(EXPW_EDEVICE, "expw_pml_create: profile upload failed");
    }
    staging.push_back(std::move(buf));
  }
  // largest c^2 (partials in the Faber buffer, which is free until a step)
  double* part = reinterpret_cast<double*>(op->ws + L.big);
  const int64_t N = g->nx * g->ny;
  const unsigned nb = red_grid_for(N);
  if (g->dtype == EXPW_F32)
    k_c2_max<float><<<nb, kBlock, 0, op->stream>>>(static_cast<const float*>(c2_dev), N, part);
  else
    k_c2_max<double><<<nb, kBlock, 0, op->stream>>>(static_cast<const double*>(c2_dev), N, part);
  std::vector<double> parts(nb);
  hipError_t e = hipMemcpyAsync(parts.data(), part, nb * sizeof(double), hipMemcpyDeviceToHost, op->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(op->stream);
  if (e != hipSuccess || hipGetLastError() != hipSuccess) {
    delete op;
    return fail(EXPW_EDEVICE, "expw_pml_create: device error: %s", hipGetErrorString(e));
  }
  double c2max = -INFINITY;
  for (double v : parts) c2max = std::fmax(c2max, v);
  if (!std::isfinite(c2max)) {
    delete op;
    return fail(EXPW_ENONFINITE, "c2 holds a non-finite or non-positive value");
  }
  op->c2max = c2max;
  expw_pml_spectrum_rectangle(g, c2max, &op->x_lo, &op->B);
  expw_ellipse(op->x_lo, op->B, &op->gamma, &op->c0, &op->c1);
  *out = op;
  return EXPW_OK;
}

int32_t expw_pml_destroy(expw_pml* op) {
  delete op;
  return EXPW_OK;
}

int32_t expw_pml_get_ellipse(const expw_pml* op, double* gamma, double* c0, double* c1) {
  if (int32_t rc = check_pml(op)) return rc;
  if (gamma) *gamma = op->gamma;
  if (c0) *c0 = op->c0;
  if (c1) *c1 = op->c1;
  return EXPW_OK;
}

int32_t expw_pml_apply(expw_pml* op, const void* x, void* y) {
  if (int32_t rc = check_pml(op)) return rc;
  if (!x || !y) return fail(EXPW_EINVAL, "NULL state");
  if (x == y) return fail(EXPW_EINVAL, "y must not alias x");
  const int64_t N = op->g.nx * op->g.ny;
  if (op->g.dtype == EXPW_F32)
    k_pml_apply<float><<<grid_for(N), kBlock, 0, op->stream>>>(make_pml_geo<float>(op), static_cast<const float*>(x), static_cast<float*>(y));
  else
    k_pml_apply<double><<<grid_for(N), kBlock, 0, op->stream>>>(make_pml_geo<double>(op), static_cast<const double*>(x), static_cast<double*>(y));
  return check_launch("pml apply");
}

int32_t expw_pml_set_source_ricker(expw_pml* op, int32_t n_src, const int64_t* idx, const double* amp,
                                   double f_peak, double t_delay, int32_t taylor_p) {
  if (int32_t rc = check_pml(op)) return rc;
  if (n_src < 0 || n_src > EXPW_MAX_SOURCES) return fail(EXPW_EINVAL, "n_src must be in [0, %d]", EXPW_MAX_SOURCES);
  if (n_src == 0) {
    op->n_src = 0;
    return EXPW_OK;
  }
  if (!idx || !amp) return fail(EXPW_EINVAL, "NULL source arrays");
  if (!(f_peak > 0.0) || !std::isfinite(f_peak) || !std::isfinite(t_delay)) return fail(EXPW_EINVAL, "f_peak must be > 0");
  if (taylor_p < 1 || taylor_p > op->pmax) return fail(EXPW_EINVAL, "taylor_p must be in [1, %d] (max_taylor_p at create)", op->pmax);
  const int64_t N = op->g.nx * op->g.ny;
  for (int s = 0; s < n_src; ++s) {
    if (idx[s] < 0 || idx[s] >= N) return fail(EXPW_EINVAL, "source %d index %lld out of range", s, (long long)idx[s]);
    if (!std::isfinite(amp[s])) return fail(EXPW_EINVAL, "source %d amplitude not finite", s);
  }
  std::vector<char> ampbuf(n_src * (op->g.dtype == EXPW_F32 ? 4 : 8));
  for (int s = 0; s < n_src; ++s) {
    if (op->g.dtype == EXPW_F32) reinterpret_cast<float*>(ampbuf.data())[s] = static_cast<float>(amp[s]);
    else reinterpret_cast<double*>(ampbuf.data())[s] = amp[s];
  }
  if (hipMemcpyAsync(op->ws + op->off_src_idx, idx, n_src * sizeof(int64_t), hipMemcpyHostToDevice, op->stream) != hipSuccess ||
      hipMemcpyAsync(op->ws + op->off_src_amp, ampbuf.data(), ampbuf.size(), hipMemcpyHostToDevice, op->stream) != hipSuccess ||
      hipStreamSynchronize(op->stream) != hipSuccess)
    return fail(EXPW_EDEVICE, "source upload failed");
  op->n_src = n_src;
  op->src_lo = *std::min_element(idx, idx + n_src);
  op->src_hi = *std::max_element(idx, idx + n_src);
  op->f_peak = f_peak;
  op->t_delay = t_delay;
  op->taylor_p = taylor_p;
  return EXPW_OK;
}

int32_t expw_pml_set_receivers(expw_pml* op, int32_t n_rec, const int64_t* idx_dev) {
  if (int32_t rc = check_pml(op)) return rc;
  if (n_rec < 0) return fail(EXPW_EINVAL, "n_rec must be >= 0");
  if (n_rec > 0 && !idx_dev) return fail(EXPW_EINVAL, "NULL receiver indices");
  op->n_rec = n_rec;
  op->rec_dev = n_rec > 0 ? idx_dev : nullptr;
  return EXPW_OK;
}

int32_t expw_pml_step_faber(expw_pml* op, void* state, double t0, double dt, int32_t m, int64_t nsteps,
                            void* traces) {
  if (int32_t rc = check_pml(op)) return rc;
  if (!state) return fail(EXPW_EINVAL, "state is NULL");
  if (!(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(t0)) return fail(EXPW_EINVAL, "dt must be > 0");
  if (nsteps < 0) return fail(EXPW_EINVAL, "nsteps must be >= 0");
  if (m < 1 || m > 1024) return fail(EXPW_EINVAL, "Faber degree m must be in [1, 1024]");
  if (op->g.dtype == EXPW_F32)
    return pml_faber_impl<float>(op, static_cast<float*>(state), t0, dt, m, nsteps, static_cast<float*>(traces));
  return pml_faber_impl<double>(op, static_cast<double*>(state), t0, dt, m, nsteps, static_cast<double*>(traces));
}

int32_t expw_pml_step_krylov(expw_pml* op, void* state, double t0, double dt, int32_t k, int64_t nsteps,
                             void* traces) {
  if (int32_t rc = check_pml(op)) return rc;
  if (!state) return fail(EXPW_EINVAL, "state is NULL");
  if (!(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(t0)) return fail(EXPW_EINVAL, "dt must be > 0");
  if (nsteps < 0) return fail(EXPW_EINVAL, "nsteps must be >= 0");
  if (k < 1 || k > op->kmax) return fail(EXPW_EINVAL, "Krylov dimension k must be in [1, %d] (max_krylov_k at create)", op->kmax);
  if (op->g.dtype == EXPW_F32)
    return pml_krylov_impl<float>(op, static_cast<float*>(state), t0, dt, k, nsteps, static_cast<float*>(traces));
  return pml_krylov_impl<double>(op, static_cast<double*>(state), t0, dt, k, nsteps, static_cast<double*>(traces));
}

int32_t expw_pml_step_rk4(expw_pml* op, void* state, double t0, double dt, int64_t nsteps, void* traces) {
  if (int32_t rc = check_pml(op)) return rc;
  if (!state) return fail(EXPW_EINVAL, "state is NULL");
  if (!(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(t0)) return fail(EXPW_EINVAL, "dt must be > 0");
  if (nsteps < 0) return fail(EXPW_EINVAL, "nsteps must be >= 0");
  if (op->g.dtype == EXPW_F32)
    return pml_rk4_impl<float>(op, static_cast<float*>(state), t0, dt, nsteps, static_cast<float*>(traces));
  return pml_rk4_impl<double>(op, static_cast<double*>(state), t0, dt, nsteps, static_cast<double*>(traces));
}

int32_t expw_pml_set_path(expw_pml* op, int32_t path) {
  if (int32_t rc = check_pml(op)) return rc;
  if (path < 0 || path > 4)
    return fail(EXPW_EINVAL,
                "path must be 0 (automatic), 1 (per node), 2 (LDS tiles), 3 (pairs of terms) or 4 (row-streamed passes)");
  op->path = path;
  return EXPW_OK;
}

int32_t expw_pml_path_for(const expw_pml* op, int32_t m, int32_t* path) {
  if (int32_t rc = check_pml(op)) return rc;
  if (!path || m < 1) return fail(EXPW_EINVAL, "invalid argument");
  *path = pml_path_for(op, m);
  return EXPW_OK;
}

int32_t expw_pml_sync_status(expw_pml* op) {
  if (int32_t rc = check_pml(op)) return rc;
  const hipError_t e = hipStreamSynchronize(op->stream);
  if (e != hipSuccess) return fail(EXPW_EDEVICE, "device error: %s", hipGetErrorString(e));
  const hipError_t e2 = hipGetLastError();
  if (e2 != hipSuccess) return fail(EXPW_EDEVICE, "device error: %s", hipGetErrorString(e2));
  return EXPW_OK;
}

}  // extern "C"
