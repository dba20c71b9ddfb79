// Unfused kernels of the hot path: one matrix-vector product of H per HBM
// sweep. Each thread owns one grid point and all its fields.
#pragma once

#include "device_common.h"

namespace expw {

// y = H x
template <typename T, int K, int BC, int DIM>
__global__ __launch_bounds__(kBlock) void k_apply(Geo<T, K, DIM> g, const T* __restrict__ x,
                                                  T* __restrict__ y) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x;
  if (idx >= g.N) return;
  int64_t ic[3];
  decompose<DIM>(g.n, idx, ic);
  T o[DIM + 1], s[DIM + 1];
  apply_point<T, K, BC, DIM>(g, x, idx, ic, o, s);
#pragma unroll
  for (int f = 0; f <= DIM; ++f) y[f * g.N + idx] = o[f];
}

// Coefficients of one Faber term j (Sec. 3.2, Faber recurrence):
//   v_j = (H~ v_{j-1}) / gamma - c0 v_{j-1} - cpp v_{j-2}
//   sum = (first ? a_first v_{j-1} : sum) + a_j v_j
// cpp is 0 for j = 1, 2 c1 for j = 2 and c1 beyond; the source adds
// src.q * amp_s to the pressure of v_j at each source node.
//
// Precision: every term is computed from the stored values of precision T
// with the stencil's difference sums in T over integer weights and
// everything after them in FP64 (apply_point_m), and stored back in T; the
// partial sum is FP64 in memory and the step's result is rounded to T once.
// With FP32 storage two things would otherwise accumulate over many steps:
// weights rounded to FP32 (a slightly different wave speed, the same in
// every term of every step) and the rounding of a partial sum whose terms
// cancel (nearly the same data in consecutive steps rounds nearly the same
// way, so those errors add up coherently).
struct FaberTerm {
  double inv_gamma, c0, cpp, a_first, a_j;
  int32_t first;
};

// The two parts of a weight in T.
template <typename T>
inline void split_weight(double a, T* hi, T* lo) {
  *hi = static_cast<T>(a);
  *lo = static_cast<T>(a - static_cast<double>(*hi));
}

// acc + (hi + lo) x, hi and lo the two parts of one weight.
template <typename T>
__device__ __forceinline__ T add_weighted(T acc, T hi, T lo, T x) {
  acc = fma(hi, x, acc);
  if constexpr (sizeof(T) == 4) acc = fma(lo, x, acc);
  return acc;
}

// vout may alias vpp (pointwise reuse); vp is read with a halo and must not
// alias any output. vout == nullptr skips storing v_j (last term of a step).
// The sum goes to state_out (rounded to T: the step's result) when it is
// given, else to acc_out (FP64; may alias acc_in); both null skips the sum
// (terms recomputed for the adjoint).
template <typename T, int K, int BC, int DIM>
__global__ __launch_bounds__(kBlock) void k_faber_term(Geo<T, K, DIM> g, const T* vp,
                                                       const T* vpp, T* vout,
                                                       const double* acc_in, double* acc_out,
                                                       T* state_out, FaberTerm c, Src<T> src) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x;
  if (idx >= g.N) return;
  int64_t ic[3];
  decompose<DIM>(g.n, idx, ic);
  double o[DIM + 1], s[DIM + 1];
  apply_point_m<T, K, BC, DIM>(g, vp, idx, ic, o, s);
#pragma unroll
  for (int f = 0; f <= DIM; ++f) {
    const int64_t e = f * g.N + idx;
    double v = o[f] * c.inv_gamma - c.c0 * s[f];
    if (vpp) v -= c.cpp * static_cast<double>(vpp[e]);
    if (f == 0) v += src_value_d(src, idx);
    const T vt = static_cast<T>(v);
    if (vout) vout[e] = vt;
    if (acc_out || state_out) {
      // the sum takes the stored term, the one the recurrence continues from
      double acc = c.first ? c.a_first * s[f] : acc_in[e];
      acc = fma(c.a_j, static_cast<double>(vt), acc);
      if (state_out) state_out[e] = static_cast<T>(acc);
      else acc_out[e] = acc;
    }
  }
}

// One classical RK4 stage: k = H y + s(t_stage);
//   ynext = u + cy k (if ynext), acc_out = (acc_in ? acc_in : u) + ca k.
template <typename T, int K, int BC, int DIM>
// (rec: receivers recorded from the pressure written to acc_out, in the last stage)
__global__ __launch_bounds__(kBlock) void k_rk4_stage(Geo<T, K, DIM> g, const T* y, const T* u,
                                                      const T* acc_in, T* ynext, T* acc_out,
                                                      T cy, T ca, Src<T> src, RecRun<T> rec) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x;
  if (idx >= g.N) return;
  int64_t ic[3];
  decompose<DIM>(g.n, idx, ic);
  T o[DIM + 1], s[DIM + 1];
  apply_point<T, K, BC, DIM>(g, y, idx, ic, o, s);
  o[0] += src_value(src, idx);
#pragma unroll
  for (int f = 0; f <= DIM; ++f) {
    const int64_t e = f * g.N + idx;
    const T ue = u ? u[e] : T(0);
    if (ynext) ynext[e] = ue + cy * o[f];
    const T base = acc_in ? acc_in[e] : ue;
    const T r = base + ca * o[f];
    acc_out[e] = r;
    if (f == 0) rec_run_put(rec, idx, r);
  }
}

// Staggered leap-frog, velocity half: v_a <- ((1 - s dt/2) v_a - dt D+_a p) / (1 + s dt/2)
template <typename T, int K, int BC, int DIM>
__global__ __launch_bounds__(kBlock) void k_lf_v(Geo<T, K, DIM> g, T* x, T dt) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x;
  if (idx >= g.N) return;
  int64_t ic[3];
  decompose<DIM>(g.n, idx, ic);
  const T* p = x;
  const T half = T(0.5) * dt;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    T dp = T(0);
#pragma unroll
    for (int l = 1; l <= K; ++l)
      dp += g.w[l - 1] * (ldn<T, BC>(p, idx, ic[a], g.n[a], g.st[a], l) -
                          ldn<T, BC>(p, idx, ic[a], g.n[a], g.st[a], 1 - l));
    const T sg = g.shalf[a][ic[a]];
    T* v = x + (1 + a) * g.N;
    v[idx] = ((T(1) - half * sg) * v[idx] - dt * dp) / (T(1) + half * sg);
  }
}

// Staggered leap-frog, pressure half:
//   p <- ((1 - s_p dt/2) p - dt c2 sum_a D-_a v_a + dt s(t + dt/2)) / (1 + s_p dt/2)
// (src.q carries dt g(t + dt/2) / h^d).
template <typename T, int K, int BC, int DIM>
__global__ __launch_bounds__(kBlock) void k_lf_p(Geo<T, K, DIM> g, T* x, T dt, Src<T> src,
                                                 RecRun<T> rec) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x;
  if (idx >= g.N) return;
  int64_t ic[3];
  decompose<DIM>(g.n, idx, ic);
  T div = T(0), sp = T(0);
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const T* v = x + (1 + a) * g.N;
#pragma unroll
    for (int l = 1; l <= K; ++l)
      div += g.w[l - 1] * (ldn<T, BC>(v, idx, ic[a], g.n[a], g.st[a], l - 1) -
                           ldn<T, BC>(v, idx, ic[a], g.n[a], g.st[a], -l));
    sp += g.sint[a][ic[a]];
  }
  const T half = T(0.5) * dt;
  const T pc = x[idx];
  const T pn = ((T(1) - half * sp) * pc - dt * g.c2[idx] * div + src_value(src, idx)) /
               (T(1) + half * sp);
  x[idx] = pn;
  rec_run_put(rec, idx, pn);
}

// traces_row[r] = p[rec[r]]
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather(const T* __restrict__ p,
                                                   const int64_t* __restrict__ rec, int32_t n,
                                                   T* __restrict__ out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] = p[rec[i]];
}

// Dense output: out[i * n_rec + r] = sum_j coef[i * (m + 1) + j] *
// term[(step_i * (m + 1) + j) * n_rec + r] (FP64 sums); a step index outside
// [0, nsteps) gives NaN. Grid-stride over the n_samples * n_rec items.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dense_combine(int32_t m, int32_t n_rec, int64_t n_samples,
                                                          const int64_t* __restrict__ sample_step,
                                                          const double* __restrict__ coef,
                                                          const T* __restrict__ term, int64_t nsteps,
                                                          T* __restrict__ out) {
  const int64_t items = n_samples * n_rec;
  for (int64_t it = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; it < items;
       it += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int64_t i = it / n_rec, r = it - i * n_rec;
    const int64_t st = sample_step[i];
    double acc = 0.0;
    if (st < 0 || st >= nsteps) {
      acc = __builtin_nan("");
    } else {
      const T* tv = term + st * (m + 1) * n_rec + r;
      const double* c = coef + i * (m + 1);
      for (int j = 0; j <= m; ++j) acc += c[j] * static_cast<double>(tv[static_cast<int64_t>(j) * n_rec]);
    }
    out[it] = static_cast<T>(acc);
  }
}

// max over c2 with non-finite or non-positive entries mapped to +inf
template <typename T>
__global__ __launch_bounds__(kBlock) void k_c2_max(const T* __restrict__ c2, int64_t n,
                                                   double* partials) {
  double m = -INFINITY;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    const double v = static_cast<double>(c2[i]);
    m = fmax(m, (isfinite(v) && v > 0.0) ? v : INFINITY);
  }
  store_partial<true>(m, partials);
}

// ---------------------------------------------------------------- Krylov (Arnoldi)
// Basis vectors hold the augmented vector [state | tail(p) | zero pad]. Column
// j is stored unnormalized as Q_j with its scale s_j = 1 / h_{j,j-1} kept in
// sc[j] (s_0 = 1: Q_0 is normalized), so that q_j = s_j Q_j without a separate
// normalization sweep; a breakdown column has s_j = 0.

// q0 = [S ; e_p] / beta, beta = sqrt(|S|^2 + tail2) (tail2 = 1 with a source);
// |S|^2 arrives as nin partials of the preceding k_norm2.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_kry_init(const T* __restrict__ S, int64_t ns,
                                                     T* __restrict__ q0, int64_t naug,
                                                     const double* pin, int nin, double tail2,
                                                     double* beta_out, double* sc) {
  const double b = sqrt(load_reduced<false>(pin, nin) + tail2);
  const double inv = b > 0.0 ? 1.0 / b : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *beta_out = b;
    sc[0] = 1.0;
  }
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < naug;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    double v = 0.0;
    if (i < ns)
      v = static_cast<double>(S[i]) * inv;
    else if (i == naug - 1 && tail2 > 0.0)
      v = inv;
    q0[i] = static_cast<T>(v);
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_norm2(const T* __restrict__ x, int64_t n,
                                                  double* pout) {
  double acc = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    const double v = static_cast<double>(x[i]);
    acc += v * v;
  }
  store_partial<false>(acc, pout);
}

// Source coupling of the augmented matrix for the Krylov basis: the pressure
// at source s gains amp_s * sum_c G[c] q_tail[c] (G scaled by 1/h^d).
struct KrySrc {
  int32_t n;
  int32_t p;
  int64_t lo, hi;
  const int64_t* idx;
  double G[16];
};

// h_{j,j-1} = sqrt(reduced partials of |w|^2) and s_j = 1/h_{j,j-1}, or 0
// when h_{j,j-1} <= tol * beta (breakdown).
__device__ __forceinline__ double column_scale(const double* pin, int nin, double tol,
                                               const double* beta, double* h_store, double* sc_store) {
  const double h = sqrt(load_reduced<false>(pin, nin));
  const double s = (h > tol * (*beta)) ? 1.0 / h : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *h_store = h;
    *sc_store = s;
  }
  return s;
}

// Column j: w = H~ q_j = s_j H~ Q_j (s_j from the norm partials pin of the
// previous column, or 1 for j = 0 when pin == nullptr); stores the partials of
// w . q_0 (the first Gram-Schmidt coefficient of the column).
template <typename T, int K, int BC, int DIM>
__global__ __launch_bounds__(kBlock) void k_kry_matvec(Geo<T, K, DIM> g, const T* __restrict__ q,
                                                       T* __restrict__ w,
                                                       const T* __restrict__ q0, KrySrc src,
                                                       const T* __restrict__ amp,
                                                       const double* pin, int nin, double tol,
                                                       const double* beta, double* h_store,
                                                       double* sc_store,
                                                       double* __restrict__ pout) {
  const int64_t ns = (DIM + 1) * g.N;
  const int64_t items = g.N + src.p;
  const double sj = pin ? column_scale(pin, nin, tol, beta, h_store, sc_store) : 1.0;
  const T st = static_cast<T>(sj);
  double acc = 0.0;
  for (int64_t it = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; it < items;
       it += static_cast<int64_t>(gridDim.x) * kBlock) {
    if (it < g.N) {
      const int64_t idx = it;
      int64_t ic[3];
      decompose<DIM>(g.n, idx, ic);
      T o[DIM + 1], s[DIM + 1];
      apply_point<T, K, BC, DIM>(g, q, idx, ic, o, s);
      if (src.n > 0 && idx >= src.lo && idx <= src.hi) {
        for (int i = 0; i < src.n; ++i)
          if (src.idx[i] == idx) {
            double gt = 0.0;
            for (int c = 0; c < src.p; ++c) gt += src.G[c] * static_cast<double>(q[ns + c]);
            o[0] += static_cast<T>(gt * static_cast<double>(amp[i]));
          }
      }
#pragma unroll
      for (int f = 0; f <= DIM; ++f) {
        const int64_t e = f * g.N + idx;
        const T v = o[f] * st;
        w[e] = v;
        acc += static_cast<double>(v) * static_cast<double>(q0[e]);
      }
    } else {
      const int c = static_cast<int>(it - g.N);
      const T val = (c + 1 < src.p) ? q[ns + c + 1] * st : T(0);  // J q_tail
      w[ns + c] = val;
      acc += static_cast<double>(val) * static_cast<double>(q0[ns + c]);
    }
  }
  store_partial<false>(acc, pout);
}

// After the last column: h_{k,k-1} and s_k from the norm partials (one block).
__global__ __launch_bounds__(kBlock) void k_kry_finish(const double* pin, int nin, double tol,
                                                       const double* beta, double* h_store,
                                                       double* sc_store) {
  (void)column_scale(pin, nin, tol, beta, h_store, sc_store);
}

struct KryCoef {
  double y[64];
};

// S = beta sum_{c < keff} y_c q_c (state part), q_c = sc[c] Q_c; y, keff and
// beta from the host
template <typename T>
__global__ __launch_bounds__(kBlock) void k_kry_combine(T* __restrict__ S,
                                                        const T* __restrict__ Q, int64_t ldq,
                                                        int64_t ns, int32_t keff, KryCoef y,
                                                        double beta, const double* sc) {
  __shared__ double ys[64];
  if (threadIdx.x < 64) ys[threadIdx.x] = (threadIdx.x < keff) ? y.y[threadIdx.x] * sc[threadIdx.x] : 0.0;
  __syncthreads();
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < ns;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    double acc = 0.0;
    for (int c = 0; c < keff; ++c) acc += ys[c] * static_cast<double>(Q[c * ldq + i]);
    S[i] = static_cast<T>(beta * acc);
  }
}

// The same with y, keff and beta read from device memory (written by k_kry_expm)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_kry_combine_dev(T* __restrict__ S,
                                                            const T* __restrict__ Q, int64_t ldq,
                                                            int64_t ns, const double* y_dev,
                                                            const int* keff_dev,
                                                            const double* beta_dev,
                                                            const double* sc, RecRun<T> rec) {
  __shared__ double y[64];
  const int keff = *keff_dev;
  const double beta = *beta_dev;
  if (threadIdx.x < 64) y[threadIdx.x] = (threadIdx.x < keff) ? y_dev[threadIdx.x] * sc[threadIdx.x] : 0.0;
  __syncthreads();
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < ns;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    double acc = 0.0;
    for (int c = 0; c < keff; ++c) acc += y[c] * static_cast<double>(Q[c * ldq + i]);
    const T v = static_cast<T>(beta * acc);
    S[i] = v;
    rec_run_put(rec, i, v);  // only pressure nodes (i < N) are on the run
  }
}

// C = A B for keff x keff matrices in LDS (leading dimension LD), one
// workgroup; ends with a barrier.
// (A B)_{rc} for matrices in LDS (leading dimension LD): operands are read
// eight at a time ahead of the multiply-adds
template <int LD>
__device__ __forceinline__ double lds_dot(const double* A, const double* B, int r, int c, int n) {
  double acc = 0.0;
  for (int l0 = 0; l0 < n; l0 += 8) {
    double a[8], b[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const bool in = l0 + t < n;
      a[t] = in ? A[r * LD + l0 + t] : 0.0;
      b[t] = in ? B[(l0 + t) * LD + c] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) acc += a[t] * b[t];
  }
  return acc;
}

template <int LD>
__device__ __forceinline__ void lds_matmul(const double* A, const double* B, double* C, int n) {
  for (int e = threadIdx.x; e < n * n; e += kBlock) {
    const int r = e / n, c = e - r * n;
    C[r * LD + c] = lds_dot<LD>(A, B, r, c, n);
  }
  __syncthreads();
}

// y = exp(dt H_keff) e_1 in FP64 on one workgroup, with keff the Krylov
// dimension after the breakdown test h_{j+1,j} <= tol * beta (the leading
// keff x keff block of the upper Hessenberg matrix is used, ld = 64).
// Scaling and squaring: A = dt H / 2^s with |A|_1 <= 1/2, the degree-16
// Taylor polynomial by Horner's rule (truncation below 2^-17 / 17!), then s
// squarings; y is the first column. The number of products is bounded by
// 15 + s with s <= 1100 for any finite matrix; a non-finite matrix yields NaN.
// (The augmented source block makes |dt H_k| large, of order dt |W|, so the
// squarings are what keeps the cost logarithmic in the norm.)
__global__ __launch_bounds__(kBlock) void k_kry_expm(const double* __restrict__ hess, int k,
                                                     double dt, double tol,
                                                     const double* __restrict__ beta_p,
                                                     double* __restrict__ y_out,
                                                     int* __restrict__ keff_out) {
  constexpr int LD = 65;
  __shared__ double A[64 * LD], T[64 * LD], W[64 * LD];
  __shared__ double cs[64], sub[64];
  __shared__ int s_keff, s_sq;
  const int tid = threadIdx.x;
  // the subdiagonal is loaded in parallel, then scanned in LDS. Only the
  // columns 0..k-2 are read: a breakdown in the last column would give
  // k_eff = k anyway, and the persistent Arnoldi kernel does not produce
  // h_{k,k-1} (its entry holds an older value)
  if (tid < k - 1) sub[tid] = hess[(tid + 1) * 64 + tid];
  const double beta = *beta_p;
  __syncthreads();
  if (tid == 0) {
    int ke = k;
    if (!(beta > 0.0)) {
      ke = 0;
    } else {
      for (int j = 0; j + 1 < k; ++j)
        if (!(sub[j] > tol * beta)) {
          ke = j + 1;
          break;
        }
    }
    s_keff = ke;
  }
  __syncthreads();
  const int n = s_keff;
  for (int e = tid; e < n * n; e += kBlock) {
    const int r = e / n, c = e - r * n;
    A[r * LD + c] = (r <= c + 1) ? dt * hess[r * 64 + c] : 0.0;
  }
  __syncthreads();
  if (tid < n) {
    double sc = 0.0;
    for (int r = 0; r < n; ++r) sc += fabs(A[r * LD + tid]);
    cs[tid] = sc;
  }
  __syncthreads();
  if (tid == 0) {
    double nm = 0.0;
    for (int c = 0; c < n; ++c) nm = fmax(nm, cs[c]);
    int sq = -1;  // -1: non-finite
    if (isfinite(nm)) {
      sq = 0;
      while (nm > 0.5 && sq < 1100) {
        nm *= 0.5;
        ++sq;
      }
    }
    s_sq = sq;
  }
  __syncthreads();
  const int sq = s_sq;
  if (sq < 0) {
    if (tid < 64) y_out[tid] = NAN;
    if (tid == 0) *keff_out = n;
    return;
  }
  const double scale = ldexp(1.0, -sq);
  for (int e = tid; e < n * n; e += kBlock) {
    const int r = e / n, c = e - r * n;
    A[r * LD + c] *= scale;
    T[r * LD + c] = (r == c ? 1.0 : 0.0) + A[r * LD + c] / 16.0;
  }
  __syncthreads();
  // Horner: P <- I + A P / j for j = 15 .. 1, alternating between T and W
  double* cur = T;
  double* nxt = W;
  for (int j = 15; j >= 1; --j) {
    const double inv = 1.0 / j;
    for (int e = tid; e < n * n; e += kBlock) {
      const int r = e / n, c = e - r * n;
      nxt[r * LD + c] = (r == c ? 1.0 : 0.0) + lds_dot<LD>(A, cur, r, c, n) * inv;
    }
    __syncthreads();
    double* t = cur;
    cur = nxt;
    nxt = t;
  }
  // squarings
  for (int i = 0; i < sq; ++i) {
    lds_matmul<LD>(cur, cur, nxt, n);
    double* t = cur;
    cur = nxt;
    nxt = t;
  }
  if (tid < 64) y_out[tid] = (tid < n) ? cur[tid * LD + 0] : 0.0;
  if (tid == 0) *keff_out = n;
}

// Non-finite guard: sets *flag when any of the n values is NaN or infinite
// (vector atomic store; the flag is only ever set here).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_guard(const T* __restrict__ x, int64_t n, int* flag) {
  bool bad = false;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock)
    bad = bad || !isfinite(x[i]);
  if (bad) __hip_atomic_store(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace expw
