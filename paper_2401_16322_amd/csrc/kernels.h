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
//   acc = (first ? a_first v_{j-1} : acc) + a_j v_j
// cpp is 0 for j = 1, 2 c1 for j = 2 and c1 beyond; the source adds
// src.q * amp_s to the pressure of v_j at each source node.
template <typename T>
struct FaberTerm {
  T inv_gamma, c0, cpp, a_first, a_j;
  int32_t first;
};

// vout may alias vpp and acc_out may alias acc_in or vpp (pointwise reuse);
// vp is read with a halo and must not alias any output. vout == nullptr skips
// storing v_j (last term of a step).
template <typename T, int K, int BC, int DIM>
__global__ __launch_bounds__(kBlock) void k_faber_term(Geo<T, K, DIM> g, const T* vp,
                                                       const T* vpp, T* vout, const T* acc_in,
                                                       T* acc_out, FaberTerm<T> c, Src<T> src) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x;
  if (idx >= g.N) return;
  int64_t ic[3];
  decompose<DIM>(g.n, idx, ic);
  T o[DIM + 1], s[DIM + 1];
  apply_point<T, K, BC, DIM>(g, vp, idx, ic, o, s);
#pragma unroll
  for (int f = 0; f <= DIM; ++f) {
    const int64_t e = f * g.N + idx;
    T v = o[f] * c.inv_gamma - c.c0 * s[f];
    if (vpp) v -= c.cpp * vpp[e];
    if (f == 0) v += src_value(src, idx);
    T acc = c.first ? c.a_first * s[f] : acc_in[e];
    acc += c.a_j * v;
    if (vout) vout[e] = v;
    acc_out[e] = acc;
  }
}

// One classical RK4 stage: k = H y + s(t_stage);
//   ynext = u + cy k (if ynext), acc_out = (acc_in ? acc_in : u) + ca k.
template <typename T, int K, int BC, int DIM>
__global__ __launch_bounds__(kBlock) void k_rk4_stage(Geo<T, K, DIM> g, const T* y, const T* u,
                                                      const T* acc_in, T* ynext, T* acc_out,
                                                      T cy, T ca, Src<T> src) {
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
    acc_out[e] = base + ca * o[f];
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
__global__ __launch_bounds__(kBlock) void k_lf_p(Geo<T, K, DIM> g, T* x, T dt, Src<T> src) {
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
  x[idx] = ((T(1) - half * sp) * pc - dt * g.c2[idx] * div + src_value(src, idx)) /
           (T(1) + half * sp);
}

// traces_row[r] = p[rec[r]]
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather(const T* __restrict__ p,
                                                   const int64_t* __restrict__ rec, int32_t n,
                                                   T* __restrict__ out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] = p[rec[i]];
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
// Basis vectors hold the augmented vector [state | tail(p) | zero pad].

// q0 = [S ; e_p] / beta, beta = sqrt(|S|^2 + tail2) (tail2 = 1 with a source);
// |S|^2 arrives as nin partials of the preceding k_norm2.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_kry_init(const T* __restrict__ S, int64_t ns,
                                                     T* __restrict__ q0, int64_t naug,
                                                     const double* pin, int nin, double tail2,
                                                     double* beta_out) {
  const double b = sqrt(load_reduced<false>(pin, nin) + tail2);
  const double inv = b > 0.0 ? 1.0 / b : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *beta_out = b;
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

// w = H~ q; stores the partials of w . q0 (first Gram-Schmidt coefficient of the column)
template <typename T, int K, int BC, int DIM>
__global__ __launch_bounds__(kBlock) void k_kry_matvec(Geo<T, K, DIM> g, const T* __restrict__ q,
                                                       T* __restrict__ w,
                                                       const T* __restrict__ q0, KrySrc src,
                                                       const T* __restrict__ amp,
                                                       double* __restrict__ pout) {
  const int64_t ns = (DIM + 1) * g.N;
  const int64_t items = g.N + src.p;
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
        w[e] = o[f];
        acc += static_cast<double>(o[f]) * static_cast<double>(q0[e]);
      }
    } else {
      const int c = static_cast<int>(it - g.N);
      const T val = (c + 1 < src.p) ? q[ns + c + 1] : T(0);  // J q_tail
      w[ns + c] = val;
      acc += static_cast<double>(val) * static_cast<double>(q0[ns + c]);
    }
  }
  store_partial<false>(acc, pout);
}

// Modified Gram-Schmidt update fused with the next dot:
//   h = (reduced partials pin), stored to *h_store by block 0;
//   w -= h q_i;  partials of w . qn into pout  (qn == nullptr: w . w)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_kry_mgs(T* __restrict__ w, const T* __restrict__ qi,
                                                    const T* __restrict__ qn, int64_t n,
                                                    const double* __restrict__ pin, int nin,
                                                    double* h_store, double* __restrict__ pout) {
  const double h = load_reduced<false>(pin, nin);
  if (blockIdx.x == 0 && threadIdx.x == 0) *h_store = h;
  double acc = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    const T wt = static_cast<T>(static_cast<double>(w[i]) - h * static_cast<double>(qi[i]));
    w[i] = wt;
    const double o = qn ? static_cast<double>(qn[i]) : static_cast<double>(wt);
    acc += static_cast<double>(wt) * o;
  }
  store_partial<false>(acc, pout);
}

// q_{j+1} = w / h with h = |w| (reduced from the partials of w . w); a column with h <= tol * beta is a
// breakdown: it is zeroed and the host truncates the basis there.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_kry_normalize(T* __restrict__ w, int64_t n,
                                                          const double* __restrict__ pin, int nin,
                                                          double* h_out, const double* beta,
                                                          double tol) {
  const double h = sqrt(load_reduced<false>(pin, nin));
  const double sc = (h > tol * (*beta)) ? 1.0 / h : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *h_out = h;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock)
    w[i] = static_cast<T>(static_cast<double>(w[i]) * sc);
}

struct KryCoef {
  double y[64];
};

// S = beta sum_{c < keff} y_c Q_c (state part)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_kry_combine(T* __restrict__ S,
                                                        const T* __restrict__ Q, int64_t ldq,
                                                        int64_t ns, int32_t keff, KryCoef y,
                                                        double beta) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < ns;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    double acc = 0.0;
    for (int c = 0; c < keff; ++c) acc += y.y[c] * static_cast<double>(Q[c * ldq + i]);
    S[i] = static_cast<T>(beta * acc);
  }
}

}  // namespace expw
