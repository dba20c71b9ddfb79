// Adjoint of the Faber step (Sec. 3.2, Faber recurrence, transposed) and of
// the operator: the kernels of a reverse sweep for gradients with respect to
// c^2. With (D+)^T = -D- (zero ghosts or periodic),
//   (H^T y)_p   = sum_a D-_a y_{v_a} - sigma_p y_p
//   (H^T y)_v_a = D+_a (c^2 y_p) - sigma_a(half) y_{v_a}
// and for u' = sum_j a_j v_j (v_j = A v_{j-1} - c_j v_{j-2}, A = H/gamma - c0)
// the derivatives mu_j of <lam, u'> with respect to v_j run from j = m down:
//   mu_j = a_j lam + A^T mu_{j+1} - c_{j+2} mu_{j+2},
// with d<lam, u'>/du = mu_0 and
//   d<lam, u'>/dc^2 = -(1/gamma) sum_{j>=1} mu_{j,p} (sum_a D-_a v_{j-1,a}).
// As in the forward step, every reverse term is computed in FP64 from the
// stored values and stored in T (see FaberTerm).
#pragma once

#include "device_common.h"
#include "expwave.h"
#include "kernels.h"

namespace expw {

// (H^T y) at one point for every field; self = y at the point.
template <typename T, int K, int BC, int DIM>
__device__ __forceinline__ void apply_point_adjoint(const Geo<T, K, DIM>& g,
                                                    const T* __restrict__ y, int64_t idx,
                                                    const int64_t* ic, T* out, T* self) {
  const T* __restrict__ p = y;
  const T pc = p[idx];
  self[0] = pc;
  T div = T(0), sp = T(0);
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const T* __restrict__ v = y + (1 + a) * g.N;
    T dv = T(0), dcp = T(0);
#pragma unroll
    for (int l = 1; l <= K; ++l) {
      dv += g.w[l - 1] * (ldn<T, BC>(v, idx, ic[a], g.n[a], g.st[a], l - 1) -
                          ldn<T, BC>(v, idx, ic[a], g.n[a], g.st[a], -l));
      dcp += g.w[l - 1] * (ldn<T, BC>(g.c2, idx, ic[a], g.n[a], g.st[a], l) *
                               ldn<T, BC>(p, idx, ic[a], g.n[a], g.st[a], l) -
                           ldn<T, BC>(g.c2, idx, ic[a], g.n[a], g.st[a], 1 - l) *
                               ldn<T, BC>(p, idx, ic[a], g.n[a], g.st[a], 1 - l));
    }
    div += dv;
    sp += g.sint[a][ic[a]];
    const T vc = v[idx];
    self[1 + a] = vc;
    out[1 + a] = dcp - g.shalf[a][ic[a]] * vc;
  }
  out[0] = div - sp * pc;
}

// (H^T y) at one point in FP64 from stored values of precision T.
template <typename T, int K, int BC, int DIM>
__device__ __forceinline__ void apply_point_adjoint_d(const Geo<T, K, DIM>& g,
                                                      const T* __restrict__ y, int64_t idx,
                                                      const int64_t* ic, double* out,
                                                      double* self) {
  const T* __restrict__ p = y;
  const double pc = static_cast<double>(p[idx]);
  self[0] = pc;
  double div = 0.0, sp = 0.0;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const T* __restrict__ v = y + (1 + a) * g.N;
    double dv = 0.0, dcp = 0.0;
#pragma unroll
    for (int l = 1; l <= K; ++l) {
      dv += g.wd[l - 1] * (static_cast<double>(ldn<T, BC>(v, idx, ic[a], g.n[a], g.st[a], l - 1)) -
                           static_cast<double>(ldn<T, BC>(v, idx, ic[a], g.n[a], g.st[a], -l)));
      dcp += g.wd[l - 1] *
             (static_cast<double>(ldn<T, BC>(g.c2, idx, ic[a], g.n[a], g.st[a], l)) *
                  static_cast<double>(ldn<T, BC>(p, idx, ic[a], g.n[a], g.st[a], l)) -
              static_cast<double>(ldn<T, BC>(g.c2, idx, ic[a], g.n[a], g.st[a], 1 - l)) *
                  static_cast<double>(ldn<T, BC>(p, idx, ic[a], g.n[a], g.st[a], 1 - l)));
    }
    div += dv;
    sp += static_cast<double>(g.sint[a][ic[a]]);
    const double vc = static_cast<double>(v[idx]);
    self[1 + a] = vc;
    out[1 + a] = dcp - static_cast<double>(g.shalf[a][ic[a]]) * vc;
  }
  out[0] = div - sp * pc;
}

// sum_a D-_a v_a at one point in FP64 (the factor of c^2 in the pressure row of H).
template <typename T, int K, int BC, int DIM>
__device__ __forceinline__ double velocity_divergence_d(const Geo<T, K, DIM>& g,
                                                        const T* __restrict__ x, int64_t idx,
                                                        const int64_t* ic) {
  double div = 0.0;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const T* __restrict__ v = x + (1 + a) * g.N;
#pragma unroll
    for (int l = 1; l <= K; ++l)
      div += g.wd[l - 1] * (static_cast<double>(ldn<T, BC>(v, idx, ic[a], g.n[a], g.st[a], l - 1)) -
                            static_cast<double>(ldn<T, BC>(v, idx, ic[a], g.n[a], g.st[a], -l)));
  }
  return div;
}

// sum_a D-_a v_a at one point (the factor of c^2 in the pressure row of H).
template <typename T, int K, int BC, int DIM>
__device__ __forceinline__ T velocity_divergence(const Geo<T, K, DIM>& g, const T* __restrict__ x,
                                                 int64_t idx, const int64_t* ic) {
  T div = T(0);
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const T* __restrict__ v = x + (1 + a) * g.N;
#pragma unroll
    for (int l = 1; l <= K; ++l)
      div += g.w[l - 1] * (ldn<T, BC>(v, idx, ic[a], g.n[a], g.st[a], l - 1) -
                           ldn<T, BC>(v, idx, ic[a], g.n[a], g.st[a], -l));
  }
  return div;
}

// y = H^T x
template <typename T, int K, int BC, int DIM>
__global__ __launch_bounds__(kBlock) void k_apply_adjoint(Geo<T, K, DIM> g, const T* __restrict__ x,
                                                          T* __restrict__ y) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x;
  if (idx >= g.N) return;
  int64_t ic[3];
  decompose<DIM>(g.n, idx, ic);
  T o[DIM + 1], s[DIM + 1];
  apply_point_adjoint<T, K, BC, DIM>(g, x, idx, ic, o, s);
#pragma unroll
  for (int f = 0; f <= DIM; ++f) y[f * g.N + idx] = o[f];
}

// Coefficients of one reverse term j: mu_j = a_j lam + (H^T mu1)/gamma
// - c0 mu1 - cnext mu2 (cnext = c_{j+2}).
struct AdjointTerm {
  double inv_gamma, c0, cnext, a_j;
};

// One reverse term. mu1 (read with a halo) and mu2 may be NULL (zero);
// vprev = v_{j-1} (read with a halo) and grad are NULL for j = 0. mu_out may
// alias lam (pointwise); it must not alias mu1, mu2 or vprev.
template <typename T, int K, int BC, int DIM>
__global__ __launch_bounds__(kBlock) void k_faber_adjoint_term(Geo<T, K, DIM> g, const T* mu1,
                                                               const T* mu2, const T* lam,
                                                               const T* vprev, T* mu_out, T* grad,
                                                               AdjointTerm c) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x;
  if (idx >= g.N) return;
  int64_t ic[3];
  decompose<DIM>(g.n, idx, ic);
  double o[DIM + 1], s[DIM + 1];
  if (mu1) {
    apply_point_adjoint_d<T, K, BC, DIM>(g, mu1, idx, ic, o, s);
  } else {
#pragma unroll
    for (int f = 0; f <= DIM; ++f) o[f] = s[f] = 0.0;
  }
  double mp = 0.0;
#pragma unroll
  for (int f = 0; f <= DIM; ++f) {
    const int64_t e = f * g.N + idx;
    double mu = c.a_j * static_cast<double>(lam[e]);
    mu += o[f] * c.inv_gamma - c.c0 * s[f];
    if (mu2) mu -= c.cnext * static_cast<double>(mu2[e]);
    const T mt = static_cast<T>(mu);
    mu_out[e] = mt;
    if (f == 0) mp = static_cast<double>(mt);
  }
  if (grad)
    grad[idx] = static_cast<T>(static_cast<double>(grad[idx]) -
                               c.inv_gamma * mp * velocity_divergence_d<T, K, BC, DIM>(g, vprev, idx, ic));
}

// Two reverse terms per launch on 2D grids with zero ghosts: mu_j and
// mu_{j-1} (j - 1 >= 1), with the gradient contributions of both. A
// workgroup owns a kAdjTX x kAdjTZ tile, one thread per tile point. Phase 1
// computes mu_j on the tile grown by K (the reach of H^T) exactly as
// k_faber_adjoint_term does, from mu1 = mu_{j+1} and mu2 = mu_{j+2} in
// global memory, and keeps it, rounded to T, in LDS (zero outside the grid,
// the ghost rule). Phase 2 applies H^T to mu_j from LDS, forms mu_{j-1} on
// the tile, stores both terms and updates the gradient with term j, then
// term j - 1. Every value takes the arithmetic of k_faber_adjoint_term in the
// same order; the launches and the reads of lam and grad are halved. mu1 and
// mu2 may be NULL (zero); vprev1 = v_{j-1}, vprev2 = v_{j-2}. mu_j and
// mu_{j-1} must not alias mu1, mu2, lam, the vprev or each other.
constexpr int kAdjTX = 64, kAdjTZ = 16, kAdjNT = kAdjTX * kAdjTZ;  // one thread per tile point

template <typename T, int K>
__global__ __launch_bounds__(kAdjNT) void k_faber_adjoint_pair(Geo<T, K, 2> g, const T* mu1, const T* mu2,
                                                               const T* __restrict__ lam,
                                                               const T* __restrict__ vprev1,
                                                               const T* __restrict__ vprev2, T* mu_j, T* mu_jm1,
                                                               T* __restrict__ grad, AdjointTerm c1,
                                                               AdjointTerm c2, int32_t tiles_x) {
  constexpr int GX = kAdjTX + 2 * K, GZ = kAdjTZ + 2 * K;
  __shared__ T sm[3][GX * GZ];  // mu_j on the grown tile: p, v_x, v_z
  const int bx = static_cast<int>(blockIdx.x) % tiles_x, bz = static_cast<int>(blockIdx.x) / tiles_x;
  const int64_t nx = g.n[0], nz = g.n[1];
  const int64_t x0 = static_cast<int64_t>(bx) * kAdjTX, z0 = static_cast<int64_t>(bz) * kAdjTZ;
  // phase 1: mu_j on the grown tile
  for (int i = threadIdx.x; i < GX * GZ; i += kAdjNT) {
    const int64_t x = x0 - K + i % GX, z = z0 - K + i / GX;
    if (x < 0 || x >= nx || z < 0 || z >= nz) {
      sm[0][i] = sm[1][i] = sm[2][i] = T(0);
      continue;
    }
    const int64_t idx = z * nx + x;
    const int64_t ic[3] = {x, z, 0};
    double o[3], s[3];
    if (mu1) {
      apply_point_adjoint_d<T, K, 0, 2>(g, mu1, idx, ic, o, s);
    } else {
#pragma unroll
      for (int f = 0; f < 3; ++f) o[f] = s[f] = 0.0;
    }
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const int64_t e = f * g.N + idx;
      double mu = c1.a_j * static_cast<double>(lam[e]);
      mu += o[f] * c1.inv_gamma - c1.c0 * s[f];
      if (mu2) mu -= c1.cnext * static_cast<double>(mu2[e]);
      sm[f][i] = static_cast<T>(mu);
    }
  }
  __syncthreads();
  // phase 2: mu_{j-1} on the tile
  {
    const int i = threadIdx.x;
    const int64_t x = x0 + i % kAdjTX, z = z0 + i / kAdjTX;
    if (x >= nx || z >= nz) return;
    const int64_t idx = z * nx + x;
    const int64_t ic[3] = {x, z, 0};
    const int l = (i / kAdjTX + K) * GX + (i % kAdjTX + K);  // the point in the grown tile
    // H^T mu_j at the point, as apply_point_adjoint_d with LDS neighbours
    double o[3], s[3];
    {
      const double pc = static_cast<double>(sm[0][l]);
      s[0] = pc;
      double div = 0.0, sp = 0.0;
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const T* v = sm[1 + a];
        const int ls = a == 0 ? 1 : GX;
        double dv = 0.0, dcp = 0.0;
#pragma unroll
        for (int q = 1; q <= K; ++q) {
          dv += g.wd[q - 1] * (static_cast<double>(v[l + (q - 1) * ls]) - static_cast<double>(v[l - q * ls]));
          dcp += g.wd[q - 1] *
                 (static_cast<double>(ldn<T, 0>(g.c2, idx, ic[a], g.n[a], g.st[a], q)) *
                      static_cast<double>(sm[0][l + q * ls]) -
                  static_cast<double>(ldn<T, 0>(g.c2, idx, ic[a], g.n[a], g.st[a], 1 - q)) *
                      static_cast<double>(sm[0][l + (1 - q) * ls]));
        }
        div += dv;
        sp += static_cast<double>(g.sint[a][ic[a]]);
        const double vc = static_cast<double>(v[l]);
        s[1 + a] = vc;
        o[1 + a] = dcp - static_cast<double>(g.shalf[a][ic[a]]) * vc;
      }
      o[0] = div - sp * pc;
    }
    double mp = 0.0;
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const int64_t e = f * g.N + idx;
      mu_j[e] = sm[f][l];
      double mu = c2.a_j * static_cast<double>(lam[e]);
      mu += o[f] * c2.inv_gamma - c2.c0 * s[f];
      if (mu1) mu -= c2.cnext * static_cast<double>(mu1[e]);
      const T mt = static_cast<T>(mu);
      mu_jm1[e] = mt;
      if (f == 0) mp = static_cast<double>(mt);
    }
    const T g1 = static_cast<T>(static_cast<double>(grad[idx]) -
                                c1.inv_gamma * static_cast<double>(sm[0][l]) *
                                    velocity_divergence_d<T, K, 0, 2>(g, vprev1, idx, ic));
    grad[idx] = static_cast<T>(static_cast<double>(g1) -
                               c2.inv_gamma * mp * velocity_divergence_d<T, K, 0, 2>(g, vprev2, idx, ic));
  }
}

// Krylov adjoint (Sec. 3.2, Krylov subspace projection, differentiated): the
// state adjoint is the Krylov approximation of exp(dt H^T) lam (Arnoldi on
// H^T from lam, no augmentation), and the c^2 derivative of
// <lam, exp(dt H~) [u; e_p]> is
//   dt int_0^1 <exp((1-s) dt H^T) lam, dH/dc^2[x] exp(s dt H~) [u; e_p]> ds
//   = -dt sum_{a,b} C_ab W_{a,p}[x] (sum_d D-_d V_{b,v_d})[x]
// with V, W the two bases and C = beta beta' int_0^1 exp((1-s) dt G_k) e_1
// e_1^T exp(s dt H_k^T) ds (formed on the host from one block exponential).

// Column j of the Arnoldi process on H^T: w = s_j H^T Q_j (s_j from the norm
// partials pin of the previous column, or 1 for j = 0 when pin == nullptr),
// in FP64 from the stored values; stores the partials of w . q_0.
template <typename T, int K, int BC, int DIM>
__global__ __launch_bounds__(kBlock) void k_kry_matvec_adj(Geo<T, K, DIM> g, const T* __restrict__ q,
                                                           T* __restrict__ w, const T* __restrict__ q0,
                                                           const double* pin, int nin, double tol,
                                                           const double* beta, double* h_store,
                                                           double* sc_store, double* __restrict__ pout) {
  const double sj = pin ? column_scale(pin, nin, tol, beta, h_store, sc_store) : 1.0;
  double acc = 0.0;
  for (int64_t idx = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; idx < g.N;
       idx += static_cast<int64_t>(gridDim.x) * kBlock) {
    int64_t ic[3];
    decompose<DIM>(g.n, idx, ic);
    double o[DIM + 1], s[DIM + 1];
    apply_point_adjoint_d<T, K, BC, DIM>(g, q, idx, ic, o, s);
#pragma unroll
    for (int f = 0; f <= DIM; ++f) {
      const int64_t e = f * g.N + idx;
      const T v = static_cast<T>(o[f] * sj);
      w[e] = v;
      acc += static_cast<double>(v) * static_cast<double>(q0[e]);
    }
  }
  store_partial<false>(acc, pout);
}

// grad[x] += scale * sum_{a < kw} W_a,p[x] sum_{b < kv} M[a kv + b]
// (sum_d D-_d V_b,v_d)[x] for the unnormalized basis columns V_b (leading
// dimension ldv) and W_a (ldw); M (kw x kv, row-major, FP64) carries the
// column scales. The divergences are formed eight columns at a time.
template <typename T, int K, int BC, int DIM>
__global__ __launch_bounds__(kBlock) void k_kry_grad(Geo<T, K, DIM> g, const T* __restrict__ V,
                                                     int64_t ldv, int32_t kv, const T* __restrict__ W,
                                                     int64_t ldw, int32_t kw,
                                                     const double* __restrict__ M, double scale,
                                                     T* __restrict__ grad) {
  __shared__ double sm[EXPW_MAX_KRYLOV * EXPW_MAX_KRYLOV];
  for (int i = threadIdx.x; i < kw * kv; i += kBlock) sm[i] = M[i];
  __syncthreads();
  const int64_t idx = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x;
  if (idx >= g.N) return;
  int64_t ic[3];
  decompose<DIM>(g.n, idx, ic);
  constexpr int CB = 8;
  double acc = 0.0;
  for (int b0 = 0; b0 < kv; b0 += CB) {
    double d[CB];
#pragma unroll
    for (int u = 0; u < CB; ++u)
      d[u] = (b0 + u < kv) ? velocity_divergence_d<T, K, BC, DIM>(g, V + (b0 + u) * ldv, idx, ic) : 0.0;
    const int nb = min(CB, kv - b0);
    for (int a = 0; a < kw; ++a) {
      const double* row = sm + a * kv + b0;
      double t = 0.0;
#pragma unroll
      for (int u = 0; u < CB; ++u)
        if (u < nb) t += row[u] * d[u];
      acc += static_cast<double>(W[a * ldw + idx]) * t;
    }
  }
  grad[idx] = static_cast<T>(static_cast<double>(grad[idx]) + scale * acc);
}

// state_p[rec[r]] += scale * vals[r] (adjoint sources at the receivers;
// repeated receivers add up).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scatter_add(const T* __restrict__ vals,
                                                        const int64_t* __restrict__ rec, int32_t n,
                                                        T scale, T* state) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) atomicAdd(state + rec[i], scale * vals[i]);
}

}  // namespace expw
