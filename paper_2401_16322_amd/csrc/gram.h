// Gram-Schmidt of the launch-per-column Arnoldi process in four launches
// per column, for vectors too large for the persistent kernel (Sec. 3.2,
// Krylov subspace projection). As in the persistent kernel, modified
// Gram-Schmidt's projections h_{i,j} = <w - sum_{l<i} h_{l,j} q_l, q_i> are
// taken from one batched reduction: h_{i,j} = r_i - sum_{l<i} h_{l,j}
// <q_l, q_i> with r_i = <w, q_i> (an identity for any basis, not only an
// exactly orthonormal one), so a column needs
//   k_gram_dots:   one sweep over w and Q_0..Q_j, block partials of r_i
//                  (i <= j) and of the new Gram row <q_j, q_l> (l < j);
//   k_gram_reduce: one workgroup per value sums its partials in block order;
//   k_gram_subst:  one thread stores the Gram row and runs the forward
//                  substitution;
//   k_gram_update: one sweep applying w -= h_i q_i in MGS's order (rounded to
//                  T after each, as the literal MGS kernels do) and the block
//                  partials of |w|^2 (the next column's scale);
// instead of j + 1 launches that each stream w, q_i and q_{i+1}. The columns
// are stored unnormalized with their scales sc (q_i = sc[i] Q_i), as in the
// other Arnoldi paths. Every sum across threads is FP64 and in a fixed order.
#pragma once

#include "device_common.h"
#include "expwave.h"

namespace expw {

constexpr int kGramChunk = 16;            // columns per accumulation sweep of k_gram_dots
constexpr int kGramPartials = 640 * 127;  // doubles of block partials (grid x (2j + 1) <= this)
constexpr int kGramMaxBlocks = 2048;      // grid cap of k_gram_dots
constexpr int kGramLd = EXPW_MAX_KRYLOV + 1;  // leading dimension of the Gram table
constexpr int kGramTot = kGramLd * kGramLd;   // offset of the 2j + 1 totals after the table

// Workgroups of k_gram_dots for column j: as many as the partials area holds
// for its 2j + 1 values, at most kGramMaxBlocks and one per 1024 elements.
inline unsigned gram_dots_grid(int64_t n, int j) {
  int64_t nb = kGramPartials / (2 * j + 1);
  if (nb > kGramMaxBlocks) nb = kGramMaxBlocks;
  const int64_t need = (n + 4 * kBlock - 1) / (4 * kBlock);
  if (nb > need) nb = need;
  return static_cast<unsigned>(nb < 1 ? 1 : nb);
}

// Block partials of r_i = sum_e w_e Q_i,e (i = 0..j) and of
// sum_e Q_j,e Q_l,e (l = 0..j-1), unscaled, at pout[block * (2j + 1) + v]
// (v = i for r_i, v = j + 1 + l for the Gram row).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gram_dots(const T* __restrict__ w, const T* __restrict__ Q,
                                                      int64_t ld, int64_t n, int j, double* __restrict__ pout) {
  const int nv = 2 * j + 1;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  const T* qj = Q + j * ld;
  for (int c0 = 0; c0 <= j; c0 += kGramChunk) {
    const int ci = min(kGramChunk, j + 1 - c0);  // r_i, i = c0 .. c0 + ci - 1
    double ar[kGramChunk], ag[kGramChunk];
#pragma unroll
    for (int u = 0; u < kGramChunk; ++u) ar[u] = ag[u] = 0.0;
    for (int64_t e = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; e < n; e += stride) {
      const double we = static_cast<double>(w[e]);
      const double je = static_cast<double>(qj[e]);
#pragma unroll
      for (int u = 0; u < kGramChunk; ++u)
        if (u < ci) {
          const double v = static_cast<double>(Q[(c0 + u) * ld + e]);
          ar[u] += we * v;
          ag[u] += je * v;
        }
    }
#pragma unroll
    for (int u = 0; u < kGramChunk; ++u) {
      if (u >= ci) break;  // block-uniform
      const double sr = block_reduce<false>(ar[u]);
      const double sg = block_reduce<false>(ag[u]);
      if (threadIdx.x == 0) {
        const int i = c0 + u;
        pout[static_cast<int64_t>(blockIdx.x) * nv + i] = sr;
        if (i < j) pout[static_cast<int64_t>(blockIdx.x) * nv + j + 1 + i] = sg;
      }
    }
  }
}

// The totals of the 2j + 1 values over the nb block partials: workgroup v
// sums value v (each thread every 256th block, then the fixed block tree).
__global__ __launch_bounds__(kBlock) void k_gram_reduce(const double* __restrict__ pin, int nb, int nv,
                                                        double* __restrict__ tot) {
  const int v = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += kBlock) acc += pin[static_cast<int64_t>(b) * nv + v];
  const double t = block_reduce<false>(acc);
  if (threadIdx.x == 0) tot[v] = t;
}

// One thread: r_i = sc_i t_i, the Gram row <q_j, q_l> = sc_j sc_l t_{j+1+l}
// into gram[j][l], the forward substitution h_i = r_i - sum_{l<i} h_l
// <q_i, q_l>, h_i into the Hessenberg column j and h_i sc_i (the factor of the
// unnormalized Q_i) into hs[i].
__global__ __launch_bounds__(64) void k_gram_subst(const double* __restrict__ tot, int j,
                                                   const double* __restrict__ sc, double* gram, double* hess,
                                                   int hess_ld, double* hs) {
  if (threadIdx.x != 0) return;
  double h[EXPW_MAX_KRYLOV];
  for (int l = 0; l < j; ++l) gram[j * kGramLd + l] = sc[j] * sc[l] * tot[j + 1 + l];
  for (int i = 0; i <= j; ++i) {
    double r = sc[i] * tot[i];
    for (int l = 0; l < i; ++l) r -= h[l] * gram[i * kGramLd + l];
    h[i] = r;
    hess[i * hess_ld + j] = r;
    hs[i] = r * sc[i];
  }
}

// w -= hs_i Q_i for i = 0..j in order (each rounded to T), and the block
// partials of |w|^2 into pout[block].
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gram_update(T* __restrict__ w, const T* __restrict__ Q, int64_t ld,
                                                        int64_t n, int j, const double* __restrict__ hs,
                                                        double* __restrict__ pout) {
  __shared__ double s_hs[EXPW_MAX_KRYLOV];
  if (threadIdx.x <= j) s_hs[threadIdx.x] = hs[threadIdx.x];
  __syncthreads();
  double acc = 0.0;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; e < n;
       e += static_cast<int64_t>(gridDim.x) * kBlock) {
    T x = w[e];
    for (int i = 0; i <= j; ++i)
      x = static_cast<T>(static_cast<double>(x) - s_hs[i] * static_cast<double>(Q[i * ld + e]));
    w[e] = x;
    acc += static_cast<double>(x) * static_cast<double>(x);
  }
  store_partial<false>(acc, pout);
}

}  // namespace expw
