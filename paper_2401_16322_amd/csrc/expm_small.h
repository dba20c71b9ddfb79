// y = exp(dt H_keff) e_1 for Krylov dimensions k <= 32 (Sec. 3.2, the
// exponential of the small projected matrix), one workgroup of TS x TS
// threads for tiles of TS = 16 or 32.
//
// The same arithmetic as k_kry_expm (breakdown test, 1-norm scaling to
// |A|_1 <= 1/2, degree-16 Taylor polynomial by Horner's rule, s squarings,
// each product summed over l = 0, 1, ... in order), laid out for the small
// case: thread t owns entry (t / TS, t % TS) of every TS x TS matrix, the
// keff x keff matrices sit in the leading block of zero-padded TS x TS tiles,
// and every product is an unrolled TS-term dot product whose LDS operands are
// loaded 16 at a time. The padding leaves the leading block unchanged
// (A is zero outside it, so the Horner iterate and its squares stay
// block-diagonal with an identity trailing block), and a product against a
// zero operand adds an exact zero, so the leading block holds the values that
// k_kry_expm computes.
#pragma once

#include "device_common.h"

namespace expw {

constexpr int kExpmSmallK = 32;  // largest k of the tiled kernels

// 1 / j for the Horner steps j = 1..15 (correctly rounded at compile time,
// the value a run-time division gives)
__device__ constexpr double kInvJ[16] = {0.0,        1.0 / 1,  1.0 / 2,  1.0 / 3,  1.0 / 4,  1.0 / 5,
                                         1.0 / 6,    1.0 / 7,  1.0 / 8,  1.0 / 9,  1.0 / 10, 1.0 / 11,
                                         1.0 / 12,   1.0 / 13, 1.0 / 14, 1.0 / 15};

// (X Y)_{rc} over TS x TS tiles in LDS (row-major, ld TS), summed over
// l = 0 .. TS-1 in order
template <int TS>
__device__ __forceinline__ double tile_dot(const double* X, const double* Y, int r, int c) {
  double acc = 0.0;
#pragma unroll
  for (int l0 = 0; l0 < TS; l0 += 16) {
    double x[16], y[16];
#pragma unroll
    for (int l = 0; l < 16; ++l) {
      x[l] = X[r * TS + l0 + l];
      y[l] = Y[(l0 + l) * TS + c];
    }
#pragma unroll
    for (int l = 0; l < 16; ++l) acc += x[l] * y[l];
  }
  return acc;
}

// hess: (k + 1) x k upper Hessenberg matrix, leading dimension 64; requires
// 1 <= k <= TS and blockDim.x == TS * TS. Outputs as k_kry_expm: y_out[0..63]
// (zero beyond keff, NaN if dt H is not finite) and *keff_out.
template <int TS>
__global__ __launch_bounds__(TS * TS) void k_kry_expm_tile(const double* __restrict__ hess, int k,
                                                          double dt, double tol,
                                                          const double* __restrict__ beta_p,
                                                          double* __restrict__ y_out,
                                                          int* __restrict__ keff_out) {
  static_assert(TS == 16 || TS == 32, "tiles of 16 x 16 or 32 x 32");
  __shared__ double A[TS * TS], P0[TS * TS], P1[TS * TS];
  __shared__ int s_keff, s_sq;
  const int tid = threadIdx.x;
  const int r = tid / TS, c = tid % TS;
  const int lane = tid & 63;
  // the entry this thread owns, loaded while wave 0 finds keff
  const double hrc = (r < k && c < k && r <= c + 1) ? hess[r * 64 + c] : 0.0;
  if (tid < 64) {
    // keff: one more than the first column whose subdiagonal entry fails the
    // breakdown test, else k (0 when beta is not positive). Columns 0..k-2
    // only: a breakdown in the last column gives keff = k anyway, and the
    // persistent Arnoldi kernel does not produce h_{k,k-1}
    const double beta = *beta_p;
    const bool brk = lane + 1 < k && !(hess[(lane + 1) * 64 + lane] > tol * beta);
    const unsigned long long m = __ballot(brk);
    int ke = m ? __ffsll(static_cast<long long>(m)) : k;
    if (!(beta > 0.0)) ke = 0;
    if (lane == 0) s_keff = ke;
  }
  __syncthreads();
  const int n = s_keff;
  const double a = (r < n && c < n) ? dt * hrc : 0.0;
  A[tid] = a;
  __syncthreads();
  if (tid < 64) {
    // 1-norm: largest column sum of |A| (columns summed over r in order)
    double cs = 0.0;
    if (lane < TS) {
      for (int i = 0; i < TS; ++i) cs += fabs(A[i * TS + lane]);
    }
    double nm = cs;
    for (int off = 32; off >= 1; off >>= 1) nm = fmax(nm, __shfl_xor(nm, off));
    if (lane == 0) {
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
  }
  __syncthreads();
  const int sq = s_sq;
  if (sq < 0) {
    if (tid < 64) y_out[tid] = NAN;
    if (tid == 0) *keff_out = n;
    return;
  }
  const double id = (r == c) ? 1.0 : 0.0;
  const double as = a * ldexp(1.0, -sq);
  A[tid] = as;
  P0[tid] = id + as / 16.0;
  __syncthreads();
  // Horner: P <- I + A P / j for j = 15 .. 1
  double* cur = P0;
  double* nxt = P1;
  for (int j = 15; j >= 1; --j) {
    nxt[tid] = id + tile_dot<TS>(A, cur, r, c) * kInvJ[j];
    __syncthreads();
    double* t = cur;
    cur = nxt;
    nxt = t;
  }
  for (int i = 0; i < sq; ++i) {
    nxt[tid] = tile_dot<TS>(cur, cur, r, c);
    __syncthreads();
    double* t = cur;
    cur = nxt;
    nxt = t;
  }
  if (tid < 64) y_out[tid] = (tid < n) ? cur[tid * TS] : 0.0;
  if (tid == 0) *keff_out = n;
}

}  // namespace expw
