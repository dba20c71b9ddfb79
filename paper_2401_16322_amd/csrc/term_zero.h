// One Faber term per sweep for the staggered stencils of order 4 and 8 (K = 2
// or 4 weights per side) with zero ghost values (Sec. 2.1), in 2D and 3D: the
// one-term path of the Faber step (3D steps, a single final term after fused
// passes, depth 1).
//
// A 64 x 4 workgroup covers 64 consecutive x-points of 4 consecutive rows
// (one plane z in 3D), so every wave reads 64 consecutive values of a row.
// Each point's 2K neighbour values of p and of v_a along each axis are loaded
// with 32-bit offsets that are clamped to the point itself when the
// neighbour lies outside the grid (the loaded value is then replaced by
// zero), so no load sits behind a branch and the compiler issues all of a
// point's loads together; x-neighbours hit in L1, y- and z-neighbours in
// L1/L2 (the planes a workgroup reads are read again by the workgroups of the
// next planes). Arithmetic and precision as in k_faber_term: with SC = T the
// difference sums use the integer weights in T and everything after them
// (the weight factor, c^2, damping, recurrence and sum) is FP64
// (apply_point_m); with SC = double the whole stencil is FP64. The arrays
// touched once per point (v_{j-2}, the sum, the outputs) are read and
// written as streaming (non-temporal) accesses, so that v_{j-1}, whose
// neighbour values are read again by other workgroups, and c^2 keep the
// caches.
#pragma once

#include "device_common.h"
#include "kernels.h"

namespace expw {

constexpr int kTzX = 64, kTzY = 4;

template <typename T>
__device__ __forceinline__ T ld_or0(const T* __restrict__ f, int base, int off, bool ok) {
  const T v = f[base + (ok ? off : 0)];
  return ok ? v : T(0);
}

template <typename SC, typename T>
__device__ __forceinline__ SC to_sc(T v) {
  return static_cast<SC>(v);
}

// grid: (ceil(nx / 64), ceil(n1 / 4), n2) for 3D (n1 = ny, n2 = nz), and
// (ceil(nx / 64), ceil(nz / 4), 1) in 2D. Requires (DIM + 1) * points < 2^31.
// Outputs as in k_faber_term (vout may alias vpp, acc_out may alias acc_in,
// state_out may alias vpp; vp must not alias any output).
template <typename T, int K, int DIM, typename SC>
__global__ __launch_bounds__(kTzX * kTzY) void k_faber_term_zero(Geo<T, K, DIM> g, const T* __restrict__ vp,
                                                                const T* vpp, T* vout,
                                                                const double* acc_in, double* acc_out,
                                                                T* state_out, FaberTerm c, Src<T> src) {
  static_assert(K == 2 || K == 4, "order 4 or 8");
  const int nx = static_cast<int>(g.n[0]), n1 = static_cast<int>(g.n[1]);
  const int i = blockIdx.x * kTzX + (threadIdx.x & (kTzX - 1));
  const int j = blockIdx.y * kTzY + (threadIdx.x >> 6);
  const int k = DIM == 3 ? static_cast<int>(blockIdx.z) : 0;
  if (i >= nx || j >= n1) return;
  const int n2 = DIM == 3 ? static_cast<int>(g.n[2]) : 1;
  const int N = static_cast<int>(g.N);
  const int sy = nx, sz = nx * n1;
  const int idx = (k * n1 + j) * nx + i;
  const int coord[3] = {i, j, k};
  const int ext[3] = {nx, n1, n2};
  const int str[3] = {1, sy, sz};
  const T* p = vp;
  // loads: p at the point and at 1-K .. -1, +1 .. +K along each axis (pk[a][l]
  // = p at offset l - K + 1, l = 0..2K-1, the point itself at l = K - 1); v_a at
  // -K .. K-1 along axis a (vk[a][l] at offset l - K, the point at l = K)
  T pk[DIM][2 * K], vk[DIM][2 * K];
  const T pc = p[idx];
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const T* v = vp + (1 + a) * N;
    const int x = coord[a], n = ext[a], s = str[a];
#pragma unroll
    for (int l = 0; l < 2 * K; ++l) {
      const int op = l - K + 1, ov = l - K;
      pk[a][l] = op == 0 ? pc : ld_or0(p, idx, op * s, x + op >= 0 && x + op < n);
      vk[a][l] = ov == 0 ? v[idx] : ld_or0(v, idx, ov * s, x + ov >= 0 && x + ov < n);
    }
  }
  const T c2 = g.c2[idx];
  T old[DIM + 1];
#pragma unroll
  for (int f = 0; f <= DIM; ++f) old[f] = vpp ? __builtin_nontemporal_load(vpp + f * N + idx) : T(0);
  double acc[DIM + 1];
#pragma unroll
  for (int f = 0; f <= DIM; ++f) acc[f] = c.first ? 0.0 : __builtin_nontemporal_load(acc_in + f * N + idx);

  // H v at the point: difference sums in SC (integer weights unless SC is
  // FP64), the weight factor and the rest in FP64
  constexpr bool kInt = !(sizeof(SC) == 8 && sizeof(T) == 4);
  SC w[K];
#pragma unroll
  for (int l = 0; l < K; ++l) w[l] = kInt ? static_cast<SC>(g.wi[l]) : static_cast<SC>(g.wd[l]);
  const double wsc = kInt ? g.wscale : 1.0;
  SC div = SC(0);
  double o[DIM + 1], s[DIM + 1];
  double sp = 0.0;
  s[0] = static_cast<double>(pc);
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    // dv = sum_l w_l (v[x + l - 1] - v[x - l]), dp = sum_l w_l (p[x + l] - p[x + 1 - l])
    SC dv, dp;
    if constexpr (K == 2) {
      dv = w[0] * (to_sc<SC>(vk[a][2]) - to_sc<SC>(vk[a][1])) + w[1] * (to_sc<SC>(vk[a][3]) - to_sc<SC>(vk[a][0]));
      dp = w[0] * (to_sc<SC>(pk[a][2]) - to_sc<SC>(pc)) + w[1] * (to_sc<SC>(pk[a][3]) - to_sc<SC>(pk[a][0]));
    } else {
      dv = w[0] * (to_sc<SC>(vk[a][K]) - to_sc<SC>(vk[a][K - 1]));
      dp = w[0] * (to_sc<SC>(pk[a][K]) - to_sc<SC>(pc));
#pragma unroll
      for (int l = 2; l <= K; ++l) {
        dv += w[l - 1] * (to_sc<SC>(vk[a][K + l - 1]) - to_sc<SC>(vk[a][K - l]));
        dp += w[l - 1] * (to_sc<SC>(pk[a][K + l - 1]) - to_sc<SC>(pk[a][K - l]));
      }
    }
    div += dv;
    sp += static_cast<double>(g.sint[a][coord[a]]);
    s[1 + a] = static_cast<double>(vk[a][K]);
    o[1 + a] = -static_cast<double>(dp) * wsc - static_cast<double>(g.shalf[a][coord[a]]) * s[1 + a];
  }
  o[0] = -static_cast<double>(c2) * (static_cast<double>(div) * wsc) - sp * s[0];
  const double q = src.n > 0 ? src_value_d(src, idx) : 0.0;
#pragma unroll
  for (int f = 0; f <= DIM; ++f) {
    const int e = f * N + idx;
    double v = o[f] * c.inv_gamma - c.c0 * s[f];
    if (vpp) v -= c.cpp * static_cast<double>(old[f]);
    if (f == 0) v += q;
    const T vt = static_cast<T>(v);
    if (vout) __builtin_nontemporal_store(vt, vout + e);
    if (acc_out || state_out) {
      double a_ = c.first ? c.a_first * s[f] : acc[f];
      a_ = fma(c.a_j, static_cast<double>(vt), a_);
      if (state_out) __builtin_nontemporal_store(static_cast<T>(a_), state_out + e);
      else __builtin_nontemporal_store(a_, acc_out + e);
    }
  }
}

template <int DIM>
inline dim3 term_zero_grid(const int64_t* n) {
  return DIM == 3 ? dim3(static_cast<unsigned>((n[0] + kTzX - 1) / kTzX),
                         static_cast<unsigned>((n[1] + kTzY - 1) / kTzY), static_cast<unsigned>(n[2]))
                  : dim3(static_cast<unsigned>((n[0] + kTzX - 1) / kTzX),
                         static_cast<unsigned>((n[1] + kTzY - 1) / kTzY), 1u);
}

}  // namespace expw
