// Device-side building blocks: grid geometry, the staggered operator at one
// point, source injection and deterministic grid-wide FP64 reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace expw {

constexpr int kBlock = 256;        // threads per workgroup (4 wave64)
constexpr int kRedMaxBlocks = 1024;  // grid cap (and partials length) of reduction kernels

// Geometry and coefficients of H on one grid, passed to kernels by value.
// Axis a has extent n[a] and flat stride st[a] (axis 0 fastest); w[l-1] =
// alpha_l / h in the state precision and wd[l-1] in FP64 (for the kernels that
// compute in FP64 from stored values of precision T); sint/shalf are the
// damping profiles at integer / half points.
template <typename T, int K, int DIM>
struct Geo {
  int64_t n[3];
  int64_t st[3];
  int64_t N;  // points per field
  T w[K];
  double wd[K];
  // the weights as small integers (exact in T) times one FP64 factor:
  // alpha_l / h = wscale * wi[l-1]
  T wi[K];
  double wscale;
  const T* __restrict__ c2;
  const T* __restrict__ sint[3];
  const T* __restrict__ shalf[3];
};

template <int DIM>
__device__ __forceinline__ void decompose(const int64_t* n, int64_t idx, int64_t* ic) {
  ic[0] = idx % n[0];
  const int64_t r = idx / n[0];
  if (DIM == 2) {
    ic[1] = r;
    ic[2] = 0;
  } else {
    ic[1] = r % n[1];
    ic[2] = r / n[1];
  }
}

// f at the point shifted by s along an axis of extent n and stride st, for a
// point at coordinate i of that axis: zero outside (Sec. 2.1 ghost rule), or
// wrapped for the periodic closed-form tests.
template <typename T, int BC>
__device__ __forceinline__ T ldn(const T* __restrict__ f, int64_t idx, int64_t i, int64_t n,
                                 int64_t st, int s) {
  const int64_t j = i + s;
  if (BC == 0) return (j >= 0 && j < n) ? f[idx + s * st] : T(0);
  int64_t jj = j % n;
  if (jj < 0) jj += n;
  return f[idx + (jj - i) * st];
}

// out = H x at one point (all DIM+1 fields), self = x at that point:
//   out_p   = -c2 sum_a D-_a v_a - (sum_a sigma_a) p
//   out_v_a = -D+_a p - sigma_a(half) v_a
template <typename T, int K, int BC, int DIM>
__device__ __forceinline__ void apply_point(const Geo<T, K, DIM>& g, const T* __restrict__ x,
                                            int64_t idx, const int64_t* ic, T* out, T* self) {
  const T* __restrict__ p = x;
  const T pc = p[idx];
  self[0] = pc;
  T div = T(0), sp = T(0);
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const T* __restrict__ v = x + (1 + a) * g.N;
    T dv = T(0), dp = T(0);
#pragma unroll
    for (int l = 1; l <= K; ++l) {
      dv += g.w[l - 1] * (ldn<T, BC>(v, idx, ic[a], g.n[a], g.st[a], l - 1) -
                          ldn<T, BC>(v, idx, ic[a], g.n[a], g.st[a], -l));
      dp += g.w[l - 1] * (ldn<T, BC>(p, idx, ic[a], g.n[a], g.st[a], l) -
                          ldn<T, BC>(p, idx, ic[a], g.n[a], g.st[a], 1 - l));
    }
    div += dv;
    sp += g.sint[a][ic[a]];
    const T vc = v[idx];
    self[1 + a] = vc;
    out[1 + a] = -dp - g.shalf[a][ic[a]] * vc;
  }
  out[0] = -g.c2[idx] * div - sp * pc;
}

// out = H x at one point in FP64 from stored values of precision T (all DIM+1
// fields), self = x at that point. The differences of stored neighbours are
// exact in FP64, and so is every product with the FP64 weights up to one
// rounding: the operator applied is H itself, not H with weights rounded to T.
template <typename T, int K, int BC, int DIM>
__device__ __forceinline__ void apply_point_d(const Geo<T, K, DIM>& g, const T* __restrict__ x,
                                              int64_t idx, const int64_t* ic, double* out,
                                              double* self) {
  const T* __restrict__ p = x;
  const double pc = static_cast<double>(p[idx]);
  self[0] = pc;
  double div = 0.0, sp = 0.0;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const T* __restrict__ v = x + (1 + a) * g.N;
    double dv = 0.0, dp = 0.0;
#pragma unroll
    for (int l = 1; l <= K; ++l) {
      dv += g.wd[l - 1] * (static_cast<double>(ldn<T, BC>(v, idx, ic[a], g.n[a], g.st[a], l - 1)) -
                           static_cast<double>(ldn<T, BC>(v, idx, ic[a], g.n[a], g.st[a], -l)));
      dp += g.wd[l - 1] * (static_cast<double>(ldn<T, BC>(p, idx, ic[a], g.n[a], g.st[a], l)) -
                           static_cast<double>(ldn<T, BC>(p, idx, ic[a], g.n[a], g.st[a], 1 - l)));
    }
    div += dv;
    sp += static_cast<double>(g.sint[a][ic[a]]);
    const double vc = static_cast<double>(v[idx]);
    self[1 + a] = vc;
    out[1 + a] = -dp - static_cast<double>(g.shalf[a][ic[a]]) * vc;
  }
  out[0] = -static_cast<double>(g.c2[idx]) * div - sp * pc;
}

// out = H x at one point in mixed precision (the Faber kernels): each
// staggered difference sum_l wi_l (f_{+} - f_{-}) with the integer weights is
// formed in T, and everything after it in FP64: the factor wscale (so the
// operator applied is H itself, not H with weights rounded to T; a rounded
// weight would change the wave speed slightly and, repeated every term of
// every step, shift the phase coherently), c^2, the damping and the sums.
template <typename T, int K, int BC, int DIM>
__device__ __forceinline__ void apply_point_m(const Geo<T, K, DIM>& g, const T* __restrict__ x,
                                              int64_t idx, const int64_t* ic, double* out,
                                              double* self) {
  const T* __restrict__ p = x;
  const double pc = static_cast<double>(p[idx]);
  self[0] = pc;
  double div = 0.0, sp = 0.0;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const T* __restrict__ v = x + (1 + a) * g.N;
    T dv = T(0), dp = T(0);
#pragma unroll
    for (int l = 1; l <= K; ++l) {
      dv += g.wi[l - 1] * (ldn<T, BC>(v, idx, ic[a], g.n[a], g.st[a], l - 1) -
                           ldn<T, BC>(v, idx, ic[a], g.n[a], g.st[a], -l));
      dp += g.wi[l - 1] * (ldn<T, BC>(p, idx, ic[a], g.n[a], g.st[a], l) -
                           ldn<T, BC>(p, idx, ic[a], g.n[a], g.st[a], 1 - l));
    }
    div += static_cast<double>(dv);
    sp += static_cast<double>(g.sint[a][ic[a]]);
    const double vc = static_cast<double>(v[idx]);
    self[1 + a] = vc;
    out[1 + a] = -static_cast<double>(dp) * g.wscale - static_cast<double>(g.shalf[a][ic[a]]) * vc;
  }
  out[0] = -static_cast<double>(g.c2[idx]) * (div * g.wscale) - sp * pc;
}

// Receivers on a run of consecutive pressure nodes first .. first + n - 1,
// recorded by the kernel that writes a step's final pressure: out is the
// step's row of the traces (nullptr: not recorded in the kernel).
template <typename T>
struct RecRun {
  T* out;
  int64_t first, n;
};

template <typename T>
__device__ __forceinline__ void rec_run_put(const RecRun<T>& r, int64_t idx, T v) {
  if (r.out) {
    const int64_t d = idx - r.first;
    if (d >= 0 && d < r.n) r.out[d] = v;
  }
}

// Point sources: flat pressure indices idx[s] with amplitudes amp[s];
// [lo, hi] bounds the indices so that other threads skip the search.
template <typename T>
struct Src {
  int32_t n;
  int64_t lo, hi;
  const int64_t* __restrict__ idx;
  const T* __restrict__ amp;
  double q;  // scalar multiplying every amplitude for this launch
};

template <typename T>
__device__ __forceinline__ T src_value(const Src<T>& s, int64_t idx) {
  T r = T(0);
  if (s.n > 0 && idx >= s.lo && idx <= s.hi)
    for (int i = 0; i < s.n; ++i)
      if (s.idx[i] == idx) r += static_cast<T>(s.q) * s.amp[i];
  return r;
}

// The source term at a pressure node in FP64 (the kernels that compute in FP64).
template <typename T>
__device__ __forceinline__ double src_value_d(const Src<T>& s, int64_t idx) {
  double r = 0.0;
  if (s.n > 0 && idx >= s.lo && idx <= s.hi)
    for (int i = 0; i < s.n; ++i)
      if (s.idx[i] == idx) r += s.q * static_cast<double>(s.amp[i]);
  return r;
}

// ---------------------------------------------------------------- reductions

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  return v;
}

// x moved across lanes by one DPP pattern (lanes of rows outside ROW_MASK get 0).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROW_MASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROW_MASK, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave (all lanes active), returned to every lane.
// Lane shuffles by DPP: pairs and quads (quad permutations), the four quads of
// each 16-lane row (row rotations by 4 and 8), then rows 0+1 and 2+3 (row
// broadcast of lane 15) and finally all four (row broadcast of lane 31). The
// value of lane 63 is taken, so the order of the additions is fixed and every
// wave with the same inputs gets the same bits.
__device__ __forceinline__ double wave_sum_fixed(double v) {
  v += dpp_move<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x124, 0xF>(v);  // row_ror:4
  v += dpp_move<0x128, 0xF>(v);  // row_ror:8
  v += dpp_move<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// Block-wide reduction over NT threads; the result is valid in thread 0.
// Ends with a barrier so that the shared scratch can be reused right away.
template <bool MAX, int NT = kBlock>
__device__ __forceinline__ double block_reduce(double v) {
  static_assert(NT % 64 == 0 && NT <= 1024, "block of whole waves");
  __shared__ double sh[NT / 64];
  v = MAX ? wave_max(v) : wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = MAX ? -INFINITY : 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < NT / 64; ++i) r = MAX ? fmax(r, sh[i]) : r + sh[i];
  __syncthreads();
  return r;
}

// Grid-wide reductions go through the kernel boundary: a producing kernel
// stores one partial per workgroup, and the kernel that needs the value
// (launched after it on the same stream, so the partials are visible on every
// XCD) sums them in block order. The result is deterministic and needs no
// atomics or intra-kernel cross-XCD coherence.
template <bool MAX>
__device__ __forceinline__ void store_partial(double v, double* __restrict__ partials) {
  const double b = block_reduce<MAX>(v);
  if (threadIdx.x == 0) partials[blockIdx.x] = b;
}

// Sum (or max) of n partials in a fixed order; the value is returned to every thread.
template <bool MAX>
__device__ __forceinline__ double load_reduced(const double* __restrict__ partials, int n) {
  __shared__ double s_val;
  double acc = MAX ? -INFINITY : 0.0;
  for (int i = threadIdx.x; i < n; i += kBlock) acc = MAX ? fmax(acc, partials[i]) : acc + partials[i];
  const double tot = block_reduce<MAX>(acc);
  if (threadIdx.x == 0) s_val = tot;
  __syncthreads();
  return s_val;
}

}  // namespace expw
