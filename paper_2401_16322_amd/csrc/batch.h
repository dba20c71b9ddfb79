// Faber steps of many independent problems (shots) in the same launches
// (Sec. 3.2, Faber recurrence; the shots share nothing but the launch). Term
// j of every shot whose degree is at least j runs in one launch: the shots
// are sorted by degree, so the participating shots are a prefix of the list
// and a block finds its shot by a binary search over the prefix sums of the
// shots' block counts. Every per-shot constant (grid, buffers, ellipse,
// coefficients, source, receivers) sits in a device table built once; the
// source scalar of a term is formed on the device from the Ricker
// derivatives at the step time (the same FP64 formula as the host path) and
// per-shot tail projections, so nothing is uploaded per step. One launch per
// term index instead of one per term and shot.
#pragma once

#include "device_common.h"
#include "expwave.h"
#include "fused.h"
#include "kernels.h"

namespace expw {

constexpr int kBatchMaxM = 64;

// Time base of the batch's kernels in device memory: step st of a sequence
// runs at t0 + (step0 + st) dt of each shot and records into trace row
// trace0 + st. Kept in memory (set by k_batch_set_clock before a sequence)
// so that a captured sequence of launches can be replayed at other times.
struct BatchClock {
  double t0;
  int64_t step0, trace0;
};

__global__ void k_batch_set_clock(BatchClock* clk, double t0, int64_t step0, int64_t trace0) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    clk->t0 = t0;
    clk->step0 = step0;
    clk->trace0 = trace0;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_batch_copy(T* __restrict__ dst, const T* __restrict__ src,
                                                       int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock)
    dst[i] = src[i];
}

template <typename T, int K, int DIM>
struct BatchShot {
  Geo<T, K, DIM> g;
  T *S, *A, *B;  // state and two term vectors of the shot
  double* C;     // the shot's FP64 partial sum
  int32_t m, n_src, p, n_rec;
  int64_t src_lo, src_hi;
  const int64_t* src_idx;
  const T* src_amp;
  const int64_t* rec;
  T* traces;  // NULL: not recorded
  double f_peak, t_delay, dt;
  double inv_gamma, c0, c1;
  double kappa, inv_ws;  // wscale / gamma and 1 / wscale (the fused passes' form)
  double a[kBatchMaxM + 1];
  double qtab[kBatchMaxM][EXPW_MAX_TAYLOR];  // source scalar of term j: sum_c G_c(t) qtab[j-1][c]
};

// g^(k)(t), k = 0..p-1, of the Ricker wavelet (physicists' Hermite form, as
// the host computes it).
__device__ __forceinline__ void ricker_derivatives_dev(double t, double f_peak, double t_delay,
                                                       int p, double* out) {
  const double pi = 3.14159265358979323846264338327950;
  const double a = (pi * f_peak) * (pi * f_peak);
  const double tau = t - t_delay;
  const double sa = sqrt(a);
  const double xs = sa * tau;
  const double e = exp(-a * tau * tau);
  double hm1 = 1.0, h0 = 2.0 * xs;  // H_0, H_1
  double apow = a;
  for (int n = 1; n < p + 2; ++n) {  // H_{n+1}
    const double h1 = 2.0 * xs * h0 - 2.0 * n * hm1;
    hm1 = h0;
    h0 = h1;
    const int k = n - 1;  // H_{k+2} = h0
    if (k < p) {
      out[k] = -(1.0 / (2.0 * a)) * ((k % 2 == 0) ? 1.0 : -1.0) * apow * h0 * e;
      apow *= sa;
    }
  }
}

// Shot of item b among the first n_part shots (prefix[s] = first item of shot s).
__device__ __forceinline__ int batch_shot_of(const int64_t* prefix, int n_part, int64_t b) {
  int lo = 0, hi = n_part - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Shot of this block among the first n_part shots (prefix[s] = first block of shot s).
__device__ __forceinline__ int batch_shot(const int64_t* prefix, int n_part) {
  return batch_shot_of(prefix, n_part, blockIdx.x);
}

// Term j of every shot with m >= j. Buffers per shot as in the one-shot
// unfused step: v1 -> A, v2 -> B, then v_j overwrites v_{j-2}; the FP64 sum
// in C, the last term rounds it into S (degree >= 2). Terms are computed in
// FP64 and stored in T (see FaberTerm).
template <typename T, int K, int BC, int DIM>
__global__ __launch_bounds__(kBlock) void k_faber_batch_term(const BatchShot<T, K, DIM>* shots,
                                                             const int64_t* prefix, int n_part,
                                                             int j, const BatchClock* clk,
                                                             int64_t st) {
  const int s = batch_shot(prefix, n_part);
  const BatchShot<T, K, DIM>& sh = shots[s];
  const Geo<T, K, DIM>& g = sh.g;
  const int64_t idx = (static_cast<int64_t>(blockIdx.x) - prefix[s]) * kBlock + threadIdx.x;
  if (idx >= g.N) return;
  const bool fin = (j == sh.m);
  const T *vp, *vpp;
  T* vout;
  T* state_out = fin ? sh.S : nullptr;
  double cpp;
  if (j == 1) {
    vp = sh.S, vpp = nullptr, vout = sh.A, cpp = 0.0;
  } else if (j == 2) {
    vp = sh.A, vpp = sh.S, vout = fin ? nullptr : sh.B;
    cpp = 2.0 * sh.c1;
  } else {
    vp = (j & 1) ? sh.B : sh.A;
    vpp = (j & 1) ? sh.A : sh.B;
    vout = fin ? nullptr : const_cast<T*>(vpp);
    cpp = sh.c1;
  }
  int64_t ic[3];
  decompose<DIM>(g.n, idx, ic);
  double o[DIM + 1], sv[DIM + 1];
  apply_point_m<T, K, BC, DIM>(g, vp, idx, ic, o, sv);
  // source at this point (rare): scalar of term j at the step time
  double src = 0.0;
  if (sh.n_src > 0 && idx >= sh.src_lo && idx <= sh.src_hi) {
    double am = 0.0;
    for (int k = 0; k < sh.n_src; ++k)
      if (sh.src_idx[k] == idx) am += static_cast<double>(sh.src_amp[k]);
    if (am != 0.0) {
      double der[EXPW_MAX_TAYLOR];
      ricker_derivatives_dev(clk->t0 + (clk->step0 + st) * sh.dt, sh.f_peak, sh.t_delay, sh.p, der);
      double q = 0.0;
      for (int c = 0; c < sh.p; ++c) q += der[sh.p - 1 - c] * sh.qtab[j - 1][c];
      src = q * am;
    }
  }
#pragma unroll
  for (int f = 0; f <= DIM; ++f) {
    const int64_t e = f * g.N + idx;
    double v = o[f] * sh.inv_gamma - sh.c0 * sv[f];
    if (vpp) v -= cpp * static_cast<double>(vpp[e]);
    if (f == 0) v += src;
    const T vt = static_cast<T>(v);
    double acc = (j == 1) ? sh.a[0] * sv[f] : sh.C[e];
    acc = fma(sh.a[j], static_cast<double>(vt), acc);
    if (vout) vout[e] = vt;
    if (state_out) state_out[e] = static_cast<T>(acc);
    else sh.C[e] = acc;
  }
}

// traces of every recording shot for one step (prefix_rec[s] = first item of shot s).
template <typename T, int K, int DIM>
__global__ __launch_bounds__(kBlock) void k_batch_gather(const BatchShot<T, K, DIM>* shots,
                                                         const int64_t* prefix_rec, int n_shots,
                                                         const BatchClock* clk, int64_t st) {
  const int64_t it = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x;
  if (it >= prefix_rec[n_shots]) return;
  int lo = 0, hi = n_shots - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix_rec[mid] <= it) lo = mid;
    else hi = mid - 1;
  }
  const BatchShot<T, K, DIM>& sh = shots[lo];
  const int64_t r = it - prefix_rec[lo];
  if (sh.traces && r < sh.n_rec) sh.traces[(clk->trace0 + st) * sh.n_rec + r] = sh.S[sh.rec[r]];
}

// Fused passes for batches of 2D order-4 zero-ghost shots: pass p of every
// shot still running applies its terms 1 + p S .. min(m, (p + 1) S) over the
// shot's tiles in one launch (a last pass with n < S terms runs the last n
// terms of the S-term tile schedule). Buffers per shot as in the one-shot
// fused step: (A, B) and (D, E) alternate as (v_last, v_prev), C holds the
// FP64 sum, the last pass rounds it into S (a shot of one pass writes A,
// copied afterwards).
constexpr int kBatchFuse = 4;  // default depth (2, 4 or 6)

template <typename T>
struct FusedShot {
  Geo<T, 2, 2> g;
  T *S, *A, *B, *D, *E;
  double* C;
  int32_t m, tiles_x, tiles_y, n_src, p, pad_;
  int64_t src_lo, src_hi;
  const int64_t* src_idx;
  const T* src_amp;
  double f_peak, t_delay, dt;
  double kappa, inv_ws, c0, c1;
  double a[kBatchMaxM + 1];
  T cpp[kBatchMaxM + 1];  // coefficient of v_{j-2} in term j (0, 2 c1, c1, ...), in T
  double qtab[kBatchMaxM][EXPW_MAX_TAYLOR];
};

// The source scalars of every term of shot sh for step st (one thread):
// q_j = sum_c g^(p-1-c)(t) qtab[j - 1][c], with the Ricker derivatives g^(k)
// at the step time from the Hermite recurrence (the host's FP64 formula);
// zero without a source.
template <typename T>
__device__ __forceinline__ void batch_shot_source_q(const FusedShot<T>& sh, const BatchClock* clk,
                                                    int64_t st, T* q) {
  double gk[EXPW_MAX_TAYLOR];
  const int p = sh.n_src > 0 ? sh.p : 0;
  if (p > 0) ricker_derivatives_dev(clk->t0 + (clk->step0 + st) * sh.dt, sh.f_peak, sh.t_delay, p, gk);
  for (int j = 1; j <= sh.m; ++j) {
    double v = 0.0;
    for (int c = 0; c < p; ++c) v += gk[p - 1 - c] * sh.qtab[j - 1][c];
    q[j - 1] = static_cast<T>(v);
  }
}

// The per-step table of source scalars (kBatchMaxM per shot), one thread per shot.
template <typename T>
__global__ __launch_bounds__(64) void k_batch_source_q(const FusedShot<T>* shots, int n, const BatchClock* clk,
                                                       int64_t st, T* qstep) {
  const int s = blockIdx.x * 64 + threadIdx.x;
  if (s < n) batch_shot_source_q(shots[s], clk, st, qstep + static_cast<int64_t>(s) * kBatchMaxM);
}

// Tile t of pass `pass` of one shot (the whole workgroup); qs: the shot's
// source scalars of this step (k_batch_source_q).
template <typename T, int S>
__device__ __forceinline__ void batch_fused_tile(const FusedShot<T>& sh, const T* __restrict__ qs, int t,
                                                 int pass) {
  const int tx_ = t % sh.tiles_x, ty_ = t / sh.tiles_x;
  const int j0 = 1 + pass * S;
  const int n = min(S, sh.m - j0 + 1);
  const int r0 = S - n;
  const bool first = (pass == 0);
  const bool last = (j0 + n - 1 == sh.m);
  FusedArgs<T, S> c{};
  c.kappa = static_cast<T>(sh.kappa);
  c.inv_ws = static_cast<T>(sh.inv_ws);
  c.c0 = static_cast<T>(sh.c0);
  c.first = first ? 1 : 0;
  c.a_first = sh.a[0];
#pragma unroll
  for (int r = 0; r < S; ++r) {
    const int j = j0 + (r - r0);
    const bool on = r >= r0;
    c.a[r] = on ? sh.a[j] : 0.0;
    c.cpp[r] = on ? sh.cpp[j] : T(0);
    c.q[r] = on ? qs[j - 1] : T(0);
  }
  const bool odd_in = ((pass - 1) & 1) != 0, odd_out = (pass & 1) != 0;
  const T* vp = first ? sh.S : (odd_in ? sh.D : sh.A);
  const T* vpp = first ? nullptr : (odd_in ? sh.E : sh.B);
  T* ol = last ? nullptr : (odd_out ? sh.D : sh.A);
  T* opv = last ? nullptr : (odd_out ? sh.E : sh.B);
  double* acc_out = last ? nullptr : sh.C;
  T* state_out = last ? (first ? sh.A : sh.S) : nullptr;
  Src<T> src{};
  src.n = sh.n_src;
  src.lo = sh.src_lo;
  src.hi = sh.src_hi;
  src.idx = sh.src_idx;
  src.amp = sh.src_amp;
  fused2d_pass<T, S>(sh.g, vp, vpp, first ? nullptr : sh.C, ol, opv, acc_out, state_out, c, src,
                     tx_, ty_, r0);
}

template <typename T, int S>
__global__ __launch_bounds__(kFusedNT, sizeof(T) == 4 ? 8 : 4) void k_faber_fused2d_batch(
    const FusedShot<T>* __restrict__ shots, const int64_t* __restrict__ prefix, int n_part, int pass,
    const T* __restrict__ qstep) {
  const int s = batch_shot(prefix, n_part);
  batch_fused_tile<T, S>(shots[s], qstep + static_cast<int64_t>(s) * kBatchMaxM,
                         static_cast<int>(static_cast<int64_t>(blockIdx.x) - prefix[s]), pass);
}

// One launch per batched step (cooperative: every workgroup is resident).
// The workgroups take the tiles of pass p of every shot still running in
// turn (tile i, i + grid, ...), then meet at a grid-wide barrier before pass
// p + 1; after the last pass, one-pass shots copy their result into the
// state, and the receivers are recorded, each behind a barrier. The barrier
// is a counter and a generation word: arriving, a workgroup's first thread
// releases its writes at agent scope (written back past its XCD's L2) and
// adds one to the counter; the last to arrive resets it and advances the
// generation, the others wait for that, and each then acquires at agent
// scope (its XCD's caches drop lines other XCDs may have written). Every
// wait is bounded: past spin_limit polls (1024 once err is set) it sets err
// and goes on, so every wave reaches the end of the kernel; the host then
// reports the step as failed.
struct BatchSync {
  unsigned count, gen;
  int err, pad;
};

constexpr int kBatchMaxPasses = kBatchMaxM;

struct BatchPersist {
  int32_t count_pass[kBatchMaxPasses];
  int32_t max_passes, n_shots, any_single;
  uint32_t spin_limit;
};

__device__ __forceinline__ void batch_grid_sync(BatchSync* bs, unsigned spin_limit) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned g = __hip_atomic_load(&bs->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned prev = __hip_atomic_fetch_add(&bs->count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (prev + 1 == gridDim.x) {
      __hip_atomic_store(&bs->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&bs->gen, g + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      unsigned polls = 0;
      unsigned limit = __hip_atomic_load(&bs->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ? 1024u : spin_limit;
      while (__hip_atomic_load(&bs->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
        if (++polls > limit) {
          __hip_atomic_store(&bs->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        if ((polls & 1023u) == 0 && __hip_atomic_load(&bs->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
          limit = polls + 1024u < limit ? polls + 1024u : limit;
        __builtin_amdgcn_s_sleep(2);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

template <typename T, int S>
__global__ __launch_bounds__(kFusedNT) void k_faber_batch_persistent(
    const FusedShot<T>* fshots, const int64_t* fprefix, const BatchShot<T, 2, 2>* shots,
    const int64_t* prefix_rec, BatchPersist pa, const BatchClock* clk, int64_t st, BatchSync* bs,
    T* qstep) {
  // the step's source scalars, one thread per shot, before the first pass
  for (int s = blockIdx.x * kFusedNT + threadIdx.x; s < pa.n_shots; s += gridDim.x * kFusedNT)
    batch_shot_source_q(fshots[s], clk, st, qstep + static_cast<int64_t>(s) * kBatchMaxM);
  batch_grid_sync(bs, pa.spin_limit);
  for (int p = 0; p < pa.max_passes; ++p) {
    const int np = pa.count_pass[p];
    const int64_t total = fprefix[np];
    for (int64_t vt = blockIdx.x; vt < total; vt += gridDim.x) {
      const int s = batch_shot_of(fprefix, np, vt);
      batch_fused_tile<T, S>(fshots[s], qstep + static_cast<int64_t>(s) * kBatchMaxM,
                             static_cast<int>(vt - fprefix[s]), p);
      __syncthreads();  // the next tile reuses the LDS
    }
    batch_grid_sync(bs, pa.spin_limit);
  }
  const int64_t tid = blockIdx.x * static_cast<int64_t>(kFusedNT) + threadIdx.x;
  const int64_t nth = static_cast<int64_t>(gridDim.x) * kFusedNT;
  if (pa.any_single) {
    for (int s = 0; s < pa.n_shots; ++s) {
      const FusedShot<T>& sh = fshots[s];
      if (sh.m > S) continue;
      const int64_t ns = 3 * sh.g.N;
      for (int64_t i = tid; i < ns; i += nth) sh.S[i] = sh.A[i];
    }
    batch_grid_sync(bs, pa.spin_limit);
  }
  const int64_t items = prefix_rec[pa.n_shots];
  for (int64_t it = tid; it < items; it += nth) {
    const int s = batch_shot_of(prefix_rec, pa.n_shots, it);
    const BatchShot<T, 2, 2>& sh = shots[s];
    const int64_t r = it - prefix_rec[s];
    if (sh.traces && r < sh.n_rec) sh.traces[(clk->trace0 + st) * sh.n_rec + r] = sh.S[sh.rec[r]];
  }
}

}  // namespace expw
