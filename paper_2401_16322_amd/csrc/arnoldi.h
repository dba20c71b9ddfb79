// Persistent Arnoldi (modified Gram-Schmidt) for one Krylov step, for
// augmented vectors small enough to live in registers across the grid.
//
// One cooperative launch runs the whole basis construction: each thread owns
// UN elements of the flat augmented vector (element e = tid + u * threads),
// and keeps its slice of w, q_0 and the current q_i in registers. An MGS step
// then costs one grid barrier (to reduce the dot) and one read of the next
// basis vector, instead of a kernel launch that streams w, q_i, q_{i+1} and w
// again. Columns are written unnormalized with their scale s_j = 1/h_{j,j-1}
// (s_0 = 1), as in the launch-per-step path.
//
// Data that crosses workgroups inside the launch (reduction partials and the
// basis vectors Q_j) is read and written with device-coherent accesses
// (agent-scope relaxed atomics, i.e. sc1 loads and stores that do not stop in
// an XCD's L2), so no cache-wide writeback or invalidation is needed. A
// grid-wide reduction is also the barrier, and uses no read-modify-write:
// each block's partial is its own arrival word. Slots start out holding a
// signalling-NaN pattern that no arithmetic produces; block b stores its
// partial (after waiting for its earlier stores, s_waitcnt 0) into slot b of
// the barrier's buffer, and every block waits, one thread per slot, until the
// slot no longer holds that pattern, taking the value it finds. Three
// buffers rotate: when barrier s completes, every block has read the values
// of barrier s-1, so each block then restores the pattern in its slot of that
// buffer, which is next written at barrier s+2. One store and one successful
// load per block and barrier, against two of each with separate flags. Every
// wait is bounded: a wait longer than spin_limit polls sets *err and gives up,
// and once *err is set no wait lasts more than 1024 polls, so every wave
// always reaches the end of the kernel.
#pragma once

#include "device_common.h"
#include "kernels.h"

namespace expw {

constexpr int kArnNT = 1024;  // threads per block of the persistent kernel

template <typename T>
__device__ __forceinline__ T ld_coherent(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ void st_coherent(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Contents of an empty slot of the grid-wide reduction (a signalling NaN;
// a NaN partial is stored as the default quiet NaN instead).
constexpr unsigned long long kSlotEmpty = 0x7FF4DEADBEEF0001ull;
constexpr int kSlotBuffers = 3;

// Grid-wide sum of v (blocks of NT threads, at most 1024 blocks): returns the
// sum of the per-block partials, added in a fixed order, to every thread. slots holds
// kSlotBuffers buffers of kRedMaxBlocks words, all kSlotEmpty at launch; seq
// numbers the barriers of the launch (1, 2, ...). after() runs in every
// thread once this block has arrived: loads it issues overlap the wait (the
// s_waitcnt before the arrival waits for every outstanding memory operation,
// so loads issued earlier would be waited for there).
template <int NT, typename F>
__device__ __forceinline__ double grid_sum(double v, unsigned long long* slots, unsigned seq,
                                           unsigned spin_limit, int* err, F&& after) {
  static_assert(NT % 64 == 0 && NT <= 1024, "block of whole waves");
  __shared__ double s_part[NT / 64];
  __shared__ double s_poll[2][kRedMaxBlocks / 64];
  unsigned long long* cur = slots + (seq % kSlotBuffers) * kRedMaxBlocks;
  unsigned long long* prev = slots + ((seq + kSlotBuffers - 1) % kSlotBuffers) * kRedMaxBlocks;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  // the block's partial: wave sums, then wave 0 sums them
  v = wave_sum_fixed(v);
  if (lane == 0) s_part[wid] = v;
  __builtin_amdgcn_s_waitcnt(0);  // this thread's coherent stores have completed
  __syncthreads();
  if (wid == 0) {
    double b = lane < NT / 64 ? s_part[lane] : 0.0;
    b = wave_sum_fixed(b);
    if (lane == 0) {
      const unsigned long long bits = (b != b) ? 0x7FF8000000000000ull : __double_as_longlong(b);
      st_coherent(cur + blockIdx.x, bits);
    }
  }
  after();
  // every block's partial, one thread per slot
  double pv = 0.0;
  if (threadIdx.x < gridDim.x) {
    unsigned polls = 0;
    unsigned long long x;
    while ((x = ld_coherent(cur + threadIdx.x)) == kSlotEmpty) {
      __builtin_amdgcn_s_sleep(1);
      if (++polls > spin_limit ||
          ((polls & 1023u) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
    pv = __longlong_as_double(x);
  }
  // sum in block order: per wave of slots, then the waves in order (every
  // thread adds the same values in the same order)
  const int nw = (static_cast<int>(gridDim.x) + 63) / 64;
  double* sp = s_poll[seq & 1u];
  if (wid < nw) {
    pv = wave_sum_fixed(pv);
    if (lane == 0) sp[wid] = pv;
  }
  __syncthreads();
  double tot = 0.0;
  for (int w = 0; w < nw; ++w) tot += sp[w];
  if (threadIdx.x == 0) {
    // all blocks arrived at this barrier, so all have read barrier seq-1's
    // values; the store completes before this block's next arrival (s_waitcnt)
    st_coherent(prev + blockIdx.x, kSlotEmpty);
  }
  return tot;
}

// x at the point shifted by s along one axis (zero outside or wrapped), read
// with a device-coherent load.
template <typename T, int BC>
__device__ __forceinline__ T ldn_coherent(const T* f, int64_t idx, int64_t i, int64_t n, int64_t st,
                                          int s) {
  const int64_t j = i + s;
  if (BC == 0) return (j >= 0 && j < n) ? ld_coherent(f + idx + s * st) : T(0);
  int64_t jj = j % n;
  if (jj < 0) jj += n;
  return ld_coherent(f + idx + (jj - i) * st);
}

// (H x)_f at one point: field f = 0 (pressure) or 1 + a (velocity along a),
// with x read coherently (c^2 and the damping profiles are read-only).
template <typename T, int K, int BC, int DIM>
__device__ __forceinline__ T apply_field(const Geo<T, K, DIM>& g, const T* x, int f, int64_t idx,
                                         const int64_t* ic) {
  if (f == 0) {
    T div = T(0), sp = T(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      const T* v = x + (1 + a) * g.N;
#pragma unroll
      for (int l = 1; l <= K; ++l)
        div += g.w[l - 1] * (ldn_coherent<T, BC>(v, idx, ic[a], g.n[a], g.st[a], l - 1) -
                             ldn_coherent<T, BC>(v, idx, ic[a], g.n[a], g.st[a], -l));
      sp += g.sint[a][ic[a]];
    }
    return -g.c2[idx] * div - sp * ld_coherent(x + idx);
  }
  const int a = f - 1;
  T dp = T(0);
#pragma unroll
  for (int l = 1; l <= K; ++l)
    dp += g.w[l - 1] * (ldn_coherent<T, BC>(x, idx, ic[a], g.n[a], g.st[a], l) -
                        ldn_coherent<T, BC>(x, idx, ic[a], g.n[a], g.st[a], 1 - l));
  return -dp - g.shalf[a][ic[a]] * ld_coherent(x + f * g.N + idx);
}

struct ArnArgs {
  int64_t ns, naug, ld;
  int k;
  double tail2;  // |e_p|^2: 1 with a source, else 0
  double tol;
  unsigned spin_limit;
};

template <typename T, int K, int BC, int DIM, int UN>
__global__ __launch_bounds__(kArnNT) void k_arnoldi_persistent(
    Geo<T, K, DIM> g, const T* __restrict__ S, T* Q, KrySrc src, const T* __restrict__ amp,
    ArnArgs a, unsigned long long* slots, int* err, double* hess, double* sc, double* beta_out) {
  __shared__ double s_scale[65];
  const unsigned nb = gridDim.x;
  const int64_t nthreads = static_cast<int64_t>(nb) * kArnNT;
  const int64_t gtid = static_cast<int64_t>(blockIdx.x) * kArnNT + threadIdx.x;
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  unsigned seq = 0;

  // grid-wide sums double as the barriers between Gram-Schmidt steps
  auto publish = [&](double v) {
    return grid_sum<kArnNT>(v, slots, ++seq, a.spin_limit, err, [] {});
  };

  // q_0 = [S; e_p] / beta
  double acc = 0.0;
#pragma unroll
  for (int u = 0; u < UN; ++u) {
    const int64_t e = gtid + u * nthreads;
    if (e < a.ns) {
      const double v = static_cast<double>(S[e]);
      acc += v * v;
    }
  }
  const double beta = sqrt(publish(acc) + a.tail2);
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  if (lead) {
    *beta_out = beta;
    sc[0] = 1.0;
  }
  if (threadIdx.x == 0) s_scale[0] = 1.0;
  T q0[UN];
#pragma unroll
  for (int u = 0; u < UN; ++u) {
    const int64_t e = gtid + u * nthreads;
    double v = 0.0;
    if (e < a.ns)
      v = static_cast<double>(S[e]) * inv;
    else if (e == a.naug - 1 && a.tail2 > 0.0)
      v = inv;
    q0[u] = static_cast<T>(v);
    if (e < a.naug) st_coherent(Q + e, q0[u]);
  }
  (void)publish(0.0);  // Q_0 complete everywhere

  // qa holds q_i's stored column Q_i, qb the next one Q_{i+1}; the next
  // column is loaded as soon as this block has arrived at a grid-wide sum, so
  // the load overlaps the wait for the other blocks
  T w[UN], qa[UN], qb[UN];
  auto load_col = [&](T* dst, int col) {
    const T* qc = Q + col * a.ld;
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const int64_t e = gtid + u * nthreads;
      dst[u] = (e < a.naug) ? ld_coherent(qc + e) : T(0);
    }
  };
  for (int j = 0; j < a.k; ++j) {
    const T* qj = Q + j * a.ld;
    T* wout = Q + (j + 1) * a.ld;
    const T sj = static_cast<T>(s_scale[j]);
    // w = s_j H~ Q_j, and the first dot w . q_0
    acc = 0.0;
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const int64_t e = gtid + u * nthreads;
      T v = T(0);
      if (e < a.ns) {
        const int f = static_cast<int>(e / g.N);
        const int64_t idx = e - f * g.N;
        int64_t ic[3];
        decompose<DIM>(g.n, idx, ic);
        v = apply_field<T, K, BC, DIM>(g, qj, f, idx, ic);
        if (f == 0 && src.n > 0 && idx >= src.lo && idx <= src.hi) {
          for (int s = 0; s < src.n; ++s)
            if (src.idx[s] == idx) {
              double gt = 0.0;
              for (int cc = 0; cc < src.p; ++cc)
                gt += src.G[cc] * static_cast<double>(ld_coherent(qj + a.ns + cc));
              v += static_cast<T>(gt * static_cast<double>(amp[s]));
            }
        }
        v *= sj;
      } else if (e < a.naug) {
        const int cc = static_cast<int>(e - a.ns);
        v = (cc + 1 < src.p) ? ld_coherent(qj + a.ns + cc + 1) * sj : T(0);  // J q_tail
      }
      w[u] = v;
      qa[u] = q0[u];
      acc += static_cast<double>(v) * static_cast<double>(q0[u]);
    }
    double h = grid_sum<kArnNT>(acc, slots, ++seq, a.spin_limit, err, [&] {
      if (j >= 1) load_col(qb, 1);
    });
    if (lead) hess[0 * 64 + j] = h;
    double sa = 1.0;
    for (int i = 0; i <= j; ++i) {
      const bool lastc = (i == j);
      const double hs = h * sa;
      const double sb = lastc ? 1.0 : s_scale[i + 1];
      acc = 0.0;
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        const int64_t e = gtid + u * nthreads;
        const T wt = static_cast<T>(static_cast<double>(w[u]) - hs * static_cast<double>(qa[u]));
        w[u] = wt;
        if (!lastc) {
          acc += static_cast<double>(wt) * sb * static_cast<double>(qb[u]);
        } else {
          if (e < a.naug) st_coherent(wout + e, wt);
          acc += static_cast<double>(wt) * static_cast<double>(wt);
        }
      }
      if (!lastc) {
#pragma unroll
        for (int u = 0; u < UN; ++u) qa[u] = qb[u];
      }
      const double r = grid_sum<kArnNT>(acc, slots, ++seq, a.spin_limit, err, [&] {
        if (!lastc && i + 2 <= j) load_col(qb, i + 2);
      });
      if (!lastc) {
        h = r;
        if (lead) hess[(i + 1) * 64 + j] = h;
        sa = sb;
      } else {
        const double hn = sqrt(r);
        const double s = (hn > a.tol * beta) ? 1.0 / hn : 0.0;
        if (lead) {
          hess[(j + 1) * 64 + j] = hn;
          sc[j + 1] = s;
        }
        if (threadIdx.x == 0) s_scale[j + 1] = s;
        __syncthreads();
      }
    }
  }
}

__global__ void k_zero_u32(unsigned* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__global__ void k_fill_u64(unsigned long long* p, int n, unsigned long long v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace expw
