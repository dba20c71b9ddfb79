// Row-streaming Faber pass for 2D grids (order 4 or 8, zero ghost values): S
// consecutive recurrence terms per HBM sweep (Sec. 3.2, Faber recurrence),
// with no recomputation along z. The description below is for order 4 (K = 2
// weights per side); at order 8 (K = 4) every lag, reach and halo of 2 is K
// (a level K rows behind the previous one, K columns of halo per level, queues
// of 2K + 1 rows).
//
// A workgroup of 512 threads owns a band of 512 - 4S output columns and a
// segment of rows; thread t owns column t of the band grown by 2S on each
// side and walks down the segment one row per iteration. (Against 256-thread
// bands: 2 KB instead of 1 KB of each array per row and workgroup, and half
// the halo share; at 8192 x 4096, FP32, six terms, 775 us per pass instead
// of 866.) Term r (level r,
// r = 0..S-1) lags two rows behind term r-1: at iteration k the input row k
// of v_{j-1} is loaded (level -1) and level r computes its row k - 2(r + 1)
// from level r-1's rows k - 2r - 3 .. k - 2r (its own column) and its row
// k - 2(r + 1) at columns t - 2 .. t + 2 (the x-stencil). Every level keeps
// its last rows in per-thread register queues: the z-stencil and the values
// at the point come from there; only the x-neighbours cross threads, through
// one LDS row per level (double-buffered: one barrier per iteration). Level
// r is valid on columns 2(r + 1) .. 511 - 2(r + 1) of the band, so the last
// level covers the output band exactly. Rows outside the grid are zero at
// every level (the ghost rule), and a segment starts 2S rows early, so no
// row is recomputed beyond that warm-up. Level r's rows before the segment
// start minus 2(S - 1 - r) feed nothing (the next level's stencil, the older
// term and the sum start there), so a level begins 4(r + 1) iterations into
// the walk and pushes zeros before.
//
// The partial sum of an output row is formed when the last level reaches
// it, in FP64: acc_in + sum_r a_r v_r (+ a_0 v_0 on the first pass), each
// level's value at that row taken from its queue (level r's queue is 2(S -
// 1 - r) + 1 rows deep for this).
//
// Arithmetic: a term is computed entirely in T as
//   v_j = kappa (-c^2 S_v - (sigma / wscale) p | -S_p - (sigma / wscale) v)
//         - c0 v_{j-1} - cpp v_{j-2} + q amp,
// with S the difference sums over the integer weights (alpha_l / h = wscale
// wi_l) and kappa = wscale / gamma. The step's ellipse is chosen so that
// kappa, c0 and c1 are exact in T (the coefficients are computed for that
// ellipse): the only systematic rounding left is 1 / wscale, which scales the
// damping inside the absorbing layer by a relative 1e-8 at most. The partial
// sum is FP64.
//
// Per point and pass: reads v_{j-1}, v_{j-2} (3 T each), c^2 (1 T) and the
// FP64 sum (3 doubles); writes v_last, v_prev (3 T each) and the sum (3
// doubles), or the step's result (3 T) on the last pass.
#pragma once

#include "device_common.h"
#include "kernels.h"
#include "profiler.h"

namespace expw {

constexpr int kStrNT = 512;

template <typename T, int S>
struct StreamArgs {
  T kappa, c0, inv_ws;  // wscale / gamma, c0, 1 / wscale (see the arithmetic note)
  T cpp[S], q[S];
  double a_first;
  double a[S];
  int32_t bands, zseg;
  RecRun<T> rec;
};

// Queue depth of level L (-1 = the input): the z-stencil and the point
// value of the next level need the last 2K + 1 rows, the sum at the last
// level's row needs K(S - 1 - L) + 1.
template <int K, int S, bool FIRST>
constexpr int queue_depth(int L) {
  const int need = (L < 0 && !FIRST) ? 2 * K + 1 : K * (S - 1 - L) + 1;
  return need > 2 * K + 1 ? need : 2 * K + 1;
}

template <typename T, int D>
struct RowQueue {
  T p[D], vx[D], vz[D];  // slot d: the row produced d iterations ago
  __device__ __forceinline__ void push(T np, T nvx, T nvz) {
#pragma unroll
    for (int d = D - 1; d > 0; --d) {
      p[d] = p[d - 1];
      vx[d] = vx[d - 1];
      vz[d] = vz[d - 1];
    }
    p[0] = np;
    vx[0] = nvx;
    vz[0] = nvz;
  }
  __device__ __forceinline__ void clear() {
#pragma unroll
    for (int d = 0; d < D; ++d) p[d] = vx[d] = vz[d] = T(0);
  }
};

template <typename T, int K, int S, bool FIRST>
struct Levels {
  RowQueue<T, queue_depth<K, S, FIRST>(-1)> in;
  RowQueue<T, queue_depth<K, S, FIRST>(0)> l0;
  RowQueue<T, queue_depth<K, S, FIRST>(1)> l1;
  RowQueue<T, queue_depth<K, S, FIRST>(2)> l2;
  RowQueue<T, queue_depth<K, S, FIRST>(3)> l3;
  RowQueue<T, queue_depth<K, S, FIRST>(4)> l4;
  RowQueue<T, queue_depth<K, S, FIRST>(5)> l5;
};

template <int L, typename Q>
__device__ __forceinline__ auto& level_q(Q& q) {
  if constexpr (L < 0) return q.in;
  else if constexpr (L == 0) return q.l0;
  else if constexpr (L == 1) return q.l1;
  else if constexpr (L == 2) return q.l2;
  else if constexpr (L == 3) return q.l3;
  else if constexpr (L == 4) return q.l4;
  else return q.l5;
}

// One pass over band (blockIdx.x % bands) and row segment (blockIdx.x /
// bands). acc_in: the FP64 sum of the previous passes (FIRST: unused); the
// sum goes to acc_out (FP64), or to state_out rounded to T on a step's last
// pass (state_out must not alias vp or vpp). out_last / out_prev: the pass's
// last two terms (nullptr on the last pass). Requires 3 * points < 2^31.
template <typename T, int K, int S, bool FIRST>
__global__ __launch_bounds__(kStrNT) void k_faber_stream2d(
    Geo<T, K, 2> g, const T* __restrict__ vp, const T* __restrict__ vpp,
    const double* __restrict__ acc_in, T* __restrict__ out_last, T* __restrict__ out_prev,
    double* __restrict__ acc_out, T* __restrict__ state_out, StreamArgs<T, S> c, Src<T> src) {
  static_assert(S >= 2 && S <= 6, "2 to 6 terms per pass");
  static_assert(K == 2 || K == 4, "order 4 or 8");
  constexpr int W = kStrNT - 2 * K * S;
  __shared__ T s_p[2][S][kStrNT];
  __shared__ T s_vx[2][S][kStrNT];
  const int nx = static_cast<int>(g.n[0]), nz = static_cast<int>(g.n[1]);
  const int N = static_cast<int>(g.N);
  const int band = static_cast<int>(blockIdx.x) % c.bands, seg = static_cast<int>(blockIdx.x) / c.bands;
  const int t = threadIdx.x;
  const int x = band * W - K * S + t;
  const bool xin = x >= 0 && x < nx;
  const int xc = xin ? x : 0;
  const int z0 = seg * c.zseg;
  const int z1 = min(z0 + c.zseg, nz);
  const bool out_col = t >= K * S && t < kStrNT - K * S && xin;
  const T sxi = xin ? g.sint[0][xc] : T(0);
  const T sxh = xin ? g.shalf[0][xc] : T(0);
  const T w0 = g.wi[0], w1 = g.wi[1];
  const T kap = c.kappa, c0 = c.c0, iws = c.inv_ws;
  const T sxi_s = sxi * iws, sxh_s = sxh * iws;
  // sources in this column: only rows whose flat index falls in [lo, hi]
  const bool src_col = src.n > 0 && xin;

  Levels<T, K, S, FIRST> q;
  q.in.clear();
  q.l0.clear();
  q.l1.clear();
  q.l2.clear();
  q.l3.clear();
  q.l4.clear();
  q.l5.clear();

  // the values v_{j-2} of level 0's row (k - K) and the input row k + 1,
  // loaded one iteration ahead
  const int kbeg = z0 - K * S, kend = z1 - 1 + K * S;
  auto ld_row = [&](int z, const T* f, T* out3) {
    const bool in = xin && z >= 0 && z < nz;
    const int gi = in ? z * nx + x : 0;
    out3[0] = in ? f[gi] : T(0);
    out3[1] = in ? f[N + gi] : T(0);
    out3[2] = in ? f[2 * N + gi] : T(0);
  };
  T nxt_in[3], nxt_old[3];
  ld_row(kbeg, vp, nxt_in);
  if (!FIRST) ld_row(kbeg - K, vpp, nxt_old);
  else nxt_old[0] = nxt_old[1] = nxt_old[2] = T(0);
  // c^2 of the last KS + 1 rows (level r reads row k - K(r + 1): slot K(r + 1)),
  // loaded with the input row
  T c2q[K * S + 1];
#pragma unroll
  for (int d = 0; d <= K * S; ++d) c2q[d] = T(0);
  auto ld_c2 = [&](int z) -> T {
    const bool in = xin && z >= 0 && z < nz;
    return in ? g.c2[z * nx + x] : T(0);
  };
  T nxt_c2 = ld_c2(kbeg);
  // the FP64 sum of the output row, loaded one iteration ahead
  const bool out_any = out_col;
  auto ld_acc = [&](int zo, double* o3) {
    const bool in = !FIRST && out_any && zo >= z0 && zo < z1;
    const int gi = in ? zo * nx + x : 0;
    o3[0] = in ? acc_in[gi] : 0.0;
    o3[1] = in ? acc_in[N + gi] : 0.0;
    o3[2] = in ? acc_in[2 * N + gi] : 0.0;
  };
  double nxt_acc[3];
  ld_acc(kbeg - K * S, nxt_acc);

  for (int k = kbeg; k <= kend; ++k) {
    const int buf = k & 1;
    // 1. every level's row that the next level needs at this iteration (the
    //    row K behind its newest after this iteration's push) goes to LDS for
    //    the x-stencil
#define EXPW_STAGE(L)                                                       \
    if constexpr (L + 1 < S) {                                              \
      auto& Q_ = level_q<L>(q);                                             \
      s_p[buf][L + 1][t] = Q_.p[K - 1];                                     \
      s_vx[buf][L + 1][t] = Q_.vx[K - 1];                                   \
    }
    EXPW_STAGE(-1) EXPW_STAGE(0) EXPW_STAGE(1) EXPW_STAGE(2) EXPW_STAGE(3) EXPW_STAGE(4)
#undef EXPW_STAGE
    // 2. the input row k enters level -1; the next loads are issued
    const T cur_in[3] = {nxt_in[0], nxt_in[1], nxt_in[2]};
    const T old0[3] = {nxt_old[0], nxt_old[1], nxt_old[2]};
    const double acc_row[3] = {nxt_acc[0], nxt_acc[1], nxt_acc[2]};
#pragma unroll
    for (int d = K * S; d > 0; --d) c2q[d] = c2q[d - 1];
    c2q[0] = nxt_c2;
    if (k < kend) {
      ld_row(k + 1, vp, nxt_in);
      if (!FIRST) ld_row(k + 1 - K, vpp, nxt_old);
      nxt_c2 = ld_c2(k + 1);
      ld_acc(k + 1 - K * S, nxt_acc);
    }
    q.in.push(cur_in[0], cur_in[1], cur_in[2]);
    __syncthreads();

    // 3. levels 0..S-1 in order: level r computes row k - K(r + 1)
    T lastv[3] = {T(0), T(0), T(0)};  // level S-1's new row
#define EXPW_LEVEL(R)                                                                      \
    if constexpr (R < S) {                                                                 \
      auto& P_ = level_q<R - 1>(q);                                                        \
      const int z = k - K * (R + 1);                                                       \
      T nv[3] = {T(0), T(0), T(0)};                                                        \
      const bool act = t >= K * (R + 1) && t < kStrNT - K * (R + 1) && xin && z >= 0 && z < nz && \
                       k >= kbeg + 2 * K * (R + 1);                                        \
      if (act) {                                                                           \
        const T* LP = s_p[buf][R];                                                         \
        const T* LX = s_vx[buf][R];                                                        \
        const T pc = P_.p[K], vxc = P_.vx[K], vzc = P_.vz[K];                              \
        T dvx, dvz, dpx, dpz;                                                              \
        if constexpr (K == 2) {                                                            \
          dvx = w0 * (vxc - LX[t - 1]) + w1 * (LX[t + 1] - LX[t - 2]);                     \
          dvz = w0 * (vzc - P_.vz[3]) + w1 * (P_.vz[1] - P_.vz[4]);                        \
          dpx = w0 * (LP[t + 1] - pc) + w1 * (LP[t + 2] - LP[t - 1]);                      \
          dpz = w0 * (P_.p[1] - pc) + w1 * (P_.p[0] - P_.p[3]);                            \
        } else {                                                                           \
          dvx = g.wi[0] * (vxc - LX[t - 1]);                                               \
          dvz = g.wi[0] * (vzc - P_.vz[K + 1]);                                            \
          dpx = g.wi[0] * (LP[t + 1] - pc);                                                \
          dpz = g.wi[0] * (P_.p[K - 1] - pc);                                              \
          _Pragma("unroll") for (int l = 2; l <= K; ++l) {                                 \
            dvx += g.wi[l - 1] * (LX[t + l - 1] - LX[t - l]);                              \
            dvz += g.wi[l - 1] * (P_.vz[K - l + 1] - P_.vz[K + l]);                        \
            dpx += g.wi[l - 1] * (LP[t + l] - LP[t + 1 - l]);                              \
            dpz += g.wi[l - 1] * (P_.p[K - l] - P_.p[K - 1 + l]);                          \
          }                                                                                \
        }                                                                                  \
        const int gi = z * nx + x;                                                         \
        const T sp_s = sxi_s + g.sint[1][z] * iws;                                         \
        const T hp = -c2q[K * (R + 1)] * (dvx + dvz) - sp_s * pc;                          \
        const T hvx = -dpx - sxh_s * vxc;                                                  \
        const T hvz = -dpz - g.shalf[1][z] * iws * vzc;                                    \
        T o0, o1, o2;                                                                      \
        if constexpr (R == 0) {                                                            \
          o0 = old0[0];                                                                    \
          o1 = old0[1];                                                                    \
          o2 = old0[2];                                                                    \
        } else {                                                                           \
          auto& O_ = level_q<R - 2>(q);                                                    \
          o0 = O_.p[2 * K];                                                                \
          o1 = O_.vx[2 * K];                                                               \
          o2 = O_.vz[2 * K];                                                               \
        }                                                                                  \
        T src_v = T(0);                                                                    \
        if (src_col && gi >= src.lo && gi <= src.hi) src_v = src_value(src, gi) * c.q[R];  \
        const T cpp = c.cpp[R];                                                            \
        nv[0] = kap * hp - c0 * pc - cpp * o0 + src_v;                                     \
        nv[1] = kap * hvx - c0 * vxc - cpp * o1;                                           \
        nv[2] = kap * hvz - c0 * vzc - cpp * o2;                                           \
      }                                                                                    \
      if constexpr (R + 1 < S) level_q<R>(q).push(nv[0], nv[1], nv[2]);                    \
      else {                                                                               \
        lastv[0] = nv[0];                                                                  \
        lastv[1] = nv[1];                                                                  \
        lastv[2] = nv[2];                                                                  \
      }                                                                                    \
    }
    EXPW_LEVEL(0) EXPW_LEVEL(1) EXPW_LEVEL(2) EXPW_LEVEL(3) EXPW_LEVEL(4) EXPW_LEVEL(5)
#undef EXPW_LEVEL

    // 4. the output row k - KS: v_last, v_prev and the sum
    const int zo = k - K * S;
    if (out_col && zo >= z0 && zo < z1) {
      const int gi = zo * nx + x;
      double s3[3];
      if constexpr (FIRST) {
        auto& I_ = q.in;  // v_0 at row zo: slot KS of the input queue
        s3[0] = c.a_first * static_cast<double>(I_.p[K * S]);
        s3[1] = c.a_first * static_cast<double>(I_.vx[K * S]);
        s3[2] = c.a_first * static_cast<double>(I_.vz[K * S]);
      } else {
        s3[0] = acc_row[0];
        s3[1] = acc_row[1];
        s3[2] = acc_row[2];
      }
#define EXPW_SUM(R)                                                              \
      if constexpr (R + 1 < S) {                                                 \
        auto& Q_ = level_q<R>(q);                                                \
        constexpr int d = K * (S - 1 - R);                                       \
        s3[0] = fma(c.a[R], static_cast<double>(Q_.p[d]), s3[0]);                \
        s3[1] = fma(c.a[R], static_cast<double>(Q_.vx[d]), s3[1]);               \
        s3[2] = fma(c.a[R], static_cast<double>(Q_.vz[d]), s3[2]);               \
      }
      EXPW_SUM(0) EXPW_SUM(1) EXPW_SUM(2) EXPW_SUM(3) EXPW_SUM(4)
#undef EXPW_SUM
      s3[0] = fma(c.a[S - 1], static_cast<double>(lastv[0]), s3[0]);
      s3[1] = fma(c.a[S - 1], static_cast<double>(lastv[1]), s3[1]);
      s3[2] = fma(c.a[S - 1], static_cast<double>(lastv[2]), s3[2]);
      if (out_last) {
        auto& V_ = level_q<S - 2>(q);  // v_prev at row zo: slot K of level S-2
        out_last[gi] = lastv[0];
        out_last[N + gi] = lastv[1];
        out_last[2 * N + gi] = lastv[2];
        out_prev[gi] = V_.p[K];
        out_prev[N + gi] = V_.vx[K];
        out_prev[2 * N + gi] = V_.vz[K];
      }
      if (state_out) {
        const T pv = static_cast<T>(s3[0]);
        state_out[gi] = pv;
        rec_run_put(c.rec, gi, pv);
        state_out[N + gi] = static_cast<T>(s3[1]);
        state_out[2 * N + gi] = static_cast<T>(s3[2]);
      } else {
        acc_out[gi] = s3[0];
        acc_out[N + gi] = s3[1];
        acc_out[2 * N + gi] = s3[2];
      }
    }
  }
}

// Workgroups of a pass kernel resident on the device at once (CUs times the
// occupancy of the kernel; 1024 when the runtime cannot say).
template <typename T, int K, int S, bool FIRST>
int stream2d_capacity() {
  static int cap = 0;  // per kernel, at first use
  if (cap == 0) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per, reinterpret_cast<const void*>(k_faber_stream2d<T, K, S, FIRST>), kStrNT, 0) == hipSuccess &&
        cus > 0 && per > 0)
      cap = cus * per;
    else
      cap = 1024;
  }
  return cap;
}

// Rows per segment. Every workgroup of a pass runs about as long (its rows
// plus a warm-up of 2S rows), and the resident workgroups run in rounds, so
// a pass takes about ceil(bands * segments / capacity) * (rows per segment +
// 2S) row times: a second, nearly empty round costs as much as a full one.
// The segment count (segments of 64 rows or more) minimizes that.
inline int stream2d_zseg(int64_t nz, int bands, int capacity, int S) {
  const int64_t smax = nz / 64 > 1 ? nz / 64 : 1;
  int64_t best_segs = 1, best_cost = -1;
  for (int64_t segs = 1; segs <= smax; ++segs) {
    const int64_t zs = (nz + segs - 1) / segs;
    const int64_t rounds = (static_cast<int64_t>(bands) * segs + capacity - 1) / capacity;
    const int64_t cost = rounds * (zs + 2 * S);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best_segs = segs;
    }
  }
  return static_cast<int>((nz + best_segs - 1) / best_segs);
}

template <typename T, int K, int S>
int32_t launch_stream2d(hipStream_t st, Profiler* prof, const Geo<T, K, 2>& g, Src<T> src,
                        const T* vp, const T* vpp, const double* acc_in, T* out_last, T* out_prev,
                        double* acc_out, T* state_out, int j, bool first, const double* a,
                        const double* qv, double kappa, double inv_ws, double c0, double c1,
                        RecRun<T> rec) {
  constexpr int W = kStrNT - 2 * K * S;
  StreamArgs<T, S> c{};
  c.rec = rec;
  c.kappa = static_cast<T>(kappa);
  c.inv_ws = static_cast<T>(inv_ws);
  c.c0 = static_cast<T>(c0);
  if (first) c.a_first = a[0];
  for (int r = 0; r < S; ++r) {
    const int jj = j + r;
    c.a[r] = a[jj];
    c.cpp[r] = static_cast<T>(jj == 1 ? 0.0 : (jj == 2 ? 2.0 * c1 : c1));
    c.q[r] = static_cast<T>(qv[jj - 1]);
  }
  c.bands = static_cast<int>((g.n[0] + W - 1) / W);
  // (the cost model's warm-up in units of 2 rows: S at order 4, 2S at order 8)
  c.zseg = stream2d_zseg(g.n[1], c.bands,
                         first ? stream2d_capacity<T, K, S, true>() : stream2d_capacity<T, K, S, false>(), K * S / 2);
  const int64_t blocks = static_cast<int64_t>(c.bands) * ((g.n[1] + c.zseg - 1) / c.zseg);
  if (blocks > INT32_MAX) return fail(EXPW_EUNSUPPORTED, "streamed Faber pass: grid too large");
  // the source term of a level is q_r amp: src.q is set to 1 so that
  // src_value returns the amplitude sum
  src.q = 1.0;
  const double bytes = (3 + 1 + (first ? 0 : 3) + (out_last ? 6 : 0) + (state_out ? 3 : 0)) * sizeof(T) +
                       ((first ? 0 : 3) + (state_out ? 0 : 3)) * sizeof(double);
  if (first)
    launch_timed(prof, st, EXPW_KERNEL_FABER, bytes * g.N, k_faber_stream2d<T, K, S, true>,
                 dim3(static_cast<unsigned>(blocks)), dim3(kStrNT), g, vp, vpp, acc_in, out_last,
                 out_prev, acc_out, state_out, c, src);
  else
    launch_timed(prof, st, EXPW_KERNEL_FABER, bytes * g.N, k_faber_stream2d<T, K, S, false>,
                 dim3(static_cast<unsigned>(blocks)), dim3(kStrNT), g, vp, vpp, acc_in, out_last,
                 out_prev, acc_out, state_out, c, src);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(EXPW_EDEVICE, "streamed Faber pass: %s", hipGetErrorString(e));
  return EXPW_OK;
}

// The streamed passes need long row segments to amortize their 4S-row
// warm-up; a grid too small to give the chip 512 workgroups with segments
// of 64 rows or more takes the tiled passes (fused.h).
inline bool stream2d_fits(int64_t nx, int64_t nz, int S, int K = 2) {
  const int W = kStrNT - 2 * K * S;
  const int64_t bands = (nx + W - 1) / W;
  return bands * ((nz + 63) / 64) >= 512;
}

template <typename T, int K>
int32_t launch_stream_pass(int n, hipStream_t st, Profiler* prof, const Geo<T, K, 2>& g, Src<T> src,
                           const T* vp, const T* vpp, const double* acc_in, T* out_last, T* out_prev,
                           double* acc_out, T* state_out, int j, bool first, const double* a,
                           const double* q, double kappa, double inv_ws, double c0, double c1,
                           RecRun<T> rec) {
#define EXPW_SPASS(S_)                                                                           \
  case S_:                                                                                       \
    return launch_stream2d<T, K, S_>(st, prof, g, src, vp, vpp, acc_in, out_last, out_prev, acc_out, \
                                  state_out, j, first, a, q, kappa, inv_ws, c0, c1, rec);
  if constexpr (sizeof(T) == 4 && K == 2) {
    switch (n) {
      EXPW_SPASS(2) EXPW_SPASS(3) EXPW_SPASS(4) EXPW_SPASS(5) EXPW_SPASS(6)
      default: break;
    }
  } else if constexpr (sizeof(T) == 8 && K == 4) {
    // (four terms of order 8 in FP64 spill: at most three)
    switch (n) {
      EXPW_SPASS(2) EXPW_SPASS(3)
      default: break;
    }
  } else {
    switch (n) {
      EXPW_SPASS(2) EXPW_SPASS(3) EXPW_SPASS(4)
      default: break;
    }
  }
#undef EXPW_SPASS
  return fail(EXPW_EUNSUPPORTED, "no streamed pass of %d terms", n);
}

}  // namespace expw
