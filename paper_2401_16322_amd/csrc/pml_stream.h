// Row-streaming Faber pass on the PML operator (Sec. 2, 2.1, 2.2 and the
// free-surface appendix; Sec. 3.2, Faber recurrence): S consecutive terms per
// HBM sweep with no recomputation along y.
//
// A workgroup of NT threads (ps_nt: 512 at FP32, 256 at FP64, whose
// two-term kernel needs more than 256 registers per lane) owns a band of
// NT - 8S output columns and a segment of rows; thread t owns column t of the
// band grown by 4S on each side. The operator's stencils reach 4 nodes along each axis (u: -4..4,
// w_x along x and w_y along y: -4..3) and the free-surface rows 0..3 read u
// down to row 8 and w_y down to row 7, so the walk goes upwards (decreasing
// row index): the first rows of the walk are the bottom ones, and by the
// time a level reaches the surface rows everything below them is known. At
// iteration k the input row jin of v_{j-1} is loaded (level -1) and level r
// computes its row jin + 4(r + 1), from level r-1's rows jin + 4r ..
// jin + 4r + 8. Every level keeps its last rows in per-thread register
// queues (slot d: the row pushed d iterations ago), whose fixed slots hold
// every y-neighbour and the values at the point; only the x-neighbours cross
// threads, through one LDS row per level (u and w_x, double-buffered: one
// barrier per iteration). Rows outside the grid (below the bottom and above
// the surface) are zero at every level and are pushed like any other row, so
// a surface row j < 4 finds level r-1's row y in slot 4 + y - j; the queues
// of u and w_y are 13 and 12 rows deep for that. Level r is valid on columns
// 4(r + 1) .. NT - 1 - 4(r + 1) of the band, so the last level covers the
// output band exactly. Level r's rows below the segment end plus 4(S - 1 - r)
// feed nothing, so a level begins 8(r + 1) iterations into the walk and
// pushes zeros before.
//
// Each level forms v_{j+r} = F_1 v_{j+r-1} - c_{j+r} v_{j+r-2} (+ q_r times
// the source amplitude on the v equation) with the arithmetic of the one-term
// kernels (pml.h), and the partial sum of an output row acc_in + sum_r
// a_{j+r} v_{j+r} (hi + lo weights, in T) is formed when the last level
// reaches it, from the queues (level r's row is 4(S - 1 - r) rows behind).
// Per point and pass: reads v_{j-1}, v_{j-2} and the sum (4 T each) and c^2,
// writes the last two terms and the sum (4 T each): 25 words for S terms
// against 12.5 per term for the pair kernel.
#pragma once

#include "device_common.h"
#include "kernels.h"
#include "pml.h"

namespace expw {

// threads per workgroup of the streamed pass (8192 x 4096, FP32, m = 16: 108
// G grid-pt matvecs/s with 512, 103.5 with 256)
template <typename T>
constexpr int ps_nt() {
  return sizeof(T) == 4 ? 512 : 256;
}

template <typename T, int S>
struct PmlStreamArgs {
  T inv_gamma, c0;
  T cpp[S];         // c of term j + r (0, 2 c1 or c1)
  T a[S], a_lo[S];  // weights of terms j .. j + S - 1 (hi + lo)
  T a_first, a_first_lo;
  double q[S];  // source scalar of each term
  int32_t bands, zseg;
};

// Queue depths of level L (-1 = the input) in a pass of S terms. Every level
// below S - 1 feeds the next one: u in slots 0..12 and w_y in 0..11 (the
// surface rows), v and w_x in slot 4. A level two below another gives it
// v_{j-2} in slot 8. The output row is in slot 4(S - 1 - L) of level L (of
// the input on a first pass: slot 4S, for a_0 v_0).
template <int S, bool FIRST>
struct PsDepth {
  static constexpr int mx(int a, int b) { return a > b ? a : b; }
  static constexpr int sum_slot(int L) { return L >= 0 ? 4 * (S - 1 - L) : (FIRST ? 4 * S : 0); }
  static constexpr int old(int L) { return L + 2 <= S - 1 ? 9 : 5; }
  static constexpr int u(int L) { return mx(13, sum_slot(L) + 1); }
  static constexpr int wy(int L) { return mx(mx(12, old(L)), sum_slot(L) + 1); }
  static constexpr int v(int L) { return mx(old(L), sum_slot(L) + 1); }
};

template <typename T, int DU, int DV, int DY>
struct PsQueue {
  T u[DU], v[DV], wx[DV], wy[DY];
  __device__ __forceinline__ void push(const T n[4]) {
#pragma unroll
    for (int d = DU - 1; d > 0; --d) u[d] = u[d - 1];
#pragma unroll
    for (int d = DV - 1; d > 0; --d) {
      v[d] = v[d - 1];
      wx[d] = wx[d - 1];
    }
#pragma unroll
    for (int d = DY - 1; d > 0; --d) wy[d] = wy[d - 1];
    u[0] = n[0];
    v[0] = n[1];
    wx[0] = n[2];
    wy[0] = n[3];
  }
  __device__ __forceinline__ void clear() {
#pragma unroll
    for (int d = 0; d < DU; ++d) u[d] = T(0);
#pragma unroll
    for (int d = 0; d < DV; ++d) v[d] = wx[d] = T(0);
#pragma unroll
    for (int d = 0; d < DY; ++d) wy[d] = T(0);
  }
};

template <typename T, int S, bool FIRST, int L>
using PsQ = PsQueue<T, PsDepth<S, FIRST>::u(L), PsDepth<S, FIRST>::v(L), PsDepth<S, FIRST>::wy(L)>;

template <typename T, int S, bool FIRST>
struct PsLevels {
  PsQ<T, S, FIRST, -1> in;
  PsQ<T, S, FIRST, 0> l0;
  PsQ<T, S, FIRST, 1> l1;
  PsQ<T, S, FIRST, 2> l2;
};

template <int L, typename Q>
__device__ __forceinline__ auto& ps_level(Q& q) {
  if constexpr (L < 0) return q.in;
  else if constexpr (L == 0) return q.l0;
  else if constexpr (L == 1) return q.l1;
  else return q.l2;
}

// The y-derivative sums of pml_point_acc at a row known at compile time:
// JT = 0..3 a surface row (j = JT), JT < 0 an interior row (j >= 4). U(0,
// dj) and WY(dj) as there; s0 = u at the node. d*: over the integer interior
// weights; p*, l*: over the surface tables' hi and lo parts (l* in FP32 only).
template <int JT, typename T, typename FU, typename FY>
__device__ __forceinline__ void pml_y_sums(const PmlGeo<T>& g, FU&& U, FY&& WY, T s0, T& dyy, T& dwy, T& dyu,
                                           T& pyy, T& pwy, T& pyu, T& lyy, T& lwy, T& lyu) {
  constexpr bool LO = sizeof(T) == 4;
  dyy = dwy = dyu = pyy = pwy = pyu = lyy = lwy = lyu = T(0);
  if constexpr (JT >= 0) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const T uk = U(0, k - JT);
      pyy += g.s2[JT][k] * uk;
      if constexpr (LO) lyy += g.s2_lo[JT][k] * uk;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const T wk = WY(k - JT);
      pwy += g.sw[JT][k] * wk;
      if constexpr (LO) lwy += g.sw_lo[JT][k] * wk;
    }
  } else {
    dyy = g.d2c * s0;
#pragma unroll
    for (int l = 1; l <= 4; ++l) {
      dyy += g.d2[l - 1] * (U(0, l) + U(0, -l));
      dwy += g.a[l - 1] * (WY(-l) - WY(l - 1));
    }
  }
  if constexpr (JT >= 0 && JT < 3) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const T uk = U(0, k - JT);
      pyu += g.s1[JT][k] * uk;
      if constexpr (LO) lyu += g.s1_lo[JT][k] * uk;
    }
  } else {
#pragma unroll
    for (int l = 1; l <= 4; ++l) dyu += g.a[l - 1] * (U(0, 1 - l) - U(0, l));
  }
}

// The four components o of H x at node (i, j) and x there (s), as
// pml_point_acc (the same sums in the same order), with the row's
// y-derivative sums taken for the surface row j < 4 or the interior; bx, bxh
// at the column, by, byh at the row, c2 at the node.
template <typename T, typename FU, typename FX, typename FY>
__device__ __forceinline__ void pml_point_row(const PmlGeo<T>& g, int j, T vc, FU&& U, FX&& WX, FY&& WY, T bx,
                                              T bxh, T by, T byh, T c2, T o[4], T s[4]) {
  s[0] = U(0, 0);
  s[1] = vc;
  s[2] = WX(0);
  s[3] = WY(0);
  T dxx = g.d2c * s[0], dwx = T(0), dxu = T(0);
#pragma unroll
  for (int l = 1; l <= 4; ++l) {
    dxx += g.d2[l - 1] * (U(l, 0) + U(-l, 0));
    dwx += g.a[l - 1] * (WX(l - 1) - WX(-l));
    dxu += g.a[l - 1] * (U(l, 0) - U(1 - l, 0));
  }
  T dyy, dwy, dyu, pyy, pwy, pyu, lyy, lwy, lyu;
  if (j >= 4) pml_y_sums<-1>(g, U, WY, s[0], dyy, dwy, dyu, pyy, pwy, pyu, lyy, lwy, lyu);
  else if (j == 3) pml_y_sums<3>(g, U, WY, s[0], dyy, dwy, dyu, pyy, pwy, pyu, lyy, lwy, lyu);
  else if (j == 2) pml_y_sums<2>(g, U, WY, s[0], dyy, dwy, dyu, pyy, pwy, pyu, lyy, lwy, lyu);
  else if (j == 1) pml_y_sums<1>(g, U, WY, s[0], dyy, dwy, dyu, pyy, pwy, pyu, lyy, lwy, lyu);
  else pml_y_sums<0>(g, U, WY, s[0], dyy, dwy, dyu, pyy, pwy, pyu, lyy, lwy, lyu);
  pml_combine(g, bx, bxh, by, byh, c2, dxx + dyy, dwx + dwy, dxu, dyu, pyy, pwy, pyu, lyy, lwy, lyu, j < 4, o, s);
}

// One pass over band (blockIdx.x % bands) and row segment (blockIdx.x /
// bands): terms j .. j + S - 1 from vp = v_{j-1} and vpp = v_{j-2} (FIRST: j
// = 1, vp = v_0, no vpp, the sum starts from a_0 v_0). acc_in: the sum of the
// earlier passes (FIRST: unused); acc_out: the new sum (the step's result on
// the last pass). out_last, out_prev: v_{j+S-1} and v_{j+S-2} (nullptr on the
// last pass). No output may alias vp, vpp or another output; acc_out may
// alias acc_in. The sum is FP64; state_out (acc_out null): the step's result,
// rounded to T.
template <typename T, int S, bool FIRST>
__global__ __launch_bounds__(ps_nt<T>()) void k_pml_faber_stream(PmlGeo<T> g, const T* __restrict__ vp,
                                                            const T* __restrict__ vpp, const double* acc_in,
                                                            T* __restrict__ out_last, T* __restrict__ out_prev,
                                                            double* acc_out, T* state_out, PmlStreamArgs<T, S> c,
                                                            Src<T> src) {
  static_assert(S >= 2 && S <= 4, "2 to 4 terms per pass");
  constexpr int NT = ps_nt<T>();
  constexpr int H = 4, W = NT - 2 * H * S;
  __shared__ T s_u[2][S][NT];
  __shared__ T s_x[2][S][NT];
  const int nx = g.nx, ny = g.ny;
  const int64_t N = g.N;
  const int band = static_cast<int>(blockIdx.x) % c.bands, seg = static_cast<int>(blockIdx.x) / c.bands;
  const int t = threadIdx.x;
  const int i = band * W - H * S + t;
  const bool xin = i >= 0 && i < nx;
  const int ic = xin ? i : 0;
  const int z0 = seg * c.zseg;
  const int z1 = min(z0 + c.zseg, ny);
  const bool out_col = t >= H * S && t < NT - H * S && xin;
  const T bxv = xin ? g.bx[ic] : T(0), bxhv = xin ? g.bxh[ic] : T(0);
  // the walk: input rows jstart, jstart - 1, ..., z0 - 4S
  const int jstart = z1 - 1 + 4 * S;
  const int niter = (z1 - z0) + 8 * S;

  PsLevels<T, S, FIRST> q;
  q.in.clear();
  q.l0.clear();
  q.l1.clear();
  q.l2.clear();

  auto ld4 = [&](const T* f, int j, bool use, T out[4]) {
    const bool in = use && xin && j >= 0 && j < ny;
    const int64_t n = in ? static_cast<int64_t>(j) * nx + i : 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = in ? f[k * N + n] : T(0);
  };
  auto ld4d = [&](const double* f, int j, bool use, double out[4]) {
    const bool in = use && xin && j >= 0 && j < ny;
    const int64_t n = in ? static_cast<int64_t>(j) * nx + i : 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = in ? f[k * N + n] : 0.0;
  };
  auto ld_c2 = [&](int j) -> T {
    const bool in = xin && j >= 0 && j < ny;
    return in ? g.c2[static_cast<int64_t>(j) * nx + i] : T(0);
  };
  // loaded one iteration ahead: the input row, v_{j-2} at level 0's row, the
  // sum at the output row and c^2 at every level's row
  T nxt_in[4], nxt_old[4], nxt_c2[S];
  double nxt_acc[4];
  ld4(vp, jstart, true, nxt_in);
  ld4(vpp, jstart + 4, !FIRST, nxt_old);
  {
    const int jo = jstart + 4 * S;
    ld4d(acc_in, jo, !FIRST && out_col && jo >= z0 && jo < z1, nxt_acc);
  }
#pragma unroll
  for (int r = 0; r < S; ++r) nxt_c2[r] = ld_c2(jstart + 4 * (r + 1));

  for (int k = 0; k < niter; ++k) {
    const int jin = jstart - k;
    const int buf = k & 1;
    // 1. level r's x-neighbours: level r-1's row jin + 4(r + 1), three rows
    //    behind its newest before this iteration's pushes
#define EXPW_PS_STAGE(L)                          \
    if constexpr (L + 1 < S) {                    \
      auto& Q_ = ps_level<L>(q);                  \
      s_u[buf][L + 1][t] = Q_.u[3];               \
      s_x[buf][L + 1][t] = Q_.wx[3];              \
    }
    EXPW_PS_STAGE(-1) EXPW_PS_STAGE(0) EXPW_PS_STAGE(1) EXPW_PS_STAGE(2)
#undef EXPW_PS_STAGE
    // 2. the input row enters level -1; the next loads are issued
    const T cur_in[4] = {nxt_in[0], nxt_in[1], nxt_in[2], nxt_in[3]};
    const T old0[4] = {nxt_old[0], nxt_old[1], nxt_old[2], nxt_old[3]};
    const double acc_row[4] = {nxt_acc[0], nxt_acc[1], nxt_acc[2], nxt_acc[3]};
    T c2l[S];
#pragma unroll
    for (int r = 0; r < S; ++r) c2l[r] = nxt_c2[r];
    if (k + 1 < niter) {
      const int jn = jin - 1;
      ld4(vp, jn, true, nxt_in);
      ld4(vpp, jn + 4, !FIRST, nxt_old);
      const int jo = jn + 4 * S;
      ld4d(acc_in, jo, !FIRST && out_col && jo >= z0 && jo < z1, nxt_acc);
#pragma unroll
      for (int r = 0; r < S; ++r) nxt_c2[r] = ld_c2(jn + 4 * (r + 1));
    }
    q.in.push(cur_in);
    __syncthreads();

    // 3. levels 0..S-1 in order: level r computes row jin + 4(r + 1)
    T lastv[4] = {T(0), T(0), T(0), T(0)};
#define EXPW_PS_LEVEL(R)                                                                           \
    if constexpr (R < S) {                                                                         \
      auto& P_ = ps_level<R - 1>(q);                                                               \
      const int jr = jin + 4 * (R + 1);                                                            \
      T nv[4] = {T(0), T(0), T(0), T(0)};                                                          \
      const bool act = t >= H * (R + 1) && t < NT - H * (R + 1) && xin && jr >= 0 && jr < ny &&   \
                       k >= 8 * (R + 1);                                                           \
      if (act) {                                                                                   \
        const T* LU = s_u[buf][R];                                                                 \
        const T* LX = s_x[buf][R];                                                                 \
        auto U = [&](int di, int dj) -> T { return di == 0 ? P_.u[4 + dj] : LU[t + di]; };         \
        auto WX = [&](int di) -> T { return di == 0 ? P_.wx[4] : LX[t + di]; };                    \
        auto WY = [&](int dj) -> T { return P_.wy[4 + dj]; };                                      \
        const T byv = g.by[jr], byhv = g.byh[jr];                                                  \
        T o[4], sc[4];                                                                             \
        pml_point_row(g, jr, P_.v[4], U, WX, WY, bxv, bxhv, byv, byhv, c2l[R], o, sc);            \
        T old[4];                                                                                  \
        if constexpr (R == 0) {                                                                    \
          old[0] = old0[0]; old[1] = old0[1]; old[2] = old0[2]; old[3] = old0[3];                  \
        } else {                                                                                   \
          auto& O_ = ps_level<R - 2>(q);                                                           \
          old[0] = O_.u[8]; old[1] = O_.v[8]; old[2] = O_.wx[8]; old[3] = O_.wy[8];                \
        }                                                                                          \
        Src<T> s_ = src;                                                                           \
        s_.q = c.q[R];                                                                             \
        const int64_t n_ = static_cast<int64_t>(jr) * nx + i;                                      \
        _Pragma("unroll") for (int f = 0; f < 4; ++f) {                                            \
          T val = o[f] * c.inv_gamma - c.c0 * sc[f] - c.cpp[R] * old[f];                           \
          if (f == 1) val += src_value(s_, n_);                                                    \
          nv[f] = val;                                                                             \
        }                                                                                          \
      }                                                                                            \
      if constexpr (R + 1 < S) ps_level<R>(q).push(nv);                                            \
      else {                                                                                       \
        lastv[0] = nv[0]; lastv[1] = nv[1]; lastv[2] = nv[2]; lastv[3] = nv[3];                    \
      }                                                                                            \
    }
    EXPW_PS_LEVEL(0) EXPW_PS_LEVEL(1) EXPW_PS_LEVEL(2) EXPW_PS_LEVEL(3)
#undef EXPW_PS_LEVEL

    // 4. the output row jin + 4S: the last two terms and the sum
    const int jo = jin + 4 * S;
    if (out_col && jo >= z0 && jo < z1) {
      const int64_t n = static_cast<int64_t>(jo) * nx + i;
      double acc[4];
      if constexpr (FIRST) {
        auto& I_ = q.in;  // v_0 at the output row
        constexpr int d = 4 * S;
        acc[0] = sum_add(0.0, c.a_first, c.a_first_lo, I_.u[d]);
        acc[1] = sum_add(0.0, c.a_first, c.a_first_lo, I_.v[d]);
        acc[2] = sum_add(0.0, c.a_first, c.a_first_lo, I_.wx[d]);
        acc[3] = sum_add(0.0, c.a_first, c.a_first_lo, I_.wy[d]);
      } else {
#pragma unroll
        for (int f = 0; f < 4; ++f) acc[f] = acc_row[f];
      }
#define EXPW_PS_SUM(R)                                                     \
      if constexpr (R + 1 < S) {                                           \
        auto& Q_ = ps_level<R>(q);                                         \
        constexpr int d = 4 * (S - 1 - R);                                 \
        acc[0] = sum_add(acc[0], c.a[R], c.a_lo[R], Q_.u[d]);              \
        acc[1] = sum_add(acc[1], c.a[R], c.a_lo[R], Q_.v[d]);              \
        acc[2] = sum_add(acc[2], c.a[R], c.a_lo[R], Q_.wx[d]);             \
        acc[3] = sum_add(acc[3], c.a[R], c.a_lo[R], Q_.wy[d]);             \
      }
      EXPW_PS_SUM(0) EXPW_PS_SUM(1) EXPW_PS_SUM(2)
#undef EXPW_PS_SUM
#pragma unroll
      for (int f = 0; f < 4; ++f) acc[f] = sum_add(acc[f], c.a[S - 1], c.a_lo[S - 1], lastv[f]);
      if (out_last) {
        auto& V_ = ps_level<S - 2>(q);  // v_{j+S-2} at the output row
        const T pv[4] = {V_.u[4], V_.v[4], V_.wx[4], V_.wy[4]};
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          out_last[f * N + n] = lastv[f];
          out_prev[f * N + n] = pv[f];
        }
      }
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        if (state_out) state_out[f * N + n] = static_cast<T>(acc[f]);
        else acc_out[f * N + n] = acc[f];
      }
    }
  }
}

// Workgroups of a streamed PML pass resident at once (CUs times the
// occupancy of the kernel; 1024 when the runtime cannot say).
template <typename T, int S, bool FIRST>
int pml_stream_capacity() {
  static int cap = 0;
  if (cap == 0) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per, reinterpret_cast<const void*>(k_pml_faber_stream<T, S, FIRST>), ps_nt<T>(), 0) == hipSuccess &&
        cus > 0 && per > 0)
      cap = cus * per;
    else
      cap = 1024;
  }
  return cap;
}

// Rows per segment: a pass takes about ceil(bands * segments / capacity) *
// (rows per segment + 8S) row times; the segment count (segments of 64 rows
// or more) minimizes that.
inline int pml_stream_zseg(int64_t ny, int bands, int capacity, int S) {
  const int64_t smax = ny / 64 > 1 ? ny / 64 : 1;
  int64_t best_segs = 1, best_cost = -1;
  for (int64_t segs = 1; segs <= smax; ++segs) {
    const int64_t zs = (ny + segs - 1) / segs;
    const int64_t rounds = (static_cast<int64_t>(bands) * segs + capacity - 1) / capacity;
    const int64_t cost = rounds * (zs + 8 * S);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best_segs = segs;
    }
  }
  return static_cast<int>((ny + best_segs - 1) / best_segs);
}

// The streamed passes need long row segments to amortize their 8S-row
// warm-up: taken automatically when the grid gives 512 workgroups (of the
// 256-thread kind; 256 of 512 threads) with segments of 64 rows or more.
template <typename T>
bool pml_stream_fits(int64_t nx, int64_t ny, int S) {
  const int W = ps_nt<T>() - 8 * S;
  const int64_t bands = (nx + W - 1) / W;
  return bands * ((ny + 63) / 64) * ps_nt<T>() >= 512 * 256;
}

// Terms j .. j + n - 1 in one streamed pass (n <= S of the instantiations).
template <typename T, int S>
int32_t launch_pml_stream(hipStream_t st, const PmlGeo<T>& g, Src<T> src, const T* vp, const T* vpp,
                          const double* acc_in, T* out_last, T* out_prev, double* acc_out, T* state_out,
                          int j, const double* a,
                          const double* q, double gs, double c0s, double c1s) {
  constexpr int NT = ps_nt<T>();
  constexpr int W = NT - 8 * S;
  const bool first = j == 1;
  PmlStreamArgs<T, S> c{};
  c.inv_gamma = static_cast<T>(1.0 / gs);
  c.c0 = static_cast<T>(c0s);
  if (first) split_weight(a[0], &c.a_first, &c.a_first_lo);
  for (int r = 0; r < S; ++r) {
    const int jj = j + r;
    c.cpp[r] = static_cast<T>(jj == 1 ? 0.0 : (jj == 2 ? 2.0 * c1s : c1s));
    split_weight(a[jj], &c.a[r], &c.a_lo[r]);
    c.q[r] = q[jj - 1];
  }
  c.bands = static_cast<int>((g.nx + W - 1) / W);
  c.zseg = pml_stream_zseg(g.ny, c.bands,
                           first ? pml_stream_capacity<T, S, true>() : pml_stream_capacity<T, S, false>(), S);
  const int64_t blocks = static_cast<int64_t>(c.bands) * ((g.ny + c.zseg - 1) / c.zseg);
  if (blocks > INT32_MAX) return fail(EXPW_EUNSUPPORTED, "streamed PML pass: grid too large");
  if (first)
    k_pml_faber_stream<T, S, true><<<static_cast<unsigned>(blocks), NT, 0, st>>>(
        g, vp, nullptr, nullptr, out_last, out_prev, acc_out, state_out, c, src);
  else
    k_pml_faber_stream<T, S, false><<<static_cast<unsigned>(blocks), NT, 0, st>>>(
        g, vp, vpp, acc_in, out_last, out_prev, acc_out, state_out, c, src);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(EXPW_EDEVICE, "streamed PML pass: %s", hipGetErrorString(e));
  return EXPW_OK;
}

}  // namespace expw
