// Temporally blocked Faber pass for 2D grids: S consecutive terms of the
// three-term recurrence per HBM sweep.
//
// A workgroup owns a TX x TY output tile. Term r of the pass is computed on the
// tile grown by K*(S-1-r) cells (the ring the next term needs), so after S
// terms the tile itself is exact and no other workgroup's data was needed.
// The tile size follows S so that the largest region is exactly 64 columns by
// 48 rows: wave w of the 16 handles rows w, w+16, w+32 of it, lane l column
// l, so every LDS row access of a wave is one contiguous 64-element segment
// and every point's role is fixed for the whole pass. The current generation
// v_{j-1} (three fields) lives in LDS over the tile plus a halo of K*S cells
// and is read with its stencil neighbours; everything the recurrence needs
// only at the point itself stays in registers: v_{j-2}, c^2, the damping
// values, the last term in which the point is still needed, its source
// amplitude and the new values. Each term computes into registers, then
// (after a barrier) writes v_j over v_{j-1} in LDS. The tile's Faber partial
// sum is kept in LDS. Only the tile is written back: v_last, v_last-1 and the
// partial sum, i.e. 19 words per point per pass instead of 16 per term for
// one-term sweeps.
//
// Every term is computed entirely in T as in the row-streamed passes
// (stream2d.h): the difference sums over the integer weights, kappa =
// wscale / gamma, c0 and c1 exact in T on the step's ellipse, the damping
// scaled by 1 / wscale; the partial sum is FP64 (in LDS and between passes),
// and the last pass rounds it to T once.
//
// Tiles are mapped to workgroups so that each XCD (block id mod 8) owns a
// band of tile columns walked row by row: halo rows shared by neighbouring
// tiles then hit in that XCD's L2.
#pragma once

#include "device_common.h"
#include "internal.h"
#include "profiler.h"

namespace expw {

constexpr int kMaxFuse = 8;
constexpr int kFusedNT = 1024;             // 16 waves
constexpr int kFusedRX = 64, kFusedRY = 48;  // largest region of a pass

// Output tile of a pass of S terms (stencil half-width K: 2 for order 4, 4 for order 8).
template <int S, int K = 2>
struct FusedTile {
  static constexpr int TX = kFusedRX - 2 * K * (S - 1);
  static constexpr int TY = kFusedRY - 2 * K * (S - 1);
};

template <typename T, int S>
struct FusedArgs {
  T kappa, c0, inv_ws;  // wscale / gamma, c0, 1 / wscale
  double a_first;
  int32_t first;  // first pass of a step: acc = a_first * v0, no v_{j-2}
  int32_t tiles_x, tiles_y, band_w;
  double a[S];
  T cpp[S], q[S];
  RecRun<T> rec;  // receivers recorded from the sum (last pass of a step only)
  // when set, every term j0 + r of the pass is also stored, over the tiles,
  // at terms + (j0 + r - 1) * terms_ld (the terms of a step recomputed for
  // its reverse sweep)
  T* terms;
  int64_t terms_ld;
  int32_t j0;
};

// One pass over tile (tx_, ty_) of the recurrence terms r0..S-1 of an S-term
// pass (r0 > 0 runs the last S - r0 terms only: a shorter pass on the same
// tile). 2D grids with 3 * points < 2^31.
// acc_in: the FP64 sum of the previous passes (not read on the first); the
// sum goes to acc_out (FP64) or, on a step's last pass, to state_out rounded
// to T (state_out must not alias vp or vpp); with neither, the sum is not
// formed (a pass that only stores its terms through c.terms).
template <typename T, int S, int K = 2>
__device__ __forceinline__ void fused2d_pass(const Geo<T, K, 2>& g, const T* __restrict__ vp,
                                             const T* __restrict__ vpp,
                                             const double* __restrict__ acc_in,
                                             T* __restrict__ out_last, T* __restrict__ out_prev,
                                             double* __restrict__ acc_out, T* __restrict__ state_out,
                                             const FusedArgs<T, S>& c, const Src<T>& src, int tx_,
                                             int ty_, int r0) {
  constexpr int H = K * S;
  constexpr int TX = FusedTile<S, K>::TX, TY = FusedTile<S, K>::TY;
  constexpr int EX = TX + 2 * H, EY = TY + 2 * H, E = EX * EY;
  constexpr int X0 = H - K * (S - 1);  // first column/row of the largest region (= K)
  constexpr int NSL = kFusedRY / 16;   // rows per wave
  static_assert(TX + 2 * K * (S - 1) == 64, "largest region is one wave wide");
  __shared__ T cur[3 * E];
  __shared__ double sacc[3 * TX * TY];

  const int nx = static_cast<int>(g.n[0]), nz = static_cast<int>(g.n[1]);
  const int N = static_cast<int>(g.N);
  const int x0 = tx_ * TX - H;  // global x of LDS column 0
  const int z0 = ty_ * TY - H;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;

  // v_{j-1} over tile + halo into LDS (zero outside the domain)
#pragma unroll 4
  for (int e = tid; e < E; e += kFusedNT) {
    const int ly = e / EX, lx = e - ly * EX;
    const int gx = x0 + lx, gz = z0 + ly;
    const bool in = gx >= 0 && gx < nx && gz >= 0 && gz < nz;
    const int gi = in ? gz * nx + gx : 0;
    cur[e] = in ? vp[gi] : T(0);
    cur[E + e] = in ? vp[N + gi] : T(0);
    cur[2 * E + e] = in ? vp[2 * N + gi] : T(0);
  }
  // this thread's points: column X0 + lane of rows X0 + wave + 16 i
  const int lx = X0 + lane;
  const int gx = x0 + lx;
  const int dx = lx < H ? H - lx : (lx >= H + TX ? lx - (H + TX - 1) : 0);
  const T iws = c.inv_ws;
  const T sxi = (gx >= 0 && gx < nx) ? g.sint[0][gx] : T(0);
  const T sxh_s = ((gx >= 0 && gx < nx) ? g.shalf[0][gx] : T(0)) * iws;
  int last[NSL];  // last term that needs the point (-1: outside the domain)
  T old[NSL][3], cc2[NSL], sp[NSL], szh[NSL], amp[NSL], nv[NSL][3];  // sp, szh: scaled by 1 / wscale
#pragma unroll
  for (int i = 0; i < NSL; ++i) {
    const int ly = X0 + wave + 16 * i;
    const int gz = z0 + ly;
    const bool in = gx >= 0 && gx < nx && gz >= 0 && gz < nz;
    const int dz = ly < H ? H - ly : (ly >= H + TY ? ly - (H + TY - 1) : 0);
    const int ring = dx > dz ? dx : dz;  // cells outside the tile
    last[i] = in ? S - 1 - (ring + K - 1) / K : -1;
    const int gi = in ? gz * nx + gx : 0;
    const bool rd = in && !c.first;
    old[i][0] = rd ? vpp[gi] : T(0);
    old[i][1] = rd ? vpp[N + gi] : T(0);
    old[i][2] = rd ? vpp[2 * N + gi] : T(0);
    cc2[i] = in ? g.c2[gi] : T(0);
    const T szi = in ? g.sint[1][gz] : T(0);
    szh[i] = (in ? g.shalf[1][gz] : T(0)) * iws;
    sp[i] = sxi * iws + szi * iws;
    // sum of the source amplitudes at this point
    T am = T(0);
    if (in && src.n > 0 && gi >= src.lo && gi <= src.hi)
      for (int s2 = 0; s2 < src.n; ++s2)
        if (src.idx[s2] == gi) am += src.amp[s2];
    amp[i] = am;
    nv[i][0] = nv[i][1] = nv[i][2] = T(0);
  }
  const bool sum = acc_out != nullptr || state_out != nullptr;
  // the partial sum of the tile (not read on the first pass)
  if (!c.first && sum) {
    for (int t = tid; t < TX * TY; t += kFusedNT) {
      const int ty = t / TX, tx = t - ty * TX;
      const int gxx = x0 + H + tx, gz = z0 + H + ty;
      const bool in = gxx < nx && gz < nz;
      const int gi = in ? gz * nx + gxx : 0;
      sacc[t] = in ? acc_in[gi] : 0.0;
      sacc[TX * TY + t] = in ? acc_in[N + gi] : 0.0;
      sacc[2 * TX * TY + t] = in ? acc_in[2 * N + gi] : 0.0;
    }
  }
  __syncthreads();
  if (c.first) {
    for (int t = tid; t < TX * TY; t += kFusedNT) {
      const int ty = t / TX, tx = t - ty * TX;
      const int l = (ty + H) * EX + tx + H;
      sacc[t] = c.a_first * static_cast<double>(cur[l]);
      sacc[TX * TY + t] = c.a_first * static_cast<double>(cur[E + l]);
      sacc[2 * TX * TY + t] = c.a_first * static_cast<double>(cur[2 * E + l]);
    }
  }

  const T* cp = cur;
  const T* cvx = cur + E;
  const T* cvz = cur + 2 * E;
#pragma unroll
  for (int r = 0; r < S; ++r) {
    if (r < r0) continue;  // block-uniform
    const T cpp = c.cpp[r];
    const T qr = c.q[r];
    const T kap = c.kappa, cz = c.c0;
#pragma unroll
    for (int i = 0; i < NSL; ++i) {
      if (r <= last[i]) {
        const int l = (X0 + wave + 16 * i) * EX + lx;
        const T pc = cp[l], vxc = cvx[l], vzc = cvz[l];
        // difference sums over the integer weights; the term in T
        T dvx = T(0), dvz = T(0), dpx = T(0), dpz = T(0);
#pragma unroll
        for (int q = 1; q <= K; ++q) {
          const T wq = g.wi[q - 1];
          dvx += wq * (cvx[l + q - 1] - cvx[l - q]);
          dvz += wq * (cvz[l + (q - 1) * EX] - cvz[l - q * EX]);
          dpx += wq * (cp[l + q] - cp[l + 1 - q]);
          dpz += wq * (cp[l + q * EX] - cp[l + (1 - q) * EX]);
        }
        const T hp = -cc2[i] * (dvx + dvz) - sp[i] * pc;
        const T hvx = -dpx - sxh_s * vxc;
        const T hvz = -dpz - szh[i] * vzc;
        nv[i][0] = kap * hp - cz * pc - cpp * old[i][0] + qr * amp[i];
        nv[i][1] = kap * hvx - cz * vxc - cpp * old[i][1];
        nv[i][2] = kap * hvz - cz * vzc - cpp * old[i][2];
        // v_{j-1} at the point becomes the next term's v_{j-2}
        old[i][0] = pc;
        old[i][1] = vxc;
        old[i][2] = vzc;
      }
    }
    __syncthreads();  // every read of v_{j-1} is done
    const double aj = c.a[r];
#pragma unroll
    for (int i = 0; i < NSL; ++i) {
      if (r <= last[i]) {
        const int ly = X0 + wave + 16 * i;
        const int l = ly * EX + lx;
        cur[l] = nv[i][0];
        cur[E + l] = nv[i][1];
        cur[2 * E + l] = nv[i][2];
        if (last[i] == S - 1 && lx >= H && lx < H + TX && ly >= H && ly < H + TY) {
          const int t = (ly - H) * TX + (lx - H);
          sacc[t] = fma(aj, static_cast<double>(nv[i][0]), sacc[t]);
          sacc[TX * TY + t] = fma(aj, static_cast<double>(nv[i][1]), sacc[TX * TY + t]);
          sacc[2 * TX * TY + t] = fma(aj, static_cast<double>(nv[i][2]), sacc[2 * TX * TY + t]);
          if (c.terms) {
            T* tr = c.terms + static_cast<int64_t>(c.j0 + r - 1) * c.terms_ld + (z0 + ly) * nx + gx;
            tr[0] = nv[i][0];
            tr[N] = nv[i][1];
            tr[2 * N] = nv[i][2];
          }
        }
      }
    }
    __syncthreads();  // v_j complete in LDS
  }

  // write back the tile: the pair (v_last, v_last-1) from registers, the sum from LDS
  if (out_last) {
#pragma unroll
    for (int i = 0; i < NSL; ++i) {
      const int ly = X0 + wave + 16 * i;
      if (last[i] == S - 1 && lx >= H && lx < H + TX && ly >= H && ly < H + TY) {
        const int gi = (z0 + ly) * nx + gx;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
          out_last[f * N + gi] = nv[i][f];
          out_prev[f * N + gi] = old[i][f];
        }
      }
    }
  }
  for (int t = tid; t < TX * TY && sum; t += kFusedNT) {
    const int ty = t / TX, tx = t - ty * TX;
    const int gxx = x0 + H + tx, gz = z0 + H + ty;
    if (gxx >= nx || gz >= nz) continue;
    const int gi = gz * nx + gxx;
    if (state_out) {
      const T pv = static_cast<T>(sacc[t]);
      state_out[gi] = pv;
      rec_run_put(c.rec, gi, pv);
      state_out[N + gi] = static_cast<T>(sacc[TX * TY + t]);
      state_out[2 * N + gi] = static_cast<T>(sacc[2 * TX * TY + t]);
    } else {
      acc_out[gi] = sacc[t];
      acc_out[N + gi] = sacc[TX * TY + t];
      acc_out[2 * N + gi] = sacc[2 * TX * TY + t];
    }
  }
}

// One pass of exactly S recurrence terms over every tile of the grid.
// XCD-aware tile order: block b runs on XCD b % 8, which owns a band of
// band_w tile columns and walks it row by row (k = b / 8), so the tiles above
// and below a tile run on the same XCD at about the same time and their
// shared halo rows are read from its L2.
template <typename T, int S, int K>
__global__ __launch_bounds__(kFusedNT, sizeof(T) == 4 ? 8 : 4) void k_faber_fused2d(
    Geo<T, K, 2> g, const T* __restrict__ vp, const T* __restrict__ vpp, const double* acc_in,
    T* __restrict__ out_last, T* __restrict__ out_prev, double* acc_out, T* state_out,
    FusedArgs<T, S> c, Src<T> src) {
  const int b = blockIdx.x;
  const int kk = b >> 3;
  const int ty_ = kk / c.band_w;
  const int tx_ = (b & 7) * c.band_w + (kk - ty_ * c.band_w);
  if (tx_ >= c.tiles_x || ty_ >= c.tiles_y) return;
  fused2d_pass<T, S, K>(g, vp, vpp, acc_in, out_last, out_prev, acc_out, state_out, c, src, tx_, ty_, 0);
}

// Fusion depth actually used for a request (1 = unfused kernels): 2D order 4
// with zero ghosts up to 6 (FP32) or 4 (FP64) terms, default 6 (FP32) or 4; 2D order 8
// with zero ghosts up to 4 terms, default 3; 3D FP32 order 4 with zero ghosts
// 2 terms unless fuse = 1 is asked for.
template <typename T, int K, int BC, int DIM>
int fused_depth(int requested, int m, int64_t npts) {
  if (BC != 0) return 1;
  // 3D FP32 order 4: passes of two terms by default (fused3d.h; 52 against 48
  // G grid-pt matvecs/s for one term per sweep at 256^3), fuse = 1 forces one
  // term per sweep; FP64 runs one term per sweep (the two-term pass spills)
  if (DIM == 3) return (K == 2 && sizeof(T) == 4 && requested != 1 && m >= 2) ? 2 : 1;
  if (3 * npts >= (int64_t(1) << 31)) return 1;
  // order 4: the row-streaming or tiled passes, up to 6 terms at FP32 and 4
  // at FP64, default 6 (FP32) and 4 (FP64); order 8: the tiled or
  // row-streaming passes, up to 4, default 3 (the Faber step raises it to 4
  // for streamed FP32 passes and caps streamed FP64 passes at 3)
  const int smax = (K == 2 && sizeof(T) == 4) ? 6 : 4;
  int s = requested == 0 ? (K == 2 ? (sizeof(T) == 4 ? 6 : 4) : 3) : requested;
  if (s > smax) s = smax;
  if (s > m) s = m;
  return s < 2 ? 1 : s;
}

template <typename T, int S, int K>
int32_t launch_fused(hipStream_t st, Profiler* prof, const Geo<T, K, 2>& g, Src<T> src,
                     const T* vp, const T* vpp, const double* acc_in, T* out_last, T* out_prev,
                     double* acc_out, T* state_out, int j, bool first, const double* a,
                     const double* q, double kappa, double inv_ws, double c0, double c1, RecRun<T> rec,
                     T* terms = nullptr) {
  FusedArgs<T, S> c{};
  c.terms = terms;
  c.terms_ld = 3 * g.N;
  c.j0 = j;
  c.rec = rec;
  c.kappa = static_cast<T>(kappa);
  c.inv_ws = static_cast<T>(inv_ws);
  c.c0 = static_cast<T>(c0);
  c.first = first ? 1 : 0;
  if (first) c.a_first = a[0];
  for (int r = 0; r < S; ++r) {
    const int jj = j + r;
    c.a[r] = a[jj];
    c.cpp[r] = static_cast<T>(jj == 1 ? 0.0 : (jj == 2 ? 2.0 * c1 : c1));
    c.q[r] = static_cast<T>(q[jj - 1]);
  }
  constexpr int TX = FusedTile<S, K>::TX, TY = FusedTile<S, K>::TY;
  const int tx = static_cast<int>((g.n[0] + TX - 1) / TX);
  const int ty = static_cast<int>((g.n[1] + TY - 1) / TY);
  c.tiles_x = tx;
  c.tiles_y = ty;
  c.band_w = (tx + 7) / 8;
  const unsigned blocks = 8u * static_cast<unsigned>(c.band_w) * static_cast<unsigned>(ty);
  // algorithmic bytes per point: reads v_{j-1} (3 T), c^2 (1 T), and unless
  // first v_{j-2} (3 T) and the FP64 sum (3 doubles); writes the sum (3
  // doubles, or the step's result: 3 T), and unless last the pair (6 T)
  const bool sum = acc_out != nullptr || state_out != nullptr;
  const double bytes = (3 + 1 + (first ? 0 : 3) + (out_last ? 6 : 0) + (state_out ? 3 : 0) + (terms ? 3 * S : 0)) *
                           sizeof(T) +
                       ((first || !sum ? 0 : 3) + (state_out || !sum ? 0 : 3)) * sizeof(double);
  launch_timed(prof, st, EXPW_KERNEL_FABER, bytes * g.N, k_faber_fused2d<T, S, K>,
               dim3(blocks), dim3(kFusedNT), g, vp, vpp, acc_in, out_last, out_prev, acc_out,
               state_out, c, src);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(EXPW_EDEVICE, "fused Faber pass: %s", hipGetErrorString(e));
  return EXPW_OK;
}

template <typename T, int K>
int32_t launch_pass(int n, hipStream_t st, Profiler* prof, const Geo<T, K, 2>& g, Src<T> src,
                    const T* vp, const T* vpp, const double* acc_in, T* out_last, T* out_prev,
                    double* acc_out, T* state_out, int j, bool first, const double* a,
                    const double* q, double kappa, double inv_ws, double c0, double c1, RecRun<T> rec,
                    T* terms = nullptr) {
#define EXPW_PASS(S_)                                                                          \
  case S_:                                                                                     \
    return launch_fused<T, S_, K>(st, prof, g, src, vp, vpp, acc_in, out_last, out_prev,      \
                                  acc_out, state_out, j, first, a, q, kappa, inv_ws, c0, c1, rec, terms);
  if constexpr (sizeof(T) == 4 && K == 2) {
    switch (n) {
      EXPW_PASS(2) EXPW_PASS(3) EXPW_PASS(4) EXPW_PASS(5) EXPW_PASS(6) EXPW_PASS(7) EXPW_PASS(8)
      default: break;
    }
  } else {
    switch (n) {
      EXPW_PASS(2) EXPW_PASS(3) EXPW_PASS(4)
      default: break;
    }
  }
#undef EXPW_PASS
  return fail(EXPW_EUNSUPPORTED, "no fused pass of %d terms", n);
}

// The buffers of a Faber step: the FP64 partial sum C and two (v_last,
// v_prev) pairs of the storage precision.
template <typename T>
struct FaberBufs {
  double* C;
  T *A, *B, *D, *E;
};

// One Faber step of degree m in passes of s terms (the last pass takes the
// remainder; a remainder of one term runs as an unfused final term).
// S0 = state (v0); A/B and D/E alternate as (v_last, v_prev); C holds the
// FP64 partial sum between passes. The last pass rounds the sum into S0,
// except when it is also the first (it reads S0 with its halo): then into A,
// copied to S0 afterwards.
// pass(n, vp, vpp, acc_in, out_last, out_prev, acc_out, state_out, j, first)
// launches one pass of n terms starting at term j; final_term(vp, vpp,
// acc_in, state_out, j) the unfused last term.
template <typename T, class Term, class Pass>
int32_t faber_fused_passes(hipStream_t st, int64_t ns, T* S0, const FaberBufs<T>& b, int m, int s,
                           Term&& final_term, Pass&& pass) {
  const T* in_last = S0;
  const T* in_prev = nullptr;
  T* pair[2][2] = {{b.A, b.B}, {b.D, b.E}};
  int which = 0;
  int j = 1;
  while (j <= m) {
    int n = std::min(s, m - j + 1);
    const bool first = (j == 1);
    if (n == 1) {  // a single final term: v_m from (in_last, in_prev), result into S0
      int32_t rc = final_term(in_last, in_prev, b.C, S0, j);
      if (rc != EXPW_OK) return rc;
      break;
    }
    const bool last = (j + n - 1 == m);
    T* ol = last ? nullptr : pair[which][0];
    T* opv = last ? nullptr : pair[which][1];
    double* acc_out = last ? nullptr : b.C;
    T* state_out = last ? (first ? b.A : S0) : nullptr;
    int32_t rc = pass(n, in_last, in_prev, first ? nullptr : b.C, ol, opv, acc_out, state_out, j, first);
    if (rc != EXPW_OK) return rc;
    if (last && first)
      if (hipMemcpyAsync(S0, b.A, ns * sizeof(T), hipMemcpyDeviceToDevice, st) != hipSuccess)
        return fail(EXPW_EDEVICE, "fused Faber: copy failed");
    in_last = ol;
    in_prev = opv;
    which ^= 1;
    j += n;
  }
  return EXPW_OK;
}

}  // namespace expw
