// Temporally blocked Faber pass for 2D grids: S consecutive terms of the
// three-term recurrence per HBM sweep.
//
// A workgroup owns a TX x TY output tile. It stages v_{j-1}, v_{j-2} (all
// three fields) and c^2 over the tile plus a halo of K*S cells in LDS, then
// runs S recurrence terms in LDS: term r is computed on the tile grown by
// K*(n-1-r) cells (n = terms of this pass), each term reading only the ring
// the previous term produced, so no other workgroup's data is needed until
// the pass ends. v_j overwrites v_{j-2} in place (the recurrence reads
// v_{j-2} only at the same point). The Faber sum for the tile's own points
// stays in registers. Only the tile is written back: v_{last}, v_{last-1}
// and the partial sum, i.e. 19 words per point per pass instead of 16 per
// term for one-term sweeps.
//
// Tiles are mapped to workgroups so that each XCD (block id mod 8) gets a
// contiguous range of tiles in raster order: halo rows shared by adjacent
// tiles then hit in that XCD's L2.
#pragma once

#include "device_common.h"
#include "internal.h"
#include "profiler.h"

namespace expw {

constexpr int kMaxFuse = 8;
constexpr int kFusedTX = 64, kFusedTY = 16, kFusedNT = 512;

template <typename T, int S>
struct FusedArgs {
  T inv_gamma, c0, a_first;
  int32_t first;  // first pass of a step: acc = a_first * v0, no v_{j-2}
  int32_t tiles_x, tiles, tiles_per_xcd;
  T a[S], cpp[S], q[S];
};

// One pass of exactly S recurrence terms. 2D grids with 3 * points < 2^31.
template <typename T, int S, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_faber_fused2d(Geo<T, 2, 2> g, const T* __restrict__ vp,
                                                      const T* __restrict__ vpp,
                                                      const T* acc_in, T* __restrict__ out_last,
                                                      T* __restrict__ out_prev, T* acc_out,
                                                      FusedArgs<T, S> c, Src<T> src) {
  constexpr int K = 2;
  constexpr int H = K * S;
  constexpr int EX = TX + 2 * H, EY = TY + 2 * H, E = EX * EY;
  constexpr int PPT = TX * TY / NT;
  static_assert(TX * TY % NT == 0, "tile must be a multiple of the block");
  __shared__ T lds[7 * E];
  __shared__ T s_xi[EX], s_xh[EX], s_zi[EY], s_zh[EY];

  // XCD-aware tile index: block b runs on XCD b % 8 and takes tile
  // (b % 8) * tiles_per_xcd + b / 8.
  const int b = blockIdx.x;
  const int tile = (b & 7) * c.tiles_per_xcd + (b >> 3);
  if (tile >= c.tiles) return;
  const int ty_ = tile / c.tiles_x, tx_ = tile - ty_ * c.tiles_x;
  const int nx = static_cast<int>(g.n[0]), nz = static_cast<int>(g.n[1]);
  const int N = static_cast<int>(g.N);
  const int x0 = tx_ * TX - H;  // global x of LDS column 0
  const int z0 = ty_ * TY - H;
  const int tid = threadIdx.x;

  T* cur = lds;
  T* old = lds + 3 * E;
  T* lc2 = lds + 6 * E;

#pragma unroll 4
  for (int e = tid; e < E; e += NT) {
    const int ly = e / EX, lx = e - ly * EX;
    const int gx = x0 + lx, gz = z0 + ly;
    const bool in = gx >= 0 && gx < nx && gz >= 0 && gz < nz;
    const int gi = in ? gz * nx + gx : 0;
    const T p0 = in ? vp[gi] : T(0), p1 = in ? vp[N + gi] : T(0), p2 = in ? vp[2 * N + gi] : T(0);
    const bool rd = in && !c.first;
    const T o0 = rd ? vpp[gi] : T(0), o1 = rd ? vpp[N + gi] : T(0), o2 = rd ? vpp[2 * N + gi] : T(0);
    const T cc = in ? g.c2[gi] : T(0);
    cur[e] = p0;
    cur[E + e] = p1;
    cur[2 * E + e] = p2;
    old[e] = o0;
    old[E + e] = o1;
    old[2 * E + e] = o2;
    lc2[e] = cc;
  }
  for (int e = tid; e < EX; e += NT) {
    const int gx = x0 + e;
    const bool in = gx >= 0 && gx < nx;
    s_xi[e] = in ? g.sint[0][gx] : T(0);
    s_xh[e] = in ? g.shalf[0][gx] : T(0);
  }
  for (int e = tid; e < EY; e += NT) {
    const int gz = z0 + e;
    const bool in = gz >= 0 && gz < nz;
    s_zi[e] = in ? g.sint[1][gz] : T(0);
    s_zh[e] = in ? g.shalf[1][gz] : T(0);
  }

  // the partial Faber sum of this thread's tile points (read before the barrier
  // so that the global loads overlap the LDS fill)
  T acc[PPT][3];
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    const int t = tid + i * NT;
    const int ty = t / TX, tx = t - ty * TX;
    const int gx = x0 + H + tx, gz = z0 + H + ty;
    const bool in = !c.first && gx < nx && gz < nz;
    const int gi = in ? gz * nx + gx : 0;
#pragma unroll
    for (int f = 0; f < 3; ++f) acc[i][f] = in ? acc_in[f * N + gi] : T(0);
  }
  __syncthreads();
  if (c.first) {
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const int t = tid + i * NT;
      const int ty = t / TX, tx = t - ty * TX;
      const int l = (ty + H) * EX + tx + H;
#pragma unroll
      for (int f = 0; f < 3; ++f) acc[i][f] = c.a_first * cur[f * E + l];
    }
  }

  const T w0 = g.w[0], w1 = g.w[1];
#pragma unroll
  for (int r = 0; r < S; ++r) {
    const int ext = K * (S - 1 - r);
    const int RW = TX + 2 * ext, RH = TY + 2 * ext;
    const int lx0 = H - ext, ly0 = H - ext;
    const T cpp = c.cpp[r];
    Src<T> sr = src;
    sr.q = c.q[r];
    const T* cp = cur;
    const T* cvx = cur + E;
    const T* cvz = cur + 2 * E;
    T* op_ = old;
    T* ovx = old + E;
    T* ovz = old + 2 * E;
    for (int e = tid; e < RW * RH; e += NT) {
      const int ry = e / RW;
      const int lx = lx0 + (e - ry * RW), ly = ly0 + ry;
      const int gx = x0 + lx, gz = z0 + ly;
      if (gx < 0 || gx >= nx || gz < 0 || gz >= nz) continue;  // ghosts stay zero
      const int l = ly * EX + lx;
      const T dvx = w0 * (cvx[l] - cvx[l - 1]) + w1 * (cvx[l + 1] - cvx[l - 2]);
      const T dvz = w0 * (cvz[l] - cvz[l - EX]) + w1 * (cvz[l + EX] - cvz[l - 2 * EX]);
      const T dpx = w0 * (cp[l + 1] - cp[l]) + w1 * (cp[l + 2] - cp[l - 1]);
      const T dpz = w0 * (cp[l + EX] - cp[l]) + w1 * (cp[l + 2 * EX] - cp[l - EX]);
      const T pc = cp[l], vxc = cvx[l], vzc = cvz[l];
      const T hp = -lc2[l] * (dvx + dvz) - (s_xi[lx] + s_zi[ly]) * pc;
      const T hvx = -dpx - s_xh[lx] * vxc;
      const T hvz = -dpz - s_zh[ly] * vzc;
      T np = hp * c.inv_gamma - c.c0 * pc - cpp * op_[l];
      np += src_value(sr, static_cast<int64_t>(gz) * nx + gx);
      const T nvx = hvx * c.inv_gamma - c.c0 * vxc - cpp * ovx[l];
      const T nvz = hvz * c.inv_gamma - c.c0 * vzc - cpp * ovz[l];
      op_[l] = np;
      ovx[l] = nvx;
      ovz[l] = nvz;
    }
    __syncthreads();
    T* tmp = cur;
    cur = old;
    old = tmp;
    const T aj = c.a[r];
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const int t = tid + i * NT;
      const int ty = t / TX, tx = t - ty * TX;
      const int l = (ty + H) * EX + tx + H;
#pragma unroll
      for (int f = 0; f < 3; ++f) acc[i][f] += aj * cur[f * E + l];
    }
  }

#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    const int t = tid + i * NT;
    const int ty = t / TX, tx = t - ty * TX;
    const int gx = x0 + H + tx, gz = z0 + H + ty;
    if (gx >= nx || gz >= nz) continue;
    const int l = (ty + H) * EX + tx + H;
    const int gi = gz * nx + gx;
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      if (out_last) {
        out_last[f * N + gi] = cur[f * E + l];
        out_prev[f * N + gi] = old[f * E + l];
      }
      acc_out[f * N + gi] = acc[i][f];
    }
  }
}

// Fusion depth actually used for a request (1 = unfused kernels).
template <typename T, int K, int BC, int DIM>
int fused_depth(int requested, int m, int64_t npts) {
  if (DIM != 2 || K != 2 || BC != 0) return 1;
  if (3 * npts >= (int64_t(1) << 31)) return 1;
  const int smax = sizeof(T) == 4 ? 8 : 4;
  int s = requested == 0 ? 4 : requested;  // default depth
  if (s > smax) s = smax;
  if (s > m) s = m;
  return s < 2 ? 1 : s;
}

inline int32_t check_tiles(int ndim, int tile_x, int tile_y) {
  (void)ndim;
  if ((tile_x != 0 && tile_x != kFusedTX) || (tile_y != 0 && tile_y != kFusedTY))
    return fail(EXPW_EUNSUPPORTED, "fused tile must be %dx%d", kFusedTX, kFusedTY);
  return EXPW_OK;
}

template <typename T, int S>
int32_t launch_fused(hipStream_t st, Profiler* prof, const Geo<T, 2, 2>& g, Src<T> src,
                     const T* vp, const T* vpp, const T* acc_in, T* out_last, T* out_prev,
                     T* acc_out, int j, bool first, const double* a, const double* q,
                     double gamma, double c0, double c1) {
  FusedArgs<T, S> c{};
  c.inv_gamma = static_cast<T>(1.0 / gamma);
  c.c0 = static_cast<T>(c0);
  c.first = first ? 1 : 0;
  c.a_first = first ? static_cast<T>(a[0]) : T(0);
  for (int r = 0; r < S; ++r) {
    const int jj = j + r;
    c.a[r] = static_cast<T>(a[jj]);
    c.cpp[r] = static_cast<T>(jj == 1 ? 0.0 : (jj == 2 ? 2.0 * c1 : c1));
    c.q[r] = static_cast<T>(q[jj - 1]);
  }
  const int tx = static_cast<int>((g.n[0] + kFusedTX - 1) / kFusedTX);
  const int ty = static_cast<int>((g.n[1] + kFusedTY - 1) / kFusedTY);
  c.tiles_x = tx;
  c.tiles = tx * ty;
  c.tiles_per_xcd = (c.tiles + 7) / 8;
  const unsigned blocks = 8u * static_cast<unsigned>(c.tiles_per_xcd);
  // algorithmic words per point: v_{j-1} (3), c^2 (1), and unless first v_{j-2}
  // and the partial sum (3 + 3); writes: the sum (3), and unless last the pair (3 + 3)
  const double words = 3 + 1 + (first ? 0 : 6) + 3 + (out_last ? 6 : 0);
  launch_timed(prof, st, EXPW_KERNEL_FABER, words * g.N * sizeof(T),
               k_faber_fused2d<T, S, kFusedTX, kFusedTY, kFusedNT>, dim3(blocks), dim3(kFusedNT), g,
               vp, vpp, acc_in, out_last, out_prev, acc_out, c, src);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(EXPW_EDEVICE, "fused Faber pass: %s", hipGetErrorString(e));
  return EXPW_OK;
}

template <typename T>
int32_t launch_pass(int n, hipStream_t st, Profiler* prof, const Geo<T, 2, 2>& g, Src<T> src,
                    const T* vp, const T* vpp, const T* acc_in, T* out_last, T* out_prev,
                    T* acc_out, int j, bool first, const double* a, const double* q,
                    double gamma, double c0, double c1) {
#define EXPW_PASS(S_)                                                                          \
  case S_:                                                                                     \
    return launch_fused<T, S_>(st, prof, g, src, vp, vpp, acc_in, out_last, out_prev, acc_out, \
                               j, first, a, q, gamma, c0, c1);
  if constexpr (sizeof(T) == 4) {
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

// One Faber step of degree m in passes of s terms (the last pass takes the
// remainder; a remainder of one term runs as an unfused final term).
// Buffers: S0 = state (v0), A/B and D/E alternate as (v_last, v_prev), C holds
// the partial sum; the last pass writes the sum into S0 unless it also read S0.
template <typename T, class Term>
int32_t faber_fused_2d(hipStream_t st, Profiler* prof, const Geo<T, 2, 2>& g, Src<T> src, T* S0,
                       T* A, T* B, T* C, T* D, T* E, const double* a, const double* q, int m,
                       int s, double gamma, double c0, double c1, Term&& final_term) {
  const int64_t ns = 3 * g.N;
  const T* in_last = S0;
  const T* in_prev = nullptr;
  T* pair[2][2] = {{A, B}, {D, E}};
  int which = 0;
  int j = 1;
  while (j <= m) {
    int n = std::min(s, m - j + 1);
    const bool first = (j == 1);
    if (n == 1) {  // a single final term: v_m from (in_last, in_prev), sum into S0
      int32_t rc = final_term(in_last, in_prev, C, S0, j);
      if (rc != EXPW_OK) return rc;
      break;
    }
    const bool last = (j + n - 1 == m);
    T* acc_out = (last && !first) ? S0 : C;
    T* ol = last ? nullptr : pair[which][0];
    T* opv = last ? nullptr : pair[which][1];
    int32_t rc = launch_pass<T>(n, st, prof, g, src, in_last, in_prev, first ? nullptr : C, ol,
                                opv, acc_out, j, first, a, q, gamma, c0, c1);
    if (rc != EXPW_OK) return rc;
    if (last && first)
      if (hipMemcpyAsync(S0, C, ns * sizeof(T), hipMemcpyDeviceToDevice, st) != hipSuccess)
        return fail(EXPW_EDEVICE, "fused Faber: copy failed");
    in_last = ol;
    in_prev = opv;
    which ^= 1;
    j += n;
  }
  return EXPW_OK;
}

}  // namespace expw
