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

namespace expw {

constexpr int kMaxFuse = 8;
constexpr int kFusedTX = 64, kFusedTY = 16;

template <typename T, int S>
struct FusedArgs {
  T inv_gamma, c0, a_first;
  int32_t first;   // first pass of a step: acc = a_first * v0, no v_{j-2}
  int32_t nterms;  // terms in this pass, 1..S
  int32_t tiles_x, tiles, tiles_per_xcd;
  T a[S], cpp[S], q[S];
};

template <typename T, int S, int TX, int TY>
__global__ __launch_bounds__(kBlock) void k_faber_fused2d(Geo<T, 2, 2> g, const T* __restrict__ vp,
                                                          const T* __restrict__ vpp,
                                                          const T* acc_in, T* __restrict__ out_last,
                                                          T* __restrict__ out_prev, T* acc_out,
                                                          FusedArgs<T, S> c, Src<T> src) {
  constexpr int K = 2;
  constexpr int H = K * S;
  constexpr int EX = TX + 2 * H, EY = TY + 2 * H, E = EX * EY;
  constexpr int PPT = TX * TY / kBlock;
  static_assert(TX * TY % kBlock == 0, "tile must be a multiple of the block");
  __shared__ T lds[7 * E];
  __shared__ T s_xi[EX], s_xh[EX], s_zi[EY], s_zh[EY];

  // XCD-aware tile index: block b runs on XCD b % 8 and takes tile
  // (b % 8) * tiles_per_xcd + b / 8.
  const int b = blockIdx.x;
  const int tile = (b & 7) * c.tiles_per_xcd + (b >> 3);
  if (tile >= c.tiles) return;
  const int ty_ = tile / c.tiles_x, tx_ = tile - ty_ * c.tiles_x;
  const int64_t nx = g.n[0], nz = g.n[1], N = g.N;
  const int64_t x0 = static_cast<int64_t>(tx_) * TX - H;  // global x of LDS column 0
  const int64_t z0 = static_cast<int64_t>(ty_) * TY - H;
  const int tid = threadIdx.x;

  T* cur = lds;
  T* old = lds + 3 * E;
  T* lc2 = lds + 6 * E;

  for (int e = tid; e < E; e += kBlock) {
    const int ly = e / EX, lx = e - ly * EX;
    const int64_t gx = x0 + lx, gz = z0 + ly;
    const bool in = gx >= 0 && gx < nx && gz >= 0 && gz < nz;
    const int64_t gi = gz * nx + gx;
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      cur[f * E + e] = in ? vp[f * N + gi] : T(0);
      old[f * E + e] = (in && !c.first) ? vpp[f * N + gi] : T(0);
    }
    lc2[e] = in ? g.c2[gi] : T(0);
  }
  for (int e = tid; e < EX; e += kBlock) {
    const int64_t gx = x0 + e;
    const bool in = gx >= 0 && gx < nx;
    s_xi[e] = in ? g.sint[0][gx] : T(0);
    s_xh[e] = in ? g.shalf[0][gx] : T(0);
  }
  for (int e = tid; e < EY; e += kBlock) {
    const int64_t gz = z0 + e;
    const bool in = gz >= 0 && gz < nz;
    s_zi[e] = in ? g.sint[1][gz] : T(0);
    s_zh[e] = in ? g.shalf[1][gz] : T(0);
  }
  __syncthreads();

  // the partial Faber sum of this thread's tile points
  T acc[PPT][3];
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    const int t = tid + i * kBlock;
    const int ty = t / TX, tx = t - ty * TX;
    const int l = (ty + H) * EX + tx + H;
    const int64_t gx = x0 + H + tx, gz = z0 + H + ty;
    const bool in = gx < nx && gz < nz;
    const int64_t gi = gz * nx + gx;
#pragma unroll
    for (int f = 0; f < 3; ++f)
      acc[i][f] = c.first ? c.a_first * cur[f * E + l] : (in ? acc_in[f * N + gi] : T(0));
  }

  const T w0 = g.w[0], w1 = g.w[1];
  for (int r = 0; r < c.nterms; ++r) {
    const int ext = K * (c.nterms - 1 - r);
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
    for (int e = tid; e < RW * RH; e += kBlock) {
      const int ry = e / RW;
      const int lx = lx0 + (e - ry * RW), ly = ly0 + ry;
      const int64_t gx = x0 + lx, gz = z0 + ly;
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
      np += src_value(sr, gz * nx + gx);
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
      const int t = tid + i * kBlock;
      const int ty = t / TX, tx = t - ty * TX;
      const int l = (ty + H) * EX + tx + H;
#pragma unroll
      for (int f = 0; f < 3; ++f) acc[i][f] += aj * cur[f * E + l];
    }
  }

#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    const int t = tid + i * kBlock;
    const int ty = t / TX, tx = t - ty * TX;
    const int64_t gx = x0 + H + tx, gz = z0 + H + ty;
    if (gx >= nx || gz >= nz) continue;
    const int l = (ty + H) * EX + tx + H;
    const int64_t gi = gz * nx + gx;
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
int fused_depth(int requested, int m) {
  if (DIM != 2 || K != 2 || BC != 0) return 1;
  int s = requested;
  if (s == 0) s = sizeof(T) == 4 ? 4 : 2;  // default depth
  if (sizeof(T) == 8 && s > 4) s = 4;
  if (s > m) s = m;
  if (s < 2) return 1;
  // supported instantiations
  if (sizeof(T) == 4) {
    if (s >= 8) return 8;
    if (s >= 6) return 6;
    return s;  // 2, 3, 4, 5 -> below
  }
  return s >= 4 ? 4 : 2;
}

inline int32_t check_tiles(int ndim, int tile_x, int tile_y) {
  (void)ndim;
  if ((tile_x != 0 && tile_x != kFusedTX) || (tile_y != 0 && tile_y != kFusedTY))
    return fail(EXPW_EUNSUPPORTED, "fused tile must be %dx%d", kFusedTX, kFusedTY);
  return EXPW_OK;
}

template <typename T, int S>
int32_t launch_fused(hipStream_t st, const Geo<T, 2, 2>& g, Src<T> src, const T* vp,
                     const T* vpp, const T* acc_in, T* out_last, T* out_prev, T* acc_out,
                     FusedArgs<T, S> c) {
  const int tx = static_cast<int>((g.n[0] + kFusedTX - 1) / kFusedTX);
  const int ty = static_cast<int>((g.n[1] + kFusedTY - 1) / kFusedTY);
  c.tiles_x = tx;
  c.tiles = tx * ty;
  c.tiles_per_xcd = (c.tiles + 7) / 8;
  const unsigned blocks = 8u * static_cast<unsigned>(c.tiles_per_xcd);
  k_faber_fused2d<T, S, kFusedTX, kFusedTY><<<blocks, kBlock, 0, st>>>(g, vp, vpp, acc_in, out_last,
                                                                       out_prev, acc_out, c, src);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(EXPW_EDEVICE, "fused Faber pass: %s", hipGetErrorString(e));
  return EXPW_OK;
}

// One Faber step of degree m in passes of S terms. Buffers: S0 = state (v0),
// A/B and D/E alternate as (v_last, v_prev) pairs, C holds the partial sum.
template <typename T, int S>
int32_t faber_fused_s(hipStream_t st, const Geo<T, 2, 2>& g, Src<T> src, T* S0, T* A, T* B, T* C,
                      T* D, T* E, const double* a, const double* q, int m, double gamma, double c0,
                      double c1) {
  FusedArgs<T, S> c{};
  c.inv_gamma = static_cast<T>(1.0 / gamma);
  c.c0 = static_cast<T>(c0);
  const int64_t ns = 3 * g.N;
  const T* in_last = S0;
  const T* in_prev = nullptr;
  T* pair[2][2] = {{A, B}, {D, E}};
  int which = 0;
  int j = 1;
  while (j <= m) {
    const int n = std::min(S, m - j + 1);
    const bool first = (j == 1), last = (j + n - 1 == m);
    c.first = first ? 1 : 0;
    c.a_first = first ? static_cast<T>(a[0]) : T(0);
    c.nterms = n;
    for (int r = 0; r < S; ++r) {
      const int jj = j + r;
      c.a[r] = (r < n) ? static_cast<T>(a[jj]) : T(0);
      c.cpp[r] = static_cast<T>(jj == 1 ? 0.0 : (jj == 2 ? 2.0 * c1 : c1));
      c.q[r] = (r < n) ? static_cast<T>(q[jj - 1]) : T(0);
    }
    T* acc_out = (last && !first) ? S0 : C;
    T* ol = last ? nullptr : pair[which][0];
    T* opv = last ? nullptr : pair[which][1];
    int32_t rc = launch_fused<T, S>(st, g, src, in_last, in_prev, first ? nullptr : C, ol, opv,
                                    acc_out, c);
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

template <typename T, int K, int BC, int DIM>
int32_t faber_fused(hipStream_t st, const Geo<T, K, DIM>& g, Src<T> src, T* S0, T* A, T* B, T* C,
                    T* D, T* E, const double* a, const double* q, int m, int s, double gamma,
                    double c0, double c1) {
  if constexpr (DIM == 2 && K == 2 && BC == 0) {
    if constexpr (sizeof(T) == 4) {
      switch (s) {
        case 2: return faber_fused_s<T, 2>(st, g, src, S0, A, B, C, D, E, a, q, m, gamma, c0, c1);
        case 3: return faber_fused_s<T, 3>(st, g, src, S0, A, B, C, D, E, a, q, m, gamma, c0, c1);
        case 4:
        case 5: return faber_fused_s<T, 4>(st, g, src, S0, A, B, C, D, E, a, q, m, gamma, c0, c1);
        case 6:
        case 7: return faber_fused_s<T, 6>(st, g, src, S0, A, B, C, D, E, a, q, m, gamma, c0, c1);
        default: return faber_fused_s<T, 8>(st, g, src, S0, A, B, C, D, E, a, q, m, gamma, c0, c1);
      }
    } else {
      if (s >= 4) return faber_fused_s<T, 4>(st, g, src, S0, A, B, C, D, E, a, q, m, gamma, c0, c1);
      return faber_fused_s<T, 2>(st, g, src, S0, A, B, C, D, E, a, q, m, gamma, c0, c1);
    }
  } else {
    return fail(EXPW_EUNSUPPORTED, "fused Faber pass needs a 2D order-4 zero-ghost grid");
  }
}

}  // namespace expw
