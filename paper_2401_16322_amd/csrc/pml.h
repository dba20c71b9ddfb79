// The paper's own spatial operator (Sec. 2, 2.1, 2.2 and the appendix on the
// free surface): the 2D acoustic PML system in (u, v, w_x, w_y),
//   (H x)_u  = v
//   (H x)_v  = -b_x b_y u + c^2 (d_xx u + d_yy u) - (b_x + b_y) v + c^2 (d_x w_x + d_y w_y)
//   (H x)_wx = (b_y - b_x) d_x u - b_x w_x        at (i + 1/2, j)
//   (H x)_wy = (b_x - b_y) d_y u - b_y w_y        at (i, j + 1/2)
// with u, v, c at nodes (i, j), row j = 0 the free surface (y = -j h, y up),
// 8th-order staggered first derivatives and centred second derivatives,
// zero values outside the two sides and the bottom, and at the top rows the
// appendix's one-sided stencils (d_yy u at rows 0..3, d_y u at half rows
// 0..2) and Fornberg weights for d_y w_y at rows 0..3 (w_y = 0 on the
// surface). Layout: four fields of ny x nx points, x fastest.
#pragma once

#include "device_common.h"
#include "kernels.h"

namespace expw {

// Coefficients of one Faber term on the PML operator (Sec. 3.2, Faber
// recurrence): as FaberTerm, computed in the storage precision with each
// weight a as hi + lo in T (lo = a - hi, zero in FP64), so that the rounding
// of a weight does not repeat in every step.
template <typename T>
struct PmlTerm {
  T inv_gamma, c0, cpp, a_first, a_j, a_first_lo, a_j_lo;
  int32_t first;
};

// The interior stencils use their integer weights, exact in T, and scale
// each sum once by sc1 = 1/(107520 h) (first derivative) or sc2 = 1/(5040
// h^2) (second derivative). With the weights rounded to FP32 one by one, a
// stencil loses its exact consistency (the second-derivative weights no
// longer sum to zero, for one): an error term of order u / h^2 that a whole
// FP32 run accumulates as phase error. The rounding of a scale only rescales
// the operator by at most 2^-24. The one-sided tables of the four surface
// rows, which are not integers, and 1/h, 1/h^2 are held as hi + lo in T (lo
// = w - hi rounded to T, zero in FP64).
template <typename T>
struct PmlGeo {
  int32_t nx, ny;
  int64_t N;
  T ih, ih2, ih_lo, ih2_lo;  // 1/h, 1/h^2
  T sc1, sc2;                // 1/(107520 h), 1/(5040 h^2)
  T a[4];                    // staggered first derivative: 107520 alpha_l (integers)
  T d2c, d2[4];              // centred second derivative times 5040: d2c u_i + sum d2_l (u_{i+l} + u_{i-l})
  T s2[4][9], s2_lo[4][9];   // h^2 d_yy u at rows 0..3 from u_0..u_8
  T s1[3][8], s1_lo[3][8];   // h d_y u at half rows 0..2 from u_0..u_7
  T sw[4][8], sw_lo[4][8];   // h d_y w_y at rows 0..3 from w_0..w_7
  const T* __restrict__ c2;
  const T* __restrict__ bx;   // beta_x at nodes, at half points
  const T* __restrict__ bxh;
  const T* __restrict__ by;   // beta_y at rows, at half rows
  const T* __restrict__ byh;
};

// f(i, j) with zero outside the grid
template <typename T>
__device__ __forceinline__ T pml_at(const PmlGeo<T>& g, const T* f, int i, int j) {
  return (i >= 0 && i < g.nx && j >= 0 && j < g.ny) ? f[static_cast<int64_t>(j) * g.nx + i] : T(0);
}

// The components of H x at a node from its derivative sums: i* over the
// integer interior weights (units of the scales sc2 for ixy, sc1 for iw, ixu,
// iyu), p* over the surface tables' hi parts and l* over their lo parts
// (units of 1/h^2 for pxy, lxy and 1/h for the others); s, c^2 and the
// profiles at the node; surf: a surface row (j < 4), where the tables apply.
// The partial sum of a Faber step on the PML operator is FP64 between terms
// and passes (FP32 sums drift over long FP32 runs): acc + a x with a given
// as hi + lo in T.
template <typename T>
__device__ __forceinline__ double sum_add(double acc, T hi, T lo, T x) {
  return fma(static_cast<double>(hi) + static_cast<double>(lo), static_cast<double>(x), acc);
}

template <typename T>
__device__ __forceinline__ void pml_combine(const PmlGeo<T>& g, T bx, T bxh, T by, T byh, T c2, T ixy, T iw,
                                            T ixu, T iyu, T pxy, T pw, T pyu, T lxy, T lw, T lyu, bool surf,
                                            T o[4], const T s[4]) {
  T sxy, sw, sxu, syu;
  if constexpr (sizeof(T) == 4) {
    sxy = ixy * g.sc2;
    sw = iw * g.sc1;
    sxu = ixu * g.sc1;
    syu = iyu * g.sc1;
    if (surf) {  // the tables' sums (zero below the surface rows)
      const T qxy = pxy + lxy, qw = pw + lw, qyu = pyu + lyu;
      sxy = sxy + (qxy * g.ih2 + qxy * g.ih2_lo);
      sw = sw + (qw * g.ih + qw * g.ih_lo);
      syu = syu + (qyu * g.ih + qyu * g.ih_lo);
    }
  } else {
    sxy = ixy * g.sc2;
    sw = iw * g.sc1;
    sxu = ixu * g.sc1;
    syu = iyu * g.sc1;
    if (surf) {
      sxy = sxy + pxy * g.ih2;
      sw = sw + pw * g.ih;
      syu = syu + pyu * g.ih;
    }
  }
  o[0] = s[1];
  o[1] = -bx * by * s[0] + c2 * sxy - (bx + by) * s[1] + c2 * sw;
  o[2] = (by - bxh) * sxu - bxh * s[2];
  o[3] = (bx - byh) * syu - byh * s[3];
}

// The four components o of H x at node (i, j), and x itself there (s), with
// the neighbours read through accessors relative to the node, each zero
// outside the grid: U(di, dj) = u(i + di, j + dj) for |di|, |dj| <= 4 and, at
// the four top rows, dj up to 8 - j; WX(di) = w_x(i + di, j) for -4 <= di <= 3;
// WY(dj) = w_y(i, j + dj) for -4 <= dj <= 3 and, at the top rows, up to 7 - j.
template <typename T, typename FU, typename FX, typename FY>
__device__ __forceinline__ void pml_point_acc(const PmlGeo<T>& g, int i, int j, T vc, FU&& U, FX&& WX,
                                              FY&& WY, T o[4], T s[4]) {
  s[0] = U(0, 0);
  s[1] = vc;
  s[2] = WX(0);
  s[3] = WY(0);
  constexpr bool LO = sizeof(T) == 4;  // add the surface tables' lo parts
  // x: integer weights
  T dxx = g.d2c * s[0], dwx = T(0), dxu = T(0);
#pragma unroll
  for (int l = 1; l <= 4; ++l) {
    dxx += g.d2[l - 1] * (U(l, 0) + U(-l, 0));
    dwx += g.a[l - 1] * (WX(l - 1) - WX(-l));
    dxu += g.a[l - 1] * (U(l, 0) - U(1 - l, 0));
  }
  // y: integer weights in the interior, the tables at the surface rows
  T dyy = T(0), dwy = T(0), dyu = T(0);
  T pyy = T(0), pwy = T(0), pyu = T(0), lyy = T(0), lwy = T(0), lyu = T(0);
  if (j < 4) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const T uk = U(0, k - j);
      pyy += g.s2[j][k] * uk;
      if constexpr (LO) lyy += g.s2_lo[j][k] * uk;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const T wk = WY(k - j);
      pwy += g.sw[j][k] * wk;
      if constexpr (LO) lwy += g.sw_lo[j][k] * wk;
    }
  } else {
    dyy = g.d2c * s[0];
#pragma unroll
    for (int l = 1; l <= 4; ++l) {
      dyy += g.d2[l - 1] * (U(0, l) + U(0, -l));
      dwy += g.a[l - 1] * (WY(-l) - WY(l - 1));
    }
  }
  if (j < 3) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const T uk = U(0, k - j);
      pyu += g.s1[j][k] * uk;
      if constexpr (LO) lyu += g.s1_lo[j][k] * uk;
    }
  } else {
#pragma unroll
    for (int l = 1; l <= 4; ++l) dyu += g.a[l - 1] * (U(0, 1 - l) - U(0, l));
  }
  const int64_t n = static_cast<int64_t>(j) * g.nx + i;
  pml_combine(g, g.bx[i], g.bxh[i], g.by[j], g.byh[j], g.c2[n], dxx + dyy, dwx + dwy, dxu, dyu, pyy, pwy, pyu,
              lyy, lwy, lyu, j < 4, o, s);
}

// The same with every read from global memory.
template <typename T>
__device__ __forceinline__ void pml_point(const PmlGeo<T>& g, const T* x, int i, int j, T o[4],
                                          T s[4]) {
  const T* u = x;
  const T* wx = x + 2 * g.N;
  const T* wy = x + 3 * g.N;
  pml_point_acc(
      g, i, j, x[g.N + static_cast<int64_t>(j) * g.nx + i],
      [&](int di, int dj) { return pml_at(g, u, i + di, j + dj); },
      [&](int di) { return pml_at(g, wx, i + di, j); },
      [&](int dj) { return pml_at(g, wy, i, j + dj); }, o, s);
}

// Tiles of the LDS kernel: 64 x 16 nodes per 256-thread block (4 rows per
// thread), with 4-cell halos of u (both axes), w_x (along x) and w_y (along y).
constexpr int kPmlTX = 64, kPmlTY = 16, kPmlHalo = 4;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_pml_apply(PmlGeo<T> g, const T* __restrict__ x,
                                                      T* __restrict__ y) {
  const int64_t n = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x;
  if (n >= g.N) return;
  const int j = static_cast<int>(n / g.nx), i = static_cast<int>(n - static_cast<int64_t>(j) * g.nx);
  T o[4], s[4];
  pml_point(g, x, i, j, o, s);
#pragma unroll
  for (int f = 0; f < 4; ++f) y[f * g.N + n] = o[f];
}

// One Faber term (Sec. 3.2) on the PML operator, as k_faber_term, one thread
// per node with every read from global memory (the path for grids with few
// tiles). The source enters the v equation. The FP64 sum goes to acc_out, or
// rounded to T into state_out (the step's last term; acc_out null). acc_out
// may alias acc_in; vp is read with a halo and must not alias an output;
// vout == nullptr skips storing v_j.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pml_faber_term(PmlGeo<T> g, const T* vp, const T* vpp,
                                                           T* vout, const double* acc_in, double* acc_out,
                                                           T* state_out, PmlTerm<T> c, Src<T> src) {
  const int64_t n = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x;
  if (n >= g.N) return;
  const int j = static_cast<int>(n / g.nx), i = static_cast<int>(n - static_cast<int64_t>(j) * g.nx);
  T o[4], s[4];
  pml_point(g, vp, i, j, o, s);
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const int64_t e = f * g.N + n;
    T v = o[f] * c.inv_gamma - c.c0 * s[f];
    if (vpp) v -= c.cpp * vpp[e];
    if (f == 1) v += src_value(src, n);
    if (vout) vout[e] = v;
    double acc = c.first ? sum_add(0.0, c.a_first, c.a_first_lo, s[f]) : acc_in[e];
    acc = sum_add(acc, c.a_j, c.a_j_lo, v);
    if (state_out) state_out[e] = static_cast<T>(acc);
    else acc_out[e] = acc;
  }
}

// The same term with the stencil operands staged in LDS (the path for grids
// with many tiles).
// XCD-aware tile order of the tiled PML kernels: workgroup b runs on XCD
// b mod 8, which owns a band of band_w = ceil(tiles_x / 8) tile columns
// walked row by row, so the tiles beside and below a tile run on the same
// XCD at about the same time and their shared halo reaches its L2. The grid
// is 8 band_w tiles_y workgroups; false for the workgroups past the last
// column.
__device__ __forceinline__ bool pml_band_tile(int tiles_x, int tiles_y, int band_w, int& tx0, int& ty0) {
  const int b = static_cast<int>(blockIdx.x), kk = b >> 3;
  ty0 = kk / band_w;
  tx0 = (b & 7) * band_w + (kk - ty0 * band_w);
  return tx0 < tiles_x && ty0 < tiles_y;
}

// tiles_x = ceil(nx / 64); one block per 64 x 16 tile, in the band order above. vout may alias vpp and acc_out may alias acc_in or vpp; vp is
// read with a halo and must not alias an output; vout == nullptr skips v_j.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pml_faber_term_lds(PmlGeo<T> g, const T* vp, const T* vpp,
                                                               T* vout, const double* acc_in, double* acc_out,
                                                               T* state_out, PmlTerm<T> c, Src<T> src,
                                                               int tiles_x, int tiles_y, int band_w) {
  static_assert(kBlock == 256 && kPmlTX == 64, "4 waves, one tile column per lane");
  constexpr int TX = kPmlTX, TY = kPmlTY, HL = kPmlHalo;
  constexpr int UX = TX + 2 * HL, UY = TY + 2 * HL;
  __shared__ T su[UY][UX];  // u at rows j0 - 4 .. j0 + 19, columns i0 - 4 .. i0 + 67
  __shared__ T sx[TY][UX];  // w_x at rows j0 .. j0 + 15, columns i0 - 4 .. i0 + 67
  __shared__ T sy[UY][TX];  // w_y at rows j0 - 4 .. j0 + 19, columns i0 .. i0 + 63
  int tx0, ty0;
  if (!pml_band_tile(tiles_x, tiles_y, band_w, tx0, ty0)) return;
  const int i0 = tx0 * TX, j0 = ty0 * TY;
  const T* u = vp;
  const T* wx = vp + 2 * g.N;
  const T* wy = vp + 3 * g.N;
  for (int e = threadIdx.x; e < UY * UX; e += kBlock) {
    const int r = e / UX, q = e - r * UX;
    su[r][q] = pml_at(g, u, i0 - HL + q, j0 - HL + r);
  }
  for (int e = threadIdx.x; e < TY * UX; e += kBlock) {
    const int r = e / UX, q = e - r * UX;
    sx[r][q] = pml_at(g, wx, i0 - HL + q, j0 + r);
  }
  for (int e = threadIdx.x; e < UY * TX; e += kBlock) {
    const int r = e / TX, q = e - r * TX;
    sy[r][q] = pml_at(g, wy, i0 + q, j0 - HL + r);
  }
  __syncthreads();
  const int tx = threadIdx.x & 63, tyb = threadIdx.x >> 6;
  const int i = i0 + tx;
#pragma unroll
  for (int k = 0; k < TY / 4; ++k) {
    const int ly = tyb + 4 * k, j = j0 + ly;
    if (i >= g.nx || j >= g.ny) continue;
    const int64_t n = static_cast<int64_t>(j) * g.nx + i;
    T o[4], s[4];
    pml_point_acc(
        g, i, j, vp[g.N + n],
        [&](int di, int dj) { return su[ly + HL + dj][tx + HL + di]; },
        [&](int di) { return sx[ly][tx + HL + di]; },
        [&](int dj) { return sy[ly + HL + dj][tx]; }, o, s);
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const int64_t e = f * g.N + n;
      T v = o[f] * c.inv_gamma - c.c0 * s[f];
      if (vpp) v -= c.cpp * vpp[e];
      if (f == 1) v += src_value(src, n);
      if (vout) vout[e] = v;
      double acc = c.first ? sum_add(0.0, c.a_first, c.a_first_lo, s[f]) : acc_in[e];
      acc = sum_add(acc, c.a_j, c.a_j_lo, v);
      if (state_out) state_out[e] = static_cast<T>(acc);
      else acc_out[e] = acc;
    }
  }
}

// Two Faber terms j and j + 1 per pass on the PML operator (temporal
// blocking). A block of NT threads owns a 64 x TY tile. It stages v_{j-1} on the
// tile grown by 8 cells (u on both axes, w_x along x, w_y along y; v on the
// tile grown by 4), computes term j on the tile grown by 4 (R1) into LDS (zero
// outside the grid, so the next stencils see the zero values there), then term
// j + 1 on the tile from LDS. Per tile point it writes v_j, v_{j+1} (each
// skipped when its pointer is null) and the sum acc_in + a_j v_j + a_{j+1}
// v_{j+1} (for c0.first: a_0 v_{j-1} + ...). vpp (v_{j-2}, null for j = 1)
// is read on R1, so no output may alias vp or vpp; acc_out may alias acc_in.
// The FP64 sum goes to acc_out, or rounded to T into state_out (acc_out null).
template <typename T, int NT, int TY>
__global__ __launch_bounds__(NT) void k_pml_faber_pair_lds(PmlGeo<T> g, const T* vp, const T* vpp,
                                                           T* out0, T* out1, const double* acc_in,
                                                           double* acc_out, T* state_out, PmlTerm<T> c0,
                                                           PmlTerm<T> c1, Src<T> s0, Src<T> s1,
                                                           int tiles_x, int tiles_y, int band_w) {
  constexpr int TX = kPmlTX, NW = NT / 64;
  static_assert(NT % 64 == 0 && TY % NW == 0, "whole waves, each wave a set of tile rows");
  constexpr int AX = TX + 16, AY = TY + 16;  // tile grown by 8
  constexpr int BX = TX + 8, BY = TY + 8;    // tile grown by 4 (R1)
  __shared__ T au[AY][AX];   // v_{j-1}: u on the tile grown by 8
  __shared__ T av[BY][BX];   //          v on R1
  __shared__ T ax[BY][AX];   //          w_x on R1's rows, columns grown by 8
  __shared__ T ay[AY][BX];   //          w_y on R1's columns, rows grown by 8
  __shared__ T bu[BY][BX], bv[BY][BX], bx[BY][BX], by[BY][BX];  // v_j on R1
  int tx0, ty0;
  if (!pml_band_tile(tiles_x, tiles_y, band_w, tx0, ty0)) return;
  const int i0 = tx0 * TX, j0 = ty0 * TY;
  const T* u = vp;
  const T* v = vp + g.N;
  const T* wx = vp + 2 * g.N;
  const T* wy = vp + 3 * g.N;
  for (int e = threadIdx.x; e < AY * AX; e += NT) {
    const int r = e / AX, q = e - r * AX;
    au[r][q] = pml_at(g, u, i0 - 8 + q, j0 - 8 + r);
  }
  for (int e = threadIdx.x; e < BY * BX; e += NT) {
    const int r = e / BX, q = e - r * BX;
    av[r][q] = pml_at(g, v, i0 - 4 + q, j0 - 4 + r);
  }
  for (int e = threadIdx.x; e < BY * AX; e += NT) {
    const int r = e / AX, q = e - r * AX;
    ax[r][q] = pml_at(g, wx, i0 - 8 + q, j0 - 4 + r);
  }
  for (int e = threadIdx.x; e < AY * BX; e += NT) {
    const int r = e / BX, q = e - r * BX;
    ay[r][q] = pml_at(g, wy, i0 - 4 + q, j0 - 8 + r);
  }
  __syncthreads();
  // term j on R1: point (r, q) is node (i0 - 4 + q, j0 - 4 + r)
  for (int e = threadIdx.x; e < BY * BX; e += NT) {
    const int r = e / BX, q = e - r * BX;
    const int i = i0 - 4 + q, j = j0 - 4 + r;
    T f[4] = {T(0), T(0), T(0), T(0)};
    if (i >= 0 && i < g.nx && j >= 0 && j < g.ny) {
      const int64_t n = static_cast<int64_t>(j) * g.nx + i;
      T o[4], sc[4];
      pml_point_acc(
          g, i, j, av[r][q],
          [&](int di, int dj) { return au[r + 4 + dj][q + 4 + di]; },
          [&](int di) { return ax[r][q + 4 + di]; },
          [&](int dj) { return ay[r + 4 + dj][q]; }, o, sc);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        T val = o[k] * c0.inv_gamma - c0.c0 * sc[k];
        if (vpp) val -= c0.cpp * vpp[k * g.N + n];
        if (k == 1) val += src_value(s0, n);
        f[k] = val;
      }
    }
    bu[r][q] = f[0];
    bv[r][q] = f[1];
    bx[r][q] = f[2];
    by[r][q] = f[3];
  }
  __syncthreads();
  // term j + 1 on the tile; v_{j-1} there is the older term
  const int tx = threadIdx.x & 63, tyb = threadIdx.x >> 6;
  const int i = i0 + tx;
#pragma unroll
  for (int k4 = 0; k4 < TY / NW; ++k4) {
    const int ly = tyb + NW * k4, j = j0 + ly;
    if (i >= g.nx || j >= g.ny) continue;
    const int64_t n = static_cast<int64_t>(j) * g.nx + i;
    T o[4], sc[4];
    pml_point_acc(
        g, i, j, bv[ly + 4][tx + 4],
        [&](int di, int dj) { return bu[ly + 4 + dj][tx + 4 + di]; },
        [&](int di) { return bx[ly + 4][tx + 4 + di]; },
        [&](int dj) { return by[ly + 4 + dj][tx + 4]; }, o, sc);
    const T old[4] = {au[ly + 8][tx + 8], av[ly + 4][tx + 4], ax[ly + 4][tx + 8], ay[ly + 8][tx + 4]};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t e = k * g.N + n;
      T val = o[k] * c1.inv_gamma - c1.c0 * sc[k] - c1.cpp * old[k];
      if (k == 1) val += src_value(s1, n);
      if (out0) out0[e] = sc[k];
      if (out1) out1[e] = val;
      double acc = c0.first ? sum_add(0.0, c0.a_first, c0.a_first_lo, old[k]) : acc_in[e];
      acc = sum_add(acc, c0.a_j, c0.a_j_lo, sc[k]);
      acc = sum_add(acc, c1.a_j, c1.a_j_lo, val);
      if (state_out) state_out[e] = static_cast<T>(acc);
      else acc_out[e] = acc;
    }
  }
}

// One classical RK4 stage on the PML operator (Sec. 3.1), as k_rk4_stage:
// k = H y + s(t_stage) (source on the v equation); ynext = u + cy k (if
// ynext), acc_out = (acc_in ? acc_in : u) + ca k. y is read with a halo and
// must not alias an output.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pml_rk4_stage(PmlGeo<T> g, const T* y, const T* u,
                                                          const T* acc_in, T* ynext, T* acc_out,
                                                          T cy, T ca, Src<T> src) {
  const int64_t n = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x;
  if (n >= g.N) return;
  const int j = static_cast<int>(n / g.nx), i = static_cast<int>(n - static_cast<int64_t>(j) * g.nx);
  T o[4], s[4];
  pml_point(g, y, i, j, o, s);
  o[1] += src_value(src, n);
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const int64_t e = f * g.N + n;
    const T ue = u ? u[e] : T(0);
    if (ynext) ynext[e] = ue + cy * o[f];
    const T base = acc_in ? acc_in[e] : ue;
    acc_out[e] = base + ca * o[f];
  }
}

// Arnoldi on the PML operator (Sec. 3.2, Krylov listing), launch per step:
// w = s_j H~ q for the augmented vector q = [state; tail] (the source tail
// enters the v equation: W tail, and J shifts the tail), with the first dot
// w . q_0 into per-block partials, as k_kry_matvec for the p/v operator.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pml_kry_matvec(PmlGeo<T> g, const T* __restrict__ q,
                                                           T* __restrict__ w, const T* __restrict__ q0,
                                                           KrySrc src, const T* __restrict__ amp,
                                                           const double* pin, int nin, double tol,
                                                           const double* beta, double* h_store,
                                                           double* sc_store, double* __restrict__ pout) {
  const int64_t ns = 4 * g.N;
  const int64_t items = g.N + src.p;
  const double sj = pin ? column_scale(pin, nin, tol, beta, h_store, sc_store) : 1.0;
  const T st = static_cast<T>(sj);
  double acc = 0.0;
  for (int64_t it = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; it < items;
       it += static_cast<int64_t>(gridDim.x) * kBlock) {
    if (it < g.N) {
      const int64_t n = it;
      const int j = static_cast<int>(n / g.nx), i = static_cast<int>(n - static_cast<int64_t>(j) * g.nx);
      T o[4], s[4];
      pml_point(g, q, i, j, o, s);
      if (src.n > 0 && n >= src.lo && n <= src.hi) {
        for (int k = 0; k < src.n; ++k)
          if (src.idx[k] == n) {
            double gt = 0.0;
            for (int c = 0; c < src.p; ++c) gt += src.G[c] * static_cast<double>(q[ns + c]);
            o[1] += static_cast<T>(gt * static_cast<double>(amp[k]));
          }
      }
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        const int64_t e = f * g.N + n;
        const T v = o[f] * st;
        w[e] = v;
        acc += static_cast<double>(v) * static_cast<double>(q0[e]);
      }
    } else {
      const int c = static_cast<int>(it - g.N);
      const T val = (c + 1 < src.p) ? q[ns + c + 1] * st : T(0);  // J q_tail
      w[ns + c] = val;
      acc += static_cast<double>(val) * static_cast<double>(q0[ns + c]);
    }
  }
  store_partial<false>(acc, pout);
}

}  // namespace expw
