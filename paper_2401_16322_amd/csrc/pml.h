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

template <typename T>
struct PmlGeo {
  int32_t nx, ny;
  int64_t N;
  T ih, ih2;        // 1/h, 1/h^2
  T a[4];           // staggered first derivative
  T d2c, d2[4];     // centred second derivative: d2c u_i + sum d2_l (u_{i+l} + u_{i-l})
  T s2[4][9];       // d_yy u at rows 0..3 from u_0..u_8
  T s1[3][8];       // d_y u at half rows 0..2 from u_0..u_7
  T sw[4][8];       // d_y w_y at rows 0..3 from w_0..w_7
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

// The four components of H x at node (i, j), and x itself there.
template <typename T>
__device__ __forceinline__ void pml_point(const PmlGeo<T>& g, const T* x, int i, int j, T o[4],
                                          T s[4]) {
  const int64_t n = static_cast<int64_t>(j) * g.nx + i;
  const T* u = x;
  const T* v = x + g.N;
  const T* wx = x + 2 * g.N;
  const T* wy = x + 3 * g.N;
  s[0] = u[n];
  s[1] = v[n];
  s[2] = wx[n];
  s[3] = wy[n];
  T dxx = g.d2c * s[0], dwx = T(0), dxu = T(0);
#pragma unroll
  for (int l = 1; l <= 4; ++l) {
    dxx += g.d2[l - 1] * (pml_at(g, u, i + l, j) + pml_at(g, u, i - l, j));
    dwx += g.a[l - 1] * (pml_at(g, wx, i + l - 1, j) - pml_at(g, wx, i - l, j));
    dxu += g.a[l - 1] * (pml_at(g, u, i + l, j) - pml_at(g, u, i + 1 - l, j));
  }
  T dyy = T(0), dwy = T(0), dyu = T(0);
  if (j < 4) {
#pragma unroll
    for (int k = 0; k < 9; ++k) dyy += g.s2[j][k] * u[static_cast<int64_t>(k) * g.nx + i];
#pragma unroll
    for (int k = 0; k < 8; ++k) dwy += g.sw[j][k] * wy[static_cast<int64_t>(k) * g.nx + i];
  } else {
    dyy = g.d2c * s[0];
#pragma unroll
    for (int l = 1; l <= 4; ++l) {
      dyy += g.d2[l - 1] * (pml_at(g, u, i, j + l) + u[n - static_cast<int64_t>(l) * g.nx]);
      dwy += g.a[l - 1] * (wy[n - static_cast<int64_t>(l) * g.nx] - pml_at(g, wy, i, j + l - 1));
    }
  }
  if (j < 3) {
#pragma unroll
    for (int k = 0; k < 8; ++k) dyu += g.s1[j][k] * u[static_cast<int64_t>(k) * g.nx + i];
  } else {
#pragma unroll
    for (int l = 1; l <= 4; ++l)
      dyu += g.a[l - 1] * (u[n + static_cast<int64_t>(1 - l) * g.nx] - pml_at(g, u, i, j + l));
  }
  const T bx = g.bx[i], bxh = g.bxh[i], by = g.by[j], byh = g.byh[j];
  const T c2 = g.c2[n];
  o[0] = s[1];
  o[1] = -bx * by * s[0] + c2 * ((dxx + dyy) * g.ih2) - (bx + by) * s[1] + c2 * ((dwx + dwy) * g.ih);
  o[2] = (by - bxh) * (dxu * g.ih) - bxh * s[2];
  o[3] = (bx - byh) * (dyu * g.ih) - byh * s[3];
}

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

// One Faber term (Sec. 3.2) on the PML operator, as k_faber_term: the source
// enters the v equation. vout may alias vpp and acc_out may alias acc_in or
// vpp; vp is read with a halo and must not alias an output; vout == nullptr
// skips storing v_j.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pml_faber_term(PmlGeo<T> g, const T* vp, const T* vpp,
                                                           T* vout, const T* acc_in, T* acc_out,
                                                           FaberTerm<T> c, Src<T> src) {
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
    T acc = c.first ? add_weighted(T(0), c.a_first, c.a_first_lo, s[f]) : acc_in[e];
    acc_out[e] = add_weighted(acc, c.a_j, c.a_j_lo, v);
  }
}

}  // namespace expw
