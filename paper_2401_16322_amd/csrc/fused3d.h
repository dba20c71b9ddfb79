// Two Faber terms per HBM sweep for 3D grids (order 4, zero ghosts): a
// workgroup owns a 56 x 8 column tile and a chunk of 32 z-planes, and streams
// upwards in z. One thread per (x, y) column of the tile grown by 4 cells
// (64 x 16 threads). At iteration k the plane k of v_{j-1} (u) is loaded;
// the first term computes v_j (a) at plane k - 2 on the tile grown by 2 (the
// ring the second term's stencil needs), and the second term computes
// v_{j+1} at plane k - 4 on the tile and writes it with v_j and the partial
// sum. The x-y neighbours come from LDS rings of three planes (p, v_x, v_y of
// u and of a); the z-neighbours and the values at the point stay in
// per-thread queues of the last planes (p and v_z: five, v_x and v_y of u:
// five, of a: three). Each plane ring slot is written two iterations before
// it is read and read one iteration before it is overwritten, so one barrier
// per iteration separates all of them. Every global load of an iteration is
// issued two iterations ahead. Per point and pass: reads u and v_{j-2} (4
// words each), the FP64 sum (8 words) and c^2, writes v_{j+1}, v_j and the
// sum: 33 words for two terms against 58 for two one-term sweeps. The terms
// are computed entirely in T with the integer weights and kappa = wscale /
// gamma on an ellipse where kappa, c0 and c1 are exact in T (as in the
// streamed 2D passes, stream2d.h); the partial sum is FP64.
#pragma once

#include "device_common.h"
#include "internal.h"
#include "kernels.h"
#include "profiler.h"

namespace expw {

constexpr int k3X = 64, k3Y = 16, k3NT = k3X * k3Y;  // threads: columns of the loaded region
constexpr int k3TX = k3X - 8, k3TY = k3Y - 8;        // output tile
constexpr int k3ZC = 32;                             // output planes per workgroup
constexpr int kXcds = 8;                             // accelerator complex dies, each with its own L2

// The dispatcher deals the workgroups of a launch to the XCDs round-robin
// (workgroup i runs on XCD i mod 8). This renumbering hands each XCD a
// contiguous range of logical workgroups (a bijection on [0, nb)), so that
// tiles which share halo data run on the same XCD and meet in its L2.
__device__ __forceinline__ int xcd_contiguous(int i, int nb) {
  const int q = nb / kXcds, r = nb % kXcds;
  const int x = i % kXcds, l = i / kXcds;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + l;
}

struct Fused3Args {
  double kappa, inv_ws, c0, a_first;
  int32_t first;  // first pass: acc = a_first u, no v_{j-2}
  int32_t tiles_x, tiles_y;
  double a[2], cpp[2], q[2];
};

template <typename T>
__device__ __forceinline__ void shift_in(T* q, int n, T v) {
#pragma unroll
  for (int i = 0; i + 1 < n; ++i) q[i] = q[i + 1];
  q[n - 1] = v;
}

template <typename T>
__device__ __forceinline__ T source_amp(const Src<T>& src, int64_t gi) {
  T am = T(0);
  if (src.n > 0 && gi >= src.lo && gi <= src.hi)
    for (int s = 0; s < src.n; ++s)
      if (src.idx[s] == gi) am += src.amp[s];
  return am;
}

template <typename T>
__global__ __launch_bounds__(k3NT) void k_faber_fused3d(
    Geo<T, 2, 3> g, const T* __restrict__ vp, const T* __restrict__ vpp,
    const double* __restrict__ acc_in, T* __restrict__ out_last, T* __restrict__ out_prev,
    double* __restrict__ acc_out, T* __restrict__ state_out, Fused3Args c, Src<T> src) {
  __shared__ T su[3][3][k3NT];  // u planes: ring slot, field (p, v_x, v_y), column
  __shared__ T sa[3][3][k3NT];  // a planes
  const int b = xcd_contiguous(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
  const int txi = b % c.tiles_x;
  const int rr = b / c.tiles_x;
  const int tyi = rr % c.tiles_y;
  const int zci = rr / c.tiles_y;
  const int nx = static_cast<int>(g.n[0]), ny = static_cast<int>(g.n[1]);
  const int nz = static_cast<int>(g.n[2]);
  const int64_t N = g.N, sxy = static_cast<int64_t>(nx) * ny;
  const int tid = threadIdx.x, lx = tid & (k3X - 1), ly = tid / k3X;
  const int x = txi * k3TX - 4 + lx, y = tyi * k3TY - 4 + ly;
  const bool inxy = x >= 0 && x < nx && y >= 0 && y < ny;
  const bool in_r0 = inxy && lx >= 2 && lx < k3X - 2 && ly >= 2 && ly < k3Y - 2;
  const bool in_tile = inxy && lx >= 4 && lx < k3X - 4 && ly >= 4 && ly < k3Y - 4;
  const int64_t col = inxy ? static_cast<int64_t>(y) * nx + x : 0;
  const T sxy_int = inxy ? g.sint[0][x] + g.sint[1][y] : T(0);
  const T sxh = inxy ? g.shalf[0][x] : T(0), syh = inxy ? g.shalf[1][y] : T(0);
  const int zc0 = zci * k3ZC;
  const int zc1 = min(zc0 + k3ZC, nz);
  // every term in T (integer weights, kappa), the sum in FP64
  const T w0 = g.wi[0], w1 = g.wi[1];
  const T kap = static_cast<T>(c.kappa), iws = static_cast<T>(c.inv_ws), cz = static_cast<T>(c.c0);
  const T sxy_s = sxy_int * iws, sxh_s = sxh * iws, syh_s = syh * iws;
  constexpr int R = k3X;  // LDS row stride

  T qp[5], qvx[5], qvy[5], qvz[5];  // u at planes k-4..k (index 0 oldest)
  T ap[5], avz[5], avx[3], avy[3];  // a at planes k-6..k-2 and k-4..k-2
#pragma unroll
  for (int i = 0; i < 5; ++i) qp[i] = qvx[i] = qvy[i] = qvz[i] = ap[i] = avz[i] = T(0);
#pragma unroll
  for (int i = 0; i < 3; ++i) avx[i] = avy[i] = T(0);

  // Everything iteration k reads from global memory is loaded during
  // iteration k - 1 (u at plane k; v_{j-2} and c^2 at plane k - 2; c^2 and
  // the sum at plane k - 4), so the loads overlap a whole iteration.
  struct Ahead {
    T u[4], w[4], c2a, c2b;
    double acc[4];
  };
  auto load_ahead = [&](int k, Ahead& o) {
    const bool in = inxy && k >= 0 && k < nz;
    const int64_t gu = col + static_cast<int64_t>(in ? k : 0) * sxy;
#pragma unroll
    for (int f = 0; f < 4; ++f) o.u[f] = in ? vp[f * N + gu] : T(0);
    const int z0 = k - 2;
    const bool t0 = in_r0 && z0 >= 0 && z0 < nz && z0 >= zc0 - 2 && z0 <= zc1 + 1;
    const int64_t g0 = col + static_cast<int64_t>(t0 ? z0 : 0) * sxy;
#pragma unroll
    for (int f = 0; f < 4; ++f) o.w[f] = (t0 && !c.first) ? __builtin_nontemporal_load(vpp + f * N + g0) : T(0);
    o.c2a = t0 ? g.c2[g0] : T(0);
    const int z1 = k - 4;
    const bool t1 = in_tile && z1 >= zc0 && z1 < zc1;
    const int64_t g1 = col + static_cast<int64_t>(t1 ? z1 : 0) * sxy;
#pragma unroll
    for (int f = 0; f < 4; ++f) o.acc[f] = (t1 && !c.first) ? __builtin_nontemporal_load(acc_in + f * N + g1) : 0.0;
    o.c2b = t1 ? g.c2[g1] : T(0);
  };
  // loads run two iterations ahead
  Ahead nxt, nx2;
  load_ahead(zc0 - 4, nxt);
  load_ahead(zc0 - 3, nx2);
  for (int k = zc0 - 4; k <= zc1 + 3; ++k) {
    const Ahead cu = nxt;
    nxt = nx2;
    const T* cur = cu.u;
    if (k + 1 < zc1 + 3) load_ahead(k + 2, nx2);
    shift_in(qp, 5, cur[0]);
    shift_in(qvx, 5, cur[1]);
    shift_in(qvy, 5, cur[2]);
    shift_in(qvz, 5, cur[3]);
    const int sk = (k + 6) % 3;
    su[sk][0][tid] = cur[0];
    su[sk][1][tid] = cur[1];
    su[sk][2][tid] = cur[2];

    // first term: a = v_j at plane z0 (its u plane was stored two iterations ago)
    const int z0 = k - 2;
    T a0[4] = {T(0), T(0), T(0), T(0)};
    if (in_r0 && z0 >= 0 && z0 < nz && z0 >= zc0 - 2 && z0 <= zc1 + 1) {
      const int s0 = (z0 + 6) % 3;
      const T* P = su[s0][0];
      const T* VX = su[s0][1];
      const T* VY = su[s0][2];
      const int l = tid;
#define D_(x) static_cast<double>(x)
      const T pc = qp[2], vxc = qvx[2], vyc = qvy[2], vzc = qvz[2];
      const T dvx = w0 * (qvx[2] - VX[l - 1]) + w1 * (VX[l + 1] - VX[l - 2]);
      const T dvy = w0 * (qvy[2] - VY[l - R]) + w1 * (VY[l + R] - VY[l - 2 * R]);
      const T dvz = w0 * (qvz[2] - qvz[1]) + w1 * (qvz[3] - qvz[0]);
      const T dpx = w0 * (P[l + 1] - qp[2]) + w1 * (P[l + 2] - P[l - 1]);
      const T dpy = w0 * (P[l + R] - qp[2]) + w1 * (P[l + 2 * R] - P[l - R]);
      const T dpz = w0 * (qp[3] - qp[2]) + w1 * (qp[4] - qp[1]);
      const int64_t gi = col + static_cast<int64_t>(z0) * sxy;
      const T hp = -cu.c2a * (dvx + dvy + dvz) - (sxy_s + g.sint[2][z0] * iws) * pc;
      const T hvx = -dpx - sxh_s * vxc;
      const T hvy = -dpy - syh_s * vyc;
      const T hvz = -dpz - g.shalf[2][z0] * iws * vzc;
      const T self[4] = {pc, vxc, vyc, vzc};
      const T h[4] = {hp, hvx, hvy, hvz};
      const T cpp0 = static_cast<T>(c.cpp[0]);
      T src0 = T(0);
      if (src.n > 0) src0 = static_cast<T>(c.q[0]) * source_amp(src, gi);
#pragma unroll
      for (int f = 0; f < 4; ++f)
        a0[f] = kap * h[f] - cz * self[f] - cpp0 * cu.w[f] + (f == 0 ? src0 : T(0));
    }
    const int sz0 = (z0 + 6) % 3;
    sa[sz0][0][tid] = a0[0];
    sa[sz0][1][tid] = a0[1];
    sa[sz0][2][tid] = a0[2];
    shift_in(ap, 5, a0[0]);
    shift_in(avz, 5, a0[3]);
    shift_in(avx, 3, a0[1]);
    shift_in(avy, 3, a0[2]);

    // second term: v_{j+1} at plane z1 (its a plane was stored two iterations ago)
    const int z1 = k - 4;
    if (in_tile && z1 >= zc0 && z1 < zc1) {
      const int s1 = (z1 + 6) % 3;
      const T* P = sa[s1][0];
      const T* VX = sa[s1][1];
      const T* VY = sa[s1][2];
      const int l = tid;
      const T pc = ap[2], vxc = avx[0], vyc = avy[0], vzc = avz[2];
      const T dvx = w0 * (avx[0] - VX[l - 1]) + w1 * (VX[l + 1] - VX[l - 2]);
      const T dvy = w0 * (avy[0] - VY[l - R]) + w1 * (VY[l + R] - VY[l - 2 * R]);
      const T dvz = w0 * (avz[2] - avz[1]) + w1 * (avz[3] - avz[0]);
      const T dpx = w0 * (P[l + 1] - ap[2]) + w1 * (P[l + 2] - P[l - 1]);
      const T dpy = w0 * (P[l + R] - ap[2]) + w1 * (P[l + 2 * R] - P[l - R]);
      const T dpz = w0 * (ap[3] - ap[2]) + w1 * (ap[4] - ap[1]);
      const int64_t gi = col + static_cast<int64_t>(z1) * sxy;
      const T hp = -cu.c2b * (dvx + dvy + dvz) - (sxy_s + g.sint[2][z1] * iws) * pc;
      const T hvx = -dpx - sxh_s * vxc;
      const T hvy = -dpy - syh_s * vyc;
      const T hvz = -dpz - g.shalf[2][z1] * iws * vzc;
      const T self[4] = {pc, vxc, vyc, vzc};
      const T h[4] = {hp, hvx, hvy, hvz};
      const T uz[4] = {qp[0], qvx[0], qvy[0], qvz[0]};
      const T am = src.n > 0 ? source_amp(src, gi) : T(0);
      const T cpp1 = static_cast<T>(c.cpp[1]);
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        T vt = kap * h[f] - cz * self[f] - cpp1 * uz[f];
        if (f == 0) vt += static_cast<T>(c.q[1]) * am;
        double acc = c.first ? c.a_first * D_(uz[f]) : cu.acc[f];
        acc = fma(c.a[0], D_(self[f]), acc);
        acc = fma(c.a[1], D_(vt), acc);
        if (out_last) {
          __builtin_nontemporal_store(vt, out_last + f * N + gi);
          __builtin_nontemporal_store(self[f], out_prev + f * N + gi);
        }
        if (state_out) __builtin_nontemporal_store(static_cast<T>(acc), state_out + f * N + gi);
        else __builtin_nontemporal_store(acc, acc_out + f * N + gi);
      }
#undef D_
    }
    __syncthreads();
  }
}

template <typename T>
int32_t launch_fused3d(hipStream_t st, Profiler* prof, const Geo<T, 2, 3>& g, Src<T> src,
                       const T* vp, const T* vpp, const double* acc_in, T* out_last, T* out_prev,
                       double* acc_out, T* state_out, int j, bool first, const double* a,
                       const double* q, double kappa, double inv_ws, double c0, double c1) {
  Fused3Args c{};
  c.kappa = kappa;
  c.inv_ws = inv_ws;
  c.c0 = c0;
  c.first = first ? 1 : 0;
  if (first) c.a_first = a[0];
  for (int r = 0; r < 2; ++r) {
    const int jj = j + r;
    c.a[r] = a[jj];
    c.cpp[r] = jj == 1 ? 0.0 : (jj == 2 ? 2.0 * c1 : c1);
    c.q[r] = q[jj - 1];
  }
  c.tiles_x = static_cast<int>((g.n[0] + k3TX - 1) / k3TX);
  c.tiles_y = static_cast<int>((g.n[1] + k3TY - 1) / k3TY);
  const int64_t chunks = (g.n[2] + k3ZC - 1) / k3ZC;
  const int64_t blocks = static_cast<int64_t>(c.tiles_x) * c.tiles_y * chunks;
  if (blocks > INT32_MAX) return fail(EXPW_EUNSUPPORTED, "3D fused pass: grid too large");
  // algorithmic bytes per point: u (4 T), c^2 (1 T), unless first v_{j-2}
  // (4 T) and the sum (4 FP64); writes the sum (4 FP64, or the step's result:
  // 4 T), unless last the pair (8 T)
  const double bytes = (4 + 1 + (first ? 0 : 4) + (out_last ? 8 : 0) + (state_out ? 4 : 0)) * sizeof(T) +
                       ((first ? 0 : 4) + (state_out ? 0 : 4)) * sizeof(double);
  launch_timed(prof, st, EXPW_KERNEL_FABER, bytes * g.N, k_faber_fused3d<T>,
               dim3(static_cast<unsigned>(blocks)), dim3(k3NT), g, vp, vpp, acc_in, out_last,
               out_prev, acc_out, state_out, c, src);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(EXPW_EDEVICE, "3D fused Faber pass: %s", hipGetErrorString(e));
  return EXPW_OK;
}

}  // namespace expw
