// Bandwidth ceiling kernels: plain HBM streams (read, copy, triad) of 16-byte
// vectors, used to measure what a kernel that does nothing but stream can
// reach on the device, as the practical ceiling beside the datasheet peak.
//
// Each workgroup of 256 threads handles 4 consecutive 4 KiB blocks of every
// array (thread t touches vectors t, t + 256, t + 512, t + 768 of the chunk), so
// every wave's access is one contiguous 1 KiB run; the loads of a thread are
// issued together before any use. Non-temporal variants mark the streams as
// used once (no reuse in L2 / MALL).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace expw {

constexpr int kStreamNT = 256;
constexpr int kStreamU = 4;  // 16-byte vectors per thread

template <bool NT>
__device__ __forceinline__ float4 sload(const float4* p) {
  if constexpr (NT) {
    float4 v;
    v.x = __builtin_nontemporal_load(&p->x);
    v.y = __builtin_nontemporal_load(&p->y);
    v.z = __builtin_nontemporal_load(&p->z);
    v.w = __builtin_nontemporal_load(&p->w);
    return v;
  } else {
    return *p;
  }
}

template <bool NT>
__device__ __forceinline__ void sstore(float4* p, float4 v) {
  if constexpr (NT) {
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
    __builtin_nontemporal_store(v.z, &p->z);
    __builtin_nontemporal_store(v.w, &p->w);
  } else {
    *p = v;
  }
}

// kind 0: read a (one partial sum per workgroup into c), 1: c = a,
// 2: c = a + s b. n4 = number of 16-byte vectors per array.
template <int KIND, bool NT>
__global__ __launch_bounds__(kStreamNT) void k_stream(const float4* __restrict__ a,
                                                      const float4* __restrict__ b,
                                                      float4* __restrict__ c, int64_t n4, float s) {
  const int64_t base = static_cast<int64_t>(blockIdx.x) * (kStreamNT * kStreamU) + threadIdx.x;
  float4 va[kStreamU], vb[kStreamU];
#pragma unroll
  for (int u = 0; u < kStreamU; ++u) {
    const int64_t i = base + u * kStreamNT;
    va[u] = i < n4 ? sload<NT>(a + i) : make_float4(0.f, 0.f, 0.f, 0.f);
    if constexpr (KIND == 2) vb[u] = i < n4 ? sload<NT>(b + i) : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  if constexpr (KIND == 0) {
    float acc = 0.f;
#pragma unroll
    for (int u = 0; u < kStreamU; ++u) acc += (va[u].x + va[u].y) + (va[u].z + va[u].w);
    // one value per workgroup; the sum only keeps the loads alive
    __shared__ float red[kStreamNT];
    red[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      float t = 0.f;
      for (int k = 0; k < kStreamNT; ++k) t += red[k];
      reinterpret_cast<float*>(c)[blockIdx.x] = t;
    }
  } else {
#pragma unroll
    for (int u = 0; u < kStreamU; ++u) {
      const int64_t i = base + u * kStreamNT;
      if (i < n4) {
        float4 v = va[u];
        if constexpr (KIND == 2) {
          v.x += s * vb[u].x;
          v.y += s * vb[u].y;
          v.z += s * vb[u].z;
          v.w += s * vb[u].w;
        }
        sstore<NT>(c + i, v);
      }
    }
  }
}

inline unsigned stream_blocks(int64_t n4) {
  return static_cast<unsigned>((n4 + kStreamNT * kStreamU - 1) / (kStreamNT * kStreamU));
}

}  // namespace expw
