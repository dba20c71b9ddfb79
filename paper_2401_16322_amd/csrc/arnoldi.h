// Persistent Arnoldi for one Krylov step, for augmented vectors small
// enough to live in registers across the grid (Sec. 3.2, Krylov subspace
// projection).
//
// One cooperative launch runs the whole basis construction: each thread owns
// UN / (DIM + 1) grid points with all their fields (UN elements of the
// augmented vector, the tail elements in pressure slots of points beyond the
// grid), and keeps its slices of w, q_0 and the newest basis vector in
// registers. A thread's matvec loads all operands of a point at once.
// Columns are written unnormalized with their scale s_j = 1/h_{j,j-1}
// (s_0 = 1), as in the launch-per-step path.
//
// Gram-Schmidt with one grid-wide reduction per column. Modified
// Gram-Schmidt takes h_{i,j} = <w - sum_{l<i} h_{l,j} q_l, q_i>, which equals
// r_i - sum_{l<i} h_{l,j} <q_l, q_i> with r_i = <w, q_i>, for any basis, not
// only an exactly orthonormal one. Column j's matvec runs on the stored,
// unnormalized Q_j (H is linear, so w = s_j H Q_j is rescaled once s_j is
// known), and |Q_j|^2 rides in the same reduction as the dots <H Q_j, Q_i>
// and the new Gram row <Q_j, Q_l> (l < j), as in low-synchronization
// Gram-Schmidt (Swirydowicz et al., 2020). After that one reduction, s_j,
// a forward substitution over the Gram entries gives MGS's projections, and
// a second sweep applies them in MGS's order (w -= h_{i,j} q_i, i = 0..j,
// rounded after each), stores Q_{j+1} and takes this workgroup's part of
// |Q_{j+1}|^2 into the next column's reduction. The price is a second read of
// q_1..q_{j-1} per column; the gain is one grid-wide reduction per column
// instead of j + 2.
//
// The stencil of column j + 1 still needs Q_{j+1} from the neighbouring
// workgroups. Instead of a grid-wide barrier, each workgroup publishes a
// flag (launch epoch + column) once its slice of Q_{j+1} is stored, and
// waits only for the flags of the workgroups that own an element of a cache
// line its matvec reads: the points within the stencil's reach along the
// outermost axis plus a margin of a few cache lines, the lines that cross a
// field boundary, and, where the source tail is read, the tail's owners.
// (With periodic boundaries a workgroup waits for every other.)
//
// Reduction partials cross workgroups through device-coherent accesses
// (agent-scope relaxed atomics, i.e. sc1 loads and stores that do not stop in
// an XCD's L2). Basis vectors are written the same way, but read with plain,
// cached loads: each column Q_j is written once per launch, and no workgroup
// reads a cache line of it before every workgroup owning an element of that
// line has stored its slice (the grid-wide reductions, or the flags above,
// order the two; columns start on 256-byte boundaries), and the launch starts
// with no lines of Q in any cache, so such a read can only miss and fetch the
// written value. The stencil's neighbour reads then hit in L1 and L2 instead
// of crossing the fabric each time. A grid-wide reduction is also the
// barrier, and uses no read-modify-write:
// each block's partial is its own arrival word. Slots start out holding a
// signalling-NaN pattern that no arithmetic produces; block b stores its
// partial of value v (after waiting for its earlier stores, s_waitcnt 0) into
// slot (v, b) of the barrier's buffer; a few leader blocks wait until each
// slot no longer holds that pattern, take the values they find, and store
// the totals into their records (the same convention), which the other
// blocks poll. Three buffers rotate: when barrier s completes, the leaders
// have read every value of barrier s-1, so each block then restores the
// pattern in its slots of that buffer, which is next written at barrier s+2
// (and each leader its record of barrier s-1). Every wait is bounded: a wait
// longer than spin_limit polls sets *err and gives up, and once *err is set
// no wait lasts more than 1024 polls, so every wave always reaches the end of
// the kernel.
#pragma once

#include "device_common.h"
#include "expwave.h"
#include "kernels.h"

namespace expw {

constexpr int kArnNT = 1024;        // threads per block of the persistent kernel
constexpr int kArnMaxBlocks = 256;  // grid cap of the persistent kernel
constexpr int kArnMaxVals = 2 * EXPW_MAX_KRYLOV;  // values of one grid-wide reduction
constexpr int kArnHessLd = EXPW_MAX_KRYLOV;           // leading dimension of the Hessenberg matrix
constexpr int kArnLdsBudget = 160 * 1024 - 1024;      // LDS of one block of the persistent kernel

template <typename T>
__device__ __forceinline__ T ld_coherent(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ void st_coherent(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// base[e] for a byte offset that fits 32 bits (a uniform base plus a 32-bit
// per-lane offset, so the address needs no 64-bit vector arithmetic)
template <typename T>
__device__ __forceinline__ T ld_at(const T* base, uint32_t byte_off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}

template <typename T>
__device__ __forceinline__ void st_at(T* base, uint32_t byte_off, T v) {
  st_coherent(reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off), v);
}

// Contents of an empty slot of the grid-wide reduction (a signalling NaN;
// a NaN partial is stored as the default quiet NaN instead).
constexpr unsigned long long kSlotEmpty = 0x7FF4DEADBEEF0001ull;
constexpr int kSlotBuffers = 3;

// Sums of the slots of row0 (and of row1 when two) over the nb blocks, each
// lane adding blocks lane, lane + 64, ... in order and the lanes by a fixed
// DPP tree. All loads of the rows are issued together and the empty slots are
// polled again together, so each poll costs one round trip. Bounded: after
// spin_limit polls (1024 once *err is set) it sets *err and gives up.
template <int PER>
__device__ __forceinline__ void collect_rows(const unsigned long long* row0,
                                             const unsigned long long* row1, bool two, int nb,
                                             int lane, unsigned spin_limit, int* err, double& s0,
                                             double& s1) {
  unsigned long long x0[PER], x1[PER];
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int b = lane + 64 * r;
    x0[r] = b < nb ? ld_coherent(row0 + b) : 0ull;
    x1[r] = (two && b < nb) ? ld_coherent(row1 + b) : 0ull;
  }
  unsigned polls = 0;
  for (;;) {
    bool empty = false;
#pragma unroll
    for (int r = 0; r < PER; ++r) empty = empty || x0[r] == kSlotEmpty || x1[r] == kSlotEmpty;
    if (!empty) break;
    __builtin_amdgcn_s_sleep(1);
    if (++polls > spin_limit ||
        ((polls & 1023u) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
      __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int b = lane + 64 * r;
      if (x0[r] == kSlotEmpty) x0[r] = ld_coherent(row0 + b);
      if (x1[r] == kSlotEmpty) x1[r] = ld_coherent(row1 + b);
    }
  }
  s0 = 0.0;
  s1 = 0.0;
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    if (lane + 64 * r < nb) {
      s0 += __longlong_as_double(x0[r]);
      s1 += __longlong_as_double(x1[r]);
    }
  }
  s0 = wave_sum_fixed(s0);
  s1 = wave_sum_fixed(s1);
}

// Leader blocks of the grid-wide sums and the length of a leader's record.
constexpr int kArnLeaders = 4;  // per launch at 1001x501, k = 16, FP32: 4 leaders 326-330 us, 2: 333-335, 8: 336, 16: 336-340
constexpr int kArnRecLen = 128;
// words of the reduction area: kSlotBuffers records per leader, then
// kSlotBuffers slot buffers of up to kArnMaxVals x kArnMaxBlocks words
constexpr size_t kArnRecWords = static_cast<size_t>(kSlotBuffers) * kArnLeaders * kArnRecLen;
static_assert(kArnMaxVals <= kArnRecLen, "a record holds every value of a reduction");
// after the slot buffers: one column flag per workgroup, then the launch
// epoch (all zero when the area is set up)
constexpr size_t kArnFlagWord = kArnRecWords + static_cast<size_t>(kSlotBuffers) * kArnMaxVals * kArnMaxBlocks;
constexpr size_t kArnAreaWords = kArnFlagWord + kArnMaxBlocks + 8;
// elements on either side of a read that may share a cache line with it
// (four 128-byte lines of FP32 values)
constexpr int64_t kArnLineMargin = 128;

// The workgroups owning a point of [A, B] (points below N + tail; point P
// belongs to workgroup (P mod nt) / kArnNT, nt the grid's threads), as bits r
// of this lane for workgroup lane + 64 r.
__device__ __forceinline__ uint32_t arn_owners(int64_t A, int64_t B, int64_t nt, int nb, int lane) {
  if (A > B) return 0u;
  const bool all = B - A + 1 >= nt;
  const int64_t a = A % nt, b = B % nt;
  uint32_t m = 0;
#pragma unroll
  for (int r = 0; r < kArnMaxBlocks / 64; ++r) {
    const int c = lane + 64 * r;
    const int64_t lo = static_cast<int64_t>(c) * kArnNT, hi = lo + kArnNT - 1;
    const bool hit = all || (a <= b ? (lo <= b && hi >= a) : (hi >= a || lo <= b));
    if (c < nb && hit) m |= 1u << r;
  }
  return m;
}

// The workgroups whose stored slices of a column workgroup blk's matvec
// reads, with every element that shares a cache line with such a read
// (wave 0; bits as in arn_owners). Points P_v = blk kArnNT + v nt + t
// (t < kArnNT, v < up); reach = K times the outermost stride plus the line
// margin. Grid points read their neighbours within reach, which near the
// first or last point share lines with the neighbouring field (the last
// field's with the tail); source points and tail slots read the tail.
template <int BC>
__device__ uint32_t arn_need_mask(int lane, int blk, int nb, int up, int64_t N, int64_t ntail, int64_t reach,
                                  const KrySrc& src) {
  const int64_t nt = static_cast<int64_t>(nb) * kArnNT;
  if (BC != 0) return arn_owners(0, nt - 1, nt, nb, lane);
  const int64_t tl = N > kArnLineMargin ? N - kArnLineMargin : 0, th = N + ntail - 1;
  uint32_t m = 0;
  for (int v = 0; v < up; ++v) {
    const int64_t lo = static_cast<int64_t>(blk) * kArnNT + v * nt, hi = lo + kArnNT - 1;
    if (lo < N) {
      const int64_t gl = lo, gh = hi < N ? hi : N - 1;
      const int64_t rl = gl - reach, rh = gh + reach;
      m |= arn_owners(rl > 0 ? rl : 0, rh < N ? rh : N - 1, nt, nb, lane);
      if (rl < 0) m |= arn_owners(N + rl > 0 ? N + rl : 0, N - 1, nt, nb, lane);
      if (rh >= N) {
        m |= arn_owners(0, rh - N < N ? rh - N : N - 1, nt, nb, lane);
        if (ntail > 0) m |= arn_owners(tl, th, nt, nb, lane);
      }
      bool has_src = false;
      for (int s = lane; s < src.n; s += 64) has_src = has_src || (src.idx[s] >= gl && src.idx[s] <= gh);
      if (ntail > 0 && __any(has_src)) m |= arn_owners(tl, th, nt, nb, lane);
    }
    if (ntail > 0 && hi >= N && lo < N + ntail) m |= arn_owners(tl, th, nt, nb, lane);
  }
  return m;
}

// Wave 0: waits until every workgroup of need has stored a column flag of at
// least target. Bounded like the reductions' waits.
__device__ __forceinline__ void arn_wait_flags(const unsigned long long* flags, uint32_t need,
                                               unsigned long long target, int lane, unsigned spin_limit,
                                               int* err) {
  constexpr int R = kArnMaxBlocks / 64;
  uint32_t pend = need;
  unsigned polls = 0;
  for (;;) {
    unsigned long long x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = (pend >> r & 1u) ? ld_coherent(flags + lane + 64 * r) : target;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (x[r] >= target) pend &= ~(1u << r);
    if (!__any(pend != 0u)) break;
    __builtin_amdgcn_s_sleep(1);
    if (++polls > spin_limit ||
        ((polls & 1023u) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
      __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
  }
}

// Grid-wide sums of nv values (1 <= nv <= nvmax, at most kArnMaxBlocks
// blocks of NT threads), in two levels. Before the call, lane 0 of wave w has
// put its wave's partial of value v in wpart[v][w]. Every block stores its
// partials into its slots; leader blocks 0..kArnLeaders-1 collect every
// block's partials and store the totals into their record; every other block
// b waits for the record of leader b % kArnLeaders. So only the leaders poll
// the slots (fewer polls of the same lines than when every block collects
// everything) and the others poll one short record. On return every thread
// sees the totals in tot[0..nv). Each total is added in a fixed order: a
// block's partial is the sum of its waves in order; block b's partial goes to
// lane b % 64 of the wave that collects the value, each lane adds its blocks
// in increasing order, and the lanes are added by a fixed DPP tree; the
// followers take the leaders' bits.
// area holds the kSlotBuffers x kArnLeaders records of kArnRecLen words, then
// kSlotBuffers buffers of nvmax x gridDim.x words (row v = value v), all
// kSlotEmpty at launch; seq numbers the barriers of the launch (1, 2, ...).
// after() runs in every thread once this block has arrived: loads it issues
// overlap the wait (the s_waitcnt before the arrival waits for every
// outstanding memory operation, so loads issued earlier would be waited for
// there).
template <int NT, typename F>
__device__ __forceinline__ void grid_sum_vec(int nv, int nvmax, const double (*wpart)[NT / 64],
                                             double* tot, unsigned long long* area, unsigned seq,
                                             unsigned spin_limit, int* err, F&& after) {
  static_assert(NT % 64 == 0 && NT <= 1024, "block of whole waves");
  constexpr int NW = NT / 64;
  constexpr int PER = kArnMaxBlocks / 64;
  const int nb = static_cast<int>(gridDim.x);
  const size_t buf = static_cast<size_t>(nvmax) * nb;
  unsigned long long* slots = area + kArnRecWords;
  unsigned long long* cur = slots + (seq % kSlotBuffers) * buf;
  unsigned long long* prev = slots + ((seq + kSlotBuffers - 1) % kSlotBuffers) * buf;
  const int leader = static_cast<int>(blockIdx.x) % kArnLeaders;
  const bool is_leader = static_cast<int>(blockIdx.x) < kArnLeaders;
  unsigned long long* rcur = area + ((seq % kSlotBuffers) * kArnLeaders + leader) * kArnRecLen;
  unsigned long long* rprev =
      area + (((seq + kSlotBuffers - 1) % kSlotBuffers) * kArnLeaders + leader) * kArnRecLen;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __builtin_amdgcn_s_waitcnt(0);  // this thread's coherent stores have completed
  __syncthreads();                // ... and so have the block's; wave partials are in LDS
  if (static_cast<int>(threadIdx.x) < nv) {
    double b = 0.0;
    for (int w = 0; w < NW; ++w) b += wpart[threadIdx.x][w];
    const unsigned long long bits = (b != b) ? 0x7FF8000000000000ull : __double_as_longlong(b);
    st_coherent(cur + static_cast<size_t>(threadIdx.x) * nb + blockIdx.x, bits);
  }
  after();
  if (is_leader) {
    // every wave polls its rows at once (only the few leaders poll the
    // slots): wave w takes values w and w + NW, then the next 2 NW
    {
      for (int v0 = wid; v0 < nv; v0 += 2 * NW) {
        const int v1 = v0 + NW;
        const bool two = v1 < nv;
        double s0, s1;
        collect_rows<PER>(cur + static_cast<size_t>(v0) * nb, cur + static_cast<size_t>(two ? v1 : v0) * nb,
                          two, nb, lane, spin_limit, err, s0, s1);
        if (lane == 0) {
          tot[v0] = s0;
          if (two) tot[v1] = s1;
        }
      }
    }
    __syncthreads();
    if (static_cast<int>(threadIdx.x) < nv) {
      const double t = tot[threadIdx.x];
      st_coherent(rcur + threadIdx.x, (t != t) ? 0x7FF8000000000000ull : __double_as_longlong(t));
    }
    // every follower has stored its slot of this barrier, so it has read this
    // leader's record of the previous one
    if (static_cast<int>(threadIdx.x) < nvmax) st_coherent(rprev + threadIdx.x, kSlotEmpty);
  } else if (wid == 0) {
    // the leader's record: lane v polls values v and v + 64 (nv <= kArnMaxVals <= 2 * 64)
    unsigned long long x0 = lane < nv ? ld_coherent(rcur + lane) : 0ull;
    unsigned long long x1 = lane + 64 < nv ? ld_coherent(rcur + lane + 64) : 0ull;
    unsigned polls = 0;
    for (;;) {
      if (!__any((lane < nv && x0 == kSlotEmpty) || (lane + 64 < nv && x1 == kSlotEmpty))) break;
      __builtin_amdgcn_s_sleep(1);
      if (++polls > spin_limit ||
          ((polls & 1023u) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      if (lane < nv && x0 == kSlotEmpty) x0 = ld_coherent(rcur + lane);
      if (lane + 64 < nv && x1 == kSlotEmpty) x1 = ld_coherent(rcur + lane + 64);
    }
    if (lane < nv) tot[lane] = __longlong_as_double(x0);
    if (lane + 64 < nv) tot[lane + 64] = __longlong_as_double(x1);
  }
  __syncthreads();
  // all blocks arrived at this barrier, so the leaders have read every
  // block's values of barrier seq-1; the stores complete before this block's
  // next arrival (s_waitcnt)
  if (static_cast<int>(threadIdx.x) < nvmax)
    st_coherent(prev + static_cast<size_t>(threadIdx.x) * nb + blockIdx.x, kSlotEmpty);
}

// Extents and strides of the grid in 32 bits: the persistent kernel's
// vectors have fewer than 2^31 elements, so point indices, coordinates and
// byte offsets fit, and the stencil needs no 64-bit index arithmetic.
struct Geo32 {
  uint32_t n[3], st[3], N;
};

// x at the point shifted by s along one axis (zero outside or wrapped); x is
// a uniform field base, idx the point, i its coordinate on the axis.
template <typename T, int BC>
__device__ __forceinline__ T ldn32(const T* x, uint32_t idx, uint32_t i, uint32_t n, uint32_t st,
                                   int s) {
  const int j = static_cast<int>(i) + s;
  if (BC == 0)
    return (j >= 0 && j < static_cast<int>(n))
               ? ld_at(x, (idx + static_cast<uint32_t>(s) * st) * static_cast<uint32_t>(sizeof(T)))
               : T(0);
  int jj = j % static_cast<int>(n);
  if (jj < 0) jj += static_cast<int>(n);
  return ld_at(x, (idx + static_cast<uint32_t>(jj - static_cast<int>(i)) * st) *
                      static_cast<uint32_t>(sizeof(T)));
}

// (H x) at one grid point for every field: out[0] the pressure, out[1 + a]
// the velocity along a. No load depends on another or on a branch, so all of
// the point's operands are in flight at once.
template <typename T, int K, int BC, int DIM>
__device__ __forceinline__ void apply_point_all(const Geo<T, K, DIM>& g, const Geo32& g32, const T* x,
                                                uint32_t idx, const uint32_t* ic, T* out) {
  constexpr uint32_t es = sizeof(T);
  T div = T(0), sp = T(0);
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const T* v = x + (1 + a) * g.N;
#pragma unroll
    for (int l = 1; l <= K; ++l)
      div += g.w[l - 1] * (ldn32<T, BC>(v, idx, ic[a], g32.n[a], g32.st[a], l - 1) -
                           ldn32<T, BC>(v, idx, ic[a], g32.n[a], g32.st[a], -l));
    sp += ld_at(g.sint[a], ic[a] * es);
  }
  out[0] = -ld_at(g.c2, idx * es) * div - sp * ld_at(x, idx * es);
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    T dp = T(0);
#pragma unroll
    for (int l = 1; l <= K; ++l)
      dp += g.w[l - 1] * (ldn32<T, BC>(x, idx, ic[a], g32.n[a], g32.st[a], l) -
                          ldn32<T, BC>(x, idx, ic[a], g32.n[a], g32.st[a], 1 - l));
    out[1 + a] = -dp - ld_at(g.shalf[a], ic[a] * es) * ld_at(x + (1 + a) * g.N, idx * es);
  }
}

struct ArnArgs {
  int64_t ns, naug, ld;
  int k;
  int nvmax;     // values of the largest grid-wide reduction: 2k
  double tail2;  // |e_p|^2: 1 with a source, else 0
  double tol;
  unsigned spin_limit;
  int32_t full_last;  // 1: orthogonalize and normalize the last column too (h_{k,k-1} for an estimate)
};

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), l);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

// Sums of two values over the 64 lanes of a wave (all lanes active), a into
// sa and b into sb. One exchange of 32-lane halves (v_permlane32_swap, which
// trades lanes 32-63 of its first operand for lanes 0-31 of its second)
// leaves a_l + a_{l+32} in lanes l < 32 and b_{l-32} + b_l in lanes l >= 32;
// then every 16-lane row is summed by DPP (quad permutations, row rotations
// by 4 and 8) and rows 0+1 and 2+3 are added (row broadcast of lane 15), so
// that lane 31 holds the sum of a and lane 63 that of b. Half the DPP
// additions of two separate wave sums; the order of the additions is fixed.
__device__ __forceinline__ void wave_sum_pair(double a, double b, double& sa, double& sb) {
  const auto lo = __builtin_amdgcn_permlane32_swap(static_cast<unsigned>(__double2loint(a)),
                                                   static_cast<unsigned>(__double2loint(b)), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(static_cast<unsigned>(__double2hiint(a)),
                                                   static_cast<unsigned>(__double2hiint(b)), false, false);
  double v = __hiloint2double(static_cast<int>(hi[0]), static_cast<int>(lo[0])) +
             __hiloint2double(static_cast<int>(hi[1]), static_cast<int>(lo[1]));
  v += dpp_move<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x124, 0xF>(v);  // row_ror:4
  v += dpp_move<0x128, 0xF>(v);  // row_ror:8
  v += dpp_move<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  sa = readlane_f64(v, 31);
  sb = readlane_f64(v, 63);
}

template <typename T, int K, int BC, int DIM, int UN>
__global__ __launch_bounds__(kArnNT) void k_arnoldi_persistent(
    Geo<T, K, DIM> g, const T* __restrict__ S, T* Q, KrySrc src, const T* __restrict__ amp,
    ArnArgs a, unsigned long long* slots, int* err, unsigned* seq_io, double* hess, double* sc,
    double* beta_out) {
  constexpr int NW = kArnNT / 64;
  static_assert(UN % (DIM + 1) == 0, "whole grid points per thread");
  constexpr int UP = UN / (DIM + 1);  // grid points per thread
  __shared__ double s_scale[EXPW_MAX_KRYLOV + 1];
  // <q_i, q_l> for l < i < EXPW_MAX_KRYLOV, packed: entry i (i - 1) / 2 + l
  __shared__ double s_gt[EXPW_MAX_KRYLOV * (EXPW_MAX_KRYLOV - 1) / 2];
  __shared__ double s_wpart[kArnMaxVals][NW];
  __shared__ double s_tot[kArnMaxVals];
  __shared__ double s_h[EXPW_MAX_KRYLOV];
  __shared__ T s_qj[UN][kArnNT];  // this block's slice of Q_j, the newest stored column
  // the first NC stored columns Q_1..Q_NC also stay in LDS, as far as the
  // block's LDS allows: every later column reads them in both sweeps
  constexpr int kColLds = UN * kArnNT * static_cast<int>(sizeof(T));
  constexpr int kFixedLds =
      (3 * EXPW_MAX_KRYLOV + 1 + EXPW_MAX_KRYLOV * (EXPW_MAX_KRYLOV - 1) / 2 + kArnMaxVals * (NW + 1)) * 8;
  constexpr int kFree = kArnLdsBudget - kFixedLds - kColLds;
  constexpr int NC = kFree / kColLds < 4 ? kFree / kColLds : 4;
  __shared__ T s_cache[NC > 0 ? NC : 1][NC > 0 ? UN : 1][NC > 0 ? kArnNT : 1];
  const unsigned nb = gridDim.x;
  const int64_t nthreads = static_cast<int64_t>(nb) * kArnNT;
  const int64_t gtid = static_cast<int64_t>(blockIdx.x) * kArnNT + threadIdx.x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  // barriers continue the numbering of the previous launch (mod 3): its last
  // slot buffer and records are restored by this launch's first barrier, so
  // the area needs no fill between launches
  unsigned seq = __hip_atomic_load(seq_io, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // column flags: workgroup b stores ep + j into flags[b] once its slice of
  // Q_j is stored; the epoch grows by k + 1 per launch, so no flag of an
  // earlier launch reaches a target of this one
  unsigned long long* flags = slots + kArnFlagWord;
  unsigned long long ep = 0;
  uint32_t need = 0;
  if (wid == 0) {
    ep = ld_coherent(flags + kArnMaxBlocks);
    need = arn_need_mask<BC>(lane, static_cast<int>(blockIdx.x), static_cast<int>(nb), UP, g.N,
                             a.naug - a.ns, static_cast<int64_t>(K) * g.st[DIM - 1] + kArnLineMargin, src);
  }
  // Thread gtid owns the grid points P_v = gtid + v * nthreads (v < UP) with
  // all their fields: slot u = f * UP + v holds element f * N + P_v. The
  // pressure slot of a point beyond the grid, P_v = N + t, holds tail element
  // ns + t of the augmented vector (t < p). Every element has one slot
  // (N + p <= UP * nthreads, host check), and naug < 2^31, so element indices
  // and byte offsets are 32-bit.
  const uint32_t e0 = static_cast<uint32_t>(gtid), estep = static_cast<uint32_t>(nthreads);
  const uint32_t naug32 = static_cast<uint32_t>(a.naug), ns32 = static_cast<uint32_t>(a.ns);
  const uint32_t npts32 = static_cast<uint32_t>(g.N);
  const uint32_t ntail32 = naug32 - ns32;
  // element of slot u for the thread's first point p0, or ok = false
  auto elem = [&](int u, uint32_t p0, bool& ok) -> uint32_t {
    const uint32_t f = static_cast<uint32_t>(u / UP);
    const uint32_t P = p0 + static_cast<uint32_t>(u % UP) * estep;
    ok = P < npts32 || (f == 0 && P - npts32 < ntail32);
    return P < npts32 ? f * npts32 + P : ns32 + (P - npts32);
  };
  constexpr uint32_t kEs = sizeof(T);
  Geo32 g32;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    g32.n[d] = static_cast<uint32_t>(g.n[d]);
    g32.st[d] = static_cast<uint32_t>(g.st[d]);
  }
  g32.N = npts32;
  // per-thread partial sums and the update w -= h q run in T (FP32 partials
  // cover UN <= 9 products); every sum across threads is in FP64

  auto put = [&](int v, double x) {
    x = wave_sum_fixed(x);
    if (lane == 0) s_wpart[v][wid] = x;
  };
  auto put2 = [&](int va, double xa, int vb, double xb) {
    double sa, sb;
    wave_sum_pair(xa, xb, sa, sb);
    if (lane == 0) {
      s_wpart[va][wid] = sa;
      s_wpart[vb][wid] = sb;
    }
  };
  auto reduce = [&](int nv, auto&& after) {
    grid_sum_vec<kArnNT>(nv, a.nvmax, s_wpart, s_tot, slots, ++seq, a.spin_limit, err, after);
  };

  // x = [S; e_p]. q0 holds x until its norm beta is known: the first
  // grid-wide reduction of column 0 brings |x|^2 together with <H~ x, x>.
  // Column 0's matvec reads S, an input complete before the launch, so no
  // barrier precedes it; Q_0 is stored after that reduction (the kernel never
  // reads it back).
  if (threadIdx.x == 0) s_scale[0] = 1.0;
  // q0: q_0; w: the vector being orthogonalized; qa, qb: streamed columns
  // Q_1..Q_{j-1}
  T q0[UN], w[UN], qa[UN], qb[UN];
  double xx = 0.0;
#pragma unroll
  for (int u = 0; u < UN; ++u) {
    bool ok;
    const uint32_t e = elem(u, e0, ok);
    T v = T(0);
    if (ok && e < ns32)
      v = S[e];
    else if (ok && e + 1 == naug32 && a.tail2 > 0.0)
      v = T(1);
    q0[u] = v;
    xx += static_cast<double>(v) * static_cast<double>(v);
  }
  double beta = 0.0, inv = 0.0;

  // the thread's first point, made opaque once per column (an empty asm):
  // otherwise the per-element index math of all UN elements is hoisted out
  // of the column loop and held in registers for the whole kernel
  uint32_t ecur = e0;
  auto load_col = [&](T* dst, int col) {
    const T* qc = Q + col * a.ld;
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      bool ok;
      const uint32_t e = elem(u, ecur, ok);
      dst[u] = ok ? ld_at(qc, e * kEs) : T(0);
    }
  };
  // fn(i, column) for the n stored columns first, first + step, ..., two
  // buffers in turn; qa already holds (or is loading) Q_first
  // fn(i, column) for the cached column Q_i (1 <= i <= NC)
  auto from_lds = [&](int i, auto&& fn) {
    T qt[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) qt[u] = s_cache[i - 1][u][threadIdx.x];
    fn(i, qt);
  };
  auto stream = [&](int first, int n, int step, auto&& fn) {
    for (int t = 0; t < n; t += 2) {
      const int i = first + t * step;
      if (t + 1 < n) load_col(qb, i + step);
      fn(i, qa);
      if (t + 1 < n) {
        if (t + 2 < n) load_col(qa, i + 2 * step);
        fn(i + step, qb);
      }
    }
  };

  for (int j = 0; j < a.k; ++j) {
    const T* qcol = Q + j * a.ld;
    T* wout = Q + (j + 1) * a.ld;
    if (j >= 1) {
      // the workgroups whose slices of Q_j this matvec reads have stored them
      if (wid == 0) arn_wait_flags(flags, need, ep + static_cast<unsigned long long>(j), lane, a.spin_limit, err);
      __syncthreads();
    }
    ecur = e0;
    asm volatile("" : "+v"(ecur));
    // w = H~ Q_j, unscaled (column 0: H~ x); rescaled by s_j (1 / beta) once
    // the column's reduction has brought |Q_j|^2 (|x|^2)
    const T* xcol = j == 0 ? S : qcol;
    auto tailv = [&](int cc) -> T {
      return j == 0 ? (cc == src.p - 1 ? T(1) : T(0)) : qcol[a.ns + cc];
    };
#pragma unroll
    for (int v = 0; v < UP; ++v) {
      const uint32_t P = ecur + static_cast<uint32_t>(v) * estep;
      if (P < npts32) {
        uint32_t ic[3];
        ic[0] = P % g32.n[0];
        const uint32_t rest = P / g32.n[0];
        if (DIM == 2) {
          ic[1] = rest;
          ic[2] = 0;
        } else {
          ic[1] = rest % g32.n[1];
          ic[2] = rest / g32.n[1];
        }
        T out[DIM + 1];
        apply_point_all<T, K, BC, DIM>(g, g32, xcol, P, ic, out);
        if (src.n > 0 && static_cast<int64_t>(P) >= src.lo && static_cast<int64_t>(P) <= src.hi) {
          for (int s = 0; s < src.n; ++s)
            if (src.idx[s] == static_cast<int64_t>(P)) {
              double gt = 0.0;
              for (int cc = 0; cc < src.p; ++cc)
                gt += src.G[cc] * static_cast<double>(tailv(cc));
              out[0] += static_cast<T>(gt * static_cast<double>(amp[s]));
            }
        }
#pragma unroll
        for (int f = 0; f <= DIM; ++f) w[f * UP + v] = out[f];
      } else {
        // beyond the grid: the pressure slot may hold tail element t, J q_tail
        const uint32_t t = P - npts32;
#pragma unroll
        for (int f = 0; f <= DIM; ++f) w[f * UP + v] = T(0);
        if (t < ntail32) {
          const int cc = static_cast<int>(t);
          w[v] = (cc + 1 < src.p) ? tailv(cc + 1) : T(0);
        }
      }
    }
    // first sweep: value i <= j is <w, Q_i>, value j + 1 + l (l < j) is
    // <Q_j, Q_l>, value 2j + 1 is |Q_j|^2 (stored by the previous column's
    // second sweep; |x|^2 for column 0); columns j-1 down to 1, so that the
    // second sweep starts on the columns read last
    {
      T r = T(0), gq = T(0);
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        r += w[u] * q0[u];
        gq += s_qj[u][threadIdx.x] * q0[u];
      }
      // value 1 of column 0 is |x|^2
      put2(0, static_cast<double>(r), j >= 1 ? j + 1 : 1, j >= 1 ? static_cast<double>(gq) : xx);
    }
    auto dot1 = [&](int i, const T* q) {
      T r = T(0), gq = T(0);
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        r += w[u] * q[u];
        gq += s_qj[u][threadIdx.x] * q[u];
      }
      put2(i, static_cast<double>(r), j + 1 + i, static_cast<double>(gq));
    };
    // columns 1..j-1: the first nc in LDS, the other ns streamed from memory
    const int nc = j - 1 < NC ? (j - 1 > 0 ? j - 1 : 0) : NC;
    const int ns = j - 1 > nc ? j - 1 - nc : 0;
    stream(j - 1, ns, -1, dot1);
    for (int i = nc; i >= 1; --i) from_lds(i, dot1);
    if (j >= 1) {
      T r = T(0);
#pragma unroll
      for (int u = 0; u < UN; ++u) r += w[u] * s_qj[u][threadIdx.x];
      put(j, static_cast<double>(r));
    }
    reduce(2 * j + 2, [&] {
      if (ns > 0) load_col(qa, nc + 1);
    });
    if (j == 0) {
      // q_0 = x / beta, and w = H~ q_0
      beta = sqrt(s_tot[1]);
      inv = beta > 0.0 ? 1.0 / beta : 0.0;
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        bool ok;
        const uint32_t e = elem(u, ecur, ok);
        q0[u] = static_cast<T>(static_cast<double>(q0[u]) * inv);
        w[u] = static_cast<T>(static_cast<double>(w[u]) * inv);
        s_qj[u][threadIdx.x] = q0[u];
        if (ok) st_at(Q, e * kEs, q0[u]);
      }
      if (lead) {
        *beta_out = beta;
        sc[0] = 1.0;
      }
    }
    // s_j = 1 / h_{j,j-1} (0 at a breakdown), and w = s_j H~ Q_j
    double sjd = 1.0;
    if (j >= 1) {
      const double hn = sqrt(s_tot[2 * j + 1]);
      sjd = (hn > a.tol * beta) ? 1.0 / hn : 0.0;
      if (lead) {
        hess[j * kArnHessLd + j - 1] = hn;
        sc[j] = sjd;
      }
      if (threadIdx.x == 0) s_scale[j] = sjd;  // read by later columns, after their reductions
      const T sj = static_cast<T>(sjd);
#pragma unroll
      for (int u = 0; u < UN; ++u) w[u] *= sj;
    }
    // MGS's projections: h_i = r_i - sum_{l<i} h_l <q_l, q_i>, lane i of wave 0
    if (wid == 0) {
      const double sl = lane < j ? s_scale[lane] : (lane == j ? sjd : 0.0);
      double r = lane <= j ? s_tot[lane] * sl * sjd : 0.0;  // <s_j H~ Q_j, q_lane>
      if (j == 0) r *= inv * inv;                            // <H~ x, x> / beta^2
      const double grow = lane < j ? s_tot[j + 1 + lane] * sjd * sl : 0.0;  // <q_j, q_lane>
      // Gram entries are read from LDS eight steps ahead of the dependent chain
      for (int l0 = 0; l0 < j; l0 += 8) {
        double gb[8];
#pragma unroll
        for (int t = 0; t < 8; ++t)
          gb[t] = (l0 + t < j && lane > l0 + t && lane < j) ? s_gt[lane * (lane - 1) / 2 + l0 + t] : 0.0;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int l = l0 + t;
          if (l < j) {
            const double hl = readlane_f64(r, l);  // final: lanes below l+1 are done
            const double gil = (lane == j) ? readlane_f64(grow, l) : gb[t];
            if (lane > l && lane <= j) r -= hl * gil;
          }
        }
      }
      if (lane < j) s_gt[j * (j - 1) / 2 + lane] = grow;
      if (lane <= j) {
        s_h[lane] = r * sl;  // applied to the stored column Q_i = q_i / s_i
        if (blockIdx.x == 0) hess[lane * kArnHessLd + j] = r;
      }
    }
    __syncthreads();
    // the last column's orthogonalized vector only gives h_{k,k-1} and Q_k,
    // which neither the exponential of the k x k matrix H_k nor the
    // combination of Q_0..Q_{k-1} uses; only an error estimate needs h_{k,k-1}
    if (j + 1 == a.k && !a.full_last) break;
    // second sweep: w -= h_i q_i in order i = 0..j, then |w|^2
    {
      const T h0 = static_cast<T>(s_h[0]);
#pragma unroll
      for (int u = 0; u < UN; ++u) w[u] -= h0 * q0[u];
    }
    auto upd = [&](int i, const T* q) {
      const T hi = static_cast<T>(s_h[i]);
#pragma unroll
      for (int u = 0; u < UN; ++u) w[u] -= hi * q[u];
    };
    for (int i = 1; i <= nc; ++i) from_lds(i, upd);
    stream(nc + 1, ns, 1, upd);
    if (j >= 1) {
      const T hj = static_cast<T>(s_h[j]);
#pragma unroll
      for (int u = 0; u < UN; ++u) w[u] -= hj * s_qj[u][threadIdx.x];
    }
    T nrm = T(0);
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      bool ok;
      const uint32_t e = elem(u, ecur, ok);
      if (ok) st_at(wout, e * kEs, w[u]);
      nrm += w[u] * w[u];
      s_qj[u][threadIdx.x] = w[u];
      if (j < NC) s_cache[j < NC ? j : 0][u][threadIdx.x] = w[u];
    }
    // |Q_{j+1}|^2 goes with the next column's reduction (value 2j + 3)
    put(j + 1 < a.k ? 2 * j + 3 : 0, static_cast<double>(nrm));
    if (j + 1 < a.k) {
      // this workgroup's slice of Q_{j+1} is stored (s_waitcnt 0 in every
      // thread, then the block barrier): publish it
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (threadIdx.x == 0) st_coherent(flags + blockIdx.x, ep + static_cast<unsigned long long>(j + 1));
      if (j > NC) load_col(qa, j);  // the next first sweep starts on Q_j
    }
  }
  if (a.full_last) {
    // h_{k,k-1} = |Q_k| for the error estimate
    reduce(1, [] {});
    const double hn = sqrt(s_tot[0]);
    if (lead) {
      hess[a.k * kArnHessLd + a.k - 1] = hn;
      sc[a.k] = (hn > a.tol * beta) ? 1.0 / hn : 0.0;
    }
  }
  // every block has read seq_io and the epoch: they all passed the barriers since
  if (lead) {
    st_coherent(seq_io, seq % static_cast<unsigned>(kSlotBuffers));
    st_coherent(flags + kArnMaxBlocks, ep + static_cast<unsigned long long>(a.k + 1));
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
