// Per-step form of sliced bucket elimination on gfx950 (CDNA4): one launch
// per bucket (or merged chain of buckets) for a group of slices, the
// intermediates in HBM.  The fused form is in fused.hip.
//
// Kernels
//   prep_kernel        complex128 model entries -> complex64 prepared inputs
//                      through a gather map (layout chosen by the planner).
//   step_kernel        one bucket: result entry sum_u prod_i T_i[pext(X,
//                      mask_i)], X = (u << r) | x.  The low 8 bits of x come
//                      from the lane, so results are stored coalesced and
//                      operands holding those variables are read coalesced;
//                      lanes decode the addresses of 64 tiles at a time.
//                      HBM-bound (about 2 flop/B).
//   msum_kernel        a merged chain of buckets: the same with 2^n_sum >= 4
//                      terms per result entry, four at a time.
//   step_pair_kernel,  the same two with two tiles per thread that differ
//   msum_pair_kernel   in x bit 0: operands holding it are read with one
//                      16-byte load for both tiles, the others once for both,
//                      results stored in 16-byte pairs.
//   step_small_kernel  the same two for results of fewer than 8 variables
//   msum_small_kernel  (several slices per tile).
//   mm_kernel          outer-product buckets on MFMA (FP32 or split BF16).
//   mmb_kernel         merged two-group products as whole-block GEMMs on
//                      MFMA, the contraction running over all summed
//                      variables (A', B' staged in LDS once per block).
//   mmk_kernel         the same products as independent 16 x 16 tiles (for
//                      factor counts the block kernel does not take).
//   group_kernel,      the small launches of one dependency level (of one
//   wide_group_kernel  plan, or of all per-step instances of a batch).
//   finalize_kernel    per-slice product of the rank-0 results, in FP64.
//   reduce_kernel      deterministic FP64 sum of per-slice values (Eq. 4).
#include "device_common.hpp"

#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

namespace qbe {

// ------------------------------------------------------------------- prep --

__global__ void prep_kernel(const double2* __restrict__ raw, const int32_t* __restrict__ map,
                            float2* __restrict__ out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double2 v = raw[map[i]];
    out[i] = make_float2((float)v.x, (float)v.y);
  }
}

// --------------------------------------------------------------- per-step --

struct StepLaunch {
  float2* out;
  const float2* src[kMaxOps];
  int64_t gstride[kMaxOps];  // elements between consecutive slices (0: input)
  uint32_t mask[kMaxOps];
  uint32_t smask[kMaxOps];
  int32_t rank[kMaxOps];
  int32_t n_ops;
  int32_t r;       // bits of x
  int32_t sum_u;   // 1: sum over the top bit u of X
  int32_t n_sum;   // msum kernels: summed top bits of X
  int32_t lo;      // min(r, kLoBits)
  int64_t s0;      // first slice of the group
  int64_t G;       // slices in the group
  int64_t n_tiles;
  // msum kernels: byte offset of operand i's entry for summed value u = 1 <<
  // b above its entry for u = 0 (0 if it lacks bit b); the offset for any u
  // is the sum over u's bits (bit extraction is linear over disjoint bits).
  // And the bits of u the operand holds.
  uint32_t uw[kMaxOps][4];
  uint32_t uhold[kMaxOps];
};

// Global-memory views of addresses carried as integers (a generic pointer
// would compile to flat accesses).
typedef const __attribute__((address_space(1))) char* gcbytep;
typedef __attribute__((address_space(1))) char* gbytep;

typedef float gf32x2 __attribute__((ext_vector_type(2)));

// Load at a wave-uniform base plus a per-lane 32-bit byte offset.
__device__ __forceinline__ float2 ld_sv(uint64_t base, uint32_t byte_off) {
  const gf32x2 v = *(const __attribute__((address_space(1))) gf32x2*)((gcbytep)base + byte_off);
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void st_sv(uint64_t base, uint32_t byte_off, float2 v) {
  *(__attribute__((address_space(1))) gf32x2*)((gbytep)base + byte_off) = gf32x2{v.x, v.y};
}
typedef float gf32x4 __attribute__((ext_vector_type(4)));
// Two consecutive complex64 entries.
__device__ __forceinline__ void ld_sv2(uint64_t base, uint32_t byte_off, float2& a, float2& b) {
  const gf32x4 v = *(const __attribute__((address_space(1))) gf32x4*)((gcbytep)base + byte_off);
  a = make_float2(v.x, v.y);
  b = make_float2(v.z, v.w);
}
__device__ __forceinline__ void st_sv2(uint64_t base, uint32_t byte_off, float2 a, float2 b) {
  *(__attribute__((address_space(1))) gf32x4*)((gbytep)base + byte_off) = gf32x4{a.x, a.y, b.x, b.y};
}

// A 64-bit wave-uniform value held by lane k.
__device__ __forceinline__ uint64_t lane64(uint64_t v, int k) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, k);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), k);
  return ((uint64_t)hi << 32) | lo;
}

// Scatter the low bits of v to the set bits of m, lowest first.
__device__ __forceinline__ uint32_t pdep32(uint32_t v, uint32_t m) {
  uint32_t r = 0;
  int k = 0;
  while (m) {
    const int b = __builtin_ctz(m);
    r |= ((v >> k) & 1u) << b;
    ++k;
    m &= m - 1;
  }
  return r;
}

// XCDs of the chip (workgroups are dealt to them round robin)
constexpr uint32_t kXcds = 8;

// The workgroup's number with one XCD's workgroups (each XCD has its own
// L2) numbered consecutively: workgroup b becomes (b mod 8) * (grid / 8) +
// b / 8; the last (grid mod 8) workgroups keep their own number.  Loops
// that start at this number and step by the grid give neighbouring work --
// the tiles of one slice, which read the same factor lines -- to one L2 at
// the same time.
__device__ __forceinline__ uint32_t xcd_major_block() {
  const uint32_t n_wg = gridDim.x, per_xcd = n_wg / kXcds;
  return blockIdx.x < per_xcd * kXcds ? (blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds : blockIdx.x;
}

// Tiling of step_kernel and msum_kernel (r >= kLoBits).  A tile is 256
// consecutive result entries of one slice: the lane supplies x_lo (the low 8
// bits of x), the tile the slice g and x_hi.  A super-tile is EPT tiles that
// differ only in the lowest bits of x_hi (EPT divides 2^hib); the block
// takes super-tiles q = xcd_major_block() + j * gridDim.x.  An operand's
// entry offset is linear over disjoint bit sets, so it splits into a
// per-lane part (x_lo and the sub-tile bits, fixed for the kernel) and a
// per-super-tile part (slice and the rest of x_hi).  The per-super-tile
// addresses of 64 super-tiles at a time are worked out in vector code, lane
// l taking the l-th of them, and the tile loop reads them back with
// readlane: the per-tile index work is off the scalar unit.
// PAIR (EPT = 2): the two tiles differ in x bit 0 instead and the lane
// supplies bits 1-8; the super-tile bits are the same.
template <int K, int EPT, bool PAIR = false>
struct TileSetup {
  uint32_t lofs[EPT][K];  // per-lane byte offsets
  uint32_t hi_mask[K];    // x_hi bits of each operand
  int lo_cnt[K];          // operand bits below x_hi
  int hib;
  int64_t n_super;

  __device__ __forceinline__ TileSetup(const StepLaunch& a, uint32_t x_lo) {
    hib = a.r - kLoBits;
    n_super = a.n_tiles / EPT;
    if (PAIR) {
      static_assert(!PAIR || EPT == 2, "paired tiles come two at a time");
#pragma unroll
      for (int i = 0; i < K; ++i) {
        hi_mask[i] = (a.mask[i] >> kLoBits) & ((1u << hib) - 1u);
        lo_cnt[i] = __builtin_popcount(a.mask[i] & (kBlock - 1));
#pragma unroll
        for (int e = 0; e < EPT; ++e) lofs[e][i] = pext32((x_lo << 1) | (uint32_t)e, a.mask[i] & (2u * kBlock - 1u)) * 8u;
      }
      return;
    }
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const uint32_t m = a.mask[i];
      const uint32_t lp = pext32(x_lo, m & (kBlock - 1));
      lo_cnt[i] = __builtin_popcount(m & (kBlock - 1));
      const uint32_t hm = (m >> kLoBits) & ((1u << hib) - 1u);
      hi_mask[i] = hm;
#pragma unroll
      for (int e = 0; e < EPT; ++e) lofs[e][i] = (lp + (pext32((uint32_t)e, hm) << lo_cnt[i])) * 8u;
    }
  }

  // Lane l: operand base addresses and the result address (entry x_lo = 0
  // of the first tile) of the block's super-tile q0 + l * gridDim.x.  Lanes
  // past the end compute addresses that are never used.
  __device__ __forceinline__ void decode(const StepLaunch& a, int64_t q0, int lane, uint64_t (&pl)[K],
                                         uint64_t& ol) const {
    const int64_t tl = (q0 + (int64_t)lane * gridDim.x) * EPT;
    const int64_t g = tl >> hib;
    const uint32_t xl = (uint32_t)(tl & ((int64_t(1) << hib) - 1));
    const uint32_t s = (uint32_t)(a.s0 + g);
#pragma unroll
    for (int i = 0; i < K; ++i) {
      // element offsets in 64 bits: an input's copies of a rank-30 tensor
      // lie more than 2^32 entries apart
      const uint64_t sp = a.gstride[i] != 0 ? 0ull : (uint64_t)pext32(s, a.smask[i]) << a.rank[i];
      const uint64_t off = sp + ((uint64_t)pext32(xl, hi_mask[i]) << lo_cnt[i]);
      pl[i] = (uint64_t)(a.src[i] + g * a.gstride[i] + off);
    }
    ol = (uint64_t)(a.out + (g << a.r) + ((int64_t)xl << kLoBits));
  }

  // super-tiles of this block from q0 on that one decode covers
  __device__ __forceinline__ int count(int64_t q0) const {
    return (int)std::min<int64_t>(64, (n_super - q0 + gridDim.x - 1) / gridDim.x);
  }
};

// One bucket (n_sum <= 1) for r >= kLoBits: result entry
// sum_u prod_i T_i[pext(X, mask_i)] per lane and tile.
template <int K, int EPT>
__global__ __launch_bounds__(kBlock) void step_kernel(StepLaunch a) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int r = a.r;
  const TileSetup<K, EPT> ts(a, (uint32_t)tid);
  // bytes from an operand's u = 0 entry to its u = 1 entry: 2^(rank - 1)
  // entries, 2^32 bytes for a rank-30 operand, so 64 bits
  uint64_t ustep[K];
#pragma unroll
  for (int i = 0; i < K; ++i)
    ustep[i] = (a.sum_u && ((a.mask[i] >> r) & 1u)) ? (uint64_t(1) << (a.rank[i] - 1)) * 8u : 0u;
  for (int64_t q0 = xcd_major_block(); q0 < ts.n_super; q0 += 64 * (int64_t)gridDim.x) {
    uint64_t pl[K], ol;
    ts.decode(a, q0, lane, pl, ol);
    const int n_here = ts.count(q0);
    for (int jj = 0; jj < n_here; ++jj) {
      float2 v0[EPT][K], v1[EPT][K];
#pragma unroll
      for (int i = 0; i < K; ++i) {
        const uint64_t b = lane64(pl[i], jj), b1 = b + ustep[i];
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          v0[e][i] = ld_sv(b, ts.lofs[e][i]);
          if (a.sum_u) v1[e][i] = ld_sv(b1, ts.lofs[e][i]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
      const uint64_t o = lane64(ol, jj);
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        float2 acc = v0[e][0];
#pragma unroll
        for (int i = 1; i < K; ++i) acc = cmul(acc, v0[e][i]);
        if (a.sum_u) {
          float2 u1 = v1[e][0];
#pragma unroll
          for (int i = 1; i < K; ++i) u1 = cmul(u1, v1[e][i]);
          acc.x += u1.x;
          acc.y += u1.y;
        }
        st_sv(o, (uint32_t)((e << kLoBits) + tid) * 8u, acc);
      }
    }
  }
}

// A launch that merges a chain of buckets (r >= kLoBits): the top n_sum
// bits of X are summed, 2^n_sum >= 4 terms per result entry.  Operand i's
// entry for summed value u sits sum_b bit_b(u) uw[i][b] bytes above its
// u = 0 entry, the same for every lane and tile: the term loop adds scalar
// offsets, worked out without memory reads, to a scalar base.
template <int K, int EPT, bool LEAD>
__global__ __launch_bounds__(kBlock) void msum_kernel(StepLaunch a) {
  const int tid = threadIdx.x, lane = tid & 63;
  const TileSetup<K, EPT> ts(a, (uint32_t)tid);
  const int nu = 1 << a.n_sum;
  for (int64_t q0 = xcd_major_block(); q0 < ts.n_super; q0 += 64 * (int64_t)gridDim.x) {
    uint64_t pl[K], ol;
    ts.decode(a, q0, lane, pl, ol);
    const int n_here = ts.count(q0);
    for (int jj = 0; jj < n_here; ++jj) {
      uint64_t b[K];
#pragma unroll
      for (int i = 0; i < K; ++i) b[i] = lane64(pl[i], jj);
      float2 acc[EPT];
#pragma unroll
      for (int e = 0; e < EPT; ++e) acc[e] = make_float2(0.f, 0.f);
      // Four terms per trip, over the two lowest summed bits d: a factor
      // holding c = its bits of d has 2^popcount(c) distinct entries in the
      // trip, read once each, all loads in flight together.  Factors with
      // c = 0 are common to the four terms and multiply their sum.
      for (int u0 = 0; u0 < nu; u0 += 4) {
        float2 v[4][EPT][K];
#pragma unroll
        for (int i = 0; i < K; ++i) {
          const uint32_t c = a.uhold[i] & 3u;
          const uint32_t ob = ((u0 & 4) ? a.uw[i][2] : 0u) + ((u0 & 8) ? a.uw[i][3] : 0u);
#pragma unroll
          for (int du = 0; du < 4; ++du)
            if (((uint32_t)du & ~c) == 0u) {
              const uint32_t off = ob + ((du & 1) ? a.uw[i][0] : 0u) + ((du & 2) ? a.uw[i][1] : 0u);
              const uint64_t bu = b[i] + off;
#pragma unroll
              for (int e = 0; e < EPT; ++e) v[du][e][i] = ld_sv(bu, ts.lofs[e][i]);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        float2 cm[EPT], pr[4][EPT];
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          cm[e] = make_float2(1.f, 0.f);
#pragma unroll
          for (int du = 0; du < 4; ++du) pr[du][e] = LEAD ? v[du][e][0] : make_float2(1.f, 0.f);
        }
#pragma unroll
        for (int i = LEAD ? 1 : 0; i < K; ++i) {
          const uint32_t c = a.uhold[i] & 3u;
          if (c == 0u) {
#pragma unroll
            for (int e = 0; e < EPT; ++e) cm[e] = cmul(cm[e], v[0][e][i]);
          } else if (c == 1u) {
#pragma unroll
            for (int du = 0; du < 4; ++du)
#pragma unroll
              for (int e = 0; e < EPT; ++e) pr[du][e] = cmul(pr[du][e], v[du & 1][e][i]);
          } else if (c == 2u) {
#pragma unroll
            for (int du = 0; du < 4; ++du)
#pragma unroll
              for (int e = 0; e < EPT; ++e) pr[du][e] = cmul(pr[du][e], v[du & 2][e][i]);
          } else {
#pragma unroll
            for (int du = 0; du < 4; ++du)
#pragma unroll
              for (int e = 0; e < EPT; ++e) pr[du][e] = cmul(pr[du][e], v[du][e][i]);
          }
        }
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          const float2 t = make_float2(pr[0][e].x + pr[1][e].x + pr[2][e].x + pr[3][e].x,
                                       pr[0][e].y + pr[1][e].y + pr[2][e].y + pr[3][e].y);
          const float2 q = cmul(cm[e], t);
          acc[e] = make_float2(acc[e].x + q.x, acc[e].y + q.y);
        }
      }
      const uint64_t o = lane64(ol, jj);
#pragma unroll
      for (int e = 0; e < EPT; ++e) st_sv(o, (uint32_t)((e << kLoBits) + tid) * 8u, acc[e]);
    }
  }
}

// step_kernel with two tiles per thread that differ in x bit 0, paired as
// in msum_pair_kernel: the first NP operands hold bit 0 (one 16-byte load
// for both tiles), the others are read once for both.
template <int K, int NP>
__global__ __launch_bounds__(kBlock) void step_pair_kernel(StepLaunch a) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int r = a.r;
  const TileSetup<K, 2, true> ts(a, (uint32_t)tid);
  // bytes from an operand's u = 0 entry to its u = 1 entry: 2^(rank - 1)
  // entries, 2^32 bytes for a rank-30 operand, so 64 bits
  uint64_t ustep[K];
#pragma unroll
  for (int i = 0; i < K; ++i)
    ustep[i] = (a.sum_u && ((a.mask[i] >> r) & 1u)) ? (uint64_t(1) << (a.rank[i] - 1)) * 8u : 0u;
  for (int64_t q0 = xcd_major_block(); q0 < ts.n_super; q0 += 64 * (int64_t)gridDim.x) {
    uint64_t pl[K], ol;
    ts.decode(a, q0, lane, pl, ol);
    const int n_here = ts.count(q0);
    for (int jj = 0; jj < n_here; ++jj) {
      float2 v0[2][K], v1[2][K];
#pragma unroll
      for (int i = 0; i < K; ++i) {
        const uint64_t b = lane64(pl[i], jj), b1 = b + ustep[i];
        if (i < NP) {
          ld_sv2(b, ts.lofs[0][i], v0[0][i], v0[1][i]);
          if (a.sum_u) ld_sv2(b1, ts.lofs[0][i], v1[0][i], v1[1][i]);
        } else {
          v0[0][i] = ld_sv(b, ts.lofs[0][i]);
          v0[1][i] = v0[0][i];
          if (a.sum_u) {
            v1[0][i] = ld_sv(b1, ts.lofs[0][i]);
            v1[1][i] = v1[0][i];
          }
        }
      }
      __builtin_amdgcn_sched_barrier(0);
      float2 acc[2];
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        acc[e] = v0[e][0];
#pragma unroll
        for (int i = 1; i < K; ++i) acc[e] = cmul(acc[e], v0[e][i]);
        if (a.sum_u) {
          float2 u1 = v1[e][0];
#pragma unroll
          for (int i = 1; i < K; ++i) u1 = cmul(u1, v1[e][i]);
          acc[e].x += u1.x;
          acc[e].y += u1.y;
        }
      }
      st_sv2(lane64(ol, jj), (uint32_t)tid * 16u, acc[0], acc[1]);
    }
  }
}

// msum_kernel with two tiles per thread that differ in x bit 0 (the lane
// supplies bits 1-8): an operand holding bit 0 -- the first NP operands, as
// the host orders them -- has its two entries side by side and is read with
// one 16-byte load; the others have the same entry for both tiles and are
// read once.  Results are written in 16-byte pairs.  Every load and store
// instruction thus serves two result entries.
template <int K, int NP, bool LEAD>
__global__ __launch_bounds__(kBlock) void msum_pair_kernel(StepLaunch a) {
  const int tid = threadIdx.x, lane = tid & 63;
  const TileSetup<K, 2, true> ts(a, (uint32_t)tid);
  const int nu = 1 << a.n_sum;
  for (int64_t q0 = xcd_major_block(); q0 < ts.n_super; q0 += 64 * (int64_t)gridDim.x) {
    uint64_t pl[K], ol;
    ts.decode(a, q0, lane, pl, ol);
    const int n_here = ts.count(q0);
    for (int jj = 0; jj < n_here; ++jj) {
      uint64_t b[K];
#pragma unroll
      for (int i = 0; i < K; ++i) b[i] = lane64(pl[i], jj);
      float2 acc[2] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
      // four terms per trip over the two lowest summed bits, as in msum_kernel
      for (int u0 = 0; u0 < nu; u0 += 4) {
        float2 v[4][2][K];
#pragma unroll
        for (int i = 0; i < K; ++i) {
          const uint32_t c = a.uhold[i] & 3u;
          const uint32_t ob = ((u0 & 4) ? a.uw[i][2] : 0u) + ((u0 & 8) ? a.uw[i][3] : 0u);
#pragma unroll
          for (int du = 0; du < 4; ++du)
            if (((uint32_t)du & ~c) == 0u) {
              const uint32_t off = ob + ((du & 1) ? a.uw[i][0] : 0u) + ((du & 2) ? a.uw[i][1] : 0u);
              const uint64_t bu = b[i] + off;
              if (i < NP) {
                ld_sv2(bu, ts.lofs[0][i], v[du][0][i], v[du][1][i]);
              } else {
                v[du][0][i] = ld_sv(bu, ts.lofs[0][i]);
                v[du][1][i] = v[du][0][i];
              }
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        float2 cm[2], pr[4][2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          cm[e] = make_float2(1.f, 0.f);
#pragma unroll
          for (int du = 0; du < 4; ++du) pr[du][e] = LEAD ? v[du][e][0] : make_float2(1.f, 0.f);
        }
#pragma unroll
        for (int i = LEAD ? 1 : 0; i < K; ++i) {
          const uint32_t c = a.uhold[i] & 3u;
          if (c == 0u) {
#pragma unroll
            for (int e = 0; e < 2; ++e) cm[e] = cmul(cm[e], v[0][e][i]);
          } else if (c == 1u) {
#pragma unroll
            for (int du = 0; du < 4; ++du)
#pragma unroll
              for (int e = 0; e < 2; ++e) pr[du][e] = cmul(pr[du][e], v[du & 1][e][i]);
          } else if (c == 2u) {
#pragma unroll
            for (int du = 0; du < 4; ++du)
#pragma unroll
              for (int e = 0; e < 2; ++e) pr[du][e] = cmul(pr[du][e], v[du & 2][e][i]);
          } else {
#pragma unroll
            for (int du = 0; du < 4; ++du)
#pragma unroll
              for (int e = 0; e < 2; ++e) pr[du][e] = cmul(pr[du][e], v[du][e][i]);
          }
        }
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const float2 t = make_float2(pr[0][e].x + pr[1][e].x + pr[2][e].x + pr[3][e].x,
                                       pr[0][e].y + pr[1][e].y + pr[2][e].y + pr[3][e].y);
          const float2 q = cmul(cm[e], t);
          acc[e] = make_float2(acc[e].x + q.x, acc[e].y + q.y);
        }
      }
      st_sv2(lane64(ol, jj), (uint32_t)tid * 16u, acc[0], acc[1]);
    }
  }
}

// Small results (r < kLoBits): a tile holds 256 >> r whole slices, so the
// slice index comes from the lane.  step_small_kernel is step_kernel's
// bucket, msum_small_kernel msum_kernel's merged chain.
template <int K>
__global__ __launch_bounds__(kBlock) void step_small_kernel(StepLaunch a) {
  const int tid = threadIdx.x;
  const int r = a.r;
  const uint32_t x = (uint32_t)tid & ((1u << r) - 1u);
  const int64_t g_sub = tid >> r;
  const int64_t spt = (int64_t)(kBlock >> r);
  uint32_t xpart[K], u_part[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    xpart[i] = pext32(x, a.mask[i]);
    u_part[i] = (a.sum_u && ((a.mask[i] >> r) & 1u)) ? (1u << (a.rank[i] - 1)) : 0u;
  }
  for (int64_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
    const int64_t g = tile * spt + g_sub;
    if (g >= a.G) continue;
    const int64_t s = a.s0 + g;
    float2 v0[K], v1[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      int64_t base;
      if (a.gstride[i] != 0)
        base = g * a.gstride[i];
      else
        base = (int64_t)pext32((uint32_t)s, a.smask[i]) << a.rank[i];
      const float2* q = a.src[i] + base + xpart[i];
      v0[i] = q[0];
      v1[i] = q[u_part[i]];
    }
    float2 acc = v0[0];
#pragma unroll
    for (int i = 1; i < K; ++i) acc = cmul(acc, v0[i]);
    if (a.sum_u) {
      float2 t = v1[0];
#pragma unroll
      for (int i = 1; i < K; ++i) t = cmul(t, v1[i]);
      acc.x += t.x;
      acc.y += t.y;
    }
    a.out[(g << r) + x] = acc;
  }
}

template <int K>
__global__ __launch_bounds__(kBlock) void msum_small_kernel(StepLaunch a) {
  const int tid = threadIdx.x;
  const int r = a.r;
  const uint32_t x = (uint32_t)tid & ((1u << r) - 1u);
  const int64_t g_sub = tid >> r;
  const int64_t spt = (int64_t)(kBlock >> r);
  const int nu = 1 << a.n_sum;
  uint32_t xpart[K];
#pragma unroll
  for (int i = 0; i < K; ++i) xpart[i] = pext32(x, a.mask[i]) * 8u;
  for (int64_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
    const int64_t g = tile * spt + g_sub;
    if (g >= a.G) continue;
    const int64_t s = a.s0 + g;
    const char* q[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      int64_t base;
      if (a.gstride[i] != 0)
        base = g * a.gstride[i];
      else
        base = (int64_t)pext32((uint32_t)s, a.smask[i]) << a.rank[i];
      q[i] = (const char*)(a.src[i] + base) + xpart[i];
    }
    float2 acc = make_float2(0.f, 0.f);
    for (int u = 0; u < nu; ++u) {
      auto uoff = [&](int i) {
        return ((u & 1) ? a.uw[i][0] : 0u) + ((u & 2) ? a.uw[i][1] : 0u) + ((u & 4) ? a.uw[i][2] : 0u) +
               ((u & 8) ? a.uw[i][3] : 0u);
      };
      float2 p = *(const float2*)(q[0] + uoff(0));
#pragma unroll
      for (int i = 1; i < K; ++i) p = cmul(p, *(const float2*)(q[i] + uoff(i)));
      acc.x += p.x;
      acc.y += p.y;
    }
    a.out[(g << r) + x] = acc;
  }
}

// --------------------------------------------------- grouped small steps --
//
// The small launches of one dependency level in one launch.  Work unit w =
// (tile t of the level's tile range, block yb of sb slices); the step owning
// tile t is found by binary search in the level's tile prefix.  A tile is
// 256 consecutive entries of the step's results for the block's sb slices
// (several slices when r < 8).  Operands are addressed as in step_kernel,
// with the bit extraction done per lane: these steps are small.
struct GroupArgs {
  const GroupStep* steps;   // the level's steps
  const uint32_t* prefix;   // count + 1 tile offsets
  int32_t count;
  int32_t sb;               // slices per block (power of two)
  float2* arena;
  const float2* step_in;
  int64_t G, s0, n_blocks;  // n_blocks = ceil(G / sb)
};

// Tile t of step d for the block of sb slices starting at slice yb * sb.
__device__ __forceinline__ void group_tile(const GroupStep& d, float2* arena, const float2* step_in, int64_t G,
                                           int64_t s0, int sb, int64_t yb, uint32_t t, int tid) {
  const int r = d.r;
  const int64_t e = (int64_t)t * kBlock + tid;
  if (e >= ((int64_t)sb << r)) return;
  const int64_t g = yb * sb + (e >> r);
  if (g >= G) return;
  const uint32_t x = (uint32_t)(e & ((int64_t(1) << r) - 1));
  const uint32_t s = (uint32_t)(s0 + g);
  float2 p0 = make_float2(1.f, 0.f), p1 = make_float2(1.f, 0.f);
  for (int i = 0; i < d.n_ops; ++i) {
    const float2* src;
    if ((d.is_input >> i) & 1u)
      src = step_in + d.base[i] + ((int64_t)pext32(s, d.smask[i]) << d.rank[i]);
    else
      src = arena + d.base[i] * G + (g << d.rank[i]);
    src += pext32(x, d.mask[i]);
    p0 = cmul(p0, src[0]);
    if (d.sum_u) p1 = cmul(p1, src[((d.mask[i] >> r) & 1u) ? (1u << (d.rank[i] - 1)) : 0u]);
  }
  if (d.sum_u) {
    p0.x += p1.x;
    p0.y += p1.y;
  }
  arena[d.out * G + (g << r) + x] = p0;
}

__global__ __launch_bounds__(kBlock) void group_kernel(GroupArgs a) {
  const int64_t total = a.prefix[a.count];
  for (int64_t w = blockIdx.x; w < total * a.n_blocks; w += gridDim.x) {
    const int64_t yb = w / total;
    const uint32_t t = (uint32_t)(w - yb * total);
    int lo = 0, hi = a.count;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (a.prefix[mid] <= t) lo = mid; else hi = mid;
    }
    group_tile(a.steps[lo], a.arena, a.step_in, a.G, a.s0, a.sb, yb, t - a.prefix[lo], threadIdx.x);
  }
}

// The grouped steps of one level of a batch's per-step instances, every
// instance with all its slices: unit w of the level's prefix is (block of
// slices, tile) of one step.
struct WideArgs {
  const WideGroupStep* steps;
  const uint64_t* prefix;   // count + 1 unit offsets
  int32_t count;
  float2* ws;               // the batch's per-step workspace
};

__global__ __launch_bounds__(kBlock) void wide_group_kernel(WideArgs a) {
  const uint64_t total = a.prefix[a.count];
  for (uint64_t w = blockIdx.x; w < total; w += gridDim.x) {
    int lo = 0, hi = a.count;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (a.prefix[mid] <= w) lo = mid; else hi = mid;
    }
    const WideGroupStep& d = a.steps[lo];
    const uint64_t local = w - a.prefix[lo];
    const int64_t yb = (int64_t)(local / (uint32_t)d.tiles);
    const uint32_t t = (uint32_t)(local - (uint64_t)yb * (uint32_t)d.tiles);
    group_tile(d.s, a.ws + d.arena, (const float2*)d.step_in, d.G, 0, d.sb, yb, t, threadIdx.x);
  }
}

// ------------------------------------------------- outer-product buckets --
//
// A bucket whose result variables all belong to two operands A and B (both
// holding u; any other operand holds only u) is a batched complex product
//   R[c, m, n] = sum_u A[c, m, u] B[c, n, u] w(u)
// over the variables of A only (m), of B only (n) and of both (c).  One
// wavefront computes a 16 x 16 tile of (m, n) with two MFMAs, for the real
// and the imaginary part, on the lowest four m- and n-variables of the
// result; the tile loop runs over the slices and the remaining variables.
// Real K = 4 stacks (Re, Im) x (u = 0, 1):
//   Re R = [Re A0, Re A1, -Im A0, -Im A1] . [Re B0; Re B1; Im B0; Im B1]
//   Im R = [Re A0, Re A1,  Im A0,  Im A1] . [Im B0; Im B1; Re B0; Re B1]
// FP32 form: v_mfma_f32_16x16x4f32.  Split-BF16 forms (bfloat16 parts,
// v_mfma_f32_16x16x16bf16 over K = 16 = four groups of the four real-K
// entries, FP32 accumulation):
//   bf16x3: x = hi + lo; one MFMA sums hi*hi + hi*lo + lo*hi as
//           [hi | hi | lo | 0] . [hi ; lo ; hi ; 0]
//   bf16x6: x = h + m + l; two MFMAs sum h*h + h*m + m*h + h*l + l*h + m*m
//           as [h | h | m | h] . [h ; m ; h ; l] + [l | m | 0 | 0] . [h ; m ; 0 ; 0]

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));


// Round-to-nearest-even conversion to bfloat16 (finite inputs).
__device__ __forceinline__ uint32_t bf16_bits(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf16_value(uint32_t b) { return __uint_as_float(b << 16); }

struct MmLaunch {
  float2* out;
  const float2* src[2];     // A, B
  int64_t gs[2];            // elements between slices (0: input tensor)
  uint32_t sm[2];           // input slice masks
  int32_t rk[2];            // ranks
  uint32_t mk[2];           // masks over X (u = bit r)
  const float2* usrc[kMaxOps];  // rank-1 operands on u
  int64_t ugs[kMaxOps];
  uint32_t usm[kMaxOps];
  int32_t n_u;
  uint32_t mtile, ntile, rest;  // result-bit masks: 4 m bits, 4 n bits, the others
  int32_t r;
  int64_t s0, G, n_tiles;
};

// bfloat16 parts of x: the first two (h, x - h) or all three (h, m, l).
__device__ __forceinline__ void split_bf16(float x, uint32_t& h, uint32_t& m, uint32_t& l) {
  h = bf16_bits(x);
  const float r1 = x - bf16_value(h);  // exact in FP32
  m = bf16_bits(r1);
  l = bf16_bits(r1 - bf16_value(m));  // exact in FP32
}

template <int kPrec>
__global__ __launch_bounds__(kBlock) void mm_kernel(MmLaunch a) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const int64_t n_waves = (int64_t)gridDim.x * (kBlock / 64);
  const int r = a.r;
  const uint32_t ubit = 1u << r;
  const int row = lane & 15, grp = lane >> 4;
  const uint32_t xm = pdep32((uint32_t)row, a.mtile), xn = pdep32((uint32_t)row, a.ntile);
  const uint32_t ao0 = pext32(xm, a.mk[0]), ao1 = pext32(xm | ubit, a.mk[0]);
  const uint32_t bo0 = pext32(xn, a.mk[1]), bo1 = pext32(xn | ubit, a.mk[1]);
  uint32_t oo[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) oo[i] = pdep32((uint32_t)(4 * grp + i), a.mtile) | xn;
  const int rb = r - 8;
  for (int64_t t = wave; t < a.n_tiles; t += n_waves) {
    const int64_t g = t >> rb;
    const uint32_t xt = pdep32((uint32_t)(t & ((int64_t(1) << rb) - 1)), a.rest);
    const int64_t s = a.s0 + g;
    int64_t base[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      base[j] = a.gs[j] ? g * a.gs[j] : ((int64_t)pext32((uint32_t)s, a.sm[j]) << a.rk[j]);
      base[j] += pext32(xt, a.mk[j]);
    }
    float2 A0 = a.src[0][base[0] + ao0], A1 = a.src[0][base[0] + ao1];
    const float2 B0 = a.src[1][base[1] + bo0], B1 = a.src[1][base[1] + bo1];
    for (int j = 0; j < a.n_u; ++j) {
      const int64_t ub = a.ugs[j] ? g * a.ugs[j] : ((int64_t)pext32((uint32_t)s, a.usm[j]) << 1);
      A0 = cmul(A0, a.usrc[j][ub]);
      A1 = cmul(A1, a.usrc[j][ub + 1]);
    }
    floatx4 cre = {0.f, 0.f, 0.f, 0.f}, cim = {0.f, 0.f, 0.f, 0.f};
    if (kPrec == QBE_PREC_FP32) {
      // lane holds real-K entry k = grp of its row (A) and of its column (B)
      const float2 Av = (grp & 1) ? A1 : A0;
      const float2 Bv = (grp & 1) ? B1 : B0;
      const float a1 = (grp >> 1) ? -Av.y : Av.x, a2 = (grp >> 1) ? Av.y : Av.x;
      const float b1 = (grp >> 1) ? Bv.y : Bv.x, b2 = (grp >> 1) ? Bv.x : Bv.y;
      cre = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, cre, 0, 0, 0);
      cim = __builtin_amdgcn_mfma_f32_16x16x4f32(a2, b2, cim, 0, 0, 0);
    } else {
      // lane holds the four real-K entries of its row / column, as the part
      // its group stands for in the layouts above
      const float ra1[4] = {A0.x, A1.x, -A0.y, -A1.y}, ra2[4] = {A0.x, A1.x, A0.y, A1.y};
      const float rb1[4] = {B0.x, B1.x, B0.y, B1.y}, rb2[4] = {B0.y, B1.y, B0.x, B1.x};
      shortx4 pa1, pa2, pb1, pb2, qa1, qa2, qb1, qb2;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        uint32_t ha1, ma1, la1, ha2, ma2, la2, hb1, mb1, lb1, hb2, mb2, lb2;
        split_bf16(ra1[v], ha1, ma1, la1);
        split_bf16(ra2[v], ha2, ma2, la2);
        split_bf16(rb1[v], hb1, mb1, lb1);
        split_bf16(rb2[v], hb2, mb2, lb2);
        if (kPrec == QBE_PREC_BF16X3) {
          pa1[v] = (short)(grp == 3 ? 0u : grp == 2 ? ma1 : ha1);
          pa2[v] = (short)(grp == 3 ? 0u : grp == 2 ? ma2 : ha2);
          pb1[v] = (short)(grp == 3 ? 0u : grp == 1 ? mb1 : hb1);
          pb2[v] = (short)(grp == 3 ? 0u : grp == 1 ? mb2 : hb2);
        } else {
          pa1[v] = (short)(grp == 2 ? ma1 : ha1);
          pa2[v] = (short)(grp == 2 ? ma2 : ha2);
          pb1[v] = (short)(grp == 1 ? mb1 : grp == 3 ? lb1 : hb1);
          pb2[v] = (short)(grp == 1 ? mb2 : grp == 3 ? lb2 : hb2);
          qa1[v] = (short)(grp == 0 ? la1 : grp == 1 ? ma1 : 0u);
          qa2[v] = (short)(grp == 0 ? la2 : grp == 1 ? ma2 : 0u);
          qb1[v] = (short)(grp == 0 ? hb1 : grp == 1 ? mb1 : 0u);
          qb2[v] = (short)(grp == 0 ? hb2 : grp == 1 ? mb2 : 0u);
        }
      }
      cre = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(pa1, pb1, cre, 0, 0, 0);
      cim = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(pa2, pb2, cim, 0, 0, 0);
      if (kPrec == QBE_PREC_BF16X6) {
        cre = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(qa1, qb1, cre, 0, 0, 0);
        cim = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(qa2, qb2, cim, 0, 0, 0);
      }
    }
    const int64_t ob = (g << r) | xt;
#pragma unroll
    for (int i = 0; i < 4; ++i) a.out[ob | oo[i]] = make_float2(cre[i], cim[i]);
  }
}

// A merged launch whose result variables all belong to two factor groups A'
// and B' (each the product of its factors; together all result bits, at
// least four private bits each), summed over the top J bits of X:
//   R[c, m, n] = sum_k A'[c, m, k] B'[c, n, k],  k in [0, 2^J)
// a batched complex product with K = 2^J.  One wavefront computes a 16 x 16
// (m, n) tile with v_mfma_f32_16x16x4f32 over the real K = 2^(J+1) entries
// [Re A' | -Im A'] . [Re B' ; Im B'] (real part) and [Re A' | Im A'] .
// [Im B' ; Re B'] (imaginary part), four entries per MFMA: lane l of a call
// supplies entry 4c + l/16, i.e. term k = (4c + l/16) mod 2^J.
struct MmkLaunch {
  float2* out;
  const float2* src[kMaxOps];
  int64_t gs[kMaxOps];      // elements between slices (0: input tensor)
  uint32_t sm[kMaxOps];     // input slice masks
  int32_t rk[kMaxOps];
  uint32_t mk[kMaxOps];     // masks over X
  int32_t n_ops;
  uint32_t side_b;          // bit i: factor i belongs to B' (else to A')
  int32_t prec;             // QBE_PREC_*: FP32 or split-BF16 MFMAs
  uint32_t mtile, ntile, rest;
  int32_t r;
  int64_t s0, G, n_tiles;
};

// acc + a * b over one lane's real-K entry in split bfloat16: slots
// (h*h, h*m, m*h, 0) for bf16x3 (x = h + m), or (h*h, h*m, m*h, h*l) then
// (l*h, m*m, 0, 0) in a second call for bf16x6 (x = h + m + l).
__device__ __forceinline__ floatx4 mfma_split(float a, float b, floatx4 acc, int prec) {
  uint32_t ha, ma, la, hb, mb, lb;
  split_bf16(a, ha, ma, la);
  split_bf16(b, hb, mb, lb);
  shortx4 pa, pb;
  pa[0] = (short)ha;
  pa[1] = (short)ha;
  pa[2] = (short)ma;
  pb[0] = (short)hb;
  pb[1] = (short)mb;
  pb[2] = (short)hb;
  if (prec == QBE_PREC_BF16X3) {
    pa[3] = 0;
    pb[3] = 0;
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(pa, pb, acc, 0, 0, 0);
  }
  pa[3] = (short)ha;
  pb[3] = (short)lb;
  acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(pa, pb, acc, 0, 0, 0);
  shortx4 qa, qb;
  qa[0] = (short)la;
  qa[1] = (short)ma;
  qa[2] = 0;
  qa[3] = 0;
  qb[0] = (short)hb;
  qb[1] = (short)mb;
  qb[2] = 0;
  qb[3] = 0;
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(qa, qb, acc, 0, 0, 0);
}

// Tiles are decoded as in step_kernel: lane l of a wavefront works out the
// slice, the tile's result bits and the operands' offsets for the wave's
// l-th next tile, and the tile loop reads them back with readlane.
template <int J, int K>
__global__ __launch_bounds__(kBlock) void mmk_kernel(MmkLaunch a) {
  constexpr int KQ = (1 << J) / 4;  // terms a lane supplies per side
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const int64_t n_waves = (int64_t)gridDim.x * (kBlock / 64);
  const int r = a.r;
  const int rb = r - 8;
  const int row = lane & 15, grp = lane >> 4;
  const uint32_t xm = pdep32((uint32_t)row, a.mtile), xn = pdep32((uint32_t)row, a.ntile);
  uint32_t oo[4];  // bytes
#pragma unroll
  for (int i = 0; i < 4; ++i) oo[i] = (pdep32((uint32_t)(4 * grp + i), a.mtile) | xn) * 8u;
  // bit extraction is linear over disjoint bit sets, so an operand's index
  // is the OR of the parts from the lane's tile bits and term (fixed per
  // lane), and from the tile's other bits (fixed per tile)
  uint32_t lofs[K][KQ];  // bytes
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const uint32_t plane = pext32(((a.side_b >> i) & 1u) ? xn : xm, a.mk[i]);
#pragma unroll
    for (int q = 0; q < KQ; ++q) lofs[i][q] = (plane | pext32((uint32_t)(4 * q + grp) << r, a.mk[i])) * 8u;
  }
  for (int64_t t0 = wave; t0 < a.n_tiles; t0 += 64 * n_waves) {
    // lane l: tile t0 + l * n_waves (lanes past the end compute values that
    // are never read)
    const int64_t tl = t0 + (int64_t)lane * n_waves;
    const int32_t gl = (int32_t)(tl >> rb);
    const uint32_t xtl = pdep32((uint32_t)(tl & ((int64_t(1) << rb) - 1)), a.rest);
    const uint32_t sl = (uint32_t)(a.s0 + gl);
    uint64_t pl[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const uint64_t off = (a.gs[i] ? 0ull : (uint64_t)pext32(sl, a.sm[i]) << a.rk[i]) + pext32(xtl, a.mk[i]);
      pl[i] = (uint64_t)(a.src[i] + (int64_t)gl * a.gs[i] + off);
    }
    const uint64_t obl = (uint64_t)(a.out + (((int64_t)gl << r) | xtl));
    const int n_here = (int)std::min<int64_t>(64, (a.n_tiles - t0 + n_waves - 1) / n_waves);
    for (int k = 0; k < n_here; ++k) {
      float2 av[KQ], bv[KQ];
#pragma unroll
      for (int q = 0; q < KQ; ++q) {
        av[q] = make_float2(1.f, 0.f);
        bv[q] = make_float2(1.f, 0.f);
      }
#pragma unroll
      for (int i = 0; i < K; ++i) {
        const uint64_t base = lane64(pl[i], k);
        float2 v[KQ];
#pragma unroll
        for (int q = 0; q < KQ; ++q) v[q] = ld_sv(base, lofs[i][q]);
        if ((a.side_b >> i) & 1u) {
#pragma unroll
          for (int q = 0; q < KQ; ++q) bv[q] = cmul(bv[q], v[q]);
        } else {
#pragma unroll
          for (int q = 0; q < KQ; ++q) av[q] = cmul(av[q], v[q]);
        }
      }
      floatx4 cre = {0.f, 0.f, 0.f, 0.f}, cim = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int c = 0; c < 2 * KQ; ++c) {
        const int q = c % KQ;
        const bool im_slot = c >= KQ;
        const float a1 = im_slot ? -av[q].y : av[q].x, b1 = im_slot ? bv[q].y : bv[q].x;
        const float a2 = im_slot ? av[q].y : av[q].x, b2 = im_slot ? bv[q].x : bv[q].y;
        if (a.prec == QBE_PREC_FP32) {
          cre = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, cre, 0, 0, 0);
          cim = __builtin_amdgcn_mfma_f32_16x16x4f32(a2, b2, cim, 0, 0, 0);
        } else {
          // split-BF16: the lane's entry of the K = 4 call above becomes its
          // four bfloat16 slots, the part products along the slot index
          cre = mfma_split(a1, b1, cre, a.prec);
          cim = mfma_split(a2, b2, cim, a.prec);
        }
      }
      const uint64_t ob = lane64(obl, k);
#pragma unroll
      for (int i = 0; i < 4; ++i) st_sv(ob, oo[i], make_float2(cre[i], cim[i]));
    }
  }
}

// Merged two-group products as whole-block GEMMs.  A block is one slice and
// one value of the result bits outside the block bits: 2^MB (A'-private) x
// 2^NB (B'-private) result entries of T = 2^J terms each.  Workgroups take
// blocks in steps of the grid, numbered so that the workgroups of one XCD
// take consecutive blocks at each step: neighbouring blocks -- neighbouring
// entries of the factors -- are read at the same time behind one L2.  Per
// block: the factors that hold no block bit (their value depends
// on the term and the block only) multiply into one value per term; A'[k][m]
// and B'[k][n] (the products of each group's other factors, A' times the
// per-term value) are staged in LDS, every load of a factor in flight at
// once; the 16 x 16 tiles run on MFMA (waves take tiles round robin; tile
// bits = the four lowest block bits of each side); each tile is written
// through a per-wave LDS buffer in result order, so that stores cover runs
// of consecutive entries.  A factor entry's offset is a sum of parts (bit
// extraction is linear over disjoint bit sets): the lane's m or n part once
// per launch, the block part once per block, the term part from per-bit
// weights.  LDS rows are padded by 16 entries so that the four term groups
// of an MFMA operand read fall in different banks.
constexpr int kMmbMaxM = 7, kMmbMaxN = 6, kMmbPad = 16, kMmbBig = 4;
// entries a thread stages per block: 2^(J + MB) / 256 <= 2^(4 + 7 - 8) of
// A', 2^(J + NB) / 256 <= 2^(4 + 6 - 8) of B'
constexpr int kMmbStageA = 8, kMmbStageB = 4;

struct MmbFactor {
  const float2* src;
  int64_t gs;        // elements between slices (0: input tensor)
  uint32_t sm;       // input slice mask
  int32_t rk;
  uint32_t mk;       // mask over X
  uint32_t kw[4];    // index weight of summed bit t (0: not held)
};

struct MmbLaunch {
  float2* out;
  MmbFactor big[kMmbBig];  // factors holding block bits: NA of A', then NB of B'
  MmbFactor kf[kMaxOps];   // the others
  int32_t n_kf;
  int32_t prec;            // QBE_PREC_*: FP32 or split-BF16 MFMAs
  uint32_t bm, bn;         // block bits of A' and B'
  uint32_t rest;           // the other result bits (fixed per block)
  int32_t r, MB, NB, rest_bits;
  int64_t s0, n_blocks;
};

__device__ __forceinline__ uint32_t lowest_bits(uint32_t m, int n) {
  uint32_t r = 0;
  for (int i = 0; i < n && m; ++i) {
    r |= m & (~m + 1u);
    m &= m - 1u;
  }
  return r;
}

// First entry of factor f for slice g (slice sl) and block bits xt.
__device__ __forceinline__ const float2* mmb_base(const MmbFactor& f, int64_t g, uint32_t sl, uint32_t xt) {
  return f.src + g * f.gs + (f.gs ? 0 : (int64_t)pext32(sl, f.sm) << f.rk) + pext32(xt, f.mk);
}

template <int J>
__device__ __forceinline__ uint32_t mmb_term(const MmbFactor& f, int k) {
  uint32_t o = 0;
#pragma unroll
  for (int t = 0; t < J; ++t) o += ((k >> t) & 1) ? f.kw[t] : 0u;
  return o;
}

template <int J, int NA, int NBF>
__global__ __launch_bounds__(kBlock) void mmb_kernel(MmbLaunch a) {
  constexpr int T = 1 << J;  // terms
  __shared__ float2 As[T * ((1 << kMmbMaxM) + kMmbPad)];
  __shared__ float2 Bs[T * ((1 << kMmbMaxN) + kMmbPad)];
  __shared__ float2 Ts[kBlock / 64][256];
  __shared__ float2 Ks[T];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int Mn = 1 << a.MB, Nn = 1 << a.NB;
  const int sa = Mn + kMmbPad, sb = Nn + kMmbPad;
  const uint32_t mt = lowest_bits(a.bm, 4), nt = lowest_bits(a.bn, 4), tt = mt | nt;
  const uint32_t mh = a.bm & ~mt, nh = a.bn & ~nt;
  const int row = lane & 15, grp = lane >> 4;
  // MFMA result layout: the lane holds tile rows 4 grp + i of column row;
  // pw: their positions in the tile's result order; qo: the result offset
  // of tile position lane + 64 j
  uint32_t pw[4], qo[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    pw[i] = pext32(pdep32((uint32_t)(4 * grp + i), mt) | pdep32((uint32_t)row, nt), tt);
    qo[i] = pdep32((uint32_t)(lane + 64 * i), tt);
  }
  // staging: thread tid takes entries tid + 256 j of A' (m = entry mod Mn,
  // k = entry / Mn; Mn divides 256, so m is fixed) and likewise of B'
  const int ma = tid & (Mn - 1), ka0 = tid >> a.MB, kas = kBlock >> a.MB;
  const int nb = tid & (Nn - 1), kb0 = tid >> a.NB, kbs = kBlock >> a.NB;
  uint32_t part[NA + NBF];
#pragma unroll
  for (int i = 0; i < NA + NBF; ++i)
    part[i] = pext32(i >= NA ? pdep32((uint32_t)nb, a.bn) : pdep32((uint32_t)ma, a.bm), a.big[i].mk);
  const int tiles_m = Mn >> 4, n_tiles = tiles_m * (Nn >> 4);
  // step i takes block number + i * grid, so that neighbouring blocks, whose
  // factor entries share cache lines, run at the same time behind one L2
  for (int64_t blk = xcd_major_block(); blk < a.n_blocks; blk += gridDim.x) {
    const int64_t g = blk >> a.rest_bits;
    const uint32_t xt = pdep32((uint32_t)(blk & ((int64_t(1) << a.rest_bits) - 1)), a.rest);
    const uint32_t sl = (uint32_t)(a.s0 + g);
    // the big factors' loads first, every entry's at once
    float2 wa[NA][kMmbStageA];
    float2 wb[NBF][kMmbStageB];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const float2* bi = mmb_base(a.big[i], g, sl, xt);
#pragma unroll
      for (int j = 0; j < kMmbStageA; ++j) {
        const int k = ka0 + j * kas;
        wa[i][j] = k < T ? bi[part[i] + mmb_term<J>(a.big[i], k)] : make_float2(1.f, 0.f);
      }
    }
#pragma unroll
    for (int i = 0; i < NBF; ++i) {
      const float2* bi = mmb_base(a.big[NA + i], g, sl, xt);
#pragma unroll
      for (int j = 0; j < kMmbStageB; ++j) {
        const int k = kb0 + j * kbs;
        wb[i][j] = k < T ? bi[part[NA + i] + mmb_term<J>(a.big[NA + i], k)] : make_float2(1.f, 0.f);
      }
    }
    __syncthreads();  // the previous block's reads of As, Bs, Ks are done
    if (tid < T) {
      float2 v = make_float2(1.f, 0.f);
      for (int i = 0; i < a.n_kf; ++i) v = cmul(v, mmb_base(a.kf[i], g, sl, xt)[mmb_term<J>(a.kf[i], tid)]);
      Ks[tid] = v;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kMmbStageA; ++j) {
      const int k = ka0 + j * kas;
      if (k < T) {
        float2 v = Ks[k];
#pragma unroll
        for (int i = 0; i < NA; ++i) v = cmul(v, wa[i][j]);
        As[k * sa + ma] = v;
      }
    }
#pragma unroll
    for (int j = 0; j < kMmbStageB; ++j) {
      const int k = kb0 + j * kbs;
      if (k < T) {
        float2 v = make_float2(1.f, 0.f);
#pragma unroll
        for (int i = 0; i < NBF; ++i) v = cmul(v, wb[i][j]);
        Bs[k * sb + nb] = v;
      }
    }
    __syncthreads();
    float2* const ob = a.out + (g << a.r) + xt;
    for (int t = wv; t < n_tiles; t += kBlock / 64) {
      const int tm = t % tiles_m, tn = t / tiles_m;
      floatx4 cre = {0.f, 0.f, 0.f, 0.f}, cim = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < T; kb += 4) {
        const float2 av = As[(kb + grp) * sa + tm * 16 + row];
        const float2 bv = Bs[(kb + grp) * sb + tn * 16 + row];
        if (a.prec == QBE_PREC_FP32) {
          cre = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv.x, cre, 0, 0, 0);
          cre = __builtin_amdgcn_mfma_f32_16x16x4f32(-av.y, bv.y, cre, 0, 0, 0);
          cim = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv.y, cim, 0, 0, 0);
          cim = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bv.x, cim, 0, 0, 0);
        } else {
          cre = mfma_split(av.x, bv.x, cre, a.prec);
          cre = mfma_split(-av.y, bv.y, cre, a.prec);
          cim = mfma_split(av.x, bv.y, cim, a.prec);
          cim = mfma_split(av.y, bv.x, cim, a.prec);
        }
      }
      // one wave's LDS accesses complete in order: the buffer needs no barrier
#pragma unroll
      for (int i = 0; i < 4; ++i) Ts[wv][pw[i]] = make_float2(cre[i], cim[i]);
      const uint32_t tb = pdep32((uint32_t)tm, mh) | pdep32((uint32_t)tn, nh);
      // streaming stores: the result is read only by later launches
#pragma unroll
      for (int j = 0; j < 4; ++j)
        __builtin_nontemporal_store(__builtin_bit_cast(uint64_t, Ts[wv][lane + 64 * j]),
                                    reinterpret_cast<uint64_t*>(ob + (tb | qo[j])));
    }
  }
}

// Where one slice group's scalar factors are: its rank-0 results in the
// arena and the scalar inputs in the prepared buffer.
struct ScalarSrc {
  const float2* arena;
  const float2* prep;
  const int64_t* arena_off;  // device arrays
  const int64_t* in_base;
  const uint32_t* in_smask;
  int32_t n_arena, n_in, n_free;
  int64_t G;
};

// FP64 product of one slice's scalar factors -- 2^n_free, the rank-0
// results, then the scalar inputs -- by a group of L lanes (L a power of two
// of at most 64, q the lane in the group): lane q multiplies factors q,
// q + L, ... in sequence (lane 0 starting from 2^n_free), then a binary tree
// over the group; its lane 0 returns the product.  ok = false: a lane past
// the last slice (factors of 1, nothing read).  Every lane of the group
// calls it (the tree shuffles within the group).
__device__ __forceinline__ double2 slice_product(const ScalarSrc& a, int64_t g, int64_t s, bool ok, uint32_t q,
                                                 uint32_t L) {
  double re = q == 0 ? ldexp(1.0, a.n_free) : 1.0, im = 0.0;
  const int n = ok ? a.n_arena + a.n_in : 0;
  for (int j = (int)q; j < n; j += (int)L) {
    const float2 v = j < a.n_arena
                         ? a.arena[a.arena_off[j] * a.G + g]
                         : a.prep[a.in_base[j - a.n_arena] + (int64_t)pext32((uint32_t)s, a.in_smask[j - a.n_arena])];
    const double vr = v.x, vi = v.y;
    const double nr = re * vr - im * vi;
    im = re * vi + im * vr;
    re = nr;
  }
  for (uint32_t w = 1; w < L; w <<= 1) {
    const double orr = __shfl_down(re, w, (int)L), oi = __shfl_down(im, w, (int)L);
    const double nr = re * orr - im * oi;
    im = re * oi + im * orr;
    re = nr;
  }
  return make_double2(re, im);
}

// Lanes per slice of slice_product: the factor count rounded up to a power
// of two, at most a wave.
static uint32_t scalar_lanes(int n_factors) {
  uint32_t L = 1;
  while ((int)L < n_factors && L < 64) L <<= 1;
  return L;
}

// Per-slice product of the scalar factors, in FP64: L lanes a slice, so
// that the factors of a slice are read at once.
struct FinalizeArgs {
  ScalarSrc src;
  uint32_t lanes;
  int64_t s0;
  double2* per_slice;  // indexed by g
};

__global__ __launch_bounds__(256) void finalize_kernel(FinalizeArgs a) {
  const uint32_t L = a.lanes, q = threadIdx.x % L;
  const int64_t per_block = 256 / L;
  // the bound is the same for every lane of a workgroup, so every group's
  // lanes reach its tree together
  for (int64_t base = (int64_t)blockIdx.x * per_block; base < a.src.G; base += (int64_t)gridDim.x * per_block) {
    const int64_t g = base + threadIdx.x / L;
    const bool ok = g < a.src.G;
    const double2 v = slice_product(a.src, g, a.s0 + g, ok, q, L);
    if (ok && q == 0) a.per_slice[g] = v;
  }
}

// FP64 slice product of the rank-0 results and the slice sum of every
// per-step instance of a batch, one workgroup per instance: the products as
// finalize_kernel computes them (L lanes a slice), 256 slices at a time into
// LDS; lane t adds slices t, t + 256, ... in sequence, then a binary tree
// over the 256 partials -- the order of reduce_kernel.
struct WideFinal {
  int64_t arena;            // complex64 offset of the instance's arena in the workspace
  const float2* prep;       // its prepared inputs
  const int64_t* arena_off; // its scalar tables (device)
  const int64_t* in_base;
  const uint32_t* in_smask;
  int32_t n_arena, n_in, n_free, plan;  // plan: index of its amplitude
  int64_t G;                // its slices (all run at once)
  uint32_t lanes;           // lanes per slice product
  uint32_t pad;
};

__global__ __launch_bounds__(256) void wide_final_kernel(const WideFinal* __restrict__ w, const float2* ws,
                                                         double2* __restrict__ amps) {
  __shared__ double sre[256], sim[256];
  const WideFinal& d = w[blockIdx.x];
  const ScalarSrc src{ws + d.arena, d.prep, d.arena_off, d.in_base, d.in_smask, d.n_arena, d.n_in, d.n_free, d.G};
  const uint32_t L = d.lanes, q = threadIdx.x % L, per = 256 / L;
  double sr = 0.0, si = 0.0;
  for (int64_t base = 0; base < d.G; base += 256) {
    for (uint32_t k = 0; k < L; ++k) {
      const uint32_t i = k * per + threadIdx.x / L;  // slice base + i of this chunk
      const bool ok = base + i < d.G;
      const double2 v = slice_product(src, base + i, base + i, ok, q, L);
      if (q == 0) {
        sre[i] = v.x;
        sim[i] = v.y;
      }
    }
    __syncthreads();
    if (base + threadIdx.x < d.G) {
      sr += sre[threadIdx.x];
      si += sim[threadIdx.x];
    }
    __syncthreads();
  }
  sre[threadIdx.x] = sr;
  sim[threadIdx.x] = si;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) {
      sre[threadIdx.x] += sre[threadIdx.x + k];
      sim[threadIdx.x] += sim[threadIdx.x + k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) amps[d.plan] = make_double2(sre[0], sim[0]);
}

// Sum of n FP64 complex values in a fixed order: lane t adds entries
// t, t + 256, ... in sequence, then a binary tree over the 256 partials.
__global__ __launch_bounds__(256) void reduce_kernel(const double2* __restrict__ v,
                                                     const int64_t* __restrict__ ranges,
                                                     int64_t n_single, double2* __restrict__ out) {
  __shared__ double sre[256], sim[256];
  int64_t b = 0, e = n_single;
  if (ranges) {
    b = ranges[2 * blockIdx.x];  // (begin, end) pairs, one per block
    e = ranges[2 * blockIdx.x + 1];
  }
  double re = 0.0, im = 0.0;
  for (int64_t i = b + threadIdx.x; i < e; i += 256) {
    re += v[i].x;
    im += v[i].y;
  }
  sre[threadIdx.x] = re;
  sim[threadIdx.x] = im;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sre[threadIdx.x] += sre[threadIdx.x + w];
      sim[threadIdx.x] += sim[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = make_double2(sre[0], sim[0]);
}

int dev_count(int* n) {
  QBE_HIP(hipGetDeviceCount(n));
  return QBE_OK;
}

int dev_set(int device) {
  QBE_HIP(hipSetDevice(device));
  return QBE_OK;
}

int dev_memcpy_d2h(void* dst, const void* src, size_t bytes, void* stream) {
  QBE_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, (hipStream_t)stream));
  QBE_HIP(hipStreamSynchronize((hipStream_t)stream));
  return QBE_OK;
}

static int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

int n_cus() {
  static int cached = 0;
  if (!cached) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      cached = prop.multiProcessorCount;
    if (cached <= 0) cached = 256;
  }
  return cached;
}

static int run_prep(Plan& p) {
  if (p.step_elems > 0) {
    prep_kernel<<<grid_for(p.step_elems, 256), 256, 0, 0>>>(
        (const double2*)p.d_raw, (const int32_t*)p.d_step_map, (float2*)p.d_step_in, p.step_elems);
    QBE_HIP(hipGetLastError());
  }
  if (p.fused_ok && p.fused_elems > 0) {
    prep_kernel<<<grid_for(p.fused_elems, 256), 256, 0, 0>>>(
        (const double2*)p.d_raw, (const int32_t*)p.d_fused_map, (float2*)p.d_fused_in, p.fused_elems);
    QBE_HIP(hipGetLastError());
  }
  for (const FusedSeg& sg : p.segs)
    if (sg.elems > 0) {
      prep_kernel<<<grid_for(sg.elems, 256), 256, 0, 0>>>((const double2*)p.d_raw, (const int32_t*)sg.d_map,
                                                            (float2*)sg.d_in, sg.elems);
      QBE_HIP(hipGetLastError());
    }
  QBE_HIP(hipDeviceSynchronize());
  return QBE_OK;
}

// Every device buffer a plan owns.
static std::vector<void**> plan_buffers(Plan& p) {
  std::vector<void**> all = {&p.d_raw,        &p.d_step_map,   &p.d_step_in, &p.d_fused_map, &p.d_fused_in,
                             &p.d_fused_prog, &p.d_scalar_tab, &p.d_state,   &p.d_group};
  for (FusedSeg& sg : p.segs) all.insert(all.end(), {&sg.d_map, &sg.d_in, &sg.d_prog});
  return all;
}

void dev_free_plan(Plan& p) {
  for (void** q : plan_buffers(p)) {
    if (*q) (void)hipFree(*q);
    *q = nullptr;
  }
}

void dev_forget_plan(Plan& p) {
  for (void** q : plan_buffers(p)) *q = nullptr;
}

int dmalloc(void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 256));
  if (e != hipSuccess) {
    set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? QBE_ERR_OOM : QBE_ERR_HIP;
  }
  return QBE_OK;
}

int upload(void** d, const void* h, size_t bytes) {
  int rc = dmalloc(d, bytes);
  if (rc) return rc;
  if (bytes) QBE_HIP(hipMemcpy(*d, h, bytes, hipMemcpyHostToDevice));
  return QBE_OK;
}

int dev_upload_plan(Plan& p) {
  int rc;
  if ((rc = upload(&p.d_raw, p.model.data.data(), p.model.data.size() * sizeof(double)))) return rc;
  if ((rc = upload(&p.d_step_map, p.step_map.data(), p.step_map.size() * 4))) return rc;
  if ((rc = dmalloc(&p.d_step_in, p.step_elems * 8))) return rc;
  {
    std::vector<char> tab(p.scalar_arena.size() * 8 + p.scalar_inputs_base.size() * 12 + 16);
    size_t o = 0;
    if (!p.scalar_arena.empty()) std::memcpy(tab.data() + o, p.scalar_arena.data(), p.scalar_arena.size() * 8);
    o += p.scalar_arena.size() * 8;
    if (!p.scalar_inputs_base.empty())
      std::memcpy(tab.data() + o, p.scalar_inputs_base.data(), p.scalar_inputs_base.size() * 8);
    o += p.scalar_inputs_base.size() * 8;
    if (!p.scalar_inputs_smask.empty())
      std::memcpy(tab.data() + o, p.scalar_inputs_smask.data(), p.scalar_inputs_smask.size() * 4);
    if ((rc = upload(&p.d_scalar_tab, tab.data(), tab.size()))) return rc;
  }
  if ((rc = dmalloc(&p.d_state, 256))) return rc;
  QBE_HIP(hipMemset(p.d_state, 0, 256));
  if (!p.group_steps.empty()) {
    const size_t sb = p.group_steps.size() * sizeof(GroupStep);
    std::vector<char> buf(sb + p.group_prefix.size() * 4);
    std::memcpy(buf.data(), p.group_steps.data(), sb);
    std::memcpy(buf.data() + sb, p.group_prefix.data(), p.group_prefix.size() * 4);
    if ((rc = upload(&p.d_group, buf.data(), buf.size()))) return rc;
  }
  if (p.fused_ok) {
    if ((rc = upload(&p.d_fused_map, p.fused_map.data(), p.fused_map.size() * 4))) return rc;
    if ((rc = dmalloc(&p.d_fused_in, p.fused_elems * 8))) return rc;
    if ((rc = upload(&p.d_fused_prog, p.fused_prog.data(), p.fused_prog.size() * 4))) return rc;
  }
  for (FusedSeg& sg : p.segs) {
    if ((rc = upload(&sg.d_map, sg.map.data(), sg.map.size() * 4))) return rc;
    if ((rc = dmalloc(&sg.d_in, sg.elems * 8))) return rc;
    if ((rc = upload(&sg.d_prog, sg.prog.data(), sg.prog.size() * 4))) return rc;
  }
  return run_prep(p);
}

int dev_update_data(Plan& p) {
  QBE_HIP(hipMemcpy(p.d_raw, p.model.data.data(), p.model.data.size() * sizeof(double),
                    hipMemcpyHostToDevice));
  return run_prep(p);
}

// Workspace layout of one call:
//   [0, 256)            result (double2) at 0, work counter at 64
//   [256, head)         per-slice FP64 values (16 B per slice of the call)
//   [head, ...)         per-step form only: the arena of G slices

size_t dev_workspace_min(const Plan& p, int64_t n) {
  if (p.exec == QBE_EXEC_FUSED) return ws_head(n);
  return ws_head(n) + (size_t)p.arena_per_slice * 8;
}

size_t dev_workspace_all(const Plan& p) {
  if (p.exec == QBE_EXEC_FUSED) return ws_head(p.n_slices);
  return ws_head(p.n_slices) + (size_t)p.arena_per_slice * 8 * (size_t)p.n_slices;
}

// A merged two-group launch as independent 16 x 16 tiles (mmk_kernel): the
// form for launches with more factors holding block bits, or term and factor
// counts, than mmb_kernel takes.
static int launch_mmk(const Plan& p, const StepProg& sp, const StepLaunch& a, int r, int64_t G, int64_t s0,
                      hipStream_t st, int wg_per_cu) {
  MmkLaunch m{};
  m.out = a.out;
  m.n_ops = sp.n_ops;
  m.side_b = sp.mmk_side;
  m.prec = p.precision;
  const uint32_t xmask = (1u << r) - 1u;
  uint32_t xa = 0, xb = 0;
  for (int i = 0; i < sp.n_ops; ++i) {
    m.src[i] = a.src[i];
    m.gs[i] = a.gstride[i];
    m.sm[i] = a.smask[i];
    m.rk[i] = a.rank[i];
    m.mk[i] = a.mask[i];
    ((sp.mmk_side >> i) & 1u ? xb : xa) |= a.mask[i] & xmask;
  }
  // the tile's column index is the lane's (16 consecutive lanes): give the
  // column side the group owning the lowest private result bit, so that
  // stores cover contiguous entries (the product is symmetric in A', B')
  const uint32_t priv = (xa ^ xb) & xmask;
  if (priv & xa & (~priv + 1u)) {
    m.side_b = ~m.side_b & ((1u << sp.n_ops) - 1u);
    std::swap(xa, xb);
  }
  uint32_t oa = xa & ~xb, ob = xb & ~xa;
  for (int k = 0; k < 4; ++k) {
    m.mtile |= oa & (~oa + 1u);
    oa &= oa - 1u;
    m.ntile |= ob & (~ob + 1u);
    ob &= ob - 1u;
  }
  m.rest = xmask & ~m.mtile & ~m.ntile;
  m.r = r;
  m.s0 = s0;
  m.G = G;
  m.n_tiles = G << (r - 8);
  if (wg_per_cu <= 0) wg_per_cu = sp.wg_per_cu > 0 ? sp.wg_per_cu : 8;
  const int64_t want = (m.n_tiles + 3) / 4;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)n_cus() * wg_per_cu));
#define QBE_MMK(JJ, KK)                                                       \
case JJ * 16 + KK:                                                          \
  mmk_kernel<JJ, KK><<<grid, kBlock, 0, st>>>(m);                           \
  break;
#define QBE_MMKS(JJ) \
QBE_MMK(JJ, 2) QBE_MMK(JJ, 3) QBE_MMK(JJ, 4) QBE_MMK(JJ, 5) QBE_MMK(JJ, 6) QBE_MMK(JJ, 7) QBE_MMK(JJ, 8)
  switch (sp.n_sum * 16 + sp.n_ops) {
    QBE_MMKS(2) QBE_MMKS(3) QBE_MMKS(4)
    default:
      set_error("merged MFMA launch with an unsupported summed-variable or operand count");
      return QBE_ERR_INTERNAL;
  }
#undef QBE_MMKS
#undef QBE_MMK
  QBE_HIP(hipGetLastError());
  return QBE_OK;
}

static int launch_step(const Plan& p, const StepProg& sp, float2* arena, int64_t G, int64_t s0,
                       hipStream_t st, int ept = 0, int wg_per_cu = 0) {
  StepLaunch a{};
  const bool sum_u = sp.out_rank >= 0;
  const int r = sum_u ? sp.out_rank : -sp.out_rank;
  a.out = arena + sp.out_base * G;
  a.n_ops = sp.n_ops;
  a.r = r;
  a.sum_u = sum_u ? 1 : 0;
  a.n_sum = sp.n_sum;
  a.lo = std::min(r, kLoBits);
  a.s0 = s0;
  a.G = G;
  for (int i = 0; i < sp.n_ops; ++i) {
    const StepOp& o = sp.ops[i];
    if (o.is_input) {
      a.src[i] = (const float2*)p.d_step_in + o.base;
      a.gstride[i] = 0;
      a.smask[i] = o.smask;
    } else {
      a.src[i] = arena + o.base * G;
      a.gstride[i] = int64_t(1) << o.rank;
      a.smask[i] = 0;
    }
    a.mask[i] = o.mask;
    a.rank[i] = o.rank;
  }
  if (sp.mmk) {
    // merged launch on MFMA: operand groups A' and B', whole blocks per
    // workgroup; the side with more private result bits is A' (up to 2^7
    // rows), the other B' (up to 2^6 columns)
    MmbLaunch m{};
    m.out = a.out;
    m.prec = p.precision;
    const uint32_t xmask = (1u << r) - 1u;
    uint32_t xa = 0, xb = 0;
    for (int i = 0; i < sp.n_ops; ++i) ((sp.mmk_side >> i) & 1u ? xb : xa) |= a.mask[i] & xmask;
    uint32_t pa = xa & ~xb, pb = xb & ~xa;
    uint32_t side_b = sp.mmk_side;
    if (__builtin_popcount(pb) > __builtin_popcount(pa)) {
      side_b = ~side_b & ((1u << sp.n_ops) - 1u);
      std::swap(pa, pb);
    }
    m.MB = std::min(__builtin_popcount(pa), kMmbMaxM);
    m.NB = std::min(__builtin_popcount(pb), kMmbMaxN);
    for (int k = 0; k < m.MB; ++k) {
      m.bm |= pa & (~pa + 1u);
      pa &= pa - 1u;
    }
    for (int k = 0; k < m.NB; ++k) {
      m.bn |= pb & (~pb + 1u);
      pb &= pb - 1u;
    }
    MmbFactor fa[kMmbBig], fb[kMmbBig];
    int na = 0, nbf = 0;
    for (int i = 0; i < sp.n_ops; ++i) {
      MmbFactor f{};
      f.src = a.src[i];
      f.gs = a.gstride[i];
      f.sm = a.smask[i];
      f.rk = a.rank[i];
      f.mk = a.mask[i];
      for (int t = 0; t < sp.n_sum && t < 4; ++t) {
        const uint32_t bit = 1u << (r + t);
        f.kw[t] = (a.mask[i] & bit) ? 1u << __builtin_popcount(a.mask[i] & (bit - 1u)) : 0u;
      }
      if (!(a.mask[i] & (m.bm | m.bn))) {
        m.kf[m.n_kf++] = f;
      } else if (na + nbf == kMmbBig) {
        return launch_mmk(p, sp, a, r, G, s0, st, wg_per_cu);
      } else if ((side_b >> i) & 1u) {
        fb[nbf++] = f;
      } else {
        fa[na++] = f;
      }
    }
    for (int i = 0; i < na; ++i) m.big[i] = fa[i];
    for (int i = 0; i < nbf; ++i) m.big[na + i] = fb[i];
    if (m.MB < 4 || m.NB < 4 || sp.n_sum < 2 || sp.n_sum > 4 || na < 1 || nbf < 1)
      return launch_mmk(p, sp, a, r, G, s0, st, wg_per_cu);
    m.rest = xmask & ~m.bm & ~m.bn;
    m.rest_bits = __builtin_popcount(m.rest);
    m.r = r;
    m.s0 = s0;
    m.n_blocks = G << m.rest_bits;
    if (wg_per_cu <= 0) wg_per_cu = sp.wg_per_cu > 0 ? sp.wg_per_cu : 4;
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(m.n_blocks, (int64_t)n_cus() * wg_per_cu));
#define QBE_MMB(JJ, A, B)                                                     \
  case (JJ * 4 + A) * 4 + B:                                                  \
    mmb_kernel<JJ, A, B><<<(int)grid, kBlock, 0, st>>>(m);                    \
    break;
#define QBE_MMBS(JJ) QBE_MMB(JJ, 1, 1) QBE_MMB(JJ, 1, 2) QBE_MMB(JJ, 2, 1) QBE_MMB(JJ, 2, 2) QBE_MMB(JJ, 1, 3) QBE_MMB(JJ, 3, 1)
    switch ((sp.n_sum * 4 + na) * 4 + nbf) {
      QBE_MMBS(2) QBE_MMBS(3) QBE_MMBS(4)
      default:
        set_error("merged MFMA launch with an unsupported summed-variable or factor count");
        return QBE_ERR_INTERNAL;
    }
#undef QBE_MMBS
#undef QBE_MMB
    QBE_HIP(hipGetLastError());
    return QBE_OK;
  }
  if (sp.mm_a >= 0 && sum_u && r >= 8) {
    MmLaunch m{};
    m.out = a.out;
    const int idx[2] = {sp.mm_a, sp.mm_b};
    for (int j = 0; j < 2; ++j) {
      m.src[j] = a.src[idx[j]];
      m.gs[j] = a.gstride[idx[j]];
      m.sm[j] = a.smask[idx[j]];
      m.rk[j] = a.rank[idx[j]];
      m.mk[j] = a.mask[idx[j]];
    }
    for (int i = 0; i < sp.n_ops; ++i) {
      if (i == sp.mm_a || i == sp.mm_b) continue;
      m.usrc[m.n_u] = a.src[i];
      m.ugs[m.n_u] = a.gstride[i];
      m.usm[m.n_u] = a.smask[i];
      ++m.n_u;
    }
    const uint32_t xmask = (1u << r) - 1u;
    uint32_t oa = m.mk[0] & xmask & ~m.mk[1], ob = m.mk[1] & xmask & ~m.mk[0];
    for (int k = 0; k < 4; ++k) {
      m.mtile |= oa & (~oa + 1u);
      oa &= oa - 1u;
      m.ntile |= ob & (~ob + 1u);
      ob &= ob - 1u;
    }
    m.rest = xmask & ~m.mtile & ~m.ntile;
    m.r = r;
    m.s0 = s0;
    m.G = G;
    m.n_tiles = G << (r - 8);
    if (wg_per_cu <= 0) wg_per_cu = sp.wg_per_cu > 0 ? sp.wg_per_cu : 8;
    const int64_t want = (m.n_tiles + 3) / 4;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)n_cus() * wg_per_cu));
    if (p.precision == QBE_PREC_BF16X3)
      mm_kernel<QBE_PREC_BF16X3><<<grid, kBlock, 0, st>>>(m);
    else if (p.precision == QBE_PREC_BF16X6)
      mm_kernel<QBE_PREC_BF16X6><<<grid, kBlock, 0, st>>>(m);
    else
      mm_kernel<QBE_PREC_FP32><<<grid, kBlock, 0, st>>>(m);
    QBE_HIP(hipGetLastError());
    return QBE_OK;
  }
  // VALU kernels: operands holding x bit 0 first (the paired kernels read
  // them with 16-byte loads and need that order at compile time), so that
  // every tile shape, paired or not, multiplies in the same order; within
  // each part, merged launches put the operands that hold both of a trip's
  // summed bits first, so that the four term products can start from
  // operand 0's entries (LEAD) instead of the constant 1 -- the same bits,
  // as 1 * v is exact
  const uint32_t trip_bits = sp.n_sum > 1 ? ((1u << sp.sum_bit[0]) | (1u << sp.sum_bit[1])) << r : 0u;
  auto holds_trip = [&](int i) { return trip_bits != 0 && (a.mask[i] & trip_bits) == trip_bits; };
  {
    StepLaunch b = a;
    int at = 0;
    for (int pass = 0; pass < 4; ++pass)
      for (int i = 0; i < sp.n_ops; ++i) {
        if (((a.mask[i] & 1u) != 0) != (pass < 2) || holds_trip(i) != (pass % 2 == 0)) continue;
        b.src[at] = a.src[i];
        b.gstride[at] = a.gstride[i];
        b.mask[at] = a.mask[i];
        b.smask[at] = a.smask[i];
        b.rank[at] = a.rank[i];
        ++at;
      }
    a = b;
  }
  const bool lead = holds_trip(0);
  if (sp.n_sum > 1) {
    if (sp.n_sum > 4) {
      set_error("merged launch with more than four summed variables");
      return QBE_ERR_INTERNAL;
    }
    const uint32_t xmask = (1u << r) - 1u;
    for (int i = 0; i < sp.n_ops; ++i) {
      if (a.rank[i] > kMergedMaxRank) {
        set_error("merged launch operand above 2^28 entries");
        return QBE_ERR_INTERNAL;
      }
      // summed variables sit above the operand's x bits, in union order;
      // the kernel's bit b of u is union bit r + sum_bit[b]
      const uint32_t um = a.mask[i] >> r;
      const int xc = __builtin_popcount(a.mask[i] & xmask);
      a.uhold[i] = 0;
      for (int b = 0; b < sp.n_sum; ++b) a.uhold[i] |= ((um >> sp.sum_bit[b]) & 1u) << b;
      for (int b = 0; b < 4; ++b) {
        a.uw[i][b] = 0;
        if (b >= sp.n_sum || !((um >> sp.sum_bit[b]) & 1u)) continue;
        // the operand's summed bits sit above its x bits in union order:
        // union bit r + sum_bit[b] is its bit xc + (held summed bits below it)
        const int below = __builtin_popcount(um & ((1u << sp.sum_bit[b]) - 1u));
        a.uw[i][b] = (1u << (xc + below)) * 8u;
      }
    }
  }
  if (wg_per_cu <= 0) wg_per_cu = sp.wg_per_cu > 0 ? sp.wg_per_cu : 16;
  if (r < kLoBits) {
    // several whole slices per tile
    a.n_tiles = (G + (kBlock >> r) - 1) / (kBlock >> r);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(a.n_tiles, (int64_t)n_cus() * wg_per_cu));
#define QBE_SMALL(KK)                                                         \
  case KK:                                                                    \
    if (sp.n_sum > 1)                                                         \
      msum_small_kernel<KK><<<grid, kBlock, 0, st>>>(a);                      \
    else                                                                      \
      step_small_kernel<KK><<<grid, kBlock, 0, st>>>(a);                      \
    break;
    switch (sp.n_ops) {
      QBE_SMALL(1) QBE_SMALL(2) QBE_SMALL(3) QBE_SMALL(4) QBE_SMALL(5) QBE_SMALL(6) QBE_SMALL(7)
      QBE_SMALL(8)
      default:
        set_error("per-step launch with an unsupported operand count");
        return QBE_ERR_INTERNAL;
    }
#undef QBE_SMALL
    QBE_HIP(hipGetLastError());
    return QBE_OK;
  }
  const int hib = r - kLoBits;
  a.n_tiles = G << hib;
  // untuned: large merged launches (32 tiles per compute unit or more) in
  // the paired form (the faster one on every such launch measured), others
  // one tile per thread
  if (ept <= 0) ept = sp.ept > 0 ? sp.ept : (sp.n_sum > 1 && a.n_tiles >= 32 * (int64_t)n_cus() ? 2 : 1);
  // a super-tile's EPT tiles share the slice: EPT divides 2^hib
  while (ept > 1 && (int64_t(1) << hib) % ept != 0) ept >>= 1;
  if (ept == 2) {
    // paired tiles (msum_pair_kernel, step_pair_kernel): x bit 0 tells them
    // apart, the lane supplies bits 1-8; the operands holding bit 0 go first
    const StepLaunch& b = a;
    int np = 0;
    for (int i = 0; i < sp.n_ops; ++i) np += (a.mask[i] & 1u) ? 1 : 0;
    const int64_t want = a.n_tiles / 2;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)n_cus() * wg_per_cu));
#define QBE_PAIR(KK, NN)                                                      \
  case KK * 16 + NN:                                                          \
    if (sp.n_sum > 1 && lead)                                                 \
      msum_pair_kernel<KK, NN, true><<<grid, kBlock, 0, st>>>(b);             \
    else if (sp.n_sum > 1)                                                    \
      msum_pair_kernel<KK, NN, false><<<grid, kBlock, 0, st>>>(b);            \
    else                                                                      \
      step_pair_kernel<KK, NN><<<grid, kBlock, 0, st>>>(b);                   \
    break;
    switch (sp.n_ops * 16 + np) {
      QBE_PAIR(1, 0) QBE_PAIR(1, 1)
      QBE_PAIR(2, 0) QBE_PAIR(2, 1) QBE_PAIR(2, 2) QBE_PAIR(3, 0) QBE_PAIR(3, 1) QBE_PAIR(3, 2) QBE_PAIR(3, 3)
      QBE_PAIR(4, 0) QBE_PAIR(4, 1) QBE_PAIR(4, 2) QBE_PAIR(4, 3) QBE_PAIR(4, 4) QBE_PAIR(5, 0) QBE_PAIR(5, 1)
      QBE_PAIR(5, 2) QBE_PAIR(5, 3) QBE_PAIR(5, 4) QBE_PAIR(5, 5) QBE_PAIR(6, 0) QBE_PAIR(6, 1) QBE_PAIR(6, 2)
      QBE_PAIR(6, 3) QBE_PAIR(6, 4) QBE_PAIR(6, 5) QBE_PAIR(6, 6) QBE_PAIR(7, 0) QBE_PAIR(7, 1) QBE_PAIR(7, 2)
      QBE_PAIR(7, 3) QBE_PAIR(7, 4) QBE_PAIR(7, 5) QBE_PAIR(7, 6) QBE_PAIR(7, 7) QBE_PAIR(8, 0) QBE_PAIR(8, 1)
      QBE_PAIR(8, 2) QBE_PAIR(8, 3) QBE_PAIR(8, 4) QBE_PAIR(8, 5) QBE_PAIR(8, 6) QBE_PAIR(8, 7) QBE_PAIR(8, 8)
      default:
        set_error("paired merged launch with an unsupported operand count");
        return QBE_ERR_INTERNAL;
    }
#undef QBE_PAIR
    QBE_HIP(hipGetLastError());
    return QBE_OK;
  }
  const int64_t want = a.n_tiles / ept;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)n_cus() * wg_per_cu));
#define QBE_CASE(KK, EE)                                                      \
  case KK * 16 + EE:                                                          \
    if (sp.n_sum > 1 && lead)                                                 \
      msum_kernel<KK, EE, true><<<grid, kBlock, 0, st>>>(a);                  \
    else if (sp.n_sum > 1)                                                    \
      msum_kernel<KK, EE, false><<<grid, kBlock, 0, st>>>(a);                 \
    else                                                                      \
      step_kernel<KK, EE><<<grid, kBlock, 0, st>>>(a);                        \
    break;
#define QBE_KS(KK) QBE_CASE(KK, 1) QBE_CASE(KK, 2) QBE_CASE(KK, 4)
  switch (sp.n_ops * 16 + ept) {
    QBE_KS(1) QBE_KS(2) QBE_KS(3) QBE_KS(4) QBE_KS(5) QBE_KS(6) QBE_KS(7) QBE_KS(8)
    default:
      set_error("per-step launch with an unsupported operand count or tile factor");
      return QBE_ERR_INTERNAL;
  }
#undef QBE_KS
#undef QBE_CASE
  QBE_HIP(hipGetLastError());
  return QBE_OK;
}

static int launch_group(const Plan& p, int g, float2* arena, int64_t G, int64_t s0, hipStream_t st) {
  GroupArgs a{};
  const int32_t first = p.group_first[g];
  a.steps = (const GroupStep*)p.d_group + first;
  a.prefix = (const uint32_t*)((const char*)p.d_group + p.group_steps.size() * sizeof(GroupStep)) + first + g;
  a.count = p.group_first[g + 1] - first;
  a.sb = p.group_sb;
  a.arena = arena;
  a.step_in = (const float2*)p.d_step_in;
  a.G = G;
  a.s0 = s0;
  a.n_blocks = (G + a.sb - 1) / a.sb;
  const int64_t units = (int64_t)p.group_prefix[first + g + a.count] * a.n_blocks;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(units, (int64_t)n_cus() * 16));
  group_kernel<<<grid, kBlock, 0, st>>>(a);
  QBE_HIP(hipGetLastError());
  return QBE_OK;
}

// Autotuner: times every large per-step launch of the plan on the device in
// each candidate tile shape (tiles per thread x workgroups per CU) and keeps
// the fastest; an FP32 merged launch on MFMA is also timed on the VALU
// kernels, and the faster form kept.  Runs the plan's own schedule on a
// slice group of G slices, so the data it reads are the intermediates of
// the group's slices.
int dev_autotune(Plan& p, void* stream, void* ws, size_t ws_bytes, int64_t min_elems) {
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = p.n_slices;
  if (ws_bytes < dev_workspace_min(p, 1)) {
    set_error("workspace too small");
    return QBE_ERR_MEM_CAP;
  }
  const int64_t per_slice_bytes = p.arena_per_slice * 8;
  const int64_t G = std::min<int64_t>(n, (int64_t)((ws_bytes - ws_head(1)) / per_slice_bytes));
  float2* arena = (float2*)((char*)ws + ws_head(1));
  hipEvent_t e0, e1;
  QBE_HIP(hipEventCreate(&e0));
  QBE_HIP(hipEventCreate(&e1));
  const int epts[] = {1, 2, 4};
  const int wgs[] = {4, 8, 16, 32};
  int rc = QBE_OK;
  // time of one configuration: the mean of two runs after a warm-up run
  auto time_config = [&](StepProg& sp, int e, int w, float& total) {
    total = 0.f;
    for (int rep = 0; rep < 3 && rc == QBE_OK; ++rep) {
      if (hipEventRecord(e0, st) != hipSuccess) rc = QBE_ERR_HIP;
      if (rc == QBE_OK) rc = launch_step(p, sp, arena, G, 0, st, e, w);
      if (rc == QBE_OK && hipEventRecord(e1, st) != hipSuccess) rc = QBE_ERR_HIP;
      if (rc == QBE_OK && hipEventSynchronize(e1) != hipSuccess) rc = QBE_ERR_HIP;
      float ms = 0.f;
      if (rc == QBE_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = QBE_ERR_HIP;
      if (rep > 0) total += ms;  // first run warms caches and code
    }
  };
  for (StepProg& sp : p.steps) {
    const int r = sp.out_rank >= 0 ? sp.out_rank : -sp.out_rank;
    if ((G << r) >= min_elems) {
      // a merged launch on MFMA in FP32 against the same launch on the
      // VALU kernels (both FP32 products: the same sum, other tiles); the
      // split-BF16 plans keep their MFMA form
      float mfma_ms = 1e30f;
      int mfma_w = 0;
      const bool both = sp.mmk && p.precision == QBE_PREC_FP32;
      if (both) {
        for (int w : wgs) {
          float total = 0.f;
          time_config(sp, 1, w, total);
          if (rc != QBE_OK) break;
          if (total < mfma_ms) {
            mfma_ms = total;
            mfma_w = w;
          }
        }
        sp.mmk = 0;
      }
      float best = 1e30f;
      int be = 1, bw = 16;
      for (int e : epts)
        for (int w : wgs) {
          float total = 0.f;
          time_config(sp, e, w, total);
          if (rc != QBE_OK) break;
          if (total < best) {
            best = total;
            be = e;
            bw = w;
          }
        }
      sp.ept = be;
      sp.wg_per_cu = bw;
      if (both && mfma_ms <= best) {
        sp.mmk = 1;
        sp.ept = 1;
        sp.wg_per_cu = mfma_w;
      }
    } else {
      // launch-bound: the first configuration is as good as any
      rc = launch_step(p, sp, arena, G, 0, st);
    }
    if (rc != QBE_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == QBE_ERR_HIP) set_error("autotune: HIP event call failed");
  return rc;
}

// One launch of the execution order for slices s0 .. s0 + G - 1.
static int launch_item(const Plan& p, const LaunchItem& li, float2* arena, int64_t G, int64_t s0, hipStream_t st) {
  if (li.seg >= 0) return seg_launch(p.segs[li.seg], arena, G, s0, st);
  if (li.group >= 0) return launch_group(p, li.group, arena, G, s0, st);
  return launch_step(p, p.steps[li.step], arena, G, s0, st);
}

// Per-slice FP64 product of the rank-0 results of slices s0 .. s0 + G - 1.
static int finalize_group(const Plan& p, float2* arena, double2* per_slice, int64_t G, int64_t s0,
                          hipStream_t st) {
  const int64_t* t_arena = (const int64_t*)p.d_scalar_tab;
  const int64_t* t_inb = t_arena + p.scalar_arena.size();
  const uint32_t* t_ism = (const uint32_t*)(t_inb + p.scalar_inputs_base.size());
  FinalizeArgs fa{};
  fa.src = ScalarSrc{arena,
                     (const float2*)p.d_step_in,
                     t_arena,
                     t_inb,
                     t_ism,
                     (int32_t)p.scalar_arena.size(),
                     (int32_t)p.scalar_inputs_base.size(),
                     (int32_t)p.sched.free_vars.size(),
                     G};
  fa.lanes = scalar_lanes(fa.src.n_arena + fa.src.n_in);
  fa.s0 = s0;
  fa.per_slice = per_slice;
  finalize_kernel<<<grid_for(G * fa.lanes, 256), 256, 0, st>>>(fa);
  QBE_HIP(hipGetLastError());
  return QBE_OK;
}

int dev_contract(const Plan& p, void* stream, void* ws, size_t ws_bytes, int64_t s_begin,
                 int64_t s_end, double* d_partial_out, double* d_per_slice) {
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = s_end - s_begin;
  char* w = (char*)ws;
  double2* per_slice = d_per_slice ? (double2*)d_per_slice : (double2*)(w + 256);
  if (ws_bytes < dev_workspace_min(p, n)) {
    set_error("workspace too small");
    return QBE_ERR_MEM_CAP;
  }
  if (p.exec == QBE_EXEC_FUSED) {
    bool reduced = false;
    int rc = fused_contract(p, st, s_begin, n, per_slice, (double2*)d_partial_out, &reduced);
    if (rc) return rc;
    if (reduced) return QBE_OK;
  } else {
    const int64_t per_slice_bytes = p.arena_per_slice * 8;
    const int64_t G = std::min<int64_t>(n, (int64_t)((ws_bytes - ws_head(n)) / per_slice_bytes));
    float2* arena = (float2*)(w + ws_head(n));
    for (int64_t g0 = 0; g0 < n; g0 += G) {
      const int64_t Gc = std::min<int64_t>(G, n - g0);
      for (const LaunchItem& li : p.launch_order) {
        int rc = launch_item(p, li, arena, Gc, s_begin + g0, st);
        if (rc) return rc;
      }
      int rc = finalize_group(p, arena, per_slice + g0, Gc, s_begin + g0, st);
      if (rc) return rc;
    }
  }
  return launch_reduce(per_slice, nullptr, n, (double2*)d_partial_out, 1, st);
}

// Per-launch timing of a per-step plan: the contraction of all slices at
// once (one slice group), with a HIP event recorded on the stream before the
// first launch and after every launch of the execution order, then the
// finalize and reduce launches.  ms_out[i] = time between events i and
// i + 1.
int dev_profile(const Plan& p, void* stream, void* ws, size_t ws_bytes, float* ms_out, int cap, int* n_out) {
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = p.n_slices;
  const int n_order = (int)p.launch_order.size();
  const int items = n_order + 2;
  *n_out = items;
  if (p.exec != QBE_EXEC_PER_STEP) {
    set_error("per-launch timing is for per-step plans (a fused plan is one launch)");
    return QBE_ERR_INVALID_ARG;
  }
  if (ws_bytes < dev_workspace_all(p)) {
    set_error("per-launch timing runs all slices at once: workspace below stats.ws_bytes_all_slices");
    return QBE_ERR_MEM_CAP;
  }
  if (cap < items) {
    set_error("ms_out holds fewer entries than the plan's launches");
    return QBE_ERR_MEM_CAP;
  }
  char* w = (char*)ws;
  double2* per_slice = (double2*)(w + 256);
  float2* arena = (float2*)(w + ws_head(n));
  std::vector<hipEvent_t> ev(items + 1, nullptr);
  int rc = QBE_OK;
  for (auto& e : ev)
    if (rc == QBE_OK && hipEventCreate(&e) != hipSuccess) rc = QBE_ERR_HIP;
  if (rc == QBE_OK && hipEventRecord(ev[0], st) != hipSuccess) rc = QBE_ERR_HIP;
  for (int i = 0; i < items && rc == QBE_OK; ++i) {
    if (i < n_order) {
      rc = launch_item(p, p.launch_order[i], arena, n, 0, st);
    } else if (i == items - 2) {
      rc = finalize_group(p, arena, per_slice, n, 0, st);
    } else {
      rc = launch_reduce(per_slice, nullptr, n, (double2*)w, 1, st);
    }
    if (rc == QBE_OK && hipEventRecord(ev[i + 1], st) != hipSuccess) rc = QBE_ERR_HIP;
  }
  if (rc == QBE_OK && hipEventSynchronize(ev[items]) != hipSuccess) rc = QBE_ERR_HIP;
  for (int i = 0; i < items && rc == QBE_OK; ++i)
    if (hipEventElapsedTime(&ms_out[i], ev[i], ev[i + 1]) != hipSuccess) rc = QBE_ERR_HIP;
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  if (rc == QBE_ERR_HIP) set_error("per-launch timing: a HIP event call failed");
  return rc;
}

// ------------------------------------------------- allocation-free entry --
//
// qbe_contract_static runs dev_contract on this fixed array instead of a
// caller's workspace.  Each device holds its own copy from the library's
// first use on it until the process ends; host code reaches it only through
// the address hipGetSymbolAddress reports on that device (the array's name
// is a host-side stand-in).  Nothing in it needs clearing: every kernel of
// the contraction writes a region before any kernel reads it.
static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};
}  // namespace

int dev_static_scratch_init(int device) {
  if (device < 0 || device >= kScratchDevices) {
    set_error("device index beyond the static scratch table");
    return QBE_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return QBE_OK;
  int cur = -1;
  QBE_HIP(hipGetDevice(&cur));
  if (cur != device) {
    set_error("static scratch set-up needs its device current");
    return QBE_ERR_INTERNAL;
  }
  void* ptr = nullptr;
  QBE_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) {
    set_error("hipGetSymbolAddress returned no address for the static scratch");
    return QBE_ERR_HIP;
  }
  g_scratch_ptr[device] = ptr;
  return QBE_OK;
}

int dev_contract_static(const Plan& p, void* stream, double* d_amp_out) {
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (p.device >= 0 && p.device < kScratchDevices) ptr = g_scratch_ptr[p.device];
  }
  if (!ptr) {
    set_error("static scratch is not set up on the plan's device");
    return QBE_ERR_INTERNAL;
  }
  const size_t need = dev_workspace_min(p, p.n_slices);
  if (need > kStaticScratchBytes) {
    set_error("plan needs a workspace of " + std::to_string(need) + " bytes, above the static scratch's " +
              std::to_string(kStaticScratchBytes));
    return QBE_ERR_MEM_CAP;
  }
  return dev_contract(p, stream, ptr, kStaticScratchBytes, 0, p.n_slices, d_amp_out, nullptr);
}

int launch_reduce(const double2* v, const int64_t* ranges, int64_t n_single, double2* out, int n_blocks,
                  hipStream_t st) {
  reduce_kernel<<<n_blocks, 256, 0, st>>>(v, ranges, n_single, out);
  QBE_HIP(hipGetLastError());
  return QBE_OK;
}

// ------------------------------------------------------------------ batch --
//
// The per-step instances of a batch run together, level by level: each has
// its own region of the workspace (all its slices at once), a level's
// single launches of every instance go first, then one launch of all their
// grouped small steps of that level; then each instance's finalize and sum.

// Largest log2(slices x result entries) of a step that the batch runs in
// its level's group launch although the plan launches it alone.
constexpr int kWideGroupMaxLog2 = 22;
// Side streams over which a level's launches of per-step batch instances
// are dealt (with the caller's stream: four, the process's hardware queues).
constexpr size_t kWideSideStreams = 3;

int step_batch_build(Batch& b) {
  b.wide_off.clear();
  b.wide_order.clear();
  b.wide_steps.clear();
  b.wide_first.assign(1, 0);
  b.wide_prefix.clear();
  size_t off = 0;
  int n_lv = 0;
  for (int i : b.wide) {
    const Plan& p = *b.plans[i];
    b.wide_off.push_back(off);
    off += (dev_workspace_all(p) + 255) / 256 * 256;
    for (int lv : p.step_level) n_lv = std::max(n_lv, lv + 1);
  }
  b.wide_ws = off;
  b.wide_level.clear();
  for (int L = 0; L < n_lv; ++L) {
    const int32_t lv0 = (int32_t)b.wide_order.size();
    std::vector<WideGroupStep> grp;
    for (size_t q = 0; q < b.wide.size(); ++q) {
      const Plan& p = *b.plans[b.wide[q]];
      const int64_t arena = (int64_t)((b.wide_off[q] + ws_head(p.n_slices)) / sizeof(float2));
      auto add = [&](const GroupStep& gs) {
        WideGroupStep d{};
        d.s = gs;
        d.step_in = p.d_step_in;
        d.arena = arena;
        d.G = p.n_slices;
        d.sb = p.group_sb;
        d.tiles = (int32_t)((((int64_t)p.group_sb << d.s.r) + kBlock - 1) / kBlock);
        grp.push_back(d);
      };
      for (const LaunchItem& li : p.launch_order) {
        if (li.group < 0) {
          if (p.step_level[li.step] != L) continue;
          // a step the plan launches alone: grouped here when it is small
          // enough for the generic kernel across instances
          const StepProg& sp = p.steps[li.step];
          const int r = sp.out_rank >= 0 ? sp.out_rank : -sp.out_rank;
          if (groupable(sp) && (p.n_slices << r) <= (int64_t(1) << kWideGroupMaxLog2))
            add(group_step_of(sp, li.step));
          else
            b.wide_order.push_back(WideItem{(int32_t)q, li.step, -1});
          continue;
        }
        const int f = p.group_first[li.group], e = p.group_first[li.group + 1];
        if (p.step_level[p.group_steps[f].step] != L) continue;
        for (int j = f; j < e; ++j) {
          WideGroupStep d{};
          d.s = p.group_steps[j];
          d.step_in = p.d_step_in;
          d.arena = arena;
          d.G = p.n_slices;
          d.sb = p.group_sb;
          d.tiles = (int32_t)((((int64_t)p.group_sb << d.s.r) + kBlock - 1) / kBlock);
          grp.push_back(d);
        }
      }
    }
    if (!grp.empty()) {
      const int g = (int)b.wide_first.size() - 1;
      uint64_t units = 0;
      b.wide_prefix.push_back(0);
      for (const WideGroupStep& d : grp) {
        units += (uint64_t)d.tiles * (uint64_t)((d.G + d.sb - 1) / d.sb);
        b.wide_prefix.push_back(units);
        b.wide_steps.push_back(d);
      }
      b.wide_first.push_back((int32_t)b.wide_steps.size());
      b.wide_order.push_back(WideItem{-1, -1, g});
    }
    if ((int32_t)b.wide_order.size() > lv0) b.wide_level.push_back(lv0);
  }
  b.wide_level.push_back((int32_t)b.wide_order.size());
  if (!b.wide.empty()) {
    std::vector<WideFinal> fin;
    for (size_t q = 0; q < b.wide.size(); ++q) {
      const Plan& p = *b.plans[b.wide[q]];
      WideFinal f{};
      f.arena = (int64_t)((b.wide_off[q] + ws_head(p.n_slices)) / sizeof(float2));
      f.prep = (const float2*)p.d_step_in;
      f.arena_off = (const int64_t*)p.d_scalar_tab;
      f.in_base = f.arena_off + p.scalar_arena.size();
      f.in_smask = (const uint32_t*)(f.in_base + p.scalar_inputs_base.size());
      f.n_arena = (int32_t)p.scalar_arena.size();
      f.n_in = (int32_t)p.scalar_inputs_base.size();
      f.n_free = (int32_t)p.sched.free_vars.size();
      f.plan = b.wide[q];
      f.G = p.n_slices;
      f.lanes = scalar_lanes(f.n_arena + f.n_in);
      fin.push_back(f);
    }
    int rc = upload(&b.d_wide_final, fin.data(), fin.size() * sizeof(WideFinal));
    if (rc) return rc;
  }
  if (!b.wide_steps.empty()) {
    const size_t sb = b.wide_steps.size() * sizeof(WideGroupStep);
    std::vector<char> buf(sb + b.wide_prefix.size() * 8);
    std::memcpy(buf.data(), b.wide_steps.data(), sb);
    std::memcpy(buf.data() + sb, b.wide_prefix.data(), b.wide_prefix.size() * 8);
    int rc = upload(&b.d_wide, buf.data(), buf.size());
    if (rc) return rc;
  }
  size_t widest = 0;
  for (size_t v = 0; v + 1 < b.wide_level.size(); ++v)
    widest = std::max<size_t>(widest, (size_t)(b.wide_level[v + 1] - b.wide_level[v]));
  const size_t n_side = std::min<size_t>(kWideSideStreams, widest > 0 ? widest - 1 : 0);
  if (n_side > 0) {
    hipEvent_t e = nullptr;
    QBE_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    b.ev_fork = e;
    for (size_t i = 0; i < n_side; ++i) {
      hipStream_t s = nullptr;
      QBE_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      b.side.push_back(s);
      QBE_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      b.ev_join.push_back(e);
    }
  }
  return QBE_OK;
}

static int launch_wide_group(const Batch& b, int g, char* wide_ws, hipStream_t st) {
  WideArgs a{};
  const int32_t first = b.wide_first[g];
  a.steps = (const WideGroupStep*)b.d_wide + first;
  a.prefix = (const uint64_t*)((const char*)b.d_wide + b.wide_steps.size() * sizeof(WideGroupStep)) + first + g;
  a.count = b.wide_first[g + 1] - first;
  a.ws = (float2*)wide_ws;
  const uint64_t units = b.wide_prefix[first + g + a.count];
  const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>(units, (uint64_t)n_cus() * 16));
  wide_group_kernel<<<grid, kBlock, 0, st>>>(a);
  QBE_HIP(hipGetLastError());
  return QBE_OK;
}

// [0, head): counter and per-item values of the fused launch; then one
// region per per-step instance (result, per-slice values, arena).
size_t dev_batch_workspace(const Batch& b) { return ws_head(b.n_items) + b.wide_ws; }

int dev_batch_contract(const Batch& b, void* stream, void* ws, size_t ws_bytes, double* d_amps) {
  hipStream_t st = (hipStream_t)stream;
  if (ws_bytes < dev_batch_workspace(b)) {
    set_error("workspace too small");
    return QBE_ERR_MEM_CAP;
  }
  char* w = (char*)ws;
  if (b.n_items > 0) {
    int rc = fused_batch_launch(b, st, (double2*)(w + 256), (double2*)d_amps);
    if (rc) return rc;
  }
  char* wide_ws = w + ws_head(b.n_items);
  // levels are dealt over the side streams when the call is captured into a
  // graph (branches replayed without host work); issued directly, the
  // events per level would cost more host time than the overlap saves
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  QBE_HIP(hipStreamIsCapturing(st, &cap));
  const size_t n_side = cap == hipStreamCaptureStatusActive ? b.side.size() : 0;
  for (size_t v = 0; v + 1 < b.wide_level.size(); ++v) {
    // a level's launches have no memory hazard with one another: deal them
    // over the caller's stream and up to n side streams, which start after
    // everything the caller's stream holds and rejoin it at the level's end
    const int32_t i0 = b.wide_level[v], i1 = b.wide_level[v + 1];
    const int n = (int)std::min<size_t>(n_side, (size_t)(i1 - i0 - 1));
    if (n > 0) {
      QBE_HIP(hipEventRecord((hipEvent_t)b.ev_fork, st));
      for (int s = 0; s < n; ++s) QBE_HIP(hipStreamWaitEvent((hipStream_t)b.side[s], (hipEvent_t)b.ev_fork, 0));
    }
    for (int32_t j = i0; j < i1; ++j) {
      const int k = (j - i0) % (n + 1);
      hipStream_t sj = k == 0 ? st : (hipStream_t)b.side[k - 1];
      const WideItem& it = b.wide_order[j];
      int rc;
      if (it.group < 0) {
        const Plan& p = *b.plans[b.wide[it.plan]];
        float2* arena = (float2*)(wide_ws + b.wide_off[it.plan] + ws_head(p.n_slices));
        rc = launch_step(p, p.steps[it.step], arena, p.n_slices, 0, sj);
      } else {
        rc = launch_wide_group(b, it.group, wide_ws, sj);
      }
      if (rc) return rc;
    }
    for (int s = 0; s < n; ++s) {
      QBE_HIP(hipEventRecord((hipEvent_t)b.ev_join[s], (hipStream_t)b.side[s]));
      QBE_HIP(hipStreamWaitEvent(st, (hipEvent_t)b.ev_join[s], 0));
    }
  }
  if (!b.wide.empty()) {
    wide_final_kernel<<<(unsigned)b.wide.size(), 256, 0, st>>>((const WideFinal*)b.d_wide_final,
                                                              (const float2*)wide_ws, (double2*)d_amps);
    QBE_HIP(hipGetLastError());
  }
  return QBE_OK;
}

}  // namespace qbe
