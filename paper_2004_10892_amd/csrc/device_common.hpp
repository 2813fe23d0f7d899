// Pieces shared by the per-step device code (device.hip) and the fused
// executor (fused.hip).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "qbe_internal.hpp"
#include "../../include/qbe.h"

namespace qbe {

#define QBE_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) {                                                             \
      set_error(std::string(#call) + ": " + hipGetErrorString(e_));                     \
      return QBE_ERR_HIP;                                                               \
    }                                                                                   \
  } while (0)

// ----------------------------------------------------------- small helpers --

__device__ __forceinline__ uint32_t pext32(uint32_t x, uint32_t m) {
  uint32_t r = 0;
  int k = 0;
  while (m) {
    const int b = __builtin_ctz(m);
    r |= ((x >> b) & 1u) << k;
    ++k;
    m &= m - 1;
  }
  return r;
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

// ------------------------------------------------ host helpers (device.hip) --

int n_cus();
int dmalloc(void** p, size_t bytes);
int upload(void** d, const void* h, size_t bytes);
// Workspace head: 256 bytes of counters, then n per-slice (or per-item)
// complex128 values, rounded up to 256 bytes.
inline size_t ws_head(int64_t n) { return 256 + ((size_t)n * 16 + 255) / 256 * 256; }
// Deterministic FP64 sums (reduce_kernel): one block per (begin, end) pair of
// ranges, or one block over v[0, n_single) when ranges is null.
int launch_reduce(const double2* v, const int64_t* ranges, int64_t n_single, double2* out, int n_blocks,
                  hipStream_t st);

// Launch order and grouped steps of a batch's per-step instances.
int step_batch_build(Batch& b);

// -------------------------------------------------- fused form (fused.hip) --

// Slices [s_begin, s_begin + n) of a fused plan: one persistent launch.
// *reduced: the launch also summed the slices into amps (else the caller
// reduces per_slice).
int fused_contract(const Plan& p, hipStream_t st, int64_t s_begin, int64_t n, double2* per_slice,
                   double2* amps, bool* reduced);
// A fused segment of a per-step plan for slices s0 .. s0 + G - 1: its
// imports come from and its exports go to the slice group's arena.
int seg_launch(const FusedSeg& sg, float2* arena, int64_t G, int64_t s0, hipStream_t st);
// The fused instances of a batch in one launch (per_item: one value per work
// item), with their per-plan sums in amps.
int fused_batch_launch(const Batch& b, hipStream_t st, double2* per_item, double2* amps);

}  // namespace qbe
