// Device side of sliced bucket elimination on gfx950 (CDNA4).
//
// Kernels
//   prep_kernel      complex128 model entries -> complex64 prepared inputs
//                    through a gather map (layout chosen by the planner).
//   step_kernel      one bucket for a group of slices (per-step form): every
//                    thread produces one result entry per tile as
//                    sum_u prod_i T_i[pext(X, mask_i)], X = (u << r) | x.
//                    The low 8 bits of x come from the lane, so the result
//                    is written with fully coalesced stores and every operand
//                    holding those low variables is read coalesced; the
//                    operand-index bits of the higher part of x are
//                    extracted once per tile.  HBM-bound (about 2 flop/B).
//   fused_kernel     whole slices in one workgroup (fused form): inputs and
//                    every intermediate live in LDS, the buckets run level by
//                    level (all buckets whose operands are ready at once), a
//                    barrier between levels.  A persistent grid pulls
//                    (instance, slice) work items from an atomic counter.
//   finalize_kernel  per-slice product of the rank-0 results, in FP64.
//   reduce_kernel    deterministic FP64 sum of per-slice values (Eq. 4).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>

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
  int32_t lo;      // min(r, kLoBits)
  int64_t s0;      // first slice of the group
  int64_t G;       // slices in the group
  int64_t n_tiles;
};

template <int K>
__global__ __launch_bounds__(kBlock) void step_kernel(StepLaunch a) {
  const int tid = threadIdx.x;
  const int r = a.r, lo = a.lo;
  const uint32_t lomask = (1u << lo) - 1u;
  const uint32_t x_lo = (uint32_t)tid & lomask;
  const int64_t g_sub = tid >> lo;  // r < kLoBits: several slices per tile
  const int64_t spt = (int64_t)(kBlock >> lo);
  const int hib = r - lo;
  uint32_t lo_part[K], u_part[K], hi_mask[K];
  int lo_cnt[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const uint32_t m = a.mask[i];
    lo_part[i] = pext32(x_lo, m & lomask);
    lo_cnt[i] = __builtin_popcount(m & lomask);
    hi_mask[i] = (m >> lo) & ((1u << hib) - 1u);
    u_part[i] = (a.sum_u && ((m >> r) & 1u)) ? (1u << (a.rank[i] - 1)) : 0u;
  }
  for (int64_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
    int64_t g;
    uint32_t x_hi;
    if (hib > 0) {
      g = tile >> hib;
      x_hi = (uint32_t)(tile & ((int64_t(1) << hib) - 1));
    } else {
      g = tile * spt + g_sub;
      x_hi = 0;
      if (g >= a.G) continue;
    }
    const int64_t s = a.s0 + g;
    const float2* p[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      int64_t base;
      if (a.gstride[i] != 0)
        base = g * a.gstride[i];
      else
        base = (int64_t)pext32((uint32_t)s, a.smask[i]) << a.rank[i];
      base += (int64_t)(pext32(x_hi, hi_mask[i]) << lo_cnt[i]) + lo_part[i];
      p[i] = a.src[i] + base;
    }
    float2 acc = p[0][0];
#pragma unroll
    for (int i = 1; i < K; ++i) acc = cmul(acc, p[i][0]);
    if (a.sum_u) {
      float2 t = p[0][u_part[0]];
#pragma unroll
      for (int i = 1; i < K; ++i) t = cmul(t, p[i][u_part[i]]);
      acc.x += t.x;
      acc.y += t.y;
    }
    a.out[(g << r) + ((int64_t)x_hi << lo) + x_lo] = acc;
  }
}

// Per-slice product of the scalar factors, in FP64.
struct FinalizeArgs {
  const float2* arena;
  const float2* prep;
  const int64_t* arena_off;   // device arrays
  const int64_t* in_base;
  const uint32_t* in_smask;
  int32_t n_arena, n_in, n_free;
  int64_t G, s0;
  double2* per_slice;  // indexed by g
};

__global__ void finalize_kernel(FinalizeArgs a) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < a.G;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = a.s0 + g;
    double re = (double)(int64_t(1) << a.n_free), im = 0.0;
    for (int j = 0; j < a.n_arena; ++j) {
      const float2 v = a.arena[a.arena_off[j] * a.G + g];
      const double vr = v.x, vi = v.y;
      const double nr = re * vr - im * vi;
      im = re * vi + im * vr;
      re = nr;
    }
    for (int j = 0; j < a.n_in; ++j) {
      const float2 v = a.prep[a.in_base[j] + (int64_t)pext32((uint32_t)s, a.in_smask[j])];
      const double vr = v.x, vi = v.y;
      const double nr = re * vr - im * vi;
      im = re * vi + im * vr;
      re = nr;
    }
    a.per_slice[g] = make_double2(re, im);
  }
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

// -------------------------------------------------------------- fused form --

struct FusedItem {
  uint32_t plan;   // index into the plan tables
  uint32_t pad;
  int64_t slice;
};

struct FusedArgs {
  const uint32_t* prog0;              // one-plan mode (items == nullptr)
  const float2* prep0;
  const uint32_t* const* progs;       // batch mode: per plan
  const float2* const* preps;
  const FusedItem* items;             // batch mode: the work items
  int64_t s_begin;                    // one-plan mode: slice of item 0
  int64_t n_items;
  uint32_t* counter;                  // work counter, zeroed before launch
  double2* out;                       // per item
};

__global__ void reset_counter_kernel(uint32_t* c) { *c = 0u; }

__global__ __launch_bounds__(kBlock) void fused_kernel(FusedArgs a) {
  extern __shared__ uint32_t lds[];
  __shared__ int64_t s_item;
  __shared__ uint32_t s_plan;
  const int tid = threadIdx.x;
  if (tid == 0) s_plan = 0xFFFFFFFFu;
  for (;;) {
    __syncthreads();
    if (tid == 0) {
      const uint32_t it = atomicAdd(a.counter, 1u);
      s_item = (int64_t)it < a.n_items ? (int64_t)it : -1;
    }
    __syncthreads();
    const int64_t item = s_item;
    if (item < 0) break;
    uint32_t plan = 0;
    int64_t slice = a.s_begin + item;
    const uint32_t* prog = a.prog0;
    const float2* prep = a.prep0;
    if (a.items) {
      const FusedItem wi = a.items[item];
      plan = wi.plan;
      slice = wi.slice;
      prog = a.progs[plan];
      prep = a.preps[plan];
    }
    if (plan != s_plan) {  // s_plan is read by every lane: the branch is uniform
      const uint32_t words = prog[FH_WORDS];
      for (uint32_t i = tid; i < words; i += kBlock) lds[i] = prog[i];
      __syncthreads();
      if (tid == 0) s_plan = plan;
    }
    const uint32_t words = lds[FH_WORDS];
    const uint32_t n_levels = lds[FH_LEVELS];
    const uint32_t n_steps = lds[FH_STEPS];
    const uint32_t n_ops = lds[FH_OPS];
    const uint32_t n_scal = lds[FH_SCALARS];
    const uint32_t inv = lds[FH_INV_ELEMS], dep = lds[FH_DEP_ELEMS];
    const uint32_t* lvl_begin = lds + kHdr;
    const uint32_t* lvl_elems = lvl_begin + n_levels + 1;
    const uint32_t* stepw = lvl_elems + n_levels;
    const uint32_t* opw = stepw + 2 * n_steps;
    const uint32_t* scal = opw + n_ops;
    float2* data = reinterpret_cast<float2*>(lds + words);
    const float2* dsrc = prep + lds[FH_DEP_SRC] + slice * (int64_t)dep;
    for (uint32_t i = tid; i < inv; i += kBlock) data[i] = prep[i];
    for (uint32_t i = tid; i < dep; i += kBlock) data[inv + i] = dsrc[i];
    __syncthreads();
    for (uint32_t l = 0; l < n_levels; ++l) {
      const uint32_t E = lvl_elems[l];
      const uint32_t b0 = lvl_begin[l], b1 = lvl_begin[l + 1];
      for (uint32_t f = tid; f < E; f += kBlock) {
        uint32_t lo = b0, hi = b1 - 1;
        while (lo < hi) {
          const uint32_t mid = (lo + hi + 1) >> 1;
          if ((stepw[2 * mid + 1] >> 16) <= f)
            lo = mid;
          else
            hi = mid - 1;
        }
        const uint32_t w0 = stepw[2 * lo], w1 = stepw[2 * lo + 1];
        const uint32_t out_off = w0 & 0xFFFFu, r = (w0 >> 16) & 31u, nops = w0 >> 21;
        const uint32_t op0 = w1 & 0xFFFFu, x = f - (w1 >> 16);
        float2 a0 = make_float2(1.f, 0.f), a1 = make_float2(1.f, 0.f);
        for (uint32_t i = 0; i < nops; ++i) {
          const uint32_t ow = opw[op0 + i];
          const uint32_t mask = ow >> 16;
          const float2* t = data + (ow & 0xFFFFu);
          const uint32_t idx = pext32(x, mask);
          a0 = cmul(a0, t[idx]);
          const uint32_t up = ((mask >> r) & 1u) ? (1u << (__builtin_popcount(mask) - 1)) : 0u;
          a1 = cmul(a1, t[idx + up]);
        }
        data[out_off + x] = make_float2(a0.x + a1.x, a0.y + a1.y);
      }
      __syncthreads();
    }
    if (tid == 0) {
      double re = (double)(1u << lds[FH_FREE]), im = 0.0;
      for (uint32_t j = 0; j < n_scal; ++j) {
        const float2 v = data[scal[j]];
        const double vr = v.x, vi = v.y;
        const double nr = re * vr - im * vi;
        im = re * vi + im * vr;
        re = nr;
      }
      a.out[item] = make_double2(re, im);
    }
  }
}

// ================================================================== host ==

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

static int n_cus() {
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
  QBE_HIP(hipDeviceSynchronize());
  return QBE_OK;
}

void dev_free_plan(Plan& p) {
  void** ptrs[] = {&p.d_raw,      &p.d_step_map,   &p.d_step_in,   &p.d_fused_map,
                   &p.d_fused_in, &p.d_fused_prog, &p.d_scalar_tab};
  for (void** q : ptrs) {
    if (*q) (void)hipFree(*q);
    *q = nullptr;
  }
}

static int dmalloc(void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 256));
  if (e != hipSuccess) {
    set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? QBE_ERR_OOM : QBE_ERR_HIP;
  }
  return QBE_OK;
}

static int upload(void** d, const void* h, size_t bytes) {
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
  if (p.fused_ok) {
    if ((rc = upload(&p.d_fused_map, p.fused_map.data(), p.fused_map.size() * 4))) return rc;
    if ((rc = dmalloc(&p.d_fused_in, p.fused_elems * 8))) return rc;
    if ((rc = upload(&p.d_fused_prog, p.fused_prog.data(), p.fused_prog.size() * 4))) return rc;
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
static size_t ws_head(int64_t n) { return 256 + ((size_t)n * 16 + 255) / 256 * 256; }

size_t dev_workspace_min(const Plan& p, int64_t n) {
  if (p.exec == QBE_EXEC_FUSED) return ws_head(n);
  return ws_head(n) + (size_t)p.arena_per_slice * 8;
}

size_t dev_workspace_all(const Plan& p) {
  if (p.exec == QBE_EXEC_FUSED) return ws_head(p.n_slices);
  return ws_head(p.n_slices) + (size_t)p.arena_per_slice * 8 * (size_t)p.n_slices;
}

static int launch_step(const Plan& p, const StepProg& sp, float2* arena, int64_t G, int64_t s0,
                       hipStream_t st) {
  StepLaunch a{};
  const bool sum_u = sp.out_rank >= 0;
  const int r = sum_u ? sp.out_rank : -sp.out_rank;
  a.out = arena + sp.out_base * G;
  a.n_ops = sp.n_ops;
  a.r = r;
  a.sum_u = sum_u ? 1 : 0;
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
  const int hib = r - a.lo;
  a.n_tiles = hib > 0 ? (G << hib) : (G + (kBlock >> a.lo) - 1) / (kBlock >> a.lo);
  const int grid = (int)std::min<int64_t>(a.n_tiles, (int64_t)n_cus() * 16);
  switch (sp.n_ops) {
#define QBE_CASE(K) \
  case K: step_kernel<K><<<grid, kBlock, 0, st>>>(a); break;
    QBE_CASE(1) QBE_CASE(2) QBE_CASE(3) QBE_CASE(4) QBE_CASE(5) QBE_CASE(6) QBE_CASE(7) QBE_CASE(8)
#undef QBE_CASE
    default:
      set_error("bucket with an unsupported operand count");
      return QBE_ERR_INTERNAL;
  }
  QBE_HIP(hipGetLastError());
  return QBE_OK;
}

static int fused_grid(int lds_bytes, int64_t n_items) {
  const int per_cu = std::max(1, std::min(8, (160 * 1024) / std::max(lds_bytes, 1)));
  return (int)std::max<int64_t>(1, std::min<int64_t>(n_items, (int64_t)n_cus() * per_cu));
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
    uint32_t* counter = (uint32_t*)(w + 64);
    reset_counter_kernel<<<1, 1, 0, st>>>(counter);
    QBE_HIP(hipGetLastError());
    FusedArgs a{};
    a.prog0 = (const uint32_t*)p.d_fused_prog;
    a.prep0 = (const float2*)p.d_fused_in;
    a.s_begin = s_begin;
    a.n_items = n;
    a.counter = counter;
    a.out = per_slice;
    fused_kernel<<<fused_grid(p.fused_lds_bytes, n), kBlock, p.fused_lds_bytes, st>>>(a);
    QBE_HIP(hipGetLastError());
  } else {
    const int64_t per_slice_bytes = p.arena_per_slice * 8;
    const int64_t G = std::min<int64_t>(n, (int64_t)((ws_bytes - ws_head(n)) / per_slice_bytes));
    float2* arena = (float2*)(w + ws_head(n));
    const int64_t* t_arena = (const int64_t*)p.d_scalar_tab;
    const int64_t* t_inb = t_arena + p.scalar_arena.size();
    const uint32_t* t_ism = (const uint32_t*)(t_inb + p.scalar_inputs_base.size());
    for (int64_t g0 = 0; g0 < n; g0 += G) {
      const int64_t Gc = std::min<int64_t>(G, n - g0);
      for (const StepProg& sp : p.steps) {
        int rc = launch_step(p, sp, arena, Gc, s_begin + g0, st);
        if (rc) return rc;
      }
      FinalizeArgs fa{};
      fa.arena = arena;
      fa.prep = (const float2*)p.d_step_in;
      fa.arena_off = t_arena;
      fa.in_base = t_inb;
      fa.in_smask = t_ism;
      fa.n_arena = (int)p.scalar_arena.size();
      fa.n_in = (int)p.scalar_inputs_base.size();
      fa.n_free = (int)p.sched.free_vars.size();
      fa.G = Gc;
      fa.s0 = s_begin + g0;
      fa.per_slice = per_slice + g0;
      finalize_kernel<<<grid_for(Gc, 256), 256, 0, st>>>(fa);
      QBE_HIP(hipGetLastError());
    }
  }
  reduce_kernel<<<1, 256, 0, st>>>(per_slice, nullptr, n, (double2*)d_partial_out);
  QBE_HIP(hipGetLastError());
  return QBE_OK;
}

// ------------------------------------------------------------------ batch --

int dev_batch_build(Batch& b) {
  const int np = (int)b.plans.size();
  std::vector<const uint32_t*> progs(np, nullptr);
  std::vector<const float2*> preps(np, nullptr);
  std::vector<int> idx;
  b.lds_bytes = 0;
  b.wide.clear();
  b.wide_ws = 0;
  for (int i = 0; i < np; ++i) {
    const Plan& p = *b.plans[i];
    if (p.exec != QBE_EXEC_FUSED) {
      b.wide.push_back(i);
      b.wide_ws = std::max(b.wide_ws, dev_workspace_all(p));
      continue;
    }
    progs[i] = (const uint32_t*)p.d_fused_prog;
    preps[i] = (const float2*)p.d_fused_in;
    b.lds_bytes = std::max(b.lds_bytes, p.fused_lds_bytes);
    idx.push_back(i);
  }
  // biggest work items first, so the tail of the persistent grid is short
  std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) {
    return b.plans[x]->cost.flops > b.plans[y]->cost.flops;
  });
  std::vector<FusedItem> items;
  std::vector<int64_t> ranges(2 * np, 0);
  for (int i : idx) {
    ranges[2 * i] = (int64_t)items.size();
    for (int64_t s = 0; s < b.plans[i]->n_slices; ++s) items.push_back(FusedItem{(uint32_t)i, 0u, s});
    ranges[2 * i + 1] = (int64_t)items.size();
  }
  b.n_items = (int64_t)items.size();
  b.item_begin = ranges;
  int rc;
  if ((rc = upload(&b.d_progs, progs.data(), np * sizeof(void*)))) return rc;
  if ((rc = upload(&b.d_preps, preps.data(), np * sizeof(void*)))) return rc;
  if ((rc = upload(&b.d_items, items.data(), items.size() * sizeof(FusedItem)))) return rc;
  if ((rc = upload(&b.d_ranges, ranges.data(), ranges.size() * 8))) return rc;
  return QBE_OK;
}

void dev_batch_free(Batch& b) {
  void** ptrs[] = {&b.d_progs, &b.d_preps, &b.d_items, &b.d_ranges};
  for (void** q : ptrs) {
    if (*q) (void)hipFree(*q);
    *q = nullptr;
  }
}

// [0, head): counter and per-item values of the fused launch; then the
// workspace of the widest per-step instance (they run one after another).
size_t dev_batch_workspace(const Batch& b) { return ws_head(b.n_items) + b.wide_ws; }

int dev_batch_contract(const Batch& b, void* stream, void* ws, size_t ws_bytes, double* d_amps) {
  hipStream_t st = (hipStream_t)stream;
  if (ws_bytes < dev_batch_workspace(b)) {
    set_error("workspace too small");
    return QBE_ERR_MEM_CAP;
  }
  char* w = (char*)ws;
  if (b.n_items > 0) {
    uint32_t* counter = (uint32_t*)(w + 64);
    double2* per_item = (double2*)(w + 256);
    reset_counter_kernel<<<1, 1, 0, st>>>(counter);
    QBE_HIP(hipGetLastError());
    FusedArgs a{};
    a.progs = (const uint32_t* const*)b.d_progs;
    a.preps = (const float2* const*)b.d_preps;
    a.items = (const FusedItem*)b.d_items;
    a.n_items = b.n_items;
    a.counter = counter;
    a.out = per_item;
    fused_kernel<<<fused_grid(b.lds_bytes, b.n_items), kBlock, b.lds_bytes, st>>>(a);
    QBE_HIP(hipGetLastError());
    // one reduction block per plan; blocks of per-step plans see an empty range
    reduce_kernel<<<(unsigned)b.plans.size(), 256, 0, st>>>(per_item, (const int64_t*)b.d_ranges, 0,
                                                             (double2*)d_amps);
    QBE_HIP(hipGetLastError());
  }
  char* wide_ws = w + ws_head(b.n_items);
  for (int i : b.wide) {
    const Plan& p = *b.plans[i];
    int rc = dev_contract(p, stream, wide_ws, b.wide_ws, 0, p.n_slices, d_amps + 2 * i, nullptr);
    if (rc) return rc;
  }
  return QBE_OK;
}

}  // namespace qbe
