// Fused form of sliced bucket elimination on gfx950 (CDNA4): whole slices
// in one workgroup.  Inputs and every intermediate live in LDS, the buckets
// run level by level (all nodes whose operands are ready at once), a barrier
// between levels; a persistent grid pulls (instance, slice) work items from
// an atomic counter, and the last workgroup of a plan sums its slices in
// FP64 (Eq. 4).
#include "device_common.hpp"

namespace qbe {

// -------------------------------------------------------------- fused form --

// The header words a workgroup needs, passed with the launch (one-plan mode)
// or with every work item (batch mode) so that no device-memory round trip
// precedes the LDS fill.
struct FusedMeta {
  uint32_t lds_tab, levels, scalars, scalar_off, free_vars, inv, dep, dep_src, bytes, exports, imports, pad;
  uint32_t lv0[4], lv1[4];  // the first two level-table entries
};

struct FusedItem {
  const uint32_t* prog;  // the item's plan: program
  const float2* prep;    //   and prepared inputs
  FusedMeta meta;
  int64_t slice;
  uint32_t plan;         // index into the batch's plans
  uint32_t pad;
};

struct FusedArgs {
  const uint32_t* prog0;              // one-plan mode (items == nullptr)
  const float2* prep0;
  FusedMeta meta0;
  const FusedItem* items;             // batch mode: the work items
  const int64_t* ranges;              // batch mode: (begin, end) items per plan
  int64_t s_begin;                    // one-plan mode: slice of item 0
  int64_t n_items;
  uint32_t* state;                    // [0] work counter, [1] exits, [2 + p] items done
  double2* out;                       // per item
  double2* amps;                      // per plan: the slice sum (when reduce_here)
  int32_t reduce_here;                // 1: the last workgroup of a plan sums its items
  uint32_t lds_ctl;                   // LDS byte offset of the workgroup's control words
  // segment mode (one-plan mode with a segment program): item g first
  // copies each import row's result (LDS element, rank, arena offset) from
  // arena[offset * G + (g << rank) + i] into LDS, and instead of the scalar
  // product copies each export row's result to its arena place
  float2* arena;
  int64_t G;
};

static FusedMeta fused_meta(const Plan& p) {
  const std::vector<uint32_t>& w = p.fused_prog;
  FusedMeta m{(uint32_t)fused_table_lds(w[FH_DATA_ELEMS]), w[FH_LEVELS], w[FH_SCALARS], w[FH_SCALAR_OFF],
              w[FH_FREE], w[FH_INV_ELEMS], w[FH_DEP_ELEMS], w[FH_DEP_SRC], w[FH_BYTE_OFFSETS], w[FH_EXPORTS],
              w[FH_IMPORTS], 0, {}, {}};
  for (int i = 0; i < 4; ++i) {
    m.lv0[i] = w[kHdr + i];
    m.lv1[i] = w[kHdr + 4 + i];
  }
  return m;
}

// LDS bytes after the data for the workgroup's control words.
constexpr int kFusedCtlBytes = 16;
// Lanes of the in-kernel slice sum: the width of reduce_kernel's tree, so
// that both sum in one order.
constexpr int kFusedReduceLanes = 256;
// Record rows (16-byte groups of words) a lane reads per level, two levels
// ahead: one half-record of up to kSplitOpsMax operands, or a whole record
// of up to kWholeOpsMax.
constexpr int kRecRows = kFusedTailRows;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) uint32_t* gu32p;
typedef const __attribute__((address_space(1))) u32x4* gu32x4p;

// The same pointer typed as device (global) memory, so that loads through it
// are global loads (waited on by their own counter) rather than flat ones.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* as_global(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}

// A pointer every lane holds the same value of, moved to scalar registers.
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }

// One lane's record words for a level.
struct Rec {
  u32x4 r[kRecRows];
};

__device__ __forceinline__ uint32_t word(const Rec& c, int i) { return c.r[i >> 2][i & 3]; }

// Reads kRecRows rows at word w (16-byte aligned; the program's zero tail
// keeps every such read inside it).  A 32-bit byte offset from a uniform
// base, so that the loads take the base from scalar registers.
__device__ __forceinline__ void load_rec(gu32p prog, uint32_t w, Rec& c) {
  typedef const __attribute__((address_space(1))) char* gcp;
  const gu32x4p q = reinterpret_cast<gu32x4p>(reinterpret_cast<gcp>(prog) + (w << 2));
#pragma unroll
  for (int i = 0; i < kRecRows; ++i) c.r[i] = q[i];
}

// Levels whose E entries x 2^lgT terms fit the workgroup give each term
// record its own lane; larger ones (two terms only) give each lane both.
__device__ __forceinline__ bool split_level(uint32_t E, uint32_t lgT) { return (E << lgT) <= (uint32_t)kFusedBlock; }

// First word this lane reads for a level (base, E, R, lgT); lanes past the
// level's end read its last record, so that every lane reads valid words.
__device__ __forceinline__ uint32_t rec_word(uint32_t base, uint32_t E, uint32_t R, uint32_t lgT, uint32_t tid) {
  if (E == 0) return base;
  return split_level(E, lgT) ? base + min(tid, (E << lgT) - 1) * 4 * R : base + min(tid, E - 1) * 8 * R;
}

// The fused kernel has no static LDS, so its dynamic LDS (the tensor
// entries) starts at LDS address 0 and a record offset is an address (byte
// offsets) or an element index (element offsets).
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) f32x2* lds_v2p;
__device__ __forceinline__ float2 lds_entry(uint32_t byte_off) {
  const f32x2 v = *(lds_v2p)(size_t)byte_off;
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void lds_store(uint32_t byte_off, float2 v) {
  *(lds_v2p)(size_t)byte_off = f32x2{v.x, v.y};
}

// LDS byte address of 16-bit slot j of the words w[w0..].
template <bool kBytes>
__device__ __forceinline__ uint32_t slot(uint32_t w, int j) {
  if (kBytes) return (j & 1) ? w >> 16 : w & 0xFFFFu;
  return (j & 1) ? (w >> 13) & 0x7FFF8u : (w << 3) & 0x7FFF8u;
}
// Slot j of a record held in registers, from word w0 on: 16-bit slots
// (element indices or LDS byte addresses), or the 32-bit LDS byte
// addresses of a wide level (flag W: at most three factors, the same
// 16-byte rows, nothing to unpack).
enum { kSlotElem = 0, kSlotBytes = 1, kSlotWide = 2 };
template <int kMode>
__device__ __forceinline__ uint32_t rec_slot(const Rec& c, int w0, int j) {
  if (kMode == kSlotWide) return word(c, w0 + j);
  return slot<kMode == kSlotBytes>(word(c, w0 + (j >> 1)), j);
}

// Product of N complex values as a balanced tree (short dependent chain).
template <int N>
__device__ __forceinline__ float2 tree_prod(float2 (&v)[N]) {
#pragma unroll
  for (int s = 1; s < N; s <<= 1)
#pragma unroll
    for (int i = 0; i + s < N; i += 2 * s) v[i] = cmul(v[i], v[i + s]);
  return v[0];
}

// Sum of a value over lane groups by DPP: pairs (quad permutation
// [1, 0, 3, 2]), quads ([2, 3, 0, 1]) and eights (half-row mirror).
template <int kCtrl>
__device__ __forceinline__ float2 dpp_add(float2 v) {
  const float x = __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v.x), kCtrl, 0xF, 0xF, false));
  const float y = __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v.y), kCtrl, 0xF, 0xF, false));
  return make_float2(v.x + x, v.y + y);
}

// Split level: lane tid holds term record tid (term tid & (T - 1) of entry
// tid >> lgT); the T lanes of an entry add their products and the first
// writes the result.  Every lane runs the same code (the DPP partners must
// be active); only the writes are guarded.
template <int K, int kMode>
__device__ __forceinline__ void level_split(const Rec& c, uint32_t E, uint32_t lgT, uint32_t tid) {
  float2 v[K];
#pragma unroll
  for (int i = 0; i < K; ++i) v[i] = lds_entry(rec_slot<kMode>(c, 0, 1 + i));
  __builtin_amdgcn_sched_barrier(0);  // every read in flight before the first product
  float2 p = dpp_add<0xB1>(tree_prod<K>(v));
  if (lgT >= 2) p = dpp_add<0x4E>(p);
  if (lgT >= 3) p = dpp_add<0x141>(p);
  if ((tid & ((1u << lgT) - 1)) == 0 && tid < (E << lgT)) lds_store(rec_slot<kMode>(c, 0, 0), p);
}

// Whole-record level (half-records of one row): lane tid holds record tid;
// records past the first kFusedBlock are read here.
template <int K, int kMode>
__device__ __forceinline__ float2 record_value(const Rec& c) {
  float2 x[K], y[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    x[i] = lds_entry(rec_slot<kMode>(c, 0, 1 + i));
    y[i] = lds_entry(rec_slot<kMode>(c, 4, 1 + i));
  }
  __builtin_amdgcn_sched_barrier(0);  // every read in flight before the first product
  return cadd(tree_prod<K>(x), tree_prod<K>(y));
}

template <int K, int kMode>
__device__ __forceinline__ void level_whole(gu32p prog, const Rec& c, uint32_t base, uint32_t E, uint32_t tid) {
  const float2 v = record_value<K, kMode>(c);
  if (tid < E) lds_store(rec_slot<kMode>(c, 0, 0), v);
  for (uint32_t f = tid + kFusedBlock; f < E; f += kFusedBlock) {
    Rec d;
    load_rec(prog, base + f * 8, d);
    lds_store(rec_slot<kMode>(d, 0, 0), record_value<K, kMode>(d));
  }
}

// Records larger than a lane's registers hold: slot by slot from memory,
// all terms of an entry in one lane.
template <bool kBytes>
__device__ __forceinline__ void level_long(gu32p prog, uint32_t base, uint32_t E, uint32_t R, uint32_t lgT,
                                           uint32_t K, uint32_t tid) {
  for (uint32_t f = tid; f < E; f += kFusedBlock) {
    const gu32p rec0 = prog + base + (f << lgT) * 4 * R;
    float2 acc = make_float2(0.f, 0.f);
    for (uint32_t t = 0; t < (1u << lgT); ++t) {
      const gu32p rec = rec0 + t * 4 * R;
      float2 a = make_float2(1.f, 0.f);
      for (uint32_t i = 1; i <= K; ++i) a = cmul(a, lds_entry(slot<kBytes>(rec[i >> 1], i)));
      acc = cadd(acc, a);
    }
    lds_store(slot<kBytes>(rec0[0], 0), acc);
  }
}

// One level: t is its table entry (base, E, R | lgT << 16, K) and c this
// lane's record words, read two levels earlier; the records of the level two
// ahead (entry tn) are read into pf here, before any of this level's work.
template <bool kBytes>
__device__ __forceinline__ void level_step(gu32p prog, const u32x4& t, const u32x4& tn, const Rec& c, Rec& pf,
                                           uint32_t tid) {
  const uint32_t ntz = uni(tn.z);
  load_rec(prog, rec_word(uni(tn.x), uni(tn.y), ntz & 0xFFFFu, (ntz >> 16) & 0xFFu, tid), pf);
  const uint32_t base = uni(t.x), E = uni(t.y), tz = uni(t.z), K = uni(t.w) & 0xFFFFu;
  const uint32_t R = tz & 0xFFFFu, lgT = (tz >> 16) & 0xFFu;
  constexpr int kMode = kBytes ? kSlotBytes : kSlotElem;
  if ((tz >> 24) & kLevelWide) {
    // at most three factors, one row a term, split or whole (host-checked)
    if (split_level(E, lgT)) {
      switch (K) {
        case 1: level_split<1, kSlotWide>(c, E, lgT, tid); break;
        case 2: level_split<2, kSlotWide>(c, E, lgT, tid); break;
        case 3: level_split<3, kSlotWide>(c, E, lgT, tid); break;
        default: break;
      }
    } else {
      switch (K) {
        case 1: level_whole<1, kSlotWide>(prog, c, base, E, tid); break;
        case 2: level_whole<2, kSlotWide>(prog, c, base, E, tid); break;
        case 3: level_whole<3, kSlotWide>(prog, c, base, E, tid); break;
        default: break;
      }
    }
  } else if (split_level(E, lgT) && K <= (uint32_t)kSplitOpsMax) {
    switch (K) {
#define QBE_SPLIT(KK) \
  case KK: level_split<KK, kMode>(c, E, lgT, tid); break;
      QBE_SPLIT(1) QBE_SPLIT(2) QBE_SPLIT(3) QBE_SPLIT(4) QBE_SPLIT(5) QBE_SPLIT(6) QBE_SPLIT(7) QBE_SPLIT(8)
      QBE_SPLIT(9) QBE_SPLIT(10) QBE_SPLIT(11) QBE_SPLIT(12) QBE_SPLIT(13) QBE_SPLIT(14) QBE_SPLIT(15)
#undef QBE_SPLIT
      default: break;
    }
  } else if (lgT == 1 && K <= (uint32_t)kWholeOpsMax) {
    switch (K) {
#define QBE_WHOLE(KK) \
  case KK: level_whole<KK, kMode>(prog, c, base, E, tid); break;
      QBE_WHOLE(1) QBE_WHOLE(2) QBE_WHOLE(3) QBE_WHOLE(4) QBE_WHOLE(5) QBE_WHOLE(6) QBE_WHOLE(7)
#undef QBE_WHOLE
      default: break;
    }
  } else {
    level_long<kBytes>(prog, base, E, R, lgT, K, tid);
  }
}

// All levels of one item: three per trip, so that the record registers
// rotate without copies (level l uses the records read at level l - 2 and
// reads those of level l + 2; entries after the last level are zero).
// lv is the program's level table; t0, t1 and the first two levels'
// records were read before the inputs were copied.
// Export rows of a segment program and where they go (one-plan mode: the
// arena of the launch's slice group, item = the slice's place in it).
struct ExportCtx {
  const __attribute__((address_space(3))) u32x4* rows;  // LDS copy of the rows
  float2* arena;
  int64_t G, item;
};

// Copies export rows [first, first + count): every lane moves entries of
// each result from LDS to the arena.
__device__ __forceinline__ void copy_exports(const ExportCtx& x, uint32_t first, uint32_t count, uint32_t tid) {
  for (uint32_t e = first; e < first + count; ++e) {
    const u32x4 r = x.rows[e];
    const uint32_t src = uni(r.x), rank = uni(r.y);
    const uint64_t off = ((uint64_t)uni(r.w) << 32) | uni(r.z);
    float2* dst = x.arena + (int64_t)off * x.G + (x.item << rank);
    for (uint32_t i = tid; i < (1u << rank); i += kFusedBlock) dst[i] = lds_entry(8u * (src + i));
  }
}

// The export rows a level copies as it starts (results of earlier levels,
// read by no later level); returns the next row.
__device__ __forceinline__ uint32_t level_exports(const ExportCtx& x, u32x4 t, uint32_t next, uint32_t tid) {
  const uint32_t n = uni(t.w) >> 16;
  if (n) copy_exports(x, next, n, tid);
  return next + n;
}

// The barrier after a level, unless the next level is another part of the
// same dependency level (flag C of its entry): such parts read only earlier
// levels' results and write fresh space, so waves run on into the next part.
__device__ __forceinline__ void level_sync(const u32x4& t) {
  if (!((uni(t.z) >> 24) & kLevelCont)) __syncthreads();
}

// The level table in device memory as constant data: read with scalar
// loads at a uniform index, its entries arrive in scalar registers.
typedef const __attribute__((address_space(4))) u32x4* cu32x4p;

template <bool kBytes>
__device__ __forceinline__ uint32_t run_levels(gu32p prog, cu32x4p lv, uint32_t n_levels, u32x4 t0, u32x4 t1,
                                               Rec& ra, Rec& rb, const ExportCtx& xc, uint32_t tid) {
  u32x4 t2 = lv[2];
  Rec rc;
  uint32_t xn = 0;  // next export row
  for (uint32_t l = 0; l < n_levels; l += 3) {
    const u32x4 t3 = lv[l + 3];
    xn = level_exports(xc, t0, xn, tid);
    level_step<kBytes>(prog, t0, t2, ra, rc, tid);
    level_sync(t0);
    if (l + 1 >= n_levels) break;
    const u32x4 t4 = lv[l + 4];
    xn = level_exports(xc, t1, xn, tid);
    level_step<kBytes>(prog, t1, t3, rb, ra, tid);
    level_sync(t1);
    if (l + 2 >= n_levels) break;
    const u32x4 t5 = lv[l + 5];
    xn = level_exports(xc, t2, xn, tid);
    level_step<kBytes>(prog, t2, t4, rc, rb, tid);
    level_sync(t2);
    t0 = t3;
    t1 = t4;
    t2 = t5;
  }
  return xn;
}

// LDS fill of one work item's inputs, in rounds whose loads are all issued
// before the first store.
// LDS fill of one work item: its inputs and the level table (n_tab rows of
// 16 bytes), in rounds whose loads are all issued before the first store.
template <int U>
__device__ __forceinline__ void fill_lds(uint64_t* dinv, const uint64_t* sinv_, uint32_t n_inv, uint64_t* ddep,
                                         const uint64_t* sdep_, uint32_t n_dep, u32x4* dtab, const u32x4* stab_,
                                         uint32_t n_tab, uint32_t tid) {
  const auto sinv = as_global(sinv_);
  const auto sdep = as_global(sdep_);
  const auto stab = as_global(stab_);
  for (uint32_t i0 = 0; i0 < n_inv || i0 < n_dep || i0 < n_tab; i0 += U * kFusedBlock) {
    uint64_t vi[U], vd[U];
    const uint32_t it = i0 + tid;
    const u32x4 vt = it < n_tab ? stab[it] : u32x4{};
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const uint32_t i = i0 + j * kFusedBlock + tid;
      vi[j] = i < n_inv ? sinv[i] : 0;
      vd[j] = i < n_dep ? sdep[i] : 0;
    }
    if (it < n_tab) dtab[it] = vt;
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const uint32_t i = i0 + j * kFusedBlock + tid;
      if (i < n_inv) dinv[i] = vi[j];
      if (i < n_dep) ddep[i] = vd[j];
    }
  }
}

// Work distribution: in one-plan mode workgroup b takes items b, b + grid,
// ...; in batch mode items are pulled from a counter (uneven sizes).  The
// program stays in device memory (all workgroups of a plan read the same
// words, so they come from the caches); LDS holds the tensor entries only.
// Registers are budgeted for two workgroups per compute unit (4 waves per
// SIMD): where LDS allows, a second workgroup's slice runs while the first
// waits on its record reads.  (A bound of one workgroup -- the register file
// for one -- keeps the hardware to one workgroup per compute unit whatever
// the LDS size, and slices then run in rounds of 256.)
constexpr int kFusedWgPerCu = 2;
__global__ __launch_bounds__(kFusedBlock) __attribute__((amdgpu_waves_per_eu(kFusedBlock / 256, kFusedWgPerCu * kFusedBlock / 256))) void fused_kernel(FusedArgs a) {
  // all of the workgroup's LDS is dynamic, so that the tensor entries start
  // at LDS address 0 and record offsets are addresses; the two shared words
  // sit after the largest data block of the launch
  extern __shared__ uint4 lds4[];
  int64_t& s_item = *reinterpret_cast<int64_t*>(reinterpret_cast<char*>(lds4) + a.lds_ctl);
  uint32_t& s_flag = *reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(lds4) + a.lds_ctl + 8);
  const uint32_t tid = threadIdx.x;
  int64_t next = blockIdx.x;
  for (;;) {
    int64_t item;
    if (a.items) {
      __syncthreads();
      if (tid == 0) {
        const uint32_t it = atomicAdd(&a.state[0], 1u);
        s_item = (int64_t)it < a.n_items ? (int64_t)it : -1;
      }
      __syncthreads();
      item = __builtin_amdgcn_readfirstlane((int)s_item);
    } else {
      __syncthreads();
      item = next < a.n_items ? next : -1;
      next += gridDim.x;
    }
    if (item < 0) break;
    uint32_t plan = 0;
    int64_t slice = a.s_begin + item;
    const uint32_t* gprog = a.prog0;
    const float2* prep = a.prep0;
    FusedMeta mt = a.meta0;
    if (a.items) {
      const FusedItem wi = a.items[item];
      plan = uni(wi.plan);
      slice = uni((uint32_t)wi.slice);
      gprog = wi.prog;
      prep = wi.prep;
      mt = FusedMeta{uni(wi.meta.lds_tab), uni(wi.meta.levels),  uni(wi.meta.scalars), uni(wi.meta.scalar_off),
                     uni(wi.meta.free_vars), uni(wi.meta.inv), uni(wi.meta.dep),     uni(wi.meta.dep_src),
                     uni(wi.meta.bytes), 0, 0, 0, {}, {}};  // batch programs export and import nothing
      for (int i = 0; i < 4; ++i) {
        mt.lv0[i] = uni(wi.meta.lv0[i]);
        mt.lv1[i] = uni(wi.meta.lv1[i]);
      }
    }
    gprog = uniform_ptr(gprog);
    const gu32p prog = as_global(gprog);
    prep = uniform_ptr(prep);
    float2* data = reinterpret_cast<float2*>(lds4);
    // level table and the records of the first two levels: issued first, so
    // that they arrive while the inputs are copied
    const u32x4 t0 = {mt.lv0[0], mt.lv0[1], mt.lv0[2], mt.lv0[3]};
    const u32x4 t1 = {mt.lv1[0], mt.lv1[1], mt.lv1[2], mt.lv1[3]};
    typedef __attribute__((address_space(3))) u32x4* lds_u32x4p;
    const lds_u32x4p lv = (lds_u32x4p)(size_t)mt.lds_tab;  // the LDS copy
    Rec ra, rb;
    load_rec(prog, rec_word(uni(t0.x), uni(t0.y), uni(t0.z) & 0xFFFFu, (uni(t0.z) >> 16) & 0xFFu, tid), ra);
    load_rec(prog, rec_word(uni(t1.x), uni(t1.y), uni(t1.z) & 0xFFFFu, (uni(t1.z) >> 16) & 0xFFu, tid), rb);
    // inputs of this slice into LDS after the constants 1 and 0
    const uint32_t inv = mt.inv, dep = mt.dep;
    const float2* dsrc = prep + mt.dep_src + slice * (int64_t)dep;
    if (tid == 0) {
      data[0] = make_float2(1.f, 0.f);
      data[kFusedZero] = make_float2(0.f, 0.f);
    }
    // the scalar factors' offsets (lane j < 64: factor j), read now for the end
    const uint32_t n_scal = mt.scalars;
    const uint32_t scal0 = tid < n_scal && tid < 64 ? prog[mt.scalar_off + tid] : 0u;
    fill_lds<4>(reinterpret_cast<uint64_t*>(data + kFusedConsts), reinterpret_cast<const uint64_t*>(prep), inv,
                reinterpret_cast<uint64_t*>(data + kFusedConsts + inv), reinterpret_cast<const uint64_t*>(dsrc), dep,
                reinterpret_cast<u32x4*>(reinterpret_cast<char*>(lds4) + mt.lds_tab),
                reinterpret_cast<const u32x4*>(gprog + kHdr), mt.levels + kFusedLevelPad + mt.exports, tid);
    if (mt.imports) {
      // results of other launches this segment reads, into their LDS slots
      const gu32p rows = prog + kHdr + 4 * (mt.levels + kFusedLevelPad + mt.exports);
      for (uint32_t e = 0; e < mt.imports; ++e) {
        const uint32_t dst = uni(rows[4 * e]), rank = uni(rows[4 * e + 1]);
        const uint64_t off = ((uint64_t)uni(rows[4 * e + 3]) << 32) | uni(rows[4 * e + 2]);
        const float2* src = a.arena + (int64_t)off * a.G + (item << rank);
        for (uint32_t i = tid; i < (1u << rank); i += kFusedBlock) lds_store(8u * (dst + i), src[i]);
      }
    }
    __syncthreads();
    const ExportCtx xc{lv + mt.levels + kFusedLevelPad, a.arena, a.G, item};
    const cu32x4p lt = (cu32x4p)(size_t)(gprog + kHdr);
    const uint32_t xn = mt.bytes ? run_levels<true>(prog, lt, mt.levels, t0, t1, ra, rb, xc, tid)
                                 : run_levels<false>(prog, lt, mt.levels, t0, t1, ra, rb, xc, tid);
    if (mt.exports) {
      // the last levels' results; the next item's LDS fill waits at the
      // loop head's barrier
      copy_exports(xc, xn, mt.exports - xn, tid);
      continue;
    }
    if (tid < 64) {
      // product of the slice's scalar factors: lane j holds factor j (and
      // j + 64, ...), then a binary tree across the wave, in FP64
      const gu32p scal = prog + mt.scalar_off;
      double re = tid == 0 ? ldexp(1.0, (int)mt.free_vars) : 1.0, im = 0.0;
      for (uint32_t j = tid; j < n_scal; j += 64) {
        const float2 v = data[j < 64 ? scal0 : scal[j]];
        const double vr = v.x, vi = v.y;
        const double nr = re * vr - im * vi;
        im = re * vi + im * vr;
        re = nr;
      }
      for (uint32_t w = 1; w < n_scal && w < 64; w <<= 1) {  // lanes >= n_scal hold 1
        const double orr = __shfl_down(re, w, 64), oi = __shfl_down(im, w, 64);
        const double nr = re * orr - im * oi;
        im = re * oi + im * orr;
        re = nr;
      }
      if (tid == 0) {
        s_flag = 0u;
        if (a.reduce_here) {
          // publish the value (device-scope atomic stores, which leave the
          // writeback of the release nothing to flush) and count it with a
          // release; only the plan's last item acquires, then sums them all
          int64_t b = 0, e = a.n_items;
          if (a.ranges) {
            b = a.ranges[2 * plan];
            e = a.ranges[2 * plan + 1];
          }
          __hip_atomic_store(&a.out[item].x, re, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&a.out[item].y, im, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const uint32_t done =
              __hip_atomic_fetch_add(&a.state[2 + plan], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) + 1u;
          if ((int64_t)done == e - b) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            s_flag = 1u;
          }
        } else {
          a.out[item] = make_double2(re, im);
        }
      }
    }
    __syncthreads();
    if (s_flag) {
      // last item of this plan: FP64 sum of its items in reduce_kernel's
      // order (lane t < 256 adds items t, t + 256, ... in sequence, then a
      // binary tree over the 256 partials), so that a plan's amplitude has
      // the same bits whether it is summed here or by reduce_kernel; then
      // re-arm the plan's counter for the next launch.  The 4 KB of partials
      // overwrite LDS data (launch_fused sizes LDS for them); no item of this
      // plan remains.  The values are visible: every item's release on the
      // counter, thread 0's acquire fence after reading its last value, then
      // the barrier.
      int64_t b = 0, e = a.n_items;
      if (a.ranges) {
        b = a.ranges[2 * plan];
        e = a.ranges[2 * plan + 1];
      }
      double* sre = reinterpret_cast<double*>(lds4);
      double* sim = sre + kFusedReduceLanes;
      if (tid < kFusedReduceLanes) {
        double re = 0.0, im = 0.0;
        for (int64_t i = b + tid; i < e; i += kFusedReduceLanes) {
          const double2 v = a.out[i];
          re += v.x;
          im += v.y;
        }
        sre[tid] = re;
        sim[tid] = im;
      }
      __syncthreads();
      for (int w = kFusedReduceLanes / 2; w > 0; w >>= 1) {
        if (tid < w) {
          sre[tid] += sre[tid + w];
          sim[tid] += sim[tid + w];
        }
        __syncthreads();
      }
      if (tid == 0) {
        a.amps[plan] = make_double2(sre[0], sim[0]);
        a.state[2 + plan] = 0u;
      }
    }
  }
  if (a.items) {
    // the last workgroup to leave re-arms the work counter
    if (tid == 0) {
      const uint32_t left = __hip_atomic_fetch_add(&a.state[1], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
      if (left == gridDim.x) {
        a.state[0] = 0u;
        a.state[1] = 0u;
      }
    }
  }
}

// ================================================================== host ==

static int launch_fused(int grid, int lds_bytes, hipStream_t st, FusedArgs a) {
  static bool attr_set = false;
  if (!attr_set) {
    QBE_HIP(hipFuncSetAttribute((const void*)fused_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                kFusedLdsMax + kFusedCtlBytes));
    attr_set = true;
  }
  // at least the in-kernel slice sum's partials below the control words
  lds_bytes = std::max(lds_bytes, kFusedReduceLanes * 16);
  a.lds_ctl = (uint32_t)lds_bytes;
  fused_kernel<<<grid, kFusedBlock, lds_bytes + kFusedCtlBytes, st>>>(a);
  QBE_HIP(hipGetLastError());
  return QBE_OK;
}

static int fused_grid(int lds_bytes, int64_t n_items) {
  // resident workgroups per compute unit: the register bound, or fewer when
  // LDS (160 KB per compute unit) holds fewer
  const int per_cu = std::max(1, std::min(kFusedWgPerCu, (160 * 1024) / (lds_bytes + kFusedCtlBytes)));
  return (int)std::max<int64_t>(1, std::min<int64_t>(n_items, (int64_t)n_cus() * per_cu));
}

int fused_contract(const Plan& p, hipStream_t st, int64_t s_begin, int64_t n, double2* per_slice,
                   double2* amps, bool* reduced) {
  FusedArgs a{};
  a.prog0 = (const uint32_t*)p.d_fused_prog;
  a.prep0 = (const float2*)p.d_fused_in;
  a.s_begin = s_begin;
  a.n_items = n;
  a.state = (uint32_t*)p.d_state;
  a.out = per_slice;
  a.amps = amps;
  a.meta0 = fused_meta(p);
  a.reduce_here = n <= kInKernelReduceMax ? 1 : 0;
  *reduced = a.reduce_here != 0;
  return launch_fused(fused_grid(p.fused_lds_bytes, n), p.fused_lds_bytes, st, a);
}

int seg_launch(const FusedSeg& sg, float2* arena, int64_t G, int64_t s0, hipStream_t st) {
  const std::vector<uint32_t>& w = sg.prog;
  FusedArgs a{};
  a.prog0 = (const uint32_t*)sg.d_prog;
  a.prep0 = (const float2*)sg.d_in;
  a.meta0 = FusedMeta{(uint32_t)fused_table_lds(w[FH_DATA_ELEMS]), w[FH_LEVELS], 0, w[FH_SCALAR_OFF], 0,
                      w[FH_INV_ELEMS], w[FH_DEP_ELEMS], w[FH_DEP_SRC], w[FH_BYTE_OFFSETS], w[FH_EXPORTS],
                      w[FH_IMPORTS], 0, {}, {}};
  for (int i = 0; i < 4; ++i) {
    a.meta0.lv0[i] = w[kHdr + i];
    a.meta0.lv1[i] = w[kHdr + 4 + i];
  }
  a.s_begin = s0;
  a.n_items = G;
  a.state = nullptr;  // one-plan mode without the in-kernel sum uses no state
  a.arena = arena;
  a.G = G;
  return launch_fused(fused_grid(sg.lds_bytes, G), sg.lds_bytes, st, a);
}

// ------------------------------------------------------------------ batch --

int dev_batch_build(Batch& b) {
  const int np = (int)b.plans.size();
  std::vector<int> idx;
  b.lds_bytes = 0;
  b.wide.clear();
  b.wide_ws = 0;
  for (int i = 0; i < np; ++i) {
    const Plan& p = *b.plans[i];
    if (p.exec != QBE_EXEC_FUSED) {
      b.wide.push_back(i);
      continue;
    }
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
    const Plan& p = *b.plans[i];
    const FusedMeta mt = fused_meta(p);
    for (int64_t s = 0; s < p.n_slices; ++s)
      items.push_back(FusedItem{(const uint32_t*)p.d_fused_prog, (const float2*)p.d_fused_in, mt, s, (uint32_t)i, 0});
    ranges[2 * i + 1] = (int64_t)items.size();
  }
  b.n_items = (int64_t)items.size();
  b.item_begin = ranges;
  int rc;
  if ((rc = upload(&b.d_items, items.data(), items.size() * sizeof(FusedItem)))) return rc;
  if ((rc = upload(&b.d_ranges, ranges.data(), ranges.size() * 8))) return rc;
  if ((rc = dmalloc(&b.d_state, (2 + (size_t)np) * 4))) return rc;
  QBE_HIP(hipMemset(b.d_state, 0, (2 + (size_t)np) * 4));
  b.reduce_here = true;
  for (int i : idx)
    if (b.plans[i]->n_slices > kInKernelReduceMax) b.reduce_here = false;
  return step_batch_build(b);
}

void dev_batch_free(Batch& b) {
  void** ptrs[] = {&b.d_items, &b.d_ranges, &b.d_state, &b.d_wide, &b.d_wide_final};
  for (void** q : ptrs) {
    if (*q) (void)hipFree(*q);
    *q = nullptr;
  }
  for (void* s : b.side) (void)hipStreamDestroy((hipStream_t)s);
  for (void* e : b.ev_join) (void)hipEventDestroy((hipEvent_t)e);
  if (b.ev_fork) (void)hipEventDestroy((hipEvent_t)b.ev_fork);
  b.side.clear();
  b.ev_join.clear();
  b.ev_fork = nullptr;
}

int fused_batch_launch(const Batch& b, hipStream_t st, double2* per_item, double2* amps) {
  FusedArgs a{};
  a.items = (const FusedItem*)b.d_items;
  a.ranges = (const int64_t*)b.d_ranges;
  a.n_items = b.n_items;
  a.state = (uint32_t*)b.d_state;
  a.out = per_item;
  a.amps = amps;
  a.reduce_here = b.reduce_here ? 1 : 0;
  int rc = launch_fused(fused_grid(b.lds_bytes, b.n_items), b.lds_bytes, st, a);
  if (rc) return rc;
  // one reduction block per plan; blocks of per-step plans see an empty range
  if (!b.reduce_here)
    return launch_reduce(per_item, (const int64_t*)b.d_ranges, 0, amps, (int)b.plans.size(), st);
  return QBE_OK;
}

}  // namespace qbe
