// Internal structures shared by the C-ABI layer (api.cpp), the plan compiler
// (program.cpp) and the device code (device.hip).  Not part of the ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "fused_format.hpp"
#include "planner.hpp"

namespace qbe {

// Largest number of operands one bucket may have in the per-step form
// (larger buckets are split into a chain of partial products by the plan
// compiler; the fused form has no limit).
constexpr int kMaxOps = 8;
// Threads per workgroup of the per-step kernels.
constexpr int kBlock = 256;
// Low index bits handled inside one workgroup tile by the per-step kernel.
constexpr int kLoBits = 8;
// Largest operand rank of a launch that sums several variables: the merged
// kernels carry an operand's per-summed-bit byte offsets in 32 bits.
constexpr int kMergedMaxRank = 28;

struct Model {
  int n_vars = 0;
  std::vector<std::vector<int>> tvars;  // per tensor
  std::vector<int64_t> data_off;        // complex element offset per tensor
  std::vector<double> data;             // interleaved complex128
};

// ---------------------------------------------------- per-step (HBM) form --

// One operand of a per-step kernel launch.
struct StepOp {
  int64_t base;     // element offset: intermediates in the arena (per-slice
                    // unit, scaled by the group size at launch), inputs in the
                    // prepared per-step buffer (version 0)
  int32_t is_input; // 1: prepared input tensor, 0: intermediate
  int32_t rank;     // rank of the operand
  uint32_t mask;    // bits of the union index X = (u << r_b) | x it reads
  uint32_t smask;   // inputs: slice bits selecting the tensor's version
};

struct StepProg {
  int32_t out_rank;   // r_b (0 for a scalar result); negative: a partial
                      // product over -out_rank variables without the sum
  int32_t n_sum = 1;  // summed variables: the top n_sum bits of the union
                      // index X = (u << r_b) | x (more than one when the
                      // launch merges a chain of buckets)
  int64_t out_base;   // arena offset (per-slice unit)
  int32_t n_ops;
  int32_t ept = 0;        // tiles per thread per pass (0: default)
  int32_t wg_per_cu = 0;  // workgroups per compute unit (0: default)
  // Outer-product buckets (two operands A, B holding u, the others only u)
  // run on MFMA in 16 x 16 result tiles: indices of A and B in ops, -1 if
  // the bucket is not of that shape.
  int32_t mm_a = -1, mm_b = -1;
  // Merged launches (n_sum > 1) that run as a batched complex product on
  // MFMA: bit i set = operand i belongs to the B group, clear = A group;
  // mmk = 0 when the launch is not of that shape.
  int32_t mmk = 0;
  uint32_t mmk_side = 0;
  // Merged launches on the multi-term kernel: the kernel's summed-value bit
  // b is union index bit r_b + sum_bit[b] (a permutation of 0..n_sum-1; the
  // kernel handles its two lowest bits four terms at a time).
  int32_t sum_bit[4] = {0, 1, 2, 3};
  StepOp ops[kMaxOps];
};

// Small per-step launches of one dependency level run as one launch
// (group_kernel): each step of a group is described by a GroupStep and owns
// a run of tiles of 256 result entries for every block of group_sb slices.
constexpr int kGroupMaxRank = 10;  // largest result rank a grouped step has
struct GroupStep {
  int64_t out;              // arena offset of the result (per-slice unit)
  int64_t base[kMaxOps];    // arena offset (per-slice unit), or prepared-input offset
  uint32_t mask[kMaxOps];   // bits of X = (u << r) | x each operand reads
  uint32_t smask[kMaxOps];  // inputs: slice bits selecting the copy
  int32_t rank[kMaxOps];
  uint32_t is_input;        // bit i: operand i is a prepared input
  int32_t n_ops, r, sum_u;  // sum_u 0: product without a summed bit
  int32_t step;             // index into the plan's steps (host checks)
};
// A step the group kernels can run (one summed variable at most, no MFMA
// form), and its descriptor.
bool groupable(const StepProg& sp);
GroupStep group_step_of(const StepProg& sp, int k);
// One entry of the per-step execution order: steps[step] alone (group < 0),
// or group `group` of small steps in one launch.
struct LaunchItem {
  int32_t step, group;
  int32_t seg = -1;  // >= 0: fused segment seg (step and group -1)
};

// A fused segment of a per-step plan: a connected run of small buckets
// (unions of at most R + 1 variables) contracted by one LDS-resident launch
// of the fused executor (fused.hip).  Its import rows copy the results of
// other launches that it reads from the arena into LDS; its export rows copy
// its results that other launches read (and its rank-0 results) from LDS to
// the arena.  The prefix -- the subtrees of small buckets above the inputs
// -- imports nothing; a later segment exports only its top bucket's result.
struct FusedSeg {
  std::vector<uint32_t> prog;   // fused program (fused_format.hpp), no scalar list
  std::vector<int32_t> map;     // its prepared-input gather map
  int64_t elems = 0;            // map entries
  int lds_bytes = 0, levels = 0, buckets = 0;
  std::vector<uint32_t> exports, imports;  // copies of the program's rows
  int64_t bytes_per_slice = 0, flops_per_slice = 0;
  int32_t level = 0;            // launch level (depth by memory hazards)
  int32_t pos = 0;              // launched before per-step step pos (in step order)
  void* d_map = nullptr;        // device copies: map, prepared inputs, program
  void* d_in = nullptr;
  void* d_prog = nullptr;
};
// A grouped step of a batch's per-step instances, which run level by level
// together: the step with its plan's context.  Its work units are `tiles`
// tiles for each of ceil(G / sb) blocks of sb slices.
struct WideGroupStep {
  GroupStep s;
  const void* step_in;   // the plan's prepared inputs (device)
  int64_t arena;         // the plan's arena: complex64 offset in the batch workspace
  int64_t G;             // the plan's slices (all run at once)
  int32_t sb, tiles;
};
struct WideItem {
  int32_t plan, step, group;  // plan's step alone (group < 0), or a group
};

struct Plan {
  // host side: the model and schedule the programs are compiled from --
  // the caller's, or (input folding) one whose tensors are products of the
  // caller's -- and the caller's schedule, whose cost model the plan reports
  Model model;
  Schedule sched;
  Schedule src_sched;
  std::vector<std::vector<int>> src_tvars;  // the caller's model structure
  std::vector<std::vector<int>> fold;       // compiled tensor -> caller's tensors
  ScheduleCost cost;
  int m = 0;
  int64_t n_slices = 1;
  int exec = 0;
  int precision = 0;
  bool merge = true;      // merge bucket chains (per-step launches, fused levels)
  int max_sums = 0;       // summed variables a merged per-step launch may hold (0: the default, 4)
  int block = kBlock;
  int n_levels = 0;       // dependency depth of the buckets
  int fused_levels = 0;   // levels of the fused program (merged buckets)

  // per-step form
  std::vector<StepProg> steps;          // launch list (chained splits included)
  std::vector<int64_t> scalar_arena;    // arena offsets of rank-0 step results
  std::vector<int64_t> scalar_inputs_base;  // prepared offsets of rank-0 inputs
  std::vector<uint32_t> scalar_inputs_smask;
  int64_t arena_per_slice = 0;          // elements
  int64_t step_bytes_per_slice = 0;     // complex64 bytes the launches read and write
  std::vector<int32_t> step_map;        // prepared per-step buffer gather map
  int64_t step_elems = 0;
  // execution order: launches level by level (dependency depth, with the
  // arena's reuse counted as a dependency), small launches of a level grouped
  std::vector<LaunchItem> launch_order;
  std::vector<GroupStep> group_steps;   // every group's steps, group by group
  std::vector<int32_t> group_first;     // group g: steps [first[g], first[g + 1])
  std::vector<uint32_t> group_prefix;   // group g: first[g + 1] - first[g] + 1 tile
                                        // offsets from index first[g] + g
  int32_t group_sb = 1;                 // slices per block of a group launch
  std::vector<int32_t> step_level;      // level of each step in that order

  // fused segments of a per-step plan (qbe_plan_opts.fused_prefix and
  // fused_segments): the prefix (segs[0] when has_prefix) and later runs
  // of small buckets, launched in launch_order
  int want_prefix = 0;                  // 0 none, 1 the largest bound that fits, else R
  bool want_segments = false;
  bool has_prefix = false;
  int seg_max_rank = -1;                // result rank bound R of their buckets (-1: none)
  std::vector<FusedSeg> segs;

  // fused form
  bool fused_ok = false;
  std::vector<uint32_t> fused_prog;
  std::vector<int32_t> fused_map;       // prepared fused buffer gather map
  int64_t fused_elems = 0;
  int fused_lds_bytes = 0;              // LDS of one workgroup

  // device side (owned)
  int device = -1;
  void* d_raw = nullptr;        // complex128 model data
  void* d_step_map = nullptr;
  void* d_step_in = nullptr;    // complex64 prepared inputs, per-step layout
  void* d_fused_map = nullptr;
  void* d_fused_in = nullptr;   // complex64 prepared inputs, fused layout
  void* d_fused_prog = nullptr;
  void* d_scalar_tab = nullptr; // int64 arena offsets, int64 input bases, uint32 smasks
  void* d_state = nullptr;      // uint32[4]: work counter, exits, items done (fused)
  void* d_group = nullptr;      // GroupStep array, then the uint32 tile prefixes
};

// A set of plans contracted together in one fused launch.
struct Batch {
  std::vector<const Plan*> plans;
  std::vector<int> wide;            // plans run in the per-step form
  size_t wide_ws = 0;               // workspace those need (all at once)
  std::vector<size_t> wide_off;     // per wide plan: its workspace region
  std::vector<WideItem> wide_order; // their launches, level by level
  std::vector<int32_t> wide_level;  // level v: wide_order [wide_level[v], wide_level[v + 1])
  std::vector<WideGroupStep> wide_steps;
  std::vector<int32_t> wide_first;  // group g: wide_steps [first[g], first[g + 1])
  std::vector<uint64_t> wide_prefix;  // group g: count + 1 unit offsets from first[g] + g
  void* d_wide = nullptr;           // wide_steps, then wide_prefix
  void* d_wide_final = nullptr;     // per wide plan: its slice product and sum
  std::vector<int64_t> item_begin;  // per plan, into the item table (+ end)
  int64_t n_items = 0;
  int lds_bytes = 0;
  void* d_items = nullptr;   // FusedItem per item
  void* d_ranges = nullptr;  // int64 (begin, end) per plan
  void* d_state = nullptr;   // uint32[2 + n_plans]: work, exits, items done per plan
  bool reduce_here = true;   // the fused kernel sums each plan's items itself
  // the launches of one level of the per-step plans are independent: they
  // are dealt over the caller's stream and these (default priority),
  // forked from and joined back to the caller's stream by the events
  std::vector<void*> side;     // hipStream_t
  void* ev_fork = nullptr;     // hipEvent_t
  std::vector<void*> ev_join;  // hipEvent_t, one per side stream
};

// -------------------------------------------------- learned proposal (GNN) --

constexpr int kGnnFeatures = 8;   // must equal kFeatures of the planner
constexpr int kGnnHidden = 64;
constexpr int kGnnLayers = 3;
constexpr int kGnnHeads = 2;      // 0: slicing score, 1: elimination priority

struct Gnn {
  int device = -1;
  int step = 0;                // optimizer steps taken
  void* d_p = nullptr;         // FP32 master parameters
  void* d_p16 = nullptr;       // FP16 copy used by the passes
  void* d_g = nullptr;         // gradients
  void* d_m = nullptr;         // Adam moments
  void* d_v = nullptr;
  void* d_ws = nullptr;        // graph + activations
  size_t ws_bytes = 0;
};

int gnn_num_params();
int gnn_alloc(Gnn& g, int device);
void gnn_free(Gnn& g);
int gnn_set_params(Gnn& g, const float* host, bool reset_optimizer);
int gnn_get_params(const Gnn& g, float* host);
// FP32 parameters, Adam moments and step count (a training checkpoint).
int gnn_get_state(const Gnn& g, float* p, float* m, float* v, int* step);
int gnn_set_state(Gnn& g, const float* p, const float* m, const float* v, int step);
int gnn_score(Gnn& g, void* stream, int head, int n, const int* rp, const int* col, const float* feats,
              float* scores);
int gnn_train_step(Gnn& g, void* stream, int head, int n, const int* rp, const int* col, const float* feats,
                   int nc, const int* cand, const float* y, float lr, float* loss_out, float* grads_out);

// Plan compilation (program.cpp).
// Input folding: the input tensors of a bucket multiplied into one tensor
// over the union of their variables (at most kFoldMaxVars of them), so that
// an entry of the bucket multiplies fewer factors.  The product is the same
// (Eq. 2 multiplies all of a bucket's tensors), formed once per plan in
// complex128.  fold_groups lists the compiled model's tensors as groups of
// the caller's (singletons for tensors left as they are); fold_model builds
// that model's structure and data.
constexpr int kFoldMaxVars = 6;
std::vector<std::vector<int>> fold_groups(const Model& m, const Schedule& s);
Model fold_model(const Model& m, const std::vector<std::vector<int>>& groups);
// Then an input factor of bucket k whose variables all lie in a result
// operand R of k (R's producer j has them all in its result) moves into
// bucket j when R has at least two variables fewer than U_k: j multiplies
// it into each of its 2^(|R| + 1) terms (it is constant in j's summed
// variable, so it passes the sum unchanged) instead of k into each of its
// 2^|U_k|.  Steps are visited from the last, so a factor moves on down
// while that holds.  Returns the number of moves.
int push_inputs(Schedule& s);

void compile_plan(Plan& p);

// Device entry points (device.hip).  All return 0 or a QBE_ERR_* code and
// set the thread-local error text on failure.
int dev_count(int* n);
int dev_set(int device);
int dev_upload_plan(Plan& p);               // allocates + prepares inputs
int dev_update_data(Plan& p);
void dev_free_plan(Plan& p);
void dev_forget_plan(Plan& p);              // clears the device pointers, frees nothing
int dev_contract(const Plan& p, void* stream, void* ws, size_t ws_bytes, int64_t s_begin,
                 int64_t s_end, double* d_partial_out, double* d_per_slice /*may be null*/);
size_t dev_workspace_min(const Plan& p, int64_t n_slices_in_call);
// Allocation-free contraction (qbe_contract_static): a fixed device array of
// kStaticScratchBytes per device serves as the workspace.  The set-up call
// looks its address up once per device (with that device current).
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
int dev_static_scratch_init(int device);
int dev_contract_static(const Plan& p, void* stream, double* d_amp_out);
size_t dev_workspace_all(const Plan& p);
int dev_autotune(Plan& p, void* stream, void* ws, size_t ws_bytes, int64_t min_elems);
int dev_profile(const Plan& p, void* stream, void* ws, size_t ws_bytes, float* ms_out, int cap, int* n_out);
int dev_batch_build(Batch& b);
void dev_batch_free(Batch& b);
size_t dev_batch_workspace(const Batch& b);
int dev_batch_contract(const Batch& b, void* stream, void* ws, size_t ws_bytes, double* d_amps);
int dev_memcpy_d2h(void* dst, const void* src, size_t bytes, void* stream);
int dev_permute(const void* in, void* out, int r, const int32_t* perm, int64_t batch, void* stream);

void set_error(const std::string& s);

}  // namespace qbe
