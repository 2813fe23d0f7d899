// Internal structures shared by the C-ABI layer (api.cpp), the plan compiler
// (program.cpp) and the device code (device.hip).  Not part of the ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "planner.hpp"

namespace qbe {

// Largest number of operands one bucket may have in the per-step form
// (larger buckets are split into a chain of partial products by the plan
// compiler; the fused form has no limit).
constexpr int kMaxOps = 8;
// Threads per workgroup of the per-step and fused kernels.
constexpr int kBlock = 256;
// Low index bits handled inside one workgroup tile by the per-step kernel.
constexpr int kLoBits = 8;
// LDS budget of one fused workgroup (bytes): program + tensors.
constexpr int kFusedLdsMax = 64 * 1024 - 256;

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
  int32_t out_rank;   // r_b (0 for a scalar result)
  int64_t out_base;   // arena offset (per-slice unit)
  int32_t n_ops;
  StepOp ops[kMaxOps];
};

// --------------------------------------------------------- fused (LDS) form --

// Word layout of a fused program (uint32 words), all offsets in elements:
//   header[kHdr]
//   level_begin[n_levels + 1]    step index ranges per level
//   level_elems[n_levels]        elements computed per level
//   steps[2 * n_steps]           w0 = out_off | out_rank << 16 | n_ops << 21
//                                w1 = op0 | elem_begin << 16
//   ops[n_ops]                   off | mask << 16
//   scalars[n_scalars]           LDS offsets of the slice's scalar factors
enum FusedHdr {
  FH_WORDS = 0,       // total program words
  FH_LEVELS,          // n_levels
  FH_STEPS,           // n_steps
  FH_OPS,             // n_ops
  FH_SCALARS,         // n_scalars
  FH_FREE,            // variables in no tensor (factor 2 each)
  FH_INV_ELEMS,       // slice-invariant input elements (LDS [0, inv))
  FH_DEP_ELEMS,       // per-slice input elements (LDS [inv, inv + dep))
  FH_DATA_ELEMS,      // total LDS data elements
  FH_INV_SRC,         // element offset of the invariant block (prepared)
  FH_DEP_SRC,         // element offset of slice 0's block (prepared)
  FH_N_SLICES,        // 2^m
  kHdr = 16
};

struct Plan {
  // host side
  Model model;
  Schedule sched;
  ScheduleCost cost;
  int m = 0;
  int64_t n_slices = 1;
  int exec = 0;
  int precision = 0;
  int block = kBlock;
  int n_levels = 0;

  // per-step form
  std::vector<StepProg> steps;          // launch list (chained splits included)
  std::vector<int64_t> scalar_arena;    // arena offsets of rank-0 step results
  std::vector<int64_t> scalar_inputs_base;  // prepared offsets of rank-0 inputs
  std::vector<uint32_t> scalar_inputs_smask;
  int64_t arena_per_slice = 0;          // elements
  std::vector<int32_t> step_map;        // prepared per-step buffer gather map
  int64_t step_elems = 0;

  // fused form
  bool fused_ok = false;
  std::vector<uint32_t> fused_prog;
  std::vector<int32_t> fused_map;       // prepared fused buffer gather map
  int64_t fused_elems = 0;
  int fused_lds_bytes = 0;

  // device side (owned)
  int device = -1;
  void* d_raw = nullptr;        // complex128 model data
  void* d_step_map = nullptr;
  void* d_step_in = nullptr;    // complex64 prepared inputs, per-step layout
  void* d_fused_map = nullptr;
  void* d_fused_in = nullptr;   // complex64 prepared inputs, fused layout
  void* d_fused_prog = nullptr;
  void* d_scalar_tab = nullptr; // int64 arena offsets, int64 input bases, uint32 smasks
};

// A set of plans contracted together in one fused launch.
struct Batch {
  std::vector<const Plan*> plans;
  std::vector<int> wide;            // plans run in the per-step form
  size_t wide_ws = 0;               // workspace those need (one at a time)
  std::vector<int64_t> item_begin;  // per plan, into the item table (+ end)
  int64_t n_items = 0;
  int lds_bytes = 0;
  void* d_progs = nullptr;   // const uint32_t* per plan
  void* d_preps = nullptr;   // const float2* per plan
  void* d_items = nullptr;   // FusedItem per item
  void* d_ranges = nullptr;  // int64 item_begin (n_plans + 1)
};

// Plan compilation (program.cpp).
void compile_plan(Plan& p);

// Device entry points (device.hip).  All return 0 or a QBE_ERR_* code and
// set the thread-local error text on failure.
int dev_count(int* n);
int dev_set(int device);
int dev_upload_plan(Plan& p);               // allocates + prepares inputs
int dev_update_data(Plan& p);
void dev_free_plan(Plan& p);
int dev_contract(const Plan& p, void* stream, void* ws, size_t ws_bytes, int64_t s_begin,
                 int64_t s_end, double* d_partial_out, double* d_per_slice /*may be null*/);
size_t dev_workspace_min(const Plan& p, int64_t n_slices_in_call);
size_t dev_workspace_all(const Plan& p);
int dev_batch_build(Batch& b);
void dev_batch_free(Batch& b);
size_t dev_batch_workspace(const Batch& b);
int dev_batch_contract(const Batch& b, void* stream, void* ws, size_t ws_bytes, double* d_amps);
int dev_memcpy_d2h(void* dst, const void* src, size_t bytes, void* stream);

void set_error(const std::string& s);

}  // namespace qbe
