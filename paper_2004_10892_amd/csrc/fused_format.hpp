// Fused (LDS-resident) form: launch constants and the program format the
// plan compiler (program.cpp) writes and the fused executor (fused.hip)
// reads.  Not part of the ABI.
#pragma once

#include <cstdint>

namespace qbe {

// Threads of a fused workgroup.
constexpr int kFusedBlock = 512;
// LDS budget of one fused workgroup (bytes): tensor entries, plus the
// program's records when they fit too (gfx950: 160 KB per workgroup).
constexpr int kFusedLdsMax = 160 * 1024 - 256;
// The largest LDS size (bytes) of which two workgroups fit one compute unit
// (with the 16 bytes of control words each).
constexpr int kFusedLdsPair = 160 * 1024 / 2 - 16;
// Largest slice count whose FP64 sum the fused kernel does itself (the
// last workgroup of a plan); above it a separate reduction kernel runs.
constexpr int64_t kInKernelReduceMax = 8192;

// --------------------------------------------------------- fused (LDS) form --

// A fused program lives in device memory (uint32 words) and is read from
// there (through the caches); the workgroup keeps the tensor entries and a
// copy of the level table in LDS.  A level holds nodes: a root bucket and
// the buckets it absorbed (the plan compiler merges buckets along chains of
// the dependency tree); an entry of a node's result sums T = 2^lgT terms,
// one per assignment of the members' eliminated variables.
// LDS data layout (complex64 elements):
//   [0], [1]                    the constants 1 (padding factor) and 0
//   [2, 2 + inv)                slice-invariant input tensors
//   [2 + inv, 2 + inv + dep)    this slice's copies of slice-dependent inputs
//   [2 + inv + dep, data)       intermediates (arena, reused level by level)
// then, from byte fused_table_lds(data), the level table (16 bytes a level)
// and the export rows after it.
// Program words:
//   header[kHdr]
//   levels[4 * (n_levels + kFusedLevelPad)]
//                               (record base, entries E, R | lgT << 16 |
//                               C << 24, factors K | X << 16), then zero
//                               entries; R = rows of a term record, T =
//                               2^lgT terms per entry, C = flags: kLevelCont
//                               when the next level is another part of the
//                               same dependency level (no barrier between
//                               the two), kLevelWide when the level's slots
//                               are 32-bit LDS byte addresses (at most three
//                               factors: one row a term either way), X =
//                               export rows copied as the level starts (the
//                               results of earlier levels)
//   exports[4 * n_exports]      a segment program's results for other
//                               launches: (LDS element, rank, arena offset
//                               lo, hi) in the order levels copy them; rows
//                               left after the last level are copied then
//   imports[4 * n_imports]      results of other launches a segment program
//                               reads: (LDS element, rank, arena offset lo,
//                               hi), copied in with the inputs
//   records                     level by level, E entries of T term records
//                               of R 16-byte rows (8R halfwords) each:
//                                 slot 0: LDS offset of the result (term 0),
//                                   0 (other terms)
//                                 slots 1..K: LDS offsets of the factor
//                                   entries for that term's assignment
//                                 rest: 0 (the constant 1); a padding term
//                                   (node with fewer terms than its level)
//                                   has slot 1 = the constant 0
//                               offsets in bytes (header FH_BYTE_OFFSETS = 1,
//                               data within 64 KB) or else in elements
//   scalars[n_scalars]          LDS element offsets of the slice's scalar
//                               factors, zero words to a multiple of 4, then
//                               4 * kFusedTailRows zero words (the executor
//                               reads kFusedTailRows rows at any record)
constexpr int kFusedTailRows = 2;
// C of a level entry: the next level reads nothing this one writes and
// writes nothing this one reads (both parts of one dependency level, whose
// results take fresh arena space), so the workgroup needs no barrier
// between them.
constexpr uint32_t kLevelCont = 1u;
// C of a level entry: its records' slots are 32-bit LDS byte addresses
// (1 + K <= 4 of them fill the 16-byte row that 16-bit slots would), so the
// executor uses them as they are.  Only on levels of at most kWideOpsMax
// factors that run in one pass: 2 terms an entry, or all term records
// within the workgroup's lanes.
constexpr uint32_t kLevelWide = 2u;
constexpr uint32_t kWideOpsMax = 3;
constexpr int kFusedLevelPad = 3;
// A level runs in one pass when every lane holds what it computes in the
// kFusedTailRows rows it read ahead: E x T <= kFusedBlock term records of
// at most kSplitOpsMax factors (a term record a lane), or, with T = 2,
// E <= kFusedBlock entries of at most kWholeOpsMax factors (both terms a
// lane).  Larger levels read further records while they run.
constexpr int kSplitOpsMax = 8 * kFusedTailRows - 1;
constexpr int kWholeOpsMax = 4 * kFusedTailRows - 1;
// Entries of a one-pass level of 2^lgT terms of K factors (kFusedBlock
// when no level of that shape runs in one pass).
inline int64_t fused_pass_entries(uint32_t lgT, uint32_t K) {
  if (lgT == 1 && K <= (uint32_t)kWholeOpsMax) return kFusedBlock;
  if (K <= (uint32_t)kSplitOpsMax) return kFusedBlock >> lgT;
  return kFusedBlock;
}
// LDS elements 0 and 1 hold the constants 1 (padding factor) and 0 (the
// factor of a padding term); inputs follow.
constexpr int kFusedConsts = 2;
constexpr uint32_t kFusedZero = 1;
// LDS byte offset of the level table's copy: after the tensor entries.
inline int64_t fused_table_lds(int64_t data_elems) { return (data_elems * 8 + 15) / 16 * 16; }
enum FusedHdr {
  FH_WORDS = 0,       // total program words
  FH_LEVELS,          // n_levels
  FH_SCALARS,         // n_scalars
  FH_SCALAR_OFF,      // word offset of the scalar list
  FH_FREE,            // variables in no tensor (factor 2 each)
  FH_INV_ELEMS,       // slice-invariant input elements
  FH_DEP_ELEMS,       // per-slice input elements
  FH_DATA_ELEMS,      // total LDS data elements (including the constant)
  FH_DEP_SRC,         // element offset of slice 0's block in the prepared buffer
  FH_N_SLICES,        // 2^m (saturated)
  FH_BYTE_OFFSETS,    // 1: record offsets are LDS bytes, 0: complex64 elements
  FH_EXPORTS,         // export rows (segment programs; 0 otherwise)
  FH_IMPORTS,         // import rows (segment programs; 0 otherwise)
  kHdr = 16
};

}  // namespace qbe
