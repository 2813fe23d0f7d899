// Host-side verification of a compiled plan: every index any kernel of the
// plan can form is checked against the size of the buffer it reads or
// writes, before anything is uploaded or launched.  Returns "" when the plan
// is sound, otherwise a description of the first violation.
#include <string>

#include "qbe_internal.hpp"

namespace qbe {

namespace {

std::string fail(const std::string& what, int64_t a, int64_t b) {
  return what + " (" + std::to_string(a) + " vs " + std::to_string(b) + ")";
}

}  // namespace

std::string check_plan(const Plan& p) {
  const int64_t raw_elems = (int64_t)p.model.data.size() / 2;
  for (size_t i = 0; i < p.step_map.size(); ++i)
    if (p.step_map[i] < 0 || p.step_map[i] >= raw_elems) return fail("step map entry out of range", p.step_map[i], raw_elems);
  if ((int64_t)p.step_map.size() != p.step_elems) return "step map size";
  for (size_t i = 0; i < p.fused_map.size(); ++i)
    if (p.fused_map[i] < 0 || p.fused_map[i] >= raw_elems) return fail("fused map entry out of range", p.fused_map[i], raw_elems);

  // per-step launches
  for (size_t k = 0; k < p.steps.size(); ++k) {
    const StepProg& sp = p.steps[k];
    const bool sum_u = sp.out_rank >= 0;
    const int r = sum_u ? sp.out_rank : -sp.out_rank;
    const int xbits = r + (sum_u ? 1 : 0);
    if (r > 30) return "result rank above 30";
    if (sp.n_ops < 1 || sp.n_ops > kMaxOps) return "operand count";
    if (sp.out_base < 0 || sp.out_base + (int64_t(1) << r) > p.arena_per_slice)
      return fail("result outside the arena", sp.out_base + (int64_t(1) << r), p.arena_per_slice);
    for (int i = 0; i < sp.n_ops; ++i) {
      const StepOp& o = sp.ops[i];
      if (__builtin_popcount(o.mask) != o.rank) return "operand mask and rank disagree";
      if (xbits < 32 && (o.mask >> xbits) != 0) return "operand mask outside the union index";
      if (sum_u && o.rank > 0 && !((o.mask >> r) & 1u) && o.rank > r) return "operand rank";
      if (o.is_input) {
        const int64_t versions = int64_t(1) << __builtin_popcount(o.smask);
        if (o.base < 0 || o.base + (versions << o.rank) > p.step_elems)
          return fail("input operand outside the prepared buffer", o.base + (versions << o.rank), p.step_elems);
        if (p.m < 32 && (o.smask >> p.m) != 0) return "input slice mask above m";
      } else {
        if (o.base < 0 || o.base + (int64_t(1) << o.rank) > p.arena_per_slice)
          return fail("intermediate operand outside the arena", o.base + (int64_t(1) << o.rank), p.arena_per_slice);
        if (o.smask != 0) return "intermediate with a slice mask";
      }
    }
  }
  for (int64_t off : p.scalar_arena)
    if (off < 0 || off >= p.arena_per_slice) return "scalar result outside the arena";
  for (size_t j = 0; j < p.scalar_inputs_base.size(); ++j) {
    const int64_t versions = int64_t(1) << __builtin_popcount(p.scalar_inputs_smask[j]);
    if (p.scalar_inputs_base[j] < 0 || p.scalar_inputs_base[j] + versions > p.step_elems)
      return "scalar input outside the prepared buffer";
  }

  // fused program
  if (p.fused_ok) {
    const auto& w = p.fused_prog;
    if (w.size() < (size_t)kHdr || w[FH_WORDS] != w.size()) return "fused header";
    const uint32_t nl = w[FH_LEVELS], ns = w[FH_STEPS], no = w[FH_OPS], nsc = w[FH_SCALARS];
    const size_t need = kHdr + (nl + 1) + nl + 2 * (size_t)ns + no + nsc;
    if (need > w.size()) return "fused program truncated";
    const uint32_t inv = w[FH_INV_ELEMS], dep = w[FH_DEP_ELEMS], data = w[FH_DATA_ELEMS];
    if ((int64_t)w.size() * 4 + (int64_t)data * 8 != p.fused_lds_bytes) return "fused LDS size";
    if (p.fused_lds_bytes > kFusedLdsMax) return "fused LDS above budget";
    if (w[FH_DEP_SRC] != inv) return "fused dependent block offset";
    if ((int64_t)inv + (int64_t)dep * p.n_slices != p.fused_elems) return "fused prepared size";
    if (inv + dep > data) return "fused inputs above data size";
    const uint32_t* lb = w.data() + kHdr;
    const uint32_t* le = lb + nl + 1;
    const uint32_t* sw = le + nl;
    const uint32_t* ow = sw + 2 * ns;
    const uint32_t* sc = ow + no;
    if (lb[0] != 0 || lb[nl] != ns) return "fused level ranges";
    for (uint32_t l = 0; l < nl; ++l) {
      if (lb[l] >= lb[l + 1]) return "empty or unordered level";
      int64_t e = 0;
      for (uint32_t j = lb[l]; j < lb[l + 1]; ++j) {
        const uint32_t w0 = sw[2 * j], w1 = sw[2 * j + 1];
        const uint32_t out = w0 & 0xFFFFu, r = (w0 >> 16) & 31u, nop = w0 >> 21;
        const uint32_t op0 = w1 & 0xFFFFu, eb = w1 >> 16;
        if (eb != e) return fail("fused element ranges", eb, e);
        if (out < inv + dep || (int64_t)out + (int64_t(1) << r) > data) return "fused result outside the arena";
        if (nop < 1 || (int64_t)op0 + nop > no) return "fused operand range";
        for (uint32_t i = 0; i < nop; ++i) {
          const uint32_t off = ow[op0 + i] & 0xFFFFu, mask = ow[op0 + i] >> 16;
          if ((mask >> (r + 1)) != 0) return "fused operand mask outside the union";
          const int rank = __builtin_popcount(mask);
          if ((int64_t)off + (int64_t(1) << rank) > data) return "fused operand outside LDS data";
        }
        e += int64_t(1) << r;
      }
      if (e != le[l]) return "fused level element count";
    }
    for (uint32_t j = 0; j < nsc; ++j)
      if (sc[j] >= data) return "fused scalar outside LDS data";
  }
  return "";
}

}  // namespace qbe
