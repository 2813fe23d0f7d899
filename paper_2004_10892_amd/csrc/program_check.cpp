// Host-side verification of a compiled plan: every index any kernel of the
// plan can form is checked against the size of the buffer it reads or
// writes, before anything is uploaded or launched.  Returns "" when the plan
// is sound, otherwise a description of the first violation.
#include <algorithm>
#include <string>

#include "qbe_internal.hpp"

namespace qbe {

namespace {

std::string fail(const std::string& what, int64_t a, int64_t b) {
  return what + " (" + std::to_string(a) + " vs " + std::to_string(b) + ")";
}

}  // namespace

// The data flow of a fused program through LDS, from its records alone.
// Time steps are the barrier groups (levels joined by continuation flags),
// 0..G-1, with the input block and the import rows filled at -1 and the
// export rows left over and the scalar list read at G.  An element is read
// only after a write (or the fill) at an earlier step; a write never lands
// at the step of a read of the same element, twice in one step, or over a
// value not yet read: every value of a contraction (input entry, result
// entry) is read by its one consumer -- a node or an export row -- at one
// step, so an overwrite before any read means a value lost.  So no result
// overwrites an operand that is still to be read, and a barrier group never
// reads what it writes.
static std::string check_fused_liveness(const std::vector<uint32_t>& w, uint32_t nl, uint32_t nx, uint32_t ni,
                                        const uint32_t* xr, uint32_t unit, uint32_t data) {
  const uint32_t* lv = w.data() + kHdr;
  const uint32_t inv = w[FH_INV_ELEMS], dep = w[FH_DEP_ELEMS];
  // per element: the step of its last write (-2: never written), and
  // whether a read since then forbids a write until a later step
  std::vector<int> last_w(data, -2), last_r(data, -2);
  std::vector<char> unread(data, 0);
  for (uint32_t e = kFusedConsts; e < kFusedConsts + inv + dep; ++e) last_w[e] = -1, unread[e] = 1;
  for (uint32_t e = nx; e < nx + ni; ++e)
    for (uint32_t i = 0; i < (1u << xr[4 * e + 1]); ++i) last_w[xr[4 * e] + i] = -1, unread[xr[4 * e] + i] = 1;
  auto read = [&](uint32_t e, int g) -> bool {
    if (e < kFusedConsts) return true;  // the constants
    if (last_w[e] == -2 || last_w[e] >= g) return false;
    last_r[e] = std::max(last_r[e], g);
    unread[e] = 0;
    return true;
  };
  auto write = [&](uint32_t e, int g) -> bool {
    // not over a value read at this step or later, nor twice in one step
    if (last_r[e] >= g || last_w[e] == g || unread[e]) return false;
    last_w[e] = g;
    unread[e] = 1;
    return true;
  };
  int g = 0;
  int64_t xn = 0;
  std::vector<uint32_t> writes;
  for (uint32_t l = 0; l < nl; ++l) {
    const uint32_t base = lv[4 * l], E = lv[4 * l + 1], R = lv[4 * l + 2] & 0xFFFFu,
                   lgT = (lv[4 * l + 2] >> 16) & 0xFFu, C = (lv[4 * l + 2] >> 24) & kLevelCont,
                   K = lv[4 * l + 3] & 0xFFFFu, X = lv[4 * l + 3] >> 16;
    const bool wide = ((lv[4 * l + 2] >> 24) & kLevelWide) != 0;
    const uint32_t su = wide ? 8u : unit;
    for (uint32_t e = 0; e < X; ++e, ++xn)
      for (uint32_t i = 0; i < (1u << xr[4 * xn + 1]); ++i)
        if (!read(xr[4 * xn] + i, g)) return "fused export row reads an element not written before it";
    for (uint32_t f = 0; f < E; ++f)
      for (uint32_t t = 0; t < (1u << lgT); ++t) {
        const uint32_t* rec = w.data() + base + ((size_t)f * (1u << lgT) + t) * 4 * R;
        auto hw = [&](uint32_t j) { return wide ? rec[j] : (rec[j / 2] >> (16 * (j % 2))) & 0xFFFFu; };
        for (uint32_t j = 1; j <= K; ++j)
          if (!read(hw(j) / su, g)) return "fused operand read before it is written, or after it is overwritten";
        if (t == 0) writes.push_back(hw(0) / su);
      }
    if (!C) {
      for (uint32_t e : writes)
        if (!write(e, g)) return "fused result overwrites a value still to be read";
      writes.clear();
      ++g;
    }
  }
  for (; xn < nx; ++xn)
    for (uint32_t i = 0; i < (1u << xr[4 * xn + 1]); ++i)
      if (!read(xr[4 * xn] + i, g)) return "fused export row reads an element not written before it";
  const uint32_t so = w[FH_SCALAR_OFF], nsc = w[FH_SCALARS];
  for (uint32_t j = 0; j < nsc; ++j)
    if (!read(w[so + j], g)) return "fused scalar read before it is written";
  return "";
}

// A fused program (fused.hip's executor) against the LDS size and prepared
// input count of its plan; "" if it holds.
static std::string check_fused_program(const std::vector<uint32_t>& w, int64_t lds_bytes, int64_t elems,
                                       int64_t n_slices) {
  if (w.size() < (size_t)kHdr || w[FH_WORDS] != w.size() || w.size() % 4) return "fused header";
  const uint32_t nl = w[FH_LEVELS], nsc = w[FH_SCALARS], so = w[FH_SCALAR_OFF];
  const uint32_t inv = w[FH_INV_ELEMS], dep = w[FH_DEP_ELEMS], data = w[FH_DATA_ELEMS], nx = w[FH_EXPORTS],
                 ni = w[FH_IMPORTS];
  if (lds_bytes != std::max<int64_t>(fused_table_lds(data) + 16 * ((int64_t)nl + kFusedLevelPad + nx), 256 * 16))
    return "fused LDS size";
  if (nx > 0 && nsc > 0) return "fused program with both exports and scalars";
  if (ni > 0 && nx == 0) return "fused program with imports but no exports";
  if (lds_bytes > kFusedLdsMax) return "fused LDS above budget";
  if (w[FH_DEP_SRC] != inv) return "fused dependent block offset";
  if ((int64_t)inv + (int64_t)dep * n_slices != elems) return "fused prepared size";
  if (kFusedConsts + inv + dep > data) return "fused inputs above data size";
  if ((int64_t)kHdr + 4 * ((int64_t)nl + kFusedLevelPad + nx + ni) > (int64_t)w.size())
    return "fused level table truncated";
  if ((int64_t)so + nsc > (int64_t)w.size()) return "fused scalar list truncated";
  const uint32_t* lv = w.data() + kHdr;
  for (uint32_t j = 4 * nl; j < 4 * (nl + kFusedLevelPad); ++j)
    if (lv[j] != 0) return "fused level table end";
  // export rows after the table: LDS results of the program, copied
  // exactly once (counts of the levels' X fields plus the rows left for the
  // end); the arena side is checked by the plan
  const uint32_t* xr = lv + 4 * ((int64_t)nl + kFusedLevelPad);
  if ((kHdr + 4 * ((int64_t)nl + kFusedLevelPad)) % 4) return "fused export rows unaligned";
  // import rows after them: LDS slots the executor fills before the first
  // level, outside the input block it copies
  for (uint32_t e = 0; e < nx + ni; ++e) {
    const uint32_t src = xr[4 * e], rank = xr[4 * e + 1];
    if (rank > 15 || src < kFusedConsts || (int64_t)src + (int64_t(1) << rank) > data)
      return "fused export or import row outside its LDS data";
    if (e >= nx && src < kFusedConsts + inv + dep) return "fused import slot inside the input block";
  }
  int64_t x_copied = 0;
  int64_t expect_base = kHdr + 4 * ((int64_t)nl + kFusedLevelPad + nx + ni);
  const bool bytes = w[FH_BYTE_OFFSETS] != 0;
  if (w[FH_BYTE_OFFSETS] > 1 || bytes != ((int64_t)data * 8 <= 65536)) return "fused offset unit";
  const uint32_t unit = bytes ? 8u : 1u;
  // results may take the space of inputs their level no longer needs (any
  // slot above the constants); 16-bit slots must reach all the data
  const uint32_t data_hi = data * unit;
  if (data_hi > 65536) return "fused offsets above 16 bits";
  // levels the executor runs without a barrier between them (flag C): the
  // group's reads (its operands and the export rows it copies) and writes
  // (its results) must be disjoint, and each result written once
  std::vector<char> wrote(data, 0);
  std::vector<uint32_t> g_reads, g_writes;
  bool cont_prev = false;
  for (uint32_t l = 0; l < nl; ++l) {
    const uint32_t base = lv[4 * l], E = lv[4 * l + 1], R = lv[4 * l + 2] & 0xFFFFu,
                   lgT = (lv[4 * l + 2] >> 16) & 0xFFu, flags = lv[4 * l + 2] >> 24, K = lv[4 * l + 3] & 0xFFFFu,
                   X = lv[4 * l + 3] >> 16;
    const uint32_t C = flags & kLevelCont;
    const bool wide = (flags & kLevelWide) != 0;
    if (base != expect_base) return fail("fused record base", base, expect_base);
    if ((flags & ~(kLevelCont | kLevelWide)) || (C && l + 1 == nl)) return "fused level flags";
    if (wide && (K > kWideOpsMax || R != 1 || !(lgT == 1 || ((int64_t)E << lgT) <= kFusedBlock)))
      return "fused wide level not of at most three factors in one pass";
    if (cont_prev && X) return "fused level copies export rows without a barrier before it";
    for (int64_t e = x_copied; e < x_copied + X && e < nx; ++e)
      for (uint32_t i = 0; i < (1u << xr[4 * e + 1]); ++i) g_reads.push_back(xr[4 * e] + i);
    x_copied += X;
    if (x_copied > nx) return "fused level copies more export rows than the program holds";
    if (base % 4 || R != (1 + K + 7) / 8 || E == 0 || K == 0 || lgT < 1 || lgT > 3) return "fused level shape";
    if (lgT > 1 && ((int64_t)E << lgT) > kFusedBlock) return "fused level of many terms above the workgroup";
    const uint32_t T = 1u << lgT;
    if ((int64_t)base + (int64_t)E * T * 4 * R > (int64_t)w.size()) return "fused records truncated";
    for (uint32_t f = 0; f < E; ++f)
      for (uint32_t t = 0; t < T; ++t) {
        const uint32_t* rec = w.data() + base + ((size_t)f * T + t) * 4 * R;
        // slot j: 16-bit (element or byte offsets), or 32-bit bytes on a
        // wide level
        const uint32_t su = wide ? 8u : unit, n_slots = wide ? 4 * R : 8 * R;
        const uint64_t s_hi = wide ? (uint64_t)data * 8 : data_hi;
        auto hw = [&](uint32_t j) { return wide ? rec[j] : (rec[j / 2] >> (16 * (j % 2))) & 0xFFFFu; };
        if (t == 0) {
          const uint32_t out = hw(0);
          if (out % su || out < kFusedConsts * su || out >= s_hi) return "fused result outside the arena";
          g_writes.push_back(out / su);
        } else if (hw(0) != 0) {
          return "fused term's result slot not zero";
        }
        for (uint32_t j = 1; j < n_slots; ++j) {
          const uint32_t v = hw(j);
          if (v % su || v >= s_hi) return "fused operand outside LDS data";
          if (j > K && v != 0) return "fused padding slot not the constant";
          if (j <= K) g_reads.push_back(v / su);
        }
      }
    expect_base += (int64_t)E * T * 4 * R;
    cont_prev = C != 0;
    if (!cont_prev) {
      for (uint32_t v : g_writes) {
        if (wrote[v]) return "fused result written twice between barriers";
        wrote[v] = 1;
      }
      for (uint32_t v : g_reads)
        if (v < data && wrote[v]) return "fused level reads a result written without a barrier between";
      for (uint32_t v : g_writes) wrote[v] = 0;
      g_reads.clear();
      g_writes.clear();
    }
  }
  if (expect_base != so) return "fused scalar list offset";
  (void)x_copied;  // the rest of the rows are copied after the last level
  if ((int64_t)(so + nsc + 3) / 4 * 4 + 4 * kFusedTailRows != (int64_t)w.size()) return "fused program tail";
  for (size_t j = so + nsc; j < w.size(); ++j)
    if (w[j] != 0) return "fused program tail not zero";
  for (uint32_t j = 0; j < nsc; ++j)
    if (w[so + j] >= data) return "fused scalar outside LDS data";
  return check_fused_liveness(w, nl, nx, ni, xr, unit, data);
}

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
    if (sum_u ? (sp.n_sum < 1 || sp.n_sum > 4) : sp.n_sum != 0) return "summed variable count";
    const int xbits = r + sp.n_sum;
    if (r > 30 || xbits > 31) return "result rank above 30";
    if (sp.n_sum > 1) {
      // the multi-term kernel's summed-value bits: a permutation
      uint32_t seen = 0;
      for (int b = 0; b < sp.n_sum; ++b) {
        if (sp.sum_bit[b] < 0 || sp.sum_bit[b] >= sp.n_sum) return "summed bit order";
        seen |= 1u << sp.sum_bit[b];
      }
      if (seen + 1 != (1u << sp.n_sum)) return "summed bit order";
    }
    if (sp.mmk) {
      // the merged MFMA kernel's assumptions
      const uint32_t xm = (1u << r) - 1u;
      if (sp.n_sum < 2 || sp.n_sum > 4 || r < 8 || sp.mm_a >= 0) return "merged product shape";
      if (sp.mmk_side == 0 || (sp.mmk_side >> sp.n_ops) != 0 || sp.mmk_side + 1 == (1u << sp.n_ops))
        return "merged product groups";
      uint32_t xa = 0, xb = 0;
      for (int i = 0; i < sp.n_ops; ++i) ((sp.mmk_side >> i) & 1u ? xb : xa) |= sp.ops[i].mask & xm;
      if (__builtin_popcount(xa & ~xb) < 4 || __builtin_popcount(xb & ~xa) < 4)
        return "merged product tile needs four private bits per group";
    }
    if (sp.mm_a >= 0 && sp.n_sum == 1) {
      // the MFMA tile kernel's assumptions
      if (!sum_u || r < 8 || sp.mm_b < 0 || sp.mm_a == sp.mm_b || sp.mm_a >= sp.n_ops || sp.mm_b >= sp.n_ops)
        return "outer-product bucket shape";
      const uint32_t ubit = 1u << r, xm = ubit - 1u;
      const uint32_t ma = sp.ops[sp.mm_a].mask, mb = sp.ops[sp.mm_b].mask;
      if (!(ma & ubit) || !(mb & ubit)) return "outer-product operand without u";
      if (((ma | mb) & xm) != xm) return "outer-product result variable outside A and B";
      if (__builtin_popcount(ma & ~mb & xm) < 4 || __builtin_popcount(mb & ~ma & xm) < 4)
        return "outer-product tile needs four private variables per side";
      for (int i = 0; i < sp.n_ops; ++i)
        if (i != sp.mm_a && i != sp.mm_b && (sp.ops[i].mask != ubit || sp.ops[i].rank != 1))
          return "outer-product extra operand not a rank-1 tensor on u";
    }
    for (int i = 0; i < sp.n_ops; ++i) {
      const StepOp& o = sp.ops[i];
      if (__builtin_popcount(o.mask) != o.rank) return "operand mask and rank disagree";
      if (xbits < 32 && (o.mask >> xbits) != 0) return "operand mask outside the union index";
      // one summed bit: an operand without it lies within x (a merged launch's
      // operands may hold any of its summed bits; the union bound covers them)
      if (sum_u && sp.n_sum == 1 && o.rank > 0 && !((o.mask >> r) & 1u) && o.rank > r) return "operand rank";
      if (sp.n_sum > 1 && (o.mask >> r) == 0 && o.rank > 0 && !o.is_input)
        return "merged launch with an intermediate that holds no summed variable";
      if (sp.n_sum > 1 && o.rank > kMergedMaxRank) return fail("merged launch operand rank", o.rank, kMergedMaxRank);
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
  // execution order: every step exactly once, alone or in one group whose
  // descriptor repeats the step's fields and whose tile prefix matches
  {
    std::vector<int> seen(p.steps.size(), 0);
    const int n_groups = (int)p.group_first.size() - 1;
    if (n_groups < 0 || p.group_first[0] != 0 || p.group_first.back() != (int32_t)p.group_steps.size())
      return "group table";
    if (p.group_prefix.size() != p.group_steps.size() + (size_t)n_groups) return "group prefix size";
    if (p.group_sb < 1 || p.group_sb > 256 || (p.group_sb & (p.group_sb - 1))) return "group slice block";
    for (const LaunchItem& li : p.launch_order) {
      if (li.seg >= 0) continue;  // checked with the segments below
      if (li.group < 0) {
        if (li.step < 0 || li.step >= (int)p.steps.size()) return "launch step index";
        ++seen[li.step];
        continue;
      }
      if (li.group >= n_groups) return "launch group index";
      const int f = p.group_first[li.group], e = p.group_first[li.group + 1];
      if (e - f < 2) return "group with fewer than two steps";
      uint32_t tiles = 0;
      if (p.group_prefix[f + li.group] != 0) return "group prefix start";
      for (int j = f; j < e; ++j) {
        const GroupStep& d = p.group_steps[j];
        if (d.step < 0 || d.step >= (int)p.steps.size()) return "group step index";
        ++seen[d.step];
        const StepProg& sp = p.steps[d.step];
        const int r = sp.out_rank >= 0 ? sp.out_rank : -sp.out_rank;
        if (d.r != r || d.r > kGroupMaxRank || d.sum_u != (sp.out_rank >= 0 ? 1 : 0) || d.n_ops != sp.n_ops ||
            d.out != sp.out_base || sp.n_sum > 1 || sp.mmk || sp.mm_a >= 0)
          return "group step fields";
        for (int i = 0; i < sp.n_ops; ++i) {
          const StepOp& o = sp.ops[i];
          if (d.base[i] != o.base || d.mask[i] != o.mask || d.rank[i] != o.rank ||
              (((d.is_input >> i) & 1u) != (uint32_t)o.is_input) || d.smask[i] != (o.is_input ? o.smask : 0u))
            return "group operand fields";
        }
        tiles += (uint32_t)((((int64_t)p.group_sb << d.r) + 255) / 256);
        if (p.group_prefix[j + 1 + li.group] != tiles) return "group prefix";
      }
    }
    for (int c : seen)
      if (c != 1) return "execution order misses or repeats a step";
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
    const std::string bad = check_fused_program(p.fused_prog, p.fused_lds_bytes, p.fused_elems, p.n_slices);
    if (!bad.empty()) return bad;
  }
  // fused segments: programs with no scalar list whose import and export
  // rows (copies kept in the segment) lie in the arena; the prefix imports
  // nothing; every segment is launched exactly once
  std::vector<int> seg_seen(p.segs.size(), 0);
  for (const LaunchItem& li : p.launch_order)
    if (li.seg >= 0) {
      if (li.seg >= (int)p.segs.size() || li.step != -1 || li.group != -1) return "launch segment index";
      ++seg_seen[li.seg];
    }
  for (size_t j = 0; j < p.segs.size(); ++j) {
    const FusedSeg& sg = p.segs[j];
    if (seg_seen[j] != 1) return "execution order misses or repeats a fused segment";
    for (size_t i = 0; i < sg.map.size(); ++i)
      if (sg.map[i] < 0 || sg.map[i] >= raw_elems) return fail("segment map entry out of range", sg.map[i], raw_elems);
    if ((int64_t)sg.map.size() != sg.elems) return "segment map size";
    const auto& w = sg.prog;
    const std::string bad = check_fused_program(w, sg.lds_bytes, sg.elems, p.n_slices);
    if (!bad.empty()) return "segment: " + bad;
    if (w[FH_SCALARS] != 0) return "segment with a scalar list";
    if (sg.exports.empty() || sg.exports.size() != 4 * (size_t)w[FH_EXPORTS]) return "segment export list";
    if (sg.imports.size() != 4 * (size_t)w[FH_IMPORTS]) return "segment import list";
    if (j == 0 && p.has_prefix && !sg.imports.empty()) return "prefix with imports";
    const size_t x_at = kHdr + 4 * ((size_t)w[FH_LEVELS] + kFusedLevelPad);
    const size_t i_at = x_at + sg.exports.size();
    if (i_at + sg.imports.size() > w.size() || !std::equal(sg.exports.begin(), sg.exports.end(), w.begin() + x_at) ||
        !std::equal(sg.imports.begin(), sg.imports.end(), w.begin() + i_at))
      return "segment rows differ from the program's";
    const int64_t lo = kFusedConsts, hi = w[FH_DATA_ELEMS];
    for (const std::vector<uint32_t>* rows : {&sg.exports, &sg.imports})
      for (size_t i = 0; i < rows->size(); i += 4) {
        const int64_t src = (*rows)[i], rank = (*rows)[i + 1];
        const int64_t off = (int64_t)(((uint64_t)(*rows)[i + 3] << 32) | (*rows)[i + 2]);
        if (rank > p.seg_max_rank + 1 || rank > 15) return "segment row above its rank bound";
        if (src < lo || src + (int64_t(1) << rank) > hi) return "segment row outside its LDS data";
        if (off < 0 || off + (int64_t(1) << rank) > p.arena_per_slice)
          return fail("segment row outside the arena", off + (int64_t(1) << rank), p.arena_per_slice);
      }
  }
  return "";
}

}  // namespace qbe
