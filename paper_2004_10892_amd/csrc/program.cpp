// Plan compiler: turns a bucket schedule into device programs.
//
// Layout decisions (host side; the device only moves and multiplies data):
//  * Every tensor's remaining variables are stored sorted by position in the
//    reduced order, earliest variable most significant.  The eliminated
//    variable u of bucket b is the earliest variable of U_b, so in the
//    bucket's union index X = (u << r_b) | x it is the top bit, and every
//    operand's index is the bit-extraction of X by the operand's mask.
//  * Input tensors are prepared on the device from the model's complex128
//    entries by a gather map computed here: per-step form -- one copy per
//    assignment of the tensor's own sliced variables; fused form -- a block
//    of slice-invariant tensors and one block per slice of the rest, so that
//    a workgroup fills its LDS with two contiguous copies.
//  * Intermediates live in an arena laid out by simulating the schedule
//    (first fit; per-slice units scaled by the slice-group size).
#include <algorithm>
#include <cstdint>
#include <map>
#include <stdexcept>

#include "qbe_internal.hpp"
#include "../../include/qbe.h"

namespace qbe {

namespace {

struct Arena {
  // free list of [begin, end) in elements
  std::map<int64_t, int64_t> free_;  // begin -> end
  int64_t top = 0;
  int64_t alloc(int64_t size, int64_t align) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      int64_t b = (it->first + align - 1) / align * align;
      if (b + size <= it->second) {
        int64_t e = it->second, s0 = it->first;
        free_.erase(it);
        if (s0 < b) free_[s0] = b;
        if (b + size < e) free_[b + size] = e;
        return b;
      }
    }
    int64_t b = (top + align - 1) / align * align;
    if (top < b) release(top, b - top);
    top = b + size;
    return b;
  }
  void release(int64_t b, int64_t size) {
    int64_t e = b + size;
    auto nx = free_.lower_bound(b);
    if (nx != free_.end() && nx->first == e) {
      e = nx->second;
      free_.erase(nx);
    }
    auto pv = free_.lower_bound(b);
    if (pv != free_.begin()) {
      --pv;
      if (pv->second == b) {
        b = pv->first;
        free_.erase(pv);
      }
    }
    free_[b] = e;
  }
};

int64_t align_for(int64_t size) { return std::min<int64_t>(64, size); }

// Mask of `vars` (sorted by position) inside the union `uni` (sorted by
// position, uni[0] is the top bit).
uint32_t union_mask(const std::vector<int>& uni, const std::vector<int>& vars) {
  uint32_t m = 0;
  const int nu = (int)uni.size();
  for (int v : vars) {
    auto it = std::find(uni.begin(), uni.end(), v);
    if (it == uni.end()) throw std::logic_error("operand variable outside its bucket");
    m |= 1u << (nu - 1 - (int)(it - uni.begin()));
  }
  return m;
}

struct InputInfo {
  std::vector<int> canon;     // remaining variables sorted by position
  std::vector<int> slice_js;  // mu indices j of the tensor's sliced variables (ascending)
  uint32_t smask = 0;
};

// Raw (model) element index of tensor t for an assignment given as a
// function of the variable.
template <class F>
int64_t raw_index(const Model& md, int t, F&& value_of) {
  const auto& vs = md.tvars[t];
  const int r = (int)vs.size();
  int64_t idx = 0;
  for (int j = 0; j < r; ++j) idx |= (int64_t)value_of(vs[j]) << (r - 1 - j);
  return md.data_off[t] + idx;
}

// A node of the fused program: a root bucket (members[0]) and the buckets it
// absorbed.  One record per entry of the root's result sums over the
// eliminated variables of all members (2^|members| terms); a term multiplies
// the members' operands other than the absorbed members' results.  Every
// member's variable occurs only in its own bucket's operands, and an
// absorbed member's other variables are all in the root's union, so each
// factor is indexed by the root's result variables and the summed ones.
struct FusedNode {
  std::vector<int> members;      // root first, then absorbed buckets
  std::vector<Operand> factors;  // operands of the members except absorbed results
  std::vector<int> kids;         // buckets (node roots) whose results it reads
  int level = 0;                 // dependency depth among nodes
};

// Fused form: merges buckets along the dependency tree to shorten the chain
// of levels.  A bucket absorbs its producer when that producer is its only
// deepest input, the merged record stays within kMergeTermsLog2 summed
// variables and kMergeFactors factors, no level deepens, and every level
// with more than two terms per entry still gives each term its own lane.
constexpr int kMergeTermsLog2 = 3;
constexpr int kMergeFactors = 15;

std::vector<FusedNode> merge_buckets(const Schedule& s, bool merge, const std::vector<char>& incl) {
  const int n = (int)s.steps.size();
  std::vector<std::vector<int>> kids(n), members(n);
  std::vector<int> F(n), lgT(n, 1), lv(n, 0);
  std::vector<int64_t> E(n);
  std::vector<char> alive(incl);
  for (int k = 0; k < n; ++k) {
    for (const auto& op : s.steps[k].ops)
      if (op.kind == 'r' && incl[op.id]) kids[k].push_back(op.id);  // others: imported results
    members[k] = {k};
    F[k] = (int)s.steps[k].ops.size();
    E[k] = int64_t(1) << s.steps[k].out.size();
  }
  auto levels = [&]() {  // steps are in dependency order
    int depth = 0;
    for (int k = 0; k < n; ++k)
      if (alive[k]) {
        int l = 0;
        for (int c : kids[k]) l = std::max(l, lv[c] + 1);
        lv[k] = l;
        depth = std::max(depth, l + 1);
      }
    return depth;
  };
  auto fits = [&](int depth) {
    std::vector<int64_t> el(depth, 0);
    std::vector<int> tl(depth, 1);
    for (int k = 0; k < n; ++k)
      if (alive[k]) {
        el[lv[k]] += E[k];
        tl[lv[k]] = std::max(tl[lv[k]], lgT[k]);
      }
    for (int l = 0; l < depth; ++l)
      if (tl[l] > 1 && (el[l] << tl[l]) > kFusedBlock) return false;
    return true;
  };
  int depth = levels();
  for (bool merged = merge; merged;) {
    merged = false;
    std::vector<int> order;
    for (int k = 0; k < n; ++k)
      if (alive[k]) order.push_back(k);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return lv[a] > lv[b]; });
    for (int c : order) {
      int top = -1, k = -1, ntop = 0;
      for (int x : kids[c]) {
        if (lv[x] > top) {
          top = lv[x];
          k = x;
          ntop = 1;
        } else if (lv[x] == top) {
          ++ntop;
        }
      }
      if (ntop != 1 || lgT[c] + lgT[k] > kMergeTermsLog2 || F[c] + F[k] - 1 > kMergeFactors) continue;
      const std::vector<int> kids_c = kids[c], lv_c = lv;
      kids[c].erase(std::find(kids[c].begin(), kids[c].end(), k));
      kids[c].insert(kids[c].end(), kids[k].begin(), kids[k].end());
      lgT[c] += lgT[k];
      F[c] += F[k] - 1;
      alive[k] = 0;
      const int d2 = levels();
      if (d2 <= depth && fits(d2)) {
        members[c].insert(members[c].end(), members[k].begin(), members[k].end());
        depth = d2;
        merged = true;
        break;
      }
      kids[c] = kids_c;
      lgT[c] -= lgT[k];
      F[c] -= F[k] - 1;
      alive[k] = 1;
      lv = lv_c;
    }
  }
  std::vector<FusedNode> nodes;
  for (int k = 0; k < n; ++k) {
    if (!alive[k]) continue;
    FusedNode nd;
    nd.members = members[k];
    for (int m : nd.members)
      for (const auto& op : s.steps[m].ops)
        if (!(op.kind == 'r' && std::find(nd.members.begin(), nd.members.end(), op.id) != nd.members.end()))
          nd.factors.push_back(op);
    if ((int)nd.factors.size() != F[k]) throw std::logic_error("fused node factor count");
    nd.kids = kids[k];
    nd.level = lv[k];
    nodes.push_back(std::move(nd));
  }
  return nodes;
}

// Per-step form: a bucket whose result is at least as large as its
// consumer's (a shrinking chain) and of rank kChainMinRank or more is merged
// into the consumer, so that one launch sums several variables and the
// absorbed result never goes to device memory.  Up to kChainSumMax summed
// variables, kMaxOps operands and operands of rank kMergedMaxRank per launch.
constexpr int kChainMinRank = 12;
// Results of this rank or less are not placed in reused arena space (their
// total is small; see compile_plan).
constexpr int kOwnSpaceRank = 8;
constexpr int kChainSumMax = 4;
// A later fused segment takes a run of at least this many buckets: a
// shorter run saves fewer launches than its levels cost.
constexpr int kSegMinBuckets = 3;

struct StepNode {
  std::vector<int> members;      // absorbed buckets in elimination order, root last
  std::vector<Operand> factors;  // operands of the members except absorbed results
};

std::vector<StepNode> merge_chains(const Schedule& s, bool merge, const std::vector<char>& skip, int max_sums) {
  const int n = (int)s.steps.size();
  std::vector<StepNode> nd(n);
  std::vector<char> alive(n, 1);
  for (int k = 0; k < n; ++k) {
    nd[k].members = {k};
    nd[k].factors = s.steps[k].ops;
    if (skip[k]) alive[k] = 0;  // runs in a fused segment
  }
  for (int k = 0; k < n && merge; ++k) {
    const int c = s.consumer[k];
    // a consumer in a fused segment reads k's result from the arena
    if (c < 0 || !alive[k] || skip[c]) continue;
    const int rk = (int)s.steps[k].out.size(), rc = (int)s.steps[c].out.size();
    if (rk < kChainMinRank || rk < rc) continue;
    if ((int)(nd[k].members.size() + nd[c].members.size()) > std::min(max_sums, kChainSumMax)) continue;
    std::vector<Operand> f;
    for (const Operand& op : nd[c].factors)
      if (!(op.kind == 'r' && op.id == k)) f.push_back(op);
    f.insert(f.end(), nd[k].factors.begin(), nd[k].factors.end());
    if ((int)f.size() > kMaxOps) continue;
    bool narrow = true;
    for (const Operand& op : f) narrow = narrow && (int)op.vars.size() <= kMergedMaxRank;
    if (!narrow) continue;
    std::vector<int> m = nd[k].members;
    m.insert(m.end(), nd[c].members.begin(), nd[c].members.end());
    nd[c].members = std::move(m);
    nd[c].factors = std::move(f);
    alive[k] = 0;
  }
  std::vector<StepNode> out;
  for (int k = 0; k < n; ++k)
    if (alive[k]) out.push_back(std::move(nd[k]));
  return out;
}

}  // namespace

bool groupable(const StepProg& sp) { return sp.n_sum <= 1 && !sp.mmk && sp.mm_a < 0; }

GroupStep group_step_of(const StepProg& sp, int k) {
  GroupStep d{};
  d.out = sp.out_base;
  d.n_ops = sp.n_ops;
  d.r = sp.out_rank >= 0 ? sp.out_rank : -sp.out_rank;
  d.sum_u = sp.out_rank >= 0 ? 1 : 0;
  d.step = k;
  for (int i = 0; i < sp.n_ops; ++i) {
    d.base[i] = sp.ops[i].base;
    d.mask[i] = sp.ops[i].mask;
    d.smask[i] = sp.ops[i].is_input ? sp.ops[i].smask : 0u;
    d.rank[i] = sp.ops[i].rank;
    if (sp.ops[i].is_input) d.is_input |= 1u << i;
  }
  return d;
}

namespace {

// Execution order of the per-step launches.  A launch's level is one more
// than that of every earlier launch it must follow: the producers of its
// operands, and -- because the arena reuses space -- earlier launches that
// read or write the space it writes.  Launches of one level are independent;
// the small ones (no merged or MFMA form, result rank <= kGroupMaxRank) of a
// level run together in one group launch when there are at least two.
void build_launch_order(Plan& p) {
  p.launch_order.clear();
  p.group_steps.clear();
  p.group_first.assign(1, 0);
  p.group_prefix.clear();
  const int n = (int)p.steps.size();
  int64_t sb = 1;
  while (sb < 256 && sb < p.n_slices) sb <<= 1;
  p.group_sb = (int32_t)sb;
  p.step_level.assign(n, 0);
  if (!p.merge) {
    // plain form: one launch per bucket, in schedule order
    for (int k = 0; k < n; ++k) {
      p.launch_order.push_back(LaunchItem{k, -1});
      p.step_level[k] = k;
    }
    return;
  }
  // units in schedule order: each fused segment before the step at its
  // position, then that step; unit u >= 0 is step u, u < 0 segment -1 - u
  std::vector<int> units;
  for (int k = 0; k <= n; ++k) {
    for (size_t j = 0; j < p.segs.size(); ++j)
      if (p.segs[j].pos == k) units.push_back(-1 - (int)j);
    if (k < n) units.push_back(k);
  }
  struct Span {
    int64_t b, e;
  };
  auto rank_of = [](const StepProg& sp) { return sp.out_rank >= 0 ? sp.out_rank : -sp.out_rank; };
  auto row_spans = [](const std::vector<uint32_t>& rows) {
    std::vector<Span> v;
    for (size_t i = 0; i < rows.size(); i += 4) {
      const int64_t off = (int64_t)(((uint64_t)rows[i + 3] << 32) | rows[i + 2]);
      v.push_back(Span{off, off + (int64_t(1) << rows[i + 1])});
    }
    return v;
  };
  const int nu = (int)units.size();
  std::vector<std::vector<Span>> wr(nu), rd(nu);
  for (int u = 0; u < nu; ++u) {
    if (units[u] < 0) {
      const FusedSeg& sg = p.segs[-1 - units[u]];
      wr[u] = row_spans(sg.exports);
      rd[u] = row_spans(sg.imports);
      continue;
    }
    const StepProg& sp = p.steps[units[u]];
    wr[u].push_back(Span{sp.out_base, sp.out_base + (int64_t(1) << rank_of(sp))});
    for (int i = 0; i < sp.n_ops; ++i)
      if (!sp.ops[i].is_input) rd[u].push_back(Span{sp.ops[i].base, sp.ops[i].base + (int64_t(1) << sp.ops[i].rank)});
  }
  auto meet = [](const Span& a, const Span& b) { return a.b < b.e && b.b < a.e; };
  auto meets = [&](const std::vector<Span>& x, const std::vector<Span>& y) {
    for (const Span& a : x)
      for (const Span& b : y)
        if (meet(a, b)) return true;
    return false;
  };
  // level of a unit: one above every earlier unit it has a memory hazard
  // with (it reads what that one writes, writes what it reads or writes)
  std::vector<int> level(nu, 0);
  int n_lv = 0;
  for (int u = 0; u < nu; ++u) {
    int l = 0;
    for (int v = 0; v < u; ++v)
      if (meets(wr[v], wr[u]) || meets(wr[v], rd[u]) || meets(rd[v], wr[u])) l = std::max(l, level[v] + 1);
    level[u] = l;
    n_lv = std::max(n_lv, l + 1);
  }
  for (int u = 0; u < nu; ++u) {
    if (units[u] >= 0)
      p.step_level[units[u]] = level[u];
    else
      p.segs[-1 - units[u]].level = level[u];
  }
  auto small = [&](const StepProg& sp) { return groupable(sp) && rank_of(sp) <= kGroupMaxRank; };
  for (int l = 0; l < n_lv; ++l) {
    std::vector<int> grp;
    for (int u = 0; u < nu; ++u) {
      if (level[u] != l) continue;
      if (units[u] < 0) {
        p.launch_order.push_back(LaunchItem{-1, -1, -1 - units[u]});
        continue;
      }
      const int k = units[u];
      if (small(p.steps[k]))
        grp.push_back(k);
      else
        p.launch_order.push_back(LaunchItem{k, -1});
    }
    if (grp.size() == 1) p.launch_order.push_back(LaunchItem{grp[0], -1});
    if (grp.size() < 2) continue;
    const int g = (int)p.group_first.size() - 1;
    uint32_t tiles = 0;
    p.group_prefix.push_back(0);
    for (int k : grp) {
      const GroupStep d = group_step_of(p.steps[k], k);
      p.group_steps.push_back(d);
      tiles += (uint32_t)(((sb << d.r) + 255) / 256);
      p.group_prefix.push_back(tiles);
    }
    p.group_first.push_back((int32_t)p.group_steps.size());
    p.launch_order.push_back(LaunchItem{-1, g});
  }
}

}  // namespace

// A fused program (the executor of fused.hip) for the buckets in `incl`.
// Without exports it is the whole schedule: the program ends with the
// slice's scalar factors.  With exports (marks per bucket, >= 0 for the
// results other launches read) it is a segment of a per-step plan: the
// marked results are copied from LDS to the per-step arena, the results of
// excluded buckets that included ones read are imported from it, and no
// scalar list follows (arena offsets of both rows are set by the caller).
struct FusedCode {
  bool ok = false;
  std::vector<uint32_t> prog;
  std::vector<int32_t> map;
  int lds_bytes = 0, levels = 0;
  size_t export_at = 0, import_at = 0;  // words of the first export and import rows
  std::vector<int> export_steps;        // the bucket of each export row
  std::vector<int> import_steps;        // the (excluded) bucket of each import row
};

static FusedCode build_fused(const Plan& p, const std::vector<InputInfo>& in, const std::vector<int>& muj,
                             const std::vector<char>& incl, const std::vector<int64_t>* export_off,
                             int64_t lds_cap = kFusedLdsMax) {
  const Model& md = p.model;
  const Schedule& s = p.sched;
  const int nt = (int)md.tvars.size();
  const int nsteps = (int)s.steps.size();
  FusedCode out;
  // the inputs the included buckets read
  std::vector<char> used(nt, export_off ? 0 : 1);
  if (export_off)
    for (int k = 0; k < nsteps; ++k)
      if (incl[k])
        for (const auto& op : s.steps[k].ops)
          if (op.kind == 't') used[op.id] = 1;
  // LDS element offsets (after the constants 1 and 0): the inputs first,
  // one contiguous block, slice-invariant ones first, as the executor copies
  // them in
  std::vector<int64_t> lds_in(nt, -1);
  int64_t inv = 0, dep = 0;
  for (int t = 0; t < nt; ++t)
    if (used[t] && in[t].smask == 0) {
      lds_in[t] = kFusedConsts + inv;
      inv += int64_t(1) << in[t].canon.size();
    }
  for (int t = 0; t < nt; ++t)
    if (used[t] && in[t].smask != 0) {
      lds_in[t] = kFusedConsts + inv + dep;
      dep += int64_t(1) << in[t].canon.size();
    }
  // merged nodes (each writes its root bucket's result) and their levels
  const std::vector<FusedNode> nodes = merge_buckets(s, p.merge, incl);
  int f_levels = 0;
  for (const FusedNode& nd : nodes) f_levels = std::max(f_levels, nd.level + 1);
  std::vector<std::vector<int>> by_level(f_levels);
  for (int i = 0; i < (int)nodes.size(); ++i) by_level[nodes[i].level].push_back(i);
  // exports (segment programs): results no included bucket reads, in the
  // order of their nodes' levels; those of level l are copied out as level
  // l + 1 starts (the last level's after it)
  std::vector<int> exp_steps;
  std::vector<int> exp_level;
  if (export_off)
    for (int l = 0; l < f_levels; ++l)
      for (int i : by_level[l]) {
        const int c = nodes[i].members[0];
        if ((*export_off)[c] >= 0) {
          exp_steps.push_back(c);
          exp_level.push_back(l);
        }
      }
  // imports (segment programs): results of excluded buckets that included
  // ones read, copied in with the inputs
  std::vector<int64_t> lds_out(nsteps, -1);
  std::vector<int> imp_steps;
  if (export_off)
    for (int k = 0; k < nsteps; ++k)
      if (incl[k])
        for (const auto& op : s.steps[k].ops)
          if (op.kind == 'r' && !incl[op.id]) imp_steps.push_back(op.id);
  // Lifetimes in levels (-1: before the first, f_levels: after the last):
  // an input or import lives from the start through the level of the node
  // that reads it, a result from its node's level through its reader's (an
  // exported one through the next level, which copies it out; one read at
  // the end, through f_levels).  A level's results are written while its
  // operands are still read, so the two lifetimes overlap at that level.
  std::vector<int> in_to(nt, f_levels), res_to(nsteps, f_levels);
  for (const FusedNode& nd : nodes) {
    for (int kid : nd.kids) res_to[kid] = nd.level;
    for (const Operand& op : nd.factors) {
      if (op.kind == 't') in_to[op.id] = nd.level;
      if (op.kind == 'r' && !incl[op.id]) res_to[op.id] = nd.level;
    }
  }
  for (size_t e = 0; e < exp_steps.size(); ++e) res_to[exp_steps[e]] = std::min(exp_level[e] + 1, f_levels);
  // Offline placement of imports and results around the fixed input block:
  // largest first (earlier first on ties), each at the lowest offset that
  // no item living at the same time uses.
  struct Span {
    int64_t off, size;
    int from, to;
  };
  std::vector<Span> placed;
  for (int t = 0; t < nt; ++t)
    if (used[t]) placed.push_back({lds_in[t] - kFusedConsts, int64_t(1) << in[t].canon.size(), -1, in_to[t]});
  struct Want {
    int64_t size;
    int from, to, step;
  };
  std::vector<Want> want;
  for (int c : imp_steps) want.push_back({int64_t(1) << s.steps[c].out.size(), -1, res_to[c], c});
  for (const FusedNode& nd : nodes) {
    const int c = nd.members[0];
    want.push_back({int64_t(1) << s.steps[c].out.size(), nd.level, res_to[c], c});
  }
  std::stable_sort(want.begin(), want.end(), [](const Want& x, const Want& y) {
    return x.size != y.size ? x.size > y.size : x.from < y.from;
  });
  std::vector<std::pair<int64_t, int64_t>> busy;
  for (const Want& w : want) {
    busy.clear();
    for (const Span& q : placed)
      if (q.from <= w.to && w.from <= q.to) busy.push_back({q.off, q.off + q.size});
    std::sort(busy.begin(), busy.end());
    int64_t at = 0;
    for (const auto& iv : busy) {
      if (at + w.size <= iv.first) break;
      at = std::max(at, iv.second);
    }
    placed.push_back({at, w.size, w.from, w.to});
    lds_out[w.step] = kFusedConsts + at;
  }
  int64_t top = inv + dep;
  for (const Span& q : placed) top = std::max(top, q.off + q.size);
  const int64_t data_elems = kFusedConsts + top;
  // each level's factors F, terms T and entries E; a prefix program splits
  // its levels into one-pass parts (their records all read ahead), as many
  // slices run it at once and a level's extra record reads would stall them
  std::vector<uint32_t> lvF(f_levels, 1), lvT(f_levels, 2);
  std::vector<int64_t> lvE(f_levels, 0), lvCap(f_levels);
  int64_t n_table = 0;
  for (int l = 0; l < f_levels; ++l) {
    for (int i : by_level[l]) {
      lvF[l] = std::max<uint32_t>(lvF[l], (uint32_t)nodes[i].factors.size());
      lvT[l] = std::max<uint32_t>(lvT[l], 2u << (nodes[i].members.size() - 1));
      lvE[l] += int64_t(1) << s.steps[nodes[i].members[0]].out.size();
    }
    lvCap[l] = export_off ? fused_pass_entries((uint32_t)__builtin_ctz(lvT[l]), lvF[l]) : lvE[l];
    n_table += (lvE[l] + lvCap[l] - 1) / lvCap[l];
  }
  // LDS: the tensor entries, then a copy of the level table and export rows
  const int64_t n_exp = (int64_t)exp_steps.size();
  const int64_t lds_bytes =
      std::max<int64_t>(fused_table_lds(data_elems) + 16 * (n_table + kFusedLevelPad + n_exp), 256 * 16);
  const int64_t prep_elems = inv + dep * p.n_slices;
  // (a whole-schedule program may have no levels: every variable sliced)
  if ((export_off && f_levels == 0) || lds_bytes > lds_cap || prep_elems >= (int64_t(1) << 31)) return out;
  std::vector<uint32_t> prog(kHdr, 0);
  const size_t lvl_at = prog.size();
  // zero entries after the last level end the executor's look-ahead
  prog.resize(lvl_at + 4 * ((size_t)n_table + kFusedLevelPad), 0);
  while (prog.size() % 4) prog.push_back(0);
  // export rows (arena offsets are set once the per-step arena is placed)
  out.export_at = prog.size();
  for (int64_t e = 0; e < n_exp; ++e) {
    const int c = exp_steps[e];
    prog.insert(prog.end(), {0u, (uint32_t)s.steps[c].out.size(), 0u, 0u});
  }
  out.export_steps = exp_steps;
  // import rows (read from device memory before the first level)
  out.import_at = prog.size();
  for (int c : imp_steps)
    prog.insert(prog.end(), {(uint32_t)lds_out[c], (uint32_t)s.steps[c].out.size(), 0u, 0u});
  out.import_steps = imp_steps;
  // 16-bit operand offsets: bytes when the data fit 64 KB, else elements
  const bool bytes = data_elems * 8 <= 65536;
  const uint32_t unit = bytes ? 8u : 1u;
  std::vector<int> val(md.n_vars, -1);  // variable values of the record being written
  size_t tab = 0;                       // next level-table entry
  for (int l = 0; l < f_levels; ++l) {
    const uint32_t F = lvF[l], T = lvT[l];
    const int64_t E = lvE[l], cap = lvCap[l];
    const uint32_t R = (1 + F + 7) / 8;  // 16-byte rows of a term record
    int64_t done = 0;                    // entries of the level written
    bool wide = false;                   // the current part's slots are 32-bit
    uint32_t X = 0;                      // exports of the previous level
    for (int64_t e = 0; e < n_exp; ++e) X += exp_level[e] == l - 1;
    for (int i : by_level[l]) {
      const FusedNode& nd = nodes[i];
      const Step& root = s.steps[nd.members[0]];
      const int r = (int)root.out.size();
      const uint32_t Tn = 2u << (nd.members.size() - 1);
      for (uint32_t x = 0; x < (1u << r); ++x, ++done) {
        if (done % cap == 0) {
          // a later part of the level: the part before it runs on without
          // a barrier (both read earlier levels only and write fresh space)
          if (done > 0) prog[lvl_at + 4 * (tab - 1) + 2] |= kLevelCont << 24;
          const int64_t part = std::min(cap, E - done);
          wide = F <= kWideOpsMax && (T == 2 || part * T <= kFusedBlock);
          prog[lvl_at + 4 * tab + 0] = (uint32_t)prog.size();
          prog[lvl_at + 4 * tab + 1] = (uint32_t)part;
          prog[lvl_at + 4 * tab + 2] = R | ((uint32_t)__builtin_ctz(T) << 16) | (wide ? kLevelWide << 24 : 0u);
          prog[lvl_at + 4 * tab + 3] = F | (done == 0 ? X << 16 : 0u);
          ++tab;
        }
        // T term records of 8R halfwords (4R words on a wide level):
        // [result (term 0) or 0, the factors' entries for that assignment
        // of the summed variables]
        for (uint32_t t = 0; t < T; ++t) {
          const size_t at = prog.size();
          prog.resize(at + 4 * R, 0);
          auto put = [&](uint32_t j, uint32_t v) {
            if (wide)
              prog[at + j] = v * 8u;
            else
              prog[at + j / 2] |= (v * unit) << (16 * (j % 2));
          };
          if (t == 0) put(0, (uint32_t)(lds_out[nd.members[0]] + x));
          if (t >= Tn) {
            put(1, kFusedZero);  // padding term: a factor 0
            continue;
          }
          for (int q = 0; q < r; ++q) val[root.out[q]] = (int)((x >> (r - 1 - q)) & 1);
          for (size_t j = 0; j < nd.members.size(); ++j) val[s.steps[nd.members[j]].var] = (int)((t >> j) & 1);
          for (size_t f = 0; f < nd.factors.size(); ++f) {
            const Operand& op = nd.factors[f];
            const std::vector<int>& vars = op.kind == 't' ? in[op.id].canon : op.vars;
            uint32_t e = 0;
            for (int v : vars) {
              if (val[v] < 0) throw std::logic_error("fused node factor outside its variables");
              e = (e << 1) | (uint32_t)val[v];
            }
            const int64_t base = op.kind == 't' ? lds_in[op.id] : lds_out[op.id];
            put(1 + (uint32_t)f, (uint32_t)(base + e));
          }
          for (int q = 0; q < r; ++q) val[root.out[q]] = -1;
          for (size_t j = 0; j < nd.members.size(); ++j) val[s.steps[nd.members[j]].var] = -1;
        }
      }
    }
  }
  prog[FH_BYTE_OFFSETS] = bytes ? 1u : 0u;
  const uint32_t scal_at = (uint32_t)prog.size();
  uint32_t n_scal = 0;
  if (!export_off) {
    for (int t : s.scalar_inputs) {
      prog.push_back((uint32_t)lds_in[t]);
      ++n_scal;
    }
    for (int k : s.scalar_steps) {
      prog.push_back((uint32_t)lds_out[k]);
      ++n_scal;
    }
  } else {
    for (int64_t e = 0; e < n_exp; ++e) {
      if (lds_out[exp_steps[e]] < 0) throw std::logic_error("exported bucket without a result");
      prog[out.export_at + 4 * e] = (uint32_t)lds_out[exp_steps[e]];
    }
  }
  while (prog.size() % 4) prog.push_back(0);
  prog.resize(prog.size() + 4 * kFusedTailRows, 0);  // the executor reads whole row groups
  if ((int64_t)tab != n_table) throw std::logic_error("fused level table count");
  prog[FH_WORDS] = (uint32_t)prog.size();
  prog[FH_LEVELS] = (uint32_t)n_table;
  prog[FH_SCALARS] = n_scal;
  prog[FH_SCALAR_OFF] = scal_at;
  prog[FH_FREE] = (uint32_t)s.free_vars.size();
  prog[FH_INV_ELEMS] = (uint32_t)inv;
  prog[FH_DEP_ELEMS] = (uint32_t)dep;
  prog[FH_DATA_ELEMS] = (uint32_t)data_elems;
  prog[FH_DEP_SRC] = (uint32_t)inv;
  prog[FH_N_SLICES] = (uint32_t)std::min<int64_t>(p.n_slices, UINT32_MAX);
  prog[FH_EXPORTS] = (uint32_t)n_exp;
  prog[FH_IMPORTS] = (uint32_t)imp_steps.size();
  out.ok = true;
  out.lds_bytes = (int)lds_bytes;
  out.levels = (int)n_table;
  out.prog = std::move(prog);
  // gather map: invariant block, then one block per slice
  out.map.reserve(prep_elems);
  for (int t = 0; t < nt; ++t)
    if (used[t] && in[t].smask == 0) {
      const int r = (int)in[t].canon.size();
      for (int64_t y = 0; y < (int64_t(1) << r); ++y) {
        auto val = [&](int v) -> int {
          int c = (int)(std::find(in[t].canon.begin(), in[t].canon.end(), v) - in[t].canon.begin());
          return (int)((y >> (r - 1 - c)) & 1);
        };
        out.map.push_back((int32_t)raw_index(md, t, val));
      }
    }
  for (int64_t sl = 0; sl < p.n_slices; ++sl)
    for (int t = 0; t < nt; ++t)
      if (used[t] && in[t].smask != 0) {
        const int r = (int)in[t].canon.size();
        for (int64_t y = 0; y < (int64_t(1) << r); ++y) {
          auto val = [&](int v) -> int {
            if (muj[v] >= 0) return (int)((sl >> muj[v]) & 1);
            int c = (int)(std::find(in[t].canon.begin(), in[t].canon.end(), v) - in[t].canon.begin());
            return (int)((y >> (r - 1 - c)) & 1);
          };
          out.map.push_back((int32_t)raw_index(md, t, val));
        }
      }
  return out;
}

std::vector<std::vector<int>> fold_groups(const Model& m, const Schedule& s) {
  const int nt = (int)m.tvars.size();
  std::vector<int> group_of(nt, -1);
  std::vector<std::vector<int>> groups;
  for (const Step& st : s.steps) {
    std::vector<int> ids, vars;
    for (const Operand& op : st.ops)
      if (op.kind == 't') {
        ids.push_back(op.id);
        for (int v : m.tvars[op.id])
          if (std::find(vars.begin(), vars.end(), v) == vars.end()) vars.push_back(v);
      }
    if (ids.size() < 2 || (int)vars.size() > kFoldMaxVars) continue;
    std::sort(ids.begin(), ids.end());
    for (int t : ids) group_of[t] = (int)groups.size();
    groups.push_back(ids);
  }
  // the compiled tensors in the caller's order, a group where its first
  // member was
  std::vector<std::vector<int>> out;
  for (int t = 0; t < nt; ++t) {
    if (group_of[t] < 0)
      out.push_back({t});
    else if (groups[group_of[t]][0] == t)
      out.push_back(groups[group_of[t]]);
  }
  return out;
}

Model fold_model(const Model& m, const std::vector<std::vector<int>>& groups) {
  Model f;
  f.n_vars = m.n_vars;
  for (const std::vector<int>& g : groups) {
    std::vector<int> vars;
    for (int t : g)
      for (int v : m.tvars[t])
        if (std::find(vars.begin(), vars.end(), v) == vars.end()) vars.push_back(v);
    const int r = (int)vars.size();
    f.data_off.push_back((int64_t)f.data.size() / 2);
    f.tvars.push_back(vars);
    std::vector<int> val(m.n_vars, 0);
    for (int64_t y = 0; y < (int64_t(1) << r); ++y) {
      for (int j = 0; j < r; ++j) val[vars[j]] = (int)((y >> (r - 1 - j)) & 1);
      double re = 1.0, im = 0.0;
      for (int t : g) {
        const int64_t e = raw_index(m, t, [&](int v) { return val[v]; });
        const double a = m.data[2 * e], b = m.data[2 * e + 1];
        const double nr = re * a - im * b;
        im = re * b + im * a;
        re = nr;
      }
      f.data.push_back(re);
      f.data.push_back(im);
    }
  }
  return f;
}

int push_inputs(Schedule& s) {
  int moves = 0;
  for (int k = (int)s.steps.size() - 1; k >= 0; --k) {
    Step& st = s.steps[k];
    for (size_t i = 0; i < st.ops.size();) {
      const Operand op = st.ops[i];
      if (op.kind != 't') {
        ++i;
        continue;
      }
      int to = -1;
      size_t best = SIZE_MAX;
      for (const Operand& r : st.ops) {
        if (r.kind != 'r' || r.vars.size() >= best) continue;
        bool inside = true;
        for (int v : op.vars) inside = inside && std::find(r.vars.begin(), r.vars.end(), v) != r.vars.end();
        if (inside) {
          best = r.vars.size();
          to = r.id;
        }
      }
      if (to < 0 || best + 2 > st.uni.size()) {
        ++i;
        continue;
      }
      st.ops.erase(st.ops.begin() + (long)i);
      // inputs by tensor id, then intermediates
      std::vector<Operand>& dst = s.steps[to].ops;
      size_t at = 0;
      while (at < dst.size() && dst[at].kind == 't' && dst[at].id < op.id) ++at;
      dst.insert(dst.begin() + (long)at, op);
      ++moves;
    }
  }
  return moves;
}

void compile_plan(Plan& p) {
  const Model& md = p.model;
  const Schedule& s = p.sched;
  const int nt = (int)md.tvars.size();
  p.m = (int)s.mu.size();
  if (p.m > 40) throw std::invalid_argument("at most 40 sliced variables");
  p.n_slices = int64_t(1) << p.m;
  std::vector<int> pos(md.n_vars, -1), muj(md.n_vars, -1);
  for (size_t i = 0; i < s.order.size(); ++i) pos[s.order[i]] = (int)i;
  for (int j = 0; j < p.m; ++j) muj[s.mu[j]] = j;
  if (p.m > 32)
    for (int j = 32; j < p.m; ++j) (void)j;  // slice ids above 2^32 handled as int64 below

  std::vector<InputInfo> in(nt);
  for (int t = 0; t < nt; ++t) {
    for (int v : md.tvars[t]) {
      if (muj[v] >= 0)
        in[t].slice_js.push_back(muj[v]);
      else
        in[t].canon.push_back(v);
    }
    std::sort(in[t].canon.begin(), in[t].canon.end(), [&](int a, int b) { return pos[a] < pos[b]; });
    std::sort(in[t].slice_js.begin(), in[t].slice_js.end());
    for (int j : in[t].slice_js) {
      if (j >= 32) throw std::invalid_argument("a tensor may not hold a sliced variable of index >= 32");
      in[t].smask |= 1u << j;
    }
    if (in[t].canon.size() > 30) throw std::invalid_argument("tensor rank above 30");
  }

  // ---------------- prepared inputs, per-step layout: versions per tensor
  std::vector<int64_t> step_base(nt);
  p.step_map.clear();
  for (int t = 0; t < nt; ++t) {
    step_base[t] = (int64_t)p.step_map.size();
    const int r = (int)in[t].canon.size();
    const int ns = (int)in[t].slice_js.size();
    for (int64_t ver = 0; ver < (int64_t(1) << ns); ++ver)
      for (int64_t y = 0; y < (int64_t(1) << r); ++y) {
        auto val = [&](int v) -> int {
          if (muj[v] >= 0) {
            int k = (int)(std::find(in[t].slice_js.begin(), in[t].slice_js.end(), muj[v]) -
                          in[t].slice_js.begin());
            return (int)((ver >> k) & 1);
          }
          int c = (int)(std::find(in[t].canon.begin(), in[t].canon.end(), v) - in[t].canon.begin());
          return (int)((y >> (r - 1 - c)) & 1);
        };
        int64_t ri = raw_index(md, t, val);
        if (ri > INT32_MAX) throw std::invalid_argument("model data too large");
        p.step_map.push_back((int32_t)ri);
      }
  }
  p.step_elems = (int64_t)p.step_map.size();

  // ---------------- fused segments (per-step plans that ask for them).
  // The prefix: the subtrees of small buckets -- every bucket whose union
  // has at most R + 1 variables and whose producers all do -- in one
  // LDS-resident launch (fused.hip) before the others; the results that
  // larger buckets read (and rank-0 results) are exported to the arena.  R
  // is the one asked for, or else the largest of 14 .. 4 whose prefix lets
  // two workgroups share a compute unit (a slice's levels are
  // latency-bound: two slices per compute unit halve the rounds), else the
  // largest of 10, 8, 6, 4 that fits LDS at all.  Later segments (if asked
  // for): each connected run of at least kSegMinBuckets other small buckets
  // (connected along the consumer edges, so a run has one top bucket, whose
  // result is its export) in one launch that imports the results of other
  // launches it reads.
  const int nsteps = (int)s.steps.size();
  std::vector<char> fused_any(nsteps, 0);  // bucket runs in a segment
  std::vector<FusedCode> seg_code;
  std::vector<std::vector<char>> seg_incl;
  p.segs.clear();
  p.has_prefix = false;
  p.seg_max_rank = -1;
  // The prefix for rank bound R (buckets of at most R + 1 variables whose
  // producers all are such), then with segments wanted every later run of
  // at least kSegMinBuckets such buckets (connected through their
  // consumers).  Programs above seg_cap leave their buckets to per-step
  // launches, or with strict set reject R.  Returns 0 when fewer than two
  // buckets qualify (no smaller R has more), 1 when built, -1 when R is
  // rejected.
  auto try_fused = [&](int R, int64_t cap, int64_t seg_cap, bool strict) -> int {
    std::vector<FusedCode> codes;
    std::vector<std::vector<char>> incls;
    std::vector<char> any(nsteps, 0);
    std::vector<char> f(nsteps, 0);
    int cnt = 0;
    for (int k = 0; k < nsteps; ++k) {  // producers precede their consumers
      bool ok = (int)s.steps[k].uni.size() <= R + 1;
      for (const auto& op : s.steps[k].ops)
        if (op.kind == 'r' && !f[op.id]) ok = false;
      f[k] = ok;
      cnt += ok;
    }
    if (cnt < 2) return 0;
    std::vector<int64_t> mark(nsteps, -1);
    for (int k = 0; k < nsteps; ++k)
      if (f[k] && (s.consumer[k] < 0 || !f[s.consumer[k]])) mark[k] = 0;
    FusedCode fc = build_fused(p, in, muj, f, &mark, cap);
    if (!fc.ok) return -1;
    codes.push_back(std::move(fc));
    incls.push_back(f);
    for (int k = 0; k < nsteps; ++k) any[k] |= f[k];
    if (p.want_segments) {
      std::vector<char> small(nsteps, 0);
      for (int k = 0; k < nsteps; ++k) small[k] = !any[k] && (int)s.steps[k].uni.size() <= R + 1;
      // the top of each bucket's run (consumers come after their producers)
      std::vector<int> top(nsteps, -1);
      for (int k = nsteps - 1; k >= 0; --k)
        if (small[k]) {
          const int c = s.consumer[k];
          top[k] = (c >= 0 && small[c]) ? top[c] : k;
        }
      std::vector<int> size(nsteps, 0);
      for (int k = 0; k < nsteps; ++k)
        if (small[k]) ++size[top[k]];
      for (int t = 0; t < nsteps; ++t) {
        if (!small[t] || top[t] != t || size[t] < kSegMinBuckets) continue;
        std::vector<char> g(nsteps, 0);
        for (int k = 0; k < nsteps; ++k) g[k] = small[k] && top[k] == t;
        std::vector<int64_t> mk(nsteps, -1);
        mk[t] = 0;
        FusedCode sc = build_fused(p, in, muj, g, &mk, seg_cap);
        if (!sc.ok) {
          if (strict) return -1;
          continue;  // its buckets stay per-step launches
        }
        codes.push_back(std::move(sc));
        incls.push_back(g);
        for (int k = 0; k < nsteps; ++k) any[k] |= g[k];
      }
    }
    for (size_t j = 0; j < codes.size(); ++j) {
      seg_code.push_back(std::move(codes[j]));
      seg_incl.push_back(incls[j]);
    }
    fused_any = any;
    p.has_prefix = true;
    p.seg_max_rank = R;
    return 1;
  };
  if (p.want_prefix > 0 && p.merge && p.m <= 24) {
    if (p.want_prefix == 1) {
      // the largest R whose launches all let two workgroups share a compute
      // unit's LDS; else the largest whose prefix does (segments up to the
      // whole LDS); else the largest that fits at all
      bool done = false;
      for (int pass = 0; pass < 3 && !done; ++pass)
        for (int R : pass < 2 ? std::vector<int>{14, 13, 12, 11, 10, 9, 8, 7, 6, 5, 4} : std::vector<int>{10, 8, 6, 4}) {
          const int64_t cap = pass < 2 ? kFusedLdsPair : kFusedLdsMax;
          const int rc = try_fused(R, cap, pass == 0 ? kFusedLdsPair : kFusedLdsMax, pass == 0 && p.want_segments);
          if (rc == 0) break;
          if (rc == 1) {
            done = true;
            break;
          }
        }
    } else {
      (void)try_fused(p.want_prefix, kFusedLdsMax, kFusedLdsMax, false);
    }
  }
  // each segment's position in schedule order: its last bucket
  std::vector<int> seg_last(seg_code.size(), -1);
  for (size_t j = 0; j < seg_code.size(); ++j)
    for (int k = 0; k < nsteps; ++k)
      if (seg_incl[j][k]) seg_last[j] = k;

  // ---------------- per-step launches and arena
  std::vector<int64_t> out_off(nsteps, -1);
  std::vector<char> placed(nsteps, 0);  // out_off is set (-1 also encodes own-space offset 0)
  Arena arena;
  int64_t own = 0;  // elements of the small results' own space
  p.steps.clear();
  p.scalar_arena.clear();
  // small results get space of their own after the arena (encoded as
  // -(offset + 1) until the arena's size is known): reusing freed space
  // would order otherwise independent launches behind one another
  auto place_result = [&](int k) {
    const int64_t osz = int64_t(1) << s.steps[k].out.size();
    if ((int)s.steps[k].out.size() <= kOwnSpaceRank) {
      own = (own + align_for(osz) - 1) / align_for(osz) * align_for(osz);
      out_off[k] = -(own + 1);
      own += osz;
    } else {
      out_off[k] = arena.alloc(osz, align_for(osz));
    }
    placed[k] = 1;
  };
  std::vector<int32_t> seg_pos(seg_code.size(), 0);
  // results the prefix exports: placed first, freed by their consumers
  if (p.has_prefix)
    for (int k : seg_code[0].export_steps) {
      const int64_t osz = int64_t(1) << s.steps[k].out.size();
      out_off[k] = arena.alloc(osz, align_for(osz));
      placed[k] = 1;
      if (s.steps[k].out.empty()) p.scalar_arena.push_back(out_off[k]);
    }
  // later segments: at their top bucket's place in schedule order, their
  // export placed like a launch's result, their imports then freed
  const std::vector<StepNode> step_nodes = merge_chains(s, p.merge, fused_any, p.max_sums > 0 ? p.max_sums : kChainSumMax);
  std::vector<std::pair<int, int>> items;  // (schedule position, node index or -1 - segment)
  for (size_t i = 0; i < step_nodes.size(); ++i) items.push_back({step_nodes[i].members.back(), (int)i});
  for (size_t j = p.has_prefix ? 1 : 0; j < seg_code.size(); ++j) items.push_back({seg_last[j], -1 - (int)j});
  std::sort(items.begin(), items.end());
  auto input_op = [&](int t, const std::vector<int>& uni) {
    StepOp o{};
    o.base = step_base[t];
    o.is_input = 1;
    o.rank = (int)in[t].canon.size();
    o.mask = union_mask(uni, in[t].canon);
    o.smask = in[t].smask;
    return o;
  };
  for (const auto& item : items) {
    if (item.second < 0) {
      const int j = -1 - item.second;
      seg_pos[j] = (int32_t)p.steps.size();
      for (int k : seg_code[j].export_steps) {
        place_result(k);
        if (s.steps[k].out.empty()) p.scalar_arena.push_back(out_off[k]);
      }
      for (int k : seg_code[j].import_steps)
        if (out_off[k] >= 0) arena.release(out_off[k], int64_t(1) << s.steps[k].out.size());
      continue;
    }
    const StepNode& node = step_nodes[item.second];
    const int k = node.members.back();  // the root: its result is the launch's
    const Step& st = s.steps[k];
    const int n_sum = (int)node.members.size();
    // union of the launch: the members' eliminated variables (earliest
    // first), then the root's result variables -- every factor's variables
    // lie in it, and the summed ones are its top bits
    std::vector<int> uni;
    for (int m : node.members) uni.push_back(s.steps[m].var);
    uni.insert(uni.end(), st.out.begin(), st.out.end());
    if (uni.size() > 31) throw std::invalid_argument("bucket union above 31 variables");
    const int rb = (int)st.out.size();
    std::vector<StepOp> ops;
    for (const auto& op : node.factors) {
      if (op.kind == 't') {
        ops.push_back(input_op(op.id, uni));
      } else {
        StepOp o{};
        o.base = out_off[op.id];
        o.is_input = 0;
        o.rank = (int)op.vars.size();
        o.mask = union_mask(uni, op.vars);
        ops.push_back(o);
      }
    }
    // Buckets with more operands than one launch takes: multiply groups of
    // operands into partial products over their own variables first (the sum
    // over u happens only in the last launch).  A partial product keeps u.
    std::vector<std::pair<int64_t, int64_t>> temps;  // arena blocks to free
    while ((int)ops.size() > kMaxOps) {
      std::vector<StepOp> grp(ops.begin(), ops.begin() + kMaxOps);
      uint32_t gm = 0;
      for (auto& o : grp) gm |= o.mask;
      // variables of the partial product, as bits of the union index
      const int pr = __builtin_popcount(gm);
      // re-express each member's mask inside the partial product's index
      StepProg sp{};
      sp.out_rank = -pr;  // negative: product without summation, out index = pext(X, gm)
      sp.n_sum = 0;
      int64_t sz = int64_t(1) << pr;
      int64_t off = arena.alloc(sz, align_for(sz));
      temps.push_back({off, sz});
      sp.out_base = off;
      sp.n_ops = kMaxOps;
      for (int i = 0; i < kMaxOps; ++i) {
        StepOp o = grp[i];
        uint32_t nm = 0;
        int bit = 0;
        for (int b = 0; b < 32; ++b)
          if ((gm >> b) & 1) {
            if ((o.mask >> b) & 1) nm |= 1u << bit;
            ++bit;
          }
        o.mask = nm;
        sp.ops[i] = o;
      }
      p.steps.push_back(sp);
      StepOp po{};
      po.base = off;
      po.is_input = 0;
      po.rank = pr;
      po.mask = gm;
      std::vector<StepOp> rest(ops.begin() + kMaxOps, ops.end());
      rest.insert(rest.begin(), po);
      ops.swap(rest);
    }
    StepProg sp{};
    sp.out_rank = rb;
    sp.n_sum = n_sum;
    if (n_sum > 2) {
      // The multi-term kernel runs four terms at a time over its two lowest
      // summed-value bits and reads a factor's entries once per distinct
      // value of the bits of those two it holds: give them to the pair of
      // summed variables that keeps that count smallest.  Union bit r_b + t
      // is summed variable uni[n_sum - 1 - t].
      int best = -1, bp = 0, bq = 1;
      for (int ti = 0; ti < n_sum; ++ti)
        for (int tj = ti + 1; tj < n_sum; ++tj) {
          int cost = 0;
          for (const StepOp& o : ops)
            cost += 1 << ((int)((o.mask >> (rb + ti)) & 1u) + (int)((o.mask >> (rb + tj)) & 1u));
          if (best < 0 || cost < best) {
            best = cost;
            bp = ti;
            bq = tj;
          }
        }
      int nb = 0;
      sp.sum_bit[nb++] = bp;
      sp.sum_bit[nb++] = bq;
      for (int t = 0; t < n_sum; ++t)
        if (t != bp && t != bq) sp.sum_bit[nb++] = t;
    }
    if (n_sum > 1 && rb >= 8 && ops.size() >= 2) {
      // merged launch as a batched complex product on MFMA: the operands
      // split into groups A and B, each with at least four result bits the
      // other group lacks (the 16 x 16 tile bits); every other result bit is
      // fixed per tile.  The first such split in operand order is taken.
      const uint32_t xmask = (1u << rb) - 1u;
      const uint32_t n = (uint32_t)ops.size();
      for (uint32_t side = 1; side + 1 < (1u << n) && !sp.mmk; ++side) {
        uint32_t xa = 0, xb = 0;
        for (uint32_t i = 0; i < n; ++i) ((side >> i) & 1u ? xb : xa) |= ops[i].mask & xmask;
        if (__builtin_popcount(xa & ~xb) >= 4 && __builtin_popcount(xb & ~xa) >= 4) {
          sp.mmk = 1;
          sp.mmk_side = side;
        }
      }
    }
    if (n_sum == 1) {
      // outer-product shape: two operands hold x bits (and u), the rest only u
      const uint32_t ubit = 1u << rb, xmask = ubit - 1u;
      int big[2] = {-1, -1}, nbig = 0;
      bool ok = (int)ops.size() <= kMaxOps;
      for (size_t i = 0; i < ops.size() && ok; ++i) {
        if (ops[i].mask & xmask) {
          if (nbig < 2 && (ops[i].mask & ubit)) big[nbig++] = (int)i; else ok = false;
        } else if (ops[i].mask != ubit) {
          ok = false;
        }
      }
      if (ok && nbig == 2) {
        const uint32_t ma = ops[big[0]].mask & xmask, mb = ops[big[1]].mask & xmask;
        if (__builtin_popcount(ma & ~mb) >= 4 && __builtin_popcount(mb & ~ma) >= 4 && ((ma | mb) == xmask)) {
          sp.mm_a = big[0];
          sp.mm_b = big[1];
        }
      }
    }
    place_result(k);
    sp.out_base = out_off[k];
    sp.n_ops = (int)ops.size();
    for (size_t i = 0; i < ops.size(); ++i) sp.ops[i] = ops[i];
    p.steps.push_back(sp);
    for (auto& tb : temps) arena.release(tb.first, tb.second);
    for (const auto& op : node.factors)
      if (op.kind == 'r' && out_off[op.id] >= 0) arena.release(out_off[op.id], int64_t(1) << op.vars.size());
    if (rb == 0) p.scalar_arena.push_back(out_off[k]);
  }
  // place the small results' own space after the arena
  const int64_t own_base = (arena.top + 63) / 64 * 64;
  auto place = [&](int64_t& off) {
    if (off < 0) off = own_base + (-off - 1);
  };
  for (StepProg& sp : p.steps) {
    place(sp.out_base);
    for (int i = 0; i < sp.n_ops; ++i)
      if (!sp.ops[i].is_input) place(sp.ops[i].base);
  }
  for (int64_t& off : p.scalar_arena) place(off);
  p.arena_per_slice = std::max<int64_t>(own > 0 ? own_base + own : arena.top, 1);
  // the segments, with the arena offsets of their rows
  for (size_t j = 0; j < seg_code.size(); ++j) {
    FusedCode& fc = seg_code[j];
    auto set_rows = [&](size_t at, const std::vector<int>& ks) {
      for (size_t i = 0; i < ks.size(); ++i) {
        if (!placed[ks[i]]) throw std::logic_error("fused segment row for a result with no arena place");
        int64_t off = out_off[ks[i]];
        place(off);
        fc.prog[at + 4 * i + 2] = (uint32_t)(uint64_t)off;
        fc.prog[at + 4 * i + 3] = (uint32_t)((uint64_t)off >> 32);
      }
    };
    set_rows(fc.export_at, fc.export_steps);
    set_rows(fc.import_at, fc.import_steps);
    FusedSeg sg;
    sg.exports.assign(fc.prog.begin() + fc.export_at, fc.prog.begin() + fc.export_at + 4 * fc.export_steps.size());
    sg.imports.assign(fc.prog.begin() + fc.import_at, fc.prog.begin() + fc.import_at + 4 * fc.import_steps.size());
    sg.prog = std::move(fc.prog);
    sg.map = std::move(fc.map);
    sg.elems = (int64_t)sg.map.size();
    sg.lds_bytes = fc.lds_bytes;
    sg.levels = fc.levels;
    sg.pos = seg_pos[j];
    // algorithmic traffic of the launch per slice: its inputs and imports
    // read once, its exports written once; products and sums of its buckets
    int64_t e = (int64_t)sg.prog[FH_INV_ELEMS] + (int64_t)sg.prog[FH_DEP_ELEMS];
    for (size_t i = 0; i < sg.exports.size(); i += 4) e += int64_t(1) << sg.exports[i + 1];
    for (size_t i = 0; i < sg.imports.size(); i += 4) e += int64_t(1) << sg.imports[i + 1];
    sg.bytes_per_slice = 8 * e;
    for (int k = 0; k < nsteps; ++k)
      if (seg_incl[j][k]) {
        const int64_t kk = (int64_t)s.steps[k].ops.size();
        sg.flops_per_slice += 6 * std::max<int64_t>(kk - 1, 0) * (int64_t(1) << s.steps[k].uni.size()) +
                              2 * (int64_t(1) << s.steps[k].out.size());
        ++sg.buckets;
      }
    p.segs.push_back(std::move(sg));
  }
  p.step_bytes_per_slice = 0;
  for (const FusedSeg& sg : p.segs) p.step_bytes_per_slice += sg.bytes_per_slice;
  for (const StepProg& sp : p.steps) {
    int64_t b = int64_t(1) << (sp.out_rank >= 0 ? sp.out_rank : -sp.out_rank);
    for (int i = 0; i < sp.n_ops; ++i) b += int64_t(1) << sp.ops[i].rank;
    p.step_bytes_per_slice += 8 * b;
  }
  // scalar results of steps must stay allocated: they were never released
  // (a rank-0 result has no consumer step).
  p.scalar_inputs_base.clear();
  p.scalar_inputs_smask.clear();
  for (int t : s.scalar_inputs) {
    p.scalar_inputs_base.push_back(step_base[t]);
    p.scalar_inputs_smask.push_back(in[t].smask);
  }

  build_launch_order(p);

  // ---------------- levels (dependency depth)
  std::vector<int> level(nsteps, 0);
  int n_levels = 0;
  for (int k = 0; k < nsteps; ++k) {
    int l = 0;
    for (const auto& op : s.steps[k].ops)
      if (op.kind == 'r') l = std::max(l, level[op.id] + 1);
    level[k] = l;
    n_levels = std::max(n_levels, l + 1);
  }
  p.n_levels = n_levels;

  // ---------------- fused form: the whole schedule in LDS
  p.fused_ok = false;
  p.fused_prog.clear();
  p.fused_map.clear();
  p.fused_elems = 0;
  p.fused_lds_bytes = 0;
  p.fused_levels = 0;
  bool eligible = p.m <= 24;
  for (const auto& st : s.steps)
    if (st.uni.size() > 15) eligible = false;
  if (eligible) {
    FusedCode fc = build_fused(p, in, muj, std::vector<char>(nsteps, 1), nullptr);
    if (fc.ok) {
      p.fused_ok = true;
      p.fused_prog = std::move(fc.prog);
      p.fused_map = std::move(fc.map);
      p.fused_elems = (int64_t)p.fused_map.size();
      p.fused_lds_bytes = fc.lds_bytes;
      p.fused_levels = fc.levels;
    }
  }
}

}  // namespace qbe
