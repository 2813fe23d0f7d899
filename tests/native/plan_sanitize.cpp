// Host driver for the sanitizer build of the planner and plan compiler
// (planner.cpp, program.cpp, program_check.cpp): reads a network and a plan
// (sliced set and reduced order), builds the schedule, compiles the device
// programs in the one-launch-per-bucket form, the merged form, and the
// merged form with a fused prefix (automatic and fixed rank bounds) and
// fused segments, each with and without input folding (and the moves of
// input factors into producer buckets), and runs the host
// bounds check of every program.  The folded model is checked against its
// definition: its tensors partition the caller's, each group is the input
// tensors of one bucket, and every entry is the product of the members'
// entries (worked out here from the variable lists, on seeded data).
// Prints "ok" and exits 0, or prints
// the failure and exits 1.  Input: n_vars n_tensors, then per tensor its
// rank and variables, then the order (count, ids) and mu (count, ids).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <string>

#include "../../paper_2004_10892_amd/csrc/qbe_internal.hpp"

namespace qbe {
void set_error(const std::string&) {}
std::string check_plan(const Plan& p);
}  // namespace qbe

int main(int argc, char** argv) {
  if (argc != 2) return 2;
  std::ifstream f(argv[1]);
  int nv = 0, nt = 0;
  f >> nv >> nt;
  qbe::Model md;
  md.n_vars = nv;
  md.tvars.resize(nt);
  int64_t off = 0;
  for (int t = 0; t < nt; ++t) {
    int r = 0;
    f >> r;
    md.tvars[t].resize(r);
    for (int& v : md.tvars[t]) f >> v;
    md.data_off.push_back(off);
    off += int64_t(1) << r;
  }
  md.data.resize(2 * off);
  uint64_t lcg = 12345;
  for (double& d : md.data) {
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    d = (double)(lcg >> 11) / 9007199254740992.0 - 0.5;
  }
  int n = 0, m = 0;
  f >> n;
  std::vector<int> order(n);
  for (int& v : order) f >> v;
  f >> m;
  std::vector<int> mu(m);
  for (int& v : mu) f >> v;
  if (!f) return 2;
  try {
    // (merge, fused prefix, fused segments)
    const int forms[][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {1, 1, 1}, {1, 6, 1}, {1, 4, 0}};
    const qbe::Schedule s0 = qbe::build_schedule(nv, md.tvars, order, mu);
    const std::vector<std::vector<int>> groups = qbe::fold_groups(md, s0);
    const qbe::Model fm = qbe::fold_model(md, groups);
    {
      std::vector<int> seen(nt, 0);
      for (const auto& g : groups)
        for (int t : g) ++seen[t];
      for (int t = 0; t < nt; ++t)
        if (seen[t] != 1) {
          std::printf("fold: tensor %d in %d groups\n", t, seen[t]);
          return 1;
        }
      for (size_t j = 0; j < groups.size(); ++j) {
        const auto& g = groups[j];
        if (g.size() < 2) continue;
        bool one_bucket = false;
        for (const auto& st : s0.steps) {
          std::vector<int> ids;
          for (const auto& op : st.ops)
            if (op.kind == 't') ids.push_back(op.id);
          std::sort(ids.begin(), ids.end());
          if (ids == g) one_bucket = true;
        }
        if (!one_bucket) {
          std::printf("fold: group %zu is not one bucket's inputs\n", j);
          return 1;
        }
        const auto& vars = fm.tvars[j];
        if ((int)vars.size() > qbe::kFoldMaxVars) return 1;
        for (int64_t y = 0; y < (int64_t(1) << vars.size()); ++y) {
          double re = 1.0, im = 0.0;
          for (int t : g) {
            int64_t e = 0;
            for (int v : md.tvars[t]) {
              const size_t q = std::find(vars.begin(), vars.end(), v) - vars.begin();
              e = 2 * e + ((y >> (vars.size() - 1 - q)) & 1);
            }
            const double a = md.data[2 * (md.data_off[t] + e)], b = md.data[2 * (md.data_off[t] + e) + 1];
            const double nr = re * a - im * b;
            im = re * b + im * a;
            re = nr;
          }
          const int64_t at = 2 * (fm.data_off[j] + y);
          if (std::abs(fm.data[at] - re) > 1e-14 || std::abs(fm.data[at + 1] - im) > 1e-14) {
            std::printf("fold: group %zu entry %lld\n", j, (long long)y);
            return 1;
          }
        }
      }
    }
    for (int folded = 0; folded < 2; ++folded)
    for (const auto& form : forms) {
      qbe::Plan p;
      p.model = folded ? fm : md;
      p.sched = qbe::build_schedule(nv, p.model.tvars, order, mu);
      if (p.sched.steps.size() != s0.steps.size()) return 1;
      if (folded) {
        (void)qbe::push_inputs(p.sched);
        // every input is a factor of one bucket, and a moved one is
        // constant in that bucket's summed variable
        std::vector<int> uses(p.model.tvars.size(), 0);
        for (int t : p.sched.scalar_inputs) ++uses[t];
        for (const auto& st : p.sched.steps)
          for (const auto& op : st.ops) {
            for (int v : op.vars)
              if (std::find(st.uni.begin(), st.uni.end(), v) == st.uni.end()) {
                std::printf("push: operand variable outside its bucket\n");
                return 1;
              }
            if (op.kind != 't') continue;
            ++uses[op.id];
            const bool holds_u = std::find(op.vars.begin(), op.vars.end(), st.var) != op.vars.end();
            if (!holds_u)
              for (int v : op.vars)
                if (std::find(st.out.begin(), st.out.end(), v) == st.out.end()) {
                  std::printf("push: moved factor outside the result\n");
                  return 1;
                }
          }
        for (size_t t = 0; t < uses.size(); ++t)
          if (uses[t] > 1) {
            std::printf("push: tensor %zu used %d times\n", t, uses[t]);
            return 1;
          }
      }
      p.cost = qbe::schedule_cost(p.sched);
      p.merge = form[0] != 0;
      p.want_prefix = form[1];
      p.want_segments = form[2] != 0;
      qbe::compile_plan(p);
      const std::string bad = qbe::check_plan(p);
      if (!bad.empty()) {
        std::printf("check failed: %s\n", bad.c_str());
        return 1;
      }
    }
    // the planner's own passes on the same graph
    const qbe::Graph g = qbe::graph_from_tensors(nv, md.tvars);
    const std::vector<int> mf = qbe::min_fill_order(g);
    (void)qbe::clique_tree(g, mf);
    (void)qbe::greedy_deletion(g, mf, std::min(3, nv), -1, qbe::SCORE_TREE_TRIMMING, 1, 2, 7);
    (void)qbe::anytime_order(g, 3, 11);
  } catch (const std::exception& e) {
    std::printf("exception: %s\n", e.what());
    return 1;
  }
  std::printf("ok\n");
  return 0;
}
