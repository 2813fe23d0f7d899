// Host driver for the sanitizer build of the planner and plan compiler
// (planner.cpp, program.cpp, program_check.cpp): reads a network and a plan
// (sliced set and reduced order), builds the schedule, compiles the device
// programs in the one-launch-per-bucket form, the merged form, and the
// merged form with a fused prefix (automatic and fixed rank bounds) and
// fused segments, and runs the host bounds check of every program.  Prints "ok" and exits 0, or prints
// the failure and exits 1.  Input: n_vars n_tensors, then per tensor its
// rank and variables, then the order (count, ids) and mu (count, ids).
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
  md.data.assign(2 * off, 0.0);
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
    for (const auto& form : forms) {
      qbe::Plan p;
      p.model = md;
      p.sched = qbe::build_schedule(nv, md.tvars, order, mu);
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
