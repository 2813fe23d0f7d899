// Host planner: simple graph, greedy min-fill order, treewidth of an order
// (Alg. 1), clique tree from an order (App. A), the tree-trimming, degree and
// direct-treewidth scores (Sec. 3.1-3.2), greedy mu-treewidth deletion
// (Alg. 2) and the bucket schedule of sliced bucket elimination (Eqs. 2-4).
//
// Graph vertices are the variables of the network; every tensor is a clique
// over its variables; self-loops and parallel edges are dropped (Sec. 2.2).
// All tie-breaks are deterministic (see each function) so that two
// independent implementations agree exactly.
#pragma once

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

namespace qbe {

// Dense bit-matrix adjacency over vertex ids [0, n).  A vertex can be
// "absent" (deleted or not part of a reduced graph).
struct Graph {
  int n = 0;
  int words = 0;
  std::vector<uint64_t> bits;   // n * words
  std::vector<uint8_t> present; // n

  void init(int n_);
  uint64_t* row(int v) { return bits.data() + (size_t)v * words; }
  const uint64_t* row(int v) const { return bits.data() + (size_t)v * words; }
  bool has(int a, int b) const { return (row(a)[b >> 6] >> (b & 63)) & 1ull; }
  void add_edge(int a, int b);
  int degree(int v) const;
  void remove_vertex(int v);
  std::vector<int> neighbours(int v) const;  // ascending ids
  int count() const;
};

Graph graph_from_tensors(int n_vars, const std::vector<std::vector<int>>& tensor_vars);

// Greedy min-fill: fewest fill edges, then smaller current degree, then
// smaller id.
std::vector<int> min_fill_order(const Graph& g);

// N+(u) for every eliminated vertex, in elimination order (ids ascending).
std::vector<std::vector<int>> eliminate(const Graph& g, const std::vector<int>& order);

// Alg. 1: max |N(u)| over the elimination (0 for an edgeless graph).
int width_of_order(const Graph& g, const std::vector<int>& order);

struct CliqueTree {
  std::vector<std::vector<int>> bags;  // maximal cliques, ids ascending,
                                       // ordered by their earliest vertex
  std::vector<int> parent;             // -1 for a root
};
// App. A read as: the maximal cliques {u} + N+(u) of the elimination, joined
// through the elimination tree.
CliqueTree clique_tree(const Graph& g, const std::vector<int>& order);

enum Score { SCORE_TREE_TRIMMING = 0, SCORE_DEGREE = 1, SCORE_TW_REDUCTION = 2, SCORE_BETWEENNESS = 3 };

int tree_trimming_pick(const Graph& g, const std::vector<int>& order);
// Sec. 3.1 betweenness centrality (unnormalised, undirected: each pair once)
// by Brandes' accumulation; the largest value rounded to 1e-9 wins, ties to
// the earliest vertex in order.
int betweenness_pick(const Graph& g, const std::vector<int>& order);
int degree_pick(const Graph& g, const std::vector<int>& order);
int tw_reduction_pick(const Graph& g, const std::vector<int>& order);

struct Deletion {
  std::vector<int> mu;             // in the order chosen
  std::vector<int> reduced_order;  // order minus mu
  int tau = 0;                     // width of the reduced order
};
// Alg. 2 without recomputing the order.  m >= 0: remove m vertices;
// m < 0: remove until the width is <= target_width.
// App. B, Alg. 5: an elimination order consistent with a tree decomposition
// (first leaf in bag order, its vertices missing from its parent in
// ascending ids; the roots' vertices last).
std::vector<int> recover_order(const CliqueTree& td);
// The anytime tree-decomposition heuristic: min-fill, then tries - 1
// min-fill runs whose (fill, degree) ties go to SplitMix64(seed) priorities
// (one draw per present vertex in id order per run); the first order of
// smallest width wins.
std::vector<int> anytime_order(const Graph& g, int tries, uint64_t seed);
// Alg. 2; with recompute_every = k > 0 its optional line runs after every
// k-th removal: the reduced order becomes Alg. 5's order of the clique tree
// of anytime_order(reduced graph, tries, seed).
Deletion greedy_deletion(const Graph& g, const std::vector<int>& order, int m, int target_width,
                         int score, int recompute_every = 0, int tries = 1, uint64_t seed = 0);
// Alg. 2 with the score f as a function (the argmax of Alg. 2's loop: it
// returns the vertex to remove from the graph and its order) and stopping
// rules: m >= 0 removes exactly m vertices; m < 0 removes until the width of
// the reduced order is <= target_width (when width_rule) and the peak live
// bytes per slice of its schedule are <= mem_cap (when mem_cap > 0).
using PickFn = std::function<int(const Graph&, const std::vector<int>&)>;
struct DeletionStop {
  int m = 0;
  bool width_rule = false;
  int target_width = 0;
  uint64_t mem_cap = 0;
  const std::vector<std::vector<int>>* tensor_vars = nullptr;  // for the memory cap
};
PickFn score_pick(int score);
Deletion greedy_deletion_with(const Graph& g, const std::vector<int>& order, const DeletionStop& stop,
                              const PickFn& pick, int recompute_every = 0, int tries = 1, uint64_t seed = 0);

// ---------------------------------------------------------------- schedule --

struct Operand {
  char kind;              // 't' input tensor, 'r' intermediate
  int id;                 // tensor id or step index
  std::vector<int> vars;  // remaining variables (inputs: original order minus
                          // sliced ones; intermediates: by position)
};

struct Step {
  int var;                     // eliminated variable u
  std::vector<Operand> ops;    // inputs by id, then intermediates by step
  std::vector<int> uni;        // U_b sorted by position in the order
  std::vector<int> out;        // U_b minus u
};

struct Schedule {
  std::vector<int> order, mu;
  std::vector<Step> steps;
  std::vector<int> scalar_inputs, scalar_steps, free_vars;
  std::vector<int> consumer;   // step index consuming step k's result (-1: scalar)
};

// Throws std::invalid_argument on inconsistent input.
Schedule build_schedule(int n_vars, const std::vector<std::vector<int>>& tensor_vars,
                        const std::vector<int>& order, const std::vector<int>& mu);

std::string dump_schedule(const Schedule& s);

// Per-slice cost of a schedule (complex64 bytes).
struct ScheduleCost {
  uint64_t flops = 0, bytes = 0, peak_bytes = 0;
  int width = 0;
};
ScheduleCost schedule_cost(const Schedule& s);

// Per-vertex features of a reduced graph and its order, for the learned
// slicing proposal: degree, relative position in the order, |N+(u)| relative
// to the width, membership of the maximum bags, number of clique-tree bags
// holding u and their total size (both relative to the maxima), and a
// constant.  Rows for vertices outside the order are zero.
constexpr int kFeatures = 8;
std::vector<float> vertex_features(const Graph& g, const std::vector<int>& order);

// ------------------------------------------------------ learned proposal --

// Greedy min-fill whose ties in fill go to the smaller priority, then the
// smaller degree, then the smaller id; rescore(g, prio) sets the priorities
// of the current elimination graph g (eliminated vertices absent, fill edges
// in) before the first elimination and after every `refresh` eliminations.
// With equal priorities this is min_fill_order.
using PrioRescore = std::function<void(const Graph&, std::vector<float>&)>;
std::vector<int> min_fill_order_learned(const Graph& g, const PrioRescore& rescore, int refresh);
// The elimination graph after eliminating order[0 .. k).
Graph eliminated_prefix(const Graph& g, const std::vector<int>& order, int k);
// The present vertices of minimum fill (ascending ids).
std::vector<int> min_fill_ties(const Graph& g);
// At most max_count of ids (a SplitMix64(seed) partial shuffle), ascending.
std::vector<int> sample_ids(std::vector<int> ids, int max_count, uint64_t seed);
// Labels of the learned proposal, the method's own exact costs (cost model):
// elimination -- for each candidate c of the state (prefix eliminated),
// log2 of the total FLOPs of the order prefix + c + greedy min-fill of the
// rest (no slicing); slicing -- log2 of the total FLOPs (2^(|mu| + 1)
// slices) of the reduced order without c and the sliced set mu + c.
std::vector<double> elim_labels(const Graph& state, const std::vector<int>& prefix,
                                const std::vector<std::vector<int>>& tensor_vars, const std::vector<int>& cand);
std::vector<double> slice_labels(const Graph& g, const std::vector<int>& order, const std::vector<int>& mu,
                                 const std::vector<std::vector<int>>& tensor_vars, const std::vector<int>& cand);

}  // namespace qbe
