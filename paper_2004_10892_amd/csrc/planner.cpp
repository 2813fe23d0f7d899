// Host planner (see planner.hpp for the contract of every function).
#include "planner.hpp"

#include <algorithm>
#include <cmath>
#include <functional>
#include <stdexcept>
#include <unordered_map>

namespace qbe {

// ------------------------------------------------------------------ graph --

void Graph::init(int n_) {
  n = n_;
  words = (n + 63) / 64;
  bits.assign((size_t)n * words, 0ull);
  present.assign(n, 1);
}

void Graph::add_edge(int a, int b) {
  if (a == b) return;
  row(a)[b >> 6] |= 1ull << (b & 63);
  row(b)[a >> 6] |= 1ull << (a & 63);
}

int Graph::degree(int v) const {
  int d = 0;
  const uint64_t* r = row(v);
  for (int i = 0; i < words; ++i) d += __builtin_popcountll(r[i]);
  return d;
}

void Graph::remove_vertex(int v) {
  for (int w : neighbours(v)) row(w)[v >> 6] &= ~(1ull << (v & 63));
  uint64_t* r = row(v);
  for (int i = 0; i < words; ++i) r[i] = 0;
  present[v] = 0;
}

std::vector<int> Graph::neighbours(int v) const {
  std::vector<int> out;
  const uint64_t* r = row(v);
  for (int i = 0; i < words; ++i) {
    uint64_t x = r[i];
    while (x) {
      int b = __builtin_ctzll(x);
      out.push_back(i * 64 + b);
      x &= x - 1;
    }
  }
  return out;
}

int Graph::count() const {
  int c = 0;
  for (uint8_t p : present) c += p;
  return c;
}

Graph graph_from_tensors(int n_vars, const std::vector<std::vector<int>>& tensor_vars) {
  Graph g;
  g.init(n_vars);
  for (const auto& vs : tensor_vars)
    for (size_t i = 0; i < vs.size(); ++i)
      for (size_t j = i + 1; j < vs.size(); ++j) g.add_edge(vs[i], vs[j]);
  return g;
}

static void check_order(const Graph& g, const std::vector<int>& order) {
  std::vector<uint8_t> seen(g.n, 0);
  int cnt = 0;
  for (int v : order) {
    if (v < 0 || v >= g.n || !g.present[v] || seen[v])
      throw std::invalid_argument("order is not a permutation of the graph's vertices");
    seen[v] = 1;
    ++cnt;
  }
  if (cnt != g.count()) throw std::invalid_argument("order does not cover the graph");
}

// One elimination step: join N(u) into a clique and delete u.
static void eliminate_vertex(Graph& g, int u, const std::vector<int>& nb) {
  const uint64_t* ru = g.row(u);
  for (int w : nb) {
    uint64_t* rw = g.row(w);
    for (int i = 0; i < g.words; ++i) rw[i] |= ru[i];
    rw[w >> 6] &= ~(1ull << (w & 63));
    rw[u >> 6] &= ~(1ull << (u & 63));
  }
  uint64_t* r = g.row(u);
  for (int i = 0; i < g.words; ++i) r[i] = 0;
  g.present[u] = 0;
}

std::vector<std::vector<int>> eliminate(const Graph& g0, const std::vector<int>& order) {
  check_order(g0, order);
  Graph g = g0;
  std::vector<std::vector<int>> out;
  out.reserve(order.size());
  for (int u : order) {
    std::vector<int> nb = g.neighbours(u);
    eliminate_vertex(g, u, nb);
    out.push_back(std::move(nb));
  }
  return out;
}

int width_of_order(const Graph& g, const std::vector<int>& order) {
  int tau = 0;
  for (const auto& nb : eliminate(g, order)) tau = std::max(tau, (int)nb.size());
  return tau;
}

// --------------------------------------------------------------- min-fill --

// Greedy min-fill; ties in (fill, degree) go to the smaller prio[v], or to
// the smaller id without priorities.
static std::vector<int> min_fill_prio(const Graph& g0, const std::vector<uint64_t>* prio);

std::vector<int> min_fill_order(const Graph& g0) { return min_fill_prio(g0, nullptr); }

static std::vector<int> min_fill_prio(const Graph& g0, const std::vector<uint64_t>* prio) {
  Graph g = g0;
  const int n = g.n;
  std::vector<int64_t> fill(n, 0);
  std::vector<int> deg(n, 0);
  auto score = [&](int v) {
    const uint64_t* rv = g.row(v);
    int d = 0;
    int64_t inner = 0;
    for (int i = 0; i < g.words; ++i) {
      uint64_t x = rv[i];
      d += __builtin_popcountll(x);
      while (x) {
        int w = i * 64 + __builtin_ctzll(x);
        x &= x - 1;
        const uint64_t* rw = g.row(w);
        for (int j = 0; j < g.words; ++j) inner += __builtin_popcountll(rw[j] & rv[j]);
      }
    }
    deg[v] = d;
    fill[v] = (int64_t)d * (d - 1) / 2 - inner / 2;
  };
  std::vector<int> alive;
  for (int v = 0; v < n; ++v)
    if (g.present[v]) {
      alive.push_back(v);
      score(v);
    }
  std::vector<int> order;
  order.reserve(alive.size());
  std::vector<int> mark(n, -1);
  for (int step = 0; !alive.empty(); ++step) {
    size_t bi = 0;
    for (size_t i = 1; i < alive.size(); ++i) {
      int a = alive[i], b = alive[bi];
      const bool tie_a = prio ? (*prio)[a] < (*prio)[b] : a < b;
      if (fill[a] < fill[b] || (fill[a] == fill[b] && (deg[a] < deg[b] || (deg[a] == deg[b] && tie_a))))
        bi = i;
    }
    int u = alive[bi];
    alive.erase(alive.begin() + bi);
    order.push_back(u);
    std::vector<int> nb = g.neighbours(u);
    eliminate_vertex(g, u, nb);
    std::vector<int> touched;
    for (int w : nb)
      if (mark[w] != step) {
        mark[w] = step;
        touched.push_back(w);
      }
    for (int w : nb)
      for (int x : g.neighbours(w))
        if (mark[x] != step) {
          mark[x] = step;
          touched.push_back(x);
        }
    for (int v : touched) score(v);
  }
  return order;
}

// ------------------------------------------------------------ clique tree --

CliqueTree clique_tree(const Graph& g, const std::vector<int>& order) {
  auto nplus = eliminate(g, order);
  const int n = g.n;
  std::vector<int> pos(n, -1);
  for (size_t i = 0; i < order.size(); ++i) pos[order[i]] = (int)i;
  std::vector<int> etp(n, -1);
  std::vector<std::vector<int>> children(n);
  for (size_t i = 0; i < order.size(); ++i) {
    int u = order[i];
    if (nplus[i].empty()) continue;
    int p = nplus[i][0];
    for (int w : nplus[i])
      if (pos[w] < pos[p]) p = w;
    etp[u] = p;
    children[p].push_back(u);  // children end up in elimination order
  }
  std::vector<int> rep(n, -1);
  std::vector<uint8_t> maximal(n, 0);
  std::vector<int> nsize(n, 0);
  for (size_t i = 0; i < order.size(); ++i) nsize[order[i]] = (int)nplus[i].size();
  for (size_t i = 0; i < order.size(); ++i) {
    int u = order[i];
    int absorbed = -1;
    for (int w : children[u])
      if (nsize[w] == nsize[u] + 1) {
        absorbed = w;
        break;
      }
    maximal[u] = absorbed < 0;
    rep[u] = maximal[u] ? u : rep[absorbed];
  }
  CliqueTree ct;
  std::vector<int> index(n, -1);
  for (size_t i = 0; i < order.size(); ++i) {
    int u = order[i];
    if (!maximal[u]) continue;
    index[u] = (int)ct.bags.size();
    std::vector<int> b = nplus[i];
    b.push_back(u);
    std::sort(b.begin(), b.end());
    ct.bags.push_back(std::move(b));
  }
  for (size_t i = 0; i < order.size(); ++i) {
    int u = order[i];
    if (!maximal[u]) continue;
    int x = u;
    while (etp[x] >= 0 && rep[etp[x]] == u) x = etp[x];
    ct.parent.push_back(etp[x] >= 0 ? index[rep[etp[x]]] : -1);
  }
  return ct;
}

// ----------------------------------------------------------------- scores --

int tree_trimming_pick(const Graph& g, const std::vector<int>& order) {
  CliqueTree ct = clique_tree(g, order);
  size_t smax = 0;
  for (const auto& b : ct.bags) smax = std::max(smax, b.size());
  const int n = g.n;
  std::vector<uint8_t> in_max(n, 0);
  std::vector<int64_t> len(n, 0), wt(n, 0);
  for (const auto& b : ct.bags) {
    for (int v : b) {
      len[v] += 1;
      wt[v] += (int64_t)b.size();
      if (b.size() == smax) in_max[v] = 1;
    }
  }
  // scan in elimination order so that the first maximum is the earliest
  int best = -1;
  for (int v : order) {
    if (!in_max[v]) continue;
    if (best < 0 || len[v] > len[best] || (len[v] == len[best] && wt[v] > wt[best])) best = v;
  }
  return best;
}

int degree_pick(const Graph& g, const std::vector<int>& order) {
  int best = -1, bd = -1;
  for (int v : order) {
    int d = g.degree(v);
    if (d > bd) {
      bd = d;
      best = v;
    }
  }
  return best;
}

int betweenness_pick(const Graph& g, const std::vector<int>& order) {
  const int n = g.n;
  std::vector<std::vector<int>> nb(n);
  for (int v : order) nb[v] = g.neighbours(v);
  std::vector<double> bc(n, 0.0), sigma(n, 0.0), delta(n, 0.0);
  std::vector<int> dist(n, -1), seq;
  std::vector<std::vector<int>> pred(n);
  seq.reserve(order.size());
  for (int s : order) {
    // shortest-path counts from s (breadth first), then the dependencies
    // of s on every vertex, accumulated from the farthest vertices back
    for (int v : order) {
      dist[v] = -1;
      sigma[v] = 0.0;
      delta[v] = 0.0;
      pred[v].clear();
    }
    seq.clear();
    dist[s] = 0;
    sigma[s] = 1.0;
    seq.push_back(s);
    for (size_t h = 0; h < seq.size(); ++h) {
      const int v = seq[h];
      for (int w : nb[v]) {
        if (dist[w] < 0) {
          dist[w] = dist[v] + 1;
          seq.push_back(w);
        }
        if (dist[w] == dist[v] + 1) {
          sigma[w] += sigma[v];
          pred[w].push_back(v);
        }
      }
    }
    for (size_t h = seq.size(); h-- > 0;) {
      const int w = seq[h];
      for (int v : pred[w]) delta[v] += sigma[v] / sigma[w] * (1.0 + delta[w]);
      if (w != s) bc[w] += delta[w];
    }
  }
  int best = -1;
  long long bk = 0;
  for (int v : order) {
    const long long k = std::llround(bc[v] / 2.0 * 1e9);
    if (best < 0 || k > bk) {
      best = v;
      bk = k;
    }
  }
  return best;
}

static Graph without(const Graph& g, int u) {
  Graph h = g;
  h.remove_vertex(u);
  return h;
}

int tw_reduction_pick(const Graph& g, const std::vector<int>& order) {
  int tau = width_of_order(g, order);
  int delta = 0, best = order[0];
  std::vector<int> red;
  for (int u : order) {
    red.clear();
    for (int v : order)
      if (v != u) red.push_back(v);
    int d = tau - width_of_order(without(g, u), red);
    if (d > delta) {
      delta = d;
      best = u;
    }
  }
  return best;
}

std::vector<int> recover_order(const CliqueTree& td) {
  const int nb = (int)td.bags.size();
  std::vector<uint8_t> alive(nb, 1);
  std::vector<int> children(nb, 0);
  for (int i = 0; i < nb; ++i)
    if (td.parent[i] >= 0) ++children[td.parent[i]];
  std::vector<int> order;
  for (;;) {
    int leaf = -1;
    for (int i = 0; i < nb && leaf < 0; ++i)
      if (alive[i] && td.parent[i] >= 0 && children[i] == 0) leaf = i;
    if (leaf < 0) break;
    const std::vector<int>& b = td.bags[leaf];
    const std::vector<int>& pb = td.bags[td.parent[leaf]];
    for (int v : b)  // bags list ids ascending
      if (!std::binary_search(pb.begin(), pb.end(), v)) order.push_back(v);
    alive[leaf] = 0;
    --children[td.parent[leaf]];
  }
  for (int i = 0; i < nb; ++i)
    if (alive[i]) order.insert(order.end(), td.bags[i].begin(), td.bags[i].end());
  return order;
}

namespace {
// SplitMix64 (Steele, Lea and Flood, 2014).
struct SplitMix64 {
  uint64_t state;
  uint64_t next() {
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
};
}  // namespace

std::vector<int> anytime_order(const Graph& g, int tries, uint64_t seed) {
  SplitMix64 rng{seed};
  std::vector<int> best = min_fill_order(g);
  int bw = width_of_order(g, best);
  std::vector<uint64_t> prio(g.n, 0);
  for (int t = 1; t < tries; ++t) {
    for (int v = 0; v < g.n; ++v)
      if (g.present[v]) prio[v] = rng.next();
    std::vector<int> o = min_fill_prio(g, &prio);
    const int w = width_of_order(g, o);
    if (w < bw) {
      best.swap(o);
      bw = w;
    }
  }
  return best;
}

Deletion greedy_deletion_with(const Graph& g0, const std::vector<int>& order, const DeletionStop& stop,
                              const PickFn& pick, int recompute_every, int tries, uint64_t seed) {
  check_order(g0, order);
  if (stop.m < 0 && !stop.width_rule && stop.mem_cap == 0)
    throw std::invalid_argument("m < 0 needs a target width or a memory cap");
  if (stop.mem_cap && !stop.tensor_vars) throw std::invalid_argument("a memory cap needs the tensors");
  Graph g = g0;
  Deletion d;
  d.reduced_order = order;
  auto peak = [&]() {
    return schedule_cost(build_schedule(g0.n, *stop.tensor_vars, d.reduced_order, d.mu)).peak_bytes;
  };
  while (!d.reduced_order.empty()) {
    if (stop.m >= 0) {
      if ((int)d.mu.size() >= stop.m) break;
    } else {
      const bool w_ok = !stop.width_rule || width_of_order(g, d.reduced_order) <= stop.target_width;
      if (w_ok && (stop.mem_cap == 0 || peak() <= stop.mem_cap)) break;
    }
    const int u = pick(g, d.reduced_order);
    if (u < 0 || u >= g.n || !g.present[u]) throw std::logic_error("score picked an absent vertex");
    g.remove_vertex(u);
    d.reduced_order.erase(std::find(d.reduced_order.begin(), d.reduced_order.end(), u));
    d.mu.push_back(u);
    if (recompute_every > 0 && d.mu.size() % (size_t)recompute_every == 0 && !d.reduced_order.empty())
      d.reduced_order = recover_order(clique_tree(g, anytime_order(g, tries, seed)));
  }
  if (stop.m >= 0 && (int)d.mu.size() < stop.m)
    throw std::invalid_argument("cannot remove more vertices than the graph has");
  d.tau = width_of_order(g, d.reduced_order);
  return d;
}

PickFn score_pick(int score) {
  switch (score) {
    case SCORE_TREE_TRIMMING: return tree_trimming_pick;
    case SCORE_DEGREE: return degree_pick;
    case SCORE_TW_REDUCTION: return tw_reduction_pick;
    case SCORE_BETWEENNESS: return betweenness_pick;
    default: throw std::invalid_argument("unknown score");
  }
}

Deletion greedy_deletion(const Graph& g0, const std::vector<int>& order, int m, int target_width,
                         int score, int recompute_every, int tries, uint64_t seed) {
  DeletionStop stop;
  stop.m = m;
  stop.width_rule = m < 0;
  stop.target_width = target_width;
  return greedy_deletion_with(g0, order, stop, score_pick(score), recompute_every, tries, seed);
}

// --------------------------------------------------------------- schedule --

Schedule build_schedule(int n_vars, const std::vector<std::vector<int>>& tensor_vars,
                        const std::vector<int>& order, const std::vector<int>& mu) {
  std::vector<int> pos(n_vars, -1);
  std::vector<uint8_t> sliced(n_vars, 0);
  for (int v : mu) {
    if (v < 0 || v >= n_vars || sliced[v]) throw std::invalid_argument("bad sliced variable");
    sliced[v] = 1;
  }
  for (size_t i = 0; i < order.size(); ++i) {
    int v = order[i];
    if (v < 0 || v >= n_vars || pos[v] >= 0 || sliced[v])
      throw std::invalid_argument("order and mu must be disjoint and repetition free");
    pos[v] = (int)i;
  }
  for (int v = 0; v < n_vars; ++v)
    if (pos[v] < 0 && !sliced[v]) throw std::invalid_argument("order + mu must cover every variable");

  Schedule s;
  s.order = order;
  s.mu = mu;
  std::vector<std::vector<Operand>> bucket(n_vars);
  for (size_t t = 0; t < tensor_vars.size(); ++t) {
    Operand op{'t', (int)t, {}};
    for (int v : tensor_vars[t])
      if (!sliced[v]) op.vars.push_back(v);
    if (op.vars.empty()) {
      s.scalar_inputs.push_back((int)t);
      continue;
    }
    int first = op.vars[0];
    for (int v : op.vars)
      if (pos[v] < pos[first]) first = v;
    bucket[first].push_back(std::move(op));
  }
  auto by_pos = [&](int a, int b) { return pos[a] < pos[b]; };
  for (int u : order) {
    auto& ops = bucket[u];
    if (ops.empty()) {
      s.free_vars.push_back(u);
      continue;
    }
    Step st;
    st.var = u;
    for (const auto& op : ops) st.uni.insert(st.uni.end(), op.vars.begin(), op.vars.end());
    std::sort(st.uni.begin(), st.uni.end(), by_pos);
    st.uni.erase(std::unique(st.uni.begin(), st.uni.end()), st.uni.end());
    for (int v : st.uni)
      if (v != u) st.out.push_back(v);
    st.ops = std::move(ops);
    int k = (int)s.steps.size();
    if (!st.out.empty())
      bucket[st.out[0]].push_back(Operand{'r', k, st.out});
    else
      s.scalar_steps.push_back(k);
    s.steps.push_back(std::move(st));
  }
  s.consumer.assign(s.steps.size(), -1);
  for (size_t k = 0; k < s.steps.size(); ++k)
    for (const auto& op : s.steps[k].ops)
      if (op.kind == 'r') s.consumer[op.id] = (int)k;
  return s;
}

static void join(std::string& out, const std::vector<int>& v) {
  for (size_t i = 0; i < v.size(); ++i) {
    if (i) out += ' ';
    out += std::to_string(v[i]);
  }
}

std::string dump_schedule(const Schedule& s) {
  std::string o;
  o += "order ";
  join(o, s.order);
  o += "\nmu ";
  join(o, s.mu);
  o += "\nscalar_inputs ";
  join(o, s.scalar_inputs);
  o += "\nfree_vars ";
  join(o, s.free_vars);
  o += "\n";
  for (size_t k = 0; k < s.steps.size(); ++k) {
    const Step& st = s.steps[k];
    o += "step " + std::to_string(k) + " var " + std::to_string(st.var) + " ops ";
    for (size_t i = 0; i < st.ops.size(); ++i) {
      if (i) o += ' ';
      o += st.ops[i].kind;
      o += std::to_string(st.ops[i].id);
    }
    o += " union ";
    join(o, st.uni);
    o += " out ";
    join(o, st.out);
    o += "\n";
  }
  o += "scalar_steps ";
  join(o, s.scalar_steps);
  o += "\n";
  return o;
}

static uint64_t sat(unsigned __int128 x) {
  return x > (unsigned __int128)UINT64_MAX ? UINT64_MAX : (uint64_t)x;
}

ScheduleCost schedule_cost(const Schedule& s) {
  ScheduleCost c;
  unsigned __int128 flops = 0, bytes = 0;
  const unsigned __int128 one = 1;
  for (const Step& st : s.steps) {
    int k = (int)st.ops.size();
    int nu = (int)st.uni.size();
    if (k > 1) flops += (unsigned __int128)6 * (k - 1) * (one << nu);
    flops += 2 * (one << (nu - 1));
    unsigned __int128 b = one << (nu - 1);
    for (const auto& op : st.ops) b += one << op.vars.size();
    bytes += 8 * b;
    c.width = std::max(c.width, nu - 1);
  }
  c.flops = sat(flops);
  c.bytes = sat(bytes);
  // peak live memory (inputs and unconsumed intermediates + current result)
  std::unordered_map<int64_t, unsigned __int128> live;
  unsigned __int128 total = 0, peak = 0;
  auto key = [](char kind, int id) { return (int64_t)(kind == 't' ? 0 : 1) << 40 | (int64_t)id; };
  for (const Step& st : s.steps)
    for (const auto& op : st.ops)
      if (op.kind == 't') {
        auto kk = key('t', op.id);
        if (!live.count(kk)) {
          live[kk] = 8 * (one << op.vars.size());
          total += live[kk];
        }
      }
  for (size_t k = 0; k < s.steps.size(); ++k) {
    const Step& st = s.steps[k];
    unsigned __int128 ob = st.out.empty() ? 0 : 8 * (one << st.out.size());
    peak = std::max(peak, total + ob);
    for (const auto& op : st.ops) {
      auto it = live.find(key(op.kind, op.id));
      if (it != live.end()) {
        total -= it->second;
        live.erase(it);
      }
    }
    if (!st.out.empty()) {
      live[key('r', (int)k)] = ob;
      total += ob;
    }
  }
  c.peak_bytes = sat(peak);
  return c;
}

std::vector<float> vertex_features(const Graph& g, const std::vector<int>& order) {
  const int n = g.n;
  std::vector<float> f((size_t)n * kFeatures, 0.f);
  if (order.empty()) return f;
  auto nplus = eliminate(g, order);
  CliqueTree ct = clique_tree(g, order);
  size_t smax = 0;
  for (const auto& b : ct.bags) smax = std::max(smax, b.size());
  std::vector<int> len(n, 0), wt(n, 0);
  std::vector<uint8_t> in_max(n, 0);
  int lmax = 1, wmax = 1;
  for (const auto& b : ct.bags)
    for (int v : b) {
      len[v] += 1;
      wt[v] += (int)b.size();
      if (b.size() == smax) in_max[v] = 1;
      lmax = std::max(lmax, len[v]);
      wmax = std::max(wmax, wt[v]);
    }
  int tau = 1;
  for (const auto& nb : nplus) tau = std::max(tau, (int)nb.size());
  const float nn = (float)order.size();
  for (size_t i = 0; i < order.size(); ++i) {
    const int u = order[i];
    float* r = f.data() + (size_t)u * kFeatures;
    r[0] = (float)g.degree(u) / 8.f;
    r[1] = (float)i / nn;
    r[2] = (float)nplus[i].size() / (float)tau;
    r[3] = in_max[u] ? 1.f : 0.f;
    r[4] = (float)len[u] / (float)lmax;
    r[5] = (float)wt[u] / (float)wmax;
    r[6] = (float)smax / 32.f;
    r[7] = 1.f;
  }
  return f;
}

// ------------------------------------------------------ learned proposal --

// Fill and degree of every present vertex of g (fill: missing edges among
// the vertex's neighbours).
static void fill_and_degree(const Graph& g, std::vector<int64_t>& fill, std::vector<int>& deg) {
  fill.assign(g.n, 0);
  deg.assign(g.n, 0);
  for (int v = 0; v < g.n; ++v) {
    if (!g.present[v]) continue;
    const uint64_t* rv = g.row(v);
    int d = 0;
    int64_t inner = 0;
    for (int i = 0; i < g.words; ++i) {
      uint64_t x = rv[i];
      d += __builtin_popcountll(x);
      while (x) {
        const int w = i * 64 + __builtin_ctzll(x);
        x &= x - 1;
        const uint64_t* rw = g.row(w);
        for (int j = 0; j < g.words; ++j) inner += __builtin_popcountll(rw[j] & rv[j]);
      }
    }
    deg[v] = d;
    fill[v] = (int64_t)d * (d - 1) / 2 - inner / 2;
  }
}

std::vector<int> min_fill_order_learned(const Graph& g0, const PrioRescore& rescore, int refresh) {
  if (refresh < 1) throw std::invalid_argument("refresh must be >= 1");
  Graph g = g0;
  std::vector<int64_t> fill;
  std::vector<int> deg;
  std::vector<float> prio(g.n, 0.f);
  std::vector<int> order;
  int left = g.count();
  for (int step = 0; left > 0; ++step, --left) {
    if (step % refresh == 0) rescore(g, prio);
    fill_and_degree(g, fill, deg);
    int u = -1;
    for (int v = 0; v < g.n; ++v) {
      if (!g.present[v]) continue;
      if (u < 0 || fill[v] < fill[u] ||
          (fill[v] == fill[u] && (prio[v] < prio[u] || (prio[v] == prio[u] && deg[v] < deg[u]))))
        u = v;  // ascending ids: a full tie keeps the smaller id
    }
    order.push_back(u);
    eliminate_vertex(g, u, g.neighbours(u));
  }
  return order;
}

Graph eliminated_prefix(const Graph& g0, const std::vector<int>& order, int k) {
  if (k < 0 || k > (int)order.size()) throw std::invalid_argument("bad elimination state");
  Graph g = g0;
  for (int i = 0; i < k; ++i) {
    const int u = order[i];
    if (u < 0 || u >= g.n || !g.present[u]) throw std::invalid_argument("bad order");
    eliminate_vertex(g, u, g.neighbours(u));
  }
  return g;
}

std::vector<int> min_fill_ties(const Graph& g) {
  std::vector<int64_t> fill;
  std::vector<int> deg;
  fill_and_degree(g, fill, deg);
  int64_t best = -1;
  std::vector<int> out;
  for (int v = 0; v < g.n; ++v) {
    if (!g.present[v]) continue;
    if (best < 0 || fill[v] < best) {
      best = fill[v];
      out.clear();
    }
    if (fill[v] == best) out.push_back(v);
  }
  return out;
}

std::vector<int> sample_ids(std::vector<int> ids, int max_count, uint64_t seed) {
  if ((int)ids.size() <= max_count) return ids;
  SplitMix64 rng{seed};
  for (int i = 0; i < max_count; ++i) {
    const int j = i + (int)(rng.next() % (uint64_t)(ids.size() - i));
    std::swap(ids[i], ids[j]);
  }
  ids.resize(max_count);
  std::sort(ids.begin(), ids.end());
  return ids;
}

std::vector<double> elim_labels(const Graph& state, const std::vector<int>& prefix,
                                const std::vector<std::vector<int>>& tensor_vars, const std::vector<int>& cand) {
  std::vector<double> y;
  for (int c : cand) {
    Graph g = state;
    eliminate_vertex(g, c, g.neighbours(c));
    std::vector<int> full = prefix;
    full.push_back(c);
    for (int v : min_fill_order(g)) full.push_back(v);
    const ScheduleCost cost = schedule_cost(build_schedule(state.n, tensor_vars, full, {}));
    y.push_back(std::log2((double)std::max<uint64_t>(cost.flops, 1)));
  }
  return y;
}

std::vector<double> slice_labels(const Graph& g, const std::vector<int>& order, const std::vector<int>& mu,
                                 const std::vector<std::vector<int>>& tensor_vars, const std::vector<int>& cand) {
  std::vector<double> y;
  for (int c : cand) {
    std::vector<int> red;
    for (int v : order)
      if (v != c) red.push_back(v);
    std::vector<int> m2 = mu;
    m2.push_back(c);
    const ScheduleCost cost = schedule_cost(build_schedule(g.n, tensor_vars, red, m2));
    y.push_back(std::log2((double)std::max<uint64_t>(cost.flops, 1)) + (double)m2.size());
  }
  return y;
}

}  // namespace qbe
