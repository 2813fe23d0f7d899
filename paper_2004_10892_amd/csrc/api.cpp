// C ABI of the library (declared in include/qbe.h).  Every entry point
// catches all C++ exceptions and turns them into error codes.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/qbe.h"
#include "qbe_internal.hpp"

struct qbe_ctx {
  int device = 0;
  void* stream = nullptr;
};

struct qbe_model {
  qbe::Model m;
  // qbe_model_create_dims: the binary variables of each original variable
  std::vector<int32_t> bit_first, bit_count;
};

struct qbe_plan {
  qbe::Plan p;
  qbe_ctx* ctx = nullptr;
};

struct qbe_gnn {
  qbe::Gnn g;
};

struct qbe_batch {
  qbe::Batch b;
  qbe_ctx* ctx = nullptr;
};

namespace qbe {
static thread_local std::string g_error;
void set_error(const std::string& s) { g_error = s; }
std::string check_plan(const Plan& p);  // program_check.cpp
}  // namespace qbe

using qbe::set_error;

#define QBE_GUARD_BEGIN try {
#define QBE_GUARD_END                                   \
  }                                                     \
  catch (const std::invalid_argument& e) {              \
    set_error(e.what());                                \
    return QBE_ERR_INVALID_ARG;                         \
  }                                                     \
  catch (const std::bad_alloc&) {                       \
    set_error("host allocation failed");                \
    return QBE_ERR_OOM;                                 \
  }                                                     \
  catch (const std::exception& e) {                     \
    set_error(std::string("internal: ") + e.what());    \
    return QBE_ERR_INTERNAL;                            \
  }                                                     \
  catch (...) {                                         \
    set_error("internal: unknown exception");           \
    return QBE_ERR_INTERNAL;                            \
  }

#define QBE_REQUIRE(cond, msg)        \
  do {                                \
    if (!(cond)) {                    \
      set_error(msg);                 \
      return QBE_ERR_INVALID_ARG;     \
    }                                 \
  } while (0)

namespace {

// A device call failed inside a host loop (a score callback): unwinds to the
// entry point, which returns its code.
struct DeviceError {
  int rc;
};

void csr_of(const qbe::Graph& g, std::vector<int32_t>& rp, std::vector<int32_t>& col) {
  rp.assign(g.n + 1, 0);
  col.clear();
  for (int v = 0; v < g.n; ++v) {
    rp[v] = (int32_t)col.size();
    for (int w : g.neighbours(v)) col.push_back(w);
  }
  rp[g.n] = (int32_t)col.size();
}

// The network's head scores on graph g with the features of (g, order).
void net_scores(qbe_ctx* ctx, qbe_gnn* gnn, int head, const qbe::Graph& g, const std::vector<int>& order,
                std::vector<float>& feats, std::vector<float>& scores) {
  feats = qbe::vertex_features(g, order);
  std::vector<int32_t> rp, col;
  csr_of(g, rp, col);
  scores.assign(g.n, 0.f);
  const int rc = qbe::gnn_score(gnn->g, ctx->stream, head, g.n, rp.data(), col.data(), feats.data(), scores.data());
  if (rc) throw DeviceError{rc};
}

}  // namespace

extern "C" {

const char* qbe_last_error(void) { return qbe::g_error.c_str(); }
int32_t qbe_version(void) { return 1; }

// ------------------------------------------------------------------ context

int qbe_create(qbe_ctx** out, int32_t device, void* hip_stream) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(out, "out is NULL");
  *out = nullptr;
  int n = 0;
  if (qbe::dev_count(&n) != QBE_OK) {
    set_error("no GPU device available (" + qbe::g_error + ")");
    return QBE_ERR_NO_DEVICE;
  }
  if (n <= 0) {
    set_error("no GPU device available");
    return QBE_ERR_NO_DEVICE;
  }
  QBE_REQUIRE(device >= 0 && device < n, "device index out of range");
  int rc = qbe::dev_set(device);
  if (rc) return rc;
  rc = qbe::dev_static_scratch_init(device);
  if (rc) return rc;
  qbe_ctx* c = new qbe_ctx;
  c->device = device;
  c->stream = hip_stream;
  *out = c;
  return QBE_OK;
  QBE_GUARD_END
}

int qbe_destroy(qbe_ctx* ctx) {
  delete ctx;
  return QBE_OK;
}

int qbe_set_stream(qbe_ctx* ctx, void* hip_stream) {
  QBE_REQUIRE(ctx, "ctx is NULL");
  ctx->stream = hip_stream;
  return QBE_OK;
}

// -------------------------------------------------------------------- model

static void fill_data(qbe::Model& m, const double* data) {
  size_t total = 0;
  for (const auto& vs : m.tvars) total += size_t(1) << vs.size();
  m.data.assign(data, data + 2 * total);
}

int qbe_model_create(int32_t n_vars, int32_t n_tensors, const int32_t* rank, const int32_t* vars,
                     const double* data, qbe_model** out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(out, "out is NULL");
  *out = nullptr;
  QBE_REQUIRE(n_vars >= 0 && n_tensors >= 0, "negative sizes");
  QBE_REQUIRE(n_tensors == 0 || (rank && data), "rank or data is NULL");
  auto* md = new qbe_model;
  qbe::Model& m = md->m;
  m.n_vars = n_vars;
  m.tvars.resize(n_tensors);
  m.data_off.resize(n_tensors);
  std::vector<uint8_t> used(n_vars, 0);
  std::vector<int> stamp(n_vars, -1);
  int64_t vp = 0, dp = 0;
  for (int t = 0; t < n_tensors; ++t) {
    if (rank[t] < 0 || rank[t] > 30) {
      delete md;
      set_error("tensor rank outside [0, 30]");
      return QBE_ERR_INVALID_ARG;
    }
    if (rank[t] > 0 && !vars) {
      delete md;
      set_error("vars is NULL");
      return QBE_ERR_INVALID_ARG;
    }
    for (int j = 0; j < rank[t]; ++j) {
      int v = vars[vp + j];
      if (v < 0 || v >= n_vars || stamp[v] == t) {
        delete md;
        set_error("variable id out of range or repeated within a tensor");
        return QBE_ERR_INVALID_ARG;
      }
      stamp[v] = t;
      used[v] = 1;
      m.tvars[t].push_back(v);
    }
    m.data_off[t] = dp;
    vp += rank[t];
    dp += int64_t(1) << rank[t];
    if (dp > (int64_t(1) << 31)) {
      delete md;
      set_error("model holds more than 2^31 complex entries");
      return QBE_ERR_INVALID_ARG;
    }
  }
  for (int v = 0; v < n_vars; ++v)
    if (!used[v]) {
      delete md;
      set_error("variable " + std::to_string(v) + " occurs in no tensor");
      return QBE_ERR_INVALID_ARG;
    }
  fill_data(m, data);
  *out = md;
  return QBE_OK;
  QBE_GUARD_END
}

int qbe_model_create_dims(int32_t n_vars, const int32_t* dims, int32_t n_tensors, const int32_t* rank,
                          const int32_t* vars, const double* data, qbe_model** out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(out, "out is NULL");
  *out = nullptr;
  QBE_REQUIRE(n_vars >= 0 && n_tensors >= 0, "negative sizes");
  QBE_REQUIRE(n_vars == 0 || dims, "dims is NULL");
  QBE_REQUIRE(n_tensors == 0 || (rank && data), "rank or data is NULL");
  // binary variables of each variable: its index bits, most significant first
  std::vector<int32_t> first(n_vars), nb(n_vars);
  int32_t nbin = 0;
  for (int v = 0; v < n_vars; ++v) {
    QBE_REQUIRE(dims[v] >= 1 && dims[v] <= (1 << 16), "dimension outside [1, 2^16]");
    int b = 0;
    while ((1 << b) < dims[v]) ++b;
    first[v] = nbin;
    nb[v] = b;
    nbin += b;
  }
  std::vector<int32_t> brank(n_tensors), bvars;
  std::vector<double> bdata;
  int64_t vp = 0, dp = 0;
  for (int t = 0; t < n_tensors; ++t) {
    QBE_REQUIRE(rank[t] >= 0 && rank[t] <= 64 && (rank[t] == 0 || vars), "bad tensor rank or vars");
    int bits = 0;
    int64_t size = 1;
    std::vector<int> tv(vars + vp, vars + vp + rank[t]);
    for (int v : tv) {
      QBE_REQUIRE(v >= 0 && v < n_vars, "variable id out of range");
      bits += nb[v];
      QBE_REQUIRE(bits <= 30, "a tensor has more than 30 binary variables");
      size *= dims[v];
      QBE_REQUIRE(size <= (int64_t(1) << 30), "tensor too large");
    }
    brank[t] = bits;
    for (int v : tv)
      for (int k = 0; k < nb[v]; ++k) bvars.push_back(first[v] + k);
    // binary index y (tensor's bits, first variable most significant) ->
    // the variables' values; a value >= L_v is padding (entry 0)
    const int64_t bsize = int64_t(1) << bits;
    const size_t o = bdata.size();
    bdata.resize(o + 2 * (size_t)bsize, 0.0);
    for (int64_t y = 0; y < bsize; ++y) {
      int64_t flat = 0;
      int shift = bits;
      bool pad = false;
      for (int v : tv) {
        shift -= nb[v];
        const int64_t val = (y >> shift) & ((int64_t(1) << nb[v]) - 1);
        if (val >= dims[v]) pad = true;
        flat = flat * dims[v] + val;
      }
      if (pad) continue;
      bdata[o + 2 * y] = data[2 * (dp + flat)];
      bdata[o + 2 * y + 1] = data[2 * (dp + flat) + 1];
    }
    vp += rank[t];
    dp += size;
  }
  qbe_model* md = nullptr;
  int rc = qbe_model_create(nbin, n_tensors, brank.data(), bvars.empty() ? nullptr : bvars.data(),
                            bdata.empty() ? nullptr : bdata.data(), &md);
  if (rc) return rc;
  md->bit_first = first;
  md->bit_count = nb;
  *out = md;
  return QBE_OK;
  QBE_GUARD_END
}

int qbe_model_var_bits(const qbe_model* model, int32_t v, int32_t* first_out, int32_t* count_out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(model && first_out && count_out, "NULL argument");
  if (model->bit_first.empty()) {
    QBE_REQUIRE(v >= 0 && v < model->m.n_vars, "variable id out of range");
    *first_out = v;
    *count_out = 1;
    return QBE_OK;
  }
  QBE_REQUIRE(v >= 0 && v < (int32_t)model->bit_first.size(), "variable id out of range");
  *first_out = model->bit_first[v];
  *count_out = model->bit_count[v];
  return QBE_OK;
  QBE_GUARD_END
}

int qbe_model_destroy(qbe_model* model) {
  delete model;
  return QBE_OK;
}

int qbe_model_set_data(qbe_model* model, const double* data) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(model && data, "NULL argument");
  fill_data(model->m, data);
  return QBE_OK;
  QBE_GUARD_END
}

// ----------------------------------------------------------------- planning

static qbe::Graph graph_of(const qbe::Model& m) { return qbe::graph_from_tensors(m.n_vars, m.tvars); }

static std::vector<int> vec(const int32_t* p, int32_t n) {
  if (n < 0) throw std::invalid_argument("negative length");
  if (n > 0 && !p) throw std::invalid_argument("NULL array");
  return std::vector<int>(p, p + n);
}

int qbe_order_min_fill(const qbe_model* model, int32_t* order_out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(model && (order_out || model->m.n_vars == 0), "NULL argument");
  auto order = qbe::min_fill_order(graph_of(model->m));
  for (size_t i = 0; i < order.size(); ++i) order_out[i] = order[i];
  return QBE_OK;
  QBE_GUARD_END
}

int qbe_width(const qbe_model* model, const int32_t* order, int32_t n, const int32_t* removed,
              int32_t n_removed, int32_t* tau_out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(model && tau_out, "NULL argument");
  qbe::Graph g = graph_of(model->m);
  for (int v : vec(removed, n_removed)) {
    QBE_REQUIRE(v >= 0 && v < g.n && g.present[v], "bad removed vertex");
    g.remove_vertex(v);
  }
  *tau_out = qbe::width_of_order(g, vec(order, n));
  return QBE_OK;
  QBE_GUARD_END
}

int qbe_slice_recompute(const qbe_model* model, const int32_t* order, int32_t n, int32_t m,
                        int32_t target_width, int32_t score, int32_t recompute_every, int32_t tries,
                        uint64_t seed, int32_t* mu_out, int32_t* m_out, int32_t* reduced_order_out,
                        int32_t* tau_out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(model && m_out && tau_out, "NULL argument");
  QBE_REQUIRE(n == model->m.n_vars, "order must list every variable");
  QBE_REQUIRE(m <= n, "m larger than the number of variables");
  QBE_REQUIRE(recompute_every >= 0 && tries >= 1, "recompute_every >= 0 and tries >= 1 required");
  auto d = qbe::greedy_deletion(graph_of(model->m), vec(order, n), m, target_width, score, recompute_every,
                                tries, seed);
  QBE_REQUIRE(d.mu.empty() || mu_out, "mu_out is NULL");
  QBE_REQUIRE(d.reduced_order.empty() || reduced_order_out, "reduced_order_out is NULL");
  for (size_t i = 0; i < d.mu.size(); ++i) mu_out[i] = d.mu[i];
  for (size_t i = 0; i < d.reduced_order.size(); ++i) reduced_order_out[i] = d.reduced_order[i];
  *m_out = (int32_t)d.mu.size();
  *tau_out = d.tau;
  return QBE_OK;
  QBE_GUARD_END
}

int qbe_order_anytime(const qbe_model* model, const int32_t* removed, int32_t n_removed, int32_t tries,
                      uint64_t seed, int32_t* order_out, int32_t* width_out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(model && order_out && width_out, "NULL argument");
  QBE_REQUIRE(tries >= 1, "tries must be >= 1");
  QBE_REQUIRE(n_removed >= 0 && (n_removed == 0 || removed), "bad removed list");
  qbe::Graph g = graph_of(model->m);
  for (int i = 0; i < n_removed; ++i) {
    QBE_REQUIRE(removed[i] >= 0 && removed[i] < g.n && g.present[removed[i]], "bad removed vertex");
    g.remove_vertex(removed[i]);
  }
  std::vector<int> o = qbe::anytime_order(g, tries, seed);
  for (size_t i = 0; i < o.size(); ++i) order_out[i] = o[i];
  *width_out = qbe::width_of_order(g, o);
  return QBE_OK;
  QBE_GUARD_END
}

int qbe_order_from_td(int32_t n_vars, int32_t n_bags, const int32_t* bag_offsets, const int32_t* bag_vars,
                      const int32_t* parent, int32_t* order_out, int32_t* n_out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(n_vars >= 0 && n_bags >= 0 && n_out && (n_bags == 0 || (bag_offsets && bag_vars && parent)),
              "bad argument");
  QBE_REQUIRE(n_bags == 0 || order_out || n_vars == 0, "order_out is NULL");
  qbe::CliqueTree td;
  td.bags.resize(n_bags);
  td.parent.assign(parent, parent + n_bags);
  for (int i = 0; i < n_bags; ++i) {
    QBE_REQUIRE(bag_offsets[i] >= 0 && bag_offsets[i] <= bag_offsets[i + 1], "bad bag offsets");
    for (int k = bag_offsets[i]; k < bag_offsets[i + 1]; ++k) {
      QBE_REQUIRE(bag_vars[k] >= 0 && bag_vars[k] < n_vars, "bag vertex out of range");
      QBE_REQUIRE(k == bag_offsets[i] || bag_vars[k - 1] < bag_vars[k], "bag ids must ascend");
      td.bags[i].push_back(bag_vars[k]);
    }
    QBE_REQUIRE(parent[i] >= -1 && parent[i] < n_bags && parent[i] != i, "bad parent");
  }
  // a forest: every bag reaches a root within n_bags steps
  for (int i = 0; i < n_bags; ++i) {
    int x = i, steps = 0;
    while (x >= 0 && steps <= n_bags) {
      x = td.parent[x];
      ++steps;
    }
    QBE_REQUIRE(x < 0, "parent array has a cycle");
  }
  std::vector<int> o = qbe::recover_order(td);
  std::vector<uint8_t> seen(n_vars, 0);
  for (int v : o) {
    QBE_REQUIRE(!seen[v], "a vertex is listed twice: not a tree decomposition");
    seen[v] = 1;
  }
  for (size_t i = 0; i < o.size(); ++i) order_out[i] = o[i];
  *n_out = (int32_t)o.size();
  return QBE_OK;
  QBE_GUARD_END
}

int qbe_clique_tree(const qbe_model* model, const int32_t* order, int32_t n, int32_t* n_bags,
                    int32_t* bag_offsets, int32_t* bag_vars, int64_t cap_vars, int32_t* parent) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(model && n_bags && bag_offsets && parent, "NULL argument");
  qbe::CliqueTree ct = qbe::clique_tree(graph_of(model->m), vec(order, n));
  *n_bags = (int32_t)ct.bags.size();
  int64_t total = 0;
  for (const auto& b : ct.bags) total += (int64_t)b.size();
  if (total > cap_vars || !bag_vars) {
    set_error("bag_vars capacity too small");
    return QBE_ERR_MEM_CAP;
  }
  int64_t o = 0;
  for (size_t i = 0; i < ct.bags.size(); ++i) {
    bag_offsets[i] = (int32_t)o;
    for (int v : ct.bags[i]) bag_vars[o++] = v;
    parent[i] = ct.parent[i];
  }
  bag_offsets[ct.bags.size()] = (int32_t)o;
  return QBE_OK;
  QBE_GUARD_END
}

int qbe_slice(const qbe_model* model, const int32_t* order, int32_t n, int32_t m, int32_t target_width,
              int32_t score, int32_t* mu_out, int32_t* m_out, int32_t* reduced_order_out,
              int32_t* tau_out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(model && m_out && tau_out, "NULL argument");
  QBE_REQUIRE(n == model->m.n_vars, "order must list every variable");
  QBE_REQUIRE(m <= n, "m larger than the number of variables");
  QBE_REQUIRE(score != QBE_SCORE_LEARNED, "the learned score needs a network: use qbe_slice_ex");
  auto d = qbe::greedy_deletion(graph_of(model->m), vec(order, n), m, target_width, score);
  QBE_REQUIRE(d.mu.empty() || mu_out, "mu_out is NULL");
  QBE_REQUIRE(d.reduced_order.empty() || reduced_order_out, "reduced_order_out is NULL");
  for (size_t i = 0; i < d.mu.size(); ++i) mu_out[i] = d.mu[i];
  for (size_t i = 0; i < d.reduced_order.size(); ++i) reduced_order_out[i] = d.reduced_order[i];
  *m_out = (int32_t)d.mu.size();
  *tau_out = d.tau;
  return QBE_OK;
  QBE_GUARD_END
}

int qbe_slice_ex(qbe_ctx* ctx, qbe_gnn* gnn, const qbe_model* model, const int32_t* order, int32_t n,
                 const qbe_slice_opts* opts, int32_t* mu_out, int32_t* m_out, int32_t* reduced_order_out,
                 int32_t* tau_out, int32_t* fell_back_out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(model && opts && m_out && tau_out, "NULL argument");
  QBE_REQUIRE(n == model->m.n_vars, "order must list every variable");
  const qbe_slice_opts& o = *opts;
  QBE_REQUIRE(o.reserved0 == 0 && o.reserved[0] == 0 && o.reserved[1] == 0, "reserved fields must be zero");
  QBE_REQUIRE(o.m <= n, "m larger than the number of variables");
  QBE_REQUIRE(o.m >= 0 || o.target_width >= 0 || o.mem_cap > 0, "m < 0 needs a target width or a memory cap");
  QBE_REQUIRE(o.recompute_every >= 0 && (o.recompute_every == 0 || o.tries >= 1), "bad recomputation options");
  const bool learned = o.score == QBE_SCORE_LEARNED;
  QBE_REQUIRE(learned || (o.score >= QBE_SCORE_TREE_TRIMMING && o.score <= QBE_SCORE_BETWEENNESS), "bad score");
  QBE_REQUIRE(!learned || (ctx && gnn), "the learned score needs a context and a network");
  if (learned) {
    int rc = qbe::dev_set(ctx->device);
    if (rc) return rc;
  }
  const qbe::Graph g = graph_of(model->m);
  qbe::DeletionStop stop;
  stop.m = o.m;
  stop.width_rule = o.m < 0 && o.target_width >= 0;
  stop.target_width = o.target_width;
  stop.mem_cap = o.m < 0 ? o.mem_cap : 0;
  stop.tensor_vars = &model->m.tvars;
  std::vector<float> feats, scores;
  qbe::PickFn pick;
  if (learned) {
    // Alg. 2's argmax with f = the network's slicing head: among the
    // vertices of the maximum bags (tree-trimming's candidates), the lowest
    // predicted cost wins; ties go to the earliest in the order
    pick = [&](const qbe::Graph& gr, const std::vector<int>& ord) {
      net_scores(ctx, gnn, QBE_HEAD_SLICING, gr, ord, feats, scores);
      int best = -1;
      for (int v : ord)
        if (feats[(size_t)v * qbe::kFeatures + 3] > 0.5f && (best < 0 || scores[v] < scores[best])) best = v;
      return best;
    };
  } else {
    pick = qbe::score_pick(o.score);
  }
  qbe::Deletion d;
  int fell_back = 0;
  try {
    d = qbe::greedy_deletion_with(g, vec(order, n), stop, pick, o.recompute_every, o.tries, o.seed);
    if (learned && o.mem_cap > 0) {
      const auto c = qbe::schedule_cost(qbe::build_schedule(n, model->m.tvars, d.reduced_order, d.mu));
      if (c.peak_bytes > o.mem_cap) {
        // the heuristic remains the fallback: tree-trimming, same rule
        d = qbe::greedy_deletion_with(g, vec(order, n), stop, qbe::score_pick(QBE_SCORE_TREE_TRIMMING),
                                      o.recompute_every, o.tries, o.seed);
        fell_back = 1;
      }
    }
  } catch (const DeviceError& e) {
    return e.rc;
  }
  QBE_REQUIRE(d.mu.empty() || mu_out, "mu_out is NULL");
  QBE_REQUIRE(d.reduced_order.empty() || reduced_order_out, "reduced_order_out is NULL");
  for (size_t i = 0; i < d.mu.size(); ++i) mu_out[i] = d.mu[i];
  for (size_t i = 0; i < d.reduced_order.size(); ++i) reduced_order_out[i] = d.reduced_order[i];
  *m_out = (int32_t)d.mu.size();
  *tau_out = d.tau;
  if (fell_back_out) *fell_back_out = fell_back;
  return QBE_OK;
  QBE_GUARD_END
}

int qbe_order_learned(qbe_ctx* ctx, qbe_gnn* gnn, const qbe_model* model, int32_t refresh, int32_t* order_out,
                      int32_t* width_out, int32_t* fell_back_out, uint64_t* flops_out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(ctx && gnn && model && order_out && width_out, "NULL argument");
  QBE_REQUIRE(refresh >= 1, "refresh must be >= 1");
  int rc = qbe::dev_set(ctx->device);
  if (rc) return rc;
  const qbe::Graph g = graph_of(model->m);
  std::vector<float> feats, scores;
  // priorities: the elimination head on the current elimination graph with
  // the features of its greedy min-fill order
  auto rescore = [&](const qbe::Graph& cur, std::vector<float>& prio) {
    net_scores(ctx, gnn, QBE_HEAD_ELIMINATION, cur, qbe::min_fill_order(cur), feats, scores);
    prio = scores;
  };
  std::vector<int> learned;
  try {
    learned = qbe::min_fill_order_learned(g, rescore, refresh);
  } catch (const DeviceError& e) {
    return e.rc;
  }
  const std::vector<int> mf = qbe::min_fill_order(g);
  const uint64_t fl = qbe::schedule_cost(qbe::build_schedule(g.n, model->m.tvars, learned, {})).flops;
  const uint64_t fm = qbe::schedule_cost(qbe::build_schedule(g.n, model->m.tvars, mf, {})).flops;
  // the heuristic remains the fallback: min-fill's order when it is cheaper
  const bool use_learned = fl <= fm;
  const std::vector<int>& best = use_learned ? learned : mf;
  std::copy(best.begin(), best.end(), order_out);
  *width_out = qbe::width_of_order(g, best);
  if (fell_back_out) *fell_back_out = use_learned ? 0 : 1;
  if (flops_out) {
    flops_out[0] = fl;
    flops_out[1] = fm;
  }
  return QBE_OK;
  QBE_GUARD_END
}

int qbe_learned_sample(const qbe_model* model, int32_t head, const int32_t* order, int32_t n, const int32_t* mu,
                       int32_t m, int32_t k_elim, int32_t max_cand, uint64_t seed, int32_t* rowptr_out,
                       int32_t* col_out, int64_t col_cap, int64_t* nnz_out, float* feats_out, int32_t* cand_out,
                       float* target_out, int32_t* n_cand_out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(model && rowptr_out && nnz_out && feats_out && n_cand_out, "NULL argument");
  QBE_REQUIRE(head == QBE_HEAD_SLICING || head == QBE_HEAD_ELIMINATION, "bad head");
  QBE_REQUIRE(max_cand >= 2 && cand_out && target_out, "max_cand must be >= 2 with output arrays");
  const int nv = model->m.n_vars;
  qbe::Graph g = graph_of(model->m);
  std::vector<int> mus = vec(mu, m);
  for (int v : mus) {
    QBE_REQUIRE(v >= 0 && v < nv && g.present[v], "bad sliced variable");
    g.remove_vertex(v);
  }
  const std::vector<int> ord = vec(order, n);
  qbe::Graph state;
  std::vector<int> cand, feat_order;
  std::vector<double> y;
  if (head == QBE_HEAD_SLICING) {
    QBE_REQUIRE(n == nv - m, "order must list every variable not in mu");
    state = g;
    const std::vector<float> f = qbe::vertex_features(g, ord);
    for (int v : ord)
      if (f[(size_t)v * qbe::kFeatures + 3] > 0.5f) cand.push_back(v);
    std::sort(cand.begin(), cand.end());
    cand = qbe::sample_ids(cand, max_cand, seed);
    feat_order = ord;
    if (cand.size() >= 2) y = qbe::slice_labels(g, ord, mus, model->m.tvars, cand);
  } else {
    QBE_REQUIRE(m == 0, "elimination samples take the whole graph (m = 0)");
    QBE_REQUIRE(n == nv, "order must list every variable");
    QBE_REQUIRE(k_elim >= 0 && k_elim < n, "bad elimination state");
    state = qbe::eliminated_prefix(g, ord, k_elim);
    cand = qbe::sample_ids(qbe::min_fill_ties(state), max_cand, seed);
    feat_order = qbe::min_fill_order(state);
    if (cand.size() >= 2)
      y = qbe::elim_labels(state, std::vector<int>(ord.begin(), ord.begin() + k_elim), model->m.tvars, cand);
  }
  int64_t nnz = 0;
  for (int v = 0; v < state.n; ++v) nnz += state.degree(v);
  *nnz_out = nnz;
  if (nnz > col_cap || (nnz > 0 && !col_out)) {
    set_error("col capacity too small");
    return QBE_ERR_MEM_CAP;
  }
  std::vector<int32_t> rp, col;
  csr_of(state, rp, col);
  std::copy(rp.begin(), rp.end(), rowptr_out);
  std::copy(col.begin(), col.end(), col_out);
  const std::vector<float> f = qbe::vertex_features(state, feat_order);
  std::copy(f.begin(), f.end(), feats_out);
  *n_cand_out = (int32_t)cand.size();
  for (size_t i = 0; i < cand.size(); ++i) cand_out[i] = cand[i];
  if (cand.size() >= 2) {
    // standardised within the state: (y - mean) / max(std, 0.05)
    double mean = 0.0, var = 0.0;
    for (double v : y) mean += v;
    mean /= (double)y.size();
    for (double v : y) var += (v - mean) * (v - mean);
    const double sd = std::max(std::sqrt(var / (double)y.size()), 0.05);
    for (size_t i = 0; i < y.size(); ++i) target_out[i] = (float)((y[i] - mean) / sd);
  }
  return QBE_OK;
  QBE_GUARD_END
}

int qbe_schedule_cost(const qbe_model* model, const int32_t* reduced_order, int32_t n, const int32_t* mu,
                      int32_t m, uint64_t* out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(model && out, "NULL argument");
  qbe::Schedule s = qbe::build_schedule(model->m.n_vars, model->m.tvars, vec(reduced_order, n), vec(mu, m));
  qbe::ScheduleCost c = qbe::schedule_cost(s);
  out[0] = c.flops;
  out[1] = c.bytes;
  out[2] = c.peak_bytes;
  out[3] = (uint64_t)c.width;
  return QBE_OK;
  QBE_GUARD_END
}

int qbe_vertex_features(const qbe_model* model, const int32_t* order, int32_t n, const int32_t* removed,
                        int32_t n_removed, float* feats_out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(model && feats_out, "NULL argument");
  qbe::Graph g = graph_of(model->m);
  for (int v : vec(removed, n_removed)) {
    QBE_REQUIRE(v >= 0 && v < g.n && g.present[v], "bad removed vertex");
    g.remove_vertex(v);
  }
  auto f = qbe::vertex_features(g, vec(order, n));
  std::copy(f.begin(), f.end(), feats_out);
  return QBE_OK;
  QBE_GUARD_END
}

// -------------------------------------------------------------------- plans

int qbe_plan_create(qbe_ctx* ctx, const qbe_model* model, const int32_t* reduced_order, int32_t n,
                    const int32_t* mu, int32_t m, const qbe_plan_opts* opts, qbe_plan** out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(model && out, "NULL argument");
  *out = nullptr;
  qbe_plan_opts o{};
  if (opts) o = *opts;
  QBE_REQUIRE(o.exec >= QBE_EXEC_AUTO && o.exec <= QBE_EXEC_FUSED, "bad exec form");
  QBE_REQUIRE(o.precision >= QBE_PREC_FP32 && o.precision <= QBE_PREC_BF16X6, "bad precision");
  QBE_REQUIRE(o.block == 0 || o.block == qbe::kBlock, "unsupported block size");
  QBE_REQUIRE(o.no_merge == 0 || o.no_merge == 1, "no_merge must be 0 or 1");
  QBE_REQUIRE(o.fused_prefix >= 0 && o.fused_prefix <= 14, "fused_prefix must be in [0, 14]");
  QBE_REQUIRE(o.fused_segments == 0 || o.fused_segments == 1, "fused_segments must be 0 or 1");
  QBE_REQUIRE(o.fused_segments == 0 || o.fused_prefix > 0, "fused_segments needs fused_prefix > 0");
  QBE_REQUIRE(o.no_fold == 0 || o.no_fold == 1, "no_fold must be 0 or 1");
  QBE_REQUIRE(o.max_sums >= 0 && o.max_sums <= 4, "max_sums must be in [0, 4]");
  auto* pl = new qbe_plan;
  std::unique_ptr<qbe_plan> guard(pl);
  qbe::Plan& p = pl->p;
  const std::vector<int> order = vec(reduced_order, n), mus = vec(mu, m);
  p.src_tvars = model->m.tvars;
  p.src_sched = qbe::build_schedule(model->m.n_vars, model->m.tvars, order, mus);
  p.cost = qbe::schedule_cost(p.src_sched);
  if (o.no_fold == 0) p.fold = qbe::fold_groups(model->m, p.src_sched);
  if (!p.fold.empty() && p.fold.size() < model->m.tvars.size()) {
    p.model = qbe::fold_model(model->m, p.fold);
    p.sched = qbe::build_schedule(p.model.n_vars, p.model.tvars, order, mus);
    // the same buckets: a folded tensor lies in its members' bucket
    QBE_REQUIRE(p.sched.steps.size() == p.src_sched.steps.size(), "internal: folding changed the buckets");
    for (size_t k = 0; k < p.sched.steps.size(); ++k)
      QBE_REQUIRE(p.sched.steps[k].var == p.src_sched.steps[k].var && p.sched.steps[k].uni == p.src_sched.steps[k].uni,
                  "internal: folding changed the buckets");
  } else {
    p.fold.clear();
    p.model = model->m;
    p.sched = p.src_sched;
  }
  if (o.no_fold == 0) (void)qbe::push_inputs(p.sched);
  p.precision = o.precision;
  p.merge = o.no_merge == 0;
  p.max_sums = o.max_sums;
  p.want_prefix = o.exec != QBE_EXEC_FUSED ? o.fused_prefix : 0;
  p.want_segments = o.fused_segments == 1;
  qbe::compile_plan(p);
  if (o.exec == QBE_EXEC_FUSED && o.precision != QBE_PREC_FP32) {
    set_error("the fused form computes in FP32 only");
    return QBE_ERR_INVALID_ARG;
  }
  if (o.exec == QBE_EXEC_FUSED && !p.fused_ok) {
    set_error("plan does not fit the fused (LDS-resident) form");
    return QBE_ERR_MEM_CAP;
  }
  p.exec = (o.exec == QBE_EXEC_PER_STEP || !p.fused_ok) ? QBE_EXEC_PER_STEP : QBE_EXEC_FUSED;
  if (p.precision != QBE_PREC_FP32 && p.exec == QBE_EXEC_FUSED && o.exec == QBE_EXEC_AUTO)
    p.exec = QBE_EXEC_PER_STEP;
  if (p.exec == QBE_EXEC_FUSED && !p.segs.empty()) {
    // the fused form is one launch: the per-step part without segments
    p.want_prefix = 0;
    p.want_segments = false;
    qbe::compile_plan(p);
  }
  std::string bad = qbe::check_plan(p);
  if (!bad.empty()) {
    set_error("internal: plan check failed: " + bad);
    return QBE_ERR_INTERNAL;
  }
  if (ctx) {
    int rc = qbe::dev_set(ctx->device);
    if (rc) return rc;
    p.device = ctx->device;
    rc = qbe::dev_upload_plan(p);
    if (rc) {
      qbe::dev_free_plan(p);
      return rc;
    }
    pl->ctx = ctx;
  }
  *out = guard.release();
  return QBE_OK;
  QBE_GUARD_END
}

int qbe_plan_destroy(qbe_plan* plan) {
  if (plan) {
    if (plan->ctx) {
      (void)qbe::dev_set(plan->p.device);
      qbe::dev_free_plan(plan->p);
    }
    delete plan;
  }
  return QBE_OK;
}

int qbe_plan_clone(const qbe_plan* src, const qbe_model* model, qbe_plan** out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(src && model && out, "NULL argument");
  *out = nullptr;
  QBE_REQUIRE(model->m.tvars == src->p.src_tvars, "model structure differs from the plan's");
  auto* pl = new qbe_plan;
  std::unique_ptr<qbe_plan> guard(pl);
  qbe::Plan& p = pl->p;
  p = src->p;  // host side: schedule, programs, layouts, tile shapes
  p.model = p.fold.empty() ? model->m : qbe::fold_model(model->m, p.fold);
  qbe::dev_forget_plan(p);  // the copied device pointers stay src's
  if (src->ctx) {
    int rc = qbe::dev_set(p.device);
    if (rc) return rc;
    rc = qbe::dev_upload_plan(p);
    if (rc) {
      qbe::dev_free_plan(p);
      return rc;
    }
    pl->ctx = src->ctx;
  }
  *out = guard.release();
  return QBE_OK;
  QBE_GUARD_END
}

int qbe_plan_update_data(qbe_plan* plan, const qbe_model* model) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(plan && model, "NULL argument");
  QBE_REQUIRE(model->m.tvars == plan->p.src_tvars, "model structure differs from the plan's");
  plan->p.model.data = plan->p.fold.empty() ? model->m.data : qbe::fold_model(model->m, plan->p.fold).data;
  if (plan->ctx) {
    int rc = qbe::dev_set(plan->p.device);
    if (rc) return rc;
    return qbe::dev_update_data(plan->p);
  }
  return QBE_OK;
  QBE_GUARD_END
}

int qbe_plan_stats(const qbe_plan* plan, qbe_stats* out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(plan && out, "NULL argument");
  const qbe::Plan& p = plan->p;
  std::memset(out, 0, sizeof(*out));
  out->n_vars = p.model.n_vars;
  out->n_tensors = (int32_t)p.src_tvars.size();
  out->m = p.m;
  out->width = p.cost.width;
  out->n_steps = (int32_t)p.sched.steps.size();
  out->n_levels = p.n_levels;
  out->exec = p.exec;
  out->lds_bytes = p.exec == QBE_EXEC_FUSED ? p.fused_lds_bytes : 0;
  out->flops_per_slice = p.cost.flops;
  out->bytes_per_slice = p.cost.bytes;
  out->peak_bytes_per_slice = p.cost.peak_bytes;
  out->ws_bytes_min = qbe::dev_workspace_min(p, p.n_slices);
  out->ws_bytes_all_slices = qbe::dev_workspace_all(p);
  out->n_mfma_steps = 0;
  for (const auto& sp : p.steps)
    if (sp.mm_a >= 0 || sp.mmk) ++out->n_mfma_steps;
  out->precision = p.precision;
  out->fused_levels = p.fused_ok ? p.fused_levels : 0;
  out->n_merged_steps = 0;
  for (const auto& sp : p.steps)
    if (sp.n_sum > 1) ++out->n_merged_steps;
  out->step_bytes_per_slice = (uint64_t)p.step_bytes_per_slice;
  out->n_launches = (int32_t)p.launch_order.size();
  out->prefix_buckets = p.has_prefix ? p.segs[0].buckets : 0;
  out->n_fused_segments = (int32_t)p.segs.size();
  out->fused_buckets = 0;
  for (const qbe::FusedSeg& sg : p.segs) out->fused_buckets += sg.buckets;
  return QBE_OK;
  QBE_GUARD_END
}

int qbe_plan_dump(const qbe_plan* plan, char* buf, size_t cap, size_t* len_out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(plan && len_out, "NULL argument");
  std::string s = qbe::dump_schedule(plan->p.src_sched);
  *len_out = s.size();
  if (buf && cap) {
    size_t n = std::min(cap, s.size() + 1);
    std::memcpy(buf, s.c_str(), n);
  }
  return QBE_OK;
  QBE_GUARD_END
}

int qbe_plan_check(const qbe_plan* plan) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(plan, "NULL argument");
  std::string bad = qbe::check_plan(plan->p);
  if (!bad.empty()) {
    set_error(bad);
    return QBE_ERR_INTERNAL;
  }
  return QBE_OK;
  QBE_GUARD_END
}

// -------------------------------------------------------------- contraction

static int check_device_call(qbe_ctx* ctx, const qbe_plan* plan, void* ws) {
  if (!ctx || !plan || !ws) {
    set_error("NULL argument");
    return QBE_ERR_INVALID_ARG;
  }
  if (!plan->ctx) {
    set_error("plan was created without a device context");
    return QBE_ERR_INVALID_ARG;
  }
  if (plan->p.device != ctx->device) {
    set_error("plan belongs to another device");
    return QBE_ERR_INVALID_ARG;
  }
  return qbe::dev_set(ctx->device);
}

int qbe_plan_autotune(qbe_ctx* ctx, qbe_plan* plan, void* d_workspace, size_t ws_bytes, int64_t min_elems) {
  QBE_GUARD_BEGIN
  int rc = check_device_call(ctx, plan, d_workspace);
  if (rc) return rc;
  if (plan->p.exec != QBE_EXEC_PER_STEP) return QBE_OK;
  return qbe::dev_autotune(plan->p, ctx->stream, d_workspace, ws_bytes, min_elems);
  QBE_GUARD_END
}

// Launch info of a per-step plan's execution order (then finalize, reduce).
namespace {

uint64_t step_bytes(const qbe::StepProg& sp) {
  const int r = sp.out_rank >= 0 ? sp.out_rank : -sp.out_rank;
  uint64_t e = uint64_t(1) << r;
  for (int i = 0; i < sp.n_ops; ++i) e += uint64_t(1) << sp.ops[i].rank;
  return 8 * e;
}

// products and sums of one launch: every result entry sums 2^n_sum terms of
// n_ops complex factors (a partial product: one term, no sum)
uint64_t step_flops(const qbe::StepProg& sp) {
  const int r = sp.out_rank >= 0 ? sp.out_rank : -sp.out_rank;
  const uint64_t terms = uint64_t(1) << sp.n_sum;
  const uint64_t per_term = 6 * (uint64_t)std::max(sp.n_ops - 1, 0);
  return (uint64_t(1) << r) * (terms * per_term + 2 * (terms - 1));
}

}  // namespace

int qbe_plan_num_launches(const qbe_plan* plan, int32_t* n_out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(plan && n_out, "NULL argument");
  const qbe::Plan& p = plan->p;
  *n_out = p.exec == QBE_EXEC_PER_STEP ? (int32_t)p.launch_order.size() + 2 : 0;
  return QBE_OK;
  QBE_GUARD_END
}

int qbe_plan_launch_info(const qbe_plan* plan, int32_t i, qbe_launch_info* out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(plan && out, "NULL argument");
  const qbe::Plan& p = plan->p;
  QBE_REQUIRE(p.exec == QBE_EXEC_PER_STEP, "launch info is for per-step plans");
  const int n_order = (int)p.launch_order.size();
  QBE_REQUIRE(i >= 0 && i < n_order + 2, "launch index out of range");
  std::memset(out, 0, sizeof(*out));
  if (i == n_order) {
    out->kind = QBE_LAUNCH_FINALIZE;
    out->bytes_per_slice = 8 * (p.scalar_arena.size() + p.scalar_inputs_base.size()) + 16;
    return QBE_OK;
  }
  if (i == n_order + 1) {
    out->kind = QBE_LAUNCH_REDUCE;
    out->bytes_per_slice = 16;
    return QBE_OK;
  }
  const qbe::LaunchItem& li = p.launch_order[i];
  if (li.seg >= 0) {
    const qbe::FusedSeg& sg = p.segs[li.seg];
    out->kind = sg.imports.empty() ? QBE_LAUNCH_PREFIX : QBE_LAUNCH_SEGMENT;
    out->n_buckets = sg.buckets;
    out->n_ops = (int32_t)(sg.imports.size() / 4);
    out->out_rank = p.seg_max_rank;
    out->bytes_per_slice = (uint64_t)sg.bytes_per_slice;
    out->flops_per_slice = (uint64_t)sg.flops_per_slice;
    out->levels = sg.levels;
    out->lds_bytes = sg.lds_bytes;
    return QBE_OK;
  }
  if (li.group >= 0) {
    out->kind = QBE_LAUNCH_GROUP;
    for (int k = p.group_first[li.group]; k < p.group_first[li.group + 1]; ++k) {
      const qbe::StepProg& sp = p.steps[p.group_steps[k].step];
      out->n_buckets += 1;
      out->bytes_per_slice += step_bytes(sp);
      out->flops_per_slice += step_flops(sp);
      out->n_ops = std::max(out->n_ops, sp.n_ops);
      out->out_rank = std::max(out->out_rank, sp.out_rank >= 0 ? sp.out_rank : -sp.out_rank);
    }
    return QBE_OK;
  }
  const qbe::StepProg& sp = p.steps[li.step];
  out->kind = sp.out_rank < 0 ? QBE_LAUNCH_PARTIAL : sp.n_sum > 1 ? QBE_LAUNCH_MERGED : QBE_LAUNCH_BUCKET;
  out->n_buckets = std::max(sp.n_sum, 1);
  out->n_ops = sp.n_ops;
  out->out_rank = sp.out_rank >= 0 ? sp.out_rank : -sp.out_rank;
  out->n_sum = sp.n_sum;
  out->mfma = (sp.mmk || sp.mm_a >= 0) ? 1 : 0;
  out->bytes_per_slice = step_bytes(sp);
  out->flops_per_slice = step_flops(sp);
  return QBE_OK;
  QBE_GUARD_END
}

int qbe_plan_profile(qbe_ctx* ctx, const qbe_plan* plan, void* d_workspace, size_t ws_bytes, float* ms_out,
                     int32_t cap, int32_t* n_out) {
  QBE_GUARD_BEGIN
  int rc = check_device_call(ctx, plan, d_workspace);
  if (rc) return rc;
  QBE_REQUIRE(ms_out && n_out, "NULL argument");
  int n = 0;
  rc = qbe::dev_profile(plan->p, ctx->stream, d_workspace, ws_bytes, ms_out, cap, &n);
  *n_out = n;
  return rc;
  QBE_GUARD_END
}

int qbe_contract_async(qbe_ctx* ctx, const qbe_plan* plan, void* d_workspace, size_t ws_bytes,
                       double* d_amp_out) {
  QBE_GUARD_BEGIN
  int rc = check_device_call(ctx, plan, d_workspace);
  if (rc) return rc;
  QBE_REQUIRE(d_amp_out, "d_amp_out is NULL");
  return qbe::dev_contract(plan->p, ctx->stream, d_workspace, ws_bytes, 0, plan->p.n_slices, d_amp_out,
                           nullptr);
  QBE_GUARD_END
}

int qbe_contract_static(qbe_ctx* ctx, const qbe_plan* plan, double* d_amp_out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(ctx && plan && d_amp_out, "NULL argument");
  QBE_REQUIRE(plan->ctx, "plan was created without a device context");
  QBE_REQUIRE(plan->p.device == ctx->device, "plan belongs to another device");
  int rc = qbe::dev_set(ctx->device);
  if (rc) return rc;
  rc = qbe::dev_static_scratch_init(ctx->device);  // no-op once qbe_create did it
  if (rc) return rc;
  return qbe::dev_contract_static(plan->p, ctx->stream, d_amp_out);
  QBE_GUARD_END
}

size_t qbe_static_scratch_bytes(void) { return qbe::kStaticScratchBytes; }

int qbe_contract_slices(qbe_ctx* ctx, const qbe_plan* plan, int64_t s_begin, int64_t s_end,
                        void* d_workspace, size_t ws_bytes, double* partial_out, double* per_slice_out) {
  QBE_GUARD_BEGIN
  int rc = check_device_call(ctx, plan, d_workspace);
  if (rc) return rc;
  QBE_REQUIRE(partial_out, "partial_out is NULL");
  QBE_REQUIRE(0 <= s_begin && s_begin < s_end && s_end <= plan->p.n_slices, "bad slice range");
  char* w = (char*)d_workspace;
  rc = qbe::dev_contract(plan->p, ctx->stream, d_workspace, ws_bytes, s_begin, s_end, (double*)w, nullptr);
  if (rc) return rc;
  rc = qbe::dev_memcpy_d2h(partial_out, w, 16, ctx->stream);
  if (rc) return rc;
  if (per_slice_out) rc = qbe::dev_memcpy_d2h(per_slice_out, w + 256, 16 * (size_t)(s_end - s_begin), ctx->stream);
  return rc;
  QBE_GUARD_END
}

int qbe_contract(qbe_ctx* ctx, const qbe_plan* plan, void* d_workspace, size_t ws_bytes, double* amp_out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(plan, "NULL argument");
  return qbe_contract_slices(ctx, plan, 0, plan->p.n_slices, d_workspace, ws_bytes, amp_out, nullptr);
  QBE_GUARD_END
}

// -------------------------------------------------------------------- batch

int qbe_batch_create(qbe_ctx* ctx, const qbe_plan* const* plans, int32_t n_plans, qbe_batch** out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(ctx && plans && out && n_plans > 0, "bad argument");
  *out = nullptr;
  auto* b = new qbe_batch;
  std::unique_ptr<qbe_batch> guard(b);
  for (int i = 0; i < n_plans; ++i) {
    QBE_REQUIRE(plans[i] && plans[i]->ctx && plans[i]->p.device == ctx->device, "bad plan in batch");
    QBE_REQUIRE(plans[i]->p.segs.empty(), "plans with fused segments are contracted alone, not in a batch");
    b->b.plans.push_back(&plans[i]->p);
  }
  int rc = qbe::dev_set(ctx->device);
  if (rc) return rc;
  rc = qbe::dev_batch_build(b->b);
  if (rc) {
    qbe::dev_batch_free(b->b);
    return rc;
  }
  b->ctx = ctx;
  *out = guard.release();
  return QBE_OK;
  QBE_GUARD_END
}

int qbe_batch_destroy(qbe_batch* batch) {
  if (batch) {
    (void)qbe::dev_set(batch->ctx->device);
    qbe::dev_batch_free(batch->b);
    delete batch;
  }
  return QBE_OK;
}

int qbe_batch_workspace(const qbe_batch* batch, size_t* ws_bytes_out) {
  QBE_REQUIRE(batch && ws_bytes_out, "NULL argument");
  *ws_bytes_out = qbe::dev_batch_workspace(batch->b);
  return QBE_OK;
}

int qbe_batch_contract_async(qbe_ctx* ctx, const qbe_batch* batch, void* d_workspace, size_t ws_bytes,
                             double* d_amps_out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(ctx && batch && d_workspace && d_amps_out, "NULL argument");
  QBE_REQUIRE(batch->ctx->device == ctx->device, "batch belongs to another device");
  int rc = qbe::dev_set(ctx->device);
  if (rc) return rc;
  return qbe::dev_batch_contract(batch->b, ctx->stream, d_workspace, ws_bytes, d_amps_out);
  QBE_GUARD_END
}

// ------------------------------------------------------------------ permute

int qbe_permute(qbe_ctx* ctx, const void* d_in, void* d_out, int32_t r, const int32_t* perm, int64_t batch) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(ctx, "NULL argument");
  QBE_REQUIRE(0 <= r && r <= 31, "r must lie in [0, 31]");
  QBE_REQUIRE(batch >= 0, "batch must be >= 0");
  QBE_REQUIRE(batch <= (int64_t(1) << (59 - r)), "tensor bytes beyond 2^62");
  if (batch == 0) return QBE_OK;
  QBE_REQUIRE(d_in && d_out, "NULL device pointer");
  QBE_REQUIRE(r == 0 || perm, "perm is NULL");
  std::vector<char> seen(r, 0);
  for (int j = 0; j < r; ++j) {
    QBE_REQUIRE(0 <= perm[j] && perm[j] < r && !seen[perm[j]], "perm is not a permutation of [0, r)");
    seen[perm[j]] = 1;
  }
  const uintptr_t bytes = (uintptr_t)(batch << r) * 8u;
  const uintptr_t a = (uintptr_t)d_in, b = (uintptr_t)d_out;
  QBE_REQUIRE(a + bytes <= b || b + bytes <= a, "d_in and d_out overlap");
  int rc = qbe::dev_set(ctx->device);
  if (rc) return rc;
  return qbe::dev_permute(d_in, d_out, r, perm, batch, ctx->stream);
  QBE_GUARD_END
}

int qbe_contract_batch(qbe_ctx* ctx, const qbe_plan* const* plans, int32_t n_plans, void* d_workspace,
                       size_t ws_bytes, double* amps_out, size_t* ws_needed_out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(ctx && plans && n_plans > 0, "bad argument");
  QBE_REQUIRE(d_workspace || ws_needed_out, "NULL argument");
  qbe_batch* b = nullptr;
  int rc = qbe_batch_create(ctx, plans, n_plans, &b);
  if (rc) return rc;
  std::unique_ptr<qbe_batch, int (*)(qbe_batch*)> guard(b, qbe_batch_destroy);
  // the batch's workspace, then the device copy of the amplitudes
  const size_t head = (qbe::dev_batch_workspace(b->b) + 255) / 256 * 256;
  const size_t need = head + 16 * (size_t)n_plans;
  if (ws_needed_out) *ws_needed_out = need;
  if (!d_workspace) return QBE_OK;
  QBE_REQUIRE(amps_out, "amps_out is NULL");
  if (ws_bytes < need) {
    set_error("workspace of " + std::to_string(ws_bytes) + " bytes, the batch needs " + std::to_string(need));
    return QBE_ERR_MEM_CAP;
  }
  double* d_amps = reinterpret_cast<double*>(static_cast<char*>(d_workspace) + head);
  rc = qbe::dev_batch_contract(b->b, ctx->stream, d_workspace, head, d_amps);
  if (rc) return rc;
  return qbe::dev_memcpy_d2h(amps_out, d_amps, 16 * (size_t)n_plans, ctx->stream);
  QBE_GUARD_END
}

// ---------------------------------------------------------- learned proposal

int32_t qbe_gnn_num_params(void) { return qbe::gnn_num_params(); }

int qbe_gnn_create(qbe_ctx* ctx, uint64_t seed, qbe_gnn** out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(ctx && out, "NULL argument");
  *out = nullptr;
  int rc = qbe::dev_set(ctx->device);
  if (rc) return rc;
  auto* n = new qbe_gnn;
  std::unique_ptr<qbe_gnn> guard(n);
  rc = qbe::gnn_alloc(n->g, ctx->device);
  if (rc) {
    qbe::gnn_free(n->g);
    return rc;
  }
  // Glorot-uniform weights, zero biases, from SplitMix64 (Steele et al. 2014)
  std::vector<float> p(qbe::gnn_num_params(), 0.f);
  uint64_t state = seed;
  auto next = [&]() {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  auto uniform = [&](float lim) { return (float)((double)(next() >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0) * lim; };
  size_t o = 0;
  for (int l = 0; l < qbe::kGnnLayers; ++l) {
    const int din = l == 0 ? qbe::kGnnFeatures : qbe::kGnnHidden;
    const float lim = std::sqrt(6.f / (float)(din + qbe::kGnnHidden));
    for (int i = 0; i < 2 * din * qbe::kGnnHidden; ++i) p[o++] = uniform(lim);
    o += qbe::kGnnHidden;
  }
  const float lim = std::sqrt(6.f / (float)(qbe::kGnnHidden + 1));
  for (int h = 0; h < qbe::kGnnHeads; ++h) {
    for (int i = 0; i < qbe::kGnnHidden; ++i) p[o++] = uniform(lim);
    o += 1;  // the head's bias
  }
  rc = qbe::gnn_set_params(n->g, p.data(), true);
  if (rc) {
    qbe::gnn_free(n->g);
    return rc;
  }
  *out = guard.release();
  return QBE_OK;
  QBE_GUARD_END
}

int qbe_gnn_destroy(qbe_gnn* gnn) {
  if (gnn) {
    (void)qbe::dev_set(gnn->g.device);
    qbe::gnn_free(gnn->g);
    delete gnn;
  }
  return QBE_OK;
}

int qbe_gnn_get_params(const qbe_gnn* gnn, float* params_out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(gnn && params_out, "NULL argument");
  int rc = qbe::dev_set(gnn->g.device);
  if (rc) return rc;
  return qbe::gnn_get_params(gnn->g, params_out);
  QBE_GUARD_END
}

int qbe_gnn_set_params(qbe_gnn* gnn, const float* params) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(gnn && params, "NULL argument");
  int rc = qbe::dev_set(gnn->g.device);
  if (rc) return rc;
  return qbe::gnn_set_params(gnn->g, params, true);
  QBE_GUARD_END
}

static const char kGnnMagic[8] = {'Q', 'B', 'E', 'G', 'N', 'N', '0', '2'};

int qbe_gnn_save(const qbe_gnn* gnn, const char* path) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(gnn && path, "NULL argument");
  int rc = qbe::dev_set(gnn->g.device);
  if (rc) return rc;
  const int32_t n = qbe::gnn_num_params();
  std::vector<float> p(n), m(n), v(n);
  int step = 0;
  rc = qbe::gnn_get_state(gnn->g, p.data(), m.data(), v.data(), &step);
  if (rc) return rc;
  std::unique_ptr<FILE, int (*)(FILE*)> f(std::fopen(path, "wb"), std::fclose);
  QBE_REQUIRE(f, std::string("cannot open ") + path + " for writing");
  const int32_t hdr[2] = {n, (int32_t)step};
  bool ok = std::fwrite(kGnnMagic, 1, 8, f.get()) == 8 && std::fwrite(hdr, 4, 2, f.get()) == 2;
  for (const std::vector<float>* a : {&p, &m, &v}) ok = ok && std::fwrite(a->data(), 4, n, f.get()) == (size_t)n;
  ok = std::fclose(f.release()) == 0 && ok;
  QBE_REQUIRE(ok, std::string("write to ") + path + " failed");
  return QBE_OK;
  QBE_GUARD_END
}

int qbe_gnn_load(qbe_gnn* gnn, const char* path) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(gnn && path, "NULL argument");
  const int32_t n = qbe::gnn_num_params();
  std::unique_ptr<FILE, int (*)(FILE*)> f(std::fopen(path, "rb"), std::fclose);
  QBE_REQUIRE(f, std::string("cannot open ") + path);
  char magic[8];
  int32_t hdr[2];
  QBE_REQUIRE(std::fread(magic, 1, 8, f.get()) == 8 && std::memcmp(magic, kGnnMagic, 8) == 0,
              std::string(path) + " is not a network checkpoint");
  QBE_REQUIRE(std::fread(hdr, 4, 2, f.get()) == 2 && hdr[0] == n && hdr[1] >= 0,
              std::string(path) + ": parameter count or step differs from this network's");
  std::vector<float> p(n), m(n), v(n);
  for (std::vector<float>* a : {&p, &m, &v})
    QBE_REQUIRE(std::fread(a->data(), 4, n, f.get()) == (size_t)n, std::string(path) + " is truncated");
  int rc = qbe::dev_set(gnn->g.device);
  if (rc) return rc;
  return qbe::gnn_set_state(gnn->g, p.data(), m.data(), v.data(), hdr[1]);
  QBE_GUARD_END
}

// Ranges and symmetry of a CSR graph (the transposed aggregation of the
// backward pass relies on symmetry).
static int check_csr(int32_t n, const int32_t* rp, const int32_t* col) {
  if (n <= 0 || !rp) return QBE_ERR_INVALID_ARG;
  if (rp[0] != 0) return QBE_ERR_INVALID_ARG;
  for (int v = 0; v < n; ++v)
    if (rp[v + 1] < rp[v]) return QBE_ERR_INVALID_ARG;
  if (rp[n] > 0 && !col) return QBE_ERR_INVALID_ARG;
  for (int v = 0; v < n; ++v)
    for (int j = rp[v]; j < rp[v + 1]; ++j) {
      const int w = col[j];
      if (w < 0 || w >= n || w == v) return QBE_ERR_INVALID_ARG;
      bool back = false;
      for (int k = rp[w]; k < rp[w + 1] && !back; ++k) back = col[k] == v;
      if (!back) return QBE_ERR_INVALID_ARG;
    }
  return QBE_OK;
}

int qbe_gnn_score_head(qbe_ctx* ctx, qbe_gnn* gnn, int32_t head, int32_t n, const int32_t* rowptr,
                       const int32_t* col, const float* feats, float* scores_out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(ctx && gnn && feats && scores_out, "NULL argument");
  QBE_REQUIRE(head >= 0 && head < qbe::kGnnHeads, "bad head");
  QBE_REQUIRE(check_csr(n, rowptr, col) == QBE_OK, "graph is not a symmetric CSR over n vertices");
  int rc = qbe::dev_set(ctx->device);
  if (rc) return rc;
  return qbe::gnn_score(gnn->g, ctx->stream, head, n, rowptr, col, feats, scores_out);
  QBE_GUARD_END
}

int qbe_gnn_score(qbe_ctx* ctx, qbe_gnn* gnn, int32_t n, const int32_t* rowptr, const int32_t* col,
                  const float* feats, float* scores_out) {
  return qbe_gnn_score_head(ctx, gnn, QBE_HEAD_SLICING, n, rowptr, col, feats, scores_out);
}

int qbe_gnn_train_step_head(qbe_ctx* ctx, qbe_gnn* gnn, int32_t head, int32_t n, const int32_t* rowptr,
                            const int32_t* col, const float* feats, int32_t n_cand, const int32_t* cand,
                            const float* target, float lr, float* loss_out, float* grads_out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(ctx && gnn && feats, "NULL argument");
  QBE_REQUIRE(head >= 0 && head < qbe::kGnnHeads, "bad head");
  QBE_REQUIRE(check_csr(n, rowptr, col) == QBE_OK, "graph is not a symmetric CSR over n vertices");
  QBE_REQUIRE(n_cand >= 0 && (n_cand == 0 || (cand && target)), "bad candidates");
  std::vector<uint8_t> seen(n, 0);
  for (int i = 0; i < n_cand; ++i) {
    QBE_REQUIRE(cand[i] >= 0 && cand[i] < n && !seen[cand[i]], "candidates must be distinct vertex ids");
    seen[cand[i]] = 1;
  }
  int rc = qbe::dev_set(ctx->device);
  if (rc) return rc;
  return qbe::gnn_train_step(gnn->g, ctx->stream, head, n, rowptr, col, feats, n_cand, cand, target, lr,
                             loss_out, grads_out);
  QBE_GUARD_END
}

int qbe_gnn_train_step(qbe_ctx* ctx, qbe_gnn* gnn, int32_t n, const int32_t* rowptr, const int32_t* col,
                       const float* feats, int32_t n_cand, const int32_t* cand, const float* target, float lr,
                       float* loss_out, float* grads_out) {
  return qbe_gnn_train_step_head(ctx, gnn, QBE_HEAD_SLICING, n, rowptr, col, feats, n_cand, cand, target, lr,
                                 loss_out, grads_out);
}

int qbe_graph_csr(const qbe_model* model, const int32_t* removed, int32_t n_removed, int32_t* rowptr_out,
                  int32_t* col_out, int64_t cap, int64_t* nnz_out) {
  QBE_GUARD_BEGIN
  QBE_REQUIRE(model && rowptr_out && nnz_out, "NULL argument");
  qbe::Graph g = graph_of(model->m);
  for (int v : vec(removed, n_removed)) {
    QBE_REQUIRE(v >= 0 && v < g.n && g.present[v], "bad removed vertex");
    g.remove_vertex(v);
  }
  int64_t nnz = 0;
  for (int v = 0; v < g.n; ++v) nnz += g.degree(v);
  *nnz_out = nnz;
  if (nnz > cap || (nnz > 0 && !col_out)) {
    set_error("col capacity too small");
    return QBE_ERR_MEM_CAP;
  }
  int64_t o = 0;
  for (int v = 0; v < g.n; ++v) {
    rowptr_out[v] = (int32_t)o;
    for (int w : g.neighbours(v)) col_out[o++] = w;
  }
  rowptr_out[g.n] = (int32_t)o;
  return QBE_OK;
  QBE_GUARD_END
}

}  // extern "C"
