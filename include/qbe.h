/*
 * qbe.h -- sliced bucket-elimination contraction of tensor networks
 * (graphical-model form), MI355X / gfx950.
 *
 * The library computes sigma = sum over all variable assignments of the
 * product of a network's tensors (Sec. 2.1, Eq. 1-2 of Schutski, Kolmakov,
 * Khakhulin and Oseledets, "Simple heuristics for efficient parallel tensor
 * contraction and quantum circuit simulation"), by bucket elimination along
 * an elimination order (Eq. 2) after fixing a set mu of variables (Eq. 3),
 * and sums the 2^|mu| independent slices (Eq. 4).  For a quantum circuit the
 * network's sum is the amplitude <x|C|0^n>.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Variables are binary (dimension L = 2) and numbered 0 .. n_vars-1.
 *  - A tensor of rank r over variables (v_0 .. v_{r-1}) holds 2^r complex
 *    entries, row-major with v_0 the most significant index; complex data is
 *    passed as interleaved (re, im) doubles.
 *  - Slice s (0 <= s < 2^m) of a sliced set mu = (mu_0 .. mu_{m-1}) fixes
 *    mu_j to bit j of s.
 *  - Every call returns QBE_OK (0) or a negative QBE_ERR_* code; no C++
 *    exception or abort crosses the ABI.  qbe_last_error() returns a
 *    thread-local description of the last failure on the calling thread.
 *  - Host arrays passed in are only read during the call; the library keeps
 *    its own copies.  Output arrays are caller-allocated with the sizes given.
 *  - Handles are opaque and owned by the caller until the matching destroy
 *    call.  A handle may be used by one thread at a time.
 */
#ifndef QBE_H
#define QBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  QBE_OK = 0,
  QBE_ERR_INVALID_ARG = -1, /* bad argument, inconsistent sizes or ids      */
  QBE_ERR_OOM = -2,         /* host or device allocation failed            */
  QBE_ERR_HIP = -3,         /* a HIP runtime call failed                   */
  QBE_ERR_MEM_CAP = -4,     /* workspace too small / plan exceeds a cap    */
  QBE_ERR_INTERNAL = -5,    /* library invariant violated (a bug)          */
  QBE_ERR_NO_DEVICE = -6    /* no usable GPU for a device call             */
};

/* Scores for the greedy mu-treewidth deletion (Alg. 2). */
enum {
  QBE_SCORE_TREE_TRIMMING = 0, /* Sec. 3.2                                 */
  QBE_SCORE_DEGREE = 1,        /* Sec. 3.1, number of neighbours            */
  QBE_SCORE_TW_REDUCTION = 2,  /* Sec. 3.1, Alg. 3 (direct width drop)      */
  QBE_SCORE_BETWEENNESS = 3,   /* Sec. 3.1, betweenness centrality
                                  (unnormalised; ties to the earliest vertex
                                  of the order after rounding to 1e-9)     */
  QBE_SCORE_LEARNED = 4        /* the network's slicing head (qbe_slice_ex
                                  only: it needs a network and a device)   */
};

/* Heads of the learned proposal's network. */
enum {
  QBE_HEAD_SLICING = 0,     /* predicted total cost after slicing a variable */
  QBE_HEAD_ELIMINATION = 1  /* predicted total cost after eliminating it next */
};

/* Device execution forms of a plan. */
enum {
  QBE_EXEC_AUTO = 0,       /* fused when a slice fits in LDS, else per-step */
  QBE_EXEC_PER_STEP = 1,   /* one kernel launch per bucket, slices batched   */
  QBE_EXEC_FUSED = 2       /* one persistent launch, a slice per workgroup,
                              all intermediates in LDS                       */
};

/* Arithmetic of the bucket products on the device. */
enum {
  QBE_PREC_FP32 = 0,    /* complex64 products, FP32 accumulation            */
  QBE_PREC_BF16X3 = 1,  /* split-BF16 products (hi*hi + hi*lo + lo*hi) with
                           FP32 accumulation in the MFMA launches of the
                           per-step form (outer-product buckets and merged
                           two-group products); other launches stay FP32.
                           Not available in the fused form.  About 2^-16
                           relative error per product.                       */
  QBE_PREC_BF16X6 = 2   /* as BF16X3 with a three-part split x = h + m + l
                           and the six products h*h, h*m, m*h, h*l, l*h,
                           m*m: about FP32 accuracy from bfloat16 MFMAs.     */
};

typedef struct qbe_ctx qbe_ctx;
typedef struct qbe_model qbe_model;
typedef struct qbe_plan qbe_plan;
typedef struct qbe_batch qbe_batch;
typedef struct qbe_gnn qbe_gnn;

typedef struct qbe_plan_opts {
  int32_t exec;        /* QBE_EXEC_*                                         */
  int32_t precision;   /* QBE_PREC_*                                         */
  int32_t block;       /* threads per workgroup for per-step kernels; 0 = tuned */
  int32_t no_merge;    /* 1: one launch per bucket in the per-step form and
                          one level per bucket depth in the fused form (no
                          merging of bucket chains); 0: merge (default)      */
  int32_t fused_prefix; /* > 0: a per-step plan contracts its small buckets
                          -- every bucket of at most R + 1 variables whose
                          producers all are such -- in one LDS-resident
                          launch of the fused form's executor (FP32,
                          whatever the plan's precision) before its
                          per-step launches, which read the results it
                          writes to the workspace.  1: R is the largest of
                          14 .. 4 whose prefix -- and with fused_segments
                          its later segments too -- lets two workgroups
                          share a compute unit's LDS, else the largest
                          whose prefix does, else the largest of 10, 8,
                          6, 4 that fits at all; 2..14: R = fused_prefix.
                          Needs merging (no_merge 0) and at most 24 sliced
                          variables; a plan with no such prefix (fewer
                          than two small buckets, or it does not fit LDS)
                          runs without one (stats.prefix_buckets 0).
                          Ignored by plans that run in the fused form.
                          0: no prefix (default); other values:
                          QBE_ERR_INVALID_ARG                               */
  int32_t fused_segments; /* 1 (with fused_prefix > 0 and a prefix): every
                          later connected run of at least three buckets of
                          at most R + 1 variables (connected through the
                          buckets that read their results) is contracted
                          by one more such launch, which reads the larger
                          results it needs from the workspace and writes
                          its top bucket's result there; a run that does
                          not fit LDS stays per-step launches.  0: none
                          (default)                                         */
  int32_t no_fold;     /* 0 (default): the input tensors of a bucket (two or
                          more, over at most 6 variables together) are
                          multiplied into one tensor once per plan, in
                          complex128, so that each entry of the bucket
                          multiplies fewer factors (Eq. 2's product,
                          regrouped); 1: every input tensor stays a factor
                          of its own.  The plan's schedule dump and cost
                          model are the caller's model's either way.       */
  int32_t max_sums;    /* 0 (default): a merged per-step launch sums up to 4
                          variables (2^4 terms per result entry); 1..4:
                          at most that many (1: one launch per bucket, as
                          no_merge for the per-step launches; fused levels
                          still merge).  Fewer terms per entry cost more
                          launches and device-memory round trips; which is
                          faster depends on the plan.  Other values:
                          QBE_ERR_INVALID_ARG                               */
} qbe_plan_opts;

typedef struct qbe_stats {
  int32_t n_vars, n_tensors, m, width; /* width: largest |U_b| - 1          */
  int32_t n_steps, n_levels;           /* levels: dependency depth of steps  */
  int32_t exec;                        /* form chosen for this plan          */
  int32_t lds_bytes;                   /* LDS per workgroup (fused form)     */
  uint64_t flops_per_slice;            /* cost model, real flops             */
  uint64_t bytes_per_slice;            /* algorithmic complex64 bytes        */
  uint64_t peak_bytes_per_slice;       /* live-tensor peak                   */
  uint64_t ws_bytes_min;               /* smallest workspace contract accepts */
  uint64_t ws_bytes_all_slices;        /* workspace for all slices at once   */
  int32_t n_mfma_steps;                /* per-step form: launches run as
                                          MFMA tiles (outer-product buckets
                                          and merged products)               */
  int32_t precision;                   /* QBE_PREC_* of the plan             */
  int32_t fused_levels;                /* fused form: levels of its program
                                          (buckets merged along chains; 0 if
                                          the plan has no fused program)     */
  int32_t n_merged_steps;              /* per-step form: launches that merge
                                          a chain of buckets (several summed
                                          variables)                         */
  uint64_t step_bytes_per_slice;       /* per-step form: complex64 bytes its
                                          launches read and write per slice
                                          (below bytes_per_slice when chains
                                          are merged)                        */
  int32_t n_launches;                  /* per-step form: contraction launches
                                          per slice group (a merged chain, a
                                          partial product or a fused segment
                                          counts once)                       */
  int32_t prefix_buckets;              /* per-step form: buckets contracted
                                          by the fused prefix (0: none)      */
  int32_t n_fused_segments;            /* per-step form: fused launches (the
                                          prefix and later segments)         */
  int32_t fused_buckets;               /* buckets they contract              */
} qbe_stats;

/* ------------------------------------------------------------------ misc -- */

/* Thread-local text of the last error ("" if none).  Never NULL. */
const char* qbe_last_error(void);
/* Library ABI version (this header: 1). */
int32_t qbe_version(void);

/* ------------------------------------------------------------- context ---- */

/* Binds device `device` and a borrowed HIP stream (hipStream_t passed as
 * void*; NULL = the default stream).  All device work of calls that take
 * the context is enqueued on that stream.  QBE_ERR_NO_DEVICE without a GPU. */
int qbe_create(qbe_ctx** out, int32_t device, void* hip_stream);
int qbe_destroy(qbe_ctx* ctx);
/* Replaces the borrowed stream. */
int qbe_set_stream(qbe_ctx* ctx, void* hip_stream);

/* --------------------------------------------------------------- model ---- */

/* The graphical model (Sec. 2.1): n_vars binary variables and n_tensors
 * tensors.  rank[t] in [0, 30]; vars holds sum(rank) variable ids
 * (tensor by tensor, no repeats within a tensor); data holds
 * 2 * sum(2^rank[t]) doubles (interleaved re, im; tensor by tensor).
 * Every variable must occur in at least one tensor.  All arrays are copied. */
int qbe_model_create(int32_t n_vars, int32_t n_tensors, const int32_t* rank, const int32_t* vars,
                     const double* data, qbe_model** out);
/* A network whose variables have any dimensions L_v = dims[v] >= 1 (Sec.
 * 2.1 allows any L; the contraction is the same sum over all assignments).
 * It is stored as the equivalent binary model: variable v becomes b_v =
 * ceil(log2 L_v) binary variables (its index bits, most significant
 * first; none for L_v = 1), numbered consecutively in v order, and every
 * tensor is re-laid out over its variables' bits with entries 0 at index
 * values >= L_v.  Every later call (orders, slicing, plans, contraction)
 * works on that binary model: slicing may fix single bits of a variable.
 * Tensor t over (v_0 .. v_{r-1}) holds prod L_{v_j} complex entries,
 * row-major with v_0 the most significant; data holds 2 * sum of those
 * doubles.  Limits: dims[v] in [1, 2^16], sum of b over a tensor's
 * variables <= 30.  Every variable must occur in a tensor.
 * QBE_ERR_INVALID_ARG otherwise. */
int qbe_model_create_dims(int32_t n_vars, const int32_t* dims, int32_t n_tensors, const int32_t* rank,
                          const int32_t* vars, const double* data, qbe_model** out);
/* The binary variables of variable v of a qbe_model_create_dims model:
 * *first_out, *count_out (count 0 for dimension 1).  For a binary model
 * every variable maps to itself (count 1). */
int qbe_model_var_bits(const qbe_model* model, int32_t v, int32_t* first_out, int32_t* count_out);
int qbe_model_destroy(qbe_model* model);
/* Replaces the tensor entries (same layout as qbe_model_create). */
int qbe_model_set_data(qbe_model* model, const double* data);

/* ------------------------------------------------------------- planning --- */

/* Greedy min-fill elimination order of the model's simple graph (tensors
 * are cliques, Sec. 2.2): fewest fill edges, then smallest degree, then
 * smallest id.  order_out: n_vars entries. */
int qbe_order_min_fill(const qbe_model* model, int32_t* order_out);

/* Alg. 1 (Sec. 2.3): the largest number of not-yet-eliminated neighbours
 * met while eliminating along `order` (n entries, a permutation of the
 * vertices that are not in `removed`).  removed: n_removed vertex ids
 * deleted from the graph first (may be NULL when n_removed == 0). */
int qbe_width(const qbe_model* model, const int32_t* order, int32_t n, const int32_t* removed,
              int32_t n_removed, int32_t* tau_out);

/* App. A: the tree decomposition of the order, as its maximal cliques.
 * Outputs: *n_bags; bag_offsets[n_bags + 1] (capacity n + 1) and bag_vars
 * (capacity cap_vars; ids ascending inside a bag); parent[n_bags] (capacity
 * n, -1 for a root).  Bags are listed by their earliest-eliminated vertex.
 * QBE_ERR_MEM_CAP if cap_vars is too small (*n_bags still set). */
int qbe_clique_tree(const qbe_model* model, const int32_t* order, int32_t n, int32_t* n_bags,
                    int32_t* bag_offsets, int32_t* bag_vars, int64_t cap_vars, int32_t* parent);

/* Alg. 2 (Sec. 3): greedy mu-treewidth deletion from the order `order`
 * (n = n_vars entries).  m >= 0 removes exactly m variables; m < 0 removes
 * variables until the width of the reduced order is <= target_width.
 * score: QBE_SCORE_*.  Outputs: mu_out (capacity n), *m_out,
 * reduced_order_out (capacity n; n - *m_out entries), *tau_out. */
int qbe_slice(const qbe_model* model, const int32_t* order, int32_t n, int32_t m,
              int32_t target_width, int32_t score, int32_t* mu_out, int32_t* m_out,
              int32_t* reduced_order_out, int32_t* tau_out);
/* Options of qbe_slice_ex: Alg. 2 with its score f, its stopping rule and
 * its optional order recomputation. */
typedef struct qbe_slice_opts {
  int32_t score;           /* QBE_SCORE_*                                     */
  int32_t m;               /* >= 0: remove exactly m variables; < 0: remove
                              until the stop rules below hold               */
  int32_t target_width;    /* m < 0: stop once the reduced order's width is
                              <= target_width (< 0: no width rule)          */
  int32_t recompute_every; /* > 0: recompute the order after every k-th
                              removal as qbe_slice_recompute does; 0: never */
  int32_t tries;           /* anytime heuristic tries of the recomputation  */
  int32_t reserved0;       /* must be zero                                  */
  uint64_t seed;           /* anytime heuristic seed                        */
  uint64_t mem_cap;        /* m < 0: also stop only once the peak live bytes
                              per slice (cost model) are <= mem_cap (0: no
                              memory rule).  QBE_SCORE_LEARNED: if the
                              network's sliced set misses the cap, the
                              result is tree-trimming's under the same rules
                              (the heuristic remains the fallback)          */
  uint64_t reserved[2];    /* must be zero                                  */
} qbe_slice_opts;

/* Alg. 2 (Sec. 3) whose score f may be the learned proposal's network
 * (QBE_SCORE_LEARNED: among the vertices of the maximum bags of App. A's
 * tree -- tree-trimming's candidates -- the one the slicing head predicts
 * cheapest, ties to the earliest in the order; the network is re-run on the
 * reduced graph after every removal).  ctx and gnn are needed only for the
 * learned score (else may be NULL).  Outputs as qbe_slice; *fell_back_out
 * (optional) = 1 when the memory-cap fallback replaced the learned result.
 * QBE_ERR_INVALID_ARG for bad options (m < 0 needs a width or memory rule). */
int qbe_slice_ex(qbe_ctx* ctx, qbe_gnn* gnn, const qbe_model* model, const int32_t* order, int32_t n,
                 const qbe_slice_opts* opts, int32_t* mu_out, int32_t* m_out, int32_t* reduced_order_out,
                 int32_t* tau_out, int32_t* fell_back_out);

/* An elimination order (Sec. 2.2's order problem) from greedy min-fill
 * whose ties in fill go to the network's elimination head (lower predicted
 * cost first; then smaller degree, then smaller id).  The head is evaluated
 * on the current elimination graph, with the features of that graph's
 * greedy min-fill order, before the first elimination and after every
 * `refresh` eliminations.  The min-fill order remains the fallback: the
 * result is whichever of the two orders has fewer exact total FLOPs
 * (cost model, no slicing); *fell_back_out (optional) = 1 when that is
 * min-fill's.  flops_out (optional, 2 entries): the learned and the
 * min-fill order's total FLOPs.  order_out: n_vars entries; *width_out its
 * width (Alg. 1). */
int qbe_order_learned(qbe_ctx* ctx, qbe_gnn* gnn, const qbe_model* model, int32_t refresh,
                      int32_t* order_out, int32_t* width_out, int32_t* fell_back_out, uint64_t* flops_out);

/* One training sample of the learned proposal, labelled with the method's
 * own exact costs (the cost model of qbe_schedule_cost):
 *  - head QBE_HEAD_SLICING: the state is the graph without mu (m entries)
 *    and its order (n = n_vars - m entries); the candidates are the
 *    vertices of the maximum bags; the label of candidate c is log2 of the
 *    total FLOPs (2^(m + 1) slices) of removing c as well;
 *  - head QBE_HEAD_ELIMINATION: the state is the elimination graph after
 *    eliminating order[0 .. k_elim) (n = n_vars, m = 0); the candidates are
 *    its vertices of minimum fill; the label of c is log2 of the total FLOPs
 *    (no slicing) of the order prefix, c, then greedy min-fill of the rest.
 * At most max_cand (>= 2) candidates are kept (a SplitMix64(seed) sample),
 * ascending ids; labels are standardised within the sample: (y - mean) /
 * max(std, 0.05).  Outputs: the state graph as CSR over all n_vars ids
 * (rowptr_out[n_vars + 1], col_out of capacity col_cap, *nnz_out; MEM_CAP if
 * short), features (feats_out[8 n_vars], qbe_vertex_features of the state
 * and -- for elimination -- its min-fill order), cand_out / target_out
 * (max_cand entries) and *n_cand_out (fewer than 2: no labels written). */
int qbe_learned_sample(const qbe_model* model, int32_t head, const int32_t* order, int32_t n, const int32_t* mu,
                       int32_t m, int32_t k_elim, int32_t max_cand, uint64_t seed, int32_t* rowptr_out,
                       int32_t* col_out, int64_t col_cap, int64_t* nnz_out, float* feats_out, int32_t* cand_out,
                       float* target_out, int32_t* n_cand_out);

/* Alg. 2 with its optional line (Sec. 3): after every recompute_every-th
 * removal (> 0) the reduced order is recomputed on the reduced graph: the
 * anytime order of qbe_order_anytime(tries, seed) is turned into its tree
 * decomposition (App. A) and back into an order by Alg. 5 (App. B), the
 * route an external tree-decomposition solver's output would take.
 * recompute_every = 0 is qbe_slice.  Arguments and outputs as qbe_slice;
 * tries >= 1.  QBE_ERR_INVALID_ARG for a bad order, m, score or tries. */
int qbe_slice_recompute(const qbe_model* model, const int32_t* order, int32_t n, int32_t m,
                        int32_t target_width, int32_t score, int32_t recompute_every, int32_t tries,
                        uint64_t seed, int32_t* mu_out, int32_t* m_out, int32_t* reduced_order_out,
                        int32_t* tau_out);

/* The project's anytime tree-decomposition heuristic, standing in for the
 * external solver of Sec. 4: greedy min-fill, then tries - 1 min-fill runs
 * whose (fill, degree) ties go to SplitMix64(seed) priorities (one draw per
 * remaining vertex in ascending id order per run); the first order of the
 * smallest width (Alg. 1) wins.  removed: vertices deleted first (may be
 * NULL when n_removed == 0).  Outputs: order_out (capacity n_vars; n_vars -
 * n_removed entries), *width_out.  tries >= 1. */
int qbe_order_anytime(const qbe_model* model, const int32_t* removed, int32_t n_removed, int32_t tries,
                      uint64_t seed, int32_t* order_out, int32_t* width_out);

/* App. B, Alg. 5: an elimination order consistent with a tree decomposition
 * of n_bags bags over vertices [0, n_vars): bag i holds bag_vars[bag_offsets
 * [i] .. bag_offsets[i + 1]) (ids ascending), parent[i] its parent bag or -1
 * for a root (a forest is allowed).  Repeatedly the first non-root leaf (in
 * bag order) gives the vertices it has and its parent lacks (ascending ids)
 * and is removed; the roots' vertices come last.  Outputs: order_out
 * (capacity n_vars), *n_out = vertices listed.  QBE_ERR_INVALID_ARG for ids
 * out of range, unsorted bags, a parent array that is not a forest, or a
 * vertex listed twice (a decomposition without the running-intersection
 * property). */
int qbe_order_from_td(int32_t n_vars, int32_t n_bags, const int32_t* bag_offsets, const int32_t* bag_vars,
                      const int32_t* parent, int32_t* order_out, int32_t* n_out);

/* Exact cost (the project's cost model for Sec. 4's per-subtask memory and
 * FLOPs) of contracting with the reduced order and sliced set, without
 * building device programs: out[0] = real FLOPs per slice, out[1] =
 * algorithmic complex64 bytes per slice, out[2] = peak live bytes per slice,
 * out[3] = largest |U_b| - 1.  Totals are 2^m times the per-slice counts. */
int qbe_schedule_cost(const qbe_model* model, const int32_t* reduced_order, int32_t n, const int32_t* mu,
                      int32_t m, uint64_t* out);

/* Features of every variable for the learned slicing proposal, computed on
 * the graph without the `removed` variables and its order `order` (a
 * permutation of the remaining ones): 8 floats per variable (degree,
 * relative order position, |N+(u)| / width, membership of a maximum bag of
 * the App. A tree, bags holding u and their total size relative to the
 * maxima, largest bag / 32, 1).  Rows of removed variables are zero.
 * feats_out: 8 * n_vars floats. */
int qbe_vertex_features(const qbe_model* model, const int32_t* order, int32_t n, const int32_t* removed,
                        int32_t n_removed, float* feats_out);

/* Compiles the bucket schedule (Eq. 2) of the reduced order and the sliced
 * set, the device programs and their memory layout.  ctx may be NULL for a
 * host-only plan (stats and dump work, contraction calls fail with
 * QBE_ERR_INVALID_ARG).  With a context the model's tensors are uploaded to
 * device memory owned by the plan.  opts may be NULL (all defaults). */
int qbe_plan_create(qbe_ctx* ctx, const qbe_model* model, const int32_t* reduced_order, int32_t n,
                    const int32_t* mu, int32_t m, const qbe_plan_opts* opts, qbe_plan** out);
int qbe_plan_destroy(qbe_plan* plan);
/* Re-uploads tensor entries from the model (same structure) to the plan. */
int qbe_plan_update_data(qbe_plan* plan, const qbe_model* model);
/* A new plan for a model with the same structure as src's (every tensor on
 * the same variables, in the same order) but other entries -- e.g. another
 * output bitstring of the same circuit, which changes only the rank-1
 * tensors on the output variables.  Slicing and schedule depend on the graph
 * alone (Sec. 2.4, Eq. 3-4), so src's order, sliced set, schedule, programs
 * and autotuned tile shapes are reused without planning or compiling again.
 * The clone is bound to src's context (if any) and owns its device memory:
 * it shares no buffer with src, and either may be destroyed first.
 * Errors: QBE_ERR_INVALID_ARG for NULL arguments or a model whose
 * structure differs from src's; device allocation errors as for
 * qbe_plan_create. */
int qbe_plan_clone(const qbe_plan* src, const qbe_model* model, qbe_plan** out);
int qbe_plan_stats(const qbe_plan* plan, qbe_stats* out);
/* Canonical text of the schedule: order, mu, scalar inputs, free
 * variables, then one line per bucket (eliminated variable, operands,
 * U_b and result variables).  Writes min(cap, len + 1) bytes (NUL
 * terminated when it fits); *len_out = full length without the NUL. */
int qbe_plan_dump(const qbe_plan* plan, char* buf, size_t cap, size_t* len_out);

/* Autotuner for the per-step form: times each bucket kernel whose launch
 * covers at least min_elems result entries in every candidate tile shape
 * (tiles per thread in {1, 2, 4} x workgroups per compute unit in {4, 8, 16,
 * 32}) on the device, with the workspace the contraction will use, and keeps
 * the fastest shape in the plan.  In an FP32 plan a merged launch that runs
 * as an MFMA product is also timed on the VALU kernels, and the faster form
 * is kept (both are FP32 products; the sums' rounding order differs, so a
 * tuned plan's bits may differ from the untuned plan's within FP32
 * rounding).  Blocks until done.  Plans in the fused form have nothing to
 * tune (QBE_OK).  The workspace contents are overwritten. */
int qbe_plan_autotune(qbe_ctx* ctx, qbe_plan* plan, void* d_workspace, size_t ws_bytes,
                      int64_t min_elems);

/* Per-launch view of a per-step plan (diagnostics and measurement): the
 * execution order's launches -- a single bucket, a merged chain of buckets
 * (several summed variables), a partial product of a wide bucket, a group
 * of small buckets of one level, or a fused segment -- then the per-slice
 * FP64 product of the rank-0 results (finalize) and the slice sum (reduce,
 * Eq. 4). */
enum {
  QBE_LAUNCH_BUCKET = 0,
  QBE_LAUNCH_MERGED = 1,
  QBE_LAUNCH_PARTIAL = 2,
  QBE_LAUNCH_GROUP = 3,
  QBE_LAUNCH_FINALIZE = 4,
  QBE_LAUNCH_REDUCE = 5,
  QBE_LAUNCH_PREFIX = 6,  /* the fused prefix: bytes_per_slice counts its
                             inputs and exported results once (its other
                             intermediates stay in LDS)                   */
  QBE_LAUNCH_SEGMENT = 7  /* a later fused segment: n_ops = its imported
                             results; bytes_per_slice also counts them    */
};
typedef struct qbe_launch_info {
  int32_t kind;              /* QBE_LAUNCH_*                                  */
  int32_t n_buckets;         /* buckets the launch contracts (chain length,
                                group size)                                   */
  int32_t n_ops;             /* operands (largest in a group; imported
                                results of a fused segment)                   */
  int32_t out_rank;          /* result rank (largest in a group; the bound R
                                of a fused segment's buckets)                 */
  int32_t n_sum;             /* summed variables per result entry             */
  int32_t mfma;              /* 1: runs on MFMA tiles                         */
  uint64_t bytes_per_slice;  /* algorithmic complex64 bytes: each operand read
                                once, the result written once                 */
  uint64_t flops_per_slice;  /* real flops: per result entry 2^n_sum terms of
                                n_ops - 1 complex products (6 flops each) and
                                their sum                                     */
  int32_t levels;            /* fused segments: levels of its program
                                (barriers per slice); 0 for other launches    */
  int32_t lds_bytes;         /* fused segments: LDS per workgroup; 0 otherwise */
} qbe_launch_info;
/* Launches of a per-step plan (its execution order + 2); 0 for a fused
 * plan. */
int qbe_plan_num_launches(const qbe_plan* plan, int32_t* n_out);
/* Launch i (0 <= i < qbe_plan_num_launches) of a per-step plan. */
int qbe_plan_launch_info(const qbe_plan* plan, int32_t i, qbe_launch_info* out);

/* ------------------------------------------------------------ contraction - */

/* Contracts all 2^m slices and sums them (Eq. 4) in FP64.  d_workspace is a
 * caller-owned device buffer of ws_bytes >= stats.ws_bytes_min (more lets
 * more slices run concurrently).  Blocks until the amplitude is on the host:
 * amp_out[0] = re, amp_out[1] = im. */
int qbe_contract(qbe_ctx* ctx, const qbe_plan* plan, void* d_workspace, size_t ws_bytes,
                 double* amp_out);

/* Contracts slices [s_begin, s_end) only; partial_out gets their FP64 sum
 * (2 doubles), per_slice_out (optional, 2 * (s_end - s_begin) doubles) each
 * slice's value. */
int qbe_contract_slices(qbe_ctx* ctx, const qbe_plan* plan, int64_t s_begin, int64_t s_end,
                        void* d_workspace, size_t ws_bytes, double* partial_out,
                        double* per_slice_out);

/* Enqueues the contraction of all slices without waiting: the FP64 result
 * (2 doubles) is written to device memory d_amp_out.  No host
 * synchronisation, allocation or copy happens inside, so the call may be
 * captured into a HIP graph; the workspace must stay untouched until the
 * stream has passed the call. */
int qbe_contract_async(qbe_ctx* ctx, const qbe_plan* plan, void* d_workspace, size_t ws_bytes,
                       double* d_amp_out);

/* ---------------------------------------------------------- slice ledger - */

/* A host record of which slice ranges of one contraction are done and their
 * FP64 partial sums, for recovery after a failure and for resuming an
 * interrupted job.  The slices are independent subtasks (Sec. 2.4) whose
 * sum is the result (Eq. 4), so a range whose result was lost or rejected is
 * contracted again alone and the others are kept.  A ledger splits slices
 * 0 .. n_slices-1 into ranges of range_size slices (the last one shorter):
 * range i = [i * range_size, min(n_slices, (i + 1) * range_size)).  `tag` is
 * the caller's 64-bit name of the work (circuit, bitstring, plan); the
 * ledger stores it and never interprets it.  Host only: no call here except
 * qbe_ledger_run touches a device. */
typedef struct qbe_ledger qbe_ledger;
/* QBE_ERR_INVALID_ARG unless n_slices >= 1 and range_size >= 1. */
int qbe_ledger_create(int64_t n_slices, int64_t range_size, uint64_t tag, qbe_ledger** out);
int qbe_ledger_destroy(qbe_ledger* ledger);
/* Any output pointer may be NULL. */
int qbe_ledger_info(const qbe_ledger* ledger, int64_t* n_slices, int64_t* range_size, uint64_t* tag,
                    int64_t* n_ranges, int64_t* n_done);
/* The lowest pending range: its index and slice bounds, or *idx_out = -1
 * (bounds 0) when every range is done. */
int qbe_ledger_next(const qbe_ledger* ledger, int64_t* idx_out, int64_t* s_begin_out, int64_t* s_end_out);
/* Records range idx's partial sum partial[2] = (re, im).  QBE_ERR_INVALID_ARG
 * (ledger unchanged) when idx is out of range, the range is already done, or
 * a value is not finite (a failed contraction is not accepted as a result). */
int qbe_ledger_record(qbe_ledger* ledger, int64_t idx, const double* partial);
/* Marks range idx pending again (its result judged lost or wrong). */
int qbe_ledger_drop(qbe_ledger* ledger, int64_t idx);
/* *done_out = 1 and partial_out[2] = the recorded sum, or 0 and (0, 0). */
int qbe_ledger_get(const qbe_ledger* ledger, int64_t idx, int32_t* done_out, double* partial_out);
/* Contracts up to max_ranges pending ranges (all if max_ranges < 0), lowest
 * first, each by qbe_contract_slices with the caller's workspace, recording
 * each as it completes; *n_run_out (may be NULL) = ranges recorded by this
 * call.  QBE_ERR_INVALID_ARG when the plan's 2^m differs from the ledger's
 * n_slices.  When a range fails, the call returns that range's error code;
 * the ranges recorded before it stay recorded, the failed one stays
 * pending. */
int qbe_ledger_run(qbe_ctx* ctx, const qbe_plan* plan, qbe_ledger* ledger, void* d_workspace, size_t ws_bytes,
                   int64_t max_ranges, int64_t* n_run_out);
/* amp_out[2] = the sum of the recorded partials in range order, in FP64.
 * QBE_ERR_INVALID_ARG while any range is pending. */
int qbe_ledger_sum(const qbe_ledger* ledger, double* amp_out);
/* The ledger as a file at a caller path.  Layout (native little-endian): the
 * 8 bytes "QBELDG01", int64 n_slices, int64 range_size, uint64 tag, then per
 * range an int64 done flag (0 or 1) and two float64 (re, im).  Loading
 * returns a new ledger; QBE_ERR_INVALID_ARG for a file that cannot be opened,
 * written or read in full, has another magic or inconsistent sizes, a flag
 * other than 0 or 1, or a non-finite recorded value, or has bytes after the
 * last range. */
int qbe_ledger_save(const qbe_ledger* ledger, const char* path);
int qbe_ledger_load(const char* path, qbe_ledger** out);

/* ------------------------------------------------ allocation-free entry - */

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the
 * contraction of qbe_contract_async with the library's own fixed device
 * workspace instead of a caller's.  Enqueues all slices on the context's
 * stream and writes the FP64 amplitude (2 doubles) to device memory
 * d_amp_out; no allocation, free, copy or synchronisation happens inside.
 * The workspace is one array of qbe_static_scratch_bytes() bytes per device,
 * held from the library's first use on that device (qbe_create) until the
 * process ends, and shared by every call on that device: calls that overlap
 * on one device (other streams or threads) race on it and must be ordered
 * by the caller.  QBE_ERR_MEM_CAP (nothing enqueued) when the plan's
 * stats.ws_bytes_min exceeds that size; other errors as qbe_contract_async. */
int qbe_contract_static(qbe_ctx* ctx, const qbe_plan* plan, double* d_amp_out);
/* Bytes of the per-device workspace of qbe_contract_static (64 MiB). */
size_t qbe_static_scratch_bytes(void);

/* Per-launch timing of a per-step plan: contracts all slices at once
 * (d_workspace of ws_bytes >= stats.ws_bytes_all_slices, else
 * QBE_ERR_MEM_CAP) with a HIP event on the context's stream before the first
 * launch and after each one; ms_out[i] (capacity cap >= the plan's launch
 * count, else QBE_ERR_MEM_CAP) receives launch i's time in milliseconds, in
 * the order of qbe_plan_launch_info, and *n_out the launch count.  Blocks
 * until done.  QBE_ERR_INVALID_ARG for a fused plan. */
int qbe_plan_profile(qbe_ctx* ctx, const qbe_plan* plan, void* d_workspace, size_t ws_bytes, float* ms_out,
                     int32_t cap, int32_t* n_out);

/* ---------------------------------------------------------------- batch - */

/* A set of independent plans (instances, e.g. circuits of uneven size)
 * contracted together.  Plans in the fused form share one persistent
 * launch: its (instance, slice) work items are pulled by a grid of
 * workgroups from a counter, biggest instances first.  Plans in the
 * per-step form (too wide for LDS) follow it level by level (Sec. 2.4: the
 * instances are independent; within a plan, launches of one level share no
 * memory): when the call is captured into a HIP graph, a level's launches
 * are dealt over the context's stream and up to three side streams that the
 * batch creates here (default priority) and owns until qbe_batch_destroy;
 * issued directly, they run on the context's stream.  The plans must outlive the batch.  The
 * work-item table is uploaded here. */
int qbe_batch_create(qbe_ctx* ctx, const qbe_plan* const* plans, int32_t n_plans, qbe_batch** out);
int qbe_batch_destroy(qbe_batch* batch);
/* Workspace bytes qbe_batch_contract_async needs. */
int qbe_batch_workspace(const qbe_batch* batch, size_t* ws_bytes_out);
/* Enqueues the batch: instance i's slices are summed in FP64 into
 * d_amps_out[2 i], d_amps_out[2 i + 1] (device memory).  No allocation, copy
 * or synchronisation inside, so the call may be captured into a HIP graph.
 * Work on the batch's side streams starts after everything enqueued on the
 * context's stream before the call, and the context's stream waits for it
 * (events) before the call's last launch: later work on the context's
 * stream sees every result.  Calls on one batch must not overlap (they share
 * its side streams and events). */
int qbe_batch_contract_async(qbe_ctx* ctx, const qbe_batch* batch, void* d_workspace, size_t ws_bytes,
                             double* d_amps_out);
/* The batch in one synchronous call (Sec. 2.4: the subtasks of all plans
 * are independent): a transient batch of the plans is built, contracted on
 * the context's stream and released; amps_out (host, 2 * n_plans doubles)
 * receives the FP64 amplitudes, plan i at [2 i], [2 i + 1].  With d_workspace
 * NULL the call only stores the workspace bytes it needs in *ws_needed_out
 * (which may otherwise be NULL).  QBE_ERR_MEM_CAP if ws_bytes is smaller than
 * that.  Allocates the batch's device tables each call: for repeated calls
 * keep a qbe_batch instead. */
int qbe_contract_batch(qbe_ctx* ctx, const qbe_plan* const* plans, int32_t n_plans, void* d_workspace,
                       size_t ws_bytes, double* amps_out, size_t* ws_needed_out);

/* ------------------------------------------------------------- permute - */

/* Re-orders the variables of complex64 tensors (Sec. 2.1: each intermediate
 * is a tensor over a clique of variables, so one tensor can be stored in any
 * order of its variables).  d_in holds `batch` tensors of 2^r complex64
 * entries each (interleaved re, im floats), one after another; in each, the
 * linear index's bit p is variable p's value (bit 0 the fastest).  Output
 * bit j takes input bit perm[j]:
 *   out[b][sum_j x_{perm[j]} 2^j] = in[b][sum_p x_p 2^p].
 * perm: host array of r distinct values in [0, r).  d_in, d_out: device
 * memory of batch * 2^r * 8 bytes each, caller-owned, not overlapping.
 * 0 <= r <= 31.  Asynchronous on the context's stream; allocates nothing.
 * QBE_ERR_INVALID_ARG for a NULL pointer, a bad perm, overlapping buffers or
 * a size beyond 2^62 bytes; batch == 0 is a no-op.  The contraction itself
 * never calls this: it reads operands in place through bit extraction. */
int qbe_permute(qbe_ctx* ctx, const void* d_in, void* d_out, int32_t r, const int32_t* perm,
                int64_t batch);

/* ------------------------------------------------------ learned proposal - */

/* A message-passing network that scores variables for slicing and for
 * elimination: 8 input features per variable (qbe_vertex_features), three
 * layers H' = relu(H Ws + mean_{neighbours} H Wn + b) of width 64 shared by
 * two linear heads (QBE_HEAD_*).  Weights are FP16 in the device passes
 * (FP32 master copy for Adam), sums are FP32.  Parameters: a flat float
 * vector of qbe_gnn_num_params() entries, layer by layer (Ws[din][64],
 * Wn[din][64], b[64]), then head 0 (w[64], c), then head 1 (w[64], c).
 * Created with Glorot-uniform weights from a SplitMix64 stream of `seed`.
 * Graphs are passed as symmetric CSR (rowptr[n + 1], col[rowptr[n]]) over n
 * vertices with feats[n * 8]; the call checks ranges and symmetry. */
int qbe_gnn_create(qbe_ctx* ctx, uint64_t seed, qbe_gnn** out);
int qbe_gnn_destroy(qbe_gnn* gnn);
int32_t qbe_gnn_num_params(void);
int qbe_gnn_get_params(const qbe_gnn* gnn, float* params_out);
/* Replaces the parameters and resets the optimizer state. */
int qbe_gnn_set_params(qbe_gnn* gnn, const float* params);
/* Training checkpoint at a caller path: the FP32 master parameters, both
 * Adam moments and the step count, so that training resumes where it
 * stopped.  File layout (native little-endian): the 8 bytes "QBEGNN02",
 * int32 parameter count, int32 step, then three float32 arrays of that count
 * (parameters, first moments, second moments).  QBE_ERR_INVALID_ARG for a
 * file that cannot be opened, written or read in full, or whose magic or
 * parameter count differs; the network is unchanged then. */
int qbe_gnn_save(const qbe_gnn* gnn, const char* path);
int qbe_gnn_load(qbe_gnn* gnn, const char* path);
/* Forward pass on the device through head `head`: scores_out[n] (host). */
int qbe_gnn_score_head(qbe_ctx* ctx, qbe_gnn* gnn, int32_t head, int32_t n, const int32_t* rowptr,
                       const int32_t* col, const float* feats, float* scores_out);
/* qbe_gnn_score_head with the slicing head. */
int qbe_gnn_score(qbe_ctx* ctx, qbe_gnn* gnn, int32_t n, const int32_t* rowptr, const int32_t* col,
                  const float* feats, float* scores_out);
/* One training step on the device through head `head`: forward, loss =
 * mean over the n_cand candidate vertices of (score - target)^2, backward
 * (the other head's gradient is zero), and (if lr > 0) one Adam step (betas
 * 0.9, 0.999, eps 1e-8) of every parameter.  loss_out (1 float) and
 * grads_out (qbe_gnn_num_params() floats, the gradient before the step) are
 * optional. */
int qbe_gnn_train_step_head(qbe_ctx* ctx, qbe_gnn* gnn, int32_t head, int32_t n, const int32_t* rowptr,
                            const int32_t* col, const float* feats, int32_t n_cand, const int32_t* cand,
                            const float* target, float lr, float* loss_out, float* grads_out);
/* qbe_gnn_train_step_head with the slicing head. */
int qbe_gnn_train_step(qbe_ctx* ctx, qbe_gnn* gnn, int32_t n, const int32_t* rowptr, const int32_t* col,
                       const float* feats, int32_t n_cand, const int32_t* cand, const float* target, float lr,
                       float* loss_out, float* grads_out);

/* The model's simple graph without `removed`, as CSR over all n_vars ids
 * (removed vertices have no neighbours): rowptr_out[n_vars + 1], col_out
 * (capacity cap, neighbours ascending); QBE_ERR_MEM_CAP if cap is short
 * (*nnz_out still set). */
int qbe_graph_csr(const qbe_model* model, const int32_t* removed, int32_t n_removed, int32_t* rowptr_out,
                  int32_t* col_out, int64_t cap, int64_t* nnz_out);

/* ----------------------------------------------------------- diagnostics - */

/* Verifies on the host that every index the plan's device programs can form
 * stays inside the buffer it addresses (prepared inputs, arena, LDS).
 * QBE_OK or QBE_ERR_INTERNAL with the first violation in qbe_last_error().
 * qbe_plan_create runs the same check before uploading anything. */
int qbe_plan_check(const qbe_plan* plan);

#ifdef __cplusplus
}
#endif
#endif /* QBE_H */
