"""Learned proposal: data, training and use of the device network.

The network (qbe_gnn_*) has two heads on a shared message-passing trunk:

* slicing (Alg. 2's score f): greedy mu-treewidth deletion keeps
  tree-trimming's candidate set (the variables of the largest bags) and
  removes the one the head predicts cheapest; the network is re-run after
  every removal (qbe_slice_ex with QBE_SCORE_LEARNED);
* elimination (Sec. 2.2's order problem): greedy min-fill whose ties in fill
  go to the vertex the head predicts cheapest, re-scored on the elimination
  graph every few eliminations (qbe_order_learned).

In both the paper's heuristic remains the fallback (tree-trimming when the
learned sliced set misses a memory cap; min-fill when the learned order
costs more FLOPs), and choices are judged by exact FLOP and peak-memory
counts.  Labels are the method's own exact costs (qbe_learned_sample: log2
total FLOPs of each candidate's continuation, standardised per state).

All planning arithmetic runs in the C++ planner behind the C ABI and all
network arithmetic in the library's HIP kernels; this module only arranges
the calls.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass
from typing import List, Sequence

import numpy as np

from . import (Gnn, Model, qbe_learned_sample, qbe_order_learned, qbe_order_min_fill, qbe_schedule_cost, qbe_slice,
               qbe_vertex_features)

MEM_CAP = 4 << 30  # bytes per slice


@dataclass
class Sample:
    rowptr: np.ndarray
    col: np.ndarray
    feats: np.ndarray
    cand: np.ndarray
    target: np.ndarray
    head: str = "slicing"


def total_log2_flops(cost: dict) -> float:
    return math.log2(max(cost["flops_per_slice"], 1)) + math.log2(cost["n_slices"])


def _sample(qm, head, order, mu=(), k_elim=0, max_cand=24, seed=0):
    s = qbe_learned_sample(qm, head, order, mu, k_elim=k_elim, max_cand=max_cand, seed=seed)
    if s is None or float(np.ptp(s[4])) == 0.0:
        return None  # fewer than two candidates, or all equally good: no signal
    return Sample(*s, head=head)


def make_dataset(circuits, states=(0, 3, 6, 9), seed=0, max_cand=24, elim_states=0, log=None):
    """Samples of each (model) circuit: slicing states along the
    tree-trimming trajectory (|mu| in `states`); with elim_states > 0, that
    many elimination states drawn from the later two thirds of its min-fill
    order (where ties in fill fall between vertices of nonzero fill)."""
    rng = np.random.default_rng(seed)
    out = []
    n_labels = 0
    for i, qm in enumerate(circuits):
        order = qbe_order_min_fill(qm)
        for k in states:
            mu, red, _ = qbe_slice(qm, order, k)
            s = _sample(qm, "slicing", red, mu, max_cand=max_cand, seed=int(rng.integers(1 << 62)))
            if s is not None:
                out.append(s)
                n_labels += len(s.cand)
        n = len(order)
        for _ in range(elim_states):
            k = int(rng.integers(n // 3, n - 1))
            s = _sample(qm, "elimination", order, k_elim=k, max_cand=max_cand, seed=int(rng.integers(1 << 62)))
            if s is not None:
                out.append(s)
                n_labels += len(s.cand)
        if log and (i + 1) % 25 == 0:
            log(f"[learned] labels: {i + 1} circuits, {n_labels} labels")
    return out, n_labels


def concat(samples: Sequence[Sample]):
    """Block-diagonal union of several graphs."""
    rps, cols, feats, cands, ys = [], [], [], [], []
    off_v = 0
    off_e = 0
    for s in samples:
        n = len(s.rowptr) - 1
        rps.append(s.rowptr[:-1] + off_e)
        cols.append(s.col + off_v)
        feats.append(s.feats)
        cands.append(s.cand + off_v)
        ys.append(s.target)
        off_v += n
        off_e += int(s.rowptr[-1])
    rp = np.concatenate(rps + [np.array([off_e], dtype=np.int32)]).astype(np.int32)
    return rp, np.concatenate(cols).astype(np.int32), np.concatenate(feats), np.concatenate(cands).astype(np.int32), \
        np.concatenate(ys)


def train(net: Gnn, samples: Sequence[Sample], epochs: int = 20, batch: int = 8, lr: float = 1e-3, seed: int = 0,
          log=None):
    """Adam on mini-batches of one head each (the heads share the trunk)."""
    rng = np.random.default_rng(seed)
    history = []
    by_head = {}
    for i, s in enumerate(samples):
        by_head.setdefault(s.head, []).append(i)
    for ep in range(epochs):
        batches = []
        for head, idx in by_head.items():
            p = rng.permutation(idx)
            batches += [(head, p[b:b + batch]) for b in range(0, len(p), batch)]
        losses = []
        for j in rng.permutation(len(batches)):
            head, sel = batches[j]
            rp, col, f, c, y = concat([samples[i] for i in sel])
            losses.append(net.train_step(rp, col, f, c, y, lr, head=head))
        history.append(float(np.mean(losses)))
        if log:
            log(f"[learned] epoch {ep} loss {history[-1]:.4f}")
    return history


def evaluate_loss(net: Gnn, samples: Sequence[Sample]) -> float:
    losses = []
    for s in samples:
        losses.append(net.train_step(s.rowptr, s.col, s.feats, s.cand, s.target, 0.0, head=s.head))
    return float(np.mean(losses))


def learned_slice(qm: Model, order: Sequence[int], net: Gnn, m: int | None = None, mem_cap: int | None = None,
                  recompute_every: int = 0, tries: int = 8, seed: int = 0):
    """Alg. 2 with the network's slicing head (qbe_slice_ex): m removals, or
    as few as bring the per-slice peak under mem_cap.  Returns (mu,
    reduced_order)."""
    mu, red, _ = qbe_slice(qm, order, m if m is not None else -1, score="learned", net=net,
                           mem_cap=mem_cap or 0, recompute_every=recompute_every, tries=tries, seed=seed)
    return mu, red


def heuristic_slice_to_cap(qm: Model, order: Sequence[int], mem_cap: int):
    """Tree-trimming deletion, as few removals as bring the per-slice peak
    under the cap."""
    mu, red, _ = qbe_slice(qm, order, -1, mem_cap=mem_cap)
    return mu, red


def compare(qm: Model, net: Gnn, mem_cap: int = MEM_CAP):
    """Heuristic vs learned slicing (with the heuristic as fallback) on one
    circuit: both slice until the per-slice peak fits the cap; compared on
    the exact total FLOPs and peak memory of the resulting plans."""
    order = qbe_order_min_fill(qm)
    t0 = time.perf_counter()
    mu_h, red_h = heuristic_slice_to_cap(qm, order, mem_cap)
    t1 = time.perf_counter()
    mu_l, red_l = learned_slice(qm, order, net, mem_cap=mem_cap)
    t2 = time.perf_counter()
    ch = qbe_schedule_cost(qm, red_h, mu_h)
    cl = qbe_schedule_cost(qm, red_l, mu_l)
    learned_ok = cl["peak_bytes_per_slice"] <= mem_cap
    use_learned = learned_ok  # the heuristic is the fallback when the plan misses the cap
    cf = cl if use_learned else ch
    return {
        "heuristic": {"m": len(mu_h), "log2_total_flops": total_log2_flops(ch), "width": ch["width"],
                      "peak_bytes": ch["peak_bytes_per_slice"], "plan_ms": (t1 - t0) * 1e3},
        "learned": {"m": len(mu_l), "log2_total_flops": total_log2_flops(cl), "width": cl["width"],
                    "peak_bytes": cl["peak_bytes_per_slice"], "plan_ms": (t2 - t1) * 1e3, "fits_cap": learned_ok},
        "chosen": "learned" if use_learned else "heuristic",
        "log2_gain": total_log2_flops(ch) - total_log2_flops(cf),
        # both plans' exact costs are known before contracting: keeping the
        # cheaper one can only gain
        "log2_gain_best_of_both": total_log2_flops(ch) - min(total_log2_flops(ch), total_log2_flops(cf)),
    }


def compare_order(qm: Model, net: Gnn, refresh: int = 16):
    """Learned elimination order vs greedy min-fill (no slicing): exact
    total FLOPs of both orders; the result keeps min-fill when it is cheaper."""
    t0 = time.perf_counter()
    order, width, fell_back, (fl, fm) = qbe_order_learned(qm, net, refresh)
    t1 = time.perf_counter()
    return {"learned_log2_flops": math.log2(max(fl, 1)), "min_fill_log2_flops": math.log2(max(fm, 1)),
            "log2_gain_raw": math.log2(max(fm, 1)) - math.log2(max(fl, 1)),
            "log2_gain": max(0.0, math.log2(max(fm, 1)) - math.log2(max(fl, 1))),
            "chosen": "min_fill" if fell_back else "learned", "width": width, "order_ms": (t1 - t0) * 1e3,
            "order": order}


def lookahead_slice(qm: Model, order: Sequence[int], mem_cap: int, max_m: int = 64):
    """Alg. 2 with the exact one-step lookahead score the slicing labels
    encode: among tree-trimming's candidates, remove the one whose removal
    gives the fewest total FLOPs (cost model), until the per-slice peak fits
    mem_cap.  A reference for the network (host only, slow)."""
    mu: List[int] = []
    red = list(order)
    while red and len(mu) < max_m:
        if qbe_schedule_cost(qm, red, mu)["peak_bytes_per_slice"] <= mem_cap:
            break
        s = qbe_learned_sample(qm, "slicing", red, mu, max_cand=max(2, len(red)), seed=0)
        if s is None:  # one candidate, or all equally good: the first in the order
            feats = qbe_vertex_features(qm, red, mu)
            u = next(v for v in red if feats[v, 3] > 0.5)
        else:
            cand, target = s[3], s[4]
            pos = {v: i for i, v in enumerate(red)}
            u = int(min(range(len(cand)), key=lambda i: (float(target[i]), pos[int(cand[i])])))
            u = int(cand[u])
        mu.append(u)
        red.remove(u)
    return mu, red
