"""Learned slicing proposal: data, training and use of the device network.

The greedy mu-treewidth deletion (Alg. 2) removes one variable at a time;
tree-trimming (Sec. 3.2) picks among the variables of the largest bags.  The
learned proposal keeps the same candidate set and replaces the pick by the
network's prediction of the total contraction cost after removing each
candidate; the network is re-run after every removal.

Labels are the method's own exact costs: for a state (mu, reduced order) on
the heuristic's trajectory and each candidate c, the label is
log2(2^(|mu|+1) * FLOPs per slice) of the schedule without c (the project's
cost model, computed by the C++ planner), standardised within the state.

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

from . import (Gnn, Model, qbe_graph_csr, qbe_order_min_fill, qbe_schedule_cost, qbe_slice,
               qbe_vertex_features)

MEM_CAP = 4 << 30  # bytes per slice


@dataclass
class Sample:
    rowptr: np.ndarray
    col: np.ndarray
    feats: np.ndarray
    cand: np.ndarray
    target: np.ndarray


def total_log2_flops(cost: dict) -> float:
    return math.log2(max(cost["flops_per_slice"], 1)) + math.log2(cost["n_slices"])


def candidates(feats: np.ndarray, order: Sequence[int]) -> List[int]:
    """Variables of the maximum bags (the tree-trimming candidate set)."""
    return [v for v in order if feats[v, 3] > 0.5]


def state_sample(qm: Model, order: Sequence[int], mu: Sequence[int], rng, max_cand: int = 24):
    feats = qbe_vertex_features(qm, order, mu)
    cand = candidates(feats, order)
    if len(cand) > max_cand:
        cand = sorted(rng.choice(cand, size=max_cand, replace=False).tolist())
    if len(cand) < 2:
        return None
    y = []
    for c in cand:
        red = [v for v in order if v != c]
        y.append(total_log2_flops(qbe_schedule_cost(qm, red, list(mu) + [c])))
    y = np.asarray(y, dtype=np.float64)
    z = (y - y.mean()) / max(y.std(), 0.05)
    rp, col = qbe_graph_csr(qm, mu)
    return Sample(rp, col, feats, np.asarray(cand, dtype=np.int32), z.astype(np.float32))


def make_dataset(circuits, states=(0, 3, 6, 9), seed=0, max_cand=24, log=None):
    """Samples along the tree-trimming trajectory of each (model) circuit."""
    rng = np.random.default_rng(seed)
    out = []
    n_labels = 0
    for i, qm in enumerate(circuits):
        order = qbe_order_min_fill(qm)
        for k in states:
            mu, red, _ = qbe_slice(qm, order, k)
            s = state_sample(qm, red, mu, rng, max_cand)
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
    rng = np.random.default_rng(seed)
    history = []
    for ep in range(epochs):
        idx = rng.permutation(len(samples))
        losses = []
        for b in range(0, len(idx), batch):
            rp, col, f, c, y = concat([samples[i] for i in idx[b:b + batch]])
            losses.append(net.train_step(rp, col, f, c, y, lr))
        history.append(float(np.mean(losses)))
        if log:
            log(f"[learned] epoch {ep} loss {history[-1]:.4f}")
    return history


def evaluate_loss(net: Gnn, samples: Sequence[Sample]) -> float:
    losses = []
    for s in samples:
        losses.append(net.train_step(s.rowptr, s.col, s.feats, s.cand, s.target, 0.0))
    return float(np.mean(losses))


def learned_slice(qm: Model, order: Sequence[int], net: Gnn, m: int | None = None, mem_cap: int | None = None,
                  max_m: int = 48):
    """Greedy deletion with the network's pick among the largest-bag
    variables; stops at m removals or once the per-slice peak fits mem_cap."""
    mu: List[int] = []
    red = list(order)
    while red:
        if m is not None and len(mu) >= m:
            break
        if mem_cap is not None:
            if qbe_schedule_cost(qm, red, mu)["peak_bytes_per_slice"] <= mem_cap or len(mu) >= max_m:
                break
        feats = qbe_vertex_features(qm, red, mu)
        cand = candidates(feats, red)
        rp, col = qbe_graph_csr(qm, mu)
        s = net.score(rp, col, feats)
        pos = {v: i for i, v in enumerate(red)}
        u = min(cand, key=lambda v: (float(s[v]), pos[v]))
        mu.append(u)
        red.remove(u)
    return mu, red


def heuristic_slice_to_cap(qm: Model, order: Sequence[int], mem_cap: int, max_m: int = 48):
    """Tree-trimming deletion, as few removals as reach the memory cap."""
    for m in range(0, max_m + 1):
        mu, red, _ = qbe_slice(qm, order, m)
        if qbe_schedule_cost(qm, red, mu)["peak_bytes_per_slice"] <= mem_cap:
            return mu, red
    return mu, red


def compare(qm: Model, net: Gnn, mem_cap: int = MEM_CAP):
    """Heuristic vs learned (with the heuristic as fallback) on one circuit:
    both slice until the per-slice peak fits the cap; compared on the exact
    total FLOPs and peak memory of the resulting plans."""
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
