"""Score-function study: which variables to fix (Sec. 3.1-3.2, Sec. 4).

For one synthetic grid circuit and each score of the greedy mu-treewidth
deletion (Alg. 2) -- degree, betweenness centrality, Alg. 3's direct width
reduction and tree-trimming -- the study removes m = 0, 1, ..., m_max
variables and reports, per m, what Sec. 4 plots: the width of the reduced
order (Fig. 7), the FLOPs of one slice (Fig. 10), the total FLOPs 2^m times
that (Fig. 11), the peak memory of one slice (Fig. 12), and the time the
heuristic took to choose the first m variables (Fig. 9).  Every figure comes
from the library's host planner and its exact cost model (no contraction is
run).  With --recompute k the reduced order is recomputed every k removals
(Alg. 2's optional line, Fig. 8's variable) by the project's anytime
tree-decomposition heuristic and Alg. 5.

Usage: python -m paper_2004_10892_amd.study [--rows 7 --cols 7 --depth 24
       --seed 0 --m-max 20 --every 1 --scores degree,betweenness,tw_reduction,
       tree_trimming --recompute 0 --tries 4 --json out.json]
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time
from typing import Dict, List, Sequence

SCORES = ("degree", "betweenness", "tw_reduction", "tree_trimming")


def study(model, scores: Sequence[str] = SCORES, m_max: int = 20, every: int = 1,
          recompute_every: int = 0, tries: int = 4, seed: int = 0) -> Dict[str, List[dict]]:
    """Rows per score for m = 0, every, 2 every, ... m_max: m, width,
    flops_per_slice, log2_total_flops, peak_bytes_per_slice, pick_ms (time to
    choose the m variables) and mu.  recompute_every > 0 runs Alg. 2 with its
    optional order recomputation (Fig. 8's variable) every that many
    removals, with the anytime heuristic's tries and seed."""
    import paper_2004_10892_amd as qbe

    order = qbe.qbe_order_min_fill(model)
    out: Dict[str, List[dict]] = {}
    for score in scores:
        rows = []
        mu_all: List[int] = []
        t_prev = 0.0
        for m in range(0, m_max + 1, every):
            # time the heuristic for exactly m removals (it restarts from
            # scratch, as a user asking for m would)
            t0 = time.perf_counter()
            mu, red, tau = qbe.qbe_slice(model, order, m, score=score, recompute_every=recompute_every,
                                         tries=tries, seed=seed)
            t_prev = (time.perf_counter() - t0) * 1e3
            if recompute_every == 0 and mu_all and mu[:len(mu_all)] != mu_all:
                raise AssertionError("greedy choices are not prefix-consistent")
            mu_all = mu
            c = qbe.qbe_schedule_cost(model, red, mu)
            rows.append({"m": m, "width": tau, "flops_per_slice": c["flops_per_slice"],
                         "log2_total_flops": math.log2(max(c["flops_per_slice"], 1)) + m,
                         "peak_bytes_per_slice": c["peak_bytes_per_slice"], "pick_ms": t_prev,
                         "mu": list(mu)})
        out[score] = rows
    return out


def table(res: Dict[str, List[dict]]) -> str:
    """Markdown table: one row per m, per score width / log2 FLOPs per slice /
    log2 total FLOPs / log2 peak bytes."""
    scores = list(res)
    head = "| m | " + " | ".join(f"{s}: width, lg F/slice, lg F total, lg peak B" for s in scores) + " |"
    sep = "|---|" + "---|" * len(scores)
    lines = [head, sep]
    n = len(next(iter(res.values())))
    for i in range(n):
        cells = []
        for s in scores:
            r = res[s][i]
            cells.append(f"{r['width']}, {math.log2(max(r['flops_per_slice'], 1)):.1f}, "
                         f"{r['log2_total_flops']:.1f}, {math.log2(max(r['peak_bytes_per_slice'], 1)):.1f}")
        lines.append(f"| {res[scores[0]][i]['m']} | " + " | ".join(cells) + " |")
    return "\n".join(lines)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--rows", type=int, default=7)
    ap.add_argument("--cols", type=int, default=7)
    ap.add_argument("--depth", type=int, default=24)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--m-max", type=int, default=20)
    ap.add_argument("--scores", default=",".join(SCORES))
    ap.add_argument("--every", type=int, default=1, help="every k-th m only")
    ap.add_argument("--recompute", type=int, default=0,
                    help="recompute the reduced order every k removals (Alg. 2's optional line)")
    ap.add_argument("--tries", type=int, default=4, help="runs of the anytime order heuristic")
    ap.add_argument("--json", help="also write the rows to this file")
    a = ap.parse_args(argv)
    import paper_2004_10892_amd as qbe
    from circuitgen import circuit_model, random_grid_circuit

    mod = circuit_model(random_grid_circuit(a.rows, a.cols, a.depth, a.seed))
    qm = qbe.Model.from_circuitgen(mod)
    res = study(qm, [s for s in a.scores.split(",") if s], a.m_max, a.every, a.recompute, a.tries, a.seed)
    print(f"{a.rows}x{a.cols} depth {a.depth} seed {a.seed}: {mod.n_vars} variables, "
          f"{len(mod.tensors)} tensors" + (f"; order recomputed every {a.recompute} removals "
                                           f"({a.tries} tries)" if a.recompute else ""))
    print(table(res))
    for s, rows in res.items():
        print(f"{s}: time to choose {a.m_max} variables {rows[-1]['pick_ms']:.1f} ms")
    if a.json:
        with open(a.json, "w") as f:
            json.dump(res, f)
    return 0


if __name__ == "__main__":
    sys.exit(main())
