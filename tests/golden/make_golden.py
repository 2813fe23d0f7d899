"""Writes tests/golden/amplitudes.json from the CPU oracle only.

Run from the repository root:  python tests/golden/make_golden.py [--only batch]
(takes a few minutes: a 2^25 statevector and 1024 slices of the 7x7 circuit).
It also writes tests/golden/batch512.json: the oracle's amplitude of every
instance of the 512-instance batch workload (circuitgen.batch_instances),
planned by the oracle's own min-fill order and Alg. 2 with the instance's m
(about a minute; --only batch writes just that file).

Contents per workload: the circuit seed and bitstring, the statevector
amplitude where the qubit count allows (<= 25), the oracle's per-slice values
and their sum.  Seeds are the smallest non-negative ones whose amplitude is
not degenerate (2^n |a|^2 >= 1e-2; shallow circuits of this family have
exact zeros when a qubit only ever receives diagonal gates).
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from circuitgen import WORKLOADS, batch_instances, circuit_model, random_grid_circuit  # noqa: E402
from oracle import contract as C  # noqa: E402
from oracle import planner as P  # noqa: E402
from oracle import statevector as SV  # noqa: E402

SEEDS = {"grid4x4_d10_m0": 0, "grid5x5_d16_m6": 1, "grid7x7_d24_m10": 0}


def plan(circ, m):
    mod = circuit_model(circ)
    tv = [v for v, _ in mod.tensors]
    adj = P.simple_graph(mod.n_vars, tv)
    order = P.min_fill_order(adj)
    mu, _, pi, tau = P.greedy_treewidth_deletion(adj, order, m)
    return mod, C.bucket_schedule(mod.n_vars, tv, pi, mu), tau


def batch_golden():
    rows_out = []
    t0 = time.time()
    for (rows, cols, depth, m, seed) in batch_instances(512):
        circ = random_grid_circuit(rows, cols, depth, seed)
        mod, sched, tau = plan(circ, m)
        total, _ = C.contract(mod.tensors, sched)
        rows_out.append({"rows": rows, "cols": cols, "depth": depth, "m": m, "seed": seed, "tau": tau,
                         "bitstring": circ.bitstring, "oracle": [total.real, total.imag]})
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch512.json"), "w") as f:
        f.write('{"instances": [\n' + ",\n".join(json.dumps(r) for r in rows_out) + "\n]}\n")
    print("batch512", len(rows_out), "%.1fs" % (time.time() - t0), flush=True)


def main():
    if "--only" in sys.argv and sys.argv[sys.argv.index("--only") + 1] == "batch":
        batch_golden()
        return
    batch_golden()
    out = {}
    for name, (rows, cols, depth, m) in WORKLOADS.items():
        t0 = time.time()
        seed = SEEDS[name]
        circ = random_grid_circuit(rows, cols, depth, seed)
        mod, sched, tau = plan(circ, m)
        total, vals = C.contract(mod.tensors, sched)
        rec = {"seed": seed, "bitstring": circ.bitstring, "m": m, "tau": tau,
               "oracle": [total.real, total.imag],
               "slices": [[v.real, v.imag] for v in vals]}
        if rows * cols <= 25:
            a = SV.amplitude(rows * cols, circ.gates, circ.bitstring)
            rec["statevector"] = [a.real, a.imag]
        out[name] = rec
        print(name, total, "%.1fs" % (time.time() - t0), flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "amplitudes.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
