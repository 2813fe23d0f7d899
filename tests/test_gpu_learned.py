"""The learned slicing proposal end to end at a small scale: labels from the
exact cost model, training on the device, and what the trained network gains
over tree-trimming alone (exact total FLOPs under a per-slice memory cap, the
heuristic as fallback)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def circuits(first_seed, count, sizes, depths, rng_seed):
    import paper_2004_10892_amd as qbe
    from circuitgen import SplitMix64, circuit_model, random_grid_circuit
    rng = SplitMix64(rng_seed)
    out = []
    for i in range(count):
        r = sizes[rng.next() % len(sizes)]
        c = sizes[rng.next() % len(sizes)]
        d = depths[0] + rng.next() % (depths[1] - depths[0] + 1)
        out.append(qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(r, c, d, first_seed + i))))
    return out


def test_learned_proposal_trains_and_is_compared():
    import torch
    assert torch.cuda.is_available()
    import paper_2004_10892_amd as qbe
    from paper_2004_10892_amd import learned as L
    print("case learned proposal", flush=True)
    ctx = qbe.Context(0)
    train_c = circuits(3000, 40, (5, 6, 7), (14, 24), 11)
    test_c = circuits(4000, 6, (7,), (20, 26), 12)
    train_s, n_train = L.make_dataset(train_c, seed=1)
    test_s, n_test = L.make_dataset(test_c, seed=2)
    assert n_train > 1000 and n_test > 100
    net = qbe.Gnn(ctx, seed=5)
    before = L.evaluate_loss(net, test_s)
    hist = L.train(net, train_s, epochs=12, batch=8, lr=2e-3)
    after = L.evaluate_loss(net, test_s)
    print(f"  train loss {hist[0]:.3f} -> {hist[-1]:.3f}; held-out loss {before:.3f} -> {after:.3f}", flush=True)
    assert hist[-1] < hist[0]
    assert after < before
    # held-out ranking: the predicted best candidate vs the average candidate
    regret, spread = [], []
    for s in test_s:
        sc = net.score(s.rowptr, s.col, s.feats)[s.cand]
        regret.append(s.target[int(np.argmin(sc))] - s.target.min())
        spread.append(s.target.mean() - s.target.min())
    print(f"  held-out regret {np.mean(regret):.3f} vs random pick {np.mean(spread):.3f} (standardised units)",
          flush=True)
    assert np.mean(regret) < np.mean(spread)
    # gains over tree-trimming under a memory cap
    cap = 1 << 20
    gains = []
    for qm in test_c:
        r = L.compare(qm, net, mem_cap=cap)
        assert (r["learned"]["peak_bytes"] if r["chosen"] == "learned" else r["heuristic"]["peak_bytes"]) <= cap
        gains.append(r["log2_gain"])
        print(f"  heuristic m={r['heuristic']['m']} log2 FLOPs {r['heuristic']['log2_total_flops']:.2f} | "
              f"learned m={r['learned']['m']} {r['learned']['log2_total_flops']:.2f} -> {r['chosen']}, "
              f"log2 gain {r['log2_gain']:+.2f}", flush=True)
    print(f"  mean log2 gain {np.mean(gains):+.3f}", flush=True)
