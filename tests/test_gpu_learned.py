"""The learned proposal end to end at a small scale: labels from the exact
cost model for both heads, training on the device, and what the trained
network gains over the method without it (exact total FLOPs; the heuristic
is the fallback), next to the exact one-step lookahead its slicing labels
encode."""
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


def test_learned_proposal_trains_and_gains():
    import torch
    assert torch.cuda.is_available()
    import paper_2004_10892_amd as qbe
    from paper_2004_10892_amd import learned as L
    print("case learned proposal", flush=True)
    ctx = qbe.Context(0)
    train_c = circuits(3000, 60, (5, 6, 7), (14, 24), 11)
    test_c = circuits(4000, 6, (7,), (20, 26), 12)
    train_s, n_train = L.make_dataset(train_c, seed=1, elim_states=6)
    test_s, n_test = L.make_dataset(test_c, seed=2, elim_states=6)
    heads = {h: sum(s.head == h for s in train_s) for h in ("slicing", "elimination")}
    print(f"  {n_train} training labels {heads}, {n_test} held-out labels", flush=True)
    assert n_train > 1000 and n_test > 100 and heads["elimination"] > 10
    net = qbe.Gnn(ctx, seed=5)
    before = {h: L.evaluate_loss(net, [s for s in test_s if s.head == h]) for h in heads}
    hist = L.train(net, train_s, epochs=12, batch=8, lr=2e-3)
    after = {h: L.evaluate_loss(net, [s for s in test_s if s.head == h]) for h in heads}
    print(f"  train loss {hist[0]:.3f} -> {hist[-1]:.3f}; held-out {before} -> {after}", flush=True)
    assert hist[-1] < hist[0]
    assert after["slicing"] < before["slicing"]
    # held-out ranking of the slicing head: predicted best vs average candidate
    regret, spread = [], []
    for s in test_s:
        if s.head != "slicing":
            continue
        sc = net.score(s.rowptr, s.col, s.feats)[s.cand]
        regret.append(s.target[int(np.argmin(sc))] - s.target.min())
        spread.append(s.target.mean() - s.target.min())
    print(f"  held-out regret {np.mean(regret):.3f} vs random pick {np.mean(spread):.3f} (standardised units)",
          flush=True)
    assert np.mean(regret) < np.mean(spread)
    # slicing under a memory cap: learned vs tree-trimming vs the lookahead
    cap = 1 << 20
    gains, look = [], []
    for qm in test_c:
        r = L.compare(qm, net, mem_cap=cap)
        assert (r["learned"]["peak_bytes"] if r["chosen"] == "learned" else r["heuristic"]["peak_bytes"]) <= cap
        mu_x, red_x = L.lookahead_slice(qm, qbe.qbe_order_min_fill(qm), cap)
        lx = L.total_log2_flops(qbe.qbe_schedule_cost(qm, red_x, mu_x))
        gains.append(r["log2_gain"])
        look.append(r["heuristic"]["log2_total_flops"] - lx)
        print(f"  heuristic m={r['heuristic']['m']} log2 FLOPs {r['heuristic']['log2_total_flops']:.2f} | "
              f"learned m={r['learned']['m']} {r['learned']['log2_total_flops']:.2f} -> {r['chosen']} | "
              f"lookahead m={len(mu_x)} {lx:.2f}", flush=True)
    print(f"  mean log2 gain over tree-trimming: learned {np.mean(gains):+.3f}, lookahead {np.mean(look):+.3f}",
          flush=True)
    assert np.mean(gains) > 0.0
    # elimination: learned tie-breaking vs greedy min-fill (min-fill is the
    # fallback, so the kept order never costs more)
    eg = []
    for qm in test_c:
        r = L.compare_order(qm, net)
        eg.append(r["log2_gain_raw"])
        assert r["log2_gain"] >= 0.0
        assert r["learned_log2_flops"] > 0 and r["min_fill_log2_flops"] > 0
    print(f"  elimination head: raw log2 gain over min-fill per circuit {np.round(eg, 2).tolist()}", flush=True)
