"""The learned loops behind the C ABI, pinned by networks whose outputs are
known functions of the features (weights written by hand, all exact in
FP16):

* a network computing tree-trimming's score (-(256 len + weight) from the
  bag-count and bag-size features) makes qbe_slice_ex's learned Alg. 2 pick
  exactly tree-trimming's variables (Sec. 3.2): same sliced set, reduced
  order and width, with and without the order recomputation;
* a network of zeros leaves greedy min-fill's own tie rule (degree, id):
  qbe_order_learned returns the min-fill order;
* a network preferring the vertices tree-trimming ranks last gives a plan
  that misses a memory cap tree-trimming meets, and the fallback returns
  tree-trimming's result."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

F, H = 8, 64


def layer_sizes():
    return [2 * (F if l == 0 else H) * H + H for l in range(3)]


def crafted_params(n_params, head, w_len, w_wt):
    """Trunk copying features 4 (bags holding u / max) and 5 (their total
    size / max) to hidden units 0 and 1 through three relu layers; head
    `head` = w_len * unit 0 + w_wt * unit 1."""
    p = np.zeros(n_params, dtype=np.float32)
    o = 0
    for l in range(3):
        din = F if l == 0 else H
        ws = p[o:o + din * H].reshape(din, H)
        if l == 0:
            ws[4, 0] = 1.0
            ws[5, 1] = 1.0
        else:
            ws[0, 0] = 1.0
            ws[1, 1] = 1.0
        o += 2 * din * H + H
    o += head * (H + 1)
    p[o + 0] = w_len
    p[o + 1] = w_wt
    return p


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    import paper_2004_10892_amd as qbe
    return qbe, qbe.Context(0)


def models(qbe):
    from circuitgen import circuit_model, random_grid_circuit
    for (r, c, d, seed) in [(4, 4, 10, 0), (5, 5, 12, 1), (5, 6, 14, 2), (6, 6, 16, 3)]:
        yield f"{r}x{c}_d{d}", qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(r, c, d, seed)))


def test_network_with_tree_trimming_score_reproduces_tree_trimming(env):
    qbe, ctx = env
    net = qbe.Gnn(ctx, seed=0)
    net.set_params(crafted_params(net.n_params, 0, -256.0, -1.0))
    for name, qm in models(qbe):
        order = qbe.qbe_order_min_fill(qm)
        for m in (1, 4, 7):
            for rec in (0, 2):
                print(f"case learned slicing pin {name} m={m} recompute={rec}", flush=True)
                want = qbe.qbe_slice(qm, order, m, recompute_every=rec, tries=4, seed=9)
                got = qbe.qbe_slice(qm, order, m, score="learned", net=net, recompute_every=rec, tries=4, seed=9)
                assert got == want, (name, m, rec)


def test_zero_network_gives_the_min_fill_order(env):
    qbe, ctx = env
    net = qbe.Gnn(ctx, seed=0)
    net.set_params(np.zeros(net.n_params, dtype=np.float32))
    for name, qm in models(qbe):
        print(f"case learned order pin {name}", flush=True)
        mf = qbe.qbe_order_min_fill(qm)
        for refresh in (1, 7):
            order, width, fell_back, (fl, fm) = qbe.qbe_order_learned(qm, net, refresh)
            assert order == mf and fl == fm and not fell_back
            assert width == qbe.qbe_width(qm, mf)


def test_memory_cap_fallback_to_tree_trimming(env):
    qbe, ctx = env
    net = qbe.Gnn(ctx, seed=0)
    # the opposite of tree-trimming's ranking: fewest, smallest bags first
    net.set_params(crafted_params(net.n_params, 0, 256.0, 1.0))
    hits = 0
    for name, qm in models(qbe):
        order = qbe.qbe_order_min_fill(qm)
        m = 4
        mu_t, pi_t, tau_t = qbe.qbe_slice(qm, order, m)
        mu_a, pi_a, tau_a = qbe.qbe_slice(qm, order, m, score="learned", net=net)
        peak_t = qbe.qbe_schedule_cost(qm, pi_t, mu_t)["peak_bytes_per_slice"]
        peak_a = qbe.qbe_schedule_cost(qm, pi_a, mu_a)["peak_bytes_per_slice"]
        if peak_a <= peak_t:
            continue
        hits += 1
        print(f"case learned fallback {name}: peaks {peak_a} (network) vs {peak_t} (tree-trimming)", flush=True)
        mu, pi, tau, fb = qbe.qbe_slice(qm, order, m, score="learned", net=net, mem_cap=peak_t,
                                         with_fallback=True)
        assert fb and (mu, pi, tau) == (mu_t, pi_t, tau_t)
        # a cap the network's plan meets: no fallback
        mu, pi, tau, fb = qbe.qbe_slice(qm, order, m, score="learned", net=net, mem_cap=peak_a,
                                         with_fallback=True)
        assert not fb and (mu, pi, tau) == (mu_a, pi_a, tau_a)
    assert hits >= 1
