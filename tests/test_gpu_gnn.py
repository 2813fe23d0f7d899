"""The device network (FP16 weights, FP32 sums) against the float64 oracle:
forward scores and gradients, plus a training sanity check.

Tolerances: with the same FP16-rounded weights on both sides, the device
differs from float64 only by FP32 rounding of sums of at most 2 * 64 + 1
terms per entry per layer (relative ~1e-6 each); 1e-4 of the largest
magnitude covers three layers and the backward pass with margin.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    import paper_2004_10892_amd as qbe
    return qbe, qbe.Context(0)


def csr(A):
    rp = [0]
    col = []
    for v in range(A.shape[0]):
        nb = np.nonzero(A[v])[0]
        col += nb.tolist()
        rp.append(len(col))
    return np.array(rp, dtype=np.int32), np.array(col, dtype=np.int32)


def case(seed, n=40, p=0.15):
    rng = np.random.default_rng(seed)
    A = (rng.random((n, n)) < p).astype(np.float64)
    A = np.triu(A, 1)
    A = A + A.T
    X = rng.standard_normal((n, 8)).astype(np.float32)
    cand = rng.choice(n, size=10, replace=False).astype(np.int32)
    y = rng.standard_normal(10).astype(np.float32)
    return A, X, cand, y


@pytest.mark.parametrize("seed,head", [(0, "slicing"), (1, "slicing"), (2, "elimination"), (3, "elimination")])
def test_forward_and_gradients_match_oracle(env, seed, head):
    qbe, ctx = env
    from oracle import gnn as G
    h = qbe.HEAD[head]
    print(f"case gnn parity seed={seed} head={head}", flush=True)
    net = qbe.Gnn(ctx, seed=seed)
    p = net.params()
    p16 = p.astype(np.float16).astype(np.float64)  # the weights the device uses
    A, X, cand, y = case(seed)
    rp, col = csr(A)
    s_dev = net.score(rp, col, X, head=head)
    s_ref, _ = G.forward(p16, A, X.astype(np.float64), h)
    assert np.max(np.abs(s_dev - s_ref)) <= 1e-4 * max(1.0, np.max(np.abs(s_ref)))
    loss_dev, g_dev = net.train_step(rp, col, X, cand, y, lr=0.0, want_grads=True, head=head)
    loss_ref, g_ref = G.loss_and_grad(p16, A, X.astype(np.float64), cand, y.astype(np.float64), h)
    assert abs(loss_dev - loss_ref) <= 1e-4 * max(1.0, loss_ref)
    assert np.max(np.abs(g_dev - g_ref)) <= 1e-4 * max(1.0, np.max(np.abs(g_ref)))
    assert np.array_equal(net.params(), p)  # lr = 0 leaves the weights alone


def test_training_reduces_loss(env):
    qbe, ctx = env
    print("case gnn training", flush=True)
    net = qbe.Gnn(ctx, seed=3)
    A, X, cand, _ = case(5, n=60)
    rp, col = csr(A)
    y = (X[cand, 0] * 0.5 - X[cand, 3]).astype(np.float32)  # a learnable target
    first = net.train_step(rp, col, X, cand, y, lr=0.0)
    for _ in range(300):
        last = net.train_step(rp, col, X, cand, y, lr=3e-3)
    assert last < 0.1 * first, (first, last)


def test_rejects_asymmetric_graphs(env):
    qbe, ctx = env
    net = qbe.Gnn(ctx, seed=0)
    rp = np.array([0, 1, 1], dtype=np.int32)
    col = np.array([1], dtype=np.int32)
    with pytest.raises(qbe.QbeError, match="INVALID_ARG"):
        net.score(rp, col, np.zeros((2, 8), np.float32))


def test_checkpoint_resumes_training_exactly(env, tmp_path):
    """qbe_gnn_save / qbe_gnn_load: a network restored from a checkpoint
    taken mid-training continues bit for bit like the original (parameters,
    Adam moments and step count all restored)."""
    qbe, ctx = env
    print("case gnn checkpoint", flush=True)
    A, X, cand, y = case(7, n=50)
    rp, col = csr(A)
    a = qbe.Gnn(ctx, seed=4)
    for _ in range(5):
        a.train_step(rp, col, X, cand, y, lr=1e-3)
    path = str(tmp_path / "net.ckpt")
    at_ckpt = a.params()
    a.save(path)
    b = qbe.Gnn(ctx, seed=99)
    b.load(path)
    assert np.array_equal(a.params(), b.params())
    for _ in range(5):
        la = a.train_step(rp, col, X, cand, y, lr=1e-3)
        lb = b.train_step(rp, col, X, cand, y, lr=1e-3)
        assert la == lb
    assert np.array_equal(a.params(), b.params())
    # the same parameters with a fresh optimizer state (set_params) take
    # other steps: the checkpoint's moments and step count matter
    c = qbe.Gnn(ctx, seed=99)
    c.set_params(at_ckpt)
    for _ in range(5):
        c.train_step(rp, col, X, cand, y, lr=1e-3)
    assert not np.array_equal(c.params(), a.params())


def test_checkpoint_rejects_bad_files(env, tmp_path):
    qbe, ctx = env
    net = qbe.Gnn(ctx, seed=1)
    before = net.params()
    with pytest.raises(qbe.QbeError, match="INVALID_ARG"):
        net.load(str(tmp_path / "missing.ckpt"))
    bad = tmp_path / "bad.ckpt"
    bad.write_bytes(b"NOTACKPT" + b"\0" * 64)
    with pytest.raises(qbe.QbeError, match="INVALID_ARG"):
        net.load(str(bad))
    good = tmp_path / "good.ckpt"
    net.save(str(good))
    data = good.read_bytes()
    short = tmp_path / "short.ckpt"
    short.write_bytes(data[: len(data) // 2])
    with pytest.raises(qbe.QbeError, match="INVALID_ARG"):
        net.load(str(short))
    assert np.array_equal(net.params(), before)
    with pytest.raises(qbe.QbeError, match="INVALID_ARG"):
        net.save(str(tmp_path / "no_such_dir" / "x.ckpt"))
