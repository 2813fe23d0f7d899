"""Pin of the float64 network reference: its hand-written gradient against
central finite differences of its own loss (float64, step 1e-6)."""
import numpy as np
import pytest

from oracle import gnn


def random_graph(n, p, rng):
    A = (rng.random((n, n)) < p).astype(np.float64)
    A = np.triu(A, 1)
    return A + A.T


@pytest.mark.parametrize("seed,head", [(0, 0), (1, 0), (2, 1), (3, 1)])
def test_gradient_matches_finite_differences(seed, head):
    rng = np.random.default_rng(seed)
    n = 12
    A = random_graph(n, 0.3, rng)
    A[0, :] = A[:, 0] = 0.0  # an isolated vertex
    X = rng.standard_normal((n, gnn.F))
    p = rng.standard_normal(gnn.n_params()) * 0.2
    cand = rng.choice(n, size=6, replace=False)
    y = rng.standard_normal(6)
    loss, g = gnn.loss_and_grad(p, A, X, cand, y, head)
    idx = rng.choice(len(p), size=80, replace=False)
    # both heads' last weights and biases (one of them has gradient 0)
    idx = np.concatenate([idx, [len(p) - 1, len(p) - 2, len(p) - 66, len(p) - 67, 0, 8 * 64]])
    eps = 1e-6
    for i in idx:
        q = p.copy()
        q[i] += eps
        lp, _ = gnn.loss_and_grad(q, A, X, cand, y, head)
        q[i] -= 2 * eps
        lm, _ = gnn.loss_and_grad(q, A, X, cand, y, head)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_mean_aggregation_by_hand():
    A = np.array([[0, 1, 1], [1, 0, 0], [1, 0, 0]], dtype=float)
    X = np.array([[1.0], [2.0], [4.0]])
    M = gnn.mean_agg(A, X)
    assert np.allclose(M[:, 0], [3.0, 1.0, 1.0])


def test_heads_share_the_trunk():
    """The two heads differ only in their last linear map: with equal head
    parameters they give equal scores, and each loss leaves the other head's
    parameters without gradient."""
    rng = np.random.default_rng(7)
    n = 10
    A = random_graph(n, 0.3, rng)
    X = rng.standard_normal((n, gnn.F))
    p = rng.standard_normal(gnn.n_params()) * 0.2
    h0 = len(p) - 2 * (gnn.H + 1)
    p[h0 + gnn.H + 1:] = p[h0:h0 + gnn.H + 1]
    s0, _ = gnn.forward(p, A, X, 0)
    s1, _ = gnn.forward(p, A, X, 1)
    assert np.array_equal(s0, s1)
    _, g0 = gnn.loss_and_grad(p, A, X, [1, 2], [0.5, -0.5], 0)
    _, g1 = gnn.loss_and_grad(p, A, X, [1, 2], [0.5, -0.5], 1)
    assert not np.any(g0[h0 + gnn.H + 1:]) and not np.any(g1[h0:h0 + gnn.H + 1])
    assert np.array_equal(g0[:h0], g1[:h0])
