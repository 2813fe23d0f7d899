"""qbe_permute (bit permutation of complex64 tensors) against the oracle's
definition, bit-exact: pure data movement, so every output entry must be
the very input entry the definition names.  Sizes span single-tile tensors,
several tiles with ragged tile-bit sets, batches, the degenerate r = 0 and
r = 1, and a 2^26-entry tensor (512 MiB, beyond the last-level cache)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    import paper_2004_10892_amd as qbe
    return qbe, qbe.Context(0), torch


def _run(env, x, r, perm):
    qbe, ctx, torch = env
    batch = x.shape[0]
    d_in = torch.from_numpy(x).to("cuda:0")
    d_out = torch.full_like(d_in, complex(float("nan"), float("nan")))
    print(f"permute r={r} batch={batch} perm={list(perm)[:8]}", flush=True)
    qbe.qbe_permute(ctx, d_in, d_out, r, perm, batch)
    torch.cuda.synchronize()
    return d_out.cpu().numpy()


def _perms(r, rng):
    yield list(range(r))
    yield list(range(r))[::-1]
    if r >= 2:
        yield [(j + 1) % r for j in range(r)]
        yield [(j + r // 2) % r for j in range(r)]
    for _ in range(3):
        yield [int(p) for p in rng.permutation(r)]


@pytest.mark.parametrize("r,batch", [(0, 1), (0, 7), (1, 3), (2, 1), (5, 2), (6, 1), (7, 3), (9, 2),
                                     (11, 1), (12, 2), (13, 1), (16, 3), (20, 1)])
def test_permute_bit_exact(env, r, batch):
    from oracle.permute import permute_bits
    rng = np.random.default_rng(1000 * r + batch)
    x = (rng.standard_normal((batch, 1 << r)) + 1j * rng.standard_normal((batch, 1 << r))).astype(np.complex64)
    for perm in _perms(r, rng):
        got = _run(env, x, r, perm)
        assert np.array_equal(got, permute_bits(x, r, perm)), perm


def test_permute_large_tensor(env):
    from oracle.permute import permute_bits
    r = 26
    rng = np.random.default_rng(26)
    x = (rng.standard_normal((1, 1 << r)) + 1j * rng.standard_normal((1, 1 << r))).astype(np.complex64)
    perm = [int(p) for p in rng.permutation(r)]
    assert np.array_equal(_run(env, x, r, perm), permute_bits(x, r, perm))


def test_permute_rejects_bad_arguments(env):
    qbe, ctx, torch = env
    a = torch.zeros(64, dtype=torch.complex64, device="cuda:0")
    b = torch.zeros(64, dtype=torch.complex64, device="cuda:0")
    for perm in ([0, 1, 2, 3, 4, 4], [0, 1, 2, 3, 4, 6], [0, 1, 2, 3, 4, -1]):
        with pytest.raises(qbe.QbeError):
            qbe.qbe_permute(ctx, a, b, 6, perm, 1)
    with pytest.raises(qbe.QbeError):  # overlapping buffers
        qbe.qbe_permute(ctx, a, a[1:], 5, list(range(5)), 1)
    with pytest.raises(ValueError):  # output too small for the batch
        qbe.qbe_permute(ctx, a, b, 6, list(range(6)), 2)
    qbe.qbe_permute(ctx, a, b, 6, list(range(6)), 0)  # no-op
    torch.cuda.synchronize()
