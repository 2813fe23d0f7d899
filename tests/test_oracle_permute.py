"""Pins of oracle.permute against facts independent of its transpose form:
the entry-by-entry definition on tiny inputs, matrix transposes, and the
composition law of permutations."""
import numpy as np
import pytest

from oracle.permute import permute_bits, permute_bits_loop


def _x(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("r", [0, 1, 2, 3, 5, 8])
def test_transpose_form_equals_entry_loop(r):
    rng = np.random.default_rng(r)
    for _ in range(4):
        perm = [int(p) for p in rng.permutation(r)]
        x = _x(rng, 1 << r)
        assert np.array_equal(permute_bits(x, r, perm), permute_bits_loop(x, r, perm))


def test_two_bit_swap_is_a_2x2_transpose():
    x = np.arange(4.0)
    # index = x0 + 2 x1; the [2, 2] C-order view is M[x1][x0]
    assert np.array_equal(permute_bits(x, 2, [1, 0]).reshape(2, 2), x.reshape(2, 2).T)


@pytest.mark.parametrize("a,b", [(1, 3), (3, 4), (5, 2), (4, 4)])
def test_moving_high_bits_down_is_a_matrix_transpose(a, b):
    # index = lo + 2^a hi with lo < 2^a: the [2^b, 2^a] view is M[hi][lo];
    # output bit j < b takes input bit a + j, output bit b + j input bit j.
    r = a + b
    perm = [a + j for j in range(b)] + list(range(a))
    x = _x(np.random.default_rng(a * 10 + b), 1 << r)
    got = permute_bits(x, r, perm).reshape(1 << a, 1 << b)
    assert np.array_equal(got, x.reshape(1 << b, 1 << a).T)


def test_composition_and_inverse():
    rng = np.random.default_rng(7)
    r = 9
    x = _x(rng, (3, 1 << r))
    for _ in range(5):
        p = [int(v) for v in rng.permutation(r)]
        q = [int(v) for v in rng.permutation(r)]
        # second output bit j = first output bit q[j] = input bit p[q[j]]
        both = permute_bits(permute_bits(x, r, p), r, q)
        assert np.array_equal(both, permute_bits(x, r, [p[q[j]] for j in range(r)]))
        inv = [0] * r
        for j in range(r):
            inv[p[j]] = j
        assert np.array_equal(permute_bits(permute_bits(x, r, p), r, inv), x)


def test_batch_rows_are_independent():
    rng = np.random.default_rng(3)
    r, perm = 6, [3, 0, 5, 1, 4, 2]
    x = _x(rng, (4, 1 << r))
    got = permute_bits(x, r, perm)
    for b in range(4):
        assert np.array_equal(got[b], permute_bits_loop(x[b], r, perm))
