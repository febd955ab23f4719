"""Pins of the oracle's reverse index and top-K selection (paper section 2.2:
the reverse index from coupled configurations to the unique set and the top-K
selection by amplitude; section 4.3 stages 2 and 3).

Each is checked against brute force of a different kind (a dictionary lookup,
a Python sort by an explicit tuple key) and against cases whose answer is fixed
by the definition alone."""
import numpy as np
import pytest

import oracle


def _keys(rng, n, W, hi):
    k = rng.integers(0, hi, size=(n, W), dtype=np.uint64)
    return k


def _tuple(row):
    # unsigned order with the last word most significant
    return tuple(int(x) for x in row[::-1])


@pytest.mark.parametrize("W", [1, 2])
def test_inverse_map_matches_dictionary(W):
    rng = np.random.Generator(np.random.PCG64(11 + W))
    u = np.unique(_keys(rng, 3000, W, 5000), axis=0)
    order = sorted(range(u.shape[0]), key=lambda i: _tuple(u[i]))
    u = u[order]
    where = {_tuple(u[i]): i for i in range(u.shape[0])}
    cand = _keys(rng, 20000, W, 5000)
    got = oracle.inverse_map(W, u, cand)
    want = np.array([where.get(_tuple(c), -1) for c in cand])
    assert np.array_equal(got, want)
    hit = got >= 0
    assert hit.any() and (~hit).any()
    assert np.array_equal(u[got[hit]], cand[hit])


def test_inverse_map_special_cases():
    u = np.array([[2], [4], [8]], dtype=np.uint64)
    assert list(oracle.inverse_map(1, u, u)) == [0, 1, 2]
    assert list(oracle.inverse_map(1, u, np.array([[1], [3], [9], [0]], dtype=np.uint64))) == [-1, -1, -1, -1]
    assert oracle.inverse_map(1, u, np.zeros((0, 1), dtype=np.uint64)).shape == (0,)
    assert list(oracle.inverse_map(1, np.zeros((0, 1), dtype=np.uint64), u)) == [-1, -1, -1]
    # the largest key value, and W=2 keys that differ only in the low word
    top = np.array([[np.uint64(2**64 - 1)]], dtype=np.uint64)
    assert list(oracle.inverse_map(1, np.vstack([u, top]), top)) == [3]
    u2 = np.array([[1, 7], [2, 7], [0, 9]], dtype=np.uint64)
    assert list(oracle.inverse_map(2, u2, np.array([[2, 7], [0, 9], [2, 9]], dtype=np.uint64))) == [1, 2, -1]
    with pytest.raises(ValueError):
        oracle.inverse_map(1, np.array([[4], [2]], dtype=np.uint64), u)
    with pytest.raises(ValueError):
        oracle.inverse_map(1, np.array([[4], [4]], dtype=np.uint64), u)


@pytest.mark.parametrize("W", [1, 2])
def test_topk_matches_sort(W):
    rng = np.random.Generator(np.random.PCG64(21 + W))
    keys = np.unique(_keys(rng, 2500, W, 1 << 40), axis=0)
    rng.shuffle(keys)
    n = keys.shape[0]
    # amplitudes with many exact magnitude ties and both signs
    psi = rng.integers(-40, 41, size=n).astype(np.float64) * 0.125
    rank = sorted(range(n), key=lambda i: (-abs(psi[i]), _tuple(keys[i])))
    for K in (0, 1, 7, 100, n - 1, n, n + 5):
        got = oracle.topk(W, keys, psi, K)
        want = np.zeros(n, dtype=bool)
        want[rank[:K]] = True
        assert np.array_equal(got, want), K
        assert got.sum() == min(K, n)
        if 0 < K < n:
            # every selected magnitude is at least every unselected one
            assert np.abs(psi[got]).min() >= np.abs(psi[~got]).max()


def test_topk_special_cases():
    keys = np.array([[9], [3], [5], [1]], dtype=np.uint64)
    # equal magnitudes: the smallest keys win, whatever the sign
    got = oracle.topk(1, keys, np.array([1.0, -1.0, 1.0, -1.0]), 2)
    assert list(got) == [False, True, False, True]
    # signed zeros are one magnitude
    got = oracle.topk(1, keys, np.array([0.0, -0.0, 0.0, 0.0]), 1)
    assert list(got) == [False, False, False, True]
    got = oracle.topk(1, keys, np.array([1e-300, -2e-300, 5e-324, 0.0]), 2)
    assert list(got) == [True, True, False, False]
    assert oracle.topk(1, np.zeros((0, 1), dtype=np.uint64), np.zeros(0), 3).shape == (0,)
    with pytest.raises(ValueError):
        oracle.topk(1, np.array([[4], [4]], dtype=np.uint64), np.array([1.0, 2.0]), 1)
