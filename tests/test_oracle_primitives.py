"""Pins for the oracle's tensor primitives (Sec. 2.1).

The matricization is checked against its index formula element by element,
the TTM against einsum, and the multi-TTM against the Kronecker identity
(eq. tucker_matrix) built with numpy.kron.
"""

import itertools

import numpy as np
import pytest

from oracle import fold, multi_ttm, ttm, unfold, vec


def _rand(shape, seed=0):
    return np.random.default_rng(seed).standard_normal(shape)


@pytest.mark.parametrize("shape", [(3, 4), (2, 3, 4), (3, 2, 4, 2)])
def test_unfold_index_formula(shape):
    x = _rand(shape)
    d = len(shape)
    for k in range(d):
        m = unfold(x, k)
        assert m.shape == (shape[k], x.size // shape[k])
        for idx in itertools.product(*[range(n) for n in shape]):
            col, stride = 0, 1
            for l in range(d):
                if l == k:
                    continue
                col += idx[l] * stride
                stride *= shape[l]
            assert m[idx[k], col] == x[idx]


@pytest.mark.parametrize("shape", [(3, 4, 5), (2, 3, 4, 5)])
def test_fold_roundtrip_and_vec(shape):
    x = _rand(shape, 1)
    for k in range(len(shape)):
        assert np.array_equal(fold(unfold(x, k), k, shape), x)
    v = vec(x)
    assert v[1] == x[(1,) + (0,) * (len(shape) - 1)]
    assert v[shape[0]] == x[(0, 1) + (0,) * (len(shape) - 2)]


def test_ttm_matches_einsum():
    x = _rand((3, 4, 5), 2)
    a = _rand((6, 4), 3)
    y = ttm(x, a, 1)
    assert y.shape == (3, 6, 5)
    np.testing.assert_allclose(y, np.einsum("ijk,mj->imk", x, a), rtol=1e-13, atol=1e-13)


def test_ttm_commutes_on_distinct_modes():
    x = _rand((3, 4, 5), 4)
    a, b = _rand((2, 3), 5), _rand((6, 5), 6)
    np.testing.assert_allclose(ttm(ttm(x, a, 0), b, 2), ttm(ttm(x, b, 2), a, 0),
                               rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("shape", [(3, 4, 5), (2, 3, 2, 3)])
def test_kronecker_identity(shape):
    rng = np.random.default_rng(7)
    x = rng.standard_normal(shape)
    mats = [rng.standard_normal((n + 1, n)) for n in shape]
    y = multi_ttm(x, mats)
    d = len(shape)
    for k in range(d):
        kron = np.ones((1, 1))
        for l in reversed(range(d)):  # A_d (x) ... (x) A_1 without A_k
            if l != k:
                kron = np.kron(kron, mats[l])
        np.testing.assert_allclose(unfold(y, k), mats[k] @ unfold(x, k) @ kron.T,
                                   rtol=1e-12, atol=1e-12)
