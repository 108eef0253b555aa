"""Pins of the oracle's TT algebra against dense brute force and invariants.

Sec. 2.1 (algebra and rank laws) and Sec. 2.2 (orthogonality conditions,
rounding bound eq. (rounding_condition_tt)) of arXiv 2512.07811.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import tt as T
from paper_2512_07811_amd import inputs as I

pytestmark = pytest.mark.filterwarnings("ignore")


def test_full_matches_explicit_sum():
    # three cores, explicit loops over every index and bond (eq. tt_format)
    x = I.random_tt([2, 3, 2], [1, 2, 3, 1], seed=1)
    ref = np.zeros((2, 3, 2), dtype=complex)
    for i, j, k in itertools.product(range(2), range(3), range(2)):
        s = 0
        for a, b in itertools.product(range(2), range(3)):
            s += x[0][0, i, a] * x[1][a, j, b] * x[2][b, k, 0]
        ref[i, j, k] = s
    assert np.allclose(T.full(x), ref, rtol=0, atol=1e-14)


def test_full_operator_matches_explicit_sum():
    A = I.random_mpo([2, 3], [3, 2], [1, 2, 1], seed=2)
    M = T.full_operator(A)
    for (i1, i2, j1, j2) in itertools.product(range(2), range(3), range(3), range(2)):
        s = sum(A[0][0, i1, j1, a] * A[1][a, i2, j2, 0] for a in range(2))
        assert abs(M[i1 * 3 + i2, j1 * 2 + j2] - s) < 1e-14


def test_tt_svd_exact_and_separable():
    g = I.rng(3)
    a = g.standard_normal((2, 3, 2, 2, 3))
    c = T.tt_svd(a, list(a.shape), 0.0)
    assert np.max(np.abs(T.full(c) - a)) < 1e-13 * np.max(np.abs(a))
    # a rank-1 (separable) tensor has all TT ranks 1
    v = [g.standard_normal(p) for p in (2, 3, 4, 2)]
    sep = np.einsum("i,j,k,l->ijkl", *v)
    c = T.tt_svd(sep, [2, 3, 4, 2], 1e-12)
    assert T.ranks(c) == [1, 1, 1, 1, 1]


def _dense(x):
    return T.full(x)


@pytest.mark.parametrize("seed", [4, 5])
def test_algebra_values_and_rank_laws(seed):
    m = [3, 2, 2, 2, 2]
    x = I.random_tt(m, [1, 2, 3, 4, 2, 1], seed)
    y = I.random_tt(m, [1, 3, 2, 2, 3, 1], seed + 100)
    A = I.random_mpo(m, m, [1, 2, 2, 3, 2, 1], seed + 200)
    X, Y = _dense(x), _dense(y)
    s = T.add(x, y)
    assert np.allclose(_dense(s), X + Y, atol=1e-13)
    assert T.ranks(s)[1:-1] == [a + b for a, b in zip(T.ranks(x)[1:-1], T.ranks(y)[1:-1])]
    d = T.sub(x, y)
    assert np.allclose(_dense(d), X - Y, atol=1e-13)
    h = T.hadamard(x, y)
    assert np.allclose(_dense(h), X * Y, atol=1e-13)
    assert T.ranks(h) == [a * b for a, b in zip(T.ranks(x), T.ranks(y))]
    z = T.mpo_apply(A, x)
    ref = (T.full_operator(A) @ X.reshape(-1)).reshape(X.shape)
    assert np.allclose(_dense(z), ref, atol=1e-12)
    assert T.ranks(z) == [a.shape[0] * b for a, b in zip(A, T.ranks(x)[:-1])] + [1]
    c = 1.7 - 0.3j
    sc = T.scale(x, c)
    assert T.ranks(sc) == T.ranks(x)
    assert np.allclose(_dense(sc), c * X, atol=1e-13)
    assert abs(T.dot(x, y) - np.vdot(X, Y)) < 1e-12 * np.linalg.norm(X) * np.linalg.norm(Y)
    # lifting a TT to a diagonal TTO gives the Hadamard product (eq. tt_to_tto)
    lifted = T.mpo_apply(T.diag_lift(y), x)
    assert np.allclose(_dense(lifted), X * Y, atol=1e-13)
    # the adjoint operator is the conjugate transpose
    assert np.allclose(T.full_operator(T.conj_transpose_mpo(A)),
                       np.conj(T.full_operator(A).T), atol=1e-13)


def test_orthogonalization_invariants():
    x = I.random_tt([3, 2, 2, 2, 2, 2], [1, 3, 5, 4, 4, 2, 1], seed=6)
    q, nrm = T.orthogonalize_left(x)
    for c in q[:-1]:
        G = T.left_gram(c)
        assert np.allclose(G, np.eye(G.shape[0]), atol=1e-13)
    assert np.allclose(T.full(q), T.full(x), atol=1e-13)
    assert abs(nrm - np.linalg.norm(T.full(x))) < 1e-13 * nrm
    # left ranks never exceed the natural bound prod(p_<=k)
    rk = T.ranks(q)
    assert rk[1] <= 3 and rk[2] <= 5


def test_round_zero_tolerance_is_exact():
    x = I.random_tt([3, 2, 2, 2, 2, 2, 2], [1, 3, 6, 8, 8, 4, 2, 1], seed=7)
    z, info = T.round_tt(x, 0.0, return_info=True)
    assert np.max(np.abs(T.full(z) - T.full(x))) < 1e-13 * np.max(np.abs(T.full(x)))
    for c in z[1:]:
        G = T.right_gram(c)
        assert np.allclose(G, np.eye(G.shape[0]), atol=1e-13)
    # natural ranks: never more than the smaller side of each unfolding
    p = T.modes(x)
    for k in range(1, len(x)):
        assert info["ranks"][k] <= min(np.prod(p[:k]), np.prod(p[k:]))


@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-8])
def test_round_bound_and_eckart_young(eps):
    m = [3] + [2] * 8
    x = I.graded_tt(m, [1, 3, 6, 8, 10, 10, 8, 6, 4, 1], decay=0.35, seed=8)
    X = T.full(x)
    z, info = T.round_tt(x, eps, return_info=True)
    Z = T.full(z)
    assert np.linalg.norm(Z - X) <= eps * np.linalg.norm(X) * (1 + 1e-10)
    # bond singular values after the left sweep are those of the dense unfoldings
    # (first bond visited by the right sweep sees the untruncated tensor)
    n = len(x)
    k = n - 1
    unf = X.reshape(int(np.prod(m[:k])), -1)
    s_ref = np.linalg.svd(unf, compute_uv=False)
    s = info["svals"][k]
    q = min(len(s), len(s_ref))
    assert np.allclose(s[:q], s_ref[:q], rtol=0, atol=1e-12 * s_ref[0])
    # every kept rank is the smallest meeting the per-bond threshold
    for k in range(1, n):
        sv = info["svals"][k]
        l = info["ranks"][k]
        assert math.sqrt(np.sum(sv[l:] ** 2)) <= info["delta"] * (1 + 1e-12)
        if l > 1:
            assert math.sqrt(np.sum(sv[l - 1:] ** 2)) > info["delta"]


def test_round_rank_cap_and_error_report():
    m = [3] + [2] * 6
    x = I.random_tt(m, [1, 3, 6, 8, 8, 4, 2, 1], seed=9)
    z, info = T.round_tt(x, 1e-12, rmax=3, return_info=True)
    assert max(T.ranks(z)) <= 3
    X, Z = T.full(x), T.full(z)
    true_err = np.linalg.norm(X - Z) / np.linalg.norm(X)
    # reported error is the Pythagorean sum of per-bond discards (upper bound)
    assert info["err"] >= true_err * (1 - 1e-10)
    assert info["err"] <= true_err * math.sqrt(len(x))
