"""Pins of the AMEn product oracle (oracle/amen.py) against the dense product.

The reference is T.full of T.mpo_apply (the exact TT x TTO contraction, pinned
in test_oracle_tt.py) or the dense matrix-vector product: exact recovery once
the frames cover the product's rank, convergence by enrichment from a rank-1
start, the tolerance, the Hadamard product through the diagonal lift, the
identity operator and the rank cap; and the right orthogonalization the
sweeps start from (the tensor kept, orthonormal rows, ranks min(r_k, p_k r_{k+1})).
"""
import numpy as np
import pytest

from oracle import amen as AM
from oracle import tt as T
from paper_2512_07811_amd import inputs as I

MODES = [3] + [2] * 7


def _problem(seed=1):
    x = I.random_tt(MODES, [1, 3, 4, 4, 4, 4, 4, 2, 1], seed=seed)
    A = I.random_mpo(MODES, MODES, [1, 2, 3, 3, 3, 3, 3, 2, 1], seed=seed + 1)
    return A, x


def _dense(A, x):
    # dense operator times dense vector: independent of the TT contraction
    return (T.full_operator(A) @ T.full(x).reshape(-1)).reshape(MODES)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_one_sweep_recovers_the_product_when_the_frames_cover_its_rank():
    A, x = _problem()
    ref = _dense(A, x)
    y0 = I.random_tt(MODES, [1] + [12] * 7 + [1], seed=3)
    z0 = I.random_tt(MODES, [1] + [4] * 7 + [1], seed=4)
    y = AM.amen_mv(A, x, y0, z0, 1e-13, sweeps=1)
    assert rel(T.full(y), ref) < 1e-12
    assert T.ranks(y) == T.ranks(T.round_tt(T.mpo_apply(A, x), 1e-13))


def test_enrichment_grows_a_rank_one_start_to_the_product():
    A, x = _problem(5)
    ref = _dense(A, x)
    y0 = I.random_tt(MODES, [1] * 9, seed=7)
    z0 = I.random_tt(MODES, [1] + [4] * 7 + [1], seed=8)
    errs = []
    for sw in (1, 2, 3, 5):
        y, info = AM.amen_mv(A, x, y0, z0, 1e-13, sweeps=sw, return_info=True)
        errs.append(rel(T.full(y), ref))
    assert errs[0] > 1e-3            # one sweep of rank <= 5 cannot hold rank 12
    assert errs[-1] < 1e-12
    assert all(b <= a * 1.0001 + 1e-14 for a, b in zip(errs, errs[1:]))


@pytest.mark.parametrize("eps", [1e-2, 1e-5])
def test_tolerance_on_a_graded_product(eps):
    ranks = [1, 3, 6, 8, 8, 8, 6, 2, 1]
    x = I.graded_tt(MODES, ranks, decay=0.5, seed=11)
    A = I.random_mpo(MODES, MODES, [1, 2, 2, 2, 2, 2, 2, 2, 1], seed=12)
    ref = _dense(A, x)
    y0 = I.random_tt(MODES, [1] + [8] * 7 + [1], seed=13)
    z0 = I.random_tt(MODES, [1] + [6] * 7 + [1], seed=14)
    y = AM.amen_mv(A, x, y0, z0, eps, sweeps=4)
    assert rel(T.full(y), ref) <= 1.5 * eps
    svd = T.round_tt(T.mpo_apply(A, x), eps)
    assert max(T.ranks(y)) <= max(T.ranks(svd)) + 2


def test_diagonal_lift_gives_the_hadamard_product():
    k = I.random_tt(MODES, [1, 2, 2, 2, 2, 2, 2, 2, 1], seed=21, is_complex=False)
    x = I.random_tt(MODES, [1, 3, 3, 3, 3, 3, 3, 2, 1], seed=22)
    y0 = I.random_tt(MODES, [1] + [8] * 7 + [1], seed=23)
    z0 = I.random_tt(MODES, [1] + [4] * 7 + [1], seed=24)
    y = AM.amen_mv(T.diag_lift(k), x, y0, z0, 1e-13, sweeps=2)
    assert rel(T.full(y), T.full(k) * T.full(x)) < 1e-12


def test_identity_operator_returns_the_train():
    x = I.random_tt(MODES, [1, 3, 4, 4, 4, 4, 4, 2, 1], seed=31)
    eye = [np.eye(p).reshape(1, p, p, 1).astype(np.complex128) for p in MODES]
    y0 = I.random_tt(MODES, [1] * 9, seed=32)
    z0 = I.random_tt(MODES, [1] + [4] * 7 + [1], seed=33)
    y = AM.amen_mv(eye, x, y0, z0, 1e-13, sweeps=4)
    assert rel(T.full(y), T.full(x)) < 1e-12


def test_rank_cap_is_near_the_best_capped_rounding():
    A, x = _problem(41)
    ref = _dense(A, x)
    y0 = I.random_tt(MODES, [1] + [12] * 7 + [1], seed=43)
    z0 = I.random_tt(MODES, [1] + [4] * 7 + [1], seed=44)
    y = AM.amen_mv(A, x, y0, z0, 1e-13, rmax=5, sweeps=3)
    best = T.round_tt(T.mpo_apply(A, x), 1e-13, rmax=5)
    assert max(T.ranks(y)) <= 5
    assert rel(T.full(y), ref) <= 1.05 * rel(T.full(best), ref)


def test_right_orthogonalization_keeps_the_train_and_orthonormalizes_its_rows():
    # ranks above the natural bound on the right (8 > 2 * 2 at the last bonds)
    # shrink to min(r_k, p_k r_{k+1}); the tensor is unchanged
    x = I.random_tt(MODES, [1, 3, 6, 12, 12, 8, 8, 8, 1], seed=51)
    y = AM.orthogonalize_right(x)
    assert rel(T.full(y), T.full(x)) < 1e-13
    for c in y[1:]:
        r, p, r2 = c.shape
        M = c.reshape(r, p * r2)
        assert np.allclose(M @ M.conj().T, np.eye(r), atol=1e-13)
    r_in, ranks = [1, 3, 6, 12, 12, 8, 8, 8, 1], T.ranks(y)
    for k in range(len(MODES) - 1, 0, -1):
        assert ranks[k] == min(r_in[k], MODES[k] * ranks[k + 1])
    assert ranks[-2] == 2 and ranks[-3] == 4
