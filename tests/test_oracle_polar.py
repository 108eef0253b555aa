"""Pins of the polar-decomposition compression oracle (oracle/polar.py).

The polar split keeps exactly the singular directions above the cutoff d~, so
on matrices and trains whose singular values keep away from d~ it must equal
a plain SVD truncation with the rule "keep sigma > d~" (numpy's SVD, written
out below); further pins: exact reconstruction at eps = 0, the tolerance
||x - x~|| <= eps ||x||, ranks never below the SVD rounding's, the reported
error equal to the dense error, and the rank cap.
"""
import math

import numpy as np
import pytest

from oracle import polar as PO
from oracle import tt as T
from paper_2512_07811_amd import inputs as I


def _unitary(n, g):
    Z = g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))
    Q, R = np.linalg.qr(Z)
    return Q * (np.diag(R) / np.abs(np.diag(R)))


@pytest.mark.parametrize("r,c", [(6, 10), (10, 6), (8, 8)])
def test_split_keeps_exactly_the_singular_values_above_the_cutoff(r, c):
    g = np.random.default_rng(5 + r + c)
    q = min(r, c)
    s = np.array([3.0, 1.5, 0.9, 0.4, 0.2, 0.05, 0.01, 0.002][:q])
    V, W = _unitary(r, g)[:, :q], _unitary(c, g)[:, :q]
    A = (V * s) @ np.conj(W.T)
    for cut in (1.0, 0.3, 0.03, 1e-3):
        core, carry, disc, l = PO.split_centre(A, cut)
        keep = int(np.sum(s > cut))
        assert l == max(keep, 1)
        ref = (V[:, :l] * s[:l]) @ np.conj(W[:, :l].T)
        assert np.linalg.norm(carry @ core - ref) <= 1e-12 * np.linalg.norm(A)
        assert abs(disc - math.sqrt(float(np.sum(s[l:] ** 2)))) <= 1e-12 * np.linalg.norm(A)
        # core rows orthonormal; carry = A core^dagger (an orthogonal projection of A)
        assert np.allclose(core @ np.conj(core.T), np.eye(l), atol=1e-12)
        assert np.allclose(carry, A @ np.conj(core.T), atol=1e-12)


def test_split_cap_keeps_the_dominant_directions():
    g = np.random.default_rng(11)
    s = np.array([2.0, 1.0, 0.5, 0.25, 0.1, 0.01])
    V, W = _unitary(6, g), _unitary(9, g)[:, :6]
    A = (V * s) @ np.conj(W.T)
    core, carry, disc, l = PO.split_centre(A, 0.05, rmax=3)
    assert l == 3
    ref = (V[:, :3] * s[:3]) @ np.conj(W[:, :3].T)
    assert np.linalg.norm(carry @ core - ref) <= 1e-12 * np.linalg.norm(A)
    assert abs(disc ** 2 - float(np.sum(s[3:] ** 2))) <= 1e-12


def _svd_threshold_rounding(tt, eps):
    """Plain right-to-left SVD sweep keeping sigma > delta / q (the rule the
    polar split realises), with the gap of the nearest singular value to the
    cutoff at every bond."""
    cores, nrm = T.orthogonalize_left(tt)
    n = len(cores)
    delta = eps * nrm / math.sqrt(n - 1)
    gaps, ranks = [], [1] * (n + 1)
    for k in range(n - 1, 0, -1):
        r, p, r2 = cores[k].shape
        U, s, Vh = np.linalg.svd(cores[k].reshape(r, p * r2), full_matrices=False)
        cut = delta / len(s)
        gaps.append(float(np.min(np.abs(s - cut))) / cut)
        l = max(int(np.sum(s > cut)), 1)
        ranks[k] = l
        cores[k] = Vh[:l].reshape(l, p, r2)
        prev = cores[k - 1]
        rp, pp, _ = prev.shape
        cores[k - 1] = (prev.reshape(rp * pp, r) @ (U[:, :l] * s[:l])).reshape(rp, pp, l)
    return cores, ranks, min(gaps)


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("eps", [1e-2, 1e-5])
def test_round_polar_equals_threshold_svd_rounding(seed, eps):
    modes = [3, 2, 2, 2, 2, 2, 2]
    tt = I.graded_tt(modes, [1, 3, 6, 8, 8, 4, 2, 1], decay=0.35, seed=40 + seed)
    ref, rref, gap = _svd_threshold_rounding(tt, eps)
    assert gap > 1e-3           # no singular value near a cutoff: the rule is unambiguous
    got, info = PO.round_polar(tt, eps, return_info=True)
    assert info["ranks"] == rref
    X = T.full(tt)
    assert np.linalg.norm(T.full(got) - T.full(ref)) <= 1e-10 * np.linalg.norm(X)


@pytest.mark.parametrize("seed", [4, 5])
@pytest.mark.parametrize("eps", [0.0, 1e-8, 1e-3, 1e-1])
def test_round_polar_tolerance_error_report_and_ranks(seed, eps):
    modes = [3, 2, 2, 2, 2, 2, 2, 2]
    tt = I.graded_tt(modes, [1, 3, 5, 8, 10, 8, 4, 2, 1], decay=0.6, seed=50 + seed)
    X = T.full(tt)
    got, info = PO.round_polar(tt, eps, return_info=True)
    G = T.full(got)
    dense = np.linalg.norm(X - G) / np.linalg.norm(X)
    assert dense <= eps * (1 + 1e-9) + 1e-13
    assert abs(info["err"] - dense) <= 1e-10 + 1e-8 * dense
    _, sinfo = T.round_tt(tt, eps, return_info=True)
    # the absolute cutoff delta / q is conservative: never fewer directions
    assert all(a >= b for a, b in zip(info["ranks"], sinfo["ranks"]))
    if eps > 0:
        for c in got[1:]:
            assert np.allclose(T.right_gram(c), np.eye(c.shape[0]), atol=1e-10)


def test_round_polar_rank_cap_reports_its_error():
    modes = [3, 2, 2, 2, 2, 2, 2]
    tt = I.random_tt(modes, [1, 3, 6, 8, 8, 4, 2, 1], seed=61)
    got, info = PO.round_polar(tt, 1e-12, rmax=3, return_info=True)
    assert max(T.ranks(got)) <= 3
    X = T.full(tt)
    dense = np.linalg.norm(X - T.full(got)) / np.linalg.norm(X)
    assert dense > 1e-3
    assert abs(info["err"] - dense) <= 1e-10


def test_round_polar_cutoff_counts_the_centres_singular_values():
    # two cores, centre A (3 x 4) with singular values 1, 0.1, 0.01: q =
    # min(3, 4) = 3, and with delta = 0.035 the cutoff delta / 3 = 0.0117
    # drops sigma = 0.01, which a cutoff over max(3, 4) = 4 (0.00875) keeps
    g = np.random.default_rng(7)
    s = np.array([1.0, 0.1, 0.01])
    U = _unitary(8, g)[:, :3]
    W = _unitary(4, g)[:, :3]
    tt = [U.reshape(1, 8, 3), (s[:, None] * np.conj(W.T)).reshape(3, 4, 1)]
    nrm = float(np.linalg.norm(s))
    got, info = PO.round_polar(tt, 0.035 / nrm, return_info=True)
    assert info["ranks"][1] == 2
    assert abs(info["disc"][1] - 0.01) <= 1e-12
