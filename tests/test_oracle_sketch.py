"""Pins of the randomized (randomize-then-orthogonalize) rounding oracle."""
import math

import numpy as np
import pytest

from oracle import sketch as SK
from oracle import tt as T
from paper_2512_07811_amd import inputs as I


def _natural(m):
    n = len(m)
    return [1] + [int(min(np.prod(m[:k]), np.prod(m[k:]))) for k in range(1, n)] + [1]


def test_rto_exact_when_sketch_covers_rank():
    m = [3, 2, 2, 2, 2, 2]
    x = I.random_tt(m, [1, 3, 4, 4, 3, 2, 1], seed=31)
    nat = _natural(m)
    ells = [1] + [min(nat[k], T.ranks(x)[k] + 3) for k in range(1, len(m))] + [1]
    om = I.gaussian_sketch(m, ells, seed=32)
    y = SK.rto(x, om)
    assert np.max(np.abs(T.full(y) - T.full(x))) < 1e-12 * np.max(np.abs(T.full(x)))
    for c in y[:-1]:
        assert np.allclose(T.left_gram(c), np.eye(c.shape[2]), atol=1e-13)


def test_rto_is_orthogonal_projection():
    m = [3] + [2] * 7
    x = I.graded_tt(m, [1, 3, 6, 8, 8, 8, 6, 4, 1], decay=0.5, seed=33)
    ells = [1, 2, 3, 4, 4, 4, 3, 2, 1]
    om = I.gaussian_sketch(m, ells, seed=34)
    y = SK.rto(x, om)
    X, Y = T.full(x), T.full(y)
    # Pythagoras: ||x||^2 = ||y||^2 + ||x - y||^2 and <x - y, y> = 0
    assert abs(np.vdot(X - Y, Y)) < 1e-12 * np.linalg.norm(X) ** 2
    assert abs(np.linalg.norm(X) ** 2 - np.linalg.norm(Y) ** 2
               - np.linalg.norm(X - Y) ** 2) < 1e-12 * np.linalg.norm(X) ** 2
    assert abs(np.linalg.norm(y[-1]) - np.linalg.norm(Y)) < 1e-13 * np.linalg.norm(X)


def test_right_sketch_definition_by_brute_force():
    # W_k = unfolding_{>=k}(x) times unfolding_{>=k}(Omega)^T
    m = [3, 2, 2, 2]
    x = I.random_tt(m, [1, 3, 4, 2, 1], seed=35)
    ells = [1, 2, 3, 2, 1]
    om = I.gaussian_sketch(m, ells, seed=36)
    W = SK.right_sketches(x, om)
    for k in range(1, len(m)):
        # explicit: contract x_{>=k} and Omega_{>=k} over all physical indices
        def right_part(cores):
            res = cores[-1][:, :, 0]                      # (r, p)
            for c in reversed(cores[:-1]):
                r, p, r2 = c.shape
                res = np.einsum("aib,bj->aij", c, res.reshape(r2, -1)).reshape(r, -1)
            return res
        Xr = right_part(x[k:])
        Or = right_part(om[k:])
        assert np.allclose(W[k], Xr @ Or.T, atol=1e-12)


@pytest.mark.parametrize("eps", [1e-3, 1e-6])
def test_sketch_round_meets_tolerance_with_oversampling(eps):
    m = [3] + [2] * 9
    x = I.graded_tt(m, [1, 3, 6, 10, 12, 12, 12, 10, 6, 3, 1], decay=0.3, seed=37)
    nat = _natural(m)
    ells = [1] + [min(nat[k], 16) for k in range(1, len(m))] + [1]
    om = I.gaussian_sketch(m, ells, seed=38)
    z, info = SK.sketch_round(x, om, eps)
    X, Z = T.full(x), T.full(z)
    assert info["ok"]
    assert np.linalg.norm(X - Z) <= eps * np.linalg.norm(X) * (1 + 1e-8)
    # compare with the deterministic SVD rounding: ranks agree within 1
    _, ref = T.round_tt(x, eps, return_info=True)
    for k in range(1, len(m)):
        assert abs(info["ranks"][k] - ref["ranks"][k]) <= 1


def test_sketch_round_noise_floor_when_over_budget():
    # bond 3's sketch width (3) is below its rank (4), so at eps = 1e-12 the
    # projection alone exhausts the budget; bond 4's width (6) exceeds its
    # rank (2): the floor 1e-14 ||x|| keeps that bond at its rank, where a
    # zero threshold keeps the sketch's noise directions as well
    modes = [2] * 6
    x = I.random_tt(modes, [1, 2, 4, 8, 2, 2, 1], seed=5)
    om = I.gaussian_sketch(modes, [1, 2, 4, 3, 6, 2, 1], seed=6)
    z, info = SK.sketch_round(x, om, 1e-12)
    assert not info["ok"]
    assert info["delta"] == pytest.approx(SK.NOISE_FLOOR * info["xnorm"], rel=1e-12)
    assert T.ranks(z)[4] == 2
    z0, info0 = SK.truncate_right(SK.rto(x, om), 0.0)
    assert T.ranks(z0)[4] > 2
    assert np.linalg.norm(T.full(z) - T.full(z0)) <= 1e-13 * info["xnorm"]


def test_capped_truncation_error_is_not_orthogonal_to_the_projection_error():
    # a rank cap truncates interior bonds of the sketched train; the result's
    # left interfaces leave the sketch's span, so ||x - z||^2 differs from
    # e_s^2 + sum tails^2 by a cross term well above rounding (brute force on
    # the dense tensors), while the linear bound e_s + sqrt(sum tails^2) holds
    m = [3] + [2] * 9
    nat = _natural(m)
    x = I.graded_tt(m, [1] + [min(v, 24) for v in nat[1:-1]] + [1], decay=0.85, seed=3)
    ells = [1] + [min(nat[k], 10) for k in range(1, len(m))] + [1]
    om = I.gaussian_sketch(m, ells, seed=7)
    z, info = SK.sketch_round(x, om, 1e-6, rmax=6)
    X, Z = T.full(x).ravel(), T.full(z).ravel()
    nx = np.linalg.norm(X)
    true = np.linalg.norm(X - Z) / nx
    tails2 = float(np.sum(np.asarray(info["disc"]) ** 2))
    quad = math.sqrt(info["sketch_err"] ** 2 + tails2) / nx
    assert abs(true - quad) > 1e-4 * true
    assert true <= info["err_bound"] * (1 + 1e-12)
    assert info["err_bound"] <= 2.0 * true


def test_uncapped_sketch_round_keeps_eps_by_the_linear_budget():
    m = [3] + [2] * 9
    x = I.graded_tt(m, [1, 3, 6, 10, 12, 12, 12, 10, 6, 3, 1], decay=0.5, seed=41)
    nat = _natural(m)
    ells = [1] + [min(nat[k], 14) for k in range(1, len(m))] + [1]
    om = I.gaussian_sketch(m, ells, seed=42)
    for eps in (1e-2, 1e-4):
        z, info = SK.sketch_round(x, om, eps)
        X, Z = T.full(x), T.full(z)
        assert info["ok"]
        assert np.linalg.norm(X - Z) <= info["err_bound"] * np.linalg.norm(X) * (1 + 1e-12)
        assert info["err_bound"] <= eps * (1 + 1e-12)
