"""TT-cross set-up (paper_2512_07811_amd/cross.py) against the oracle (CPU).

maxvol: its dominance bound; tt_cross: exact recovery of a function of known
TT rank; the cross-built Green operator: equal to the oracle's dense momentum
array (Sec. 3.1-3.2) within the rounding tolerance, with the dense build's
ranks, also on the origin and the Nyquist planes where the formula is cut.
"""
import numpy as np
import pytest

from oracle import ops as O
from oracle import tt as T
from paper_2512_07811_amd import cross as X


def test_maxvol_submatrix_dominates():
    g = np.random.default_rng(3)
    A = g.standard_normal((60, 7))
    idx = X.maxvol(A)
    assert len(set(idx.tolist())) == 7
    B = A @ np.linalg.inv(A[idx])
    assert np.abs(B).max() <= 1.05 + 1e-12
    assert np.allclose(B[idx], np.eye(7), atol=1e-12)


def test_cross_recovers_a_function_of_known_rank():
    # f(x, y, z) = sin(x) cos(y) + x y z / 10 on a 16^3 grid: TT rank 2 over
    # the axes (and at most 4 inside an axis group of the 4 bits)
    L = 4
    W = X.grid_weights(L)
    h = 2 * np.pi / 16

    def fun(c):
        x, y, z = (c[..., 0] * h, c[..., 1] * h, c[..., 2] * h)
        return np.sin(x) * np.cos(y) + x * y * z / 10

    cores, info = X.tt_cross(fun, W, [2] * (3 * L), eps=1e-13, seed=1)
    full = T.full(cores).reshape(16, 16, 16)
    i = np.arange(16)
    ref = fun(np.stack(np.meshgrid(i, i, i, indexing="ij"), axis=-1))
    assert np.abs(full - ref).max() < 1e-11 * np.abs(ref).max()
    assert T.ranks(cores)[L] <= 2 and T.ranks(cores)[2 * L] <= 2


def test_tt_eval_matches_full():
    from paper_2512_07811_amd import inputs as I
    tt = I.random_tt([3, 2, 2, 2], [1, 3, 4, 2, 1], seed=4, is_complex=False)
    d = np.stack(np.meshgrid(np.arange(3), np.arange(2), np.arange(2), np.arange(2),
                             indexing="ij"), axis=-1).reshape(-1, 4)
    got = X.tt_eval(tt, d)
    assert np.allclose(got, T.full(tt).reshape(-1), rtol=0, atol=1e-13)


@pytest.mark.parametrize("L", [3, 4, 5])
def test_green_cross_equals_the_dense_momentum_operator(L):
    from paper_2512_07811_amd import operands as P
    k0 = 5.5
    G, info = X.green_tt_cross(L, k0, eps=1e-10)
    cores = [G[0].reshape(1, 9, -1).real] + [c.real for c in G[1:]]
    full = T.full(cores).reshape(3, 3, 2 ** L, 2 ** L, 2 ** L)
    ref = O.green_momentum(L, k0)
    print(f"[cross] L={L}: ranks {T.ranks(cores)}, sweeps {info['sweeps']}, "
          f"evaluations {info['evaluations']}")
    assert np.linalg.norm(full - ref) <= 1e-10 * np.linalg.norm(ref) * 1.01
    assert np.abs(full - ref).max() <= 1e-8 * np.abs(ref).max()
    # cut entries: the origin and every Nyquist plane stay zero
    N = 2 ** L
    nyq = 1                      # momentum position of frequency -N/2
    assert np.abs(full[:, :, 0, 0, 0]).max() < 1e-9 / k0
    assert np.abs(full[:, :, nyq]).max() < 1e-9 / k0
    assert np.abs(full[:, :, :, nyq]).max() < 1e-9 / k0
    assert np.abs(full[:, :, :, :, nyq]).max() < 1e-9 / k0
    dense_ranks = T.ranks([c.real for c in P.green_tt(L, k0, 1e-10)[1:]])
    assert max(T.ranks(cores)) <= max(dense_ranks) + 2
    assert N == full.shape[2]
