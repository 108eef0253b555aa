"""Pins of the oracle's Algorithm 2 against Algorithm 1 and closed forms."""
import json
import os

import numpy as np
import pytest

from oracle import ls_tt
from oracle import ms
from oracle import tt as T
from paper_2512_07811_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("L,seed", [(2, 1), (3, 2)])
def test_tt_iterates_equal_dense_iterates_without_truncation(L, seed):
    # with exact operands and zero rounding tolerance every TT iterate of
    # Algorithm 2 equals the dense iterate of Algorithm 1
    N = 2 ** L
    g = I.rng(seed)
    k = g.uniform(1.0, 3.0, size=(N, N, N))
    k0 = 2.0
    prob = ls_tt.Problem(k, k0, op_eps=1e-14, sfft_eps=1e-14)
    E = np.array([0.3, -1.0, 0.5])
    e_tt = ls_tt.O.mean_field_tt(E, L)
    E_tt = ls_tt.O.mean_field_tt(E, L)
    e_d = np.broadcast_to(E[:, None, None, None], (3, N, N, N)).copy()
    for m in range(3):
        e_tt, r_tt = ls_tt.ls_iterate(e_tt, prob.kp, prob.S, prob.G, prob.Sinv, E_tt, E, 0.0)
        e_new = ms.ms_step(e_d, k, k0, E)
        r_d = ms.residual(e_new, e_d, E)
        e_d = e_new
        full = T.full(e_tt).reshape(3, N, N, N)
        assert np.max(np.abs(full - e_d)) < 1e-11 * np.max(np.abs(e_d))
        assert abs(r_tt - r_d) < 1e-10 * max(r_d, 1e-3)


def test_laminate_c1_tt_closed_form():
    with open(os.path.join(GOLDEN, "laminate_32.json")) as f:
        gold = json.load(f)
    k = I.laminate(5)
    prob = ls_tt.Problem(k, 5.5)
    A, its = ls_tt.effective_tensor(prob, [0, 1], eps=1e-10, tol=1e-8, max_iter=200)
    assert abs(A[0, 0] - gold["A_xx"]) < 1e-10 * gold["A_xx"]
    assert abs(A[1, 1] - gold["A_yy"]) < 1e-10 * gold["A_yy"]
    assert its[0] <= 3 and its[1] <= 2


def test_truncated_tt_solution_close_to_dense():
    # rounding at eps gives an effective tensor close to the dense one
    L = 3
    k = I.random_boxes(L, 5, edge_min=2, edge_max=5, k_min=2.0, k_max=6.0)
    k0 = (k.min() + k.max()) / 2
    prob = ls_tt.Problem(k, k0)
    A_tt, _ = ls_tt.effective_tensor(prob, [0], eps=1e-6, tol=1e-9, max_iter=300)
    A_d = ms.effective_tensor(k, k0, loads=[0], tol=1e-12, max_iter=2000)
    assert np.max(np.abs(A_tt[:, 0] - A_d[:, 0])) < 1e-5 * abs(A_d[0, 0])
