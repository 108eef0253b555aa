"""Batched solves: several microstructures times several loads in one call,
with per-instance k' operators (zero-padded to common ranks) and shared SFFT
and Green operators.  Each field must come out as when solved on its own, and
match the dense Moulinec-Suquet oracle."""
import numpy as np
import pytest

from oracle import ms
from paper_2512_07811_amd import inputs as I

pytestmark = pytest.mark.gpu

L = 3
K0 = 3.5           # common reference medium for k in [1, 6]: (1 + 6) / 2
LOADS = [[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]]


@pytest.fixture(scope="module")
def q():
    from paper_2512_07811_amd import qtt
    return qtt


@pytest.fixture(scope="module")
def ctx(q):
    c = q.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def cells():
    from paper_2512_07811_amd import operands as P
    kv = [I.random_boxes(L, 300 + s, edge_min=2, edge_max=5, k_min=2.0, k_max=6.0) for s in range(3)]
    return kv, [P.build_problem(kvox=k, k0=K0) for k in kv]


def opts(q, mode=None):
    return q.solve_opts(1e-10, 0, tol=1e-9, max_iter=120,
                        mode=q.ROUND_SKETCH if mode is None else mode, oversample=4, seed=9)


def test_batched_fields_equal_separate_solves_and_dense(q, ctx, cells):
    from paper_2512_07811_amd import operands as P
    kv, probs = cells
    assert len({max(c.shape[0] for c in p["kp"]) for p in probs}) > 1   # uneven operator ranks
    ops, e = P.upload_batch(probs, LOADS, 0)
    A, its, res, st = q.homogenize(ctx, ops, e, opts(q))
    assert st == q.QT_OK
    assert A.shape == (len(probs) * len(LOADS), 3)
    for i, prob in enumerate(probs):
        ops1, e1 = P.upload(prob, LOADS, 0)
        A1, its1, _, st1 = q.homogenize(ctx, ops1, e1, opts(q))
        assert st1 == q.QT_OK
        Ab = A[i * len(LOADS):(i + 1) * len(LOADS)]
        assert np.max(np.abs(Ab - A1)) < 1e-8 * np.max(np.abs(A1))
        Ad = ms.effective_tensor(kv[i], K0, loads=[0, 1], tol=1e-11)
        for j in range(len(LOADS)):
            assert np.max(np.abs(Ab[j] - Ad[:, j])) < 1e-7 * np.max(np.abs(Ad[:, j]))


def test_plain_iteration_rejects_per_instance_operators(q, ctx, cells):
    from paper_2512_07811_amd import operands as P
    kv, probs = cells
    ops, e = P.upload_batch(probs, LOADS, 0)
    with pytest.raises(q.QtError):
        q.ls_iterate(ctx, ops, e, opts(q, q.ROUND_SVD), 1)


def test_early_converged_fields_keep_their_own_a_eff(q, ctx, cells):
    # one cell, loads e_x and e_y: at tol 1e-4 the dense oracle converges in
    # 14 and 15 iterations, so in the batch e_x converges first and goes on
    # iterating with e_y; its A_eff must still be that of iteration 14, as in
    # its separate solve (the SVD rounding draws nothing at random)
    from paper_2512_07811_amd import operands as P
    kv, probs = cells
    loads = [[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]]
    its_dense = [ms.solve(kv[0], K0, E, tol=1e-4, max_iter=200)[1] for E in loads]
    assert its_dense == [14, 15]
    o = q.solve_opts(1e-10, 0, tol=1e-4, max_iter=120, mode=q.ROUND_SVD)
    ops, e = P.upload(probs[0], loads, 0)
    A, its, _, st = q.homogenize(ctx, ops, e, o)
    assert st == q.QT_OK
    print(f"[batch] iterations batched {list(its)}, dense {its_dense}", flush=True)
    assert list(its) == its_dense
    for j, E in enumerate(loads):
        ops1, e1 = P.upload(probs[0], [E], 0)
        A1, its1, _, st1 = q.homogenize(ctx, ops1, e1, o)
        assert st1 == q.QT_OK and int(its1[0]) == its_dense[j]
        d = np.max(np.abs(A[j] - A1[0])) / np.max(np.abs(A1[0]))
        print(f"[batch] load {j}: batched vs separate A_eff {d:.2e}", flush=True)
        assert d < 1e-9
