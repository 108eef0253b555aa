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
