"""Degenerate and edge cases of the method through the C ABI."""
import numpy as np
import pytest

from oracle import tt as T
from paper_2512_07811_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    from paper_2512_07811_amd import qtt
    return qtt


@pytest.fixture(scope="module")
def ctx(q):
    c = q.Context(0)
    yield c
    c.close()


MODES = {"svd": "ROUND_SVD", "sketch": "ROUND_SKETCH"}


@pytest.mark.parametrize("mode", ["svd", "sketch"])
def test_reference_medium_equal_to_k_gives_mean_field(q, ctx, mode):
    # k = k0 everywhere: k' = 0, every product vanishes (zero norms, zero
    # matrices in QR and SVD), e' = E up to the roundoff of re-orthogonalizing
    # E, A_eff = k0 I
    from paper_2512_07811_amd import operands as P
    L = 3
    k = np.full((2 ** L,) * 3, 2.5)
    prob = P.build_problem(kvox=k, k0=2.5)
    ops, e = P.upload(prob, [[1.0, 0.0, 0.0], [0.0, 0.0, 2.0]], 8)
    A, its, res, st = q.homogenize(ctx, ops, e, q.solve_opts(1e-8, 8, tol=1e-10, max_iter=5,
                                                             mode=getattr(q, MODES[mode]),
                                                             oversample=4, seed=1))
    assert st == q.QT_OK
    assert np.all(its == 1) and np.all(res[0] < 1e-13)
    assert np.allclose(A, [[2.5, 0, 0], [0, 0, 5.0]], atol=1e-13)


@pytest.mark.parametrize("mode", ["svd", "sketch"])
def test_homogeneous_medium_converges_in_one_step(q, ctx, mode):
    # k constant but != k0: tau = k' e is constant, its transform lives at the
    # zero frequency where the Green operator vanishes, so e_1 = E
    from paper_2512_07811_amd import operands as P
    L = 3
    k = np.full((2 ** L,) * 3, 3.0)
    prob = P.build_problem(kvox=k, k0=2.0)
    ops, e = P.upload(prob, [[0.0, 1.0, 0.0]], 8)
    A, its, res, st = q.homogenize(ctx, ops, e, q.solve_opts(1e-10, 8, tol=1e-9, max_iter=5,
                                                             mode=getattr(q, MODES[mode]),
                                                             oversample=4, seed=1))
    assert st == q.QT_OK and its[0] == 1
    assert res[0, 0] < 1e-12
    assert np.allclose(A[0], [0.0, 3.0, 0.0], atol=1e-11)


def test_zero_load_is_rejected(q, ctx):
    from paper_2512_07811_amd import operands as P
    k = I.random_boxes(3, 5, edge_min=2, edge_max=5, k_min=2.0, k_max=6.0)
    prob = P.build_problem(kvox=k, k0=4.0)
    ops, e = P.upload(prob, [[0.0, 0.0, 0.0]], 8)
    with pytest.raises(q.QtError):
        q.ls_iterate(ctx, ops, e, q.solve_opts(1e-8, 8), 1)


def test_round_zero_and_single_core_trains(q, ctx):
    # a zero train keeps rank 1 with zero error; a one-core train is only normed
    modes = [3] + [2] * 6
    z = [np.zeros((r0, p, r1), dtype=complex) for r0, p, r1 in
         zip([1, 2, 3, 3, 3, 2, 2], modes, [2, 3, 3, 3, 2, 2, 1])]
    Z = q.DeviceTT.from_cores([z])
    err, nrm = q.tt_round(ctx, Z, 1e-6)
    ctx.sync()
    assert nrm.cpu().numpy()[0] == 0.0 and err.cpu().numpy()[0] == 0.0
    assert np.all(np.isfinite(T.full(Z.to_cores()[0])))
    assert np.all(T.full(Z.to_cores()[0]) == 0)
    one = [I.random_tt([5], [1, 1], seed=3)[0]]
    X = q.DeviceTT.from_cores([one])
    err, nrm = q.tt_round(ctx, X, 1e-3)
    ctx.sync()
    assert abs(nrm.cpu().numpy()[0] - np.linalg.norm(one[0])) < 1e-14 * np.linalg.norm(one[0])
    assert np.allclose(X.to_cores()[0][0], one[0], atol=0)


@pytest.mark.parametrize("eps", [0.0, 1e-12])
def test_round_component_below_double_square_range(q, ctx, eps):
    # x = a + 1e-160 b: after the first reflection the orthogonal part of a
    # column is ~1e-160, whose squared norm is denormal; the reflector is then
    # computed from the column scaled by 2^600 (a finite, exact rounding is
    # required: the tiny component is kept at eps = 0, dropped at eps > 0)
    modes = [3] + [2] * 7
    a = I.random_tt(modes, [1] * 9, seed=91)
    b = I.random_tt(modes, [1] * 9, seed=92)
    x = T.add(a, T.scale(b, 1e-160))
    X = q.DeviceTT.from_cores([x])
    err, nrm = q.tt_round(ctx, X, eps)
    ctx.sync()
    out = X.to_cores()[0]
    ref, info = T.round_tt(x, eps, None, return_info=True)
    full_out = T.full(out)
    assert np.all(np.isfinite(full_out))
    assert T.ranks(out) == T.ranks(ref)
    assert np.linalg.norm(full_out - T.full(ref)) <= 1e-14 * np.linalg.norm(T.full(ref))
    assert abs(nrm.cpu().numpy()[0] - info["norm"]) <= 1e-14 * info["norm"]


def test_jacobi_sweep_cap_reports_diagnostics(q):
    # a one-sweep cap on SVD blocks of order 16 cannot converge: the rounding
    # returns QT_ENUMERIC with the order, the last sweep's worst off-diagonal
    # (above the tolerance) and the sweep count; the kernels exit normally
    c = q.Context(0)
    try:
        modes = [3] + [2] * 9
        x = I.random_tt(modes, [1, 3, 6, 12, 16, 16, 16, 12, 6, 3, 1], seed=123)
        X = q.DeviceTT.from_cores([x])
        with pytest.raises(q.QtError) as ei:
            q.tt_round(c, X, 0.0, 0, jacobi_max_sweeps=1)
            c.sync()
        assert ei.value.status == -5
        msg = str(ei.value)
        assert "sweep cap" in msg and ", 1 sweeps)" in msg
        worst = float(msg.split("worst off-diagonal ")[1].split(" ")[0])
        assert worst > 1.0
    finally:
        c.close()
