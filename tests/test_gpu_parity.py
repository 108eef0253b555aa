"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Gauge-invariant comparisons only: dense reconstructions, ranks, norms, dot
products and reported errors (TT cores are unique only up to gauge).
FP64 bar: relative error <= 1e-10 (per operation the kernels reach ~1e-13).
"""
import math

import numpy as np
import pytest

from oracle import ls_tt
from oracle import ops as O
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


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300)


def ragged_pair(modes, seed):
    n = len(modes)
    nat = [1] + [min(int(np.prod(modes[:k])), int(np.prod(modes[k:]))) for k in range(1, n)] + [1]
    g = I.rng(seed)
    r1 = [1] + [int(min(nat[k], g.integers(1, 7))) for k in range(1, n)] + [1]
    r2 = [1] + [int(min(nat[k], g.integers(1, 7))) for k in range(1, n)] + [1]
    return r1, r2


def test_hadamard_mpo_add_dot(q, ctx):
    modes = [3, 2, 2, 2, 2, 2, 2]
    r1, r2 = ragged_pair(modes, 1)
    xs = [I.random_tt(modes, r1, seed=10 + b) for b in range(2)]
    ys = [I.random_tt(modes, r2, seed=20 + b) for b in range(2)]
    cap = [1] + [7] * (len(modes) - 1) + [1]
    X = q.DeviceTT.from_cores(xs, cap)
    Y = q.DeviceTT.from_cores(ys, cap)
    # Hadamard (batched)
    H = q.tt_hadamard(ctx, X, Y)
    out = H.to_cores()
    for b in range(2):
        ref = T.hadamard(xs[b], ys[b])
        assert T.ranks(out[b]) == T.ranks(ref)
        assert rel(T.full(out[b]), T.full(ref)) < 1e-13
    # broadcast of a single train over the batch
    X1 = q.DeviceTT.from_cores([xs[0]], cap)
    H1 = q.tt_hadamard(ctx, X1, Y).to_cores()
    assert rel(T.full(H1[1]), T.full(T.hadamard(xs[0], ys[1]))) < 1e-13
    # general and diagonal operators
    A = I.random_mpo(modes, modes, [1, 2, 3, 2, 3, 2, 2, 1], seed=30)
    Ad = q.DeviceMPO.from_cores(A)
    Z = q.tt_mpo_apply(ctx, Ad, X).to_cores()
    for b in range(2):
        assert rel(T.full(Z[b]), T.full(T.mpo_apply(A, xs[b]))) < 1e-13
    dcores = I.random_tt(modes, [1, 2, 2, 3, 2, 2, 2, 1], seed=31)
    Dd = q.DeviceMPO.from_cores(dcores, [1] * len(modes))
    Zd = q.tt_mpo_apply(ctx, Dd, X).to_cores()
    assert rel(T.full(Zd[0]), T.full(xs[0]) * T.full(dcores)) < 1e-13
    # scaled addition
    S = q.tt_add(ctx, 0.5 - 1j, X, 2.0, Y).to_cores()
    for b in range(2):
        assert rel(T.full(S[b]), (0.5 - 1j) * T.full(xs[b]) + 2.0 * T.full(ys[b])) < 1e-13
    # dot
    d = q.tt_dot(ctx, X, Y).cpu().numpy()
    for b in range(2):
        ref = np.vdot(T.full(xs[b]), T.full(ys[b]))
        assert abs(d[b] - ref) < 1e-12 * abs(ref) + 1e-14


@pytest.mark.parametrize("eps,rmax", [(0.0, 0), (1e-3, 0), (1e-8, 0), (1e-12, 5)])
def test_round_matches_oracle(q, ctx, eps, rmax):
    modes = [3] + [2] * 9
    ranks = [1, 3, 6, 10, 14, 16, 14, 10, 6, 2, 1]
    xs = [I.graded_tt(modes, ranks, decay=0.4, seed=40 + b) for b in range(3)]
    X = q.DeviceTT.from_cores(xs)
    err, nrm = q.tt_round(ctx, X, eps, rmax)
    ctx.sync()
    out = X.to_cores()
    err = err.cpu().numpy()
    nrm = nrm.cpu().numpy()
    for b in range(3):
        ref, info = T.round_tt(xs[b], eps, rmax or None, return_info=True)
        assert T.ranks(out[b]) == T.ranks(ref)
        assert rel(T.full(out[b]), T.full(ref)) < 1e-10
        assert abs(nrm[b] - info["norm"]) < 1e-13 * info["norm"]
        assert abs(err[b] - info["err"]) <= 1e-10 * max(info["err"], 1e-300) + 1e-15
        # right-orthogonal cores after the sweep
        for c in out[b][1:]:
            G = T.right_gram(c)
            assert np.allclose(G, np.eye(G.shape[0]), atol=1e-12)


@pytest.mark.parametrize("eps", [0.0, 1e-8])
def test_round_mixed_orientation_and_subfloor_columns(q, ctx, eps):
    # one batch whose right sweep meets wide SVD blocks (A^H = QR, then the
    # second QR of R^H) and tall ones (A = QR), with ragged ranks, and an
    # instance with a component 1e-100 below the Jacobi's rotation floor:
    # those columns are never rotated, so at eps = 0 they are kept through an
    # orthonormal completion (same ranks as the oracle, orthonormal cores),
    # at eps > 0 they are truncated
    modes = [3] + [2] * 9
    xa = I.graded_tt(modes, [1, 3, 6, 12, 16, 16, 12, 6, 3, 2, 1], decay=0.5, seed=71)
    xb = I.graded_tt(modes, [1, 3, 6, 12, 24, 12, 4, 8, 4, 2, 1], decay=0.5, seed=72)
    a = I.random_tt(modes, [1, 2, 4, 4, 4, 4, 4, 4, 4, 2, 1], seed=73)
    b = I.random_tt(modes, [1, 2, 3, 3, 3, 3, 3, 3, 3, 2, 1], seed=74)
    xc = T.add(a, T.scale(b, 1e-100))
    xs = [xa, xb, xc]
    X = q.DeviceTT.from_cores(xs)
    err, nrm = q.tt_round(ctx, X, eps, 0)
    ctx.sync()
    out = X.to_cores()
    nrm = nrm.cpu().numpy()
    for i in range(3):
        ref, info = T.round_tt(xs[i], eps, None, return_info=True)
        assert T.ranks(out[i]) == T.ranks(ref)
        assert rel(T.full(out[i]), T.full(ref)) < 1e-10
        assert abs(nrm[i] - info["norm"]) < 1e-13 * info["norm"]
        for c in out[i][1:]:
            G = T.right_gram(c)
            assert np.allclose(G, np.eye(G.shape[0]), atol=1e-12)


@pytest.mark.parametrize("eps", [0.0, 1e-9])
def test_round_jacobi_orders_101_to_256_match_oracle(q, ctx, eps):
    # right-sweep SVD blocks of orders 192-220: the global-memory Jacobi with
    # each pair's columns held in registers by 32-lane groups
    modes = [3] + [2] * 16
    ranks = [1, 3, 6, 12, 24, 48, 96, 192, 220, 192, 128, 64, 32, 16, 8, 4, 2, 1]
    xs = [I.graded_tt(modes, ranks, decay=0.97, seed=170 + b) for b in range(2)]
    X = q.DeviceTT.from_cores(xs)
    err, nrm = q.tt_round(ctx, X, eps, 0)
    ctx.sync()
    out = X.to_cores()
    nrm = nrm.cpu().numpy()
    for b in range(2):
        ref, info = T.round_tt(xs[b], eps, None, return_info=True)
        assert T.ranks(out[b]) == T.ranks(ref)
        assert rel(T.full(out[b]), T.full(ref)) < 1e-10
        assert abs(nrm[b] - info["norm"]) < 1e-12 * info["norm"]
        for c in out[b][1:]:
            G = T.right_gram(c)
            assert np.allclose(G, np.eye(G.shape[0]), atol=1e-12)


@pytest.mark.parametrize("eps", [0.0, 1e-9])
def test_round_jacobi_orders_128_and_136_match_oracle(q, ctx, eps):
    # SVD blocks of orders 136 and 128: the global-memory Jacobi's 16-lane
    # pair groups (nine and eight elements per lane; a step's pairs in two
    # passes and in one)
    modes = [3] + [2] * 14
    ranks = [1, 3, 6, 12, 24, 48, 96, 136, 128, 64, 32, 16, 8, 4, 2, 1]
    xs = [I.graded_tt(modes, ranks, decay=0.96, seed=180 + b) for b in range(2)]
    X = q.DeviceTT.from_cores(xs)
    err, nrm = q.tt_round(ctx, X, eps, 0)
    ctx.sync()
    out = X.to_cores()
    nrm = nrm.cpu().numpy()
    for b in range(2):
        ref, info = T.round_tt(xs[b], eps, None, return_info=True)
        assert T.ranks(out[b]) == T.ranks(ref)
        assert rel(T.full(out[b]), T.full(ref)) < 1e-10
        assert abs(nrm[b] - info["norm"]) < 1e-12 * info["norm"]
        for c in out[b][1:]:
            G = T.right_gram(c)
            assert np.allclose(G, np.eye(G.shape[0]), atol=1e-12)


@pytest.mark.parametrize("eps", [0.0, 1e-9])
def test_round_large_ranks_matches_oracle(q, ctx, eps):
    # bond ranks up to 100: the right sweep's SVD orders exceed the LDS Jacobi
    # (68) and the left sweep's matrices exceed LDS, so the global-memory QR
    # and Jacobi kernels run
    modes = [3] + [2] * 13
    ranks = [1, 3, 6, 12, 24, 48, 90, 100, 64, 32, 16, 8, 4, 2, 1]
    xs = [I.graded_tt(modes, ranks, decay=0.9, seed=140 + b) for b in range(2)]
    X = q.DeviceTT.from_cores(xs)
    err, nrm = q.tt_round(ctx, X, eps, 0)
    ctx.sync()
    out = X.to_cores()
    nrm = nrm.cpu().numpy()
    for b in range(2):
        ref, info = T.round_tt(xs[b], eps, None, return_info=True)
        assert T.ranks(out[b]) == T.ranks(ref)
        assert rel(T.full(out[b]), T.full(ref)) < 1e-10
        assert abs(nrm[b] - info["norm"]) < 1e-12 * info["norm"]


@pytest.mark.parametrize("eps,rmax", [(0.0, 0), (1e-6, 0), (1e-12, 40)])
def test_round_blocked_qr_matches_oracle(q, ctx, eps, rmax):
    # capacities of 280 make the left sweep's unfoldings (up to 560 x 280)
    # take the blocked Householder QR (panels of 32 columns, trailing updates
    # and Q on the MFMA GEMM); the actual ranks (up to 160, the second instance
    # smaller) leave panels idle or partial inside those launches
    modes = [3] + [2] * 15
    r0 = [1, 3, 6, 12, 24, 48, 96, 160, 160, 128, 64, 32, 16, 8, 4, 2, 1]
    r1 = [1, 3, 6, 12, 24, 48, 70, 100, 90, 64, 40, 32, 16, 8, 4, 2, 1]
    cap = [1, 3, 6, 12, 24, 48, 96, 280, 280, 256, 64, 32, 16, 8, 4, 2, 1]
    xs = [I.graded_tt(modes, r0, decay=0.93, seed=170),
          I.graded_tt(modes, r1, decay=0.9, seed=171)]
    X = q.DeviceTT.from_cores(xs, cap)
    err, nrm = q.tt_round(ctx, X, eps, rmax)
    ctx.sync()
    out = X.to_cores()
    nrm = nrm.cpu().numpy()
    err = err.cpu().numpy()
    for b in range(2):
        ref, info = T.round_tt(xs[b], eps, rmax or None, return_info=True)
        assert T.ranks(out[b]) == T.ranks(ref)
        assert rel(T.full(out[b]), T.full(ref)) < 1e-10
        assert abs(nrm[b] - info["norm"]) < 1e-12 * info["norm"]
        # the discarded tails (~eps ||x||) carry absolute errors ~1e-16 ||x||
        assert abs(err[b] - info["err"]) <= 1e-6 * info["err"] + 1e-13


def test_round_product_train_and_ragged_batch(q, ctx):
    # a materialized Hadamard product is rounded exactly like the oracle does
    modes = [3] + [2] * 8
    a = I.random_tt(modes, [1, 2, 4, 5, 6, 5, 4, 3, 2, 1], seed=50)
    b = I.random_tt(modes, [1, 3, 3, 4, 4, 4, 3, 2, 2, 1], seed=51)
    prod = T.hadamard(a, b)
    X = q.DeviceTT.from_cores([prod, T.hadamard(b, b)])
    q.tt_round(ctx, X, 1e-6)
    out = X.to_cores()
    for got, src in zip(out, [prod, T.hadamard(b, b)]):
        ref = T.round_tt(src, 1e-6)
        assert T.ranks(got) == T.ranks(ref)
        assert rel(T.full(got), T.full(ref)) < 1e-10


@pytest.mark.parametrize("L", [2, 3])
def test_ls_iterates_match_oracle_without_truncation(q, ctx, L):
    from paper_2512_07811_amd import operands as P
    N = 2 ** L
    g = I.rng(60 + L)
    k = g.uniform(1.0, 3.0, size=(N, N, N))
    k0 = 2.0
    E = np.array([1.0, 0.0, 0.0])
    prob = P.build_problem(kvox=k, k0=k0, op_eps=1e-14, sfft_eps=1e-14)
    ops, e = P.upload(prob, [E], max_rank=0)
    oprob = ls_tt.Problem(k, k0, op_eps=1e-14, sfft_eps=1e-14)
    opts = q.solve_opts(0.0, 0)
    # start from E
    e_cores = [O.mean_field_tt(E, L)]
    e = q.DeviceTT.from_cores(e_cores, e.cap)
    e_ref = O.mean_field_tt(E, L)
    E_tt = O.mean_field_tt(E, L)
    for m in range(3):
        res = q.ls_iterate(ctx, ops, e, opts, 1).cpu().numpy()
        e_ref, r_ref = ls_tt.ls_iterate(e_ref, oprob.kp, oprob.S, oprob.G, oprob.Sinv, E_tt, E, 0.0)
        got = T.full(e.to_cores()[0])
        assert rel(got, T.full(e_ref)) < 1e-10
        assert abs(res[0, 0] - r_ref) < 1e-9 * max(r_ref, 1e-6)


def test_residual_dot_value_and_exact_sweep_in_one_batch(q, ctx):
    # the residual takes the environment dot value where ||e' - e|| is large
    # against ||e'|| + ||e|| and the exact left-orthogonalizing sweep close to
    # convergence; field 0 starts at E (residual 0.11, dot value), field 1
    # three oracle iterations in (residual 2.8e-4, exact sweep), one batch
    from paper_2512_07811_amd import operands as P
    L, N = 2, 4
    g = I.rng(77)
    k = g.uniform(1.0, 3.0, size=(N, N, N))
    k0 = 2.0
    E = np.array([1.0, 0.0, 0.0])
    prob = P.build_problem(kvox=k, k0=k0, op_eps=1e-14, sfft_eps=1e-14)
    oprob = ls_tt.Problem(k, k0, op_eps=1e-14, sfft_eps=1e-14)
    E_tt = O.mean_field_tt(E, L)
    x = O.mean_field_tt(E, L)
    for _ in range(3):
        x, r = ls_tt.ls_iterate(x, oprob.kp, oprob.S, oprob.G, oprob.Sinv, E_tt, E, 0.0)
    starts = [O.mean_field_tt(E, L), x]
    refs = [ls_tt.ls_iterate(s0, oprob.kp, oprob.S, oprob.G, oprob.Sinv, E_tt, E, 0.0)
            for s0 in starts]
    assert refs[0][1] > 1e-2 and refs[1][1] < 1e-3
    ops, e = P.upload(prob, [E, E], max_rank=0)
    e = q.DeviceTT.from_cores(starts, e.cap)
    res = q.ls_iterate(ctx, ops, e, q.solve_opts(0.0, 0, mode=q.ROUND_SVD), 1).cpu().numpy()
    out = e.to_cores()
    for b in range(2):
        assert rel(T.full(out[b]), T.full(refs[b][0])) < 1e-10
        assert abs(res[0, b] - refs[b][1]) < 1e-8 * refs[b][1]


def test_ls_iterates_match_oracle_with_binding_rank_cap(q, ctx):
    # a cap that binds on the middle bonds of three of the four roundings; the
    # spectra are separated at the cut, so the truncation is well defined and
    # the GPU iterates equal the oracle's (four roundings per iteration, the
    # last one of E - S^H eps^)
    from paper_2512_07811_amd import operands as P
    L = 3
    k = I.random_boxes(L, 7, edge_min=2, edge_max=5, k_min=2.0, k_max=6.0)
    k0 = (k.min() + k.max()) / 2
    E = np.array([1.0, 0.0, 0.0])
    prob = P.build_problem(kvox=k, k0=k0)
    ops, e = P.upload(prob, [E], max_rank=16)
    e = q.DeviceTT.from_cores([O.mean_field_tt(E, L)], e.cap)
    oprob = ls_tt.Problem(k, k0)
    E_tt = O.mean_field_tt(E, L)
    ref = O.mean_field_tt(E, L)
    for m in range(3):
        res = q.ls_iterate(ctx, ops, e, q.solve_opts(1e-8, 16), 1).cpu().numpy()
        ref, r = ls_tt.ls_iterate(ref, oprob.kp, oprob.S, oprob.G, oprob.Sinv, E_tt, E, 1e-8, 16)
        assert max(T.ranks(ref)) == 16
        assert rel(T.full(e.to_cores()[0]), T.full(ref)) < 1e-10
        assert abs(res[0, 0] - r) < 1e-9 * r


def test_homogenize_laminate_closed_form(q, ctx):
    from paper_2512_07811_amd import operands as P
    k = I.laminate(5)
    prob = P.build_problem(kvox=k, k0=5.5)
    ops, e = P.upload(prob, [[1, 0, 0], [0, 1, 0]], max_rank=64)
    A, its, res, st = q.homogenize(ctx, ops, e, q.solve_opts(1e-10, 64, tol=1e-8, max_iter=200))
    assert st == q.QT_OK
    assert abs(A[0, 0] - 20.0 / 11.0) < 1e-10 * (20.0 / 11.0)
    assert abs(A[1, 1] - 5.5) < 1e-10 * 5.5
    assert np.all(np.abs(A[0, 1:]) < 1e-10) and abs(A[1, 0]) < 1e-10 and abs(A[1, 2]) < 1e-10
    assert its[0] <= 3 and its[1] <= 2


def test_homogenize_boxes_matches_oracle_tt(q, ctx):
    from paper_2512_07811_amd import operands as P
    L = 3
    k = I.random_boxes(L, 5, edge_min=2, edge_max=5, k_min=2.0, k_max=6.0)
    k0 = (k.min() + k.max()) / 2
    prob = P.build_problem(kvox=k, k0=k0)
    ops, e = P.upload(prob, [[1, 0, 0]], max_rank=0)
    A, its, res, st = q.homogenize(ctx, ops, e, q.solve_opts(1e-6, 0, tol=1e-9, max_iter=300))
    oprob = ls_tt.Problem(k, k0)
    A_ref, its_ref = ls_tt.effective_tensor(oprob, [0], eps=1e-6, tol=1e-9, max_iter=300)
    assert abs(its[0] - its_ref[0]) <= 1
    assert np.max(np.abs(A[0] - A_ref[:, 0])) < 1e-8 * abs(A_ref[0, 0])


@pytest.mark.parametrize("mode", ["svd", "sketch"])
def test_jacobi_converges_on_symmetric_cell(q, ctx, mode):
    # A centred sphere's fields have bond spectra with (nearly) repeated singular
    # values from the cube symmetries.  One-sided Jacobi must converge on them:
    # the rotation of a pair with almost equal norms depends on the sign of a
    # cancelling difference, which every lane of a pair must evaluate alike.
    from paper_2512_07811_amd import operands as P
    kvox = I.sphere(4, 0.2, k_in=10.0, k_out=1.0)
    prob = P.build_problem(kvox=kvox, k0=5.5)
    ops, e = P.upload(prob, [[1.0, 0.0, 0.0]], 64)
    m = q.ROUND_SVD if mode == "svd" else q.ROUND_SKETCH
    ctx.counters(reset=True)
    A, its, res, st = q.homogenize(ctx, ops, e, q.solve_opts(1e-8, 64, tol=1e-7, max_iter=4,
                                                             mode=m, oversample=4, seed=3))
    cnt = ctx.counters(reset=True)
    assert cnt["svd_calls"] > 0
    assert cnt["svd_sweeps"] / cnt["svd_calls"] < 16
