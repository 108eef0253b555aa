"""Mixed precision (QT_PREC_F32): FP32-MFMA range finder, FP64 projection.

The contractions that only choose the bases (right sketches and sketched
products) run on v_mfma_f32_16x16x4f32; the projection, QR/SVD and the error
bookkeeping stay FP64.  What must hold whatever the FP32 noise:
  * the returned train is an exact orthogonal projection of the product, so
    the fixed-rank rounding's reported error equals the oracle's dense error
    of the returned train (squared, to 2e-14), and its cores are orthonormal;
  * with SVD truncation, ||x - x~|| <= eps ||x|| and the reported error
    bounds the dense one.
What FP32 costs (measured here, and guarded with about 2x margin; the FP32
bases tilt by the FP32 rounding of the sketched products, amplified by the
spread of the singular values, so no sharper a-priori bound is claimed):
against the FP64 oracle's RTO with the same Gaussians, a full-width sketch
(exact in FP64, errors of 1e-13) misses 7.5e-6 to 1.1e-4 of ||x|| (guard
3e-4), and truncating sketches change the error in the fourth digit; at the
solver level, after 30 iterations on a 16^3 cell the A_eff of the mixed path
differs from the FP64 path's by 1.2e-5 to 1.8e-4 relative at eps 1e-4 and
1e-6 (guard 1e-3), and its residual stalls near 1e-2 where the FP64 path's
reaches 1.4e-5: the mode is for tolerances of about 1e-3 and above (the
paper computes in complex64 throughout).
"""
import math

import numpy as np
import pytest

from oracle import sketch as SK
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


def natural(m):
    n = len(m)
    return [1] + [int(min(np.prod(m[:k]), np.prod(m[k:]))) for k in range(1, n)] + [1]


def operators(modes, seed):
    n = len(modes)
    rf = [1] + [[2, 3, 2, 3, 3, 2, 2, 3][(k - 1) % 8] for k in range(1, n)] + [1]
    rd = [1] + [[2, 3, 4, 3, 3, 2, 2, 3][(k - 1) % 8] for k in range(1, n)] + [1]
    return I.random_mpo(modes, modes, rf, seed), I.random_tt(modes, rd, seed + 1)


@pytest.mark.parametrize("kind", ["diag", "full"])
@pytest.mark.parametrize("ell_max", [3, 6, 64])
def test_mixed_fixed_rank_sketch_is_an_exact_projection(q, ctx, kind, ell_max):
    import torch
    modes = [3, 2, 2, 2, 2, 2, 2, 2]
    full, dcores = operators(modes, 80)
    ys = [I.random_tt(modes, [1, 3, 4, 5, 5, 4, 3, 2, 1], seed=81 + b) for b in range(2)]
    if kind == "diag":
        Ad, Ao = q.DeviceMPO.from_cores(dcores, [1] * len(modes)), T.diag_lift(dcores)
    else:
        Ad, Ao = q.DeviceMPO.from_cores(full), full
    nat = natural(modes)
    prod = [a.shape[0] * b for a, b in zip(Ao, [1, 3, 4, 5, 5, 4, 3, 2])] + [1]
    ells = [1] + [min(nat[k], prod[k], ell_max) for k in range(1, len(modes))] + [1]
    om = I.gaussian_sketch(modes, ells, seed=82)
    Om = q.DeviceTT.from_cores([om], ells)
    Y = q.DeviceTT.from_cores(ys, [1] + [6] * (len(modes) - 1) + [1])
    out = q.DeviceTT.empty(modes, ells, 2)
    xs = [T.mpo_apply(Ao, y) for y in ys]
    xn2 = torch.tensor([np.real(T.dot(x, x)) for x in xs], dtype=torch.float64, device="cuda")
    err, _ = q.tt_sketch_round(ctx, Ad, Y, xn2, out, omega=Om, eps=1e-3, mode=q.ROUND_LEARNED,
                               precision=q.PREC_F32)
    got = out.to_cores()
    err = err.cpu().numpy()
    for b in range(2):
        X = T.full(xs[b])
        nx = np.linalg.norm(X)
        true = np.linalg.norm(X - T.full(got[b])) / nx
        ref = SK.rto(xs[b], om)
        e64 = np.linalg.norm(X - T.full(ref)) / nx
        print(f"[mixed] {kind} l<={ell_max} field {b}: reported {err[b]:.3e} dense {true:.3e} "
              f"FP64 RTO {e64:.3e}", flush=True)
        assert abs(err[b] ** 2 - true ** 2) <= 2e-14 + 1e-6 * true ** 2
        assert T.ranks(got[b]) == T.ranks(ref)
        for c in got[b][:-1]:
            assert np.allclose(T.left_gram(c), np.eye(c.shape[2]), atol=1e-12)
        assert abs(true - e64) <= 3e-4


def test_mixed_sketch_svd_round_keeps_eps(q, ctx):
    import torch
    modes = [3] + [2] * 8
    dcores = I.random_tt(modes, [1, 3, 4, 4, 4, 3, 3, 2, 2, 1], seed=90)
    ys = [I.graded_tt(modes, [1, 3, 5, 6, 6, 6, 5, 4, 2, 1], decay=0.5, seed=91 + b)
          for b in range(2)]
    Ad = q.DeviceMPO.from_cores(dcores, [1] * len(modes))
    Ao = T.diag_lift(dcores)
    nat = natural(modes)
    ells = [1] + [min(nat[k], 24) for k in range(1, len(modes))] + [1]
    om = I.gaussian_sketch(modes, ells, seed=92)
    Om = q.DeviceTT.from_cores([om], ells)
    Y = q.DeviceTT.from_cores(ys)
    out = q.DeviceTT.empty(modes, ells, 2)
    xs = [T.mpo_apply(Ao, y) for y in ys]
    xn2 = torch.tensor([np.real(T.dot(x, x)) for x in xs], dtype=torch.float64, device="cuda")
    eps = 1e-4
    err, fail = q.tt_sketch_round(ctx, Ad, Y, xn2, out, omega=Om, eps=eps, mode=q.ROUND_SKETCH,
                                  precision=q.PREC_F32)
    got = out.to_cores()
    err = err.cpu().numpy()
    assert np.all(fail.cpu().numpy() == 0)
    for b in range(2):
        X = T.full(xs[b])
        true = np.linalg.norm(T.full(got[b]) - X) / np.linalg.norm(X)
        ref, _ = SK.sketch_round(xs[b], om, eps, xnorm=math.sqrt(np.real(T.dot(xs[b], xs[b]))))
        print(f"[mixed] svd-truncated field {b}: reported {err[b]:.3e} dense {true:.3e} ranks "
              f"{T.ranks(got[b])} FP64 {T.ranks(ref)}", flush=True)
        assert true <= eps * (1 + 1e-9)
        assert true <= err[b] * (1 + 1e-9) + 1e-12
        assert err[b] <= eps * (1 + 1e-9)


def test_precision_f32_is_refused_where_it_does_not_apply(q, ctx):
    x = q.DeviceTT.from_cores([I.random_tt([2, 2, 2], [1, 2, 2, 1], seed=3)])
    with pytest.raises(q.QtError):
        q.tt_round(ctx, x, 1e-6, precision=q.PREC_F32)


@pytest.mark.parametrize("eps", [1e-4, 1e-6])
@pytest.mark.parametrize("mode", ["sketch", "learned"])
def test_mixed_iterates_track_fp64(q, eps, mode):
    # 30 iterations from E on a 16^3 sphere cell (k = 10 in 1, k0 = 5.5,
    # contraction 0.82, no rank cap) in each precision, then A_eff of both end
    # fields
    import torch

    from paper_2512_07811_amd import learned
    from paper_2512_07811_amd import operands as P
    rmax, L, iters = 64, 4, 30
    prob = P.build_problem(kvox=I.sphere(L, 0.25, 10.0, 1.0), k0=5.5)
    loads = [[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]]
    md = q.ROUND_SKETCH if mode == "sketch" else q.ROUND_LEARNED
    ctx = q.Context(0)
    try:
        if md == q.ROUND_LEARNED:
            n_cls = learned.n_classes(rmax)
            params = torch.from_numpy(learned.flat_params(
                I.mlp_init(q.RANK_FEATURES, n_cls, 2))).cuda()
            q.set_predictor(ctx, params, n_cls, 0.9, 1.0)
        res = {}
        for prec in (q.PREC_F64, q.PREC_F32):
            ops, e = P.upload(prob, loads, rmax)
            e = q.DeviceTT.from_cores([P.mean_field(np.asarray(E), L) for E in loads], e.cap)
            q.learn_reset(ctx)
            opts = q.solve_opts(eps, rmax, mode=md, oversample=4, seed=5, precision=prec)
            r = q.ls_iterate(ctx, ops, e, opts, iters).cpu().numpy()
            A = np.stack([q.tt_dot(ctx, ops.k_sel[c], e).cpu().numpy().real / 2.0 ** (3 * L)
                          for c in range(3)], axis=1)
            res[prec] = (A, r[-1])
        (A64, r64), (A32, r32) = res[q.PREC_F64], res[q.PREC_F32]
        gap = np.abs(np.diag(A32) - np.diag(A64)) / np.abs(np.diag(A64))
        print(f"[mixed] {mode} eps {eps}: A_eff FP64 {np.diag(A64)} mixed {np.diag(A32)} rel gap "
              f"{gap}  last residuals {r64} / {r32}", flush=True)
        assert np.all(gap <= 1e-3)
    finally:
        ctx.close()
