"""The error a product-aware rounding reports is the true error of what it returns.

Each of the four roundings of a sketch-mode iteration (Algorithm 2 as the
solver runs it) reports sqrt(||x||^2 - ||x~||^2)/||x||, with ||x||^2 taken from
an identity of the operator (<e, K2 e>, ||S t|| = ||t||, <t, G t>/k0, the
environments of S E - eps^) and ||x~||^2 from its own output.  Here the oracle
materializes every product x from the same (set-up) operator trains, forms the
dense x and x~ (16^3 cell) and computes ||x - x~|| / ||x|| directly, both
where every rounding meets eps = 1e-6 and where a rank cap of 6 binds (errors
of 1e-1).  Fixed-rank (learned) mode: the reported error is the projection's
and the squared errors agree to 2e-14 (the floor of the norm identities, far
below eps^2 = 1e-12).  SVD-truncated mode: the reported value
(e_s + sqrt(tails^2)) / ||x|| bounds the true error (the truncation of
interior bonds is not orthogonal to the projection error) and is within 2x
of it.
"""
import numpy as np
import pytest

from oracle import tt as T
from paper_2512_07811_amd import inputs as I

import sketch_chain as SC

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    from paper_2512_07811_amd import qtt
    return qtt


@pytest.fixture(scope="module")
def cell():
    from paper_2512_07811_amd import operands as P
    L, k0 = 4, 50.5
    kvox = I.sphere(L, 0.2, 100.0, 1.0)
    return L, k0, P.build_problem(kvox=kvox, k0=k0)


def _full_op(cores, diag):
    return [c if not d else T.diag_lift([c])[0] for c, d in zip(cores, diag)]


@pytest.mark.parametrize("rmax", [0, 6])
@pytest.mark.parametrize("mode", ["sketch", "learned"])
def test_reported_rounding_errors_equal_dense_errors(q, cell, rmax, mode):
    from paper_2512_07811_amd import operands as P
    L, k0, prob = cell
    eps, os_ = 1e-6, 4
    n = 3 * L + 1
    E = [1.0, 0.0, 0.0]
    md = q.ROUND_SKETCH if mode == "sketch" else q.ROUND_LEARNED
    ctx = q.Context(0)
    try:
        ops, e = P.upload(prob, [E], rmax)
        e = q.DeviceTT.from_cores([P.mean_field(np.asarray(E), L)], e.cap)
        # a nontrivial field: two SVD-truncated iterations
        q.ls_iterate(ctx, ops, e, q.solve_opts(eps, rmax, mode=q.ROUND_SKETCH, oversample=os_,
                                               seed=5), 2)
        ctx.sync()
        modes = list(e.modes)
        wide = SC._cap(modes, (rmax if rmax else 10 ** 6) + os_)
        # a fixed-rank (learned) rounding keeps its sketch ranks (up to rmax + os)
        field = wide if mode == "learned" else SC._cap(modes, rmax if rmax else 10 ** 6)
        Kp = prob["kp"]
        S, Sinv = prob["S"], prob["Sinv"]
        G = _full_op(prob["G"], [0] + [1] * (n - 1))
        worst = 0.0
        y = e
        for s in range(4):
            yc = y.to_cores()[0]
            if s == 0:
                x = T.hadamard(Kp, yc)
                xn2 = q.tt_sandwich(ctx, ops.K2, y, 1.0)
                A = ops.Kp
            elif s == 1:
                x = T.mpo_apply(S, yc)
                xn2 = q.tt_dot(ctx, y, y).real.contiguous()
                A = ops.S
            elif s == 2:
                x = T.mpo_apply(G, yc)
                xn2 = q.tt_sandwich(ctx, ops.G, y, 1.0 / k0)
                A = ops.G
            else:
                x = T.mpo_apply(Sinv, yc)
                xn2 = q.tt_dot(ctx, y, y).real.contiguous()
                A = ops.Sinv
            out = q.DeviceTT.empty(modes, wide, 1)
            err, _ = q.tt_sketch_round(ctx, A, y, xn2, out, eps=eps, max_rank=rmax, mode=md,
                                       oversample=os_, seed=61 + s)
            ctx.sync()
            xd = T.full(x).reshape(-1)
            xt = T.full(out.to_cores()[0]).reshape(-1)
            nx2 = float(np.vdot(xd, xd).real)
            true2 = float(np.vdot(xd - xt, xd - xt).real) / nx2
            rep2 = float(err.cpu().numpy()[0]) ** 2
            print(f"[aposteriori] {mode} rmax {rmax} step {s}: reported {np.sqrt(rep2):.3e} "
                  f"true {np.sqrt(true2):.3e}  ||x||^2 identity rel diff "
                  f"{abs(float(xn2.cpu().numpy()[0]) - nx2) / nx2:.1e}", flush=True)
            if mode == "learned":
                # fixed rank: the reported error is the projection's, exact
                assert abs(rep2 - true2) <= 2e-14 + 1e-6 * true2
            else:
                # sketch + truncation: a rigorous bound, and not a loose one
                assert true2 <= rep2 * (1 + 1e-9) + 2e-14
                assert rep2 <= 4.0 * true2 + 2e-14
            if rmax == 0 and mode == "sketch":
                assert true2 <= (eps * (1 + 1e-6)) ** 2 + 2e-14
            worst = max(worst, true2)
            y = SC._view(out, field)
            if s == 2:
                y = q.tt_add(ctx, 1.0, ops.SE, -1.0, y)
        if rmax:
            assert worst > 1e-6          # the cap binds
    finally:
        ctx.close()
