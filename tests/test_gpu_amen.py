"""AMEn product (tt_amen_mv) against the oracle (oracle/amen.py) and the dense product.

With the same initial guess and residual guess the GPU sweeps take the
oracle's steps: the same ranks and results within 1e-10 where the rounding
has no ties (eps far below or above the spectrum), for full and diagonal
operator cores, batches, growth from a rank-1 start by enrichment, the rank
cap, and the Green operator applied to a polarization field of the LS scheme.
"""
import numpy as np
import pytest

from oracle import amen as AM
from oracle import tt as T
from paper_2512_07811_amd import inputs as I

pytestmark = pytest.mark.gpu

MODES = [3] + [2] * 7


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
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _caps(modes, rmax):
    n = len(modes)
    cap = [1]
    left = 1
    for k in range(n - 1):
        left *= modes[k]
        right = int(np.prod(modes[k + 1:]))
        cap.append(min(left, right, rmax))
    return cap + [1]


def _run(q, ctx, A, x_list, y0_list, z0_list, eps, rmax, sweeps, diag=None, ycap=16):
    Ad = q.DeviceMPO.from_cores(A, diag_flags=diag)
    X = q.DeviceTT.from_cores(x_list)
    Y = q.DeviceTT.from_cores(y0_list, cap=_caps(MODES, ycap))
    Z = q.DeviceTT.from_cores(z0_list)
    err = q.tt_amen_mv(ctx, Ad, X, Y, Z, eps, rmax, sweeps)
    ctx.sync()
    return Y.to_cores(), err.cpu().numpy()


def test_amen_full_operator_matches_oracle(q, ctx):
    x = I.random_tt(MODES, [1, 3, 4, 4, 4, 4, 4, 2, 1], seed=1)
    A = I.random_mpo(MODES, MODES, [1, 2, 3, 3, 3, 3, 3, 2, 1], seed=2)
    y0 = I.random_tt(MODES, [1, 3, 6, 12, 12, 8, 4, 2, 1], seed=3)
    z0 = I.random_tt(MODES, [1, 3, 4, 4, 4, 4, 4, 2, 1], seed=4)
    got, err = _run(q, ctx, A, [x], [y0], [z0], 1e-13, 0, 2)
    ref = AM.amen_mv(A, x, y0, z0, 1e-13, sweeps=2)
    dense = T.full(T.mpo_apply(A, x))
    print(f"[amen] full: ranks {T.ranks(got[0])} oracle {T.ranks(ref)}, "
          f"vs oracle {rel(T.full(got[0]), T.full(ref)):.2e}, vs product "
          f"{rel(T.full(got[0]), dense):.2e}", flush=True)
    assert T.ranks(got[0]) == T.ranks(ref)
    assert rel(T.full(got[0]), T.full(ref)) < 1e-10
    assert rel(T.full(got[0]), dense) < 1e-11


def test_amen_diagonal_operator_and_batch(q, ctx):
    # the Hadamard product through the diagonal lift, three instances
    k = I.random_tt(MODES, [1, 2, 2, 2, 2, 2, 2, 2, 1], seed=21, is_complex=False)
    xs = [I.random_tt(MODES, [1, 3, 3, 3, 3, 3, 3, 2, 1], seed=22 + b) for b in range(3)]
    y0 = [I.random_tt(MODES, [1, 3, 6, 8, 8, 8, 4, 2, 1], seed=30 + b) for b in range(3)]
    z0 = [I.random_tt(MODES, [1, 3, 4, 4, 4, 4, 4, 2, 1], seed=40 + b) for b in range(3)]
    kc = [c.astype(np.complex128) for c in k]
    got, _ = _run(q, ctx, kc, xs, y0, z0, 1e-13, 0, 2, diag=[1] * len(MODES))
    for b in range(3):
        ref = AM.amen_mv(T.diag_lift(kc), xs[b], y0[b], z0[b], 1e-13, sweeps=2)
        print(f"[amen] diag instance {b}: vs oracle {rel(T.full(got[b]), T.full(ref)):.2e}",
              flush=True)
        assert T.ranks(got[b]) == T.ranks(ref)
        assert rel(T.full(got[b]), T.full(ref)) < 1e-10
        assert rel(T.full(got[b]), T.full(k) * T.full(xs[b])) < 1e-11


def test_amen_enrichment_from_rank_one(q, ctx):
    x = I.random_tt(MODES, [1, 3, 4, 4, 4, 4, 4, 2, 1], seed=5)
    A = I.random_mpo(MODES, MODES, [1, 2, 3, 3, 3, 3, 3, 2, 1], seed=6)
    y0 = I.random_tt(MODES, [1] * 9, seed=7)
    z0 = I.random_tt(MODES, [1, 3, 4, 4, 4, 4, 4, 2, 1], seed=8)
    dense = T.full(T.mpo_apply(A, x))
    for sw in (1, 5):
        got, _ = _run(q, ctx, A, [x], [y0], [z0], 1e-13, 0, sw)
        ref = AM.amen_mv(A, x, y0, z0, 1e-13, sweeps=sw)
        e_gpu, e_ref = rel(T.full(got[0]), dense), rel(T.full(ref), dense)
        print(f"[amen] rank-1 start, {sw} sweeps: error {e_gpu:.2e} (oracle {e_ref:.2e}), "
              f"ranks {T.ranks(got[0])}", flush=True)
        assert T.ranks(got[0]) == T.ranks(ref)
        assert abs(e_gpu - e_ref) <= 1e-8 * max(e_ref, 1e-3) + 1e-11
    assert e_gpu < 1e-11


def test_amen_rank_cap(q, ctx):
    x = I.random_tt(MODES, [1, 3, 4, 4, 4, 4, 4, 2, 1], seed=41)
    A = I.random_mpo(MODES, MODES, [1, 2, 3, 3, 3, 3, 3, 2, 1], seed=42)
    y0 = I.random_tt(MODES, [1, 3, 5, 5, 5, 5, 4, 2, 1], seed=43)
    z0 = I.random_tt(MODES, [1, 3, 4, 4, 4, 4, 4, 2, 1], seed=44)
    got, err = _run(q, ctx, A, [x], [y0], [z0], 1e-13, 5, 3, ycap=5)
    ref = AM.amen_mv(A, x, y0, z0, 1e-13, rmax=5, sweeps=3)
    dense = T.full(T.mpo_apply(A, x))
    print(f"[amen] cap 5: error {rel(T.full(got[0]), dense):.4e} oracle "
          f"{rel(T.full(ref), dense):.4e}, reported rounding error {err[0]:.3e}", flush=True)
    assert max(T.ranks(got[0])) <= 5
    assert rel(T.full(got[0]), T.full(ref)) < 1e-8


def test_amen_green_multiply_of_a_polarization(q, ctx):
    # Algorithm 2's Green step on an 8^3 two-phase cell: tau^ = S (k' e) for the
    # mean field e, eps^ = A(G, tau^) from a random rank-16 guess (the product
    # has rank 28 at 1e-10) with an enrichment of rank 8
    from paper_2512_07811_amd import operands as P
    L = 3
    g = np.random.default_rng(3)
    kvox = np.where(g.random((8, 8, 8)) < 0.3, 10.0, 1.0)
    prob = P.build_problem(kvox=kvox, k0=5.5)
    e = P.mean_field(np.array([1.0, 0.0, 0.0]), L)
    tau = T.round_tt(T.mpo_apply(prob["S"], T.round_tt(T.hadamard(prob["kp"], e), 1e-12)),
                     1e-12)
    G = prob["G"]
    n = len(G)
    modes = [3] + [2] * (3 * L)
    nat = [min(3 * 2 ** k, 2 ** (3 * L - k)) for k in range(n - 1)]
    y0 = I.random_tt(modes, [1] + [min(16, r) for r in nat] + [1], seed=8)
    z0 = I.random_tt(modes, [1] + [min(8, r) for r in nat] + [1], seed=9)
    Ad = q.DeviceMPO.from_cores(G, diag_flags=[0] + [1] * (3 * L))
    X = q.DeviceTT.from_cores([tau])
    Y = q.DeviceTT.from_cores([y0], cap=[1] + [min(64, r) for r in nat] + [1])
    Z = q.DeviceTT.from_cores([z0])
    q.tt_amen_mv(ctx, Ad, X, Y, Z, 1e-10, 0, 3)
    ctx.sync()
    got = Y.to_cores()[0]
    Gop = [G[0]] + T.diag_lift(G[1:])
    ref = AM.amen_mv(Gop, tau, y0, z0, 1e-10, sweeps=3)
    exact = T.full(T.mpo_apply(Gop, tau))
    e_gpu, e_ref = rel(T.full(got), exact), rel(T.full(ref), exact)
    print(f"[amen] Green step: ranks {T.ranks(got)} oracle {T.ranks(ref)}, vs exact "
          f"{e_gpu:.2e} (oracle {e_ref:.2e})", flush=True)
    assert T.ranks(got) == T.ranks(ref)
    assert abs(e_gpu - e_ref) <= 1e-6 * e_ref + 1e-10
    assert rel(T.full(got), T.full(ref)) < 1e-8
