"""Linear elasticity (Voigt strain field, 6 x 6 component cores) on the GPU.

With eps = 0 and no rank cap the TT iterates are the dense Moulinec-Suquet
iterates of the oracle (materializing SVD mode and product-aware sketch mode,
within 1e-10); a laminate's effective stiffness matches its closed form (sketch
and learned-rank paths), and a random cell's matches the dense oracle's.
"""
import numpy as np
import pytest

from oracle import ms_elastic as ME
from oracle import tt as T

pytestmark = pytest.mark.gpu

LOADS6 = [list(np.eye(6)[j]) for j in range(6)]


@pytest.fixture(scope="module")
def q():
    from paper_2512_07811_amd import qtt
    return qtt


@pytest.fixture(scope="module")
def ctx(q):
    c = q.Context(0)
    yield c
    c.close()


def _cell(L, seed):
    g = np.random.default_rng(seed)
    N = 2 ** L
    ph = g.random((N, N, N)) < 0.4
    return np.where(ph, 6.0, 2.0), np.where(ph, 3.0, 1.0)


def _laminate(L, lams=(2.0, 6.0), mus=(1.0, 3.0), layers=4):
    N = 2 ** L
    lam = np.zeros((N, N, N))
    mu = np.zeros((N, N, N))
    w = N // layers
    for i in range(layers):
        lam[i * w:(i + 1) * w] = lams[i % 2]
        mu[i * w:(i + 1) * w] = mus[i % 2]
    return lam, mu


# the materializing SVD mode forms the products: at 8^3 with six components
# the first one's SVD blocks exceed 1024 columns, so it runs at 4^3 only
@pytest.mark.parametrize("mode,L,geom", [("svd", 2, "random"), ("sketch", 2, "random"),
                                         ("sketch", 3, "laminate"), ("sketch", 3, "random")])
def test_elastic_iterates_match_dense_oracle(q, ctx, mode, L, geom):
    from paper_2512_07811_amd import operands as P
    lam, mu = _cell(L, 7) if geom == "random" else _laminate(L)
    prob = P.build_problem_elastic(lam, mu, op_eps=1e-14, green_eps=1e-14)
    loads = [LOADS6[0], LOADS6[5]]
    ops, e = P.upload(prob, loads, 0)
    e = q.DeviceTT.from_cores([P.mean_field(np.asarray(E), L) for E in loads], e.cap)
    md = q.ROUND_SVD if mode == "svd" else q.ROUND_SKETCH
    opts = q.solve_opts(0.0, 0, mode=md, oversample=8, seed=3)
    N = 2 ** L
    dense = [np.zeros((6, N, N, N)) + np.asarray(E).reshape(6, 1, 1, 1) for E in loads]
    for it in range(3):
        q.ls_iterate(ctx, ops, e, opts, 1)
        ctx.sync()
        got = e.to_cores()
        for b, E in enumerate(loads):
            dense[b] = ME.ms_step(dense[b], lam, mu, prob["lam0"], prob["mu0"], E)
            g = T.full(got[b]).reshape(6, N, N, N)
            err = np.linalg.norm(g - dense[b]) / np.linalg.norm(dense[b])
            print(f"[elastic] {mode} L={L} {geom} iterate {it + 1} load {b}: {err:.2e}", flush=True)
            assert err < 1e-10


@pytest.mark.parametrize("mode", ["sketch", "learned"])
def test_elastic_laminate_stiffness_matches_closed_form(q, ctx, mode):
    import torch

    from paper_2512_07811_amd import inputs as I
    from paper_2512_07811_amd import learned
    from paper_2512_07811_amd import operands as P
    L = 4
    lam, mu = _laminate(L)
    prob = P.build_problem_elastic(lam, mu, op_eps=1e-12, green_eps=1e-13)
    ops, e = P.upload(prob, LOADS6, 64)
    md = q.ROUND_SKETCH if mode == "sketch" else q.ROUND_LEARNED
    if md == q.ROUND_LEARNED:
        n_cls = learned.n_classes(64)
        params = torch.from_numpy(learned.flat_params(I.mlp_init(q.RANK_FEATURES, n_cls, 2))).cuda()
        q.set_predictor(ctx, params, n_cls, 0.9, 1.0)
    opts = q.solve_opts(1e-10, 64, tol=1e-10, max_iter=400, mode=md, oversample=8, seed=5)
    A, its, res, st = q.homogenize(ctx, ops, e, opts)
    C = A.T                                   # column j: mean stress of load e_j
    ref = ME.laminate_closed_form([2.0, 6.0], [1.0, 3.0], [0.5, 0.5])
    err = np.abs(C - ref).max() / np.abs(ref).max()
    print(f"[elastic] laminate {mode}: iterations {its.tolist()}, max rel diff {err:.2e}",
          flush=True)
    assert st == q.QT_OK
    assert err < 1e-8
    assert np.abs(C - C.T).max() < 1e-8 * np.abs(ref).max()


def test_elastic_random_cell_stiffness_matches_dense_oracle(q, ctx):
    # 8^3 two-phase cell, six unit strains in one batch, solved to 1e-10:
    # the effective stiffness against the dense oracle's to 1e-8
    from paper_2512_07811_amd import operands as P
    L = 3
    lam, mu = _cell(L, 9)
    prob = P.build_problem_elastic(lam, mu, op_eps=1e-12, green_eps=1e-13)
    ops, e = P.upload(prob, LOADS6, 0)
    opts = q.solve_opts(1e-11, 0, tol=1e-11, max_iter=600, mode=q.ROUND_SKETCH, oversample=8,
                        seed=7)
    A, its, res, st = q.homogenize(ctx, ops, e, opts)
    ref = ME.effective_tensor(lam, mu, prob["lam0"], prob["mu0"], tol=1e-12, max_iter=3000)
    err = np.abs(A.T - ref).max() / np.abs(ref).max()
    print(f"[elastic] random 8^3: iterations {its.tolist()}, max rel diff {err:.2e}", flush=True)
    assert st == q.QT_OK
    assert err < 1e-8
