"""Learned-rank rounding: MLP kernels against the FP64 oracle MLP, rank logs,
the a-posteriori acceptance with SVD fallback, and what the trained network
gains over the product-aware rounding without it.

MLP tolerances: the kernels run in FP32 (unit roundoff 6e-8) on sums of at
most 64 terms per layer and 200 samples, so losses and gradients are compared
at 1e-4 relative (norm-wise) to the FP64 oracle; an Adam update applied to the
kernel's own gradient is compared at 1e-5 of the learning rate.
"""
import numpy as np
import pytest

from oracle import mlp as M
from oracle import ms
from paper_2512_07811_amd import inputs as I

pytestmark = pytest.mark.gpu

F, C = 24, 8


@pytest.fixture(scope="module")
def q():
    from paper_2512_07811_amd import qtt
    return qtt


@pytest.fixture(scope="module")
def ctx(q):
    c = q.Context(0)
    yield c
    c.close()


def as_dict(layers):
    P = {}
    for i in range(len(layers) // 2):
        P[f"W{i}"] = np.asarray(layers[2 * i], dtype=np.float64)
        P[f"b{i}"] = np.asarray(layers[2 * i + 1], dtype=np.float64)
    return P


def unflatten(flat, n_in=F, n_cls=C):
    dims = [n_in, 64, 64, 64, n_cls]
    out, o = [], 0
    for i in range(4):
        w = dims[i] * dims[i + 1]
        out.append(flat[o:o + w].reshape(dims[i], dims[i + 1]))
        o += w
        out.append(flat[o:o + dims[i + 1]])
        o += dims[i + 1]
    assert o == flat.size
    return out


def data(n, seed):
    g = I.rng(seed)
    X = g.uniform(-1.0, 0.2, size=(n, F)).astype(np.float32)
    Y = g.integers(0, C, size=n).astype(np.int32)
    return X, Y


def f32_layers(seed):
    return [a.astype(np.float32) for a in I.mlp_init(F, C, seed)]


@pytest.mark.parametrize("n", [1, 64, 200])
def test_mlp_loss_and_gradient_match_oracle(q, ctx, n):
    import torch

    from paper_2512_07811_amd import learned
    layers = f32_layers(3)
    X, Y = data(n, 4 + n)
    P = torch.from_numpy(learned.flat_params(layers)).cuda()
    Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    grad = torch.zeros_like(P)
    q.mlp_train_step(ctx, P, None, None, 1, Xd, Yd, C, 0.0, 1.0, 2.0, loss=loss, grad=grad)
    ctx.sync()
    lref, Gref = M.loss_and_grad(as_dict(layers), X.astype(np.float64), Y, beta=1.0, gamma=2.0)
    assert abs(loss.item() - lref) < 1e-4 * abs(lref)
    g = unflatten(grad.cpu().numpy().astype(np.float64))
    for i in range(4):
        for key, got in ((f"W{i}", g[2 * i]), (f"b{i}", g[2 * i + 1])):
            ref = Gref[key]
            scale = max(np.linalg.norm(ref), 1e-12)
            assert np.linalg.norm(got - ref) < 1e-4 * scale, key
    # lr = 0 leaves the parameters untouched
    assert np.array_equal(P.cpu().numpy(), learned.flat_params(layers))


def test_mlp_adam_update_matches_oracle(q, ctx):
    import torch

    from paper_2512_07811_amd import learned
    layers = f32_layers(5)
    X, Y = data(150, 6)
    flat0 = learned.flat_params(layers)
    P = torch.from_numpy(flat0.copy()).cuda()
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    grad = torch.zeros_like(P)
    lr = 1e-2
    Pref = as_dict(layers)
    mref, vref = M.adam_init(Pref)
    for t in range(1, 4):
        before = P.cpu().numpy().astype(np.float64)
        q.mlp_train_step(ctx, P, m, v, t, Xd, Yd, C, lr, 1.0, 2.0, grad=grad)
        ctx.sync()
        # Adam on the kernel's own gradient, in FP64 from the kernel's parameters
        Pk = as_dict(unflatten(before))
        Gk = as_dict(unflatten(grad.cpu().numpy().astype(np.float64)))
        M.adam_step(Pk, Gk, mref, vref, t, lr=lr)
        got = as_dict(unflatten(P.cpu().numpy().astype(np.float64)))
        for key in Pk:
            assert np.max(np.abs(got[key] - Pk[key])) < 1e-5 * lr * 10, (t, key)
        # and the kernel's gradient is the oracle gradient at those parameters
        _, Gref = M.loss_and_grad(as_dict(unflatten(before)), X.astype(np.float64), Y)
        for key in Gref:
            assert np.linalg.norm(Gk[key] - Gref[key]) < 1e-4 * max(np.linalg.norm(Gref[key]),
                                                                     1e-12)


def test_mlp_inference_matches_oracle(q, ctx):
    import torch

    from paper_2512_07811_amd import learned
    layers = f32_layers(7)
    X, _ = data(300, 8)
    P = torch.from_numpy(learned.flat_params(layers)).cuda()
    cap = torch.from_numpy(I.rng(9).integers(1, 70, size=300).astype(np.int32)).cuda()
    logits, ranks = q.mlp_infer(ctx, P, torch.from_numpy(X).cuda(), C, 0.8, cap)
    ctx.sync()
    Pd = as_dict(layers)
    z, _ = M.forward(Pd, X.astype(np.float64))
    assert np.max(np.abs(logits.cpu().numpy() - z)) < 1e-4 * max(np.max(np.abs(z)), 1.0)
    cls = M.predict_class(Pd, X.astype(np.float64), 0.8)
    cdf = np.cumsum(M.softmax(z), axis=1)
    clear = np.all(np.abs(cdf - 0.8) > 1e-4, axis=1)     # class decided away from the boundary
    want = np.maximum(np.minimum(8 * (cls + 1), cap.cpu().numpy()), 1)
    got = ranks.cpu().numpy()
    assert clear.sum() > 250
    assert np.array_equal(got[clear], want[clear])


def test_mlp_training_fits_a_rule(q, ctx):
    # labels given by a rule of the features: full-batch training on the device
    # drives the loss down and reproduces the rule on most samples
    import torch

    from paper_2512_07811_amd import learned
    g = I.rng(11)
    X = g.uniform(-1.0, 0.0, size=(2000, F)).astype(np.float32)
    Y = np.clip(np.floor(-X[:, 0] * C), 0, C - 1).astype(np.int32)
    pred = learned.RankPredictor(ctx, C, seed=12)
    hist = pred.train(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), epochs=300,
                      lr=3e-3)
    assert np.all(np.isfinite(hist))
    assert hist[-1] < 0.5 * hist[0]
    logits, _ = pred.infer(torch.from_numpy(X).cuda())
    acc = np.mean(np.argmax(logits.cpu().numpy(), axis=1) == Y)
    assert acc > 0.8


# ---------------------------------------------------------------- solver

# 16^3 cell whose field ranks at eps = 1e-8 (at most 60) stay below the cap, so
# every SVD-truncated rounding meets eps and the iteration converges like the
# dense one
L_SMALL = 4
EPS = 1e-8
RMAX = 64
TOL = 1e-7


@pytest.fixture(scope="module")
def cell():
    from paper_2512_07811_amd import operands as P
    kvox = I.sphere(L_SMALL, 0.2, k_in=10.0, k_out=1.0)
    prob = P.build_problem(kvox=kvox, k0=5.5)
    return kvox, prob


def fresh_field(q, cell, E):
    from paper_2512_07811_amd import operands as P
    ops, e = P.upload(cell[1], [E], RMAX)
    return ops, e


def sketch_opts(q, mode, max_iter=200):
    return q.solve_opts(EPS, RMAX, tol=TOL, max_iter=max_iter, mode=mode, oversample=4, seed=3)


@pytest.fixture(scope="module")
def trained(q, cell):
    """A context with a predictor trained on the rank log of a sketch-mode run."""
    c = q.Context(0)
    from paper_2512_07811_amd import learned
    ops, e = fresh_field(q, cell, [1.0, 0.0, 0.0])
    q.ranklog_enable(c, 200000, C)
    A, its, res, st = q.homogenize(c, ops, e, sketch_opts(q, q.ROUND_SKETCH))
    assert st == q.QT_OK
    X, Y = q.ranklog_get(c)
    q.ranklog_enable(c, 0, C)
    pred = learned.RankPredictor(c, C, seed=21)
    hist = pred.train(X, Y, epochs=400, lr=3e-3)
    pred.install(quantile=0.9)
    yield c, pred, X, Y, A, its, hist
    c.close()


def test_rank_log_contents(q, cell, trained):
    c, pred, X, Y, A, its, hist = trained
    n = 3 * L_SMALL + 1
    # one sample per bond and step, from the second iteration on
    assert X.shape[0] == (its[0] - 1) * 4 * (n - 1)
    Xh, Yh = X.cpu().numpy(), Y.cpu().numpy()
    assert np.all(np.isfinite(Xh))
    assert np.all((Yh >= 0) & (Yh < C))
    assert np.all((Xh[:, :16] >= -1.0) & (Xh[:, :16] <= 0.0))
    # step one-hot and bond position
    assert np.all(Xh[:, 19:23].sum(axis=1) == 1.0)
    pos = np.round(Xh[:, 18] * (n - 1)).astype(int)
    assert pos.min() == 1 and pos.max() == n - 1
    assert hist[-1] < hist[0]


def test_learned_homogenize_matches_svd_path_and_dense_oracle(q, cell, trained):
    c, pred, X, Y, A_sk, its_sk, hist = trained
    ops, e = fresh_field(q, cell, [1.0, 0.0, 0.0])
    c.counters(reset=True)
    A, its, res, st = q.homogenize(c, ops, e, sketch_opts(q, q.ROUND_LEARNED))
    cnt = c.counters(reset=True)
    assert st == q.QT_OK
    assert cnt["learned_roundings"] > 0
    # every rounding met the truncation tolerance (learned or fallback), so the
    # effective conductivity agrees with the SVD-truncated path to 1e-6
    assert abs(A[0, 0] - A_sk[0, 0]) < 1e-6 * abs(A_sk[0, 0])
    assert abs(its[0] - its_sk[0]) <= 2
    kvox = cell[0]
    Ad = ms.effective_tensor(kvox, 5.5, loads=[0], tol=1e-9)
    assert abs(A[0, 0] - Ad[0, 0]) < 1e-5 * Ad[0, 0]


def test_accept_factor_never_relaxes_eps(q, cell):
    # at eps 1e-3 the sketch of width rank cap + oversampling covers every
    # product of this cell, so each SVD-truncated rounding meets eps and a
    # factor above 1 must not loosen the acceptance: a network that always
    # answers rank 8 keeps and rejects the same roundings with accept 1 and 2
    import torch

    from paper_2512_07811_amd import learned
    layers = f32_layers(31)
    layers[7] = np.array([50.0] + [-50.0] * (C - 1), dtype=np.float32)
    layers[6] = np.zeros_like(layers[6])
    params = torch.from_numpy(learned.flat_params(layers)).cuda()
    opts = q.solve_opts(1e-3, RMAX, tol=TOL, max_iter=12, mode=q.ROUND_LEARNED, oversample=4,
                        seed=3)
    runs = []
    for accept in (1.0, 2.0):
        c = q.Context(0)
        try:
            q.set_predictor(c, params, C, 0.9, accept)
            ops, e = fresh_field(q, cell, [1.0, 0.0, 0.0])
            A, its, res, st = q.homogenize(c, ops, e, opts)
            runs.append((A, its, res, c.counters()))
        finally:
            c.close()
    (A1, its1, res1, cnt1), (A2, its2, res2, cnt2) = runs
    assert cnt1["learned_roundings"] > 0
    assert cnt1["learned_fallbacks"] == cnt2["learned_fallbacks"]
    assert cnt1["learned_roundings"] == cnt2["learned_roundings"]
    assert np.array_equal(its1, its2)
    assert np.array_equal(res1, res2)
    assert A1[0, 0] == A2[0, 0]


def test_forced_underprediction_falls_back(q, cell):
    # a network that always answers class 0 (rank 8) under-predicts the field
    # ranks: the a-posteriori check rejects those roundings and the SVD path runs
    import torch

    from paper_2512_07811_amd import learned
    c = q.Context(0)
    try:
        layers = f32_layers(31)
        layers[7] = np.array([50.0] + [-50.0] * (C - 1), dtype=np.float32)
        layers[6] = np.zeros_like(layers[6])
        params = torch.from_numpy(learned.flat_params(layers)).cuda()
        q.set_predictor(c, params, C, 0.9, 1.0)
        ops, e = fresh_field(q, cell, [1.0, 0.0, 0.0])
        A, its, res, st = q.homogenize(c, ops, e, sketch_opts(q, q.ROUND_LEARNED, 12))
        cnt = c.counters()
        assert cnt["learned_roundings"] > 0
        assert cnt["learned_fallbacks"] > 0
        ops2, e2 = fresh_field(q, cell, [1.0, 0.0, 0.0])
        A2, its2, res2, st2 = q.homogenize(c, ops2, e2, sketch_opts(q, q.ROUND_SKETCH, 12))
        assert np.max(np.abs(res - res2)) < 1e-4 * np.max(np.abs(res2))
    finally:
        c.close()


def test_learned_rejects_bad_arguments(q, ctx, cell):
    ops, e = fresh_field(q, cell, [1.0, 0.0, 0.0])
    c = q.Context(0)
    try:
        with pytest.raises(q.QtError):
            q.ls_iterate(c, ops, e, sketch_opts(q, q.ROUND_LEARNED), 1)   # no predictor
        import torch
        params = torch.zeros(q.mlp_num_params(F, C), dtype=torch.float32, device="cuda")
        with pytest.raises(q.QtError):
            q.set_predictor(c, params, C, 0.9, 2.5)                     # accept > 2
        with pytest.raises(q.QtError):
            q.set_predictor(c, params, 1, 0.9, 1.0)                     # one class
    finally:
        c.close()


def test_ablation_trained_network_saves_work(q, cell, trained):
    # the same iterations with and without the predictor: the learned path
    # sketches at the predicted ranks and skips the truncation SVDs, at matched
    # accuracy; an untrained network of the same shape is reported beside it
    from paper_2512_07811_amd import learned
    from paper_2512_07811_amd import operands as P
    c, pred, X, Y, A_sk, its_sk, hist = trained
    n_it = 12

    def run(mode, ctx_):
        ops, e = fresh_field(q, cell, [1.0, 0.0, 0.0])
        e = q.DeviceTT.from_cores([P.mean_field(np.array([1.0, 0.0, 0.0]), L_SMALL)], e.cap)
        q.learn_reset(ctx_)
        ctx_.counters(reset=True)
        res = q.ls_iterate(ctx_, ops, e, sketch_opts(q, mode), n_it).cpu().numpy()[:, 0]
        return res, ctx_.counters(reset=True)

    res_sk, cnt_sk = run(q.ROUND_SKETCH, c)
    res_ln, cnt_ln = run(q.ROUND_LEARNED, c)
    assert np.max(np.abs(res_ln - res_sk)) < 1e-4 * np.max(res_sk)
    assert cnt_ln["gemm_flops"] < cnt_sk["gemm_flops"]
    assert cnt_ln["svd_calls"] < cnt_sk["svd_calls"]
    c2 = q.Context(0)
    try:
        untrained = learned.RankPredictor(c2, C, seed=99)
        untrained.install(quantile=0.9)
        res_un, cnt_un = run(q.ROUND_LEARNED, c2)
    finally:
        c2.close()
    print("ablation", {"sketch": cnt_sk, "trained": cnt_ln, "untrained": cnt_un})
    assert np.max(np.abs(res_un - res_sk)) < 1e-4 * np.max(res_sk)
