"""Pins of the rank-predictor MLP oracle: finite differences, Adam and the
quantile class rule on known class probabilities."""
import numpy as np

from oracle import mlp
from paper_2512_07811_amd import inputs as I


def test_gradients_match_finite_differences():
    g = I.rng(41)
    B, F, C = 7, 11, 5
    x = g.standard_normal((B, F))
    y = g.integers(0, C, size=B)
    P = mlp.init_params(F, C, seed=42)
    for k in P:
        P[k] = P[k] + 0.1 * g.standard_normal(P[k].shape)
    _, G = mlp.loss_and_grad(P, x, y, beta=0.7, gamma=1.5)
    h = 1e-6
    for k in P:
        flat = P[k].reshape(-1)
        idx = g.choice(flat.size, size=min(6, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp, _ = mlp.loss_and_grad(P, x, y, beta=0.7, gamma=1.5)
            flat[i] = old - h
            lm, _ = mlp.loss_and_grad(P, x, y, beta=0.7, gamma=1.5)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - G[k].reshape(-1)[i]) < 1e-7 * max(1.0, abs(fd))


def test_first_adam_step_is_signed_lr():
    P = {"W0": np.array([[1.0, -2.0]]), "b0": np.array([0.5, 0.0])}
    G = {"W0": np.array([[0.3, -4.0]]), "b0": np.array([-1e-3, 2.0])}
    m, v = mlp.adam_init(P)
    mlp.adam_step(P, G, m, v, t=1, lr=0.01, eps=0.0)
    assert np.allclose(P["W0"], [[1.0 - 0.01, -2.0 + 0.01]])
    assert np.allclose(P["b0"], [0.5 + 0.01, 0.0 - 0.01])


def test_cost_matrix_is_asymmetric():
    W = mlp.cost_matrix(4, gamma=2.0)
    assert W[3, 0] == 0.75 and W[0, 3] == 2.0 and W[2, 2] == 0.0


def test_training_separates_toy_classes():
    g = I.rng(43)
    C = 4
    x = g.standard_normal((256, 3))
    y = np.clip(np.floor((x[:, 0] + 2) / 1.0).astype(int), 0, C - 1)
    P = mlp.init_params(3, C, seed=44)
    m, v = mlp.adam_init(P)
    l0, _ = mlp.loss_and_grad(P, x, y)
    for t in range(1, 301):
        l, G = mlp.loss_and_grad(P, x, y)
        mlp.adam_step(P, G, m, v, t, lr=1e-2)
    assert l < 0.5 * l0
    pred = mlp.predict_class(P, x, quantile=0.5)
    assert np.mean(pred == y) > 0.85


def test_predict_class_takes_the_quantile_of_known_probabilities():
    # zero weights: every hidden unit is tanh(0) = 0, so the logits are the
    # last bias; with bias log p the class probabilities are p, and the class
    # is the first one whose cumulative probability reaches the quantile
    P = mlp.init_params(3, 4, seed=1)
    for k in P:
        P[k] = np.zeros_like(P[k])
    last = max(int(k[1:]) for k in P if k.startswith("b"))
    P[f"b{last}"] = np.log(np.array([0.1, 0.2, 0.3, 0.4]))   # cdf 0.1, 0.3, 0.6, 1.0
    x = I.rng(5).standard_normal((7, 3))
    for q, c in ((0.05, 0), (0.25, 1), (0.55, 2), (0.9, 3), (0.95, 3)):
        assert mlp.predict_class(P, x, quantile=q).tolist() == [c] * 7
