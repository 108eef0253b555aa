"""Host set-up of the elasticity operands against the dense oracle (CPU).

The Voigt Green-Eshelby train reproduces the oracle's operator at every
momentum position (frequency rev(x') per axis), G2 = G^T G per frequency,
the material operator C - C0 and (C - C0)^T (C - C0) act on dense fields as
the oracle's Voigt stress does, and k_sel[c] holds row c of C.
"""
import numpy as np
import pytest

from oracle import ms_elastic as ME
from oracle import ops as O
from oracle import tt as T
from paper_2512_07811_amd import inputs as I
from paper_2512_07811_amd import operands as P


def _cell(L, seed):
    g = np.random.default_rng(seed)
    N = 2 ** L
    ph = g.random((N, N, N)) < 0.4
    return np.where(ph, 6.0, 2.0), np.where(ph, 3.0, 1.0)


def _momentum_q(L):
    N = 2 ** L
    f = O.freqs(N)
    f = np.where(f == N // 2, -N // 2, f)                 # signed
    fr = f[O.bitrev(L)]
    return np.meshgrid(fr, fr, fr, indexing="ij"), N


def test_green_voigt_train_matches_oracle_operator():
    L, lam0, mu0 = 2, 4.0, 2.0
    G, G2 = P.green_tt_elastic(L, lam0, mu0, 1e-13)
    (qx, qy, qz), N = _momentum_q(L)
    q2 = qx ** 2 + qy ** 2 + qz ** 2
    bad = (q2 == 0) | (qx == -N // 2) | (qy == -N // 2) | (qz == -N // 2)
    safe = [np.where(bad, 1.0, g) for g in (qx, qy, qz)]
    ref = np.stack([ME.gamma_strain(np.eye(6)[b][:, None, None, None] * np.ones((1, N, N, N)),
                                    safe, lam0, mu0) for b in range(6)], axis=1)
    ref[:, :, bad] = 0.0
    for train, want in ((G, ref), (G2, np.einsum("ca...,cb...->ab...", ref, ref))):
        dense = T.full_operator([train[0]] + T.diag_lift(train[1:]))
        diag = np.einsum("aibi->abi", dense.reshape(6, N ** 3, 6, N ** 3))
        assert np.max(np.abs(diag.reshape(6, 6, N, N, N) - want)) < 1e-10 * np.abs(want).max()


def test_material_operators_act_as_the_oracle_stress():
    L = 2
    lam, mu = _cell(L, 3)
    prob = P.build_problem_elastic(lam, mu)
    lam0, mu0 = prob["lam0"], prob["mu0"]
    N = 2 ** L
    Kp = T.full_operator([prob["Kp_op"][0]] + T.diag_lift(prob["Kp_op"][1:]))
    K2 = T.full_operator([prob["K2_op"][0]] + T.diag_lift(prob["K2_op"][1:]))
    g = np.random.default_rng(5)
    ev = g.standard_normal((6, N, N, N))
    want = ME.stress_apply(lam - lam0, mu - mu0, ev)
    assert np.allclose((Kp @ ev.reshape(-1)).real.reshape(ev.shape), want, atol=1e-9)
    assert np.allclose(K2, Kp.conj().T @ Kp, atol=1e-8 * np.abs(K2).max())
    for c in range(6):
        row = T.full(prob["k_sel"][c]).reshape(6, N, N, N).real
        for j in range(6):
            e = np.zeros((6, 1, 1, 1))
            e[j] = 1.0
            assert np.allclose(row[j], ME.stress_apply(lam, mu, e * np.ones((6, N, N, N)))[c],
                               atol=1e-9)


def test_elastic_sfft_is_identity_on_the_voigt_core():
    S, Sinv = P.sfft_3d(1, 1e-13, d=6)
    assert S[0].shape == (1, 6, 6, 1)
    assert np.allclose(S[0][0, :, :, 0], np.eye(6))
