"""Pins of the dense elasticity oracle (oracle/ms_elastic.py).

Closed forms: the exact effective stiffness of a laminate of isotropic layers
(uniform in-plane strains and tractions), and C_eff = C for a homogeneous
cell.  Properties of the Green-Eshelby operator that a wrong factor, sign or
shear convention breaks: Gamma C0 Gamma = Gamma (a projector for the C0
energy), Gamma C0 eps = eps for every compatible strain sym(q (x) u), and
Gamma C0 eps = 0 for a uniform strain.  A random microstructure: symmetric
C_eff between the Reuss and Voigt bounds.
"""
import numpy as np
import pytest

from oracle import ms_elastic as ME
from oracle.ops import freqs


def _laminate(N, lams, mus, layers=4):
    lam = np.zeros((N, N, N))
    mu = np.zeros((N, N, N))
    w = N // layers
    for i in range(layers):
        lam[i * w:(i + 1) * w] = lams[i % 2]
        mu[i * w:(i + 1) * w] = mus[i % 2]
    return lam, mu


def _ref(lam, mu):
    return 0.5 * (lam.min() + lam.max()), 0.5 * (mu.min() + mu.max())


def test_laminate_matches_closed_form():
    lams, mus = (2.0, 6.0), (1.0, 3.0)
    lam, mu = _laminate(8, lams, mus)
    lam0, mu0 = _ref(lam, mu)
    C = ME.effective_tensor(lam, mu, lam0, mu0, tol=1e-13, max_iter=3000)
    ref = ME.laminate_closed_form(lams, mus, [0.5, 0.5])
    assert np.allclose(C, ref, rtol=0, atol=1e-9 * np.abs(ref).max())


def test_homogeneous_cell_is_its_own_effective_tensor():
    lam = np.full((4, 4, 4), 2.5)
    mu = np.full((4, 4, 4), 1.5)
    C = ME.effective_tensor(lam, mu, 1.0, 1.0, tol=1e-14)
    assert np.allclose(C, ME.isotropic_voigt(2.5, 1.5), atol=1e-12)


def _green_voigt(q, lam0, mu0):
    """6 x 6 Voigt matrix of Gamma_0^ at one frequency q (columns: unit stresses)."""
    return np.stack([ME.gamma_strain(np.eye(6)[a], q, lam0, mu0) for a in range(6)], axis=1)


@pytest.mark.parametrize("q", [(1.0, 0.0, 0.0), (1.0, 2.0, 0.0), (1.0, -2.0, 3.0), (0.3, 0.7, -1.1)])
def test_green_operator_is_the_c0_energy_projector(q):
    lam0, mu0 = 2.0, 1.3
    G = _green_voigt(np.array(q), lam0, mu0)
    C0 = ME.isotropic_voigt(lam0, mu0)
    # Gamma C0 Gamma = Gamma
    assert np.allclose(G @ C0 @ G, G, atol=1e-12)
    # compatible strains sym(q (x) u) are kept by Gamma C0
    rng = np.random.default_rng(3)
    for _ in range(3):
        u = rng.standard_normal(3)
        t = 0.5 * (np.outer(q, u) + np.outer(u, q))
        ev = ME.strain_voigt(t)
        assert np.allclose(G @ (C0 @ ev), ev, atol=1e-12)
    # and a strain orthogonal to them (in the C0 energy) is removed: the rank of
    # Gamma C0 is 3, the dimension of {sym(q (x) u)}
    assert np.linalg.matrix_rank(G @ C0, tol=1e-10) == 3


def test_green_operator_vanishes_on_uniform_fields():
    N = 4
    tau = np.zeros((6, N, N, N), dtype=np.complex128)
    tau[:, 0, 0, 0] = np.arange(1, 7)         # zero frequency only
    assert np.abs(ME.green_apply(tau, 1.0, 1.0)).max() == 0.0


def test_random_cell_is_symmetric_and_within_hill_bounds():
    rng = np.random.default_rng(11)
    N = 8
    phase = rng.random((N, N, N)) < 0.35
    lam = np.where(phase, 5.0, 1.0)
    mu = np.where(phase, 4.0, 1.0)
    lam0, mu0 = _ref(lam, mu)
    C = ME.effective_tensor(lam, mu, lam0, mu0, tol=1e-12, max_iter=3000)
    assert np.allclose(C, C.T, atol=1e-8 * np.abs(C).max())
    f = phase.mean()
    Cv = (1 - f) * ME.isotropic_voigt(1.0, 1.0) + f * ME.isotropic_voigt(5.0, 4.0)
    Sr = (1 - f) * np.linalg.inv(ME.isotropic_voigt(1.0, 1.0)) + f * np.linalg.inv(
        ME.isotropic_voigt(5.0, 4.0))
    Cr = np.linalg.inv(Sr)
    assert np.linalg.eigvalsh(Cv - 0.5 * (C + C.T)).min() > -1e-8
    assert np.linalg.eigvalsh(0.5 * (C + C.T) - Cr).min() > -1e-8
