"""Pins of the dense Moulinec-Suquet oracle (Algorithm 1, scalar form).

Closed forms (laminate: harmonic mean across layers, arithmetic mean along
them), Wiener bounds, and the defining conditions of the cell problem at the
fixed point: curl-free field with mean E and divergence-free flux.
"""
import json
import os

import numpy as np
import pytest

from oracle import ms
from oracle import ops as O
from paper_2512_07811_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_laminate_closed_form_c1():
    with open(os.path.join(GOLDEN, "laminate_32.json")) as f:
        gold = json.load(f)
    k = I.laminate(5, layers=4, k_lo=1.0, k_hi=10.0)
    A = ms.effective_tensor(k, 5.5, loads=[0, 1], tol=1e-12, max_iter=50)
    assert abs(A[0, 0] - gold["A_xx"]) < 1e-12 * gold["A_xx"]
    assert abs(A[1, 1] - gold["A_yy"]) < 1e-12 * gold["A_yy"]
    assert np.all(np.abs(A[[1, 2], 0]) < 1e-13) and np.all(np.abs(A[[0, 2], 1]) < 1e-13)


def test_random_layer_profile_harmonic_mean():
    # an x-only profile: A_xx = harmonic mean, A_yy = arithmetic mean.  The
    # discrete fixed point is e_x = c/k exactly when 1/k has no Nyquist content
    # (Gamma is zero there), so odd-position resistivities permute the even ones.
    g = I.rng(21)
    N = 16
    u = g.uniform(0.25, 1.0, size=N // 2)
    res = np.empty(N)
    res[0::2] = u
    res[1::2] = g.permutation(u)
    prof = 1.0 / res
    k = np.broadcast_to(prof[:, None, None], (N, N, N)).copy()
    k0 = (prof.min() + prof.max()) / 2
    A = ms.effective_tensor(k, k0, loads=[0, 1], tol=1e-13, max_iter=400)
    assert abs(A[0, 0] - 1.0 / np.mean(1.0 / prof)) < 1e-10
    assert abs(A[1, 1] - np.mean(prof)) < 1e-12


@pytest.mark.parametrize("seed", [1, 2])
def test_boxes_fixed_point_conditions_and_bounds(seed):
    L = 4
    N = 2 ** L
    k = I.random_boxes(L, seed, edge_min=2, edge_max=8, k_min=2.0, k_max=8.0)
    k0 = (k.min() + k.max()) / 2
    A = np.zeros((3, 3))
    fields = []
    for j in range(3):
        E = np.zeros(3)
        E[j] = 1.0
        e, it, r = ms.solve(k, k0, E, tol=1e-13, max_iter=2000)
        fields.append(e)
        A[:, j] = ms.effective_column(k, e)
        # mean field equals E
        assert np.allclose(e.mean(axis=(1, 2, 3)), E, atol=1e-12)
        # curl-free: Fourier coefficients of e - E parallel to q
        m = O.freqs(N)
        q = np.stack(np.meshgrid(m, m, m, indexing="ij"))
        eh = np.fft.fftn(e - E[:, None, None, None], axes=(1, 2, 3))
        curl = np.cross(q, eh, axis=0)
        nyq = (q == -N / 2).any(axis=0)
        assert np.max(np.abs(curl[:, ~nyq])) < 1e-9 * np.max(np.abs(eh))
        # divergence-free flux: q . FFT(k e) = 0 for q != 0 off Nyquist
        fh = np.fft.fftn(k[None] * e, axes=(1, 2, 3))
        div = np.sum(q * fh, axis=0)
        assert np.max(np.abs(div[~nyq])) < 1e-9 * np.max(np.abs(fh))
    # symmetry and energy (discrete Hill-Mandel): <k e_i . e_j> = A_ij
    assert np.allclose(A, A.T, atol=1e-10)
    for i in range(3):
        for j in range(3):
            en = np.mean(k * np.sum(fields[i] * fields[j], axis=0))
            assert abs(en - A[i, j]) < 1e-9
    # Wiener bounds on the eigenvalues
    w = np.linalg.eigvalsh((A + A.T) / 2)
    assert w.min() >= 1.0 / np.mean(1.0 / k) - 1e-10
    assert w.max() <= np.mean(k) + 1e-10


def test_sphere_isotropy_and_hashin_shtrikman():
    L = 5
    k = I.sphere(L, frac=0.2, k_in=10.0, k_out=1.0)
    f = np.mean(k == 10.0)
    A = ms.effective_tensor(k, 5.5, loads=[0, 1, 2], tol=1e-11, max_iter=2000)
    assert np.allclose(np.diag(A), A[0, 0], rtol=1e-10)
    assert np.max(np.abs(A - np.diag(np.diag(A)))) < 1e-10
    # Hashin-Shtrikman bounds for an isotropic two-phase composite (3D)
    k1, k2 = 1.0, 10.0
    lo = k1 + f / (1 / (k2 - k1) + (1 - f) / (3 * k1))
    hi = k2 + (1 - f) / (1 / (k1 - k2) + f / (3 * k2))
    # voxelized inclusion on a 32^3 grid: allow a small discretization margin
    assert lo * 0.98 <= A[0, 0] <= hi


def test_first_iterate_by_hand_1d():
    # a single nonzero Fourier pair: tau = cos(2 pi x/N) along x
    N = 8
    x = np.arange(N)
    prof = 2.0 + np.cos(2 * np.pi * x / N)
    k = np.broadcast_to(prof[:, None, None], (N, N, N)).copy()
    k0 = 2.0
    e1 = ms.ms_step(np.stack([np.ones((N, N, N)), np.zeros((N, N, N)), np.zeros((N, N, N))]),
                    k, k0, [1.0, 0.0, 0.0])
    # tau_x = cos(.) has zero mean; Gamma_xx = 1/k0 on (m, 0, 0): e1_x = 1 - cos/k0
    assert np.allclose(e1[0], 1.0 - np.cos(2 * np.pi * x / N)[:, None, None] / k0, atol=1e-14)
    assert np.allclose(e1[1:], 0.0, atol=1e-14)
