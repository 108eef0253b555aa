"""Host set-up of the product path against closed forms and the oracle (CPU)."""
import numpy as np
import pytest

from oracle import ops as O
from oracle import tt as T
from paper_2512_07811_amd import inputs as I
from paper_2512_07811_amd import operands as P


@pytest.mark.parametrize("L", [1, 2, 4, 7, 9])
def test_circuit_sfft_equals_bit_reversed_fft(L):
    N = 2 ** L
    M = T.full_operator(P.sfft_1d(L))
    g = I.rng(100 + L)
    x = g.standard_normal((N, 2)) + 1j * g.standard_normal((N, 2))
    ref = np.fft.fft(x, axis=0)[O.bitrev(L)] / np.sqrt(N)
    assert np.max(np.abs(M @ x - ref)) < 1e-12 * np.max(np.abs(ref))


def test_green_tt_matches_oracle_definition():
    L, k0 = 3, 5.5
    G = P.green_tt(L, k0, 1e-12)
    lifted = [G[0]] + T.diag_lift(G[1:])
    Gref = O.green_momentum(L, k0)
    # contract the operator on unit fields and compare with the dense symbol
    dense = T.full_operator(lifted)
    N = 2 ** L
    diag = np.einsum("aibi->abi", dense.reshape(3, N ** 3, 3, N ** 3))
    assert np.max(np.abs(diag.reshape(3, 3, N, N, N) - Gref)) < 1e-11


@pytest.mark.parametrize("L", [3, 4, 5])
def test_green_expsum_matches_oracle_definition(L):
    # the exponential-sum build (grids beyond 256^3) against the oracle's dense
    # Green array: same operator to the build tolerance, Gamma(0) = 0 and the
    # Nyquist planes zero, same ranks as the dense TT-SVD
    G = P.green_tt_expsum(L, 3.5, 1e-10)
    ctrl = G[0].reshape(9, -1)
    x = ctrl
    for c in G[1:]:
        r, p, r2 = c.shape
        x = (x @ c.reshape(r, p * r2)).reshape(-1, r2)
    ref = O.green_momentum(L, 3.5)
    got = x.reshape(ref.shape)
    assert np.max(np.abs(got - ref)) <= 1e-9 * np.max(np.abs(ref))
    assert [c.shape[-1] for c in G] == [c.shape[-1] for c in P.green_tt(L, 3.5, 1e-10)]


def test_material_tt_bits_and_z_invariance():
    L = 4
    sec = I.cylinders_section(L, seed=3, count=2, r_min=2, r_max=3, k_in=5.0)
    k3 = np.broadcast_to(sec[:, :, None], (16, 16, 16))
    a = T.full(P.material_tt_z_invariant(sec, 1.0, 1e-12)).reshape(16, 16, 16)
    b = T.full(P.material_tt(k3, 1.0, 1e-12)).reshape(16, 16, 16)
    assert np.allclose(a, k3 - 1.0, atol=1e-11) and np.allclose(b, k3 - 1.0, atol=1e-11)


def test_sfft_of_mean_field_is_zero_frequency_delta():
    # S E for a constant field E: rank 1, E N^{3/2} at index 0 (zero frequency,
    # which bit reversal leaves in place), zero elsewhere
    L = 3
    N = 2 ** L
    S, _ = P.sfft_3d(L)
    E = np.array([0.3, -1.2, 2.0])
    se = P.compress(P.apply_mpo(S, P.mean_field(E, L)), 1e-14)
    assert max(c.shape[2] for c in se[:-1]) == 1
    full = se[0]
    for c in se[1:]:
        full = np.tensordot(full, c, axes=(full.ndim - 1, 0))
    full = full.reshape(3, N ** 3)
    want = np.zeros((3, N ** 3), dtype=complex)
    want[:, 0] = E * N ** 1.5
    assert np.max(np.abs(full - want)) < 1e-12 * N ** 1.5


def test_periodic_material_equals_tiled_array():
    # a 2^5 grid tiled by a 2^3 cell: free top bits (identity on the bond)
    # followed by the cell's cores, per axis; compared with the train of the
    # tiled array itself
    cell = I.sphere_lattice_cell(3, rel_radius=0.3, k_in=20.0, k_out=1.0)
    L = 5
    tiled = np.tile(cell, (4, 4, 4))
    per = P.material_tt_periodic(cell, L, 10.5, 1e-12)
    ref = P.material_tt(tiled, 10.5, 1e-12)
    assert len(per) == 3 * L
    assert np.max(np.abs(T.full(per) - T.full(ref))) < 1e-10
    assert max(c.shape[2] for c in per) <= max(c.shape[2] for c in ref)
