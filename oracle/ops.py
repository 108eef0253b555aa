"""Operands of the SFFT-based scheme (oracle).  Test infrastructure only.

Hauck, Kabel, Gauger (arXiv 2512.07811), Sec. 3.2 "Quantum Inspired
Homogenization":
  * binary discretization, eq. (binary_discretization): a grid index
    i = sum_j b_j 2^(L-j), b_1 most significant, one TT core per bit; cores are
    grouped by dimension (x bits, then y bits, then z bits);
  * an extra control core carries the outer (vector-component) index; here it
    is core 0 with mode 3 (reading: position and mode are not stated);
  * QFT_n = R_n Q_n; the SFFT operator is Q_n as a TTO (the bit-reversal R_n is
    dropped and the momentum-space operator is stored in the reversed order);
  * the Green operator is brought into that convention by reversing the bit
    order of each dimension's discretization index (complex conjugation is a
    no-op for the real conductivity Green operator).

Physics reading (the paper treats elasticity only): scalar conductivity with
Green operator Gamma_0(q) = q q^T / (k0 |q|^2), Gamma_0(0) = 0 (Moulinec and
Suquet 1998, conductivity form).  Frequencies m in {-N/2 .. N/2-1} (numpy
fftfreq order); Gamma_0 is zero wherever a component equals -N/2 (Nyquist),
which keeps real fields real.

Everything here is built by dense TT-SVD of the defining array.
"""
from __future__ import annotations

import numpy as np

from . import tt as T


def bitrev(L: int) -> np.ndarray:
    """rev[k] = integer whose L-bit binary expansion is that of k reversed."""
    k = np.arange(2 ** L)
    r = np.zeros_like(k)
    for b in range(L):
        r |= ((k >> b) & 1) << (L - 1 - b)
    return r


def freqs(N: int) -> np.ndarray:
    """Integer frequencies in fftfreq order."""
    return np.fft.fftfreq(N, d=1.0 / N)


# ------------------------------------------------------------------ SFFT

def sfft_matrix(L: int) -> np.ndarray:
    """Dense Q_L = P_rev F / sqrt(N), F[k, j] = exp(-2 pi i j k / N).

    Row k' of the result holds frequency rev(k'): the QFT without its final
    bit-reversal circuit.  Reading: sign e^{-2 pi i}, unitary normalisation.
    """
    N = 2 ** L
    j = np.arange(N)
    rv = bitrev(L)
    phase = np.outer(rv, j) % N          # exact integer phase, avoids large-argument rounding
    return np.exp(-2j * np.pi * phase / N) / np.sqrt(N)


def sfft_mpo_1d(L: int, eps: float = 1e-13):
    """Q_L as a TTO over L bit cores: TT-SVD of the dense matrix with the
    (output bit m, input bit m) pairs merged into one mode of size 4."""
    M = sfft_matrix(L)
    t = M.reshape([2] * (2 * L))                     # (i1..iL, j1..jL)
    perm = [x for m in range(L) for x in (m, L + m)]  # (i1 j1 i2 j2 ...)
    t = np.transpose(t, perm)
    cores = T.tt_svd(t.reshape([4] * L), [4] * L, eps)
    return [c.reshape(c.shape[0], 2, 2, c.shape[2]) for c in cores]


def identity_core(p: int):
    return np.eye(p, dtype=np.complex128).reshape(1, p, p, 1)


def sfft_mpo_3d(L: int, eps: float = 1e-13):
    """Operator on the full operand: identity on the control core, Q_L on each
    of the x, y, z bit groups (the 3D transform is their Kronecker product)."""
    one = sfft_mpo_1d(L, eps)
    return [identity_core(3)] + [c.copy() for _ in range(3) for c in one]


# ----------------------------------------------------------------- Green

def green_natural(L: int, k0: float) -> np.ndarray:
    """Gamma[a, b, jx, jy, jz] at natural frequency order (jx indexes fftfreq)."""
    N = 2 ** L
    m = freqs(N)
    q = np.meshgrid(m, m, m, indexing="ij")
    q2 = q[0] ** 2 + q[1] ** 2 + q[2] ** 2
    nyq = (q[0] == -N / 2) | (q[1] == -N / 2) | (q[2] == -N / 2)
    G = np.zeros((3, 3, N, N, N))
    safe = np.where(q2 > 0, q2, 1.0)
    for a in range(3):
        for b in range(3):
            g = q[a] * q[b] / (k0 * safe)
            g[q2 == 0] = 0.0
            g[nyq] = 0.0
            G[a, b] = g
    return G


def green_momentum(L: int, k0: float) -> np.ndarray:
    """Gamma in the SFFT convention: position k' along an axis holds frequency
    index rev(k') (each dimension's bit order reversed)."""
    rv = bitrev(L)
    G = green_natural(L, k0)
    return G[:, :, rv][:, :, :, rv][:, :, :, :, rv]


def green_tto(L: int, k0: float, eps: float = 1e-10):
    """Green operator as a TTO: control core (1, 3, 3, r) (out a, in b) and
    diagonal spatial cores (TT -> TTO lift of the momentum-convention TT)."""
    G = green_momentum(L, k0)
    cores = T.tt_svd(G.reshape(-1), [9] + [2] * (3 * L), eps)
    ctrl = cores[0].reshape(1, 3, 3, cores[0].shape[2]).astype(np.complex128)
    return [ctrl] + T.diag_lift([c.astype(np.complex128) for c in cores[1:]])


# ------------------------------------------------------ material and loads

def conductivity_tt(kvox: np.ndarray, k0: float, eps: float = 1e-10):
    """k' = k - k0 as a TT with an all-ones control core (broadcast over components)."""
    N = kvox.shape[0]
    L = int(round(np.log2(N)))
    sp = T.tt_svd((kvox - k0).reshape(-1), [2] * (3 * L), eps)
    return [np.ones((1, 3, 1), dtype=np.complex128)] + [c.astype(np.complex128) for c in sp]


def field_to_tt_dense(e: np.ndarray) -> np.ndarray:
    """Dense field e[c, x, y, z] -> tensor with modes [3, 2, ..., 2] (same memory order)."""
    N = e.shape[1]
    L = int(round(np.log2(N)))
    return e.reshape([3] + [2] * (3 * L))


def mean_field_tt(E, L: int):
    """Rank-1 TT of the constant field E (Alg. 2 input)."""
    return [np.asarray(E, dtype=np.complex128).reshape(1, 3, 1)] + \
        [np.ones((1, 2, 1), dtype=np.complex128) for _ in range(3 * L)]


def component_selector_tt(kvox_tt_spatial, c: int):
    """TT of (x -> k(x) on component c, 0 elsewhere): control core = unit vector."""
    e = np.zeros((1, 3, 1), dtype=np.complex128)
    e[0, c, 0] = 1.0
    return [e] + [x.astype(np.complex128) for x in kvox_tt_spatial]
