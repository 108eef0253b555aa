"""Algorithm 2 (SFFT-based homogenization) on TTs, step by step (oracle).

Test infrastructure only.  Hauck, Kabel, Gauger (arXiv 2512.07811), Sec. 3.2,
Algorithm 2, with TT rounding after every step (Sec. 4 "Accelerated Quantum
Inspired Homogenization": SVD-based compression after each step):

  tau      = round( k' (Hadamard) e_m )
  tau^     = round( S tau )                       S = SFFT operator
  eps^     = round( Gamma^ tau^ )                 Green operator, diagonal TTO
  e_{m+1}  = round( E + (-1) S^{-1} eps^ )        S^{-1} = S^dagger
  r_m      = ||e_{m+1} - e_m||_F / (|E| N^{3/2})  (norm by left orthogonalization)

Readings: the Green multiply is a diagonal-TTO apply followed by rounding (the
paper uses AMEn there); the last rounding acts on the sum of E and the
back-transformed term; the residual norm comes from orthogonalizing the
difference TT, never from expanding <a-b, a-b>.
"""
from __future__ import annotations

import math

import numpy as np

from . import tt as T
from . import ops as O


def ls_iterate(e, kp, S, G, Sinv, E_tt, E, eps, rmax=None, infos=None):
    """One LS iteration; returns (e_new, residual)."""
    L3 = len(e) - 1
    N3 = 2.0 ** L3
    tau, i1 = T.round_tt(T.hadamard(kp, e), eps, rmax, return_info=True)
    tau_h, i2 = T.round_tt(T.mpo_apply(S, tau), eps, rmax, return_info=True)
    eps_h, i3 = T.round_tt(T.mpo_apply(G, tau_h), eps, rmax, return_info=True)
    back = T.mpo_apply(Sinv, eps_h)
    e_new, i4 = T.round_tt(T.add(E_tt, T.scale(back, -1.0)), eps, rmax, return_info=True)
    res = T.norm(T.sub(e_new, e)) / (np.linalg.norm(E) * math.sqrt(N3))
    if infos is not None:
        infos.append((i1, i2, i3, i4))
    return e_new, res


class Problem:
    """Operands of one cell problem: k' TT, SFFT and its inverse, Green TTO."""

    def __init__(self, kvox, k0, op_eps=1e-10, sfft_eps=1e-13):
        self.kvox = kvox
        self.k0 = k0
        N = kvox.shape[0]
        self.L = int(round(math.log2(N)))
        self.kp = O.conductivity_tt(kvox, k0, op_eps)
        self.S = O.sfft_mpo_3d(self.L, sfft_eps)
        self.Sinv = T.conj_transpose_mpo(self.S)
        self.G = O.green_tto(self.L, k0, op_eps)
        sp = T.tt_svd(kvox.reshape(-1), [2] * (3 * self.L), op_eps)
        self.k_sel = [O.component_selector_tt(sp, c) for c in range(3)]


def solve(prob: Problem, E, eps, rmax=None, tol=1e-8, max_iter=200, infos=None):
    """Iterate from e_0 = E until r_m < tol; returns (e, iterations, residuals)."""
    E = np.asarray(E, dtype=np.float64)
    E_tt = O.mean_field_tt(E, prob.L)
    e = [c.copy() for c in E_tt]
    res = []
    it = 0
    for it in range(1, max_iter + 1):
        e, r = ls_iterate(e, prob.kp, prob.S, prob.G, prob.Sinv, E_tt, E, eps, rmax, infos)
        res.append(r)
        if r < tol:
            break
    return e, it, res


def effective_column(prob: Problem, e) -> np.ndarray:
    """A_eff[:, j] = Re <k e^(j)> per component (Appendix A, scalar form)."""
    N3 = 2.0 ** (3 * prob.L)
    return np.array([np.real(T.dot(prob.k_sel[c], e)) / N3 for c in range(3)])


def effective_tensor(prob: Problem, loads, eps, rmax=None, tol=1e-8, max_iter=200):
    A = np.full((3, 3), np.nan)
    its = {}
    for j in loads:
        E = np.zeros(3)
        E[j] = 1.0
        e, it, _ = solve(prob, E, eps, rmax, tol, max_iter)
        A[:, j] = effective_column(prob, e)
        its[j] = it
    return A, its
