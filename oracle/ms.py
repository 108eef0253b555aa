"""Dense Moulinec-Suquet basic scheme (oracle).  Test infrastructure only.

Hauck, Kabel, Gauger (arXiv 2512.07811), Sec. 3.1, Algorithm 1 (FFT-based
homogenization), written for the scalar-conductivity cell problem on a
periodic 2^L-per-axis grid (reading: the paper treats elasticity):

  e_0 = E
  loop:  tau = (k - k0) e ;  tau^ = FFT(tau) ;  e^ = Gamma_0 tau^ ;
         e_{m+1} = E - IFFT(e^) ;  stop when r_m < delta_tol

with Gamma_0(q) = q q^T/(k0 |q|^2), Gamma_0(0) = 0 and Gamma_0 = 0 on Nyquist
frequencies.  Residual reading (the printed criterion divides by a vector):
r_m = ||e_{m+1} - e_m||_F / (|E| N^(d/2)).

Effective tensor (Appendix A, scalar form): unit loads E = e_j give column j
as the mean flux, A_eff[:, j] = < k e^(j) >.
"""
from __future__ import annotations

import numpy as np

from .ops import freqs


def green_apply(tau_hat: np.ndarray, k0: float) -> np.ndarray:
    """e^_a(q) = sum_b Gamma_ab(q) tau^_b(q) on a d-dimensional natural-order grid."""
    d = tau_hat.shape[0]
    shape = tau_hat.shape[1:]
    grids = np.meshgrid(*[freqs(n) for n in shape], indexing="ij")
    q2 = sum(g ** 2 for g in grids)
    nyq = np.zeros(shape, dtype=bool)
    for g, n in zip(grids, shape):
        nyq |= g == -n / 2
    qdot = sum(grids[b] * tau_hat[b] for b in range(d))
    safe = np.where(q2 > 0, q2, 1.0)
    fac = qdot / (k0 * safe)
    fac[q2 == 0] = 0.0
    fac[nyq] = 0.0
    return np.stack([grids[a] * fac for a in range(d)])


def ms_step(e: np.ndarray, kvox: np.ndarray, k0: float, E) -> np.ndarray:
    """One basic-scheme iteration on a dense field e[c, ...] (c = component)."""
    d = e.shape[0]
    axes = tuple(range(1, d + 1))
    tau = (kvox - k0)[None] * e
    tau_hat = np.fft.fftn(tau, axes=axes)
    eh = green_apply(tau_hat, k0)
    fluct = np.fft.ifftn(eh, axes=axes)
    Ev = np.asarray(E, dtype=np.float64).reshape((d,) + (1,) * d)
    return Ev - fluct.real if np.isrealobj(e) else Ev - fluct


def residual(e_new, e_old, E) -> float:
    npts = e_new[0].size
    return float(np.linalg.norm(e_new - e_old) / (np.linalg.norm(E) * np.sqrt(npts)))


def solve(kvox: np.ndarray, k0: float, E, tol: float = 1e-8, max_iter: int = 1000,
          history: bool = False):
    """Iterate Algorithm 1 from e_0 = E; returns (e, iterations, residual list)."""
    d = kvox.ndim
    shape = kvox.shape
    e = np.broadcast_to(np.asarray(E, dtype=np.float64).reshape((d,) + (1,) * d),
                        (d,) + shape).copy()
    res = []
    it = 0
    for it in range(1, max_iter + 1):
        e_new = ms_step(e, kvox, k0, E)
        r = residual(e_new, e, E)
        res.append(r)
        e = e_new
        if r < tol:
            break
    return (e, it, res) if history else (e, it, res[-1] if res else 0.0)


def effective_column(kvox: np.ndarray, e: np.ndarray) -> np.ndarray:
    """Mean flux <k e> (Appendix A: column of the effective tensor for a unit load)."""
    return np.array([np.mean(kvox * e[c]) for c in range(e.shape[0])])


def effective_tensor(kvox: np.ndarray, k0: float, loads=None, tol: float = 1e-8,
                     max_iter: int = 1000) -> np.ndarray:
    """A_eff with NaN columns for loads not computed."""
    d = kvox.ndim
    A = np.full((d, d), np.nan)
    for j in (range(d) if loads is None else loads):
        E = np.zeros(d)
        E[j] = 1.0
        e, _, _ = solve(kvox, k0, E, tol, max_iter)
        A[:, j] = effective_column(kvox, e)
    return A
