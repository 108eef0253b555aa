"""Compression of a TT by polar decomposition (oracle).  Test infrastructure only.

Follows Hauck, Kabel, Gauger (arXiv 2512.07811), Sec. 2.2 "Stability",
"Compression via Polar Decomposition": the same two sweeps as the SVD-based
rounding (left orthogonalization, then right to left), but at every bond the
orthogonality centre is split without an SVD:

  T = U H                  polar decomposition of the centre (U isometric,
                           H positive semidefinite; H carries the singular values)
  H - d~ I = U' H'         polar decomposition of the shifted Hermitian factor:
                           U' has eigenvalue +1 on the directions whose singular
                           value exceeds d~ and -1 on the others
  P+ = (1 + U') / 2        projector onto the "above cutoff" directions
  C+ = orthonormal basis of the column space of P+
  F = U C+,  G = C+^dagger H       (T ~ F G, with l = rank(P+) columns)

with the absolute cutoff d~ = delta / q, delta = eps ||x|| / sqrt(n - 1) (the
threshold of eq. optimal_delta, read with n - 1 bonds as for the SVD rounding)
and q the number of singular values of the centre.  Keeping every singular
value above d~ discards at most sqrt(q) d~ = delta / sqrt(q) <= delta at each
bond, so ||x - x~|| <= eps ||x|| holds, with ranks at least those of the SVD
rounding.

Readings (the paper states neither):
  * Orientation: the right-to-left sweep's centre is the (r_k x p_k r_{k+1})
    unfolding A of core k; T = A^dagger, so that H is r_k x r_k, the new core
    is F^dagger = (U C+)^dagger (orthonormal rows) and G^dagger = H C+ is
    carried into core k - 1.
  * q = min(r_k, p_k r_{k+1}), the number of singular values of A.
  * C+ from an eigendecomposition of P+ (eigenvalues above 1/2): the limit of
    the paper's subspace iteration, taken with a library routine.
  * A rank cap r_max keeps the r_max eigenvectors of C+^dagger H C+ with the
    largest eigenvalues (the dominant directions of H above the cutoff).
  * At least one direction is kept (as in the SVD rounding): when no singular
    value exceeds d~, C+ is the dominant eigenvector of H.
The polar factors come from scipy.linalg.polar (a library routine serving as
one step, as the paper leaves the polar algorithm open).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from . import tt as T


def split_centre(A, delta_t, rmax=None):
    """Polar split of the centre A (r x c): returns (core rows F^dagger (l x c),
    carry G^dagger = H C+ (r x l), discarded weight ||A - carry core||_F, l)."""
    Th = np.conj(A.T)                                  # T = A^dagger, (c x r)
    U, H = sla.polar(Th, side="right")                 # T = U H, H (r x r)
    H = 0.5 * (H + np.conj(H.T))
    r = H.shape[0]
    Up, _ = sla.polar(H - delta_t * np.eye(r), side="right")
    Pp = 0.5 * (np.eye(r) + Up)
    Pp = 0.5 * (Pp + np.conj(Pp.T))
    w, V = np.linalg.eigh(Pp)
    C = V[:, w > 0.5]
    if C.shape[1] == 0:
        wh, Vh = np.linalg.eigh(H)
        C = Vh[:, -1:]
    if rmax is not None and rmax > 0 and C.shape[1] > rmax:
        wh, Vh = np.linalg.eigh(np.conj(C.T) @ H @ C)
        C = C @ Vh[:, ::-1][:, :rmax]
    F = U @ C                                          # (c x l)
    carry = H @ C                                      # (r x l)
    core = np.conj(F.T)                                # (l x c)
    disc = float(np.linalg.norm(A - carry @ core))
    return core, carry, disc, C.shape[1]


def round_polar(tt, eps: float, rmax: int | None = None, return_info: bool = False):
    """TT compression by polar decomposition (Sec. 2.2).

    1. left orthogonalization (QR sweep, as in tt.round_tt);
    2. right to left: split every centre by split_centre with d~ = delta / q,
       keep F^dagger as core k and absorb H C+ into core k-1.

    info: kept ranks, discarded weight per bond, err = sqrt(sum disc^2)/||x||,
    ||x||, delta.
    """
    cores, nrm = T.orthogonalize_left(tt)
    n = len(cores)
    delta = eps * nrm / math.sqrt(n - 1) if n > 1 else 0.0
    disc = np.zeros(n + 1)
    kept = [1] * (n + 1)
    for k in range(n - 1, 0, -1):
        r, p, r2 = cores[k].shape
        A = cores[k].reshape(r, p * r2)
        q = min(r, p * r2)
        core, carry, d, l = split_centre(A, delta / q, rmax)
        disc[k] = d
        kept[k] = l
        cores[k] = core.reshape(l, p, r2)
        prev = cores[k - 1]
        rp, pp, _ = prev.shape
        cores[k - 1] = (prev.reshape(rp * pp, r) @ carry).reshape(rp, pp, l)
    err = math.sqrt(float(np.sum(disc ** 2))) / nrm if nrm > 0 else 0.0
    if return_info:
        return cores, {"ranks": kept, "disc": disc, "err": err, "norm": nrm, "delta": delta}
    return cores
