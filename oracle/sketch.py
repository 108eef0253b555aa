"""Randomized TT rounding (oracle).  Test infrastructure only.

Randomize-then-orthogonalize (Al Daas, Ballard, Cazeaux, Hallman, Miedlar,
Pasha, Reid, Saibaba, "Randomized algorithms for rounding in the tensor-train
format", SIAM J. Sci. Comput. 45 (2023)), the range-finder idea of Halko,
Martinsson and Tropp (SIAM Review 2011) applied bond by bond.  It is the
fixed-rank alternative to SVD truncation named in Sec. 2.2 of Hauck, Kabel,
Gauger (arXiv 2512.07811) ("prescribe a fixed number of singular values").

Given x with bond ranks R_k and a Gaussian TT Omega with ranks l_k:
  right pass   W_n = 1;  W_k = sum_i X_k(i) W_{k+1} Omega_k(i)^T      (R_k x l_k)
  left pass    Z_0 = X_0;  for k = 0..n-2:
                 Y_k = Z_k W_{k+1};  Q_k = orth(Y_k)  -> core k
                 M_k = Q_k^dagger Z_k;  Z_{k+1} = M_k X_{k+1}
               core n-1 = Z_{n-1}
The result is the orthogonal projection of x onto the span of the left
interface bases, so ||x - x~||^2 = ||x||^2 - ||x~||^2.

Omega's cores are inputs (drawn by the shared seeded generator).
"""
from __future__ import annotations

import math

import numpy as np

from . import tt as T


def right_sketches(x, omega):
    """W[k] for bonds k = 1..n (W[n] = [[1]]); W[k] has shape (R_k, l_k)."""
    n = len(x)
    W = [None] * (n + 1)
    W[n] = np.ones((1, 1), dtype=np.complex128)
    for k in range(n - 1, 0, -1):
        X = x[k]
        Om = omega[k]
        acc = np.zeros((X.shape[0], Om.shape[0]), dtype=np.complex128)
        for i in range(X.shape[1]):
            acc += X[:, i, :] @ W[k + 1] @ Om[:, i, :].T
        W[k] = acc
    return W


def rto(x, omega):
    """Randomize-then-orthogonalize: fixed-rank projection of x; returns cores."""
    n = len(x)
    W = right_sketches(x, omega)
    out = []
    Z = x[0].reshape(x[0].shape[1], x[0].shape[2]).astype(np.complex128)   # (p0, R1)
    rprev = 1
    for k in range(n - 1):
        p = x[k].shape[1]
        Y = Z @ W[k + 1]
        Q, _ = np.linalg.qr(Y, mode="reduced")
        s = Q.shape[1]
        out.append(Q.reshape(rprev, p, s))
        M = np.conj(Q.T) @ Z
        nxt = x[k + 1]
        Z = (M @ nxt.reshape(nxt.shape[0], -1)).reshape(s * nxt.shape[1], nxt.shape[2])
        rprev = s
    out.append(Z.reshape(rprev, x[-1].shape[1], 1))
    return out


def truncate_right(cores, delta, rmax=None):
    """Right-to-left SVD truncation of a TT whose cores 0..n-2 are left-orthogonal
    (the second sweep of Sec. 2.2 on an already orthogonalized train)."""
    cores = [c.copy() for c in cores]
    n = len(cores)
    disc = np.zeros(n + 1)
    kept = [1] * (n + 1)
    svals = [None] * (n + 1)
    for k in range(n - 1, 0, -1):
        r, p, r2 = cores[k].shape
        U, s, Vh = np.linalg.svd(cores[k].reshape(r, p * r2), full_matrices=False)
        l = T._choose_rank(s, delta, rmax)
        svals[k] = s
        disc[k] = math.sqrt(float(np.sum(s[l:] ** 2)))
        kept[k] = l
        cores[k] = Vh[:l].reshape(l, p, r2)
        prev = cores[k - 1]
        rp, pp, _ = prev.shape
        cores[k - 1] = (prev.reshape(rp * pp, r) @ (U[:, :l] * s[:l])).reshape(rp, pp, l)
    return cores, {"disc": disc, "ranks": kept, "svals": svals}


NOISE_FLOOR = 1e-14


def sketch_round(x, omega, eps, rmax=None, xnorm=None):
    """RTO followed by SVD truncation with the remaining error budget.

    sketch error e_s^2 = ||x||^2 - ||x~||^2 (exact for the projection).  The
    truncation of interior bonds moves the left interfaces of the result out of
    the sketch's span, so the projection error x - x~ and the truncation error
    are not orthogonal: the budget is split linearly (triangle inequality),
    ||x - z|| <= e_s + sqrt(sum of discarded tails^2) <= eps ||x||, with the
    per-bond threshold (eps ||x|| - e_s)/sqrt(n-1), and at least
    NOISE_FLOOR ||x|| when eps > 0.
    Returns (cores, info) with info['ok'] = (e_s <= eps ||x||) and
    info['err_bound'] = (e_s + sqrt(sum tails^2)) / ||x||.
    """
    n = len(x)
    if xnorm is None:
        xnorm = math.sqrt(abs(T.dot(x, x)))
    y = rto(x, omega)
    ynorm = float(np.linalg.norm(y[-1]))
    es2 = max(xnorm ** 2 - ynorm ** 2, 0.0)
    es = math.sqrt(es2)
    budget = eps * xnorm - es
    ok = budget >= 0.0
    delta = max(budget, 0.0) / math.sqrt(n - 1) if n > 1 else 0.0
    if eps > 0.0 and n > 1:
        # noise floor: for eps > 0 no direction below 1e-14 ||x|| is kept, also
        # when the sketch error alone exceeds the budget
        delta = max(delta, NOISE_FLOOR * xnorm)
    z, info = truncate_right(y, delta, rmax)
    trunc = math.sqrt(float(np.sum(np.asarray(info["disc"]) ** 2)))
    info.update({"sketch_err": es, "xnorm": xnorm, "ynorm": ynorm, "ok": ok,
                 "delta": delta, "err_bound": (es + trunc) / xnorm if xnorm > 0 else 0.0})
    return z, info
