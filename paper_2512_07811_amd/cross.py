"""TT-cross construction of operator trains from entry formulas (host set-up).

A train of a tensor whose entries have a closed form is built from O(n r^2)
sampled entries instead of from its dense array: the rank-adaptive two-site
cross interpolation (DMRG cross) of Savostyanov and Oseledets (2011), with
the maximum-volume row choice of Goreinov, Oseledets, Savostyanov, Tyrtyshnikov,
Zamarashkin (2010).  Sec. 3.2 of arXiv 2512.07811 names cross approximation as
the way to bring large images and operators into QTT form without their dense
arrays; here it builds the Green operator of grids whose 9 N^3 array does not
fit the host (4096^3: 6e11 entries).

Indices are handled through coordinates: digit i of core k adds i * w[k] to a
small integer vector (the component and the x', y', z' positions of the
momentum-ordered grid), so an index set is stored as its coordinate rows, and
a superblock's entries are one broadcast sum and one call of the formula.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg


def maxvol(A: np.ndarray, tol: float = 1.05, max_iters: int = 200) -> np.ndarray:
    """Row indices of a dominant r x r submatrix of the n x r matrix A (n >= r,
    full column rank): every entry of A A[idx]^-1 is at most tol in modulus."""
    n, r = A.shape
    if n <= r:
        return np.arange(n)
    # rank-revealing start: the pivot order of a QR of A^T
    _, _, piv = scipy.linalg.qr(A.T, mode="economic", pivoting=True)
    idx = np.array(piv[:r])
    B = np.linalg.solve(A[idx].T, A.T).T
    for _ in range(max_iters):
        i, j = np.unravel_index(np.argmax(np.abs(B)), B.shape)
        if abs(B[i, j]) <= tol:
            break
        # swap row idx[j] for row i: rank-one update of B = A A[idx]^-1
        bj = B[:, j].copy()
        bi = B[i, :].copy()
        bi[j] -= 1.0
        B -= np.outer(bj, bi / B[i, j])
        idx[j] = i
    return idx


def tt_eval(cores, digits: np.ndarray) -> np.ndarray:
    """Entries of a train at the rows of digits (m x n): one GEMM per core and
    digit value over the samples holding it."""
    m = digits.shape[0]
    v = np.ones((m, 1))
    for k, c in enumerate(cores):
        out = np.empty((m, c.shape[2]), dtype=np.result_type(v, c))
        for i in range(c.shape[1]):
            sel = digits[:, k] == i
            if np.any(sel):
                out[sel] = v[sel] @ c[:, i, :]
        v = out
    return v[:, 0]


def _keep_rank(s: np.ndarray, tol: float, rmax: int) -> int:
    """Smallest rank whose discarded tail sqrt(sum s_j^2) is at most tol * ||s||."""
    tail = np.sqrt(np.cumsum((s ** 2)[::-1]))[::-1]
    thr = tol * tail[0]
    r = int(np.sum(tail > thr))
    return max(1, min(r, rmax))


def tt_cross(fun, weights, modes, eps: float = 1e-10, rmax: int = 1024, r0: int = 16,
             max_sweeps: int = 12, seed: int = 0, n_check: int = 4096, special=None,
             log=None):
    """Train of the tensor T[i_0, ..., i_{n-1}] = fun(sum_k i_k w_k).

    weights: (n, C) integer array, w_k = weights[k]; fun maps an integer array
    (..., C) of coordinates to the entries (...).  modes: the n mode sizes.
    Every superblock (two neighbouring cores with their left and right index
    sets) is truncated at eps / sqrt(n - 1) of its own norm; sweeps alternate
    direction until the sampled maximum error (n_check random entries and the
    rows of `special`, a digit array) stops improving below 10 eps of the
    largest sampled entry, or the ranks stop changing with that error met.
    Returns (cores, info) with real float64 cores (r_k, p_k, r_{k+1})."""
    W = np.asarray(weights, dtype=np.int64)
    n, C = W.shape
    modes = [int(p) for p in modes]
    rng = np.random.default_rng(seed)
    tol = eps / math.sqrt(max(n - 1, 1))
    digit_w = [np.arange(p, dtype=np.int64)[:, None] * W[k][None, :] for k, p in enumerate(modes)]
    # right index sets J[k] (coordinates of digits k..n-1), J[n] = {0}: the
    # all-zero suffix and independent random suffixes (nested random sets
    # lose the variety of their last digits within a few cores, and a
    # superblock that never sees a direction drops it for good)
    J = [None] * (n + 1)
    J[n] = np.zeros((1, C), dtype=np.int64)
    for k in range(n - 1, 0, -1):
        count = 1
        for p in modes[k:]:
            count *= p
            if count >= r0:
                break
        cnt = min(r0, count)
        suf = np.stack([rng.integers(0, p, size=cnt) for p in modes[k:]], axis=1)
        suf[0] = 0
        J[k] = np.unique(suf @ W[k:], axis=0)
    I = [None] * (n + 1)
    I[0] = np.zeros((1, C), dtype=np.int64)
    I[n] = np.zeros((1, C), dtype=np.int64)
    cores = [None] * n
    # sample set for the stopping rule
    chk = np.stack([rng.integers(0, p, size=n_check) for p in modes], axis=1)
    if special is not None:
        chk = np.concatenate([chk, np.asarray(special, dtype=chk.dtype)], axis=0)
    chk_val = fun(chk.astype(np.int64) @ W)
    scale = max(float(np.max(np.abs(chk_val))), 1e-300)
    evals = 0
    history = []
    prev_ranks = None

    def superblock(k):
        nonlocal evals
        crd = (I[k][:, None, None, None, :] + digit_w[k][None, :, None, None, :]
               + digit_w[k + 1][None, None, :, None, :] + J[k + 2][None, None, None, :, :])
        evals += crd.size // C
        return fun(crd)

    best = math.inf
    for sweep in range(max_sweeps):
        forward = sweep % 2 == 0
        order = range(n - 1) if forward else range(n - 2, -1, -1)
        for k in order:
            B = superblock(k)
            rk, pk, pk1, rk2 = B.shape
            M = B.reshape(rk * pk, pk1 * rk2)
            U, s, Vt = np.linalg.svd(M, full_matrices=False)
            r = _keep_rank(s, tol, rmax)
            if forward:
                Ur = U[:, :r]
                idx = maxvol(Ur)
                left = (I[k][:, None, :] + digit_w[k][None, :, :]).reshape(-1, C)
                I[k + 1] = left[idx]
                cores[k] = np.linalg.solve(Ur[idx].T, Ur.T).T.reshape(rk, pk, r)
                if k == n - 2:
                    cores[k + 1] = M[idx].reshape(r, pk1, rk2)
            else:
                Vr = Vt[:r].T                       # (pk1 rk2) x r
                idx = maxvol(Vr)
                right = (digit_w[k + 1][:, None, :] + J[k + 2][None, :, :]).reshape(-1, C)
                J[k + 1] = right[idx]
                cores[k + 1] = np.linalg.solve(Vr[idx].T, Vr.T).reshape(r, pk1, rk2)
                if k == 0:
                    cores[0] = M[:, idx].reshape(rk, pk, r)
        approx = tt_eval(cores, chk)
        err = float(np.max(np.abs(approx - chk_val))) / scale
        ranks = [c.shape[2] for c in cores[:-1]]
        history.append((err, max(ranks)))
        if log:
            log(f"cross sweep {sweep + 1}: max rank {max(ranks)}, sampled max error {err:.2e}")
        if sweep >= 1 and err <= 10 * eps and (ranks == prev_ranks or err >= 0.5 * best):
            break
        best = min(best, err)
        prev_ranks = ranks
    info = {"sweeps": len(history), "history": history, "evaluations": evals,
            "sampled_max_error": history[-1][0]}
    return cores, info


def green_momentum_fun(L: int, k0: float):
    """Entry formula of the conductivity Green operator in the momentum order of
    the SFFT (position x' along an axis holds the frequency of index rev(x')):
    coordinates (c, x', y', z') with c = 3 a + b give q_a q_b / (k0 |q|^2), zero
    at q = 0 and where any component is the Nyquist frequency -N/2."""
    N = 2 ** L
    idx = np.arange(N)
    rev = np.zeros_like(idx)
    for b in range(L):
        rev = (rev << 1) | ((idx >> b) & 1)
    f = np.where(rev < N // 2, rev, rev - N).astype(np.float64)

    def fun(crd):
        c = crd[..., 0]
        q = [f[crd[..., 1]], f[crd[..., 2]], f[crd[..., 3]]]
        q2 = q[0] ** 2 + q[1] ** 2 + q[2] ** 2
        a, b = c // 3, c % 3
        qa = np.choose(a, q)
        qb = np.choose(b, q)
        bad = (q2 == 0) | (q[0] == -N // 2) | (q[1] == -N // 2) | (q[2] == -N // 2)
        return np.where(bad, 0.0, qa * qb / (k0 * np.where(q2 == 0, 1.0, q2)))

    return fun


def grid_weights(L: int, control: int = 0) -> np.ndarray:
    """Coordinate weights of a 3D QTT with an optional control core first: the
    control digit adds to coordinate 0, then the L bits of each axis (most
    significant first) add 2^(L-1-j) to that axis' coordinate."""
    off = 1 if control else 0
    W = np.zeros(((1 if control else 0) + 3 * L, off + 3), dtype=np.int64)
    if control:
        W[0, 0] = 1
    for a in range(3):
        for j in range(L):
            W[(1 if control else 0) + a * L + j, off + a] = 1 << (L - 1 - j)
    return W


def green_tt_cross(L: int, k0: float, eps: float = 1e-10, rmax: int = 1024, seed: int = 0,
                   log=None):
    """The Green operator of green_tt (component core (1, 3, 3, r), spatial cores
    (r, 2, r')) by cross interpolation of its entry formula at eps / 100, then
    one TT rounding at eps.  Returns (cores, info)."""
    from .operands import compress
    n = 1 + 3 * L
    modes = [9] + [2] * (3 * L)
    # entries the stopping rule always checks: the origin and one Nyquist
    # position per axis (x' = 1 holds frequency -N/2), for every component
    special = []
    for c in range(9):
        for pos in ([], [L], [2 * L], [3 * L]):
            d = np.zeros(n, dtype=np.int64)
            d[0] = c
            for p in pos:
                d[p] = 1
            special.append(d)
    # the interpolation amplifies the superblock truncations in the maximum
    # norm: cross at eps / 100, then one TT rounding at eps
    cores, info = tt_cross(green_momentum_fun(L, k0), grid_weights(L, control=1), modes,
                           eps=eps * 1e-2, rmax=rmax, seed=seed, special=np.array(special),
                           max_sweeps=20, log=log)
    cores = compress(cores, eps)
    ctrl = cores[0].reshape(1, 3, 3, cores[0].shape[2])
    return [ctrl.astype(np.complex128)] + [c.astype(np.complex128) for c in cores[1:]], info
