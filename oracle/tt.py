"""Naive tensor-train algebra (oracle).  Test infrastructure only.

Follows Hauck, Kabel, Gauger (arXiv 2512.07811), Sec. 2 "Tensor Trains":
  * TT format, eq. (tt_format); TTO format, eq. (tto_format)
  * constant multiplication, eq. (tt_const_multiplication); addition and
    subtraction by block-diagonal cores; Hadamard product by Kronecker products
    of core slices; TT x TTO contraction; TT -> TTO lift, eq. (tt_to_tto)
    (Sec. 2.1 "Fundamental Algebra")
  * left orthogonalization by a QR sweep and compression by a right-to-left
    truncated-SVD sweep with the threshold of eq. (optimal_delta)
    (Sec. 2.2 "Stability")

Storage reading: the paper writes a core as (r_k x p x r_{k-1}); here core k is
an ndarray of shape (r_k, p_k, r_{k+1}) (left bond, physical, right bond) with
r_0 = r_n = 1.  The order of the bond axes has no effect on any result.
Operator cores are (r_k, p_out, p_in, r_{k+1}).

Threshold reading: eq. (optimal_delta) prints eps/sqrt(1-n)*||x||, imaginary
for n > 1; the TT-rounding bound it cites (Oseledets 2011) has n-1 bonds, so
delta = eps*||x||_F/sqrt(n-1) is used.
"""
from __future__ import annotations

import math

import numpy as np


def ranks(tt):
    return [c.shape[0] for c in tt] + [tt[-1].shape[2]]


def modes(tt):
    return [c.shape[1] for c in tt]


def full(tt):
    """Contract all bonds, eq. (tt_format); returns an array of shape modes(tt)."""
    res = tt[0].reshape(tt[0].shape[1], tt[0].shape[2])          # (p0, r1)
    shp = [tt[0].shape[1]]
    for c in tt[1:]:
        r, p, r2 = c.shape
        res = res @ c.reshape(r, p * r2)
        shp.append(p)
        res = res.reshape(-1, r2)
    return res.reshape(shp)


def full_operator(mpo):
    """Dense matrix of a TTO (eq. tto_format): rows = output multi-index."""
    po = [c.shape[1] for c in mpo]
    pi = [c.shape[2] for c in mpo]
    # treat the operator as a TT with merged (out, in) modes, then permute
    merged = [c.reshape(c.shape[0], c.shape[1] * c.shape[2], c.shape[3]) for c in mpo]
    t = full(merged).reshape([x for pair in zip(po, pi) for x in pair])
    n = len(mpo)
    perm = list(range(0, 2 * n, 2)) + list(range(1, 2 * n, 2))
    t = np.transpose(t, perm)
    return t.reshape(int(np.prod(po)), int(np.prod(pi)))


def tt_svd(a, mode_list, eps: float = 0.0, rmax: int | None = None):
    """TT-SVD of a dense tensor: left-to-right successive truncated SVDs.

    Each bond keeps the smallest rank whose discarded tail does not exceed
    delta = eps*||a||_F/sqrt(n-1) (Sec. 2.2).  eps = 0 keeps every nonzero
    singular direction up to the natural rank (exact reconstruction).
    """
    n = len(mode_list)
    a = np.asarray(a)
    rest = a.reshape(-1)
    nrm = np.linalg.norm(rest)
    delta = eps * nrm / math.sqrt(n - 1) if n > 1 else 0.0
    cores = []
    r = 1
    for k in range(n - 1):
        M = rest.reshape(r * mode_list[k], -1)
        U, s, Vh = np.linalg.svd(M, full_matrices=False)
        l = _choose_rank(s, delta, rmax)
        cores.append(U[:, :l].reshape(r, mode_list[k], l))
        rest = s[:l, None] * Vh[:l]
        r = l
    cores.append(rest.reshape(r, mode_list[-1], 1))
    return cores


def _choose_rank(s, delta, rmax):
    """Smallest l >= 1 with sqrt(sum_{j>l} s_j^2) <= delta, then capped by rmax."""
    s = np.asarray(s, dtype=np.float64)
    q = len(s)
    # tail[l] = sqrt(sum_{j>=l} s_j^2) for l = 0..q (tail[q] = 0)
    tail = np.zeros(q + 1)
    tail[:q] = np.sqrt(np.cumsum((s ** 2)[::-1]))[::-1]
    l = q
    for cand in range(1, q + 1):
        if tail[cand] <= delta:
            l = cand
            break
    l = max(1, l)
    if rmax is not None:
        l = min(l, rmax)
    return l


# ------------------------------------------------------------------ algebra

def scale(tt, c):
    """Constant multiplication: scale the first core (eq. tt_const_multiplication)."""
    out = [x.copy() for x in tt]
    out[0] = c * out[0]
    return out


def add(x, y):
    """Addition by block-diagonal cores; first core [A B], last core [A; B]."""
    n = len(x)
    if n == 1:
        return [x[0] + y[0]]
    out = []
    for k in range(n):
        a, b = x[k], y[k]
        ra, p, ra2 = a.shape
        rb, _, rb2 = b.shape
        dt = np.result_type(a, b)
        if k == 0:
            c = np.zeros((1, p, ra2 + rb2), dtype=dt)
            c[:, :, :ra2] = a
            c[:, :, ra2:] = b
        elif k == n - 1:
            c = np.zeros((ra + rb, p, 1), dtype=dt)
            c[:ra] = a
            c[ra:] = b
        else:
            c = np.zeros((ra + rb, p, ra2 + rb2), dtype=dt)
            c[:ra, :, :ra2] = a
            c[ra:, :, ra2:] = b
        out.append(c)
    return out


def sub(x, y):
    """Subtraction: scale y by -1, then add (Sec. 2.1)."""
    return add(x, scale(y, -1.0))


def hadamard(x, y):
    """Elementwise product: C_k(i) = A_k(i) (Kronecker) B_k(i) (Sec. 2.1).

    The product bond index is (alpha, beta) with alpha (from x) slow.
    """
    out = []
    for a, b in zip(x, y):
        ra, p, ra2 = a.shape
        rb, _, rb2 = b.shape
        c = np.einsum("aib,cid->acibd", a, b).reshape(ra * rb, p, ra2 * rb2)
        out.append(c)
    return out


def mpo_apply(mpo, x):
    """TT x TTO contraction: B_k(i) = sum_j D_k(i, j) (Kronecker) A_k(j) (Sec. 2.1).

    Product bond index (operator bond slow, TT bond fast).
    """
    out = []
    for d, a in zip(mpo, x):
        rd, po, pi, rd2 = d.shape
        ra, pa, ra2 = a.shape
        assert pa == pi
        c = np.einsum("aijb,cjd->acibd", d, a).reshape(rd * ra, po, rd2 * ra2)
        out.append(c)
    return out


def diag_lift(tt):
    """TT -> TTO with D(alpha, i, j, alpha') = B(alpha, i, alpha') delta(i, j), eq. (tt_to_tto)."""
    out = []
    for b in tt:
        r, p, r2 = b.shape
        d = np.zeros((r, p, p, r2), dtype=b.dtype)
        for i in range(p):
            d[:, i, i, :] = b[:, i, :]
        out.append(d)
    return out


def conj_transpose_mpo(mpo):
    """Adjoint operator: conjugate every core and swap (p_out, p_in)."""
    return [np.conj(np.transpose(d, (0, 2, 1, 3))) for d in mpo]


def dot(x, y):
    """sum_i conj(x_i) y_i by a left-to-right environment sweep."""
    env = np.ones((1, 1), dtype=np.result_type(x[0], y[0], np.complex128))
    for a, b in zip(x, y):
        # env[a, b] -> sum_i A(a, i, a')^* env[a, b] B(b, i, b')
        t = np.einsum("ab,bid->aid", env, b)
        env = np.einsum("aic,aid->cd", np.conj(a), t)
    return env[0, 0]


def norm(x):
    _, nrm = orthogonalize_left(x)
    return nrm


# ----------------------------------------------------------------- stability

def orthogonalize_left(tt):
    """QR sweep left to right (Sec. 2.2): Q_k kept, R absorbed into core k+1.

    Returns (cores, ||x||_F) with cores 0..n-2 left-orthogonal and the
    orthogonality centre at the last core.  The left rank after core k is
    min(r'_k * p_k, r_{k+1}) (reading: the R factor is square only when the
    unfolding is tall).
    """
    cores = [c.copy() for c in tt]
    n = len(cores)
    for k in range(n - 1):
        r, p, r2 = cores[k].shape
        Q, R = np.linalg.qr(cores[k].reshape(r * p, r2), mode="reduced")
        s = Q.shape[1]
        cores[k] = Q.reshape(r, p, s)
        nxt = cores[k + 1]
        cores[k + 1] = (R @ nxt.reshape(nxt.shape[0], -1)).reshape(s, nxt.shape[1], nxt.shape[2])
    return cores, float(np.linalg.norm(cores[-1]))


def round_tt(tt, eps: float, rmax: int | None = None, return_info: bool = False):
    """TT rounding (Sec. 2.2, "Compression via SVD").

    1. left orthogonalization (QR sweep);
    2. right-to-left sweep: SVD of the orthogonality centre reshaped
       (r_k x p_k r_{k+1}), keep the smallest l whose discarded tail does not
       exceed delta = eps*||x||/sqrt(n-1), then cap by rmax; V^dagger stays as
       core k, U Sigma is absorbed into core k-1.

    info: singular values per bond (bond k between cores k-1 and k), kept
    ranks, discarded weight per bond and err = sqrt(sum disc^2)/||x||.
    """
    cores, nrm = orthogonalize_left(tt)
    n = len(cores)
    delta = eps * nrm / math.sqrt(n - 1) if n > 1 else 0.0
    svals = [None] * (n + 1)
    disc = np.zeros(n + 1)
    kept = [1] * (n + 1)
    for k in range(n - 1, 0, -1):
        r, p, r2 = cores[k].shape
        U, s, Vh = np.linalg.svd(cores[k].reshape(r, p * r2), full_matrices=False)
        l = _choose_rank(s, delta, rmax)
        svals[k] = s
        disc[k] = math.sqrt(float(np.sum(s[l:] ** 2)))
        kept[k] = l
        cores[k] = Vh[:l].reshape(l, p, r2)
        prev = cores[k - 1]
        rp, pp, _ = prev.shape
        cores[k - 1] = (prev.reshape(rp * pp, r) @ (U[:, :l] * s[:l])).reshape(rp, pp, l)
    err = math.sqrt(float(np.sum(disc ** 2))) / nrm if nrm > 0 else 0.0
    if return_info:
        return cores, {"svals": svals, "ranks": kept, "disc": disc, "err": err, "norm": nrm,
                       "delta": delta}
    return cores


# ------------------------------------------------------------------ helpers

def rank1(vectors):
    """Rank-1 TT from a list of 1D vectors."""
    return [np.asarray(v).reshape(1, -1, 1) for v in vectors]


def left_gram(core):
    """sum_i Q(i)^dagger Q(i) for core (r, p, r') -> (r' x r'); identity if left-orthogonal."""
    r, p, r2 = core.shape
    M = core.reshape(r * p, r2)
    return np.conj(M.T) @ M


def right_gram(core):
    """sum_i V(i) V(i)^dagger for core (r, p, r') -> (r x r); identity if right-orthogonal."""
    r, p, r2 = core.shape
    M = core.reshape(r, p * r2)
    return M @ np.conj(M.T)
