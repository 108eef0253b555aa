"""Host-side set-up of the operands of Algorithm 2 (not on the hot path).

Builds, once per problem, the trains that the HIP iteration consumes:
  * k' = k - k0 in the binary (QTT) discretization of eq. (binary_discretization),
    grid bits of x, then y, then z, most significant first, with an all-ones
    component core in front (Sec. 3.2 of arXiv 2512.07811);
  * the SFFT operator Q_L (the QFT without its final bit-reversal, Sec. 3.2)
    assembled from its gate structure: every output bit m picks up the phase
    exp(-2 pi i k'_m j_m' 2^(m-1-m')) from each input bit m' >= m, i.e. one
    Hadamard-type factor per qubit and one controlled phase per pair; each
    factor is an exact rank <= 2 operator train, they are multiplied
    elementwise and recompressed as the product grows;
  * the Green operator Gamma_0(q) = q q^T/(k0 |q|^2) sampled in the SFFT's
    momentum convention (each axis' bit order reversed), compressed to a
    train with a 3 x 3 component core and diagonal spatial cores;
  * the rank-1 mean field E and the selector trains k * e_c used for A_eff.
Compression uses its own host TT-SVD (QR of the long side, SVD of the small
factor), independent of the test oracle.
"""
from __future__ import annotations

import math

import numpy as np


# ------------------------------------------------------------- host TT kit

def _keep(s, delta, rmax=None):
    """Smallest l >= 1 whose discarded tail sqrt(sum_{j>=l} s_j^2) <= delta."""
    tail = np.sqrt(np.cumsum((s ** 2)[::-1]))[::-1]
    ok = np.nonzero(tail <= delta)[0]
    l = int(ok[0]) if ok.size else len(s)
    l = max(l, 1)
    return min(l, rmax) if rmax else l


def _svd_wide(M):
    """Thin SVD of a matrix with few rows, through a QR of its transpose."""
    r, c = M.shape
    if c <= 2 * r:
        return np.linalg.svd(M, full_matrices=False)
    Q, R = np.linalg.qr(M.T)                 # M^T = Q R   (c x r) (r x r)
    U, s, Wt = np.linalg.svd(R.T)            # M = R^T Q^T = U s Wt Q^T
    return U, s, Wt @ Q.T


def ttsvd(a, modes, eps, rmax=None):
    """Train of a dense array by successive truncated SVDs (threshold eps*||a||/sqrt(n-1))."""
    n = len(modes)
    rest = np.asarray(a).reshape(-1)
    delta = eps * np.linalg.norm(rest) / math.sqrt(max(n - 1, 1))
    cores, r = [], 1
    for k in range(n - 1):
        U, s, Vt = _svd_wide(rest.reshape(r * modes[k], -1))
        l = _keep(s, delta, rmax)
        cores.append(U[:, :l].reshape(r, modes[k], l))
        rest = s[:l, None] * Vt[:l]
        r = l
    cores.append(rest.reshape(r, modes[-1], 1))
    return cores


def compress(cores, eps, rmax=None):
    """Host rounding: right-to-left LQ orthogonalization, then left-to-right SVD truncation."""
    cs = [np.array(c) for c in cores]
    n = len(cs)
    for k in range(n - 1, 0, -1):
        r, p, r2 = cs[k].shape
        Q, R = np.linalg.qr(cs[k].reshape(r, p * r2).T)       # core^T = Q R
        s = Q.shape[1]
        cs[k] = Q.T.reshape(s, p, r2)
        cs[k - 1] = np.tensordot(cs[k - 1], R.T, axes=(2, 0))
    nrm = np.linalg.norm(cs[0])
    delta = eps * nrm / math.sqrt(max(n - 1, 1))
    for k in range(n - 1):
        r, p, r2 = cs[k].shape
        U, s, Vt = np.linalg.svd(cs[k].reshape(r * p, r2), full_matrices=False)
        l = _keep(s, delta, rmax)
        cs[k] = U[:, :l].reshape(r, p, l)
        cs[k + 1] = np.tensordot(s[:l, None] * Vt[:l], cs[k + 1], axes=(1, 0))
    return cs


def elementwise(x, y):
    """Elementwise product of two trains with equal modes (Kronecker of slices)."""
    out = []
    for a, b in zip(x, y):
        ra, p, ra2 = a.shape
        rb, _, rb2 = b.shape
        c = (a[:, None, :, :, None] * b[None, :, :, None, :]).reshape(ra * rb, p, ra2 * rb2)
        out.append(c)
    return out


# --------------------------------------------------------------- geometry

def bit_reversal(L):
    idx = np.arange(2 ** L)
    rev = np.zeros_like(idx)
    for b in range(L):
        rev = (rev << 1) | ((idx >> b) & 1)
    return rev


def signed_freq(N):
    k = np.arange(N)
    return np.where(k < N // 2, k, k - N).astype(np.float64)


# ------------------------------------------------------------------ SFFT

def sfft_1d(L, eps=1e-13):
    """Q_L as (r, 2, 2, r') cores, built from its per-qubit and per-pair phase factors.

    Merged physical index (k'_c, j_c) -> 2*k'_c + j_c; the output position
    k' holds frequency rev(k').
    """
    ones = [np.ones((1, 4, 1), dtype=np.complex128) for _ in range(L)]
    kk = np.array([0, 0, 1, 1])
    jj = np.array([0, 1, 0, 1])
    train = [c.copy() for c in ones]
    for m in range(L):
        # qubit factor: (-1)^(k'_m j_m) / sqrt(2)
        g = [c.copy() for c in ones]
        g[m] = (np.where(kk * jj == 1, -1.0, 1.0) / math.sqrt(2.0)).astype(np.complex128).reshape(1, 4, 1)
        train = elementwise(train, g)
        for mp in range(m + 1, L):
            # controlled phase between output bit m and input bit mp
            ang = -2.0 * math.pi * 2.0 ** (m - mp - 1)
            g = [c.copy() for c in ones]
            first = np.zeros((1, 4, 2), dtype=np.complex128)
            first[0, kk == 0, 0] = 1.0
            first[0, kk == 1, 1] = 1.0
            g[m] = first
            for c in range(m + 1, mp):
                mid = np.zeros((2, 4, 2), dtype=np.complex128)
                mid[0, :, 0] = 1.0
                mid[1, :, 1] = 1.0
                g[c] = mid
            last = np.zeros((2, 4, 1), dtype=np.complex128)
            last[0, :, 0] = 1.0
            last[1, :, 0] = np.exp(1j * ang * jj)
            g[mp] = last
            train = compress(elementwise(train, g), eps * 1e-2)
    train = compress(train, eps)
    return [c.reshape(c.shape[0], 2, 2, c.shape[2]) for c in train]


def sfft_3d(L, eps=1e-13, d=3):
    """Identity on the component core (mode d), Q_L on each axis group; and its adjoint."""
    one = sfft_1d(L, eps)
    eye = np.eye(d, dtype=np.complex128).reshape(1, d, d, 1)
    S = [eye] + [c.copy() for _ in range(3) for c in one]
    Sinv = [np.conj(np.transpose(c, (0, 2, 1, 3))) for c in S]
    return S, Sinv


# ------------------------------------------------------------------ Green

def green_momentum_dense(L, k0):
    """Gamma[a, b, x', y', z'] where position x' along an axis holds frequency rev(x')."""
    N = 2 ** L
    f = signed_freq(N)[bit_reversal(L)]
    q = [f[:, None, None], f[None, :, None], f[None, None, :]]
    q2 = q[0] ** 2 + q[1] ** 2 + q[2] ** 2
    bad = (q2 == 0) | (q[0] == -N // 2) | (q[1] == -N // 2) | (q[2] == -N // 2)
    inv = np.where(bad, 0.0, 1.0 / np.where(q2 == 0, 1.0, q2)) / k0
    G = np.empty((3, 3, N, N, N))
    for a in range(3):
        for b in range(a, 3):
            G[a, b] = q[a] * q[b] * inv
            if b != a:
                G[b, a] = G[a, b]
    return G


def green_tt(L, k0, eps=1e-10):
    """Green operator: component core (1, 3, 3, r) and diagonal spatial cores (r, 2, r')."""
    G = green_momentum_dense(L, k0)
    cores = ttsvd(G.reshape(-1), [9] + [2] * (3 * L), eps)
    ctrl = cores[0].reshape(1, 3, 3, cores[0].shape[2])
    return [ctrl.astype(np.complex128)] + [c.astype(np.complex128) for c in cores[1:]]


def _inv_expsum(smax, tol):
    """Exponents t_m and weights w_m with 1/s ~ sum_m w_m exp(-t_m s) on [1, smax]
    to relative error below tol: the trapezoidal rule on 1/s = int exp(-s e^u + u) du,
    step pi^2 / (2 log(4/tol)) from the width of the strip where the integrand is
    analytic, range cut where each tail falls below tol."""
    h = math.pi ** 2 / (2.0 * math.log(4.0 / tol))
    u = np.arange(math.log(tol / smax) - 1.0, math.log(math.log(4.0 / tol) + 2.0) + h, h)
    return np.exp(u), h * np.exp(u)


def _split_modes(cores, split, eps):
    """Rounding of a train in which core k (mode 2**split[k], or any mode when
    split[k] == 0) becomes split[k] cores of mode 2, most significant bit first;
    every discarded tail is within eps * ||x|| / sqrt(number of bonds)."""
    cs = [np.array(c) for c in cores]
    n = len(cs)
    for k in range(n - 1, 0, -1):
        r, p, r2 = cs[k].shape
        Q, R = np.linalg.qr(cs[k].reshape(r, p * r2).T)
        cs[k] = Q.T.reshape(Q.shape[1], p, r2)
        cs[k - 1] = np.tensordot(cs[k - 1], R.T, axes=(2, 0))
    bonds = sum(max(m, 1) for m in split) - 1
    delta = eps * np.linalg.norm(cs[0]) / math.sqrt(max(bonds, 1))
    out = []
    for k in range(n):
        r, p, r2 = cs[k].shape
        pm = [2] * split[k] if split[k] > 0 else [p]
        rest = cs[k].reshape(r, -1)
        for j, q in enumerate(pm):
            rows = rest.reshape(r * q, -1)
            if k == n - 1 and j == len(pm) - 1:
                out.append(rows.reshape(r, q, r2))
                break
            U, sv, Vt = _svd_wide(rows)
            l = _keep(sv, delta)
            out.append(U[:, :l].reshape(r, q, l))
            rest = sv[:l, None] * Vt[:l]
            r = l
        if k < n - 1:
            cs[k + 1] = np.tensordot(rest, cs[k + 1], axes=(1, 0))
    return out


def green_tt_expsum(L, k0, eps=1e-10, log=None):
    """The operator of green_tt without its dense 9 N^3 array (grids beyond 256^3).

    Gamma_ab(q) = q_a q_b / (k0 |q|^2) with 1/|q|^2 as an exponential sum, so
    that every term is a product of one function per axis (the momentum order
    of green_momentum_dense).  Gamma(0) = 0 through the factor q_a q_b, and a
    Nyquist frequency on any axis zeroes every term through a per-axis
    indicator.  Each component's sum is compressed at the level of the three
    axis groups, the nine components are stacked behind the component core,
    and the axis cores are split into their L bits."""
    N = 2 ** L
    f = signed_freq(N)[bit_reversal(L)]
    keep = (f != -N // 2).astype(np.float64)
    t, w = _inv_expsum(3.0 * (N // 2) ** 2, eps * 1e-3)
    E = np.exp(-np.outer(f * f, t)) * keep[:, None]
    P = [E, E * f[:, None], E * (f * f)[:, None]]        # q_d^0, q_d^1, q_d^2 in each term
    M = len(t)
    comps = []
    for a in range(3):
        for b in range(3):
            pw = [(a == d) + (b == d) for d in range(3)]
            X = (P[pw[0]] * (w / k0)[None, :])[None, :, :]
            Y = np.zeros((M, N, M))
            Y[np.arange(M), :, np.arange(M)] = P[pw[1]].T
            Z = P[pw[2]].T[:, :, None]
            comps.append(compress([X, Y, Z], eps * 1e-3))
            if log:
                log(f"Green component {3 * a + b + 1}/9")
    R1 = np.cumsum([0] + [c[0].shape[2] for c in comps])
    R2 = np.cumsum([0] + [c[1].shape[2] for c in comps])
    ctrl = np.eye(9).reshape(1, 9, 9)
    X = np.zeros((9, N, R1[-1]))
    Y = np.zeros((R1[-1], N, R2[-1]))
    Z = np.zeros((R2[-1], N, 1))
    for c, (cx, cy, cz) in enumerate(comps):
        X[c, :, R1[c]:R1[c + 1]] = cx[0]
        Y[R1[c]:R1[c + 1], :, R2[c]:R2[c + 1]] = cy
        Z[R2[c]:R2[c + 1]] = cz
    big = compress([ctrl, X, Y, Z], eps * 1e-2)
    if log:
        log("Green axis-group train")
    cores = compress(_split_modes(big, [0, L, L, L], eps * 1e-1), eps)
    ctl = cores[0].reshape(1, 3, 3, cores[0].shape[2])
    return [ctl.astype(np.complex128)] + [c.astype(np.complex128) for c in cores[1:]]


# ------------------------------------------------------- linear elasticity

# Voigt order of the strain / stress components: (11, 22, 33, 23, 13, 12)
VOIGT_PAIRS = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


def voigt_green_momentum(L, lam0, mu0):
    """Green-Eshelby operator of the isotropic reference medium (lam0, mu0) as a
    6 x 6 Voigt matrix per frequency, G[a, b, x', y', z'] in the momentum order
    of green_momentum_dense (position x' holds frequency rev(x')): strain a
    (engineering shears) of a unit stress-like polarization b.  With
    K^-1 = (I - c q q^T / |q|^2) / (mu0 |q|^2), c = (lam0 + mu0) / (lam0 + 2 mu0),
    the strain is eps_ij = (q_i (K^-1 tau q)_j + q_j (K^-1 tau q)_i) / 2; zero at
    q = 0 and on Nyquist frequencies."""
    N = 2 ** L
    f = signed_freq(N)[bit_reversal(L)]
    q = [f[:, None, None], f[None, :, None], f[None, None, :]]
    q2 = q[0] ** 2 + q[1] ** 2 + q[2] ** 2
    bad = (q2 == 0) | (q[0] == -N // 2) | (q[1] == -N // 2) | (q[2] == -N // 2)
    s2 = np.where(bad, 1.0, q2)
    c = (lam0 + mu0) / (lam0 + 2.0 * mu0)

    def kinv(m, k):
        return (float(m == k) - c * q[m] * q[k] / s2) / (mu0 * s2)

    G = np.zeros((6, 6, N, N, N))
    for a, (i, j) in enumerate(VOIGT_PAIRS):
        scale = 1.0 if i == j else 2.0
        for b, (k, l) in enumerate(VOIGT_PAIRS):
            pairs = [(k, l)] if k == l else [(k, l), (l, k)]
            acc = 0.0
            for kk, ll in pairs:
                acc = acc + 0.5 * (q[i] * kinv(j, kk) + q[j] * kinv(i, kk)) * q[ll]
            G[a, b] = np.where(bad, 0.0, scale * acc)
    return G


def green_tt_elastic(L, lam0, mu0, eps=1e-12):
    """Green operator (component core (1, 6, 6, r), diagonal spatial cores) and
    G2 = G^T G per frequency (the exact ||G t||^2 = <t, G2 t>), dense builds."""
    G = voigt_green_momentum(L, lam0, mu0)
    G2 = np.einsum("ca...,cb...->ab...", G, G)
    out = []
    for A in (G, G2):
        cores = ttsvd(A.reshape(-1), [36] + [2] * (3 * L), eps)
        ctrl = cores[0].reshape(1, 6, 6, cores[0].shape[2])
        out.append([ctrl.astype(np.complex128)] + [c.astype(np.complex128) for c in cores[1:]])
    return out[0], out[1]


def _voigt_blocks():
    A = np.zeros((6, 6))
    A[:3, :3] = 1.0                            # lam: trace coupling
    B = np.diag([2.0, 2.0, 2.0, 1.0, 1.0, 1.0])  # mu: 2 mu eps (engineering shears)
    return A, B


def _field_operator(fields, mats, eps):
    """Operator cores of sum_t mats[t] (x) fields[t](x): component core
    (1, 6, 6, r) and diagonal spatial cores, from one TT-SVD of the stacked fields."""
    F = np.stack([np.asarray(f, dtype=np.float64) for f in fields])
    L = int(round(math.log2(F.shape[1])))
    cores = ttsvd(F.reshape(-1), [len(fields)] + [2] * (3 * L), eps)
    first = cores[0][0]                         # (t, r1)
    ctrl = np.einsum("tab,tr->abr", np.stack(mats), first)[None]
    return [ctrl.astype(np.complex128)] + [c.astype(np.complex128) for c in cores[1:]]


def _field_rows(fields, rows, eps):
    """Trains of sum_t rows[t] (x) fields[t](x) with a component core (1, 6, r)."""
    F = np.stack([np.asarray(f, dtype=np.float64) for f in fields])
    L = int(round(math.log2(F.shape[1])))
    cores = ttsvd(F.reshape(-1), [len(fields)] + [2] * (3 * L), eps)
    first = cores[0][0]
    ctrl = np.einsum("ta,tr->ar", np.stack(rows), first)[None]
    return [ctrl.astype(np.complex128)] + [c.astype(np.complex128) for c in cores[1:]]


def build_problem_elastic(lam, mu, lam0=None, mu0=None, op_eps=1e-10, sfft_eps=1e-13,
                          green_eps=1e-12, log=None):
    """Host trains of one linear-elasticity cell problem (Sec. 3.1, App. A) on an
    N^3 grid of isotropic voxels (Lame parameters lam, mu): the field is the
    Voigt strain (component core of mode 6), the material acts through the
    Voigt operator C - C0 = (lam - lam0) A + (mu - mu0) B (A the trace
    coupling, B = diag(2, 2, 2, 1, 1, 1)), the reference medium defaults to the
    midpoints of the phase ranges.  k_sel[c] holds row c of C, so that
    Re <k_sel[c], eps> / N^3 is the mean stress component c."""
    say = log or (lambda msg: None)
    lam = np.asarray(lam, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    lam0 = 0.5 * (lam.min() + lam.max()) if lam0 is None else float(lam0)
    mu0 = 0.5 * (mu.min() + mu.max()) if mu0 is None else float(mu0)
    L = int(round(math.log2(lam.shape[0])))
    A, B = _voigt_blocks()
    dl, dm = lam - lam0, mu - mu0
    Kp = _field_operator([dl, dm], [A, B], op_eps)
    # (C - C0)^T (C - C0) = dl^2 A^2 + dl dm (A B + B A) + dm^2 B^2
    K2 = _field_operator([dl * dl, dl * dm, dm * dm], [A @ A, A @ B + B @ A, B @ B],
                         op_eps * 1e-2)
    ksel = [_field_rows([lam, mu], [A[c], B[c]], op_eps) for c in range(6)]
    say(f"elastic material operators, C - C0 rank {max(c.shape[0] for c in Kp)}")
    S, Sinv = sfft_3d(L, sfft_eps, d=6)
    G, G2 = green_tt_elastic(L, lam0, mu0, green_eps)
    say(f"Green-Eshelby operator, rank {max(c.shape[0] for c in G)}")
    return {"kind": "elastic", "L": L, "k0": 1.0, "lam0": lam0, "mu0": mu0, "Kp_op": Kp,
            "K2_op": K2, "k_sel": ksel, "S": S, "Sinv": Sinv, "G": G, "G2": G2}


# ------------------------------------------------------- material, loads

def material_tt(kvox, shift=0.0, eps=1e-10):
    """Spatial train of (k - shift) on an N^3 grid (x bits, y bits, z bits, MSB first)."""
    N = kvox.shape[0]
    L = int(round(math.log2(N)))
    return ttsvd(np.asarray(kvox, dtype=np.float64) - shift, [2] * (3 * L), eps)


def material_tt_z_invariant(section, shift=0.0, eps=1e-10):
    """k(x, y, z) = section(x, y): train of the section followed by all-ones z cores."""
    N = section.shape[0]
    L = int(round(math.log2(N)))
    sp = ttsvd(np.asarray(section, dtype=np.float64) - shift, [2] * (2 * L), eps)
    return sp + [np.ones((1, 2, 1)) for _ in range(L)]


def material_tt_periodic(cell, L, shift=0.0, eps=1e-10):
    """Spatial train of (k - shift) on a 2^L grid tiled by a periodic cell of
    side 2^pL: k depends on the low pL bits of each axis only, so each axis
    group is L - pL free top bits (identity on the bond, mode 2) followed by
    the cell's own cores for that axis."""
    M = cell.shape[0]
    pL = int(round(math.log2(M)))
    sp = ttsvd(np.asarray(cell, dtype=np.float64) - shift, [2] * (3 * pL), eps)
    out = []
    for d in range(3):
        r = sp[d * pL].shape[0]
        free = np.repeat(np.eye(r)[:, None, :], 2, axis=1)
        out += [free.copy() for _ in range(L - pL)] + sp[d * pL:(d + 1) * pL]
    return out


def with_component_core(spatial, control):
    """Prepend a (1, d, 1) component core (d = len(control)) to a spatial train."""
    ctl = np.asarray(control, dtype=np.complex128)
    return [ctl.reshape(1, ctl.size, 1)] + [c.astype(np.complex128) for c in spatial]


def apply_mpo(op, x):
    """Cores of A x for operator cores (r, p_out, p_in, r') and train cores (s, p_in, s')."""
    out = []
    for A, X in zip(op, x):
        c = np.einsum("aijc,bjd->abicd", A, X)
        out.append(c.reshape(A.shape[0] * X.shape[0], A.shape[1], A.shape[3] * X.shape[2]))
    return out


def mean_field(E, L):
    return with_component_core([np.ones((1, 2, 1)) for _ in range(3 * L)], E)


def build_problem(kvox=None, k0=None, L=None, section=None, op_eps=1e-10, sfft_eps=1e-13,
                  shared=None, cell=None, log=None, green_eps=None, green=None):
    """All host trains of one cell problem (k given as N^3 voxels, a z-invariant
    section, or a periodic cell tiling a 2^L grid).

    shared: the "S", "Sinv" and "G" entries of an earlier problem with the same L and
    k0, reused instead of rebuilt (they do not depend on the microstructure).
    green_eps: compression tolerance of the Green operator.  The product-aware
    rounding takes ||G t||^2 = <t, G t> / k0, an identity of the exact operator
    (k0 G is a projector); the compressed one misses it by about 1e-3 of its
    tolerance relative to ||G t||^2 (1.5e-13 at 1e-10 on 32^3, 5e-16 at 1e-12).
    Default: min(op_eps, 1e-12) for the dense build (L <= 8, same set-up time), which
    keeps that floor far below eps^2 = 1e-12 of a field tolerance of 1e-6; op_eps
    for the exponential-sum build (L > 8), whose set-up time triples at 1e-12
    (the floor, ~1e-13 of ||G t||^2, is then below the rank-capped errors of
    those workloads by ten orders of magnitude).
    green: how the Green operator is built: "dense" (TT-SVD of its 9 N^3 array),
    "expsum" (exponential sums per axis, then split into bits) or "cross"
    (cross interpolation of its entry formula); default dense up to 256^3,
    expsum up to 1024^3, cross beyond.
    log: optional callable taking a progress message."""
    say = log or (lambda msg: None)
    if kvox is not None:
        sp_k = material_tt(kvox, 0.0, op_eps)
        sp_kp = material_tt(kvox, k0, op_eps)
        sp_k2 = material_tt((np.asarray(kvox, dtype=np.float64) - k0) ** 2, 0.0, op_eps * 1e-2)
        L = int(round(math.log2(kvox.shape[0])))
    elif cell is not None:
        # a 2^L grid tiled by a periodic cell (L given)
        sp_k = material_tt_periodic(cell, L, 0.0, op_eps)
        say(f"material train k, rank {max(c.shape[0] for c in sp_k)}")
        sp_kp = material_tt_periodic(cell, L, k0, op_eps)
        say(f"material train k', rank {max(c.shape[0] for c in sp_kp)}")
        sp_k2 = material_tt_periodic((np.asarray(cell, dtype=np.float64) - k0) ** 2, L, 0.0,
                                     op_eps * 1e-2)
    else:
        sp_k = material_tt_z_invariant(section, 0.0, op_eps)
        sp_kp = material_tt_z_invariant(section, k0, op_eps)
        sp_k2 = material_tt_z_invariant((np.asarray(section, dtype=np.float64) - k0) ** 2, 0.0,
                                        op_eps * 1e-2)
        L = int(round(math.log2(section.shape[0])))
    say(f"material trains, k' rank {max(c.shape[0] for c in sp_kp)}")
    kp = with_component_core(sp_kp, np.ones(3))
    ksel = [with_component_core(sp_k, np.eye(3)[c]) for c in range(3)]
    # (k')^2 for the exact norm ||k' e||^2 = <e, diag((k')^2) e>
    k2 = with_component_core(sp_k2, np.ones(3))
    if shared is not None:
        S, Sinv, G = shared["S"], shared["Sinv"], shared["G"]
    else:
        S, Sinv = sfft_3d(L, sfft_eps)
        say("SFFT operator")
        # the dense Green array has 9 N^3 entries: beyond 256^3 the
        # exponential-sum build (same operator, same ranks)
        how = green or ("dense" if L <= 8 else "expsum" if L <= 10 else "cross")
        geps = green_eps if green_eps is not None else (min(op_eps, 1e-12) if how == "dense"
                                                        else op_eps)
        if how == "dense":
            G = green_tt(L, k0, geps)
        elif how == "expsum":
            G = green_tt_expsum(L, k0, geps, log=say)
        else:
            from .cross import green_tt_cross
            G, cinfo = green_tt_cross(L, k0, geps, log=say)
            say(f"Green operator by cross: {cinfo['sweeps']} sweeps, {cinfo['evaluations']} "
                f"entries, sampled max error {cinfo['sampled_max_error']:.1e}")
        say(f"Green operator, rank {max(c.shape[0] for c in G)}")
    return {"L": L, "k0": float(k0), "kp": kp, "k2": k2, "k_sel": ksel, "S": S, "Sinv": Sinv,
            "G": G}


def upload(prob, loads, max_rank, device=0):
    """Device operands for a batch of loads (rows of `loads`) plus an empty field batch."""
    from . import qtt
    L = prob["L"]
    B = len(loads)
    n = 3 * L + 1
    G2 = None
    if prob.get("kind") == "elastic":
        # Voigt operators with full 6 x 6 component cores; no scalar material train
        kp = None
        Kp = qtt.DeviceMPO.from_cores(prob["Kp_op"], [0] + [1] * (n - 1), device=device)
        K2 = qtt.DeviceMPO.from_cores(prob["K2_op"], [0] + [1] * (n - 1), device=device)
        G2 = qtt.DeviceMPO.from_cores(prob["G2"], [0] + [1] * (n - 1), device=device)
    else:
        kp = qtt.DeviceTT.from_cores(prob["kp"], device=device)
        Kp = qtt.DeviceMPO.from_cores(prob["kp"], [1] * n, device=device)
        K2 = qtt.DeviceMPO.from_cores(prob["k2"], [1] * n, device=device)
    S = qtt.DeviceMPO.from_cores(prob["S"], device=device)
    Sinv = qtt.DeviceMPO.from_cores(prob["Sinv"], device=device)
    G = qtt.DeviceMPO.from_cores(prob["G"], [0] + [1] * (n - 1), device=device)
    E = qtt.DeviceTT.from_cores([mean_field(np.asarray(Ej, dtype=float), L) for Ej in loads],
                                device=device)
    ksel = [qtt.DeviceTT.from_cores(c, device=device) for c in prob["k_sel"]]
    E_norm = np.array([np.linalg.norm(Ej) for Ej in loads], dtype=np.float64)
    # S E (rank 1: the constant field maps onto the zero frequency)
    SE = qtt.DeviceTT.from_cores(
        [compress(apply_mpo(prob["S"], mean_field(np.asarray(Ej, dtype=float), L)), 1e-14)
         for Ej in loads], device=device)
    ops = qtt.DeviceOperands(L, kp, Kp, K2, prob["k0"], S, Sinv, G, E, E_norm, ksel, SE, G2)
    modes, cap = qtt.field_capacity(L, max_rank, len(loads[0]))
    e = qtt.DeviceTT.empty(modes, cap, B, device)
    return ops, e


def upload_batch(probs, loads, max_rank, device=0):
    """Device operands for several microstructures (one `build_problem` each, equal L
    and k0) times the same loads: field b = instance * len(loads) + load.  k' and (k')^2
    are per-instance operators (zero-padded to common ranks); S, S^H and the Green
    operator are shared; E, S E and the k selectors are per field."""
    from . import qtt
    L = probs[0]["L"]
    k0 = probs[0]["k0"]
    if any(p["L"] != L or p["k0"] != k0 for p in probs):
        raise ValueError("instances must share L and k0")
    nl = len(loads)
    n = 3 * L + 1
    Kp = qtt.DeviceMPO.from_cores([p["kp"] for p in probs], [1] * n, device=device,
                                  inst_group=nl)
    K2 = qtt.DeviceMPO.from_cores([p["k2"] for p in probs], [1] * n, device=device,
                                  inst_group=nl)
    S = qtt.DeviceMPO.from_cores(probs[0]["S"], device=device)
    Sinv = qtt.DeviceMPO.from_cores(probs[0]["Sinv"], device=device)
    G = qtt.DeviceMPO.from_cores(probs[0]["G"], [0] + [1] * (n - 1), device=device)
    fields = [np.asarray(Ej, dtype=float) for _ in probs for Ej in loads]
    E = qtt.DeviceTT.from_cores([mean_field(Ej, L) for Ej in fields], device=device)
    SE = qtt.DeviceTT.from_cores(
        [compress(apply_mpo(probs[0]["S"], mean_field(Ej, L)), 1e-14) for Ej in fields],
        device=device)
    ksel = [qtt.DeviceTT.from_cores([p["k_sel"][c] for p in probs for _ in loads], device=device)
            for c in range(3)]
    kp = qtt.DeviceTT.from_cores(probs[0]["kp"], device=device)   # plain path only
    E_norm = np.array([np.linalg.norm(Ej) for Ej in fields], dtype=np.float64)
    ops = qtt.DeviceOperands(L, kp, Kp, K2, k0, S, Sinv, G, E, E_norm, ksel, SE)
    modes, cap = qtt.field_capacity(L, max_rank)
    e = qtt.DeviceTT.empty(modes, cap, len(fields), device)
    return ops, e
