"""AMEn approximation of a TT x TTO product (oracle).  Test infrastructure only.

Hauck, Kabel, Gauger (arXiv 2512.07811), Sec. 2.1, the variational
alternative to contracting and then compressing: y ~ A x is built directly in
the TT format by sweeping over the cores, each core taken from the local
projection of A x, while the representation is enriched with an
approximation z of the residual A x - y (Dolgov and Savostyanov 2014, the
alternating minimal energy method); Algorithm 2 applies it to the Green
multiply, eps^ = A(Gamma^, tau^).

One sweep, left to right, with y and z right-orthogonal on entry (interfaces
Phi are contractions of conj(frame) x A x over the cores on one side):

  local solution   y_k = Phi^{yAx}_L (A_k x_k) Phi^{yAx}_R
  residual on z    z_k = Phi^{zAx}_L (A_k x_k) Phi^{zAx}_R
                         - Phi^{zy}_L y_k Phi^{zy}_R
  enrichment       e_k = Phi^{yAx}_L (A_k x_k) Phi^{zAx}_R - y_k Phi^{zy}_R
  new cores        y_k <- Q of QR([y_k | e_k]),  z_k <- Q of QR(z_k)
  the last core    y_{n-1} = local solution, z_{n-1} = residual projection.

Reading (the paper gives no further detail): each sweep ends with one TT
rounding of y at eps (the truncated-SVD sweep of Sec. 2.2 and its delta rule,
cap r_max), which leaves y right-orthogonal for the next sweep, and z is
right-orthogonalized by a QR sweep.  The initial y and z are inputs.
"""
from __future__ import annotations

import numpy as np

from . import tt as T


def orthogonalize_right(tt):
    """QR sweep right to left: cores 1..n-1 right-orthogonal (rows orthonormal)."""
    cores = [np.array(c, dtype=np.complex128) for c in tt]
    for k in range(len(cores) - 1, 0, -1):
        r, p, r2 = cores[k].shape
        Q, R = np.linalg.qr(cores[k].reshape(r, p * r2).T, mode="reduced")
        s = Q.shape[1]
        cores[k] = Q.T.reshape(s, p, r2)
        cores[k - 1] = np.tensordot(cores[k - 1], R.T, axes=(2, 0))
    return cores


def _c(spec, *ops):
    return np.einsum(spec, *ops, optimize=True)


def amen_mv(A, x, y0, z0, eps: float, rmax: int | None = None, sweeps: int = 2,
            return_info: bool = False):
    """y ~ A x for a TTO A (cores (ra, p, p, ra')) and a TT x, from the initial
    guess y0 and residual guess z0.  Returns y (and, with return_info, the
    relative change of y per sweep and its ranks)."""
    n = len(x)
    y = orthogonalize_right(y0)
    z = orthogonalize_right(z0)
    changes = []
    prev = None
    for _ in range(sweeps):
        one3 = np.ones((1, 1, 1), dtype=np.complex128)
        PyR = [None] * (n + 1)
        PzR = [None] * (n + 1)
        PzyR = [None] * (n + 1)
        PyR[n], PzR[n], PzyR[n] = one3, one3, np.ones((1, 1), dtype=np.complex128)
        for k in range(n - 1, 0, -1):
            Ak, xk = A[k], x[k]
            PyR[k] = _c("yiY,aijB,xjX,YBX->yax", np.conj(y[k]), Ak, xk, PyR[k + 1])
            PzR[k] = _c("ziZ,aijB,xjX,ZBX->zax", np.conj(z[k]), Ak, xk, PzR[k + 1])
            PzyR[k] = _c("ziZ,yiY,ZY->zy", np.conj(z[k]), y[k], PzyR[k + 1])
        PyL, PzL = one3, one3
        PzyL = np.ones((1, 1), dtype=np.complex128)
        ny, nz = [], []
        for k in range(n):
            Ak, xk = A[k], x[k]
            yk = _c("yax,aijB,xjX,YBX->yiY", PyL, Ak, xk, PyR[k + 1])
            zk = (_c("zax,aijB,xjX,ZBX->ziZ", PzL, Ak, xk, PzR[k + 1])
                  - _c("zy,yiY,ZY->ziZ", PzyL, yk, PzyR[k + 1]))
            if k == n - 1:
                ny.append(yk)
                nz.append(zk)
                break
            ek = (_c("yax,aijB,xjX,ZBX->yiZ", PyL, Ak, xk, PzR[k + 1])
                  - _c("yiY,ZY->yiZ", yk, PzyR[k + 1]))
            ry, p, rY = yk.shape
            Qy, _ = np.linalg.qr(np.concatenate([yk.reshape(ry * p, rY),
                                                 ek.reshape(ry * p, -1)], axis=1))
            Qy = Qy.reshape(ry, p, -1)
            rz, _, rZ = zk.shape
            Qz, _ = np.linalg.qr(zk.reshape(rz * p, rZ))
            Qz = Qz.reshape(rz, p, -1)
            ny.append(Qy)
            nz.append(Qz)
            PyL = _c("yax,yiY,aijB,xjX->YBX", PyL, np.conj(Qy), Ak, xk)
            PzL = _c("zax,ziZ,aijB,xjX->ZBX", PzL, np.conj(Qz), Ak, xk)
            PzyL = _c("zy,ziZ,yiY->ZY", PzyL, np.conj(Qz), Qy)
        y = T.round_tt(ny, eps, rmax)
        z = orthogonalize_right(nz)
        if prev is not None:
            d = T.norm(T.sub(y, prev)) / max(T.norm(y), 1e-300)
            changes.append(d)
        prev = y
    if return_info:
        return y, {"changes": changes, "ranks": T.ranks(y)}
    return y
