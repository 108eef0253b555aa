"""Dense Moulinec-Suquet basic scheme for linear elasticity (oracle).
Test infrastructure only.

Hauck, Kabel, Gauger (arXiv 2512.07811), Sec. 3.1 (the corrector problem,
eqs. local_strain, pol_force_eq, polarization_tensor, lippmann_schwinger,
green_conv_momentum) and Algorithm 1, on a periodic 3D grid of isotropic
phases (Lame parameters lam(x), mu(x)) with an isotropic reference medium
(lam0, mu0):

  eps_0 = E
  loop:  tau = (C - C0) : eps ;  tau^ = FFT(tau) ;
         eps_{m+1} = E - IFFT(Gamma_0^ tau^)

Gamma_0^(q) maps a stress-like tau^ to the strain of the displacement that
balances div(C0 grad^s u + tau) = 0: with the acoustic tensor
K(q)_ik = C0_ijkl q_j q_l = mu0 |q|^2 delta_ik + (lam0 + mu0) q_i q_k,
u^ = K(q)^-1 (tau^ q) (up to the factor i of the derivative, which cancels),
and Gamma_0^ tau^ = sym(q (x) u^).  Gamma_0^(0) = 0, and Gamma_0^ = 0 where a
frequency component equals -N/2 (Nyquist), as in the conductivity oracle.

Voigt notation (Appendix A): strain vector (e11, e22, e33, 2 e23, 2 e13,
2 e12) with engineering shears, stress vector (s11, s22, s33, s23, s13, s12),
so that sigma = C eps with the 6 x 6 matrix C and the energy is
sigma . eps / 2.  Unit loads E = e_j give column j of C_eff as the mean stress
<C eps^(j)> (eq. macro_ss).
"""
from __future__ import annotations

import numpy as np

from .ops import freqs

# Voigt index -> tensor index pair
VOIGT = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


def isotropic_voigt(lam, mu):
    """6 x 6 Voigt stiffness of an isotropic material (scalars)."""
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    for i in range(3):
        C[i, i] = lam + 2 * mu
        C[3 + i, 3 + i] = mu
    return C


def strain_tensor(ev):
    """Voigt strain (6, ...) with engineering shears -> symmetric tensor (3, 3, ...)."""
    t = np.empty((3, 3) + ev.shape[1:], dtype=ev.dtype)
    for a, (i, j) in enumerate(VOIGT):
        v = ev[a] if i == j else 0.5 * ev[a]
        t[i, j] = v
        t[j, i] = v
    return t


def stress_tensor(sv):
    """Voigt stress (6, ...) -> symmetric tensor (3, 3, ...)."""
    t = np.empty((3, 3) + sv.shape[1:], dtype=sv.dtype)
    for a, (i, j) in enumerate(VOIGT):
        t[i, j] = sv[a]
        t[j, i] = sv[a]
    return t


def strain_voigt(t):
    """Symmetric strain tensor -> Voigt vector with engineering shears."""
    return np.stack([t[i, j] if i == j else t[i, j] + t[j, i] for i, j in VOIGT])


def stress_apply(lam, mu, ev):
    """Voigt stress of an isotropic (possibly voxel-varying) material:
    sigma = lam tr(eps) I + 2 mu eps."""
    tr = ev[0] + ev[1] + ev[2]
    s = np.empty_like(ev)
    for a in range(3):
        s[a] = lam * tr + 2 * mu * ev[a]
    for a in range(3, 6):
        s[a] = mu * ev[a]
    return s


def gamma_strain(tau_v, q, lam0, mu0):
    """Strain (Voigt) of Gamma_0^ applied to the stress-like Voigt vector tau_v at
    frequencies q = (q1, q2, q3) (arrays of one shape, none all-zero)."""
    T = stress_tensor(tau_v)
    q2 = q[0] ** 2 + q[1] ** 2 + q[2] ** 2
    tq = [sum(T[i, j] * q[j] for j in range(3)) for i in range(3)]      # tau^ q
    # K^-1 v = (v - c q (q . v) / |q|^2) / (mu0 |q|^2), c = (lam0 + mu0) / (lam0 + 2 mu0)
    c = (lam0 + mu0) / (lam0 + 2 * mu0)
    qv = sum(q[i] * tq[i] for i in range(3))
    u = [(tq[i] - c * q[i] * qv / q2) / (mu0 * q2) for i in range(3)]
    eps = np.empty((3, 3) + np.shape(q2), dtype=np.result_type(tau_v, np.float64))
    for i in range(3):
        for j in range(3):
            eps[i, j] = 0.5 * (q[i] * u[j] + q[j] * u[i])
    return strain_voigt(eps)


def green_apply(tau_hat, lam0, mu0):
    """Strain (Voigt) Gamma_0^ tau^ for a stress-like tau^ (Voigt, (6, N, N, N))."""
    shape = tau_hat.shape[1:]
    q = np.meshgrid(*[freqs(n) for n in shape], indexing="ij")
    q2 = q[0] ** 2 + q[1] ** 2 + q[2] ** 2
    nyq = np.zeros(shape, dtype=bool)
    for g, n in zip(q, shape):
        nyq |= g == -n / 2
    zero = q2 == 0
    qs = [np.where(zero, 1.0, g) for g in q]           # placeholder where Gamma^ = 0
    ev = gamma_strain(tau_hat, qs, lam0, mu0)
    ev[:, zero] = 0.0
    ev[:, nyq] = 0.0
    return ev


def ms_step(ev, lam, mu, lam0, mu0, E):
    """One basic-scheme iteration on a dense Voigt strain field ev (6, N, N, N)."""
    tau = stress_apply(lam - lam0, mu - mu0, ev)
    th = np.fft.fftn(tau, axes=(1, 2, 3))
    fl = np.fft.ifftn(green_apply(th, lam0, mu0), axes=(1, 2, 3))
    Ev = np.asarray(E, dtype=np.float64).reshape(6, 1, 1, 1)
    return Ev - fl.real if np.isrealobj(ev) else Ev - fl


def solve(lam, mu, lam0, mu0, E, tol=1e-10, max_iter=2000):
    """Iterate from E until ||e_{m+1} - e_m|| / (|E| sqrt(N^3)) < tol; returns (eps, iters)."""
    ev = np.zeros((6,) + lam.shape)
    ev += np.asarray(E, dtype=np.float64).reshape(6, 1, 1, 1)
    for it in range(1, max_iter + 1):
        nw = ms_step(ev, lam, mu, lam0, mu0, E)
        r = np.linalg.norm(nw - ev) / (np.linalg.norm(E) * np.sqrt(lam.size))
        ev = nw
        if r < tol:
            return ev, it
    return ev, max_iter


def effective_column(lam, mu, ev):
    """Mean Voigt stress <C eps> (column j of C_eff for E = e_j)."""
    s = stress_apply(lam, mu, ev)
    return np.array([np.mean(s[a]) for a in range(6)])


def effective_tensor(lam, mu, lam0, mu0, tol=1e-10, max_iter=2000):
    cols = []
    for j in range(6):
        E = np.zeros(6)
        E[j] = 1.0
        ev, _ = solve(lam, mu, lam0, mu0, E, tol, max_iter)
        cols.append(effective_column(lam, mu, ev))
    return np.stack(cols, axis=1)


def laminate_closed_form(lams, mus, fracs):
    """Exact C_eff (Voigt) of isotropic layers normal to x1 with volume fractions fracs.

    In a laminate normal to x1 the in-plane strains e22, e33, 2 e23 and the
    traction components s11, s13, s12 are uniform across the layers.  With
    M = lam + 2 mu and <.> the layer average:
      C11 = 1/<1/M>,  C12 = C13 = <lam/M>/<1/M>,
      C22 = C33 = <M> - <lam^2/M> + <lam/M>^2/<1/M>,
      C23 = <lam> - <lam^2/M> + <lam/M>^2/<1/M>,
      C44 (23) = <mu>,  C55 (13) = C66 (12) = 1/<1/mu>."""
    lams, mus, f = map(np.asarray, (lams, mus, fracs))
    f = f / f.sum()
    av = lambda v: float(np.sum(f * v))  # noqa: E731
    M = lams + 2 * mus
    i1 = av(1.0 / M)
    lm = av(lams / M)
    l2 = av(lams ** 2 / M)
    C = np.zeros((6, 6))
    C[0, 0] = 1.0 / i1
    C[0, 1] = C[0, 2] = C[1, 0] = C[2, 0] = lm / i1
    C[1, 1] = C[2, 2] = av(M) - l2 + lm ** 2 / i1
    C[1, 2] = C[2, 1] = av(lams) - l2 + lm ** 2 / i1
    C[3, 3] = av(mus)
    C[4, 4] = C[5, 5] = 1.0 / av(1.0 / mus)
    return C
