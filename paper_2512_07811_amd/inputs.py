"""Seeded synthetic inputs shared by the oracle, the tests and the bench.

This module holds no arithmetic of the homogenization method: it only draws
microstructures (voxel conductivity arrays), random tensor-train cores and
Gaussian sketch cores from numpy's PCG64 generator.  Both the CPU oracle and
the HIP path receive the same arrays from here.

Voxel convention: voxel index i on an axis of N = 2**L points has its centre
at (i + 1/2) in voxel units; arrays are indexed [x, y, z].
"""
from __future__ import annotations

import math

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------- geometries

def laminate(L: int, layers: int = 4, k_lo: float = 1.0, k_hi: float = 10.0,
             axis: int = 0) -> np.ndarray:
    """Two-phase laminate, equal layers normal to `axis`, k_lo first."""
    N = 2 ** L
    if N % layers:
        raise ValueError("layers must divide N")
    idx = np.arange(N) // (N // layers)
    k1 = np.where(idx % 2 == 0, k_lo, k_hi)
    shape = [1, 1, 1]
    shape[axis] = N
    return np.broadcast_to(k1.reshape(shape), (N, N, N)).astype(np.float64).copy()


def sphere(L: int, frac: float = 0.2, k_in: float = 100.0, k_out: float = 1.0) -> np.ndarray:
    """Centred sphere of nominal volume fraction `frac` (voxel-centre test)."""
    N = 2 ** L
    R = N * (3.0 * frac / (4.0 * math.pi)) ** (1.0 / 3.0)
    c = (np.arange(N) + 0.5) - N / 2.0
    d2 = c[:, None, None] ** 2 + c[None, :, None] ** 2 + c[None, None, :] ** 2
    return np.where(d2 <= R * R, k_in, k_out).astype(np.float64)


def random_boxes(L: int, seed: int, n_min: int = 1, n_max: int = 8,
                 edge_min: int = 8, edge_max: int = 48,
                 k_min: float = 5.0, k_max: float = 50.0, k_matrix: float = 1.0) -> np.ndarray:
    """Periodic axis-aligned boxes, half-open [p, p+l) mod N; later boxes overwrite."""
    N = 2 ** L
    g = rng(seed)
    nb = int(g.integers(n_min, n_max + 1))
    k = np.full((N, N, N), k_matrix, dtype=np.float64)
    for _ in range(nb):
        edges = g.integers(edge_min, edge_max + 1, size=3)
        corner = g.integers(0, N, size=3)
        kb = float(g.uniform(k_min, k_max))
        ix = [(corner[a] + np.arange(edges[a])) % N for a in range(3)]
        k[np.ix_(ix[0], ix[1], ix[2])] = kb
    return k


def boxes_section(L: int, seed: int, n_min: int = 4, n_max: int = 12, edge_min: int = 8,
                  edge_max: int = 40) -> np.ndarray:
    """(N, N) phase indicator of periodic axis-aligned rectangles (1 inside,
    0 outside), half-open [p, p+l) mod N: the 2D box/multibox cells of the
    elasticity workload, repeated along z for a plane-strain cell."""
    N = 2 ** L
    g = rng(seed)
    nb = int(g.integers(n_min, n_max + 1))
    ph = np.zeros((N, N), dtype=np.float64)
    for _ in range(nb):
        edges = g.integers(edge_min, edge_max + 1, size=2)
        corner = g.integers(0, N, size=2)
        ix = [(corner[a] + np.arange(edges[a])) % N for a in range(2)]
        ph[np.ix_(ix[0], ix[1])] = 1.0
    return ph


def cylinders_section(L: int, seed: int, count: int = 16, r_min: float = 20.0,
                      r_max: float = 40.0, k_in: float = 50.0, k_out: float = 1.0,
                      max_tries: int = 100000) -> np.ndarray:
    """(N, N) cross-section of z-parallel periodic cylinders without overlap.

    The 3D microstructure is this section repeated along z.
    """
    N = 2 ** L
    g = rng(seed)
    radii = g.uniform(r_min, r_max, size=count)
    centres = []
    tries = 0
    for r in radii:
        while True:
            tries += 1
            if tries > max_tries:
                raise RuntimeError("could not place cylinders without overlap")
            c = g.uniform(0, N, size=2)
            ok = True
            for (c2, r2) in centres:
                d = np.abs(c - c2)
                d = np.minimum(d, N - d)
                if math.hypot(d[0], d[1]) <= r + r2:
                    ok = False
                    break
            if ok:
                centres.append((c, r))
                break
    x = np.arange(N) + 0.5
    sec = np.full((N, N), k_out, dtype=np.float64)
    for (c, r) in centres:
        dx = np.abs(x - c[0]); dx = np.minimum(dx, N - dx)
        dy = np.abs(x - c[1]); dy = np.minimum(dy, N - dy)
        inside = dx[:, None] ** 2 + dy[None, :] ** 2 <= r * r
        sec[inside] = k_in
    return sec


def sphere_lattice_cell(period_L: int, rel_radius: float = 0.3, k_in: float = 20.0,
                        k_out: float = 1.0) -> np.ndarray:
    """One period (2**period_L)^3 of a simple-cubic lattice of centred spheres."""
    M = 2 ** period_L
    R = rel_radius * M
    c = (np.arange(M) + 0.5) - M / 2.0
    d2 = c[:, None, None] ** 2 + c[None, :, None] ** 2 + c[None, None, :] ** 2
    return np.where(d2 <= R * R, k_in, k_out).astype(np.float64)


# --------------------------------------------------------------- random TTs

def random_tt(modes, ranks, seed: int, is_complex: bool = True, scale: float = 1.0):
    """Cores of shape (ranks[k], modes[k], ranks[k+1]) with i.i.d. N(0, 1) entries.

    `ranks` has len(modes)+1 entries with ranks[0] = ranks[-1] = 1.
    """
    g = rng(seed)
    cores = []
    for k, p in enumerate(modes):
        shp = (ranks[k], p, ranks[k + 1])
        c = g.standard_normal(shp)
        if is_complex:
            c = c + 1j * g.standard_normal(shp)
        cores.append(scale * c / math.sqrt(ranks[k] * p))
    return cores


def random_mpo(modes_out, modes_in, ranks, seed: int, is_complex: bool = True):
    """Operator cores of shape (r, p_out, p_in, r') with i.i.d. normal entries."""
    g = rng(seed)
    cores = []
    for k, (po, pi) in enumerate(zip(modes_out, modes_in)):
        shp = (ranks[k], po, pi, ranks[k + 1])
        c = g.standard_normal(shp)
        if is_complex:
            c = c + 1j * g.standard_normal(shp)
        cores.append(c / math.sqrt(ranks[k] * pi))
    return cores


def gaussian_sketch(modes, ells, seed: int):
    """Real Gaussian sketch cores (ells[k], modes[k], ells[k+1]), ells[0]=ells[-1]=1."""
    g = rng(seed)
    return [g.standard_normal((ells[k], p, ells[k + 1])) for k, p in enumerate(modes)]


def graded_tt(modes, ranks, decay: float, seed: int, is_complex: bool = True):
    """Random TT whose bond spectra decay geometrically (for truncation tests).

    Built as left-orthonormal random cores with the last core scaled, and each
    bond weighted by decay**j on its j-th rank index.
    """
    g = rng(seed)
    cores = []
    for k, p in enumerate(modes):
        shp = (ranks[k], p, ranks[k + 1])
        c = g.standard_normal(shp)
        if is_complex:
            c = c + 1j * g.standard_normal(shp)
        w = decay ** np.arange(ranks[k + 1])
        cores.append(c * w[None, None, :] / math.sqrt(ranks[k] * p))
    return cores


def mlp_init(n_in: int, n_cls: int, seed: int, hidden: int = 64, layers: int = 3):
    """Initial MLP weights: W_i ~ N(0, 1/fan_in) of shape (fan_in, fan_out), b_i = 0.

    Returned as the list [W0, b0, W1, b1, ...] in float64."""
    g = rng(seed)
    dims = [n_in] + [hidden] * layers + [n_cls]
    out = []
    for i in range(len(dims) - 1):
        out.append(g.standard_normal((dims[i], dims[i + 1])) * math.sqrt(1.0 / dims[i]))
        out.append(np.zeros(dims[i + 1]))
    return out
