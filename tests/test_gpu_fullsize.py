"""Parity at the benchmarked sizes against the dense Moulinec-Suquet oracle.

256^3 sphere (25 cores, field rank cap 64, eps 1e-6, oversample 4: the
launch configuration of `bench.py --config sphere256`): the cap binds hard, so
the TT iterates are not the dense ones.  Each product-aware rounding reports
its exact a-posteriori error (||x - x~||^2 = ||x||^2 - ||x~||^2 of the
orthogonal projection), and those errors propagate through the iteration to a
rigorous bound on the distance from the dense iterate (tests/sketch_chain.py):
after the first iteration from E, ||e_1 - e_1*|| <= a_4; after the second,
||e_2 - e_2*|| <= rho ||e_1 - e_1*|| + a_4', with rho = max|k - k0| / k0 the
contraction factor of the basic scheme.  A wrong operator, bit order or
product would be off by O(1) and fail; the test also asserts that the bound
is not vacuous (below 0.5 of the iterate's norm).

64 x 128^3 boxes (the batched workload's first 4 instances x 3 loads = 12
fields in one batch, rank cap 96, eps 1e-6, oversample 4): 12 batched
iterations against 12 dense iterations of each field, with the bound
propagated over the iterations (D_m = rho D_{m-1} + a_4 of iteration m); and
the effective-conductivity columns after those iterations against the dense
ones within the bound's effect on the mean flux (Cauchy-Schwarz).
"""
import math

import numpy as np
import pytest

from oracle import ms
from oracle import tt as T
from paper_2512_07811_amd import inputs as I

import sketch_chain as SC

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    from paper_2512_07811_amd import qtt
    return qtt


def dense_field(q, e):
    """The (3, N, N, N) array of a device field (batch 1)."""
    cores = e.to_cores()[0]
    L = (len(cores) - 1) // 3
    N = 2 ** L
    return T.full(cores).reshape(3, N, N, N)


@pytest.mark.timeout(600)
def test_sphere256_two_iterates_within_propagated_rounding_bound(q):
    from paper_2512_07811_amd import operands as P
    L, k0, rmax, eps, os_ = 8, 50.5, 64, 1e-6, 4
    kvox = I.sphere(L, 0.2, 100.0, 1.0)
    rho = float(np.max(np.abs(kvox - k0)) / k0)
    prob = P.build_problem(kvox=kvox, k0=k0)
    E = [1.0, 0.0, 0.0]
    ctx = q.Context(0)
    try:
        ops, e = P.upload(prob, [E], rmax)
        e = q.DeviceTT.from_cores([P.mean_field(np.asarray(E), L)], e.cap)
        dense = np.zeros((3,) + kvox.shape)
        dense[0] = 1.0
        prev_dist = 0.0
        for it in range(2):
            print(f"[fullsize] sphere256 iterate {it + 1}", flush=True)
            e, steps = SC.sketch_iteration(q, ctx, ops, e, eps, rmax, os_, seed=41 + 10 * it)
            assert int(e.rank_array().max()) <= rmax
            bound = rho * prev_dist + float(SC.propagated_bound(steps, k0)[0])
            dense = ms.ms_step(dense, kvox, k0, E)
            got = dense_field(q, e)
            nrm = float(np.linalg.norm(dense))
            dist = float(np.linalg.norm(got - dense))
            print(f"  errors {[round(float(s[0][0]), 5) for s in steps]}  distance {dist / nrm:.4f}  "
                  f"bound {bound / nrm:.4f}  imag {np.linalg.norm(got.imag) / nrm:.2e}", flush=True)
            assert dist <= bound * (1 + 1e-8) + 1e-9 * nrm
            assert bound <= 0.5 * nrm
            prev_dist = dist
            del got
    finally:
        ctx.close()


@pytest.mark.timeout(900)
def test_boxes128_batched_iterates_track_dense(q):
    from paper_2512_07811_amd import operands as P
    L, k0, rmax, eps, os_, iters = 7, 25.5, 96, 1e-6, 4, 12
    loads = [[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]]
    vox = [I.random_boxes(L, 1000 + i) for i in range(4)]
    first = P.build_problem(kvox=vox[0], k0=k0)
    shared = {k: first[k] for k in ("S", "Sinv", "G")}
    probs = [first] + [P.build_problem(kvox=v, k0=k0, shared=shared) for v in vox[1:]]
    ctx = q.Context(0)
    try:
        ops, e = P.upload_batch(probs, loads, rmax)
        fields = [(i, E) for i in range(len(vox)) for E in loads]
        e = q.DeviceTT.from_cores([P.mean_field(np.asarray(E), L) for _, E in fields], e.cap)
        rho = np.array([float(np.max(np.abs(vox[i] - k0)) / k0) for i, _ in fields])
        D = np.zeros(len(fields))     # propagated bound on ||e_m - e_m*|| per field
        print(f"[fullsize] boxes128 x{len(fields)} fields, {iters} iterations", flush=True)
        for it in range(iters):
            e, steps = SC.sketch_iteration(q, ctx, ops, e, eps, rmax, os_, seed=101 + 10 * it)
            D = rho * D + SC.propagated_bound(steps, k0)
        worst_err = max(float(np.max(s[0])) for s in steps)
        got = e.to_cores()
        for b, (i, E) in enumerate(fields):
            kv = vox[i]
            d = np.zeros((3,) + kv.shape)
            d += np.asarray(E).reshape(3, 1, 1, 1)
            for _ in range(iters):
                d = ms.ms_step(d, kv, k0, E)
            g = T.full(got[b]).reshape(d.shape)
            nrm = float(np.linalg.norm(d))
            dist = float(np.linalg.norm(g - d))
            A_gpu = np.array([np.mean(kv * g[c].real) for c in range(3)])
            A_ref = ms.effective_column(kv, d)
            print(f"  field {b}: distance {dist / nrm:.2e} (bound {D[b] / nrm:.2e}), A_eff rel "
                  f"diff {np.linalg.norm(A_gpu - A_ref) / np.linalg.norm(A_ref):.2e}", flush=True)
            assert dist <= D[b] * (1 + 1e-8) + 1e-9 * nrm
            # mean flux: |<k (g - d)>| <= rms(k) ||g - d|| / sqrt(N^3)
            rms = float(np.sqrt(np.mean(kv ** 2)))
            assert np.linalg.norm(A_gpu - A_ref) <= rms * dist / math.sqrt(kv.size) * (1 + 1e-8)
        print(f"  largest rounding error of the last iteration {worst_err:.2e}", flush=True)
    finally:
        ctx.close()
