"""One product-aware LS iteration (Algorithm 2 as ls_iterate runs it in the
sketch mode) assembled from the C-ABI calls, so that a test sees every
rounding's reported error and norm, plus the error bound these propagate to.

Steps and the exact norms of the products (the same identities the solver
uses): tau = R(k' e), ||k' e||^2 = <e, K2 e>; tau^ = R(S tau), ||S tau|| =
||tau||; eps^ = R(G tau^), ||G t||^2 = <t, G t>/k0; e' = R(S^H (S E - eps^)),
||S E - eps^||^2 by environments.

Bound: with a_s the absolute error after step s against the same chain with
exact roundings, a_1 = err_1 ||x_1||, a_2 = a_1 + err_2 ||x_2|| (S unitary),
a_3 = a_2 / k0 + err_3 ||x_3|| (k0 G is an orthogonal projector, so
||G|| = 1/k0), a_4 = a_3 + err_4 ||x_4||: the iterate is within a_4 of the
exact iterate of the same input (operators exact to their set-up tolerance).
"""
import dataclasses
import numpy as np


def natural_caps(modes):
    n = len(modes)
    return [1] + [int(min(np.prod(modes[:k], dtype=float), np.prod(modes[k:], dtype=float)))
                  for k in range(1, n)] + [1]


def _cap(modes, r):
    return [min(c, r) for c in natural_caps(modes)]


def _view(t, cap):
    return dataclasses.replace(t, cap=np.ascontiguousarray(np.asarray(cap, dtype=np.int32)))


def sketch_iteration(q, ctx, ops, e, eps, rmax, oversample, seed):
    """One iteration from the field batch e; returns (e', steps) with
    steps = [(err_s, ||x_s||)] for the four roundings, host arrays [batch]."""
    modes = list(e.modes)
    wide = _cap(modes, rmax + oversample)
    field = _cap(modes, rmax)
    steps = []

    def rnd(A, y, xn2, s):
        out = q.DeviceTT.empty(modes, wide, y.batch)
        err, _ = q.tt_sketch_round(ctx, A, y, xn2, out, eps=eps, max_rank=rmax,
                                   mode=q.ROUND_SKETCH, oversample=oversample, seed=seed + s)
        ctx.sync()
        steps.append((err.cpu().numpy().copy(), np.sqrt(xn2.cpu().numpy())))
        return _view(out, field)

    t1 = rnd(ops.Kp, e, q.tt_sandwich(ctx, ops.K2, e, 1.0), 0)
    n1 = q.tt_dot(ctx, t1, t1).real.contiguous()
    t2 = rnd(ops.S, t1, n1, 1)
    t3 = rnd(ops.G, t2, q.tt_sandwich(ctx, ops.G, t2, 1.0 / ops.k0), 2)
    t = q.tt_add(ctx, 1.0, ops.SE, -1.0, t3)
    t4 = rnd(ops.Sinv, t, q.tt_dot(ctx, t, t).real.contiguous(), 3)
    return t4, steps


def propagated_bound(steps, k0):
    """a_4 of the module docstring (per instance)."""
    (e1, n1), (e2, n2), (e3, n3), (e4, n4) = steps
    a = e1 * n1
    a = a + e2 * n2
    a = a / k0 + e3 * n3
    return a + e4 * n4
