"""The sphere-lattice pipeline of the 4096^3 workload at 64^3 (CPU build of the
periodic material and the cross-built Green operator, GPU iterations) against
the dense Moulinec-Suquet oracle on the exact reduction, the 16^3 period cell.

A field of the 64^3 grid tiled by a 16^3 cell is 16-periodic: it has only
frequencies that are multiples of 4, where the scale-free Green operator and
its Nyquist cut agree with the 16^3 grid's, so each iterate is the tiled
iterate of the cell.  With eps = 0 (no truncation) the TT iterates equal the
tiled dense iterates up to the operators' compression tolerances.
"""
import numpy as np
import pytest

from oracle import ms
from oracle import tt as T
from paper_2512_07811_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    from paper_2512_07811_amd import qtt
    return qtt


def test_lattice_iterates_equal_the_tiled_cell_iterates(q):
    # the product-aware rounding at eps = 0: sketch widths at the natural rank
    # bounds capture every product exactly (the materializing path's products,
    # Green rank 213 times the field's, exceed an SVD block here)
    from paper_2512_07811_amd import operands as P
    L, pL, k0 = 6, 4, 10.5
    cell = I.sphere_lattice_cell(pL, 0.3, 20.0, 1.0)
    prob = P.build_problem(cell=cell, L=L, k0=k0, op_eps=1e-12, green="cross",
                           green_eps=1e-11)
    E = [1.0, 0.0, 0.0]
    ctx = q.Context(0)
    try:
        ops, e = P.upload(prob, [E], 0)
        e = q.DeviceTT.from_cores([P.mean_field(np.asarray(E), L)], e.cap)
        opts = q.solve_opts(0.0, 0, mode=q.ROUND_SKETCH, oversample=8, seed=5)
        dense = np.zeros((3,) + cell.shape)
        dense[0] = 1.0
        reps = 2 ** (L - pL)
        for it in range(3):
            q.ls_iterate(ctx, ops, e, opts, 1)
            ctx.sync()
            dense = ms.ms_step(dense, cell, k0, E)
            got = T.full(e.to_cores()[0]).reshape(3, 2 ** L, 2 ** L, 2 ** L)
            tiled = np.tile(dense, (1, reps, reps, reps))
            err = np.linalg.norm(got - tiled) / np.linalg.norm(tiled)
            print(f"[lattice] iterate {it + 1}: ranks max {int(e.rank_array().max())}, "
                  f"distance to the tiled cell iterate {err:.2e}", flush=True)
            assert err < 1e-8
    finally:
        ctx.close()
