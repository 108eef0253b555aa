"""The allocation-free rounding entry point against tt_round.

tt_round_noalloc runs tt_round's kernels with the workspace taken from the
library's static device array; on the same input both must give the same
rounded train (bitwise equal cores, ranks, errors and norms: the same kernels
sum in the same order).  Two calls in a row, the second with a smaller input,
so that the second reuses the array the first left behind.
"""
import numpy as np
import pytest

from paper_2512_07811_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    from paper_2512_07811_amd import qtt
    return qtt


def _caps(modes, r):
    """min(r, natural rank) on every inner bond."""
    n = len(modes)
    nat = [min(int(np.prod(modes[:k])), int(np.prod(modes[k:]))) for k in range(1, n)]
    return [1] + [min(r, v) for v in nat] + [1]


def _pair(q, cores_list, cap):
    a = q.DeviceTT.from_cores(cores_list, cap)
    b = q.DeviceTT.from_cores(cores_list, cap)
    return a, b


def _compare(q, ctx, cores_list, cap, eps, max_rank):
    torch = q._torch()
    a, b = _pair(q, cores_list, cap)
    B = a.batch
    err_n = torch.full((B,), -1.0, dtype=torch.float64, device="cuda")
    nrm_n = torch.full((B,), -1.0, dtype=torch.float64, device="cuda")
    print(f"[no_alloc] batch {B} caps {list(cap)} eps {eps} max_rank {max_rank}", flush=True)
    q.tt_round_noalloc(ctx, a, eps, err_n, nrm_n, max_rank)
    err_r, nrm_r = q.tt_round(ctx, b, eps, max_rank)
    ctx.sync()
    assert np.array_equal(a.rank_array(), b.rank_array())
    ca, cb = a.to_cores(), b.to_cores()
    for x, y in zip(ca, cb):
        for u, v in zip(x, y):
            assert u.shape == v.shape
            assert np.array_equal(u, v)
    assert np.array_equal(err_n.cpu().numpy(), err_r.cpu().numpy())
    assert np.array_equal(nrm_n.cpu().numpy(), nrm_r.cpu().numpy())
    return a


def test_noalloc_matches_tt_round_twice(q):
    ctx = q.Context(0)
    modes = [3] + [2] * 12
    # first call: a batch of two graded trains of rank 48, truncated at 1e-6
    # with a cap of 40 on some bonds
    r1 = _caps(modes, 48)
    big = [I.graded_tt(modes, r1, decay=0.8, seed=71 + b) for b in range(2)]
    out = _compare(q, ctx, big, r1, 1e-6, 40)
    assert out.rank_array().max() <= 40
    # second call: one smaller train (rank 12), exact rounding (eps 0)
    r2 = _caps(modes, 12)
    small = [I.random_tt(modes, r2, seed=81)]
    _compare(q, ctx, small, r2, 0.0, 0)
    ctx.close()


def test_noalloc_rejects_workspace_above_its_scratch(q):
    ctx = q.Context(0)
    modes = [3] + [2] * 24
    cap = _caps(modes, 512)
    x = q.DeviceTT.empty(modes, cap, 1)
    torch = q._torch()
    err = torch.zeros(1, dtype=torch.float64, device="cuda")
    nrm = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(q.QtError) as ei:
        q.tt_round_noalloc(ctx, x, 0.0, err, nrm)
    assert ei.value.status == -2
    assert "scratch" in str(ei.value)
    ctx.close()
