"""Benchmark: Lippmann-Schwinger iterations per second on one MI355X.

A step is one basic-scheme iteration of Algorithm 2 (Hadamard with k', SFFT,
Green multiply, inverse SFFT and mean field, each followed by rounding, and the
FP64 residual) on one batch of fields, entirely in the HIP library.

Default workload (the configuration the headline target is stated for): the
1024^3 fibre cell (L = 10, 30 spatial QTT cores plus the component core), 16
periodic z-parallel cylinders of k = 50 in k = 1, reference k0 = 25.5, load
E = e_x, truncation tolerance 1e-6, field rank cap 128.  The rank predictor is
trained on the device from the rank log of SVD-truncated iterations run
before the timed windows (part of the warm-up).  From the same field, two
windows of K iterations are timed: the learned-rank rounding (`value`) and
the FP64 SVD-truncated product-aware rounding (the plain FP64 path, whose
materialized products cannot be formed at this size, see `comparison`); the
effective conductivity column after each window and their relative gap are
reported beside the rates.  Kernel-class timing (HIP events around launches)
runs in separate, untimed iterations after the windows.

Prints one JSON line (see the keys below).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

CONFIGS = {
    "sphere256": dict(L=8, geom="sphere", frac=0.2, k_in=100.0, k_out=1.0, k0=50.5, eps=1e-6,
                      rmax=64, loads=[[1.0, 0.0, 0.0]]),
    "laminate32": dict(L=5, geom="laminate", k0=5.5, eps=1e-10, rmax=64,
                       loads=[[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]]),
    "sphere32": dict(L=5, geom="sphere", frac=0.2, k_in=100.0, k_out=1.0, k0=50.5, eps=1e-6,
                     rmax=16, loads=[[1.0, 0.0, 0.0]]),
    # 64 instances of 128^3 with 1-8 periodic boxes (edges 8-48, k in [5, 50]) in
    # k = 1, loads e_x, e_y, e_z: 192 fields in one batched solve, per-instance k'
    # operators, one reference medium k0 = (1 + 50) / 2 for all instances
    "boxes128": dict(L=7, geom="boxes", instances=64, seed0=1000, k0=25.5, eps=1e-6, rmax=96,
                     loads=[[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]]),
    # 1024^3 fibre cell: 16 z-parallel periodic cylinders, radii 20-40 voxels,
    # k = 50 in k = 1 (seed 4), load e_x; z-invariant, so k' is built from the
    # 1024^2 section, and the Green operator by its exponential-sum form
    "cyl1024": dict(L=10, geom="cylinders", seed=4, k0=25.5, eps=1e-6, rmax=128,
                    loads=[[1.0, 0.0, 0.0]]),
    # 4096^3 simple-cubic lattice of 8^3 spheres (period 512, radius 0.3 of the
    # period = 153.6 voxels), k = 20 in k = 1, load e_x: k' from the 512^3 period
    # cell, the Green operator by cross interpolation of its entry formula
    "lattice4096": dict(L=12, geom="lattice", period_L=9, rel_radius=0.3, k_in=20.0, k_out=1.0,
                        k0=10.5, eps=1e-5, rmax=256, loads=[[1.0, 0.0, 0.0]]),
    # linear elasticity (Voigt strain, 6 components): a plane-strain cell of
    # 4-12 periodic rectangles (the 2D box/multibox workload repeated along z),
    # rectangles E = 10, nu = 0.25 (lam = mu = 4) in E = 1, nu = 0.3
    # (lam = 0.577, mu = 0.385), reference medium at the midpoints, load e_11
    "elastic128": dict(L=7, geom="elastic_boxes", seed=21, eps=1e-6, rmax=64,
                       phases=((0.5769230769230769, 0.38461538461538464), (4.0, 4.0)),
                       loads=[[1.0, 0.0, 0.0, 0.0, 0.0, 0.0]]),
}


# HBM bytes per k_gemm_ex launch from two copy-calibrated rocprofv3 counter runs
# (FETCH_SIZE, WRITE_SIZE) of this bench on the learned path; the summary with the
# commands is in profiles/.  Reported only for the workload and mode it was
# measured on, and only while the kernel is the one measured.
GEMM_TRAFFIC = {("cyl1024", "learned"): 25.50e6}

# iterations per kernel class in the class-timing runs (after the timed windows)
SPLIT_ITERS = 4


def voxels(cfg, inst=0):
    import numpy as np

    from paper_2512_07811_amd import inputs as I
    if cfg["geom"] == "boxes":
        return I.random_boxes(cfg["L"], cfg["seed0"] + inst)
    if cfg["geom"] == "sphere":
        return I.sphere(cfg["L"], cfg["frac"], cfg["k_in"], cfg["k_out"])
    if cfg["geom"] == "laminate":
        return I.laminate(cfg["L"])
    if cfg["geom"] == "lattice":        # one period cell (the exact reduction)
        return I.sphere_lattice_cell(cfg["period_L"], cfg["rel_radius"], cfg["k_in"], cfg["k_out"])
    if cfg["geom"] == "cylinders":      # the (N, N) section of a z-invariant cell
        return I.cylinders_section(cfg["L"], cfg["seed"])
    if cfg["geom"] == "elastic_boxes":  # Lame fields (lam, mu) of the plane-strain cell
        ph = I.boxes_section(cfg["L"], cfg["seed"])
        N = ph.shape[0]
        (l0, m0), (l1, m1) = cfg["phases"]
        ph3 = np.broadcast_to(ph[:, :, None], (N, N, N))
        return np.where(ph3 > 0, l1, l0), np.where(ph3 > 0, m1, m0)
    raise ValueError(cfg["geom"])


_WORKER = {}


def _init_worker(cfg, shared):
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)          # one BLAS thread per worker process
    _WORKER["cfg"] = cfg
    _WORKER["shared"] = shared


def _instance_problem(i):
    from paper_2512_07811_amd import operands as P
    cfg = _WORKER["cfg"]
    return P.build_problem(kvox=voxels(cfg, i), k0=cfg["k0"], shared=_WORKER["shared"])


def _oracle_rate(args):
    """Dense Moulinec-Suquet oracle iterations (Algorithm 1) for about budget_s
    seconds in this process; returns (iterations, seconds)."""
    cfg, budget_s = args
    import numpy as np

    from oracle import ms
    if cfg["geom"] == "elastic_boxes":
        from oracle import ms_elastic as ME
        lam, mu = voxels(cfg)
        lam0, mu0 = 0.5 * (lam.min() + lam.max()), 0.5 * (mu.min() + mu.max())
        E = cfg["loads"][0]
        ev = np.zeros((6,) + lam.shape) + np.asarray(E, dtype=float).reshape(6, 1, 1, 1)
        t0 = time.perf_counter()
        its = 0
        while True:
            ev = ME.ms_step(ev, lam, mu, lam0, mu0, E)
            its += 1
            if time.perf_counter() - t0 > budget_s or its >= 200:
                break
        return its, time.perf_counter() - t0
    kvox = voxels(cfg)
    d = kvox.ndim          # a z-invariant cell is timed on its exact 2D reduction
    E = cfg["loads"][0][:d]
    e = np.broadcast_to(np.asarray(E, dtype=float).reshape((d,) + (1,) * d),
                        (d,) + kvox.shape).copy()
    t0 = time.perf_counter()
    its = 0
    while True:
        e = ms.ms_step(e, kvox, cfg["k0"], E)
        its += 1
        if time.perf_counter() - t0 > budget_s or its >= 200:
            break
    return its, time.perf_counter() - t0


def cpu_baseline(cfg, budget_s=20.0):
    """The oracle, unchanged (single-threaded numpy FFTs), on every host core:
    one worker process per core (at most 16, the machine's CPU share; fewer for 3D
    grids whose dense fields need GBs each), each iterating the same workload
    for budget_s; the rate is the sum of the workers' iterations per second.
    Forked before the GPU is touched."""
    import multiprocessing as mp
    kvox = voxels(cfg)
    if isinstance(kvox, tuple):         # elasticity: (lam, mu), a 6-component field
        kvox = kvox[0]
    workers = min(16, os.cpu_count() or 1)
    if kvox.ndim == 3 and kvox.shape[0] >= 256:
        workers = min(workers, 8)
    if kvox.ndim == 3 and kvox.shape[0] >= 512:
        workers = 1                     # one 512^3 step holds about 36 GB
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_oracle_rate, [(cfg, budget_s)] * workers)
    its = sum(r[0] for r in res)
    rate = sum(r[0] / r[1] for r in res)
    d = kvox.ndim
    return {"value": rate, "unit": "LS iters/s", "cores": workers, "kind": "oracle",
            "sample": f"{its} dense Moulinec-Suquet iterations (Algorithm 1, numpy pocketfft, "
                      f"one thread per process) in {workers} processes of about {budget_s:.0f} s "
                      f"each, on the same {kvox.shape[0]}^{d} microstructure and load"
                      + (" (the exact 2D reduction of the z-invariant cell)" if d == 2 else "")
                      + (f" (the {kvox.shape[0]}^3 period cell: the exact reduction of the "
                         f"{2 ** cfg['L']}^3 lattice)" if cfg["geom"] == "lattice" else "")
                      + "; the naive TT oracle cannot form this workload's product ranks"}


def round_model_flops(modes, r_in, r_out):
    """Real flops of one rounding by the Householder/Golub-Reinsch model (complex = 4x).

    Left QR sweep over the cores (absorb the carried R factor, factor the
    unfolding), then the right truncated-SVD sweep (QR of the unfolding, square
    SVD of its triangle, carried factor, absorb into the next core), Sec. 2.2.
    r_in are the input ranks, r_out the ranks after rounding."""
    n = len(modes)

    def qr(m, N):
        big, small = max(m, N), min(m, N)
        return 2.0 * big * small * small - 2.0 / 3.0 * small ** 3

    f = 0.0
    rl = [1] * (n + 1)
    for k in range(n):
        f += 2.0 * rl[k] * r_in[k] * modes[k] * r_in[k + 1]          # absorb
        if k < n - 1:
            m, N = rl[k] * modes[k], r_in[k + 1]
            f += qr(m, N)
            rl[k + 1] = min(m, N)
    for k in range(n - 1, 0, -1):
        m, N = rl[k], modes[k] * r_out[k + 1]
        small = min(m, N)
        f += qr(m, N) + 21.0 * small ** 3                                # QR + square SVD
        f += 2.0 * m * N * r_out[k]                                     # carried factor
        f += 2.0 * rl[k - 1] * modes[k - 1] * rl[k] * r_out[k]           # absorb into k-1
    return 4.0 * f


def round_microbench(ctx, ranks, batches=(1,), L=8, max_runs=100, budget_s=3.0):
    """tt_round on i.i.d. complex N(0, 1) cores of uniform rank R, zero tolerance
    (nothing is truncated beyond the natural ranks: pure cost), mean time per
    call over up to `max_runs` runs; the input is restored between runs outside
    the timed events.  A call rounds `batch` independent trains at once."""
    import numpy as np
    import torch

    from paper_2512_07811_amd import inputs as I
    from paper_2512_07811_amd import qtt
    modes = [3] + [2] * (3 * L)
    n = len(modes)
    out = []
    for R, B in ((R, B) for R in ranks for B in batches):
        rk = [1] + [R] * (n - 1) + [1]
        x = qtt.DeviceTT.from_cores([I.random_tt(modes, rk, seed=100 + R + 7919 * b)
                                     for b in range(B)], cap=rk)
        d0, r0 = x.data.clone(), x.ranks.clone()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        times = []
        t_start = time.perf_counter()
        while len(times) < max_runs and (len(times) < 2 or time.perf_counter() - t_start < budget_s):
            x.data.copy_(d0)
            x.ranks.copy_(r0)
            ev0.record()
            qtt.tt_round(ctx, x, 0.0)
            ev1.record()
            ev1.synchronize()
            times.append(ev0.elapsed_time(ev1))
        times = times[1:]                      # the first run pays the workspace set-up
        r_out = x.rank_array()[0].tolist()
        ms = float(np.mean(times))
        # the same trains compressed by polar decomposition (QT_ROUND_POLAR)
        ptimes = []
        t_start = time.perf_counter()
        while len(ptimes) < max_runs and (len(ptimes) < 3 or time.perf_counter() - t_start < budget_s):
            x.data.copy_(d0)
            x.ranks.copy_(r0)
            ev0.record()
            qtt.tt_round(ctx, x, 0.0, mode=qtt.ROUND_POLAR, seed=1)
            ev1.record()
            ev1.synchronize()
            ptimes.append(ev0.elapsed_time(ev1))
        pms = float(np.mean(ptimes[1:]))
        fl = B * round_model_flops(modes, rk, r_out)
        out.append({"R": R, "batch": B, "runs": len(times), "ms": ms, "model_gflop": fl / 1e9,
                    "gflops": fl / (ms * 1e-3) / 1e9, "frac_fp64_peak": fl / (ms * 1e-3) / 78.6e12,
                    "polar_ms": pms, "chi_polar_over_svd": pms / ms})
        print(f"[bench] tt_round R={R} batch {B}: {ms:.3f} ms, {out[-1]['gflops']:.1f} GFLOP/s "
              f"({len(times)} runs); polar {pms:.3f} ms", file=sys.stderr, flush=True)
        del x, d0, r0
    return {"family": f"i.i.d. complex N(0,1) cores, {n} cores (modes 3, 2, ..., 2), uniform "
                      f"rank R, eps 0", "flop_model": "Householder QR 2mN^2 - 2N^3/3, square "
                      "SVD 21N^3, absorb/carry products 2mnk; x4 for complex",
            "polar": "the same calls with QT_ROUND_POLAR (polar-decomposition truncation on the "
                     "GEMM); chi = tau_polar / tau_SVD as the paper's appendix defines it",
            "results": out}


def _qr_flops(m, N):
    big, small = max(m, N), min(m, N)
    return 2.0 * big * small * small - 2.0 / 3.0 * small ** 3


def sketch_widths(modes, r_op, cap_y, rmax, oversample):
    """Sketch ranks l_k = min(natural, r_A r_y, rmax + oversample) of one
    product-aware rounding (the library's plan)."""
    n = len(modes)
    out = [1] * (n + 1)
    for k in range(1, n):
        nat = min(math.prod(modes[:k]), math.prod(modes[k:]))
        out[k] = max(1, min(nat, r_op[k] * cap_y[k], rmax + oversample))
    return out


def sketch_round_model_flops(modes, ell, rmax):
    """Real flops of the rounding kernels of one product-aware rounding (complex = 4x),
    by the Householder / Golub-Reinsch model:
      qr:  the QR of every sketch Y_k (l_k p_k x l_{k+1}) with Q formed (twice the
           factorization);
      svd: per bond of the truncation sweep, the block (l_k x p_k min(l_{k+1}, rmax)):
           QR of the block with Q formed, a second QR (R only) when it is wide, and
           the square SVD 21 N^3 of its N x N triangle."""
    n = len(modes)
    qr = 0.0
    for k in range(n - 1):
        qr += 2.0 * _qr_flops(ell[k] * modes[k], ell[k + 1])
    svd = 0.0
    for k in range(n - 1, 0, -1):
        m, c = ell[k], modes[k] * min(ell[k + 1], rmax)
        N = min(m, c)
        svd += 2.0 * _qr_flops(m, c) + (_qr_flops(N, N) if m < c else 0.0) + 21.0 * N ** 3
    return 4.0 * qr, 4.0 * svd


def iteration_model(ops, field_cap, rmax, oversample):
    """Rounding-kernel model flops of one iteration (four product-aware roundings)."""
    modes = [int(v) for v in field_cap[0]]
    cap = [int(v) for v in field_cap[1]]
    def capmin(v):
        return [min(x, rmax) if 0 < k < len(v) - 1 else x for k, x in enumerate(v)]
    tot_qr = tot_svd = 0.0
    y = cap
    for A in (ops.Kp, ops.S, ops.G, None):
        if A is None:       # S^H (S E - eps^): input rank r + 1
            A = ops.Sinv
            y = [1] + [v + 1 for v in y[1:-1]] + [1]
        ell = sketch_widths(modes, [int(v) for v in A.ranks], y, rmax, oversample)
        q, sv = sketch_round_model_flops(modes, ell, rmax)
        tot_qr += q
        tot_svd += sv
        y = capmin(ell)
    return tot_qr, tot_svd


def mat_rank(prob):
    """Largest bond of the material train (or operator, for elasticity)."""
    return max(c.shape[0] for c in (prob["Kp_op"] if prob.get("kind") == "elastic" else prob["kp"]))


def max_op_rank(prob) -> int:
    """Largest bond over the operators an iteration multiplies the field by."""
    names = ("Kp_op", "S", "G", "Sinv") if prob.get("kind") == "elastic" else ("kp", "S", "G", "Sinv")
    return max(c.shape[0] for n in names for c in prob[n])


def green_step(qtt, ctx, ops, prev, e, cfg, args):
    """Algorithm 2's Green multiply eps^ ~ Gamma^ tau^ on this workload's
    polarization two ways: the product-aware rounding (sketch + SVD truncation,
    with the exact norm from <tau^, Gamma^ tau^>) and AMEn (tt_amen_mv, 2 sweeps,
    enrichment rank 8, warm start: the Green output of the field `prev`, as in
    an iteration that starts from the previous one's eps^).  tau^ = R(S R(k' e))
    by the product-aware rounding.  Returns times, GEMM work and the distance
    between the two results."""
    import numpy as np

    from paper_2512_07811_amd import inputs as I
    rmax, eps, p_over = cfg["rmax"], cfg["eps"], args.oversample
    modes = [int(m) for m in e.modes]
    B = e.batch
    nat = []
    for k in range(1, len(modes)):
        nat.append(min(int(np.prod(modes[:k])), int(np.prod(modes[k:]))))
    cap = [1] + [min(r, rmax + p_over) for r in nat] + [1]

    def rounded(A, y, n2):
        out = qtt.DeviceTT.empty(modes, cap, B)
        qtt.tt_sketch_round(ctx, A, y, n2, out, eps=eps, max_rank=rmax, mode=qtt.ROUND_SKETCH,
                            oversample=p_over, seed=args.sketch_seed)
        return out

    def tau_hat(f):
        t1 = rounded(ops.Kp, f, qtt.tt_sandwich(ctx, ops.K2, f))
        return rounded(ops.S, t1, qtt.tt_dot(ctx, t1, t1).real.contiguous())

    def green_n2(t):
        return (qtt.tt_sandwich(ctx, ops.G2, t) if ops.G2 is not None
                else qtt.tt_sandwich(ctx, ops.G, t, 1.0 / ops.k0))

    t_prev, t_cur = tau_hat(prev), tau_hat(e)
    y0 = rounded(ops.G, t_prev, green_n2(t_prev))          # the warm start
    z_host = [I.random_tt(modes, [1] + [min(8, r) for r in nat] + [1], seed=77 + b)
              for b in range(B)]

    def fresh():
        y = qtt.DeviceTT.empty(modes, cap, B)
        y.data.copy_(y0.data)
        y.ranks.copy_(y0.ranks)
        return y, qtt.DeviceTT.from_cores(z_host)

    # one untimed call first: its GEMM shapes are new to the tile-shape tuner
    y, z = fresh()
    qtt.tt_amen_mv(ctx, ops.G, t_cur, y, z, eps, rmax, 2)
    y, z = fresh()
    ctx.sync()
    ctx.counters(reset=True)
    t0 = time.perf_counter()
    y_rto = rounded(ops.G, t_cur, green_n2(t_cur))
    ctx.sync()
    dt_rto = time.perf_counter() - t0
    f_rto = ctx.counters(reset=True)["gemm_flops"]
    t0 = time.perf_counter()
    qtt.tt_amen_mv(ctx, ops.G, t_cur, y, z, eps, rmax, 2)
    ctx.sync()
    dt_amen = time.perf_counter() - t0
    f_amen = ctx.counters(reset=True)["gemm_flops"]
    d = qtt.tt_add(ctx, 1.0, y, -1.0, y_rto)
    dn = qtt.tt_dot(ctx, d, d).real.cpu().numpy()
    yn = qtt.tt_dot(ctx, y_rto, y_rto).real.cpu().numpy()
    return {"product_aware_ms": 1000.0 * dt_rto, "amen_ms": 1000.0 * dt_amen,
            "amen_sweeps": 2, "amen_enrichment_rank": 8,
            "gemm_tflop_product_aware": f_rto / 1e12, "gemm_tflop_amen": f_amen / 1e12,
            "amen_over_product_aware_time": dt_amen / dt_rto,
            "rel_distance": float(np.sqrt(np.max(dn / yn))),
            "ranks_amen": y.rank_array()[0].tolist(), "ranks_product_aware":
                y_rto.rank_array()[0].tolist(),
            "note": "the rank cap binds, so the two rank-capped results differ at the level of "
                    "the truncation error; the product-aware rounding's time includes the exact "
                    "norm <tau^, Gamma^ tau^> it needs for its error budget"}


def dominant_class(cls_ms, window_svd_calls_per_step):
    """The kernel class with the most time per iteration of the timed window.
    `cls_ms` holds per-iteration averages of the class-timing iterations, which
    run past the window: their SVDs come only from fallbacks, whose number
    differs from the window's, so the SVD class's time is scaled to the
    window's SVD calls per step.  Returns (class, the SVD class's scaled ms)."""
    s_svd = cls_ms["svd"]["svd_calls"]

    def window_ms(k):
        if k != "svd":
            return cls_ms[k]["ms"]
        return cls_ms[k]["ms"] * window_svd_calls_per_step / s_svd if s_svd > 0 else 0.0
    return max(cls_ms, key=window_ms), window_ms("svd")


def under_profiler() -> bool:
    """rocprofv3 preloads its library, which initialises the GPU before this
    program starts: no worker processes may be forked then."""
    return any(k.startswith("ROCPROF") for k in os.environ) or \
        "rocprofiler" in os.environ.get("LD_PRELOAD", "")


def a_eff(q, ctx, ops, e, L):
    """A_eff[:, j] = Re <k_sel[c], e> / N^3 per field (Appendix A)."""
    import numpy as np
    N3 = 2.0 ** (3 * L)
    cols = [q.tt_dot(ctx, ops.k_sel[c], e).cpu().numpy().real / N3
            for c in range(len(ops.k_sel))]
    return np.stack(cols, axis=1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="cyl1024", choices=sorted(CONFIGS))
    ap.add_argument("--mode", default="learned", choices=["learned", "sketch", "svd"],
                    help="path of `value`; learned also times the SVD-truncated path")
    ap.add_argument("--log-iters", type=int, default=8,
                    help="SVD-truncated iterations logged for training the rank predictor")
    ap.add_argument("--epochs", type=int, default=400)
    ap.add_argument("--graph", action="store_true",
                    help="sketch mode: replay a captured HIP graph of one iteration")
    ap.add_argument("--instances", type=int, default=0,
                    help="override the instance count of a batched config")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 512 MiB device copy first (HBM counter calibration)")
    ap.add_argument("--oversample", type=int, default=4)
    ap.add_argument("--sketch-seed", type=int, default=17,
                    help="Philox seed of the sketch Gaussians")
    ap.add_argument("--accept", type=float, default=1.25,
                    help="learned mode: where the step's last SVD-truncated error e_s exceeds "
                         "eps (rank cap), keep a rounding iff its error <= accept * e_s (eps "
                         "always holds where e_s <= eps)")
    ap.add_argument("--quantile", type=float, default=0.9,
                    help="learned mode: the predicted rank is the class at this quantile")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-split", action="store_true",
                    help="skip the untimed kernel-class timing iterations")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision (FP32 range finder) windows")
    ap.add_argument("--no-amen", action="store_true",
                    help="skip the Green-step comparison with AMEn")
    ap.add_argument("--no-compare", action="store_true",
                    help="learned mode: skip the SVD-truncated window")
    ap.add_argument("--round-ranks", default="64,128",
                    help="uniform ranks of the tt_round micro-benchmark ('' skips it)")
    ap.add_argument("--round-batches", default="1,64",
                    help="batch sizes of the tt_round micro-benchmark (trains per call)")
    ap.add_argument("--round-only", action="store_true",
                    help="run only the tt_round micro-benchmark and print its JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: independent solves would shard across GPUs "
                                   "with no exchange, and one large train by core blocks with "
                                   "point-to-point sends of the carried factor; neither is "
                                   "launched", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np

    cfg = dict(CONFIGS[args.config])
    batched = "instances" in cfg
    if batched and args.instances > 0:
        cfg["instances"] = args.instances
    profiled = under_profiler()
    # host work that forks worker processes runs before anything touches the GPU
    cpu = None
    if not args.no_cpu_baseline and not args.round_only and not profiled:
        print("[bench] cpu baseline (oracle on the host cores)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(cfg, args.cpu_budget)

    import torch

    from paper_2512_07811_amd import operands as P
    from paper_2512_07811_amd import qtt

    if args.round_only:
        ctx = qtt.Context(0)
        res = round_microbench(ctx, [int(v) for v in args.round_ranks.split(",")],
                               [int(v) for v in args.round_batches.split(",")])
        ctx.close()
        print(json.dumps({"tt_round": res}), flush=True)
        return

    t0 = time.perf_counter()
    say = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)  # noqa: E731
    if batched:
        first = P.build_problem(kvox=voxels(cfg, 0), k0=cfg["k0"], log=say)
        shared = {k: first[k] for k in ("S", "Sinv", "G")}
        if profiled:
            probs = [first] + [P.build_problem(kvox=voxels(cfg, i), k0=cfg["k0"], shared=shared)
                               for i in range(1, cfg["instances"])]
        else:
            import multiprocessing as mp
            with mp.get_context("fork").Pool(min(16, os.cpu_count() or 1),
                                             initializer=_init_worker,
                                             initargs=(cfg, shared)) as pool:
                probs = [first] + pool.map(_instance_problem, range(1, cfg["instances"]))
        prob = first
        fields = [E for _ in probs for E in cfg["loads"]]
    elif cfg["geom"] == "lattice":
        prob = P.build_problem(cell=voxels(cfg), L=cfg["L"], k0=cfg["k0"], log=say)
        probs = [prob]
        fields = list(cfg["loads"])
    elif cfg["geom"] == "cylinders":
        prob = P.build_problem(section=voxels(cfg), k0=cfg["k0"], log=say)
        probs = [prob]
        fields = list(cfg["loads"])
    elif cfg["geom"] == "elastic_boxes":
        lam, mu = voxels(cfg)
        prob = P.build_problem_elastic(lam, mu, log=say)
        probs = [prob]
        fields = list(cfg["loads"])
    else:
        prob = P.build_problem(kvox=voxels(cfg), k0=cfg["k0"], log=say)
        probs = [prob]
        fields = list(cfg["loads"])
    t_setup = time.perf_counter() - t0
    say(f"setup {t_setup:.1f}s  instances {len(probs)}  fields {len(fields)}  material max rank "
        f"{max(mat_rank(p) for p in probs)}  "
        f"G max rank {max(c.shape[0] for c in prob['G'])}")
    if args.calibrate_copy:
        # a plain copy of known size: 512 MiB read, 512 MiB written
        src = torch.ones(1 << 26, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ctx = qtt.Context(0)
    if batched:
        ops, e = P.upload_batch(probs, cfg["loads"], cfg["rmax"])
    else:
        ops, e = P.upload(prob, cfg["loads"], cfg["rmax"])
    mode = {"learned": qtt.ROUND_LEARNED, "sketch": qtt.ROUND_SKETCH, "svd": qtt.ROUND_SVD}[args.mode]
    opts = qtt.solve_opts(cfg["eps"], cfg["rmax"], mode=mode, oversample=args.oversample,
                          seed=args.sketch_seed, graph=args.graph)
    sk_opts = qtt.solve_opts(cfg["eps"], cfg["rmax"], mode=qtt.ROUND_SKETCH,
                             oversample=args.oversample, seed=args.sketch_seed)
    e = qtt.DeviceTT.from_cores([P.mean_field(np.asarray(E), ops.L) for E in fields], e.cap)
    train_info = None
    if args.mode == "learned":
        from paper_2512_07811_amd import learned
        t0 = time.perf_counter()
        n_cls = learned.n_classes(cfg["rmax"])
        qtt.ranklog_enable(ctx, 1 << 20, n_cls)
        qtt.ls_iterate(ctx, ops, e, sk_opts, args.log_iters)
        X, Y = qtt.ranklog_get(ctx)
        qtt.ranklog_enable(ctx, 0, n_cls)
        pred = learned.RankPredictor(ctx, n_cls=n_cls, seed=5)
        hist = pred.train(X, Y, epochs=args.epochs)
        pred.install(quantile=args.quantile, accept_factor=args.accept)
        train_info = {"samples": int(X.shape[0]), "epochs": args.epochs, "classes": n_cls,
                      "trained_on": f"rank log of the first {args.log_iters} SVD-truncated "
                                    f"iterations of this workload",
                      "loss_first": float(hist[0]), "loss_last": float(hist[-1]),
                      "log_and_train_s": time.perf_counter() - t0}
        say(f"predictor trained on {X.shape[0]} samples, loss {hist[0]:.3f} -> {hist[-1]:.4f}")
    if args.warmup:
        qtt.ls_iterate(ctx, ops, e, opts, args.warmup)
    ctx.sync()
    torch.cuda.synchronize()
    say(f"warmup done, ranks {e.rank_array()[0].tolist()}")
    snap = (e.data.clone(), e.ranks.clone())
    B = len(fields)

    def window(o, label):
        """K timed iterations from the snapshot; returns (seconds, residuals, counters)."""
        e.data.copy_(snap[0])
        e.ranks.copy_(snap[1])
        ctx.counters(reset=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        res = qtt.ls_iterate(ctx, ops, e, o, args.steps)
        ctx.sync()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        cnt = ctx.counters(reset=True)
        r = res.cpu().numpy()
        say(f"{label}: {args.steps} steps in {dt:.3f}s; fallbacks {cnt['learned_fallbacks']} of "
            f"{cnt['learned_roundings']}; residuals {r[:, 0].tolist()}")
        return dt, r, cnt

    def class_split(o, restore, iters=SPLIT_ITERS):
        """`iters` more iterations per kernel class (GEMM, QR, SVD) with HIP
        events around every launch of that class, outside the timed window;
        per-iteration averages."""
        if restore:
            e.data.copy_(snap[0])
            e.ranks.copy_(snap[1])
        cls_ms = {}
        for cname, cls in (("gemm", ctx.PROF_GEMM), ("qr", ctx.PROF_QR), ("svd", ctx.PROF_SVD)):
            c0 = ctx.counters()
            ctx.profile(cls)
            qtt.ls_iterate(ctx, ops, e, o, iters)
            ms_, n_ = ctx.profile_read()
            c1 = ctx.counters()
            cls_ms[cname] = {"ms": ms_ / iters, "launches": n_ / iters,
                             "svd_calls": (c1["svd_calls"] - c0["svd_calls"]) / iters,
                             "gemm_flops": (c1["gemm_flops"] - c0["gemm_flops"]) / iters,
                             "gemm_bytes": (c1["gemm_bytes"] - c0["gemm_bytes"]) / iters,
                             "fallbacks": c1["learned_fallbacks"] - c0["learned_fallbacks"]}
        ctx.profile(0)
        return cls_ms

    # GEMM tile-shape signatures timed so far (a first call of a signature
    # inside the window is timed there: its four shapes run on the stream)
    tuned0 = ctx.autotune(1)
    dt, res, cnt = window(opts, args.mode)
    tuned1 = ctx.autotune(1)
    A_main = a_eff(qtt, ctx, ops, e, ops.L)
    # kernel classes of the main path: the iterations continue from the end of
    # the timed window (the rank predictor's features belong to that field)
    split = {}
    split_paths = [args.mode] + (["svd_truncated"] if args.mode == "learned" and not args.no_compare
                                 else [])
    if not args.no_split:
        split[args.mode] = class_split(opts, restore=False)
        ctx.counters(reset=True)
    comparison = accuracy = None
    cnt_sk = None
    if args.mode == "learned" and not args.no_compare:
        dt_sk, res_sk, cnt_sk = window(sk_opts, "SVD-truncated")
        A_sk = a_eff(qtt, ctx, ops, e, ops.L)
        gap = float(np.linalg.norm(A_main - A_sk) / np.linalg.norm(A_sk))
        comparison = {
            "svd_truncated_iters_per_s": args.steps * B / dt_sk,
            "svd_truncated_ms_per_step": 1000.0 * dt_sk / args.steps,
            "speedup_learned_over_svd_truncated": dt_sk / dt,
            "learned_roundings": cnt["learned_roundings"],
            "learned_fallbacks": cnt["learned_fallbacks"],
            "svd_calls_learned": cnt["svd_calls"], "svd_calls_svd_truncated": cnt_sk["svd_calls"],
            "gemm_flops_ratio": cnt["gemm_flops"] / max(cnt_sk["gemm_flops"], 1),
            "plain_fp64": "the FP64 SVD-truncated product-aware rounding stands in for the "
                          "plain (materializing) FP64 path, which cannot run here: its "
                          "products have ranks up to the operator's times the field's, "
                          f"{max_op_rank(prob)} x {cfg['rmax']} per bond (an SVD block holds "
                          "at most 1024 columns)",
        }
        accuracy = {
            "A_eff_column_learned": A_main[0].tolist(), "A_eff_column_svd_truncated": A_sk[0].tolist(),
            "A_eff_rel_gap": gap, "meets_1e-6": bool(gap <= 1e-6),
            "residual_last_learned": float(res[-1, 0]), "residual_last_svd_truncated": float(res_sk[-1, 0]),
            "note": "after the same K iterations from the same field; the rank cap binds on every "
                    "middle bond (each rounding's error is a few per cent, far above eps), so two "
                    "different roundings give iterates, and A_eff, that differ at that level",
        }
    amen = None
    if B == 1 and not args.no_amen:
        pf = qtt.DeviceTT.empty(e.modes, e.cap, e.batch)
        pf.data.copy_(snap[0])
        pf.ranks.copy_(snap[1])
        amen = green_step(qtt, ctx, ops, pf, e, cfg, args)
        say(f"Green step: product-aware {amen['product_aware_ms']:.1f} ms, AMEn "
            f"{amen['amen_ms']:.1f} ms, distance {amen['rel_distance']:.2e}")
    # mixed precision (FP32-MFMA range finder, FP64 projection and bookkeeping):
    # the same windows from the same snapshot, against their FP64 counterparts
    mixed = None
    if args.mode in ("learned", "sketch") and not args.no_mixed:
        mixed = {"scheme": "right sketches and sketched products on v_mfma_f32_16x16x4f32; "
                           "projection, QR, SVD and error bookkeeping FP64"}
        pairs = [(args.mode, opts, A_main, dt)]
        if comparison:
            pairs.append(("svd_truncated", sk_opts, A_sk, dt_sk))
        for name, o64, A64, dt64 in pairs:
            o32 = qtt.solve_opts(cfg["eps"], cfg["rmax"], mode=o64.round.mode,
                                 oversample=args.oversample, seed=args.sketch_seed,
                                 precision=qtt.PREC_F32)
            dt32, res32, cnt32 = window(o32, f"{name} mixed")
            A32 = a_eff(qtt, ctx, ops, e, ops.L)
            g32 = float(np.linalg.norm(A32 - A64) / np.linalg.norm(A64))
            mixed[name] = {"iters_per_s": args.steps * B / dt32, "speedup_over_fp64": dt64 / dt32,
                           "A_eff_column": A32[0].tolist(), "A_eff_rel_gap_vs_fp64": g32,
                           "meets_1e-6": bool(g32 <= 1e-6),
                           "residual_last": float(res32[-1, 0]),
                           "fallbacks": cnt32["learned_fallbacks"]}
    if not args.no_split and "svd_truncated" in split_paths:
        split["svd_truncated"] = class_split(sk_opts, restore=True)
        ctx.counters(reset=True)
    value = args.steps * B / dt
    out = {
        "metric": "LS iters/s", "value": value, "unit": "LS iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1000.0 * dt / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": args.config, "L": cfg["L"], "grid": f"{2 ** cfg['L']}^3",
                   "physics": ("linear elasticity (Voigt strain, 6 components)"
                               if cfg["geom"] == "elastic_boxes"
                               else "scalar conductivity (3 gradient components)"),
                   "instances": len(probs),
                   "rounding": args.mode, "eps": cfg["eps"], "max_rank": cfg["rmax"],
                   "oversample": args.oversample,
                   "quantile": args.quantile if args.mode == "learned" else None,
                   "accept": args.accept if args.mode == "learned" else None,
                   "graph": bool(args.graph and args.mode == "sketch"),
                   "batch": B, "parallelism": "single GPU"},
    }
    if comparison:
        out["comparison"] = comparison
        out["accuracy"] = accuracy
    if mixed:
        out["mixed_precision"] = mixed
    if amen:
        out["green_step_amen"] = amen
    if split:
        main = split[args.mode]
        qr_model, svd_model = iteration_model(ops, (e.modes, e.cap), cfg["rmax"], args.oversample)
        dom, svd_window_ms = dominant_class(main, cnt["svd_calls"] / args.steps)
        g = main["gemm"]
        g_ach = g["gemm_flops"] / (g["ms"] * 1e-3) / 1e12 if g["ms"] > 0 else None
        classes = {"gemm": {"achieved": g_ach, "flops_per_step": g["gemm_flops"],
                            "bytes_per_step": g["gemm_bytes"],
                            "algorithmic_bytes_per_launch": g["gemm_bytes"] / max(g["launches"], 1),
                            "model": "structured GEMMs: 8 flops per complex multiply-add, counted "
                                     "on the device per launch"},
                   "qr": {"achieved": qr_model * B / (main["qr"]["ms"] * 1e-3) / 1e12
                          if main["qr"]["ms"] > 0 else None, "flops_per_step": qr_model * B,
                          "model": "Householder QR of every sketch with Q formed, 4 roundings"}}
        if cnt_sk and cnt_sk["svd_calls"] > 0 and main["svd"]["ms"] > 0:
            # the SVD model of a full SVD-truncated step, scaled to the
            # class-timing iterations' share of its SVD calls
            share = main["svd"]["svd_calls"] / (cnt_sk["svd_calls"] / args.steps)
            classes["svd"] = {"achieved": svd_model * B * share / (main["svd"]["ms"] * 1e-3) / 1e12,
                              "flops_per_step": svd_model * B * share,
                              "model": "square SVD 21N^3 per block (x4 complex) on the "
                                       "fallbacks' SVD calls"}
        ach = classes[dom]["achieved"] if dom in classes else None
        out["roofline"] = {
            "kernel": {"gemm": "structured GEMM (k_gemm_ex with its split-K sums)",
                       "qr": "QR of the sketches (register-panel blocked QR and its products)",
                       "svd": "truncated SVD (QRs + one-sided Jacobi)"}[dom],
            "bound": "alu", "achieved": ach, "peak": 78.6, "unit": "TFLOP/s",
            "frac": ach / 78.6 if ach else None,
            "traffic": GEMM_TRAFFIC.get((args.config, args.mode)) if dom == "gemm" else None,
            "avg_launch_us": 1000.0 * main[dom]["ms"] / max(main[dom]["launches"], 1),
            "kernel_ms_per_step": {k: v["ms"] for k, v in main.items()},
            "launches_per_step": {k: v["launches"] for k, v in main.items()},
            "classes": classes, "dominant_class": dom,
            "class_timing_fallbacks": {k: v["fallbacks"] for k, v in main.items()},
            "svd_ms_per_step_window": svd_window_ms,
        }
        if "svd_truncated" in split:
            sv = split["svd_truncated"]
            r_qr = qr_model * B / (sv["qr"]["ms"] * 1e-3) / 1e12 if sv["qr"]["ms"] > 0 else None
            r_sv = svd_model * B / (sv["svd"]["ms"] * 1e-3) / 1e12 if sv["svd"]["ms"] > 0 else None
            out["rounding_roofline"] = {
                "path": "svd_truncated", "peak": 78.6, "unit": "TFLOP/s",
                "qr": {"achieved": r_qr, "frac": r_qr / 78.6 if r_qr else None,
                       "ms_per_step": sv["qr"]["ms"], "model_flops_per_step": qr_model * B},
                "svd": {"achieved": r_sv, "frac": r_sv / 78.6 if r_sv else None,
                        "ms_per_step": sv["svd"]["ms"], "model_flops_per_step": svd_model * B},
                "kernel_ms_per_step": {k: v["ms"] for k, v in sv.items()},
                "model": "Householder 2mN^2 - 2N^3/3 per QR (Q formed: twice), square SVD "
                         "21N^3 (Golub-Reinsch), complex x4, on the plan's sketch widths",
            }
    out["counters"] = {"svd_calls_per_step": cnt["svd_calls"] / args.steps,
                       "gemm_flops_timed_window": cnt["gemm_flops"],
                       "gemm_bytes_timed_window": cnt["gemm_bytes"],
                       "jacobi_sweeps_per_svd": (cnt["svd_sweeps"] / cnt["svd_calls"]
                                                 if cnt["svd_calls"] else None),
                       "sketch_over_budget": cnt["sketch_over_budget"],
                       "gemm_signatures_tuned_before_window": tuned0,
                       "gemm_signatures_tuned_in_window": tuned1 - tuned0}
    if train_info:
        out["predictor"] = train_info
    if args.round_ranks:
        out["tt_round"] = round_microbench(ctx, [int(v) for v in args.round_ranks.split(",")],
                                           [int(v) for v in args.round_batches.split(",")])
    if cpu:
        out["cpu_baseline"] = cpu
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
