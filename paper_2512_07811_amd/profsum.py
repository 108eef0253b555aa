"""Summaries of rocprofv3 result databases (``<dir>/<name>_results.db``).

    python -m paper_2512_07811_amd.profsum kernels DB [--top N] [--warmup W --steps K]
    python -m paper_2512_07811_amd.profsum counters DB [--calib-kib KIB] [--kernel SUBSTR]
                                                       [--warmup W --steps K]
    python -m paper_2512_07811_amd.profsum schema DB

``kernels``: per-kernel dispatch counts, total and average durations over the
whole run, and, with --steps, over the timed LS iterations of a ``bench.py``
run: the iterations after the last rank-predictor training launch
(``k_mlp_train``), of which the first W are the warm-up (one ``k_residual``
launch ends every iteration).

``counters``: per-kernel averages of a ``--pmc`` run's counter values (KiB for
FETCH_SIZE / WRITE_SIZE), and, with --calib-kib, the value the largest
dispatch of the plain copy kernel (``__amd_rocclr_copyBuffer`` or torch's
elementwise copy: ``bench.py --calibrate-copy`` runs one copy of 512 MiB =
524288 KiB) read, the scale factor, and the scaled values; with --steps, of
the dispatches of the timed iterations only.
"""
from __future__ import annotations

import argparse
import collections
import re
import sqlite3


def _short(name: str) -> str:
    s = re.sub(r"\(.*", "", name).replace("void ", "").replace("qt::", "")
    return s.replace("HIP_vector_type<double, 2u>", "cplx")


def kernel_rows(con):
    return list(con.execute("select name, start, end, duration from kernels order by start"))


def timed_window(rows, warmup: int, steps: int):
    last = max(i for i, r in enumerate(rows) if "k_mlp_train" in r[0])
    ends = [i for i in range(last + 1, len(rows)) if "k_residual" in rows[i][0]]
    if len(ends) < warmup + steps:
        raise SystemExit(f"only {len(ends)} iterations after training")
    lo = ends[warmup - 1] + 1 if warmup > 0 else last + 1
    hi = ends[warmup + steps - 1] + 1
    return rows[lo:hi]


def table(rows, top: int):
    agg = collections.defaultdict(lambda: [0, 0.0])
    for name, _, _, dur in rows:
        a = agg[_short(name)]
        a[0] += 1
        a[1] += dur
    tot = sum(a[1] for a in agg.values())
    out = ["| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for k, (c, t) in sorted(agg.items(), key=lambda x: -x[1][1])[:top]:
        out.append(f"| `{k}` | {c} | {t / 1e6:.1f} | {t / c / 1e3:.1f} | {100 * t / tot:.1f} |")
    out.append(f"\nall kernels: {tot / 1e6:.1f} ms over {sum(a[0] for a in agg.values())} "
               f"dispatches")
    return "\n".join(out), agg


def cmd_kernels(a):
    con = sqlite3.connect(a.db)
    rows = kernel_rows(con)
    txt, _ = table(rows, a.top)
    print("## whole run\n")
    print(txt)
    if a.steps:
        w = timed_window(rows, a.warmup, a.steps)
        txt, agg = table(w, a.top)
        wall = (w[-1][2] - w[0][1]) / 1e6
        print(f"\n## timed window: {a.steps} iterations after {a.warmup} warm-up "
              f"(wall {wall:.1f} ms, {wall / a.steps:.1f} ms per iteration)\n")
        print(txt)
        g = [v for k, v in agg.items() if k.startswith("k_gemm_ex")]
        n = sum(c for c, _ in g)
        t = sum(x for _, x in g)
        if n:
            print(f"\nk_gemm_ex (all tile shapes) in the window: {n} launches, {t / 1e6:.1f} ms, "
                  f"average {t / n / 1e3:.2f} us per launch, {n / a.steps:.1f} launches per "
                  f"iteration")


def cmd_schema(a):
    con = sqlite3.connect(a.db)
    for (name,) in con.execute("select name from sqlite_master where type = 'view'"):
        cols = [r[1] for r in con.execute(f"pragma table_info({name})")]
        print(name, cols)


def cmd_counters(a):
    con = sqlite3.connect(a.db)
    cols = [r[1] for r in con.execute("pragma table_info(counters_collection)")]
    kcol = "kernel_name" if "kernel_name" in cols else "name"
    rows = list(con.execute(f"select {kcol}, counter_name, value, dispatch_id, dispatch_id "
                            f"from counters_collection order by dispatch_id"))
    keep = None
    if a.steps:
        # dispatches of the timed LS iterations (as for ``kernels``)
        seq, seen = [], set()
        for k, _, _, d, t in rows:
            if d not in seen:
                seen.add(d)
                seq.append((k, t, t, 0.0, d))
        w = timed_window([r[:4] for r in seq], a.warmup, a.steps)
        first, last = w[0][1], w[-1][1]
        keep = {r[4] for r in seq if first <= r[1] <= last}
    agg = collections.defaultdict(lambda: [0, 0.0])
    copy_max = {}
    for k, cname, v, d, _ in rows:
        if "copyBuffer" in k or "copy_kernel" in k or "CopyFunctor" in k:
            copy_max[cname] = max(copy_max.get(cname, 0.0), v)
        if keep is not None and d not in keep:
            continue
        x = agg[(_short(k), cname)]
        x[0] += 1
        x[1] += v
    scale = {}
    if a.calib_kib:
        # the calibration copy is the largest copy dispatch of the run
        for cname, v in copy_max.items():
            scale[cname] = v / a.calib_kib
    print("| kernel | counter | dispatches | avg (KiB) | scaled avg (MiB) |")
    print("|---|---|---|---|---|")
    for (k, cname), (c, v) in sorted(agg.items(), key=lambda x: -x[1][1]):
        if a.kernel and a.kernel not in k:
            continue
        s = scale.get(cname)
        sc = f"{v / c / s / 1024:.3f}" if s else "-"
        print(f"| `{k}` | {cname} | {c} | {v / c:.1f} | {sc} |")
    for cname, s in scale.items():
        print(f"\ncalibration {cname}: the copy of {a.calib_kib:.0f} KiB read {s * a.calib_kib:.1f} "
              f"KiB, scale {s:.5f}")
    if a.kernel:
        for cname in sorted({c for _, c in agg}):
            sel = [(c, v) for (k, cn), (c, v) in agg.items() if cn == cname and a.kernel in k]
            n = sum(c for c, _ in sel)
            v = sum(v for _, v in sel)
            s = scale.get(cname, 1.0)
            if n:
                print(f"\n{a.kernel} (all variants) {cname}: {n} dispatches, {v / n / s / 1024:.3f} "
                      f"MiB per dispatch (scaled), {v / n / s * 1024 / 1e6:.3f} MB")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("db")
    k.add_argument("--top", type=int, default=25)
    k.add_argument("--warmup", type=int, default=2)
    k.add_argument("--steps", type=int, default=0)
    c = sub.add_parser("counters")
    c.add_argument("db")
    c.add_argument("--calib-kib", type=float, default=0.0)
    c.add_argument("--kernel", default="")
    c.add_argument("--warmup", type=int, default=1)
    c.add_argument("--steps", type=int, default=0)
    s = sub.add_parser("schema")
    s.add_argument("db")
    a = ap.parse_args()
    {"kernels": cmd_kernels, "counters": cmd_counters, "schema": cmd_schema}[a.cmd](a)


if __name__ == "__main__":
    main()
