"""Autotuner for the streaming evaluation kernels.

Axes: the launch shape (unroll, block, workgroups per CU) of every kernel
family, and for the forward the segment locate (index map, or the paper's
branch-free binary search over the knots, Sec. IV-V) and the arrangement of
the per-segment data in LDS (packed records or structure of arrays, Sec. V).
Every candidate is timed on the caller's own table and points with
fence-free HIP events on the current stream, after a time-based warm-up;
the fastest is installed.  save() writes the choices in the format the
binding applies when it loads the library (tuned_mi355x.json beside this
file), so the shipped configuration is the tuner's.

    python -m paper_1510_02975_amd.autotune [--log2n 28] [--bwd-log2n 26] [--batch] [--out FILE]
"""

import argparse
import itertools
import json
import os

import torch

from . import binding as B
from .timing import timed_median, warm_up

DEFAULT_CANDIDATES = {
    "unroll": (1, 2, 4),
    "block": (256, 512, 768, 1024),
    "wg_per_cu": (1, 2, 3, 4, 6, 8, 16, 24, 32),
}
LOCATE_NAMES = {B.LOCATE_MAP: "map", B.LOCATE_SEARCH: "search"}
RECORDS_NAMES = {B.RECORDS_PACKED: "packed", B.RECORDS_SOA: "soa", B.RECORDS_PAIRS: "pairs"}


def _time(fn, reps, warm_seconds=0.05):
    return timed_median(torch, fn, reps=reps, warm_seconds=warm_seconds)


def tune(kernel, run, candidates=None, reps=10, verbose=False):
    """run(i) launches the kernel once on buffer set i; returns (best config,
    seconds, all results) and installs the best config."""
    cand = dict(DEFAULT_CANDIDATES)
    cand.update(candidates or {})
    results = []
    warm_up(torch, run)
    for u, blk, w in itertools.product(cand["unroll"], cand["block"], cand["wg_per_cu"]):
        B.pwl_set_launch(kernel, u, blk, w)
        t = _time(run, reps)
        results.append((t, (u, blk, w)))
        if verbose:
            print("  kernel %d unroll %d block %4d wg/CU %d: %.1f us" % (kernel, u, blk, w, t * 1e6), flush=True)
    results.sort()
    best_t, best = results[0]
    B.pwl_set_launch(kernel, *best)
    return best, best_t, results


def tune_batch(tables, offsets, x, y, g=None, dx=None, dv=None, candidates=None, reps=5, verbose=False):
    """Batched kernels: the launch grids are planned when the batch is
    created, so every candidate gets its own batch.  Tunes PWL_KERNEL_BATCH
    on the forward and, when g is given, PWL_KERNEL_BATCH_BACKWARD on the
    fused backward; installs the best shapes and returns {kernel: (best, s)}."""
    cand = dict(DEFAULT_CANDIDATES)
    cand.update(candidates or {})
    out = {}
    kinds = [(B.KERNEL_BATCH, lambda bt: (lambda i: B.pwl_batch_eval(bt, x, y)))]
    if g is not None:
        kinds.append((B.KERNEL_BATCH_BACKWARD,
                      lambda bt: (lambda i: B.pwl_batch_eval_backward(bt, x, g, y, dx, dv))))
    for kernel, make in kinds:
        results = []
        for u, blk, w in itertools.product(cand["unroll"], cand["block"], cand["wg_per_cu"]):
            B.pwl_set_launch(kernel, u, blk, w)
            bt = B.pwl_batch_create(tables, offsets)
            t = _time(make(bt), reps)
            bt.free()
            results.append((t, (u, blk, w)))
            if verbose:
                print("  batch kernel %d unroll %d block %4d wg/CU %d: %.1f us" % (kernel, u, blk, w, t * 1e6),
                      flush=True)
        results.sort()
        B.pwl_set_launch(kernel, *results[0][1])
        out[kernel] = (results[0][1], results[0][0])
    return out


def tune_layout(run, reps=10, verbose=False):
    """The forward's layout A/B at its current launch shape: every
    (locate, records) pair, timed by run(i); installs and returns the best
    pair, its seconds and all results {(locate, records): seconds}."""
    warm_up(torch, run)
    res = {}
    for loc, rec in itertools.product((B.LOCATE_MAP, B.LOCATE_SEARCH), tuple(RECORDS_NAMES)):
        B.pwl_set_locate(loc)
        B.pwl_set_records(rec)
        res[loc, rec] = _time(run, reps)
        if verbose:
            print("  forward locate %-6s records %-6s: %.1f us"
                  % (LOCATE_NAMES[loc], RECORDS_NAMES[rec], res[loc, rec] * 1e6), flush=True)
    best = min(res, key=res.get)
    B.pwl_set_locate(best[0])
    B.pwl_set_records(best[1])
    return best, res[best], res


def save(path, launch, locate=None, records=None, source=None, timings=None):
    """Write the tuned choices: launch {kernel family: (unroll, block,
    wg_per_cu)}, the forward's locate mode and record layout."""
    rec = {"source": source or "paper_1510_02975_amd.autotune",
           "launch": {str(k): list(v) for k, v in launch.items()}}
    if locate is not None:
        rec["locate"] = int(locate)
    if records is not None:
        rec["records"] = int(records)
    if timings:
        rec["timings_us"] = timings
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)


def load(path):
    """Install the choices saved by save(); a missing file is a no-op."""
    return B.apply_tuned(path)


def main():
    import workloads as W
    ap = argparse.ArgumentParser()
    ap.add_argument("--log2n", type=int, default=28, help="points for the forward and batch kernels")
    ap.add_argument("--bwd-log2n", type=int, default=26, help="points for the fused backward")
    ap.add_argument("--out", default=None)
    ap.add_argument("--batch", action="store_true")
    args = ap.parse_args()
    B.load_library()
    dev = torch.device("cuda", 0)
    best = {}
    # forward: the headline table and points
    n = 1 << args.log2n
    spec = W.GAUSS_BIG
    t = B.pwl_build(spec["func"], spec["params"], spec["a"], spec["b"], spec["N"], spec["partition"],
                    spec["values"])
    xh = W.gauss_big_points(n)
    xs = [torch.from_numpy(xh).to(dev) for _ in range(3)]
    del xh
    ys = [torch.empty(n, device=dev) for _ in range(3)]
    fwd = lambda i: B.pwl_eval(t, xs[i % 3], ys[i % 3])
    B.pwl_set_locate(B.LOCATE_MAP)
    B.pwl_set_records(B.RECORDS_PACKED)
    best_f, tf, _ = tune(B.KERNEL_FORWARD, fwd, verbose=True)
    print("forward best", best_f, "%.1f GB/s" % (8.0 * n / tf / 1e9), flush=True)
    best[B.KERNEL_FORWARD] = best_f
    (loc, rec), tl, lres = tune_layout(fwd, verbose=True)
    print("forward layout A/B at %s (locate x records, us):" % (best_f,), flush=True)
    for (lo, rc), sec in sorted(lres.items()):
        print("  %-6s %-6s %8.1f us  %6.1f Gpoints/s" % (LOCATE_NAMES[lo], RECORDS_NAMES[rc], sec * 1e6, n / sec / 1e9),
              flush=True)
    print("forward layout best: locate %s, records %s" % (LOCATE_NAMES[loc], RECORDS_NAMES[rec]), flush=True)
    timings = {"forward_%s_%s" % (LOCATE_NAMES[lo], RECORDS_NAMES[rc]): sec * 1e6 for (lo, rc), sec in lres.items()}
    del xs, ys
    # fused backward: the gradient workload (x, g ~ N(0, 1))
    gs = W.GRAD
    nb = 1 << args.bwd_log2n
    tg = B.pwl_build(gs["func"], gs["params"], gs["a"], gs["b"], gs["N"], gs["partition"], gs["values"])
    xh, gh = W.grad_inputs(nb)
    xb = [torch.from_numpy(xh).to(dev) for _ in range(2)]
    gg = [torch.from_numpy(gh).to(dev) for _ in range(2)]
    yb = [torch.empty(nb, device=dev) for _ in range(2)]
    dx = [torch.empty(nb, device=dev) for _ in range(2)]
    dv = torch.empty(gs["N"] + 1, device=dev)
    best_b, tb, _ = tune(B.KERNEL_BACKWARD,
                         lambda i: B.pwl_eval_backward(tg, xb[i % 2], gg[i % 2], yb[i % 2], dx[i % 2], dv),
                         verbose=True)
    print("backward best", best_b, "%.1f GB/s" % (16.0 * nb / tb / 1e9), flush=True)
    best[B.KERNEL_BACKWARD] = best_b
    del xb, gg, yb, dx
    if args.batch:
        specs = W.many_tables(T=4096, total_points=n, seed=2)
        tabs = [B.pwl_build(s["func"], s["params"], s["a"], s["b"], s["N"], s["partition"], s["values"])
                for s in specs]
        xh, offs = W.many_tables_points(specs, seed=0)
        xm = torch.from_numpy(xh).to(dev)
        del xh
        ym = torch.empty_like(xm)
        gm = torch.from_numpy(W.upstream_grad(xm.numel(), 1)).to(dev)
        dxm = torch.empty_like(xm)
        bt = B.pwl_batch_create(tabs, offs)
        dvm = torch.empty(bt.dv_len, device=dev)
        bt.free()
        res = tune_batch(tabs, offs, xm, ym, gm, dxm, dvm, verbose=True)
        for kernel, (shape, sec) in res.items():
            print("batch kernel %d best" % kernel, shape, "%.1f us, %.1f Gpoints/s" % (sec * 1e6, xm.numel() / sec / 1e9),
                  flush=True)
            best[kernel] = shape
    if args.out:
        save(args.out, best, locate=loc, records=rec, timings=timings,
             source="paper_1510_02975_amd.autotune --log2n %d --bwd-log2n %d%s on MI355X"
                    % (args.log2n, args.bwd_log2n, " --batch" if args.batch else ""))


if __name__ == "__main__":
    main()
