"""Launch-shape autotuner for the streaming evaluation kernels.

Times every candidate (unroll, block, workgroups per CU) of a kernel family
on the caller's own table and points with HIP events on the current stream,
keeps the fastest, and installs it with pwl_set_launch.  Results can be saved
to and loaded from a JSON file keyed by kernel family.

    python -m paper_1510_02975_amd.autotune [--log2n 28] [--bwd-log2n 26] [--batch]
"""

import argparse
import itertools
import json
import os

import numpy as np
import torch

from . import binding as B

DEFAULT_CANDIDATES = {
    "unroll": (1, 2, 4),
    "block": (256, 512, 768, 1024),
    "wg_per_cu": (1, 2, 4, 8, 16, 24),
}


def _time(fn, reps, warm=2):
    for i in range(warm):
        fn(i)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for i, (s, e) in enumerate(ev):
        s.record()
        fn(i)
        e.record()
    torch.cuda.synchronize()
    return float(np.median([s.elapsed_time(e) for s, e in ev])) * 1e-3


def tune(kernel, run, candidates=None, reps=10, verbose=False):
    """run(i) launches the kernel once on buffer set i; returns (best config,
    seconds, all results) and installs the best config."""
    cand = dict(DEFAULT_CANDIDATES)
    cand.update(candidates or {})
    results = []
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


def save(path, configs):
    with open(path, "w") as fh:
        json.dump({str(k): list(v) for k, v in configs.items()}, fh, indent=1)


def load(path):
    """Install the configs saved by save(); missing file is a no-op."""
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        raw = json.load(fh)
    out = {}
    for k, v in raw.items():
        B.pwl_set_launch(int(k), *v)
        out[int(k)] = tuple(v)
    return out


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
    best_f, tf, _ = tune(B.KERNEL_FORWARD, lambda i: B.pwl_eval(t, xs[i % 3], ys[i % 3]), verbose=True)
    print("forward best", best_f, "%.1f GB/s" % (8.0 * n / tf / 1e9), flush=True)
    best[B.KERNEL_FORWARD] = best_f
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
        save(args.out, best)


if __name__ == "__main__":
    main()
