"""Benchmark of the CPWL evaluation path on one MI355X.

Workload (the headline one): f(x) = exp(-x^2/2) on [-5, 5], quasi-optimal
partition with N = 1024 segments, L2-projection vertex values; 2^28 FP32
points x = clip(1.5 Z, -5, 5), seed 0, resident in HBM.  One step is one pass
of the whole path: a table is rebuilt in place on the GPU (density scan,
knot inversion, index map, quadrature, FP64 tridiagonal solve, packing) and
then all 2^28 points are evaluated with it.  Steps are pipelined over three
tables and three streams: step i rebuilds table i % 3 on a build stream, up
to two steps ahead (each build waits for the evaluation that last used its
table), and evaluates on stream i % 2 once its table is built, so that the
tail of one evaluation overlaps the start of the next.  Every step does all
the work.  Inputs rotate over three buffers and outputs over four (two
steps' evaluations may run at once), so no step reads the previous step's
cache residue.

Before anything is timed the GPU runs at least WARM_SECONDS of sustained
steps (whatever --warmup says): it raises its clocks under load, and a short
warm-up times the ramp.  The roofline figure is the forward kernel's own
average duration: back-to-back launches on one stream, each between two
fence-free HIP events.  The same steps run back to back on one stream are
reported too ("serial_step_gpoints_s").

Prints one JSON line.  Secondary figures ride along in "extra": the fused
forward+backward on the gradient workload, direct expf, the copy ceiling,
the Lorentzian and J0 tables at N = 256, 1024, 4096, the many-table workload
(one batched launch, its graph replay, the fused backward, one launch per
table from a captured graph and from a host loop, and the unscaled draw of
the point counts), the paper's sample application (per-pixel sums of
Gaussian kernels through a uniform and an optimal table, expf and __expf),
and the paper's own timings with the hardware they were taken on.

    python bench.py [--gpus 1] [--steps 50] [--warmup 20]
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1510_02975_amd.timing import WARM_SECONDS, launch_durations, timed_median, warm_up  # noqa: E402

METRIC = "Gpoints/s fwd and fwd+bwd, % HBM roofline, max err vs FP64 oracle"
HBM_PEAK_GBS = 8000.0
FWD_BYTES_PER_POINT = 8      # x in, y out (FP32)
FUSED_BYTES_PER_POINT = 16   # x, g in; y, dx out
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_eval_fwd_gauss_n1024.json")
CPU_THREADS_MAX = 16         # the GPU machine's CPU share for one GPU
KERNEL_SOURCES = ["paper_1510_02975_amd/csrc/pwl_eval.hip", "paper_1510_02975_amd/csrc/pwl_stream.h",
                  "paper_1510_02975_amd/csrc/pwl_locate.h", "paper_1510_02975_amd/csrc/pwl_internal.h"]


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the kernel sources' code: comments and whitespace are
    dropped, so a reworded comment keeps the counters it was measured with."""
    import re
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the forward kernel from the committed counter
    summary, or None if absent or taken on different kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def host_description():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, os.cpu_count(), avail


def _oracle_rate(work, npoints, seconds):
    """Passes of work() for about `seconds`; returns (Gpoints/s, passes, s)."""
    reps, t0 = 0, time.perf_counter()
    while True:
        work()
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return reps * npoints / el / 1e9, reps, el


def cpu_baseline_leg(spec, x_sample, y_gpu_sample, gspec, xg_sample, gg_sample, seconds):
    """The FP64 oracle (test infrastructure, untuned) on bounded samples of
    the workloads, on one host core and on a thread pool over chunks (NumPy
    releases the GIL inside its array loops): forward = oracle table build +
    evaluation of the headline sample; backward = table build + fused
    forward and backward of the gradient workload's sample.  Also returns the
    GPU output's max error against the oracle on the headline sample."""
    import concurrent.futures as cf
    import oracle as O
    model, ncpu, avail = host_description()
    threads = max(1, min(CPU_THREADS_MAX, avail))
    pool = cf.ThreadPoolExecutor(threads)

    def chunks(a):
        return np.array_split(a, threads)

    x64 = x_sample.astype(np.float64)
    xc = chunks(x64)
    last = {}

    def build(sp):
        return O.build_table(sp["func"], sp["params"], sp["a"], sp["b"], sp["N"], sp["partition"], sp["values"])

    def fwd1():
        tb = build(spec)
        last["y"] = O.evaluate(tb["X"], tb["v"], x64)

    def fwdn():
        tb = build(spec)
        list(pool.map(lambda c: O.evaluate(tb["X"], tb["v"], c), xc))

    xg64, gg64 = xg_sample.astype(np.float64), gg_sample.astype(np.float64)
    xgc, ggc = chunks(xg64), chunks(gg64)

    def bwd1():
        tb = build(gspec)
        O.evaluate_backward(tb["X"], tb["v"], xg64, gg64)

    def bwdn():
        tb = build(gspec)
        list(pool.map(lambda a: O.evaluate_backward(tb["X"], tb["v"], a[0], a[1]), zip(xgc, ggc)))

    f1 = _oracle_rate(fwd1, len(x64), seconds)
    fn = _oracle_rate(fwdn, len(x64), seconds)
    b1 = _oracle_rate(bwd1, len(xg64), seconds)
    bn = _oracle_rate(bwdn, len(xg64), seconds)
    pool.shutdown()
    fmax = float(np.max(np.abs(O.f_value(spec["func"], spec["params"], np.linspace(spec["a"], spec["b"], 100001)))))
    err = float(np.max(np.abs(y_gpu_sample.astype(np.float64) - last["y"]))) / fmax
    return {"value": fn[0], "unit": "Gpoints/s", "cores": threads, "kind": "oracle",
            "sample": "first %d points of the headline workload, table build + evaluation per pass; "
                      "%d threads over chunks: %d passes in %.1f s; one core: %.4f Gpoints/s (%d passes)"
                      % (len(x64), threads, fn[1], fn[2], f1[0], f1[1]),
            "value_1core": f1[0], "host_model": model, "host_cpus": ncpu, "host_cpus_available": avail,
            "bwd": {"workload": "gradient workload (N = 512 projection), first %d points: table build + "
                                "fused forward and backward per pass" % len(xg64),
                    "value": bn[0], "cores": threads, "value_1core": b1[0], "unit": "Gpoints/s"}}, err


# The paper's own timings (Table I and the application table of Sec. VI-A,
# Sec. VI-B, Sec. VI-C): mean per-evaluation times of its synthetic benchmark
# (Gaussian on [0, 8], N + 1 = 32 ... 512 knots) and per-pixel times of its
# application, on an Intel Core i7-2600K (one core) and an NVIDIA GTX 580.
# Context only: another workload on other hardware.
def paper_figures():
    def g(ps):
        return round(1e3 / ps, 4)   # Gpoints/s from picoseconds per evaluation
    knots = [32, 64, 128, 256, 512]
    return {
        "source": "Table I (Sec. VI-A); Sec. VI-B (Lorentzian), Sec. VI-C (J0); application table (Sec. VI-A)",
        "hardware": {"cpu": "Intel Core i7-2600K, sequential, one core", "gpu": "NVIDIA GTX 580"},
        "workload": "Gaussian exp(-x^2/2)/sqrt(2 pi) on [0, 8], N + 1 = 32..512 knots; per-evaluation times",
        "gpoints_s": {
            "cpu_expf": g(13710),
            "cpu_uniform": [g(1780), g(1750)],
            "cpu_optimal_by_knots": dict(zip(map(str, knots), map(g, [8900, 11230, 13830, 16910, 20120]))),
            "gpu_expf": g(33.3),
            "gpu_fast_expf": g(14.2),
            "gpu_uniform_manual": [g(19.8), g(19.7)],
            "gpu_uniform_texture": [g(7.9), g(7.8)],
            "gpu_optimal_manual_by_knots": dict(zip(map(str, knots), map(g, [142.0, 161.9, 181.8, 203.1, 224.1]))),
            "gpu_optimal_texture_by_knots": dict(zip(map(str, knots), map(g, [122.7, 142.9, 163.2, 188.3, 211.1]))),
            "lorentzian_exact_cpu_gpu_gpu_fastdiv": [g(576), g(19.5), g(9.2)],
            "j0_exact_gpu": g(78), "j0_first_asymptotic_term_gpu": g(42),
        },
        "application_ns_per_pixel": {"uniform_texture": 286, "fast_expf": 324, "expf": 391},
    }


def _kernel_rows(csv_path):
    import csv
    with open(csv_path) as fh:
        return list(csv.DictReader(fh))


def _find(dirname, suffix):
    for root, _, files in os.walk(dirname):
        for f in files:
            if f.endswith(suffix):
                return os.path.join(root, f)
    raise FileNotFoundError("no *%s under %s" % (suffix, dirname))


def ingest_pmc(fetch_dir, write_dir, command, n_points):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the forward kernel,
    scaled by the copy kernel's counters over its known 4 n bytes each way;
    writes the traffic record bench.py reports and a text summary."""
    out = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = _kernel_rows(_find(d, "counter_collection.csv"))
        per = {}
        for r in rows:
            if r.get("Counter_Name") != counter:
                continue
            name = r["Kernel_Name"]
            key = "k_eval_fwd" if "k_eval_fwd" in name else ("k_copy" if "k_copy" in name else None)
            if key:
                per.setdefault(key, []).append(float(r["Counter_Value"]) * 1024.0)
        copy_bytes = 4.0 * n_points
        factor = copy_bytes / float(np.median(per["k_copy"]))
        out[counter] = {"k_eval_fwd_raw_bytes": float(np.median(per["k_eval_fwd"])),
                        "k_copy_raw_bytes": float(np.median(per["k_copy"])),
                        "copy_known_bytes": copy_bytes, "scale": factor,
                        "k_eval_fwd_bytes": float(np.median(per["k_eval_fwd"])) * factor,
                        "dispatches": len(per["k_eval_fwd"])}
    total = out["FETCH_SIZE"]["k_eval_fwd_bytes"] + out["WRITE_SIZE"]["k_eval_fwd_bytes"]
    rec = {"kernel": "k_eval_fwd", "workload": "gauss_optimal_n1024_proj_2^%d" % int(np.log2(n_points)),
           "algorithmic_bytes_per_launch": FWD_BYTES_PER_POINT * n_points,
           "hbm_bytes_per_launch": total, "counters": out,
           "kernel_source_hash": kernel_source_hash(), "command": command}
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec, indent=1))


def ingest_trace(trace_dir, out_md, command):
    """Text summary of a rocprofv3 --kernel-trace --stats run: the tool's
    per-kernel statistics, then per (kernel, grid, workgroup) launch shape
    from the dispatch trace, which separates the headline launches from the
    small per-table ones of the same kernel."""
    rows = _kernel_rows(_find(trace_dir, "kernel_stats.csv"))

    def short(name):
        name = name.replace("(anonymous namespace)::", "")
        return name.split("(")[0] if "(" in name else name
    lines = ["# rocprofv3 kernel statistics", "", "Command (from the repository root):", "",
             "    " + command, "", "## Per kernel (rocprofv3 --stats)", "",
             "| kernel | calls | average us | min us | max us | share |",
             "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append("| %s | %s | %.2f | %.2f | %.2f | %.1f%% |" % (
            short(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    trace = _kernel_rows(_find(trace_dir, "kernel_trace.csv"))
    groups = {}
    for r in trace:
        key = (short(r["Kernel_Name"]), int(r["Grid_Size_X"]), int(r["Workgroup_Size_X"]))
        groups.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    lines += ["", "## Per launch shape (dispatch trace; grid in threads)", "",
              "| kernel | grid | workgroup | calls | average us | median us | min us | max us |",
              "|---|---|---|---|---|---|---|---|"]
    for (name, grid, wg), d in sorted(groups.items(), key=lambda kv: -sum(kv[1]))[:24]:
        lines.append("| %s | %d | %d | %d | %.2f | %.2f | %.2f | %.2f |" % (
            name, grid, wg, len(d), float(np.mean(d)), float(np.median(d)), min(d), max(d)))
    # the headline steps: every dispatch before the first copy-kernel launch
    seq = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short(r["Kernel_Name"]),
                  int(r["Grid_Size_X"])) for r in trace)
    first_copy = min([s0 for s0, _, nm, _ in seq if nm.endswith("k_copy")] or [float("inf")])
    head = [(s0, e0, nm, g) for s0, e0, nm, g in seq if s0 < first_copy]
    if head:
        lines += ["", "## Headline steps (the dispatches before the first copy-kernel launch)", "",
                  "| kernel | grid | calls | average us | median us | min us | max us |",
                  "|---|---|---|---|---|---|---|"]
        hg = {}
        for s0, e0, nm, g in head:
            hg.setdefault((nm, g), []).append((e0 - s0) / 1e3)
        for (nm, g), d in sorted(hg.items(), key=lambda kv: -sum(kv[1])):
            lines.append("| %s | %d | %d | %.2f | %.2f | %.2f | %.2f |" % (
                nm, g, len(d), float(np.mean(d)), float(np.median(d)), min(d), max(d)))
        # the evaluation launches that no other dispatch overlaps (the serial
        # steps: the kernel's own duration) and those that share the GPU (the
        # pipelined steps)
        evs = [(s0, e0, g) for s0, e0, nm, g in head if "k_eval_fwd" in nm]
        if evs:
            gmax = max(g for _, _, g in evs)
            alone, shared = [], []
            for s0, e0, g in evs:
                if g != gmax:
                    continue
                hit = any(s1 < e0 and e1 > s0 and (s1, e1) != (s0, e0) for s1, e1, _, _ in head)
                (shared if hit else alone).append((e0 - s0) / 1e3)
            lines += ["", "Evaluation launches of the headline steps (grid %d):" % gmax, "",
                      "| launches | calls | average us | median us | min us | max us |",
                      "|---|---|---|---|---|---|"]
            for label, d in (("no other dispatch running (serial steps)", alone),
                             ("overlapping other dispatches (pipelined steps)", shared)):
                if d:
                    lines.append("| %s | %d | %.2f | %.2f | %.2f | %.2f |" % (
                        label, len(d), float(np.mean(d)), float(np.median(d)), min(d), max(d)))
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def ingest_counters(pmc_dirs, out_md, command):
    """Text summary of rocprofv3 --pmc runs (one directory per pass): per
    kernel and counter, the median value per dispatch."""
    per = {}
    for d in pmc_dirs:
        for r in _kernel_rows(_find(d, "counter_collection.csv")):
            name = r["Kernel_Name"].replace("(anonymous namespace)::", "")
            name = name.split("(")[0] if "(" in name else name
            per.setdefault(name, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    counters = sorted({c for k in per.values() for c in k})
    lines = ["# rocprofv3 counters (median per dispatch)", "", "Commands (from the repository root), one per pass:", ""]
    lines += ["    " + c for c in command.split(" ;; ")]
    lines += ["", "| kernel | dispatches | " + " | ".join(counters) + " |",
              "|---|---|" + "---|" * len(counters)]
    for name, cs in sorted(per.items(), key=lambda kv: kv[0]):
        nd = max(len(v) for v in cs.values())
        cells = ["%.4g" % float(np.median(cs[c])) if c in cs else "" for c in counters]
        lines.append("| %s | %d | %s |" % (name, nd, " | ".join(cells)))
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def batch_extra(torch, P, W, dev, args):
    """Many-table workload: 4096 tables of uneven N and uneven point counts
    (about 2^28 points in total), one batched launch (eager and replayed
    from its captured graph), the fused forward+backward, and the same
    forward as one pwl_eval launch per table, replayed from one captured HIP
    graph (no host overhead) and issued from a host loop; then the same
    tables with the unscaled draw of the point counts."""
    log("batch: building 4096 tables")
    specs = W.many_tables(T=4096, total_points=1 << args.batch_log2n, seed=2)
    tabs = [P.pwl_build(s["func"], s["params"], s["a"], s["b"], s["N"], s["partition"], s["values"],
                        check=False) for s in specs]
    for t in tabs:
        P.pwl_table_check(t)
    x_h, offs = W.many_tables_points(specs, seed=0)
    n = int(offs[-1])
    log("batch: %d points" % n)
    x = torch.from_numpy(x_h).to(dev)
    del x_h
    y = torch.empty_like(x)
    bt = P.pwl_batch_create(tabs, offs)
    t_fwd = timed_median(torch, lambda i: P.pwl_batch_eval(bt, x, y), reps=10)
    P.pwl_batch_capture(bt, x, y)
    t_graph = timed_median(torch, lambda i: P.pwl_batch_replay(bt), reps=10)
    g = torch.from_numpy(W.upstream_grad(n, 1)).to(dev)
    dx = torch.empty_like(x)
    dv = torch.empty(bt.dv_len, dtype=torch.float32, device=dev)
    t_fb = timed_median(torch, lambda i: P.pwl_batch_eval_backward(bt, x, g, y, dx, dv), reps=10)
    if args.quick:   # profiling runs: the batched launches only
        bt.free()
        for t in tabs:
            t.free()
        return {"batch_fwd_gpoints_s": n / t_fwd / 1e9, "batch_fwd_bwd_gpoints_s": n / t_fb / 1e9}
    o = [int(v) for v in offs]
    views = [(t, x[o[k]:o[k + 1]], y[o[k]:o[k + 1]]) for k, t in enumerate(tabs) if o[k + 1] > o[k]]

    def per_table(i):
        for t, xs, ys in views:
            P.pwl_eval(t, xs, ys)
    t_loop = timed_median(torch, per_table, reps=3, warm_seconds=0.0)
    # the same launches captured into one graph: replaying it costs no host time
    gr = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cap):
        per_table(0)   # one eager pass on the capture stream first
    torch.cuda.current_stream().wait_stream(cap)
    torch.cuda.synchronize()
    with torch.cuda.graph(gr, stream=cap, capture_error_mode="thread_local"):
        per_table(0)
    t_per = timed_median(torch, lambda i: gr.replay(), reps=5)
    del gr
    table_bytes = sum(28 * s["N"] for s in specs)
    out = {"batch_workload": "4096 tables (Gaussian/Lorentzian/J0, N log-uniform 16..4096), %d points" % n,
           "batch_fwd_gpoints_s": n / t_fwd / 1e9,
           "batch_fwd_hbm_frac": FWD_BYTES_PER_POINT * n / t_fwd / 1e9 / HBM_PEAK_GBS,
           "batch_fwd_graph_gpoints_s": n / t_graph / 1e9,
           "batch_fwd_bwd_gpoints_s": n / t_fb / 1e9,
           "batch_fwd_bwd_hbm_frac": FUSED_BYTES_PER_POINT * n / t_fb / 1e9 / HBM_PEAK_GBS,
           "batch_per_table_launches_graph_gpoints_s": n / t_per / 1e9,
           "batch_per_table_launches_host_loop_gpoints_s": n / t_loop / 1e9,
           "batch_speedup_vs_per_table_graph": t_per / t_fwd,
           "batch_grid_fwd": bt.grid_fwd, "batch_runs_fwd": bt.runs_fwd,
           "batch_grid_bwd": bt.grid_bwd, "batch_runs_bwd": bt.runs_bwd,
           "batch_table_bytes": table_bytes}
    bt.free()
    del x, y, g, dx, dv, views
    if not args.no_unscaled:
        # the configuration's raw draw of the counts (about 2^29.2 points)
        specs_u = W.many_tables(T=4096, seed=2, scale_to_total=False)
        xu_h, offs_u = W.many_tables_points(specs_u, seed=0)
        nu = int(offs_u[-1])
        log("batch: unscaled draw, %d points" % nu)
        xu = torch.from_numpy(xu_h).to(dev)
        del xu_h
        yu = torch.empty_like(xu)
        btu = P.pwl_batch_create(tabs, offs_u)
        tu = timed_median(torch, lambda i: P.pwl_batch_eval(btu, xu, yu), reps=5)
        gu = torch.from_numpy(W.upstream_grad(nu, 1)).to(dev)
        dxu = torch.empty_like(xu)
        dvu = torch.empty(btu.dv_len, dtype=torch.float32, device=dev)
        tub = timed_median(torch, lambda i: P.pwl_batch_eval_backward(btu, xu, gu, yu, dxu, dvu), reps=5)
        out.update({"batch_unscaled_points": nu,
                    "batch_unscaled_counts_min_max": [int(np.min(np.diff(offs_u))), int(np.max(np.diff(offs_u)))],
                    "batch_unscaled_fwd_gpoints_s": nu / tu / 1e9,
                    "batch_unscaled_fwd_hbm_frac": FWD_BYTES_PER_POINT * nu / tu / 1e9 / HBM_PEAK_GBS,
                    "batch_unscaled_fwd_bwd_gpoints_s": nu / tub / 1e9,
                    "batch_unscaled_fwd_bwd_hbm_frac": FUSED_BYTES_PER_POINT * nu / tub / 1e9 / HBM_PEAK_GBS})
        btu.free()
        del xu, yu, gu, dxu, dvu
    for t in tabs:
        t.free()
    return out


def c3_extra(torch, P, W, dev):
    """Lorentzian on [-20, 20] and J0 on [0, 50], optimal partition, N in
    {256, 1024, 4096}, projection values, 2^27 uniform points: forward
    throughput per table size (the LDS footprint grows with N)."""
    out = {}
    for spec in (W.LORENTZ, W.BESSEL):
        n = spec["n"]
        x_h = W.uniform_points(spec["a"], spec["b"], n, 0)
        xs = [torch.from_numpy(x_h).to(dev) for _ in range(2)]
        del x_h
        ys = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(2)]
        for N in (256, 1024, 4096):
            t = P.pwl_build(spec["func"], spec["params"], spec["a"], spec["b"], N, spec["partition"], W.PROJ)
            s = timed_median(torch, lambda i: P.pwl_eval(t, xs[i % 2], ys[i % 2]))
            key = "%s_n%d" % (spec["name"].split("_")[0], N)
            out[key + "_gpoints_s"] = n / s / 1e9
            out[key + "_hbm_frac"] = FWD_BYTES_PER_POINT * n / s / 1e9 / HBM_PEAK_GBS
            t.free()
        del xs, ys
    return out


def kde_extra(torch, P, W, dev):
    """The sample application (per-pixel sums of Gaussian kernels, T = 16
    reference frames, 5 x 5 windows: 1200 kernel values per pixel) at CIF
    and 1080p, with the kernel through a table of exp(-u^2/2) on [0, 8] -
    uniform partition (the paper's choice for this application), N = 64 and
    1024, and the optimal partition, N = 1024 - and through expf and __expf:
    mean time per pixel."""
    c = W.KDE_CIF
    tables = {"table_uniform_n64": P.pwl_build(0, (1.0, 1.0), 0.0, 8.0, 64, 0, 1),
              "table_uniform_n1024": P.pwl_build(0, (1.0, 1.0), 0.0, 8.0, 1024, 0, 1),
              "table_optimal_n1024": P.pwl_build(0, (1.0, 1.0), 0.0, 8.0, 1024, 1, 1)}
    out = {}
    for label, H, Wd in (("cif", c["H"], c["W"]), ("1080p", 1080, 1920)):
        f_h, h_h = W.kde_frames(H, Wd, c["T"], seed=4)
        f, h = torch.from_numpy(f_h).to(dev), torch.from_numpy(h_h).to(dev)
        y = torch.empty((H, Wd), dtype=torch.float32, device=dev)
        runs = [(name, P.KDE_TABLE, t) for name, t in tables.items()]
        runs += [("expf", P.KDE_EXPF, None), ("fast_expf", P.KDE_FAST_EXPF, None)]
        for name, mode, t in runs:
            s = timed_median(torch, lambda i: P.pwl_kde(t, mode, f, h, c["radius"], c["sigma"], y), reps=10)
            out["kde_%s_%s_ns_per_pixel" % (label, name)] = s / (H * Wd) * 1e9
        del f, h, y
    for t in tables.values():
        t.free()
    out["kde_kernel_values_per_pixel"] = 3 * c["T"] * (2 * c["radius"] + 1) ** 2
    return out


def layout_extra(torch, P, table, xs, ys, n):
    """The forward's locate (index map, or the paper's binary search over
    the knots, Sec. IV-V) and record layout (packed or structure of arrays,
    Sec. V) on the headline table and points: every pair, and which one the
    library runs."""
    mode, rec = P.pwl_get_locate(), P.pwl_get_records()
    out = {}
    for lo, ln in ((P.LOCATE_MAP, "map"), (P.LOCATE_SEARCH, "search")):
        for rc, rn in ((P.RECORDS_PACKED, "packed"), (P.RECORDS_SOA, "soa"), (P.RECORDS_PAIRS, "pairs")):
            P.pwl_set_locate(lo)
            P.pwl_set_records(rc)
            t = timed_median(torch, lambda i: P.pwl_eval(table, xs[i % len(xs)], ys[i % len(ys)]))
            out["fwd_%s_%s_us" % (ln, rn)] = t * 1e6
    P.pwl_set_locate(mode)
    P.pwl_set_records(rec)
    out["fwd_layout_in_use"] = "%s_%s" % ("map" if mode == P.LOCATE_MAP else "search",
                                          {P.RECORDS_PACKED: "packed", P.RECORDS_SOA: "soa",
                                           P.RECORDS_PAIRS: "pairs"}[rec])
    return out


def fused_extra(torch, P, W, dev):
    """Fused forward + backward on the gradient workload (N = 512 projection,
    2^26 points, x and g ~ N(0, 1)): the library's launch shape and a few
    others timed in the same run."""
    gs = dict(W.GRAD)
    ng = gs["n"]
    xg_h, gg_h = W.grad_inputs(ng)
    tg = P.pwl_build(gs["func"], gs["params"], gs["a"], gs["b"], gs["N"], gs["partition"], gs["values"])
    xg = [torch.from_numpy(xg_h).to(dev) for _ in range(2)]
    gg = [torch.from_numpy(gg_h).to(dev) for _ in range(2)]
    yg = [torch.empty(ng, dtype=torch.float32, device=dev) for _ in range(2)]
    dxg = [torch.empty(ng, dtype=torch.float32, device=dev) for _ in range(2)]
    dvg = torch.empty(gs["N"] + 1, dtype=torch.float32, device=dev)
    fb = lambda i: P.pwl_eval_backward(tg, xg[i % 2], gg[i % 2], yg[i % 2], dxg[i % 2], dvg)
    lib_shape = P.pwl_get_launch(P.KERNEL_BACKWARD)
    shapes = {}
    for shape in (lib_shape, (2, 512, 2), (2, 256, 4), (4, 1024, 1)):
        P.pwl_set_launch(P.KERNEL_BACKWARD, *shape)
        shapes["x".join(str(v) for v in shape)] = timed_median(torch, fb)
    P.pwl_set_launch(P.KERNEL_BACKWARD, *lib_shape)
    default = "x".join(str(v) for v in lib_shape)
    d = launch_durations(torch, fb, reps=20)
    t_fb = float(np.mean(d))
    best = min(shapes, key=shapes.get)
    out = {"fwd_bwd_workload": "gauss_optimal_n512_proj, 2^26 points x~N(0,1), g~N(0,1)",
           "fwd_bwd_gpoints_s": ng / t_fb / 1e9,
           "fwd_bwd_hbm_frac": FUSED_BYTES_PER_POINT * ng / t_fb / 1e9 / HBM_PEAK_GBS,
           "fwd_bwd_us_mean": t_fb * 1e6,
           "fwd_bwd_launch": default, "fwd_bwd_best_launch": best,
           "fwd_bwd_best_gpoints_s": ng / shapes[best] / 1e9,
           "fwd_bwd_us_by_launch": {k: v * 1e6 for k, v in shapes.items()}}
    del xg, gg, yg, dxg
    tg.free()
    return out, xg_h, gg_h


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--ingest-pmc":
        # --ingest-pmc FETCH_DIR WRITE_DIR LOG2N "command"
        ingest_pmc(sys.argv[2], sys.argv[3], sys.argv[5], 1 << int(sys.argv[4]))
        return 0
    if len(sys.argv) > 1 and sys.argv[1] == "--ingest-counters":
        # --ingest-counters OUT_MD "cmd1 ;; cmd2 ..." DIR...
        ingest_counters(sys.argv[4:], sys.argv[2], sys.argv[3])
        return 0
    if len(sys.argv) > 1 and sys.argv[1] == "--ingest-trace":
        # --ingest-trace TRACE_DIR OUT_MD "command"
        ingest_trace(sys.argv[2], sys.argv[3], sys.argv[4])
        return 0
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--cpu-seconds", type=float, default=6.0)
    ap.add_argument("--cpu-sample-log2", type=int, default=23)
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-unscaled", action="store_true")
    ap.add_argument("--batch-log2n", type=int, default=28)
    ap.add_argument("--legs", default="layout,direct,fused,c3,kde,batch",
                    help="secondary measurements to run (comma list; --no-extra runs none)")
    ap.add_argument("--quick", action="store_true",
                    help="for profiler runs: the batch leg times only its batched launches")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        return 2

    import torch
    import workloads as W
    import paper_1510_02975_amd as P
    from paper_1510_02975_amd import build as B
    if not os.path.exists(P.binding.LIB_PATH):
        B.build()
    P.load_library()
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)

    spec = dict(W.GAUSS_BIG)
    n = 1 << args.log2n
    log("generating %d points" % n)
    x_host = W.gauss_big_points(n)
    sets = 3
    xs = [torch.from_numpy(x_host).to(dev) for _ in range(sets)]
    ys = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(sets + 1)]
    # three tables: step i rebuilds table i % 3 on the build stream, up to
    # two steps ahead of its evaluation
    ntab = 3
    tables = [P.pwl_build(spec["func"], spec["params"], spec["a"], spec["b"], spec["N"],
                          spec["partition"], spec["values"]) for _ in range(ntab)]
    main = torch.cuda.current_stream()
    other = torch.cuda.Stream()   # default priority, like every stream here
    side = torch.cuda.Stream()

    def rebuild(t, stream):
        P.pwl_rebuild(t, spec["func"], spec["params"], spec["a"], spec["b"], spec["partition"],
                      spec["values"], stream=stream)

    def run_steps(steps):
        """Pipelined steps: the evaluation of step i (stream i % 2) waits for
        the build of its table; the build of step i + 2 waits for the
        evaluation (step i - 1) that last used its table."""
        evs = (main, other)
        built = [torch.cuda.Event() for _ in range(ntab)]
        used = [torch.cuda.Event() for _ in range(ntab)]
        other.wait_stream(main)
        side.wait_stream(main)
        ahead = ntab - 1
        for j in range(min(ahead, steps)):
            rebuild(tables[j % ntab], side)
            built[j % ntab].record(side)
        for i in range(steps):
            k = i % ntab
            s = evs[i % 2]
            s.wait_event(built[k])
            P.pwl_eval(tables[k], xs[i % sets], ys[i % len(ys)], stream=s)
            used[k].record(s)
            j = i + ahead
            if j < steps:
                if i >= 1:
                    side.wait_event(used[j % ntab])
                rebuild(tables[j % ntab], side)
                built[j % ntab].record(side)
        main.wait_stream(other)
        main.wait_stream(side)

    def serial_steps(steps):
        for i in range(steps):
            rebuild(tables[0], main)
            P.pwl_eval(tables[0], xs[i % sets], ys[i % sets], stream=main)

    # warm-up: --warmup steps, and at least WARM_SECONDS of them
    log("warmup: %d steps and at least %.2f s" % (args.warmup, WARM_SECONDS))
    t0 = time.perf_counter()
    run_steps(args.warmup)
    torch.cuda.synchronize()
    while time.perf_counter() - t0 < WARM_SECONDS:
        run_steps(max(4, args.warmup))
        torch.cuda.synchronize()
    warm_s = time.perf_counter() - t0
    for t in tables:
        assert P.pwl_table_check(t) == 0
    torch.cuda.synchronize()

    log("timing %d steps" % args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_steps(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    m_cpu = min(n, 1 << args.cpu_sample_log2)
    y_sample = ys[(args.steps - 1) % len(ys)][:m_cpu].cpu().numpy()   # before anything reuses ys
    # the same steps on one stream, for reference
    warm_up(torch, lambda i: serial_steps(1))
    torch.cuda.synchronize()
    ts0 = time.perf_counter()
    serial_steps(args.steps)
    torch.cuda.synchronize()
    serial_wall = time.perf_counter() - ts0
    # the forward kernel alone: back-to-back launches on one stream
    reps = max(20, args.steps)
    d_eval = launch_durations(torch, lambda i: P.pwl_eval(tables[0], xs[i % sets], ys[i % len(ys)]), reps=reps)
    eval_s = float(np.mean(d_eval))
    # the build alone (all its kernels, one stream)
    d_build = launch_durations(torch, lambda i: rebuild(tables[0], main), reps=20)
    build_s = float(np.mean(d_build))
    value = n * args.steps / wall / 1e9
    achieved = FWD_BYTES_PER_POINT * n / eval_s / 1e9
    log("step %.3f ms, eval kernel %.1f us (%.0f GB/s), build %.1f us"
        % (wall / args.steps * 1e3, eval_s * 1e6, achieved, build_s * 1e6))
    traffic = measured_traffic()

    extra = {"warmup_seconds": warm_s,
             "eval_kernel_us": eval_s * 1e6, "eval_kernel_us_median": float(np.median(d_eval)) * 1e6,
             "eval_kernel_launches_timed": reps, "build_us": build_s * 1e6,
             "eval_only_gpoints_s": n / eval_s / 1e9,
             "pipelined_step_us": wall / args.steps * 1e6,
             "serial_step_gpoints_s": n * args.steps / serial_wall / 1e9,
             "kernel_source_hash": kernel_source_hash(),
             "launch": {"forward": P.pwl_get_launch(P.KERNEL_FORWARD),
                        "backward": P.pwl_get_launch(P.KERNEL_BACKWARD),
                        "batch_forward": P.pwl_get_launch(P.KERNEL_BATCH),
                        "batch_backward": P.pwl_get_launch(P.KERNEL_BATCH_BACKWARD),
                        "locate": "search" if P.pwl_get_locate() == P.LOCATE_SEARCH else "map",
                        "tuned_from": P.binding.TUNED_SOURCE}}
    # the copy kernel in the forward's launch shape: the practical HBM ceiling
    d_copy = launch_durations(torch, lambda i: P.pwl_copy(xs[i % sets], ys[i % len(ys)]), reps=20)
    extra["copy_GBs"] = 8.0 * n / float(np.mean(d_copy)) / 1e9
    extra["eval_vs_copy"] = float(np.mean(d_copy)) / eval_s
    extra["paper"] = paper_figures()
    xg_h = gg_h = None
    legs = set() if args.no_extra else set(args.legs.split(","))
    if args.no_batch:
        legs.discard("batch")
    if "layout" in legs:
        log("extras: locate and record-layout A/B")
        extra.update(layout_extra(torch, P, tables[0], xs, ys, n))
    if "direct" in legs:
        log("extras: direct expf")
        for fast in (0, 1):
            t = timed_median(torch, lambda i: P.pwl_direct_gaussian(xs[i % sets], ys[i % sets], 1.0, 1.0, fast))
            extra["direct_%s_gpoints_s" % ("fast_expf" if fast else "expf")] = n / t / 1e9
    if "fused" in legs:
        log("extras: fused forward+backward")
        fx, xg_h, gg_h = fused_extra(torch, P, W, dev)
        extra.update(fx)
    if "c3" in legs:
        log("extras: Lorentzian and J0 tables, 2^27 points")
        extra.update(c3_extra(torch, P, W, dev))
    if "kde" in legs:
        log("extras: sample application (per-pixel kernel sums)")
        extra.update(kde_extra(torch, P, W, dev))
    if "batch" in legs:
        del xs, ys
        extra.update(batch_extra(torch, P, W, dev, args))

    cpu = None
    max_err = None
    if not args.no_cpu:
        if xg_h is None:
            xg_h, gg_h = W.grad_inputs(W.GRAD["n"])
        mg = min(len(xg_h), 1 << (args.cpu_sample_log2 - 1))
        log("cpu baseline on %d + %d points" % (m_cpu, mg))
        cpu, max_err = cpu_baseline_leg(spec, x_host[:m_cpu], y_sample, dict(W.GRAD), xg_h[:mg], gg_h[:mg],
                                        args.cpu_seconds)
        extra["max_err_rel_maxf_on_cpu_sample"] = max_err

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "Gpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "gauss_optimal_n1024_proj_2^%d" % args.log2n,
                   "f": "exp(-x^2/2)", "domain": [-5.0, 5.0], "N": 1024, "partition": "optimal",
                   "values": "L2 projection", "points": n, "x": "clip(1.5 Z, -5, 5), seed 0",
                   "step": "GPU table rebuild + forward evaluation of all points; builds run up to two "
                           "steps ahead on their own stream (three tables), evaluations alternate over "
                           "two streams"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_eval_fwd", "algorithmic_bytes_per_launch": FWD_BYTES_PER_POINT * n},
        "cpu_baseline": cpu,
        "max_err": max_err,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)
    for t in tables:
        t.free()
    return 0


if __name__ == "__main__":
    sys.exit(main())
