"""Batched multi-table evaluation (one launch per direction) against per-table
launches and the FP64 oracle, and its captured HIP graph replayed several
times with the program's own work in between."""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests.gpu_util import GRAD_TOL, Y_TOL, device, fmax_abs, launch_shape, library, say

pytestmark = pytest.mark.gpu


def _tables(P, T=40, seed=7, max_n=4096):
    """Mixed tables (the many-table recipe at a small total) plus the points."""
    specs = W.many_tables(T=T, total_points=1 << 21, seed=seed)
    rng = np.random.default_rng(seed)
    for k, s in enumerate(specs):
        s["N"] = int(min(s["N"], max_n))
        if k % 9 == 4:
            s["n"] = 0                    # empty tables
        elif k % 7 == 3:
            s["n"] = int(rng.integers(1, 6))   # a handful of points, odd offsets
    tabs = [P.pwl_build(s["func"], s["params"], s["a"], s["b"], s["N"], s["partition"], s["values"])
            for s in specs]
    x, offs = W.many_tables_points(specs, seed=0)
    return specs, tabs, x, offs


def test_batch_forward_matches_per_table_and_oracle():
    import paper_1510_02975_amd as P
    library()
    dev = device()
    specs, tabs, x, offs = _tables(P)
    say("batch forward: %d tables, %d points" % (len(tabs), len(x)))
    xt = torch.from_numpy(x).to(dev)
    bt = P.pwl_batch_create(tabs, offs)
    assert bt.npoints == len(x) and bt.T == len(tabs)
    y = P.pwl_batch_eval(bt, xt).cpu().numpy()
    for t, s, o0, o1 in zip(tabs, specs, offs[:-1], offs[1:]):
        if o1 == o0:
            continue
        y1 = P.pwl_eval(t, xt[o0:o1]).cpu().numpy()
        assert np.array_equal(y[o0:o1], y1)          # same kernel body, bit for bit
        d = P.pwl_table_download(t)
        yr = O.evaluate(d["knots"].astype(np.float64), d["values"].astype(np.float64),
                        x[o0:o1].astype(np.float64))
        assert np.max(np.abs(y[o0:o1] - yr)) <= Y_TOL * fmax_abs(s["func"], s["params"], s["a"], s["b"])
    bt.free()


def test_batch_backward_matches_per_table():
    import paper_1510_02975_amd as P
    library()
    dev = device()
    specs, tabs, x, offs = _tables(P, T=25, seed=3)
    g = W.upstream_grad(len(x), 5)
    xt, gt = torch.from_numpy(x).to(dev), torch.from_numpy(g).to(dev)
    bt = P.pwl_batch_create(tabs, offs)
    y, dx, dv = P.pwl_batch_eval_backward(bt, xt, gt)
    y, dx, dv = y.cpu().numpy(), dx.cpu().numpy(), dv.cpu().numpy()
    # without y and dx (dL/dv is summed from per-workgroup partials with FP32
    # atomics, so two calls agree to the error bound, not bit for bit)
    _, _, dv2 = P.pwl_batch_eval_backward(bt, xt, gt, want=())
    dv2 = dv2.cpu().numpy()
    for i, (t, o0, o1) in enumerate(zip(tabs, offs[:-1], offs[1:])):
        d0, d1 = bt.dv_offsets[i], bt.dv_offsets[i + 1]
        if o1 == o0:
            assert np.all(dv[d0:d1] == 0.0) and np.all(dv2[d0:d1] == 0.0)
            continue
        y1, dx1, dv1 = P.pwl_eval_backward(t, xt[o0:o1], gt[o0:o1])
        assert np.array_equal(y[o0:o1], y1.cpu().numpy())
        assert np.array_equal(dx[o0:o1], dx1.cpu().numpy())
        d = P.pwl_table_download(t)
        X = d["knots"].astype(np.float64)
        _, _, dvr = O.evaluate_backward(X, d["values"].astype(np.float64), x[o0:o1].astype(np.float64),
                                        g[o0:o1].astype(np.float64))
        _, _, wk = O.evaluate_backward(X, np.zeros(len(X)), x[o0:o1].astype(np.float64),
                                       np.abs(g[o0:o1]).astype(np.float64))
        assert np.all(np.abs(dv[d0:d1] - dvr) <= GRAD_TOL * wk + 1e-30)
        assert np.all(np.abs(dv2[d0:d1] - dvr) <= GRAD_TOL * wk + 1e-30)
    bt.free()


def test_batch_graph_replays_match_eager():
    import paper_1510_02975_amd as P
    library()
    dev = device()
    specs, tabs, x, offs = _tables(P, T=30, seed=11)
    g = W.upstream_grad(len(x), 2)
    xt, gt = torch.from_numpy(x).to(dev), torch.from_numpy(g).to(dev)
    bt = P.pwl_batch_create(tabs, offs)
    y_e = P.pwl_batch_eval(bt, xt).clone()
    ye, dxe, dve = P.pwl_batch_eval_backward(bt, xt, gt)
    ye, dxe, dve = ye.clone(), dxe.clone(), dve.clone()
    y = torch.full_like(xt, 7.0)
    P.pwl_batch_capture(bt, xt, y)
    for rep in range(4):
        y.fill_(float(rep))                    # eager work between replays
        torch.cuda.synchronize()
        P.pwl_batch_replay(bt)
        torch.cuda.synchronize()
        assert torch.equal(y, y_e), rep
    yb, dxb = torch.empty_like(xt), torch.empty_like(xt)
    dvb = torch.full((bt.dv_len,), 3.0, device=dev)
    P.pwl_batch_capture(bt, xt, yb, g=gt, dx=dxb, dv=dvb)
    # dL/dv sums per-workgroup partials with FP32 atomics in no fixed order:
    # two runs agree to the gradient tolerance, normwise per entry (the scale
    # of entry k is the sum over its table's points of |g phi_k(x)|)
    scale = np.concatenate([_abs_weights(t, x[o0:o1], g[o0:o1]) for t, o0, o1 in zip(tabs, offs[:-1], offs[1:])])
    for rep in range(4):
        dvb.fill_(float(rep + 1))              # the graph must clear dv itself
        yb.zero_()
        torch.cuda.synchronize()
        P.pwl_batch_replay(bt)
        torch.cuda.synchronize()
        assert torch.equal(yb, ye) and torch.equal(dxb, dxe), rep
        diff = np.abs(dvb.cpu().numpy().astype(np.float64) - dve.cpu().numpy())
        assert np.all(diff <= 2 * GRAD_TOL * scale + 1e-30), rep
    bt.free()


def _abs_weights(table, x, g):
    """Per entry k of a table's dL/dv: the sum over the points of |g| times
    the hat weight phi_k(x), from the oracle on the table's own knots."""
    import paper_1510_02975_amd as P
    X = P.pwl_table_download(table)["knots"].astype(np.float64)
    _, _, w = O.evaluate_backward(X, np.zeros(len(X)), x.astype(np.float64), np.abs(g.astype(np.float64)))
    return w


def test_batch_misaligned_and_degenerate_shapes():
    import paper_1510_02975_amd as P
    library()
    dev = device()
    t = P.pwl_build(O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 300, O.OPTIMAL, O.PROJ)
    u = P.pwl_build(O.BESSEL_J0, (1.0,), 0.0, 50.0, 40, O.UNIFORM, O.INTERP)
    base = torch.from_numpy(W.uniform_points(-6.0, 51.0, 20011, 9)).to(dev)
    for off in (0, 1, 2, 3):
        x = base[off:off + 20003]
        offs = [0, 7, 7, 12345, 20003]
        bt = P.pwl_batch_create([t, u, t, u], offs)
        y = torch.empty(20006, device=dev)[off % 3:off % 3 + 20003]
        P.pwl_batch_eval(bt, x, y)
        ref = torch.cat([P.pwl_eval(t, x[0:7]), P.pwl_eval(t, x[7:12345]), P.pwl_eval(u, x[12345:20003])])
        assert torch.equal(y, ref), off
        bt.free()
    # the batch holds its own copy of the tables: a freed table is not needed
    t2 = P.pwl_build(O.LORENTZIAN, (1.0, 1.0), -20.0, 20.0, 700, O.OPTIMAL, O.INTERP)
    ref = P.pwl_eval(t2, base)
    bt = P.pwl_batch_create([t2], [0, base.numel()])
    t2.free()
    assert torch.equal(P.pwl_batch_eval(bt, base), ref)
    bt.free()
    # a single table equals pwl_eval; zero points is valid
    bt = P.pwl_batch_create([t], [0, 20011])
    assert torch.equal(P.pwl_batch_eval(bt, base), P.pwl_eval(t, base))
    bt.free()
    bt = P.pwl_batch_create([t, u], [0, 0, 0])
    P.pwl_batch_eval(bt, base[:0], base[:0].clone())
    _, _, dv = P.pwl_batch_eval_backward(bt, base[:0], base[:0], want=())
    assert torch.all(dv == 0.0) and dv.numel() == 301 + 41
    bt.free()


def _expected_runs(offs, slice_pts):
    """Runs of the slice plan: one per (slice, table with points in it)."""
    total = int(offs[-1])
    runs = 0
    for s0 in range(0, total, slice_pts):
        s1 = min(total, s0 + slice_pts)
        runs += int(np.count_nonzero((offs[:-1] < s1) & (offs[1:] > s0) & (offs[1:] > offs[:-1])))
    return runs


@pytest.mark.parametrize("shapes", [((4, 1024, 3), (4, 1024, 32)), ((2, 512, 2), (1, 256, 4))],
                         ids=["tuned", "small"])
def test_batch_plan_slices(shapes):
    """The slice plan as the host builds it: slices of 2 (forward) and 4
    (backward) vector iterations of the launch shape, one run per table per
    slice it meets (empty tables none), no more workgroups than wg_per_cu
    per CU; and the outputs of both directions equal the per-table kernels'."""
    import paper_1510_02975_amd as P
    library()
    dev = device()
    num_cu = torch.cuda.get_device_properties(dev).multi_processor_count
    t1 = P.pwl_build(O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 300, O.OPTIMAL, O.PROJ)
    t2 = P.pwl_build(O.BESSEL_J0, (1.0,), 0.0, 50.0, 64, O.UNIFORM, O.INTERP)
    counts = [100000, 0, 1, 70001, 3, 0, 250000, 17, 40000]
    tabs = [t1 if k % 2 == 0 else t2 for k in range(len(counts))]
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    n = int(offs[-1])
    x = torch.from_numpy(W.uniform_points(-6.0, 51.0, n, 13)).to(dev)
    g = torch.from_numpy(W.upstream_grad(n, 14)).to(dev)
    (uf, bf, wf), (ub, bb, wb) = shapes
    with launch_shape(P, P.KERNEL_BATCH, shapes[0]), launch_shape(P, P.KERNEL_BATCH_BACKWARD, shapes[1]):
        bt = P.pwl_batch_create(tabs, offs)
        say("plan: grid fwd %d bwd %d, runs fwd %d bwd %d" % (bt.grid_fwd, bt.grid_bwd, bt.runs_fwd, bt.runs_bwd))
        assert bt.runs_fwd == _expected_runs(offs, 2 * 4 * bf * uf)
        assert bt.runs_bwd == _expected_runs(offs, 4 * 4 * bb * ub)
        assert 1 <= bt.grid_fwd <= num_cu * wf and 1 <= bt.grid_bwd <= num_cu * wb
        y = P.pwl_batch_eval(bt, x)
        yb, dxb, _ = P.pwl_batch_eval_backward(bt, x, g)
        for t, o0, o1 in zip(tabs, offs[:-1], offs[1:]):
            if o1 > o0:
                assert torch.equal(y[o0:o1], P.pwl_eval(t, x[o0:o1]))
                y1, dx1, _ = P.pwl_eval_backward(t, x[o0:o1], g[o0:o1], want=("y", "dx"))
                assert torch.equal(yb[o0:o1], y1) and torch.equal(dxb[o0:o1], dx1)
        bt.free()
    t1.free()
    t2.free()


@pytest.mark.parametrize("shape", [(4, 1024, 3), (1, 256, 1), (2, 512, 8)], ids=["u4", "u1-256", "u2-512"])
def test_batch_forward_slices_cross_tables(shape):
    """The forward's slices against table boundaries: runs of 1 to 300
    points (a wave's 256 points then cross several tables, and a vector
    holds points of up to four), tables of N = 16 .. 4096 (different
    unrolled compare depths in one slice), and a stretch of N = 4096
    tables with 97 points each, whose images cannot share LDS, so its
    slices are split at every table; x and y at every 4-byte phase.  Every
    table's points match pwl_eval bit for bit."""
    import paper_1510_02975_amd as P
    library()
    dev = device()
    rng = np.random.default_rng(11)
    kinds = [(O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0), (O.LORENTZIAN, (1.0, 1.0), -20.0, 20.0),
             (O.BESSEL_J0, (1.0,), 0.0, 50.0)]
    built = {}

    def table(k, N):
        if (k, N) not in built:
            f, p, a, b = kinds[k]
            built[k, N] = P.pwl_build(f, p, a, b, N, O.OPTIMAL if N % 2 else O.UNIFORM, O.PROJ)
        return built[k, N]
    tabs, counts = [], []
    for i in range(600):
        tabs.append(table(i % 3, int(rng.choice([16, 33, 200, 1000, 4096]))))
        counts.append(int(rng.integers(1, 301)))
    for i in range(40):
        tabs.append(table(i % 3, 4096))
        counts.append(97)
    for i in range(30):
        tabs.append(table(i % 3, int(rng.choice([64, 777]))))
        counts.append(int(rng.integers(0, 70000)))
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    n = int(offs[-1])
    base = torch.from_numpy(W.uniform_points(-25.0, 55.0, n + 8, 12)).to(dev)
    with launch_shape(P, P.KERNEL_BATCH, shape):
        bt = P.pwl_batch_create(tabs, offs)
        say("%d tables, %d points, shape %s: grid %d, %d runs" % (len(tabs), n, shape, bt.grid_fwd, bt.runs_fwd))
        for ph in (0, 1, 2, 3):
            x = base[ph:ph + n]
            y = torch.full((n + 8,), 7.0, device=dev)[(ph * 3) % 4:(ph * 3) % 4 + n]
            P.pwl_batch_eval(bt, x, y)
            ref = torch.cat([P.pwl_eval(t, x[o0:o1]) for t, o0, o1 in zip(tabs, offs[:-1], offs[1:])])
            bad = torch.nonzero(y != ref).flatten()
            assert bad.numel() == 0, (ph, int(np.searchsorted(offs, int(bad[0]), side="right")) - 1)
        bt.free()
    for t in built.values():
        t.free()


@pytest.mark.parametrize("shapes", [((2, 1024, 16), (1, 1024, 16)), ((4, 1024, 1), (2, 512, 1))],
                         ids=["16-per-CU", "1-per-CU"])
def test_batch_mixed_table_sizes(shapes):
    """Tables of very different LDS footprints (N = 4096, 64, 1000), each
    appearing several times, cut for 16 workgroups per CU (many rounds) and
    for one: a workgroup per non-empty chunk, plus one for every split of a
    chunk whose tables' images do not fit in LDS together (at most one per
    table), plus (backward) at most 8 idle ones that round the grid to the
    XCDs; y and dx match the per-table evaluator bit for bit and dL/dv
    matches the oracle."""
    import paper_1510_02975_amd as P
    library()
    dev = device()
    with launch_shape(P, P.KERNEL_BATCH, shapes[0]), launch_shape(P, P.KERNEL_BATCH_BACKWARD, shapes[1]):
        _mixed_sizes(P, dev, shapes)


def _mixed_sizes(P, dev, shapes):
    num_cu = torch.cuda.get_device_properties(dev).multi_processor_count
    big = P.pwl_build(O.LORENTZIAN, (1.0, 1.0), -20.0, 20.0, 4096, O.OPTIMAL, O.PROJ)
    small = P.pwl_build(O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 64, O.UNIFORM, O.INTERP)
    mid = P.pwl_build(O.BESSEL_J0, (1.0,), 0.0, 50.0, 1000, O.OPTIMAL, O.INTERP)
    tabs = [big, small, mid, big, small, big, mid]
    counts = [70001, 5, 33333, 0, 128000, 3, 257]
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    n = int(offs[-1])
    x = W.uniform_points(-25.0, 55.0, n, 4)
    g = W.upstream_grad(n, 6)
    xt, gt = torch.from_numpy(x).to(dev), torch.from_numpy(g).to(dev)
    bt = P.pwl_batch_create(tabs, offs)
    say("grid fwd %d bwd %d, runs fwd %d bwd %d" % (bt.grid_fwd, bt.grid_bwd, bt.runs_fwd, bt.runs_bwd))
    assert 1 <= bt.grid_fwd <= num_cu * shapes[0][2] + len(tabs)
    assert 1 <= bt.grid_bwd <= num_cu * shapes[1][2] + len(tabs) + 8
    y = P.pwl_batch_eval(bt, xt)
    yb, dxb, dvb = P.pwl_batch_eval_backward(bt, xt, gt)
    dvb = dvb.cpu().numpy()
    for i, (t, o0, o1) in enumerate(zip(tabs, offs[:-1], offs[1:])):
        d0, d1 = bt.dv_offsets[i], bt.dv_offsets[i + 1]
        if o1 == o0:
            assert np.all(dvb[d0:d1] == 0.0)
            continue
        assert torch.equal(y[o0:o1], P.pwl_eval(t, xt[o0:o1])), i
        y1, dx1, _ = P.pwl_eval_backward(t, xt[o0:o1], gt[o0:o1])
        assert torch.equal(yb[o0:o1], y1) and torch.equal(dxb[o0:o1], dx1), i
        d = P.pwl_table_download(t)
        X = d["knots"].astype(np.float64)
        xs, gs = x[o0:o1].astype(np.float64), g[o0:o1].astype(np.float64)
        _, _, dvr = O.evaluate_backward(X, d["values"].astype(np.float64), xs, gs)
        _, _, wk = O.evaluate_backward(X, np.zeros(len(X)), xs, np.abs(gs))
        assert np.all(np.abs(dvb[d0:d1] - dvr) <= GRAD_TOL * wk + 1e-30), i
    bt.free()
    for t in (big, small, mid):
        t.free()
