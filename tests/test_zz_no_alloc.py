"""pwl_eval_backward_noalloc (the fused backward with the dL/dv partial sums
in the library's fixed device scratch) against pwl_eval_backward: the same
kernels and launch shape, so every output must be bit-identical.  Two calls
in a row, the second on a smaller input and another table, check that the
shared scratch carries nothing over from the first."""

import numpy as np
import pytest

from tests.gpu_util import device, library, say

pytestmark = pytest.mark.gpu


def _inputs(n, seed, sigma):
    import torch
    rng = np.random.default_rng(seed)
    x = (sigma * rng.standard_normal(n)).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    dev = device()
    return torch.from_numpy(x).to(dev), torch.from_numpy(g).to(dev)


def _both(P, t, x, g):
    import torch
    ref = P.pwl_eval_backward(t, x, g)
    out = (torch.full_like(x, float("nan")), torch.full_like(x, float("nan")),
           torch.full((t.N + 1,), float("nan"), dtype=torch.float32, device=x.device))
    P.pwl_eval_backward_noalloc(t, x, g, *out)
    torch.cuda.synchronize()
    return ref, out


def test_noalloc_backward_matches_backward_twice():
    import torch
    import oracle as O
    import paper_1510_02975_amd as P
    library()
    # second call: smaller input, another table (N = 24: its dL/dv in 16 LDS copies)
    cases = [(1024, (1 << 22) + 3, 1.5), (24, 4099, 1.0)]
    for N, n, sigma in cases:
        say("noalloc backward: Gaussian optimal N=%d projection, n=%d" % (N, n))
        t = P.pwl_build(O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, N, O.OPTIMAL, O.PROJ)
        x, g = _inputs(n, N, sigma)
        (y0, dx0, dv0), (y1, dx1, dv1) = _both(P, t, x, g)
        assert torch.equal(y0, y1)
        assert torch.equal(dx0, dx1)
        assert torch.equal(dv0, dv1)
        # and dL/dv against the oracle on the GPU's own table (normwise per entry)
        d = P.pwl_table_download(t)
        X, v = d["knots"].astype(np.float64), d["values"].astype(np.float64)
        xh, gh = x.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64)
        _, _, dvr = O.evaluate_backward(X, v, xh, gh)
        i = O.locate(X, xh)
        xc = np.clip(xh, X[0], X[-1])
        w1 = (xc - X[i]) / (X[i + 1] - X[i])
        scale = np.bincount(i, np.abs((1 - w1) * gh), N + 1) + np.bincount(i + 1, np.abs(w1 * gh), N + 1)
        assert np.all(np.abs(dv1.cpu().numpy() - dvr) <= 1e-5 * scale + 1e-30)
        t.free()


def test_noalloc_backward_without_dv_and_empty():
    import torch
    import oracle as O
    import paper_1510_02975_amd as P
    library()
    t = P.pwl_build(O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 512, O.OPTIMAL, O.PROJ)
    x, g = _inputs(10007, 3, 1.0)
    y0, dx0, _ = P.pwl_eval_backward(t, x, g, want=("y", "dx"))
    y1, dx1 = torch.empty_like(x), torch.empty_like(x)
    P.pwl_eval_backward_noalloc(t, x, g, y1, dx1, None)
    dv = torch.full((513,), 7.0, dtype=torch.float32, device=x.device)
    P.pwl_eval_backward_noalloc(t, x[:0], g[:0], None, None, dv)   # no points: dL/dv = 0
    torch.cuda.synchronize()
    assert torch.equal(y0, y1) and torch.equal(dx0, dx1)
    assert torch.count_nonzero(dv).item() == 0
    t.free()


def test_noalloc_backward_rejects_oversized_scratch():
    """A backward launch whose partial sums exceed the fixed scratch is
    refused on the host before anything is enqueued."""
    import torch
    import oracle as O
    import paper_1510_02975_amd as P
    from tests.gpu_util import launch_shape
    library()
    t = P.pwl_build(O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 4096, O.OPTIMAL, O.PROJ)
    n = 240 * (1 << 20)   # enough points for 4 workgroups per CU at N = 4096
    dev = device()
    x = torch.zeros(n, dtype=torch.float32, device=dev)
    g = torch.zeros(n, dtype=torch.float32, device=dev)
    dv = torch.empty(4097, dtype=torch.float32, device=dev)
    with launch_shape(P, P.KERNEL_BACKWARD, (2, 1024, 4)):
        with pytest.raises(P.PWLError) as ei:
            P.pwl_eval_backward_noalloc(t, x, g, None, None, dv)
    assert ei.value.status == -5   # PWL_ECAPACITY
    torch.cuda.synchronize()
    del x, g
    t.free()
