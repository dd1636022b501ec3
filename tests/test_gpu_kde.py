"""The sample application (Sec. VI-A), per-pixel sums of Gaussian kernels,
on the GPU against the FP64 oracle: with expf and __expf against the exact
Gaussian; through a table of exp(-u^2/2) on [0, 8] (the paper's interval)
against the oracle evaluating the same table, and against the exact
Gaussian within three times the table's L-infinity error (a product of three
kernel values, each at most 1)."""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests.gpu_util import device, library, say

pytestmark = pytest.mark.gpu

SIGMA = (6.0, 6.0, 6.0)


def _run(P, dev, H, W_, T, r, table_N):
    f_h, h_h = W.kde_frames(H, W_, T, seed=4)
    f, h = torch.from_numpy(f_h).to(dev), torch.from_numpy(h_h).to(dev)
    exact = O.kde_likelihood(f_h, h_h, r, SIGMA)
    t = P.pwl_build(O.GAUSSIAN, (1.0, 1.0), 0.0, 8.0, table_N, O.OPTIMAL, O.PROJ)
    d = P.pwl_table_download(t)
    X, v = d["knots"].astype(np.float64), d["values"].astype(np.float64)
    via_table = O.kde_likelihood(f_h, h_h, r, SIGMA, g=lambda u: O.evaluate(X, v, np.abs(u)))
    linf = O.linf_error(O.GAUSSIAN, (1.0, 1.0), X, v)
    out = {}
    for mode in (P.KDE_TABLE, P.KDE_EXPF, P.KDE_FAST_EXPF):
        out[mode] = P.pwl_kde(t, mode, f, h, r, SIGMA).cpu().numpy().astype(np.float64)
    e_exp = np.max(np.abs(out[P.KDE_EXPF] - exact))
    e_fast = np.max(np.abs(out[P.KDE_FAST_EXPF] - exact))
    e_tab = np.max(np.abs(out[P.KDE_TABLE] - via_table))
    e_tab_exact = np.max(np.abs(out[P.KDE_TABLE] - exact))
    say("  %dx%d T=%d r=%d: expf %.2e, __expf %.2e, table vs oracle table %.2e, table vs exact %.2e "
        "(table L-inf %.2e)" % (H, W_, T, r, e_exp, e_fast, e_tab, e_tab_exact, linf))
    assert e_exp <= 1e-6
    assert e_fast <= 1e-5
    assert e_tab <= 1e-6
    assert e_tab_exact <= 3.0 * linf + 1e-6
    t.free()


def test_kde_small_frame():
    import paper_1510_02975_amd as P
    library()
    _run(P, device(), 37, 53, 3, 2, 256)


def test_kde_cif_frame():
    import paper_1510_02975_amd as P
    library()
    c = W.KDE_CIF
    _run(P, device(), c["H"], c["W"], c["T"], c["radius"], 1024)


def test_kde_expf_modes_need_no_table():
    import paper_1510_02975_amd as P
    library()
    dev = device()
    f_h, h_h = W.kde_frames(9, 11, 2, seed=5)
    f, h = torch.from_numpy(f_h).to(dev), torch.from_numpy(h_h).to(dev)
    y = P.pwl_kde(None, P.KDE_EXPF, f, h, 1, SIGMA).cpu().numpy()
    assert np.max(np.abs(y - O.kde_likelihood(f_h, h_h, 1, SIGMA))) <= 1e-6
    with pytest.raises(P.PWLError):
        P.pwl_kde(None, P.KDE_TABLE, f, h, 1, SIGMA)
