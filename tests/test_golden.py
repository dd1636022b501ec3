"""The stored oracle tables under tests/golden/ (written by make_golden.py)
must still be reproduced exactly, and they must satisfy the paper's
structural facts on their own."""

import os

import numpy as np
import pytest

import oracle as O
from tests.golden_util import read_table

NAMES = ["gauss_uniform_n64.txt", "gauss_optimal_n32.txt", "j0_optimal_n16.txt"]


@pytest.mark.parametrize("name", NAMES)
def test_oracle_reproduces_stored_tables(golden_dir, name):
    meta, arr = read_table(os.path.join(golden_dir, name))
    func, N, part = int(meta["func"]), int(meta["N"]), int(meta["partition"])
    p = tuple(float(t) for t in meta["params"].split())
    a, b = float(meta["a"]), float(meta["b"])
    ti = O.build_table(func, p, a, b, N, part, O.INTERP)
    tp = O.build_table(func, p, a, b, N, part, O.PROJ)
    assert np.array_equal(ti["X"], arr[:, 1])
    assert np.max(np.abs(ti["v"] - arr[:, 2])) <= 1e-15
    assert np.max(np.abs(tp["v"] - arr[:, 3])) <= 1e-14


def test_stored_uniform_table_structure(golden_dir):
    meta, arr = read_table(os.path.join(golden_dir, "gauss_uniform_n64.txt"))
    X = arr[:, 1]
    assert np.array_equal(X, -4.0 + np.arange(65) / 8.0)
    # even function on a symmetric uniform partition: symmetric values
    assert np.array_equal(arr[:, 2], arr[::-1, 2])
    assert np.max(np.abs(arr[:, 3] - arr[::-1, 3])) <= 1e-15
