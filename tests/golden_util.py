"""Readers for the text fixtures under tests/golden/."""

import os

import numpy as np


def paper_constants(golden_dir):
    out = {}
    with open(os.path.join(golden_dir, "paper_constants.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, value = line.split()[:2]
            out[name] = float(value)
    return out


def read_table(path):
    """A fixture table: header lines '# key value', then rows 'k X v'."""
    meta = {}
    rows = []
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line:
                continue
            if line.startswith("#"):
                parts = line[1:].split(None, 1)
                if len(parts) == 2:
                    meta[parts[0]] = parts[1]
                continue
            rows.append([float(t) for t in line.split()])
    arr = np.array(rows)
    return meta, arr
