"""Writes the stored oracle tables under tests/golden/.

Calls only the oracle.  Run from the repository root:
    python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402

FIXTURES = [
    ("gauss_uniform_n64.txt", O.GAUSSIAN, (1.0, 1.0), -4.0, 4.0, 64, O.UNIFORM),
    ("gauss_optimal_n32.txt", O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 32, O.OPTIMAL),
    ("j0_optimal_n16.txt", O.BESSEL_J0, (1.0,), 0.0, 50.0, 16, O.OPTIMAL),
]


def main():
    for name, func, p, a, b, N, part in FIXTURES:
        ti = O.build_table(func, p, a, b, N, part, O.INTERP)
        tp = O.build_table(func, p, a, b, N, part, O.PROJ)
        with open(os.path.join(HERE, name), "w") as fh:
            fh.write("# written by tests/golden/make_golden.py from the FP64 oracle\n")
            fh.write("# func %d\n# params %s\n# a %r\n# b %r\n# N %d\n# partition %d\n"
                     % (func, " ".join(repr(x) for x in p), a, b, N, part))
            fh.write("# columns: k  X_k(FP32 knot)  interp v_k  projection c_k\n")
            for k in range(N + 1):
                fh.write("%d %r %r %r\n" % (k, float(ti["X"][k]), float(ti["v"][k]), float(tp["v"][k])))


if __name__ == "__main__":
    main()
