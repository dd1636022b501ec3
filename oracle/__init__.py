"""FP64 CPU oracle (test infrastructure only; see pwl_oracle)."""
from .pwl_oracle import *  # noqa: F401,F403
from .pwl_oracle import (GAUSSIAN, LORENTZIAN, BESSEL_J0, POLY, EXP, UNIFORM, OPTIMAL,  # noqa: F401
                         INTERP, PROJ, FLAG_DEGENERATE, FLAG_KNOTS_COLLAPSED, KnotCollapse)
