"""Optimality-criteria design update (the paper's Section 2.1 cites the
textbook OC method for eq. (3)); support step of the optimisation loop.

Reading (the paper gives no parameters): move limit 0.2, damping exponent
0.5, bisection on the Lagrange multiplier in [0, 1e9] until
(l2 - l1) / (l1 + l2) <= 1e-3 or 200 halvings, and the volume constraint of
eq. (3) evaluated on the filtered density.
"""

from __future__ import annotations

import numpy as np

from . import filt


def oc_update(x, dc, dv, H, Hs, volfrac, move=0.2, eta=0.5, gap=1e-3, max_halvings=200):
    """Return (x_new, rho~_new, lambda)."""
    x = np.asarray(x, dtype=np.float64).ravel()
    n = x.size
    l1, l2 = 0.0, 1e9
    lo = np.maximum(0.0, x - move)
    hi = np.minimum(1.0, x + move)
    B = np.maximum(0.0, -np.asarray(dc).ravel()) / np.asarray(dv).ravel()
    xnew, xphys, lmid = x, x, 0.0
    for _ in range(max_halvings):
        if (l2 - l1) / (l1 + l2) <= gap:
            break
        lmid = 0.5 * (l1 + l2)
        xnew = np.clip(x * (B / lmid) ** eta, lo, hi)
        xphys = filt.forward(H, Hs, xnew)
        if xphys.sum() > volfrac * n:
            l1 = lmid
        else:
            l2 = lmid
    return xnew, xphys, lmid
