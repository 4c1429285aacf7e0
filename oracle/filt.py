"""Density filter (eqs. 2, 31, 32) and its chain rule (eq. 33).

rho~_i = sum_j w_ij rho_j / sum_j w_ij with the cone weight
w_ij = max(0, r - ||x_i - x_j||) over element centres (eq. 32).  The
neighbourhood is truncated at the domain boundary and each row is normalised
by its own in-domain weight sum Hs_i.  The adjoint (eq. 33) is
dC/drho_e = sum_i (w_ie / Hs_i) dC/drho~_i.

The matrix is built by an explicit loop over elements and offsets so that it
can be checked by eye; it is slow and meant for small grids.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


def filter_matrix(nx: int, ny: int, nz: int, r: float):
    """Return (H, Hs): sparse weights and row sums."""
    R = int(math.ceil(r)) - 1  # offsets with a positive weight satisfy |d| < r
    rows, cols, vals = [], [], []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                e = i + nx * (j + ny * k)
                for dk in range(-R, R + 1):
                    for dj in range(-R, R + 1):
                        for di in range(-R, R + 1):
                            ii, jj, kk = i + di, j + dj, k + dk
                            if not (0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz):
                                continue
                            w = r - math.sqrt(di * di + dj * dj + dk * dk)
                            if w > 0.0:
                                rows.append(e)
                                cols.append(ii + nx * (jj + ny * kk))
                                vals.append(w)
    n = nx * ny * nz
    H = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    Hs = np.asarray(H.sum(axis=1)).ravel()
    return H, Hs


def forward(H, Hs, rho):
    """eq. (31)."""
    return (H @ np.asarray(rho).ravel()) / Hs


def adjoint(H, Hs, g):
    """eq. (33): H^T (g / Hs)."""
    return H.T @ (np.asarray(g).ravel() / Hs)


def brute_force_forward(nx, ny, nz, r, rho):
    """O(N^2) distance loop over all element pairs (tiny grids only)."""
    rho = np.asarray(rho).ravel()
    cen = np.array([(i, j, k) for k in range(nz) for j in range(ny) for i in range(nx)],
                   dtype=np.float64)
    out = np.zeros(len(rho))
    for a in range(len(rho)):
        d = np.sqrt(((cen - cen[a]) ** 2).sum(axis=1))
        w = np.maximum(0.0, r - d)
        out[a] = (w * rho).sum() / w.sum()
    return out
