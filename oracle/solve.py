"""Direct FP64 solution of the equilibrium equation K u = f (eq. 7).

Fixed DOFs are eliminated: K_ff u_f = f_f and u = 0 on fixed DOFs.  The
factorisation is a Cholesky factorisation, dense for tiny systems and banded
(LAPACK ``pbtrf`` through :func:`scipy.linalg.cholesky_banded`) otherwise,
with nodes renumbered so that the longest grid axis varies slowest, which
keeps the half-bandwidth at about three node planes.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import fem

DENSE_LIMIT = 3000


def band_permutation(nx: int, ny: int, nz: int) -> np.ndarray:
    """AoS DOF permutation that orders nodes with the longest axis slowest,
    then the middle axis, then the shortest (fastest)."""
    dims = [nx + 1, ny + 1, nz + 1]
    order = sorted(range(3), key=lambda a: -dims[a])  # slowest first
    I, J, K = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1),
                          indexing="ij")
    coords = [I.ravel(), J.ravel(), K.ravel()]
    nodes = fem.node_id(nx, ny, coords[0], coords[1], coords[2])
    keys = tuple(coords[a] for a in reversed(order))  # lexsort: last key is primary
    node_order = nodes[np.lexsort(keys)]
    return (3 * node_order[:, None] + np.arange(3)[None, :]).ravel()


class DirectSolver:
    """Cholesky factorisation of the free-DOF block of K, reusable for
    several right-hand sides."""

    def __init__(self, K: sp.spmatrix, fixed: np.ndarray, dims=None):
        n = K.shape[0]
        free = fem.free_mask(n, fixed)
        if dims is not None:
            perm = band_permutation(*dims)
            perm = perm[free[perm]]
        else:
            perm = np.nonzero(free)[0]
        self.n = n
        self.perm = perm
        Kff = K.tocsr()[perm][:, perm].tocoo()
        m = len(perm)
        if m <= DENSE_LIMIT:
            self.mode = "dense"
            self.fac = sla.cho_factor(Kff.toarray(), lower=True)
        else:
            self.mode = "banded"
            lower = Kff.row >= Kff.col
            r, c, v = Kff.row[lower], Kff.col[lower], Kff.data[lower]
            kd = int((r - c).max())
            ab = np.zeros((kd + 1, m))
            ab[r - c, c] = v  # LAPACK lower band storage: ab[i-j, j] = A[i, j]
            self.kd = kd
            self.fac = sla.cholesky_banded(ab, lower=True, check_finite=False)

    def solve(self, f: np.ndarray) -> np.ndarray:
        b = np.asarray(f, dtype=np.float64)[self.perm]
        if self.mode == "dense":
            x = sla.cho_solve(self.fac, b)
        else:
            x = sla.cho_solve_banded((self.fac, True), b, check_finite=False)
        u = np.zeros(self.n)
        u[self.perm] = x
        return u


def solve_direct(K: sp.spmatrix, f: np.ndarray, fixed: np.ndarray, dims=None) -> np.ndarray:
    """u with K_ff u_f = f_f and u = 0 on fixed DOFs (loads there ignored)."""
    return DirectSolver(K, fixed, dims).solve(f)


def residual_norm(K: sp.spmatrix, u: np.ndarray, f: np.ndarray, fixed: np.ndarray) -> float:
    """Relative force residual on the free DOFs, ||f - K u||_f / ||f||_f, the
    criterion form of eq. (29) used as the solver tolerance."""
    free = fem.free_mask(K.shape[0], fixed)
    r = (np.asarray(f) - K @ u)[free]
    return float(np.linalg.norm(r) / np.linalg.norm(np.asarray(f)[free]))
