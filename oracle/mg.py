"""Multigrid-preconditioned conjugate gradients (MGCG), Algorithm 2.

The paper preconditions CG with a V-cycle (Algorithm 2): damped-Jacobi
pre-smoothing, restriction of the residual with P^T, a coarse-grid solve with
the Galerkin operator P^T K P, interpolation with P and damped-Jacobi
post-smoothing, recursively over the grid levels.  Readings taken where the
paper is silent:

* "grid level" counts all levels including the finest; coarsening is 2:1 per
  axis and P is trilinear interpolation;
* the pre-smoother uses the current iterate (the u0 in its first line is read
  as the current u, zero on entry to the preconditioner);
* fixed DOFs: the fine operator is A = Df K Df + (I - Df) and the fine
  interpolation is masked, Df P, so the first coarse operator is
  (Df P)^T K (Df P); a coarse DOF that no free DOF interpolates from gets an
  identity row;
* the coarsest level is solved exactly (dense Cholesky).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import fem


def prolongation(ncx: int, ncy: int, ncz: int) -> sp.csr_matrix:
    """Trilinear interpolation from the coarse grid (ncx x ncy x ncz elements)
    to the 2:1 refined grid, AoS on both sides (acts per component)."""
    nfx, nfy, nfz = 2 * ncx, 2 * ncy, 2 * ncz

    def axis(f):
        return [(f // 2, 1.0)] if f % 2 == 0 else [((f - 1) // 2, 0.5), ((f + 1) // 2, 0.5)]

    rows, cols, vals = [], [], []
    for fk in range(nfz + 1):
        for fj in range(nfy + 1):
            for fi in range(nfx + 1):
                fn = fem.node_id(nfx, nfy, fi, fj, fk)
                for ci, wi in axis(fi):
                    for cj, wj in axis(fj):
                        for ck, wk in axis(fk):
                            cn = fem.node_id(ncx, ncy, ci, cj, ck)
                            for c in range(3):
                                rows.append(3 * fn + c)
                                cols.append(3 * cn + c)
                                vals.append(wi * wj * wk)
    nf = 3 * (nfx + 1) * (nfy + 1) * (nfz + 1)
    nc = 3 * (ncx + 1) * (ncy + 1) * (ncz + 1)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf, nc))


def prolongation_kron(ncx: int, ncy: int, ncz: int) -> sp.csr_matrix:
    """The same trilinear interpolation as `prolongation`, formed as the
    Kronecker product of the three 1D interpolations (z slowest, then y, x,
    and the 3 components fastest, the AoS node order), for grids too large
    for the node loop.  Equal to `prolongation` entry for entry."""

    def axis1d(nc):
        rows, cols, vals = [], [], []
        for f in range(2 * nc + 1):
            if f % 2 == 0:
                rows.append(f); cols.append(f // 2); vals.append(1.0)
            else:
                rows += [f, f]; cols += [(f - 1) // 2, (f + 1) // 2]; vals += [0.5, 0.5]
        return sp.csr_matrix((vals, (rows, cols)), shape=(2 * nc + 1, nc + 1))

    P = sp.kron(axis1d(ncz), sp.kron(axis1d(ncy), sp.kron(axis1d(ncx), sp.identity(3))))
    return P.tocsr()


def prolongation2(ncx: int, ncy: int) -> sp.csr_matrix:
    """Bilinear interpolation from the coarse 2D grid (ncx x ncy elements) to
    the 2:1 refined grid, AoS with 2 components per node."""
    nfx, nfy = 2 * ncx, 2 * ncy

    def axis(f):
        return [(f // 2, 1.0)] if f % 2 == 0 else [((f - 1) // 2, 0.5), ((f + 1) // 2, 0.5)]

    rows, cols, vals = [], [], []
    for fj in range(nfy + 1):
        for fi in range(nfx + 1):
            fn = fi + (nfx + 1) * fj
            for ci, wi in axis(fi):
                for cj, wj in axis(fj):
                    cn = ci + (ncx + 1) * cj
                    for c in range(2):
                        rows.append(2 * fn + c)
                        cols.append(2 * cn + c)
                        vals.append(wi * wj)
    nf = 2 * (nfx + 1) * (nfy + 1)
    nc = 2 * (ncx + 1) * (ncy + 1)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf, nc))


def _fix_empty_rows(A: sp.csr_matrix) -> sp.csr_matrix:
    d = A.diagonal()
    dead = (d == 0.0).astype(np.float64)
    return (A + sp.diags(dead)).tocsr() if dead.any() else A


class Hierarchy:
    """Galerkin hierarchy A_0 .. A_{L-1} with per-level Jacobi diagonals."""

    def __init__(self, K: sp.spmatrix, fixed: np.ndarray, dims, levels: int):
        """dims: (nx, ny, nz) elements, or (nx, ny) for the 2D plane-stress grid."""
        two_d = len(dims) == 2
        nx, ny, nz = (dims[0], dims[1], 1) if two_d else dims
        if levels < 2:
            raise ValueError("need at least two levels")
        s = 2 ** (levels - 1)
        if nx % s or ny % s or (not two_d and nz % s):
            raise ValueError("grid not divisible by 2^(levels-1)")
        n = K.shape[0]
        df = fem.free_mask(n, fixed).astype(np.float64)
        self.A = [fem.operator_with_bc(K, fixed)]
        self.P = []
        for l in range(levels - 1):
            f = 2 ** (l + 1)
            P = prolongation2(nx // f, ny // f) if two_d else prolongation(nx // f, ny // f, nz // f)
            if l == 0:
                P = (sp.diags(df) @ P).tocsr()
            self.P.append(P)
            Ac = (P.T @ self.A[-1] @ P).tocsr()
            self.A.append(_fix_empty_rows(Ac))
        self.D = [A.diagonal().copy() for A in self.A]
        self.coarse_fac = sla.cho_factor(self.A[-1].toarray(), lower=True)
        self.levels = levels

    def vcycle(self, b: np.ndarray, omega: float = 0.6, nu1: int = 1, nu2: int = 1,
               level: int = 0) -> np.ndarray:
        """Algorithm 2 applied to b with zero initial guess, recursively."""
        if level == self.levels - 1:
            return sla.cho_solve(self.coarse_fac, b)
        A, D, P = self.A[level], self.D[level], self.P[level]
        x = np.zeros_like(b)
        for _ in range(nu1):                                  # line 1: pre-smooth
            x = x + omega * (b - A @ x) / D
        e = P.T @ (b - A @ x)                                 # line 2: restrict
        xc = self.vcycle(e, omega, nu1, nu2, level + 1)       # line 3: coarse solve
        x = x + P @ xc                                        # line 4: interpolate
        for _ in range(nu2):                                  # line 5: post-smooth
            x = x + omega * (b - A @ x) / D
        return x


def mgcg(K, f, fixed, dims, levels, u0=None, rtol=1e-8, maxit=1000, omega=0.6,
         nu1=1, nu2=1):
    """Preconditioned CG on A u = f (A with identity rows on fixed DOFs, f
    zeroed there) with one V-cycle as preconditioner; stops when
    ||f - A u|| <= rtol ||f||.  Returns (u, iterations, rel_residual)."""
    H = Hierarchy(K, fixed, dims, levels)
    A = H.A[0]
    free = fem.free_mask(K.shape[0], fixed)
    f = np.where(free, f, 0.0)
    u = np.zeros_like(f) if u0 is None else np.where(free, u0, 0.0)
    r = f - A @ u
    nf = np.linalg.norm(f)
    it = 0
    rel = np.linalg.norm(r) / nf
    if rel <= rtol:
        return u, 0, rel
    z = H.vcycle(r, omega, nu1, nu2)
    p = z.copy()
    rz = r @ z
    while it < maxit:
        q = A @ p
        alpha = rz / (p @ q)
        u = u + alpha * p
        r = r - alpha * q
        it += 1
        rel = np.linalg.norm(r) / nf
        if rel <= rtol:
            break
        z = H.vcycle(r, omega, nu1, nu2)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return u, it, rel
