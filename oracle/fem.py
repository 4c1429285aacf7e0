"""Discretisation: SIMP stiffness (eq. 1), hex8 element stiffness, assembly.

The paper discretises 3D domains with 1x1x1 hexahedral elements (Section
4.2.2) and fixes E0=1, Emin=1e-9, nu=0.3, p=3 (Section 4).  It does not print
the element stiffness matrix; here it is the standard trilinear hexahedron
for isotropic linear elasticity integrated exactly with 2x2x2 Gauss points.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def lame(E: float, nu: float):
    """Lame parameters of an isotropic solid."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def elasticity_matrix(E: float, nu: float) -> np.ndarray:
    """6x6 isotropic D for strains (xx, yy, zz, xy, yz, zx), engineering shear."""
    lam, mu = lame(E, nu)
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[0, 0] = D[1, 1] = D[2, 2] = lam + 2.0 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    return D


def local_corner(a: int):
    """Corner offsets of local node ``a`` (bit order a = dx + 2 dy + 4 dz)."""
    return (a & 1, (a >> 1) & 1, (a >> 2) & 1)


def strain_displacement(x: float, y: float, z: float) -> np.ndarray:
    """6x24 B matrix of the unit-cube trilinear element at (x, y, z)."""
    B = np.zeros((6, 24))
    for a in range(8):
        i, j, k = local_corner(a)
        fx, fy, fz = (x if i else 1 - x), (y if j else 1 - y), (z if k else 1 - z)
        sx, sy, sz = (1 if i else -1), (1 if j else -1), (1 if k else -1)
        dNx, dNy, dNz = sx * fy * fz, fx * sy * fz, fx * fy * sz
        B[0, 3 * a + 0] = dNx
        B[1, 3 * a + 1] = dNy
        B[2, 3 * a + 2] = dNz
        B[3, 3 * a + 0] = dNy
        B[3, 3 * a + 1] = dNx
        B[4, 3 * a + 1] = dNz
        B[4, 3 * a + 2] = dNy
        B[5, 3 * a + 0] = dNz
        B[5, 3 * a + 2] = dNx
    return B


def hex8_ke(E: float = 1.0, nu: float = 0.3) -> np.ndarray:
    """24x24 element stiffness of the unit cube: integral of B^T D B with
    2x2x2 Gauss-Legendre points (exact for the trilinear cube)."""
    D = elasticity_matrix(E, nu)
    g = 0.5 + 0.5 * np.array([-1.0, 1.0]) / np.sqrt(3.0)
    KE = np.zeros((24, 24))
    for x in g:
        for y in g:
            for z in g:
                B = strain_displacement(x, y, z)
                KE += B.T @ D @ B * 0.125  # each Gauss weight is 1/8 on [0,1]^3
    return KE


def simp(rho_phys: np.ndarray, E0: float = 1.0, Emin: float = 1e-9, p: float = 3.0):
    """Modified SIMP interpolation, eq. (1): E = Emin + (E0 - Emin) rho~^p.
    Complex input is kept complex (complex-step derivative checks)."""
    rho = np.asarray(rho_phys)
    if not np.iscomplexobj(rho):
        rho = rho.astype(np.float64)
    return Emin + (E0 - Emin) * rho ** p


def node_id(nx, ny, i, j, k):
    return i + (nx + 1) * (j + (ny + 1) * k)


def element_dofs(nx: int, ny: int, nz: int) -> np.ndarray:
    """(n_elem, 24) global AoS DOF ids of every element's local DOFs."""
    ne = nx * ny * nz
    edof = np.zeros((ne, 24), dtype=np.int64)
    e = 0
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                for a in range(8):
                    di, dj, dk = local_corner(a)
                    n = node_id(nx, ny, i + di, j + dj, k + dk)
                    edof[e, 3 * a:3 * a + 3] = 3 * n + np.arange(3)
                e += 1
    return edof


def element_dofs_grid(nx: int, ny: int, nz: int) -> np.ndarray:
    """element_dofs built with array operations (same numbering), for grids
    too large for the element loop."""
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()  # element order e = i + nx (j + ny k)
    cols = []
    for a in range(8):
        di, dj, dk = local_corner(a)
        n = node_id(nx, ny, i + di, j + dj, k + dk)
        cols += [3 * n + c for c in range(3)]
    return np.stack(cols, axis=1).astype(np.int64)


def apply_ebe(nx: int, ny: int, nz: int, Ee: np.ndarray, KE: np.ndarray, v: np.ndarray,
              edof: np.ndarray = None) -> np.ndarray:
    """K v = sum_e E_e L_e^T KE L_e v element by element, without assembling
    K (eq. 7's product for grids whose assembled K would not fit); AoS."""
    if edof is None:
        edof = element_dofs_grid(nx, ny, nz)
    ye = (np.asarray(v)[edof] @ KE.T) * np.asarray(Ee, dtype=np.float64)[:, None]
    return np.bincount(edof.ravel(), weights=ye.ravel(), minlength=3 * (nx + 1) * (ny + 1) * (nz + 1))


def apply_ebe_at_nodes(nx: int, ny: int, nz: int, Ee: np.ndarray, KE: np.ndarray,
                       dof_value, nodes) -> np.ndarray:
    """(K v) at the listed nodes only, (len(nodes), 3): for each node, the sum
    over the up to eight elements that contain it of E_e times the node's three
    rows of KE applied to the element's 24 values (eq. 7's product, row by
    row).  ``dof_value(ids)`` returns v at AoS DOF ids, so v may live in any
    layout; meant for sampled checks on grids too large for apply_ebe."""
    out = np.zeros((len(nodes), 3))
    for t, n in enumerate(nodes):
        n = int(n)
        i, j, k = n % (nx + 1), (n // (nx + 1)) % (ny + 1), n // ((nx + 1) * (ny + 1))
        for a in range(8):  # the node is local corner a of element (i, j, k) - corner(a)
            di, dj, dk = local_corner(a)
            ei, ej, ek = i - di, j - dj, k - dk
            if not (0 <= ei < nx and 0 <= ej < ny and 0 <= ek < nz):
                continue
            ids = []
            for b in range(8):
                bi, bj, bk = local_corner(b)
                nb = node_id(nx, ny, ei + bi, ej + bj, ek + bk)
                ids += [3 * nb, 3 * nb + 1, 3 * nb + 2]
            ve = np.asarray(dof_value(np.array(ids, dtype=np.int64)), dtype=np.float64)
            out[t] += float(Ee[ei + nx * (ej + ny * ek)]) * (KE[3 * a:3 * a + 3, :] @ ve)
    return out


def assemble(nx: int, ny: int, nz: int, Ee: np.ndarray, KE: np.ndarray) -> sp.csr_matrix:
    """Global stiffness K = sum_e E_e L_e^T KE L_e (no boundary conditions)."""
    edof = element_dofs(nx, ny, nz)
    ne = edof.shape[0]
    ndof = 3 * (nx + 1) * (ny + 1) * (nz + 1)
    rows = np.repeat(edof, 24, axis=1).ravel()
    cols = np.tile(edof, (1, 24)).ravel()
    Ee = np.asarray(Ee)
    if not np.iscomplexobj(Ee):
        Ee = Ee.astype(np.float64)
    vals = (Ee.reshape(ne, 1, 1) * KE[None]).ravel()
    K = sp.coo_matrix((vals, (rows, cols)), shape=(ndof, ndof)).tocsr()
    K.sum_duplicates()
    return K


def dof_vector_aos(prob, case: int = 0) -> np.ndarray:
    """Load vector of one load case in AoS layout (loads on fixed DOFs kept;
    the solver drops them)."""
    f = np.zeros(3 * prob.n_node)
    for (i, j, k, c, v) in prob.loads[case]:
        f[3 * node_id(prob.nx, prob.ny, i, j, k) + c] += v
    return f


def fixed_dofs_aos(prob) -> np.ndarray:
    s = {3 * node_id(prob.nx, prob.ny, i, j, k) + c for (i, j, k, c) in prob.fixed}
    return np.array(sorted(s), dtype=np.int64)


def free_mask(ndof: int, fixed: np.ndarray) -> np.ndarray:
    m = np.ones(ndof, dtype=bool)
    m[fixed] = False
    return m


def operator_with_bc(K: sp.csr_matrix, fixed: np.ndarray) -> sp.csr_matrix:
    """The full-size operator the solvers work with: K on the free block,
    identity on fixed rows and columns (A = Df K Df + (I - Df))."""
    n = K.shape[0]
    d = free_mask(n, fixed).astype(np.float64)
    Df = sp.diags(d)
    return (Df @ K @ Df + sp.diags(1.0 - d)).tocsr()


def aos_to_soa(v: np.ndarray) -> np.ndarray:
    """(3 n_node,) AoS -> (3, n_node) SoA."""
    return np.asarray(v).reshape(-1, 3).T.copy()


def soa_to_aos(v: np.ndarray) -> np.ndarray:
    return np.asarray(v).reshape(3, -1).T.ravel().copy()
