"""Plane-stress discretisation of the paper's 2D examples (Sections 4.1, 4.2.1
and 4.3): 1x1 bilinear quadrilateral (Q4) elements of unit thickness, E0=1,
Emin=1e-9, nu=0.3, p=3 (Section 4).  The paper prints no element matrix;
here it is the standard Q4 for plane stress integrated exactly with 2x2 Gauss
points.  Test infrastructure only (see the package docstring).

Layout: nodes x-fastest, node = i + (nx+1) j; local corner a = dx + 2 dy;
AoS DOF 2 node + c (c = 0: x, 1: y).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def plane_stress_D(E: float, nu: float) -> np.ndarray:
    """3x3 constitutive matrix of plane stress for strains (xx, yy, xy),
    engineering shear."""
    c = E / (1.0 - nu * nu)
    return c * np.array([[1.0, nu, 0.0], [nu, 1.0, 0.0], [0.0, 0.0, 0.5 * (1.0 - nu)]])


def local_corner2(a: int):
    return (a & 1, (a >> 1) & 1)


def strain_displacement2(x: float, y: float) -> np.ndarray:
    """3x8 B matrix of the unit-square bilinear element at (x, y)."""
    B = np.zeros((3, 8))
    for a in range(4):
        i, j = local_corner2(a)
        fx, fy = (x if i else 1 - x), (y if j else 1 - y)
        sx, sy = (1 if i else -1), (1 if j else -1)
        dNx, dNy = sx * fy, fx * sy
        B[0, 2 * a] = dNx
        B[1, 2 * a + 1] = dNy
        B[2, 2 * a] = dNy
        B[2, 2 * a + 1] = dNx
    return B


def q4_ke(E: float = 1.0, nu: float = 0.3) -> np.ndarray:
    """8x8 element stiffness: integral of B^T D B over the unit square with
    2x2 Gauss-Legendre points (exact for the bilinear square)."""
    D = plane_stress_D(E, nu)
    g = 0.5 + 0.5 * np.array([-1.0, 1.0]) / np.sqrt(3.0)
    KE = np.zeros((8, 8))
    for x in g:
        for y in g:
            B = strain_displacement2(x, y)
            KE += B.T @ D @ B * 0.25
    return KE


def node_id2(nx: int, i: int, j: int) -> int:
    return i + (nx + 1) * j


def element_dofs2(nx: int, ny: int) -> np.ndarray:
    """(n_elem, 8) AoS DOF ids of every element's local DOFs."""
    edof = np.zeros((nx * ny, 8), dtype=np.int64)
    e = 0
    for j in range(ny):
        for i in range(nx):
            for a in range(4):
                di, dj = local_corner2(a)
                n = node_id2(nx, i + di, j + dj)
                edof[e, 2 * a:2 * a + 2] = 2 * n + np.arange(2)
            e += 1
    return edof


def assemble2(nx: int, ny: int, Ee: np.ndarray, KE: np.ndarray) -> sp.csr_matrix:
    """Global stiffness K = sum_e E_e L_e^T KE L_e (no boundary conditions)."""
    edof = element_dofs2(nx, ny)
    ne = edof.shape[0]
    ndof = 2 * (nx + 1) * (ny + 1)
    rows = np.repeat(edof, 8, axis=1).ravel()
    cols = np.tile(edof, (1, 8)).ravel()
    Ee = np.asarray(Ee)
    if not np.iscomplexobj(Ee):
        Ee = Ee.astype(np.float64)
    vals = (Ee.reshape(ne, 1, 1) * KE[None]).ravel()
    K = sp.coo_matrix((vals, (rows, cols)), shape=(ndof, ndof)).tocsr()
    K.sum_duplicates()
    return K


def spring_matrix2(prob) -> sp.csr_matrix:
    """Diagonal matrix of the problem's linear springs to ground: k on the
    DOF (i, j, c) of each spring (Section 4.3's k_in, k_out)."""
    n = 2 * prob.n_node
    d = np.zeros(n)
    for (i, j, c, k) in getattr(prob, "springs", []):
        d[2 * node_id2(prob.nx, i, j) + c] += k
    return sp.diags(d).tocsr()


def dof_vector_aos2(prob, case: int = 0) -> np.ndarray:
    f = np.zeros(2 * prob.n_node)
    for (i, j, c, v) in prob.loads[case]:
        f[2 * node_id2(prob.nx, i, j) + c] += v
    return f


def fixed_dofs_aos2(prob) -> np.ndarray:
    s = {2 * node_id2(prob.nx, i, j) + c for (i, j, c) in prob.fixed}
    return np.array(sorted(s), dtype=np.int64)


def aos_to_soa2(v: np.ndarray) -> np.ndarray:
    """(2 n_node,) AoS -> (2, n_node) SoA."""
    return np.asarray(v).reshape(-1, 2).T.copy()


def soa_to_aos2(v: np.ndarray) -> np.ndarray:
    return np.asarray(v).reshape(2, -1).T.ravel().copy()


def analyse2(prob, rho_phys, KE=None, E0=1.0, Emin=1e-9, p=3.0):
    """Plain definition of the 2D analysis for every load case: direct solve
    on the free DOFs of K + springs, C_l = f_l^T u_l (eq. 3), summed
    dC/drho~ (eq. 6; the springs do not depend on rho~).
    Returns (u_list AoS, C_list, dc_phys)."""
    from . import fem, sens, solve

    if KE is None:
        KE = q4_ke(1.0, 0.3)
    rho = np.asarray(rho_phys).ravel()
    Ee = fem.simp(rho, E0, Emin, p)
    K = (assemble2(prob.nx, prob.ny, Ee, KE) + spring_matrix2(prob)).tocsr()
    fixed = fixed_dofs_aos2(prob)
    ds = solve.DirectSolver(K, fixed)
    edof = element_dofs2(prob.nx, prob.ny)
    free = fem.free_mask(K.shape[0], fixed)
    us, Cs = [], []
    dc = np.zeros(prob.n_elem)
    for l in range(prob.n_case):
        f = dof_vector_aos2(prob, l) * free
        u = ds.solve(f)
        us.append(u)
        Cs.append(sens.compliance(f, u))
        dc += sens.dc_drho_phys(rho, sens.element_energy(u, edof, KE), E0, Emin, p)
    return us, Cs, dc


def mutual_energy(u: np.ndarray, w: np.ndarray, edof: np.ndarray, KE: np.ndarray) -> np.ndarray:
    """Per-element u_e^T KE w_e."""
    return np.einsum("ei,ij,ej->e", u[edof], KE, w[edof])


def mechanism2(prob, rho_phys, KE=None, E0=1.0, Emin=1e-9, p=3.0):
    """The non-self-adjoint analysis of Section 4.3: load case 0 (input force)
    and case 1 (unit dummy load at the output DOF) solved with the springs;
    the output displacement u_out = f_1^T u_0 and its sensitivity by the
    adjoint method: d u_out / d rho~_e = -dE_e/drho~_e u1_e^T KE u0_e (K
    symmetric, so case 1's solution is the adjoint).  Evaluated with the
    approximate displacements of the reduced model in place of u0, u1 this
    is the paper's approximate sensitivity (eq. 34's form).
    Returns (u0, u1 AoS, u_out, dout_phys)."""
    from . import fem

    if KE is None:
        KE = q4_ke(1.0, 0.3)
    us, _, _ = analyse2(prob, rho_phys, KE, E0, Emin, p)
    u0, u1 = us[0], us[1]
    free = fem.free_mask(2 * prob.n_node, fixed_dofs_aos2(prob))
    f1 = dof_vector_aos2(prob, 1) * free
    rho = np.asarray(rho_phys).ravel()
    dE = p * (E0 - Emin) * rho ** (p - 1)
    mut = mutual_energy(u0, u1, element_dofs2(prob.nx, prob.ny), KE)
    return u0, u1, float(f1 @ u0), -dE * mut
