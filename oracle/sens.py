"""Compliance and its sensitivity (eqs. 3-6 and 34).

C = f^T u (equal to u^T K u at equilibrium, eq. 3).  With a
design-independent load, the adjoint derivation of eqs. (4)-(5) leaves
dC/drho~_e = -u^T (dK/drho~_e) u (eq. 6), and under SIMP (eq. 1)
dK/drho~_e = p rho~_e^(p-1) (E0 - Emin) L_e^T KE L_e.  When the displacement
is the reduced-model one, u = R~ y, this is exactly eq. (34).
"""

from __future__ import annotations

import numpy as np

from . import fem


def element_energy(u: np.ndarray, edof: np.ndarray, KE: np.ndarray) -> np.ndarray:
    """e_e = u_e^T KE u_e for every element (unit Young's modulus)."""
    ue = np.asarray(u)[edof]  # (ne, 24)
    return np.einsum("ei,ij,ej->e", ue, KE, ue)


def compliance(f: np.ndarray, u: np.ndarray) -> float:
    return float(np.dot(f, u))


def dc_drho_phys(rho_phys, energy, E0=1.0, Emin=1e-9, p=3.0):
    """eq. (6) with eq. (1): -p rho~^(p-1) (E0 - Emin) e_e."""
    return -p * np.asarray(rho_phys) ** (p - 1.0) * (E0 - Emin) * energy


def analyse(prob, rho_phys, KE=None, E0=1.0, Emin=1e-9, p=3.0, case=None):
    """Plain definition of the analysis step for every load case: direct
    solve, compliance C_l = f_l^T u_l, summed sensitivity dC/drho~.

    Returns (u_list AoS, C_list, dc_phys)."""
    from . import solve

    if KE is None:
        KE = fem.hex8_ke(1.0, 0.3)
    Ee = fem.simp(rho_phys.ravel(), E0, Emin, p)
    K = fem.assemble(prob.nx, prob.ny, prob.nz, Ee, KE)
    fixed = fem.fixed_dofs_aos(prob)
    ds = solve.DirectSolver(K, fixed, (prob.nx, prob.ny, prob.nz))
    edof = fem.element_dofs(prob.nx, prob.ny, prob.nz)
    cases = range(prob.n_case) if case is None else [case]
    us, Cs = [], []
    dc = np.zeros(prob.n_elem)
    free = fem.free_mask(K.shape[0], fixed)
    for l in cases:
        f = fem.dof_vector_aos(prob, l) * free
        u = ds.solve(f)
        us.append(u)
        Cs.append(compliance(f, u))
        dc += dc_drho_phys(rho_phys.ravel(), element_energy(u, edof, KE), E0, Emin, p)
    return us, Cs, dc
