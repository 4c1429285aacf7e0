"""Combined-approximation reanalysis with a projection auxiliary model.

Followed in the paper's order and notation (Section 2.2, Section 3.1,
Algorithm 1):

* classic CA (eqs. 8-14): B = -K0^-1 dK, r_1 = u_0, r_i = B r_(i-1),
  K R y = f solved in the least-squares/Galerkin sense R^T K R y = R^T f;
* PARM (eqs. 15-18, 27-28): Phi = [u_i / ||u_i||], K_Phi = Phi^T K0 Phi and
  the approximate inverse K0^-1 ~ Phi K_Phi^-1 Phi^T;
* CARM basis (eqs. 19-20, 26): r_1 = u_last, r_i = -Phi K_Phi^-1 Phi^T dK r_(i-1);
* orthogonalisation by SVD (eq. 21), reduced system (eqs. 22-25);
* force-residual fidelity criterion (eq. 29) with the MGCG fallback and the
  first-in-first-out PARM update (Algorithm 1, lines 6-10).

All operators are the full-size boundary-condition operators
A = Df K Df + (I - Df) (identity on fixed DOFs) and loads are zero on fixed
DOFs, so every basis vector vanishes on fixed DOFs.  The exact solve stands in
for MGCG: MGCG converges to it, and the oracle needs the plain definition.

Readings taken where the paper is silent or inconsistent: K0 is the stiffness
of the previous design cycle and u_last the previous accepted displacement;
Algorithm 1 line 5 is read as (R^T K R) y = R^T f (eq. 23); the criterion
accepts iff eps < eps_tol; the SVD keeps singular vectors with
sigma_i / sigma_1 > tau on column-normalised R.
"""

from __future__ import annotations

from typing import List, Optional

import numpy as np
import scipy.linalg as sla

from . import fem, solve


def parm_vector(u: np.ndarray) -> np.ndarray:
    """eq. (28): phi(u) = u / ||u||."""
    return u / np.linalg.norm(u)


def parm_fifo(Phi: List[np.ndarray], u: np.ndarray, Ns: int) -> List[np.ndarray]:
    """PARM update: drop the earliest vector once Ns are held, append the
    newest normalised displacement (eq. 27 and its update rule)."""
    out = list(Phi) + [parm_vector(u)]
    return out[-Ns:]


def k_phi(A0, Phi: np.ndarray) -> np.ndarray:
    """eq. (15): K_Phi = Phi^T K0 Phi (s x s)."""
    return Phi.T @ (A0 @ Phi)


def approximate_inverse_apply(Phi: np.ndarray, KPhi: np.ndarray, x: np.ndarray) -> np.ndarray:
    """eq. (18): K0^-1 x ~ Phi K_Phi^-1 Phi^T x."""
    return Phi @ np.linalg.solve(KPhi, Phi.T @ x)


def carm_basis(A, A0, Phi: np.ndarray, u_last: np.ndarray, m: int) -> np.ndarray:
    """eqs. (20)/(26): R = [r_1, C r_1, ..., C^(m-1) r_1] with r_1 = u_last and
    C = -Phi K_Phi^-1 Phi^T dK, dK = K - K0."""
    KPhi = k_phi(A0, Phi)
    R = [np.asarray(u_last, dtype=np.float64)]
    for _ in range(1, m):
        t = A @ R[-1] - A0 @ R[-1]
        R.append(-approximate_inverse_apply(Phi, KPhi, t))
    return np.stack(R, axis=1)


def orthogonalise_svd(R: np.ndarray, tau: float = 1e-10) -> np.ndarray:
    """eq. (21): R = R~ Sigma V^T; keep columns of R~ whose singular value
    exceeds tau times the largest (columns of R are normalised first)."""
    norms = np.linalg.norm(R, axis=0)
    Rn = R[:, norms > 0] / norms[norms > 0]
    U, S, _ = np.linalg.svd(Rn, full_matrices=False)
    keep = S > tau * S[0]
    return U[:, keep]


def reduced_solve(A, Rt: np.ndarray, f: np.ndarray):
    """eqs. (22)-(25): K_R~ = R~^T K R~, f_R~ = R~^T f, solve, u~ = R~ y.
    Returns (u~, y, K R~)."""
    KR = A @ Rt
    KRt = Rt.T @ KR
    fR = Rt.T @ f
    y = sla.solve(KRt, fR, assume_a="pos")
    return Rt @ y, y, KR


def force_residual(A, u: np.ndarray, f: np.ndarray) -> float:
    """eq. (29): ||K u - f|| / ||f||."""
    return float(np.linalg.norm(A @ u - f) / np.linalg.norm(f))


def ca_approximation(A, A0, Phi: np.ndarray, u_last, f, m: int, tau: float = 1e-10):
    """Algorithm 1 lines 4-6: basis, orthogonalisation, reduced solve and
    criterion.  Returns (u~, eps, rank)."""
    R = carm_basis(A, A0, Phi, u_last, m)
    Rt = orthogonalise_svd(R, tau)
    u, _, _ = reduced_solve(A, Rt, f)
    return u, force_residual(A, u, f), Rt.shape[1]


def classic_ca(A0, A, f, m: int) -> np.ndarray:
    """eqs. (8)-(14) with the exact reference inverse: r_1 = u_0 = K0^-1 f,
    r_i = -K0^-1 dK r_(i-1), then R^T K R y = R^T f and u = R y."""
    solve0 = lambda b: sla.solve(A0.toarray() if hasattr(A0, "toarray") else A0, b,
                                 assume_a="pos")
    R = [solve0(f)]
    for _ in range(1, m):
        R.append(-solve0(A @ R[-1] - A0 @ R[-1]))
    R = np.stack(R, axis=1)
    y = sla.solve(R.T @ (A @ R), R.T @ f, assume_a="pos")
    return R @ y


class AARMRState:
    """Per-load-case state of Algorithm 1: PARM vectors, last displacement."""

    def __init__(self, Ns: int):
        self.Ns = Ns
        self.Phi: List[np.ndarray] = []
        self.u_last: Optional[np.ndarray] = None


class AARMR:
    """Algorithm 1 on one problem with the exact solve in place of MGCG.

    ``cycle(loop, rho_phys)`` runs one design cycle (1-based ``loop``):
    loops 1..N_on solve exactly and record the last Ns normalised solutions
    into PARM; later loops build the CARM from K0 = K(rho~ of the previous
    cycle), accept u~ if eps < eps_tol and otherwise solve exactly and update
    PARM first-in-first-out."""

    def __init__(self, prob, Ns=2, Nm=2, N_on=20, eps_tol=1e-3, tau=1e-10,
                 E0=1.0, Emin=1e-9, p=3.0, nu=0.3):
        self.prob = prob
        self.Ns, self.Nm, self.N_on, self.eps_tol, self.tau = Ns, Nm, N_on, eps_tol, tau
        self.E0, self.Emin, self.p = E0, Emin, p
        self.KE = fem.hex8_ke(1.0, nu)
        self.fixed = fem.fixed_dofs_aos(prob)
        n = 3 * prob.n_node
        self.free = fem.free_mask(n, self.fixed)
        self.f = [fem.dof_vector_aos(prob, l) * self.free for l in range(prob.n_case)]
        self.states = [AARMRState(Ns) for _ in range(prob.n_case)]
        self.A_prev = None

    def operator(self, rho_phys):
        Ee = fem.simp(np.ravel(rho_phys), self.E0, self.Emin, self.p)
        K = fem.assemble(self.prob.nx, self.prob.ny, self.prob.nz, Ee, self.KE)
        return K, fem.operator_with_bc(K, self.fixed)

    def cycle(self, loop: int, rho_phys):
        K, A = self.operator(rho_phys)
        dims = (self.prob.nx, self.prob.ny, self.prob.nz)
        direct = None
        out = []
        for l, st in enumerate(self.states):
            f = self.f[l]
            if loop <= self.N_on or self.A_prev is None or len(st.Phi) < self.Ns:
                if direct is None:
                    direct = solve.DirectSolver(K, self.fixed, dims)
                u = direct.solve(f)
                if loop > self.N_on - self.Ns:
                    st.Phi = parm_fifo(st.Phi, u, self.Ns)
                path, eps, rank = "mgcg", 0.0, 0
            else:
                Phi = np.stack(st.Phi, axis=1)
                u, eps, rank = ca_approximation(A, self.A_prev, Phi, st.u_last, f,
                                                self.Nm, self.tau)
                path = "ca"
                if not eps < self.eps_tol:
                    if direct is None:
                        direct = solve.DirectSolver(K, self.fixed, dims)
                    u = direct.solve(f)
                    st.Phi = parm_fifo(st.Phi, u, self.Ns)
                    path = "fallback"
            st.u_last = u
            out.append((u, path, eps, rank))
        self.A_prev = A
        return out
