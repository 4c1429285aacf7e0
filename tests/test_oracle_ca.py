"""Pins of the oracle's combined-approximation reanalysis (eqs. 8-29,
Algorithm 1) and OC update against exact identities and textbook PCG."""

import numpy as np
import scipy.linalg as sla

import synth
from oracle import ca, fem, filt, oc, solve


def _ops(dims, seed, amp=0.2):
    prob = synth.cantilever(*dims)
    rng = np.random.default_rng(seed)
    rho0 = rng.uniform(0.3, 1.0, prob.n_elem)
    rho1 = np.clip(rho0 + rng.uniform(-amp, amp, prob.n_elem), 0.05, 1.0)
    KE = fem.hex8_ke()
    fixed = fem.fixed_dofs_aos(prob)
    K0 = fem.assemble(*dims, fem.simp(rho0), KE)
    K1 = fem.assemble(*dims, fem.simp(rho1), KE)
    A0 = fem.operator_with_bc(K0, fixed)
    A1 = fem.operator_with_bc(K1, fixed)
    free = fem.free_mask(K0.shape[0], fixed)
    f = fem.dof_vector_aos(prob) * free
    return prob, A0, A1, f, free, K0, K1, fixed


def textbook_pcg(A, f, Minv, m):
    """Plain preconditioned CG from x0 = 0, m iterations."""
    x = np.zeros_like(f)
    r = f.copy()
    z = Minv(r)
    p = z.copy()
    for _ in range(m):
        q = A @ p
        a = (r @ z) / (p @ q)
        x = x + a * p
        rn = r - a * q
        zn = Minv(rn)
        p = zn + ((rn @ zn) / (r @ z)) * p
        r, z = rn, zn
    return x


def test_kirsch_equivalence_classic_ca_is_pcg():
    """Classic CA with the exact K0^-1 and r_1 = K0^-1 f gives the m-th
    iterate of K0-preconditioned CG (the equivalence the paper cites in its
    introduction)."""
    _, A0, A1, f, free, *_ = _ops((4, 2, 2), 0, amp=0.3)
    A0d = A0.toarray()
    Minv = lambda r: sla.solve(A0d, r, assume_a="pos")
    for m in (1, 2, 3, 4):
        u_ca = ca.classic_ca(A0, A1, f, m)
        u_cg = textbook_pcg(A1, f, Minv, m)
        assert np.linalg.norm(u_ca - u_cg) <= 1e-9 * np.linalg.norm(u_cg)


def test_eq18_exact_for_square_phi():
    """eq. (18): with Phi square and invertible, Phi K_Phi^-1 Phi^T = K0^-1."""
    _, A0, _, _, _, *_ = _ops((1, 1, 1), 1)
    A0d = A0.toarray()
    Phi = np.random.default_rng(3).standard_normal(A0d.shape)
    KPhi = ca.k_phi(A0d, Phi)
    approx = Phi @ np.linalg.solve(KPhi, Phi.T)
    assert np.abs(approx - np.linalg.inv(A0d)).max() <= 1e-8 * np.abs(np.linalg.inv(A0d)).max()


def test_basis_rank_at_most_ns_plus_one():
    _, A0, A1, f, free, K0, K1, fixed = _ops((6, 3, 3), 2)
    us = [solve.solve_direct(K, f, fixed) for K in (K0, K0 + 0.5 * K1)]
    Phi = np.stack([ca.parm_vector(u) for u in us], axis=1)
    u_last = solve.solve_direct(K0, f, fixed) * 1.1 + 0.01 * free
    R = ca.carm_basis(A1, A0, Phi, u_last, 6)
    s = np.linalg.svd(R / np.linalg.norm(R, axis=0), compute_uv=False)
    assert (s > 1e-10 * s[0]).sum() <= Phi.shape[1] + 1
    assert ca.orthogonalise_svd(R).shape[1] <= Phi.shape[1] + 1


def test_gram_schmidt_basis_gives_same_solution():
    """u~ depends only on span(R~): the SVD basis (eq. 21) and a QR
    (Gram-Schmidt) basis of the same columns agree."""
    _, A0, A1, f, free, K0, K1, fixed = _ops((6, 3, 3), 3)
    rng = np.random.default_rng(5)
    Phi = np.stack([ca.parm_vector(rng.standard_normal(len(f)) * free) for _ in range(3)], 1)
    u_last = solve.solve_direct(K0, f, fixed)
    R = ca.carm_basis(A1, A0, Phi, u_last, 3)
    u_svd, _, _ = ca.reduced_solve(A1, ca.orthogonalise_svd(R), f)
    Q, _ = np.linalg.qr(R)
    u_qr, _, _ = ca.reduced_solve(A1, Q, f)
    assert np.linalg.norm(u_svd - u_qr) <= 1e-10 * np.linalg.norm(u_qr)


def test_no_change_exact_u_last_is_exact():
    _, A0, _, f, free, K0, _, fixed = _ops((4, 2, 2), 4)
    u = solve.solve_direct(K0, f, fixed)
    Phi = np.stack([ca.parm_vector(u), ca.parm_vector(np.roll(u, 3) * free)], 1)
    ut, eps, rank = ca.ca_approximation(A0, A0, Phi, u, f, 2)
    assert rank == 1  # dK = 0 makes r_2 = 0
    assert np.linalg.norm(ut - u) <= 1e-12 * np.linalg.norm(u)
    assert eps < 1e-12


def test_full_span_basis_is_exact_and_galerkin_identity():
    _, A0, A1, f, free, K0, K1, fixed = _ops((1, 1, 1), 6)
    n_free = int(free.sum())
    rng = np.random.default_rng(7)
    R = np.zeros((len(f), n_free))
    R[free] = rng.standard_normal((n_free, n_free))
    u_t, y, KR = ca.reduced_solve(A1, ca.orthogonalise_svd(R), f)
    u = solve.solve_direct(K1, f, fixed)
    assert np.linalg.norm(u_t - u) <= 1e-10 * np.linalg.norm(u)
    # Galerkin: u~^T K u~ = f^T u~ for any basis
    R2 = R[:, :3]
    u2, _, _ = ca.reduced_solve(A1, ca.orthogonalise_svd(R2), f)
    assert abs(u2 @ (A1 @ u2) - f @ u2) <= 1e-12 * abs(f @ u2)


def test_aarmr_loop_paths_and_accuracy():
    """Algorithm 1 on a short perturbation sequence: loops <= N_on solve
    exactly; later loops accept the CA approximation only when eps < tol,
    and an accepted u~ has force residual eps."""
    prob = synth.cantilever(6, 3, 3)
    rng = np.random.default_rng(8)
    rho = rng.uniform(0.3, 1.0, prob.n_elem)
    alg = ca.AARMR(prob, Ns=2, Nm=3, N_on=3, eps_tol=0.11)
    paths = []
    for loop in range(1, 9):
        rho = np.clip(rho + rng.uniform(-0.01, 0.01, prob.n_elem), 0.05, 1.0)
        (u, path, eps, rank), = alg.cycle(loop, rho)
        paths.append(path)
        K, A = alg.operator(rho)
        if path == "ca":
            assert eps < 0.11
            assert abs(ca.force_residual(A, u, alg.f[0]) - eps) < 1e-12
            assert rank <= 3
        else:
            assert solve.residual_norm(K, u, alg.f[0], alg.fixed) < 1e-10
    assert paths[:3] == ["mgcg"] * 3
    assert "ca" in paths[3:]
    assert len(alg.states[0].Phi) == 2


def test_oc_volume_and_bounds():
    nx, ny, nz = 6, 4, 4
    n = nx * ny * nz
    H, Hs = filt.filter_matrix(nx, ny, nz, 1.5)
    rng = np.random.default_rng(9)
    x = np.full(n, 0.3)
    dc = -rng.uniform(0.1, 2.0, n)
    dv = filt.adjoint(H, Hs, np.ones(n))
    xn, xp, lam = oc.oc_update(x, dc, dv, H, Hs, 0.3)
    assert np.all(xn >= np.maximum(0, x - 0.2) - 1e-15)
    assert np.all(xn <= np.minimum(1, x + 0.2) + 1e-15)
    assert abs(xp.sum() / n - 0.3) < 1e-2


def test_reduced_solve_and_force_residual_by_hand():
    """eqs. 22-25 and 29 on a 3x3 case solved by hand: K = diag(1, 2, 4),
    f = (1, 1, 1).  With the basis e1: K_R = 1, y = 1, u~ = (1, 0, 0), the
    force residual K u~ - f = (0, -1, -1) and eps = sqrt(2) / sqrt(3).  With
    the basis (1, 1, 0)/sqrt(2): K_R = 3/2, f_R = sqrt(2), u~ = (2/3, 2/3, 0),
    K u~ - f = (-1/3, 1/3, -1) and eps = sqrt(11/9) / sqrt(3).  eps is relative
    to the load, not to the displacement."""
    K = np.diag([1.0, 2.0, 4.0])
    f = np.ones(3)
    u, y, KR = ca.reduced_solve(K, np.array([[1.0], [0.0], [0.0]]), f)
    assert np.allclose(u, [1.0, 0.0, 0.0], atol=1e-15) and np.allclose(y, [1.0])
    assert abs(ca.force_residual(K, u, f) - np.sqrt(2.0 / 3.0)) < 1e-15
    Rt = np.array([[1.0], [1.0], [0.0]]) / np.sqrt(2.0)
    u, y, KR = ca.reduced_solve(K, Rt, f)
    assert np.allclose(y, [np.sqrt(2.0) / 1.5], rtol=1e-15)
    assert np.allclose(u, [2.0 / 3.0, 2.0 / 3.0, 0.0], atol=1e-15)
    assert np.allclose(KR[:, 0], K @ Rt[:, 0], atol=1e-15)
    assert abs(ca.force_residual(K, u, f) - np.sqrt(11.0 / 27.0)) < 1e-15


def test_svd_cutoff_is_relative_to_largest_singular_value():
    """eq. 21 truncation, read as sigma_i / sigma_1 > tau on column-normalised
    R.  Two columns 3 e1 and 5 (e1 + d e2) normalise to unit vectors with
    cosine c = 1 / sqrt(1 + d^2); their Gram matrix [[1, c], [c, 1]] gives
    sigma_1 = sqrt(1 + c) and sigma_2 = sqrt(1 - c), the leading singular
    vector along the sum of the two unit columns.  A tau between sigma_2 and
    sigma_2 / sigma_1 separates the relative cut-off (rank 1) from an absolute
    one (rank 2)."""
    d = 1e-3
    R = np.zeros((4, 2))
    R[0, 0] = 3.0
    R[0, 1], R[1, 1] = 5.0, 5.0 * d
    s = np.sqrt(1.0 + d * d)
    one_minus_c = d * d / (s * (1.0 + s))
    s1, s2 = np.sqrt(2.0 - one_minus_c), np.sqrt(one_minus_c)
    assert s2 / s1 < s2 / 1.2 < s2
    Rt = ca.orthogonalise_svd(R, tau=s2 / 1.2)
    assert Rt.shape == (4, 1)
    lead = np.array([1.0, 0.0, 0.0, 0.0]) + np.array([1.0, d, 0.0, 0.0]) / s
    lead /= np.linalg.norm(lead)
    assert abs(abs(Rt[:, 0] @ lead) - 1.0) < 1e-14
    Rt2 = ca.orthogonalise_svd(R, tau=s2 / s1 / 1.2)
    assert Rt2.shape == (4, 2)
    assert np.allclose(Rt2.T @ Rt2, np.eye(2), atol=1e-12)
    assert ca.orthogonalise_svd(R, tau=s2 / s1 * 1.2).shape == (4, 1)


def test_oc_volume_constraint_is_on_the_filtered_density():
    """eq. 3 constrains the volume of the filtered density rho~ = H x / Hs, not
    of x.  The volume of the filtered trial design is non-increasing in the
    multiplier, so the bisection's final multiplier must bracket the target
    within its stopping gap (a relative width of 1e-3, hence a factor
    1 +- 3e-3 on the multiplier).  The sensitivities favour boundary elements,
    whose filter column sums differ from one, so the unfiltered volume misses
    the target by far more than the gap."""
    nx, ny, nz = 6, 4, 4
    n = nx * ny * nz
    H, Hs = filt.filter_matrix(nx, ny, nz, 2.0)
    cw = filt.adjoint(H, Hs, np.ones(n))
    rng = np.random.default_rng(3)
    x = np.full(n, 0.4)
    dc = -np.where(cw > 1.0, 10.0, 0.1) * rng.uniform(0.9, 1.1, n)
    xn, xp, lam = oc.oc_update(x, dc, cw, H, Hs, 0.4)

    def filtered_volume(l):
        B = np.maximum(0.0, -dc) / cw
        t = np.clip(x * np.sqrt(B / l), np.maximum(0.0, x - 0.2), np.minimum(1.0, x + 0.2))
        return (H @ t / Hs).sum()

    target = 0.4 * n
    assert filtered_volume(lam * (1 - 3e-3)) >= target >= filtered_volume(lam * (1 + 3e-3))
    assert np.allclose(xp, (H @ xn) / Hs, rtol=1e-15)
    assert abs(xn.sum() - target) > 0.02 * target
