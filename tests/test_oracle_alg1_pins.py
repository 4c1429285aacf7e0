"""Pins of the oracle's Algorithm 1 pieces that the GPU path shares readings
with: K_Phi built from the reference stiffness K0 (eqs. 15, 18, 20), the
first-in-first-out PARM rule (eqs. 27-28, Algorithm 1 line 10), which design
cycles record into the PARM and which design supplies K0 (Algorithm 1 lines
1-3, Section 3.1), and the OC update against a hand-solved two-element case.

Each pin is chosen so that a plausible slip in the oracle (K in place of K0,
keeping the oldest PARM vectors, recording one cycle too early, freezing K0,
another damping exponent) turns at least one test red.
"""

import numpy as np
import scipy.linalg as sla

import synth
from oracle import ca, fem, filt, oc, solve


def _pair(dims, seed, amp=0.3):
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


def _pcg_iterate(A, f, Minv, m):
    """m iterations of preconditioned CG from zero, written independently of
    the oracle (the equivalence in the paper's introduction: classic CA with
    the exact reference inverse reproduces these iterates)."""
    x = np.zeros_like(f)
    r = f.copy()
    z = Minv(r)
    p = z.copy()
    rz = r @ z
    for _ in range(m):
        q = A @ p
        a = rz / (p @ q)
        x += a * p
        r -= a * q
        z = Minv(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x


def test_carm_with_square_phi_reproduces_reference_preconditioned_cg():
    """eq. (18) makes Phi K_Phi^-1 Phi^T the exact K0^-1 when Phi is square and
    invertible; then the CARM basis from r_1 = K0^-1 f is the classic CA basis
    and its reduced solution is the m-th K0-preconditioned CG iterate.  Using
    the current K in K_Phi (instead of K0) gives a different Krylov space and
    fails this."""
    _, A0, A1, f, free, *_ = _pair((3, 2, 2), 11)
    A0d, A1d = A0.toarray(), A1.toarray()
    n = A0d.shape[0]
    Phi = np.random.default_rng(12).standard_normal((n, n))
    Minv = lambda r: sla.solve(A0d, r, assume_a="pos")
    r1 = Minv(f)
    for m in (2, 3, 4):
        R = ca.carm_basis(A1d, A0d, Phi, r1, m)
        u_carm, _, _ = ca.reduced_solve(A1d, ca.orthogonalise_svd(R), f)
        u_pcg = _pcg_iterate(A1d, f, Minv, m)
        assert np.linalg.norm(u_carm - u_pcg) <= 1e-8 * np.linalg.norm(u_pcg), m
        # and the same through the classic CA the paper starts from
        u_cls = ca.classic_ca(A0d, A1d, f, m)
        assert np.linalg.norm(u_cls - u_pcg) <= 1e-8 * np.linalg.norm(u_pcg), m


def test_carm_second_vector_uses_reference_stiffness():
    """r_2 = -K0^-1 (K - K0) r_1 with square Phi: K0 r_2 = -(K - K0) r_1 holds
    to rounding, which fixes both the operator inverted (K0) and the sign and
    order of the difference (eq. 20)."""
    _, A0, A1, f, free, *_ = _pair((2, 2, 1), 13)
    A0d, A1d = A0.toarray(), A1.toarray()
    n = A0d.shape[0]
    Phi = np.random.default_rng(14).standard_normal((n, n))
    r1 = np.random.default_rng(15).standard_normal(n) * free
    R = ca.carm_basis(A1d, A0d, Phi, r1, 3)
    lhs = A0d @ R[:, 1]
    rhs = -(A1d - A0d) @ r1
    assert np.linalg.norm(lhs - rhs) <= 1e-9 * np.linalg.norm(rhs)
    lhs3 = A0d @ R[:, 2]
    rhs3 = -(A1d - A0d) @ R[:, 1]
    assert np.linalg.norm(lhs3 - rhs3) <= 1e-9 * np.linalg.norm(rhs3)


def test_parm_fifo_keeps_newest_in_order():
    """Algorithm 1 line 10 and the PARM update rule: the earliest vector is
    removed and the latest normalised displacement appended (eqs. 27-28)."""
    rng = np.random.default_rng(16)
    us = [rng.standard_normal(30) * (k + 1) for k in range(5)]
    for Ns in (1, 2, 3):
        Phi = []
        for k, u in enumerate(us):
            Phi = ca.parm_fifo(Phi, u, Ns)
            held = us[max(0, k + 1 - Ns):k + 1]
            assert len(Phi) == len(held)
            for got, want in zip(Phi, held):
                assert np.allclose(got, want / np.linalg.norm(want), rtol=0, atol=1e-15)
                assert abs(np.linalg.norm(got) - 1.0) < 1e-14


def _exact(prob, rho):
    KE = fem.hex8_ke()
    K = fem.assemble(prob.nx, prob.ny, prob.nz, fem.simp(rho), KE)
    fixed = fem.fixed_dofs_aos(prob)
    f = fem.dof_vector_aos(prob) * fem.free_mask(K.shape[0], fixed)
    return solve.solve_direct(K, f, fixed)


def test_parm_records_exactly_the_last_ns_warmup_cycles():
    """Loops 1..N_on use MGCG, and the PARM holds the normalised solutions of
    loops N_on-Ns+1..N_on: after loop N_on-1 it holds one vector (loop
    N_on-1's), after loop N_on the two of loops N_on-1 and N_on."""
    prob = synth.cantilever(4, 2, 2)
    rng = np.random.default_rng(17)
    designs = [rng.uniform(0.3, 1.0, prob.n_elem) for _ in range(5)]
    alg = ca.AARMR(prob, Ns=2, Nm=3, N_on=4, eps_tol=1e-3)
    for loop in range(1, 5):
        (u, path, _, _), = alg.cycle(loop, designs[loop - 1])
        assert path == "mgcg"
        held = alg.states[0].Phi
        if loop <= 2:
            assert held == []
        elif loop == 3:
            assert len(held) == 1
            want = _exact(prob, designs[2])
            assert np.allclose(held[0], want / np.linalg.norm(want), rtol=0, atol=1e-12)
        else:
            assert len(held) == 2
            for got, d in zip(held, (designs[2], designs[3])):
                want = _exact(prob, d)
                assert np.allclose(got, want / np.linalg.norm(want), rtol=0, atol=1e-12)
    # the first CA cycle uses u_last = loop N_on's solution
    assert np.allclose(alg.states[0].u_last, _exact(prob, designs[3]), rtol=0, atol=1e-10)


def test_reference_stiffness_is_the_previous_cycle():
    """K0 = K(rho~ of the previous design cycle) (Section 3.1): a design that
    repeats the previous cycle's gives dK = 0, so the CARM has rank 1 and,
    with an exact u_last (the previous cycle fell back to the exact solve),
    the reduced solution is exact.  A K0 frozen at an earlier design makes
    dK nonzero and the rank larger."""
    prob = synth.cantilever(4, 2, 2)
    rng = np.random.default_rng(18)
    designs = [rng.uniform(0.3, 1.0, prob.n_elem) for _ in range(3)]
    alg = ca.AARMR(prob, Ns=2, Nm=4, N_on=3, eps_tol=1e-8)
    for loop in range(1, 4):
        alg.cycle(loop, designs[loop - 1])
    far = rng.uniform(0.3, 1.0, prob.n_elem)  # a large change: CA rejected
    (u4, path4, eps4, rank4), = alg.cycle(4, far)
    assert path4 == "fallback" and eps4 >= 1e-8
    (u5, path5, eps5, rank5), = alg.cycle(5, far)  # repeat of cycle 4's design
    assert rank5 == 1
    assert path5 == "ca" and eps5 < 1e-10
    assert np.linalg.norm(u5 - _exact(prob, far)) <= 1e-9 * np.linalg.norm(u5)


def test_accepted_ca_solution_becomes_u_last_and_leaves_parm():
    """An accepted cycle (Algorithm 1 line 7) keeps the PARM unchanged and its
    u~ is the next cycle's r_1; a rejected one appends the exact solution."""
    prob = synth.cantilever(4, 2, 2)
    rng = np.random.default_rng(19)
    rho = rng.uniform(0.3, 1.0, prob.n_elem)
    alg = ca.AARMR(prob, Ns=2, Nm=3, N_on=2, eps_tol=0.5)
    step = lambda r, k: np.clip(r + rng.uniform(-0.02, 0.02, r.size), 0.05, 1.0)
    rho1 = step(rho, 0)
    rho2 = step(rho1, 1)
    rho3 = step(rho2, 2)
    alg.cycle(1, rho1)
    alg.cycle(2, rho2)
    before = [p.copy() for p in alg.states[0].Phi]
    (u3, path3, eps3, _), = alg.cycle(3, rho3)
    assert path3 == "ca"
    assert all(np.array_equal(a, b) for a, b in zip(before, alg.states[0].Phi))
    assert np.array_equal(alg.states[0].u_last, u3)
    alg.eps_tol = 1e-14
    rho4 = rng.uniform(0.3, 1.0, prob.n_elem)
    (u4, path4, _, _), = alg.cycle(4, rho4)
    assert path4 == "fallback"
    want = _exact(prob, rho4)
    assert np.allclose(alg.states[0].Phi[-1], want / np.linalg.norm(want), rtol=0, atol=1e-12)
    assert np.allclose(alg.states[0].Phi[0], before[-1], rtol=0, atol=0)


def test_oc_two_element_hand_solution():
    """Two elements, no filtering (r = 1 leaves only the self weight), equal
    start x: OC scales x_e by (B_e / lambda)^eta with B_e = -dc_e / dv_e, so
    the constraint x1 + x2 = 2 V gives x_e = 2 V B_e^eta / (B_1^eta + B_2^eta)
    while no move limit is active.  The bisection stops at a relative
    multiplier gap of 1e-3, which moves x by less than eta * 1e-3
    relatively."""
    H, Hs = filt.filter_matrix(2, 1, 1, 1.0)
    assert np.allclose(H.toarray(), np.eye(2))
    x = np.array([0.5, 0.5])
    dv = np.ones(2)
    for B1, B2, V in ((1.0, 1.21, 0.5), (2.0, 0.9, 0.45), (0.3, 0.3, 0.4)):
        dc = -np.array([B1, B2])
        xn, xp, lam = oc.oc_update(x, dc, dv, H, Hs, V)
        s = np.sqrt(np.array([B1, B2]))
        want = 2 * V * s / s.sum()
        assert np.all(np.abs(want - x) < 0.2)  # no move limit active
        assert np.allclose(xn, want, rtol=1e-3, atol=0), (xn, want)
        assert np.allclose(xp, xn, rtol=0, atol=0)
        # the multiplier that produced it
        assert np.allclose(x * np.sqrt(np.array([B1, B2]) / lam), xn, rtol=1e-12)


def test_oc_move_limit_and_box():
    """A large sensitivity ratio drives one element to its move limit (x +/-
    0.2) or the box [0, 1]; the other takes the remaining volume."""
    H, Hs = filt.filter_matrix(2, 1, 1, 1.0)
    x = np.array([0.5, 0.5])
    xn, _, _ = oc.oc_update(x, np.array([-100.0, 0.0]), np.ones(2), H, Hs, 0.5)
    assert abs(xn[0] - 0.7) < 1e-15 and abs(xn[1] - 0.3) < 1e-15
    x = np.array([0.95, 0.05])
    xn, _, _ = oc.oc_update(x, np.array([-100.0, 0.0]), np.ones(2), H, Hs, 0.5)
    assert xn[0] == 1.0 and xn[1] == 0.0
