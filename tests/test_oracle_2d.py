"""Pins of the 2D plane-stress oracle (Q4, Sections 4.1, 4.2.1, 4.3) against
closed forms and independent computations."""

import numpy as np
import pytest

import synth
from oracle import fem, fem2d, mg, solve


def test_q4_ke_closed_forms():
    nu = 0.3
    KE = fem2d.q4_ke(1.0, nu)
    assert np.allclose(KE, KE.T, atol=1e-15)
    # diagonal: E/(1-nu^2) * (1/3 + (1-nu)/2 * 1/3) = (3 - nu) / (6 (1 - nu^2))
    assert np.allclose(np.diag(KE), (3.0 - nu) / (6.0 * (1.0 - nu * nu)), rtol=0, atol=1e-15)
    w, V = np.linalg.eigh(KE)
    assert np.sum(np.abs(w) < 1e-12) == 3 and w.min() > -1e-13
    # rigid modes: two translations and the in-plane rotation
    xy = np.array([[a & 1, a >> 1] for a in range(4)], dtype=float)
    modes = [np.tile([1.0, 0.0], 4), np.tile([0.0, 1.0], 4),
             np.column_stack([-xy[:, 1], xy[:, 0]]).ravel()]
    for r in modes:
        assert np.abs(KE @ r).max() < 1e-14


@pytest.mark.parametrize("strain", [(1, 0, 0), (0, 1, 0), (0, 0, 1), (0.3, -0.7, 0.2)])
def test_q4_constant_strain_energy(strain):
    """u = (exx x + gxy/2 y, eyy y + gxy/2 x): energy u^T KE u = eps^T D eps (unit area)."""
    nu = 0.3
    exx, eyy, gxy = strain
    xy = np.array([[a & 1, a >> 1] for a in range(4)], dtype=float)
    u = np.column_stack([exx * xy[:, 0] + 0.5 * gxy * xy[:, 1],
                         eyy * xy[:, 1] + 0.5 * gxy * xy[:, 0]]).ravel()
    eps = np.array([exx, eyy, gxy])
    D = np.array([[1, nu, 0], [nu, 1, 0], [0, 0, (1 - nu) / 2]]) / (1 - nu * nu)
    assert abs(u @ fem2d.q4_ke(1.0, nu) @ u - eps @ D @ eps) < 1e-14


def test_patch_test_plane_stress():
    """Symmetry rollers (u_x = 0 on x = 0, u_y = 0 on y = 0), uniform traction
    sigma on x = nx with consistent nodal forces: u_x = sigma x / E,
    u_y = -nu sigma y / E exactly, C = sigma^2 V / E."""
    nx, ny, sigma, nu = 6, 4, 2.0, 0.3
    fixed = [(0, j, 0) for j in range(ny + 1)] + [(i, 0, 1) for i in range(nx + 1)]
    w = np.ones(ny + 1) / ny
    w[0] = w[-1] = 0.5 / ny
    loads = [[(nx, j, 0, sigma * ny * w[j]) for j in range(ny + 1)]]
    prob = synth.Problem2D(nx, ny, fixed, loads, "patch2d")
    us, Cs, _ = fem2d.analyse2(prob, np.ones(prob.n_elem), Emin=0.0)
    u = us[0].reshape(-1, 2)
    for j in range(ny + 1):
        for i in range(nx + 1):
            n = fem2d.node_id2(nx, i, j)
            assert abs(u[n, 0] - sigma * i) < 1e-12
            assert abs(u[n, 1] + nu * sigma * j) < 1e-12
    assert abs(Cs[0] - sigma ** 2 * nx * ny) < 1e-10


def test_sensitivity_complex_step_2d():
    prob = synth.cantilever2d(4, 2)
    rho = np.random.default_rng(5).uniform(0.3, 1.0, prob.n_elem)
    _, Cs, dc = fem2d.analyse2(prob, rho)
    KE = fem2d.q4_ke()
    fixed = fem2d.fixed_dofs_aos2(prob)
    free = fem.free_mask(2 * prob.n_node, fixed)
    f = fem2d.dof_vector_aos2(prob) * free
    h = 1e-30
    for e in range(prob.n_elem):
        r = rho.astype(complex)
        r[e] += 1j * h
        K = fem2d.assemble2(prob.nx, prob.ny, fem.simp(r), KE).toarray()
        idx = np.nonzero(free)[0]
        u = np.zeros(2 * prob.n_node, dtype=complex)
        u[idx] = np.linalg.solve(K[np.ix_(idx, idx)], f[idx])
        assert abs((f @ u).imag / h - dc[e]) <= 1e-12 * abs(dc[e])


def test_multigrid_2d_symmetric_and_mgcg_matches_direct():
    prob = synth.cantilever2d(16, 8)
    rho = np.random.default_rng(6).uniform(0.2, 1.0, prob.n_elem)
    K = fem2d.assemble2(16, 8, fem.simp(rho), fem2d.q4_ke())
    fixed = fem2d.fixed_dofs_aos2(prob)
    H = mg.Hierarchy(K, fixed, (16, 8), 3)
    rng = np.random.default_rng(7)
    free = fem.free_mask(K.shape[0], fixed)
    x, y = rng.standard_normal(K.shape[0]) * free, rng.standard_normal(K.shape[0]) * free
    assert abs(H.vcycle(x) @ y - x @ H.vcycle(y)) < 1e-11 * np.linalg.norm(x) * np.linalg.norm(y)
    f = fem2d.dof_vector_aos2(prob)
    u, its, rel = mg.mgcg(K, f, fixed, (16, 8), 3, rtol=1e-12)
    ud = solve.solve_direct(K, f * free, fixed)
    assert rel <= 1e-12 and np.linalg.norm(u - ud) <= 1e-9 * np.linalg.norm(ud)


def test_springs_proportional_to_traction_give_uniform_strain():
    """A strip on rollers (u_x = 0 on x = 0, u_y = 0 on y = 0) pulled by the
    consistent nodal forces of a uniform traction sigma on x = nx, with
    grounded springs kappa * ny * w_j proportional to the same weights:
    the uniform strain state u_x = eps x, u_y = -nu eps y is exact with
    eps = sigma / (E + kappa nx), and C = sigma ny eps nx."""
    nx, ny, sigma, kappa, nu = 6, 4, 2.0, 0.05, 0.3
    fixed = [(0, j, 0) for j in range(ny + 1)] + [(i, 0, 1) for i in range(nx + 1)]
    w = np.ones(ny + 1) / ny
    w[0] = w[-1] = 0.5 / ny
    loads = [[(nx, j, 0, sigma * ny * w[j]) for j in range(ny + 1)]]
    springs = [(nx, j, 0, kappa * ny * w[j]) for j in range(ny + 1)]
    prob = synth.Problem2D(nx, ny, fixed, loads, "spring_strip", springs)
    us, Cs, _ = fem2d.analyse2(prob, np.ones(prob.n_elem), Emin=0.0)
    eps = sigma / (1.0 + kappa * nx)
    u = us[0].reshape(-1, 2)
    for j in range(ny + 1):
        for i in range(nx + 1):
            n = fem2d.node_id2(nx, i, j)
            assert abs(u[n, 0] - eps * i) < 1e-12
            assert abs(u[n, 1] + nu * eps * j) < 1e-12
    assert abs(Cs[0] - sigma * ny * eps * nx) < 1e-10


def test_mechanism_sensitivity_complex_step():
    """The inverter's output displacement f_1^T u_0 (springs included)
    differentiated by a complex step in each element's modulus equals the
    adjoint sensitivity, and Maxwell-Betti reciprocity f_1^T u_0 = f_0^T u_1
    holds."""
    prob = synth.inverter2d(6, 4)
    rho = np.random.default_rng(8).uniform(0.3, 1.0, prob.n_elem)
    u0, u1, uout, dout = fem2d.mechanism2(prob, rho)
    fixed = fem2d.fixed_dofs_aos2(prob)
    free = fem.free_mask(2 * prob.n_node, fixed)
    f0 = fem2d.dof_vector_aos2(prob, 0) * free
    f1 = fem2d.dof_vector_aos2(prob, 1) * free
    assert abs(f1 @ u0 - f0 @ u1) <= 1e-12 * abs(uout)
    assert abs(f1 @ u0 - uout) == 0.0
    KE = fem2d.q4_ke()
    S = fem2d.spring_matrix2(prob).toarray()
    idx = np.nonzero(free)[0]
    h = 1e-30
    for e in range(prob.n_elem):
        r = rho.astype(complex)
        r[e] += 1j * h
        K = fem2d.assemble2(prob.nx, prob.ny, fem.simp(r), KE).toarray() + S
        u = np.zeros(2 * prob.n_node, dtype=complex)
        u[idx] = np.linalg.solve(K[np.ix_(idx, idx)], f0[idx])
        assert abs((f1 @ u).imag / h - dout[e]) <= 1e-10 * np.abs(dout).max()


def test_mechanism_springs_enter_the_objective():
    """Raising k_out stiffens the output: |u_out| falls; with both springs
    zero the objective is the spring-free analysis."""
    rho = np.full(8 * 4, 0.6)
    outs = [fem2d.mechanism2(synth.inverter2d(8, 4, 1.0, k), rho)[2] for k in (0.0, 0.1, 10.0)]
    assert abs(outs[0]) > abs(outs[1]) > abs(outs[2])
    bare = synth.inverter2d(8, 4, 0.0, 0.0)
    us, _, _ = fem2d.analyse2(synth.Problem2D(8, 4, bare.fixed, bare.loads), rho)
    assert abs(fem2d.mechanism2(bare, rho)[2] - us[0][2 * fem2d.node_id2(8, 8, 0)]) < 1e-15


def test_mutual_sensitivity_reduces_to_compliance():
    """With the dummy load equal to the input load, the mutual-energy
    sensitivity is the (pinned) compliance sensitivity."""
    base = synth.inverter2d(6, 4)
    prob = synth.Problem2D(6, 4, base.fixed, [base.loads[0], base.loads[0]], "same", base.springs)
    rho = np.random.default_rng(9).uniform(0.3, 1.0, prob.n_elem)
    _, _, uout, dout = fem2d.mechanism2(prob, rho)
    _, Cs, dc = fem2d.analyse2(synth.Problem2D(6, 4, base.fixed, [base.loads[0]], "c", base.springs), rho)
    assert abs(uout - Cs[0]) <= 1e-13 * Cs[0]
    assert np.abs(dout - dc).max() <= 1e-12 * np.abs(dc).max()


def test_springs_and_loads_on_one_dof_add_up():
    """Linearity of the boundary data: two springs (or two point loads) listed
    on the same DOF act as one with the summed stiffness (or force), so a
    problem split that way has the same operator, solution and compliance."""
    import dataclasses

    prob = synth.inverter2d(8, 4)
    i, j, c, k = prob.springs[0]
    split = dataclasses.replace(prob, springs=[(i, j, c, 0.25 * k), (i, j, c, 0.75 * k)]
                                + list(prob.springs[1:]))
    assert abs(fem2d.spring_matrix2(split) - fem2d.spring_matrix2(prob)).max() == 0.0
    (li, lj, lc, lv) = prob.loads[0][0]
    loads = [list(case) for case in prob.loads]
    loads[0] = [(li, lj, lc, 0.5 * lv), (li, lj, lc, 0.5 * lv)] + list(prob.loads[0][1:])
    split2 = dataclasses.replace(prob, loads=loads)
    assert np.array_equal(fem2d.dof_vector_aos2(split2, 0), fem2d.dof_vector_aos2(prob, 0))
    rho = np.full(prob.n_elem, 0.5)
    _, C1, _ = fem2d.analyse2(split2, rho)
    _, C0, _ = fem2d.analyse2(prob, rho)
    assert abs(C1[0] - C0[0]) <= 1e-12 * abs(C0[0])
