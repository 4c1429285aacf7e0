"""Pins of the oracle's discretisation, direct solve and sensitivities
against closed forms, invariants and brute force (no GPU)."""

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import fem, sens, solve


def rigid_modes(coords):
    """Three translations and three infinitesimal rotations, AoS, built from
    node coordinates only."""
    n = len(coords)
    modes = np.zeros((3 * n, 6))
    for a, (x, y, z) in enumerate(coords):
        modes[3 * a:3 * a + 3, 0] = (1, 0, 0)
        modes[3 * a:3 * a + 3, 1] = (0, 1, 0)
        modes[3 * a:3 * a + 3, 2] = (0, 0, 1)
        modes[3 * a:3 * a + 3, 3] = (-y, x, 0)
        modes[3 * a:3 * a + 3, 4] = (0, -z, y)
        modes[3 * a:3 * a + 3, 5] = (z, 0, -x)
    return modes


def test_ke_symmetric_psd_rank(gold):
    g = gold("hex8_closed_forms.txt")
    KE = fem.hex8_ke(1.0, 0.3)
    assert np.abs(KE - KE.T).max() < 1e-15
    w = np.linalg.eigvalsh(KE)
    assert w.min() > -1e-14
    assert int((w > 1e-10).sum()) == int(g["ke_rank"])


def test_ke_null_space_is_rigid_motion():
    KE = fem.hex8_ke(1.0, 0.3)
    coords = [fem.local_corner(a) for a in range(8)]
    assert np.abs(KE @ rigid_modes(coords)).max() < 1e-14


def test_ke_diagonal_closed_form(gold):
    g = gold("hex8_closed_forms.txt")
    KE = fem.hex8_ke(1.0, 0.3)
    assert np.allclose(np.diag(KE), g["ke_diag"], rtol=0, atol=1e-15)


def test_ke_constant_strain_energy(gold):
    g = gold("hex8_closed_forms.txt")
    KE = fem.hex8_ke(1.0, 0.3)
    coords = np.array([fem.local_corner(a) for a in range(8)], dtype=float)
    for comp in range(3):  # u_c = x_c  -> unit axial strain
        u = np.zeros(24)
        u[comp::3] = coords[:, comp]
        assert abs(u @ KE @ u - g["axial_energy"]) < 1e-14
    for (a, b) in [(0, 1), (1, 2), (0, 2)]:  # u_a = x_b -> unit engineering shear
        u = np.zeros(24)
        u[a::3] = coords[:, b]
        assert abs(u @ KE @ u - g["shear_energy"]) < 1e-14


def test_ke_scales_with_E():
    assert np.allclose(fem.hex8_ke(7.0, 0.3), 7.0 * fem.hex8_ke(1.0, 0.3), rtol=1e-14)


def test_global_k_rigid_modes_and_diag(gold):
    nx, ny, nz = 3, 2, 2
    rng = np.random.default_rng(0)
    Ee = rng.uniform(0.1, 1.0, nx * ny * nz)
    KE = fem.hex8_ke()
    K = fem.assemble(nx, ny, nz, Ee, KE)
    assert abs(K - K.T).max() < 1e-14
    coords = [(i, j, k) for k in range(nz + 1) for j in range(ny + 1) for i in range(nx + 1)]
    assert np.abs(K @ rigid_modes(coords)).max() < 1e-12
    # diag K at a node = KE_ii * sum of adjacent E (every KE_ii is equal)
    d = K.diagonal().reshape(-1, 3)
    want = np.zeros(len(coords))
    for e, (i, j, k) in enumerate([(i, j, k) for k in range(nz) for j in range(ny) for i in range(nx)]):
        for a in range(8):
            di, dj, dk = fem.local_corner(a)
            want[fem.node_id(nx, ny, i + di, j + dj, k + dk)] += Ee[e]
    assert np.allclose(d, gold("hex8_closed_forms.txt")["ke_diag"] * want[:, None], rtol=1e-14)


def test_patch_test_linear_solution(gold):
    g = gold("patch_test.txt")
    nx, ny, nz = 4, 2, 2
    prob = synth.patch_test(nx, ny, nz, sigma=g["sigma"])
    rho = np.ones(prob.n_elem)
    us, Cs, _ = sens.analyse(prob, rho)
    u = us[0].reshape(-1, 3)
    for k in range(nz + 1):
        for j in range(ny + 1):
            for i in range(nx + 1):
                n = fem.node_id(nx, ny, i, j, k)
                want = (g["sigma"] * i / g["E"], -g["nu"] * g["sigma"] * j / g["E"],
                        -g["nu"] * g["sigma"] * k / g["E"])
                assert np.allclose(u[n], want, atol=1e-12)
    assert abs(Cs[0] - g["sigma"] ** 2 * nx * ny * nz / g["E"]) < 1e-11


@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 1, 1), (2, 2, 2), (4, 2, 2), (6, 4, 4)])
def test_direct_solve_vs_dense_lu(dims):
    nx, ny, nz = dims
    prob = synth.cantilever(nx, ny, nz)
    rng = np.random.default_rng(1)
    Ee = fem.simp(rng.uniform(0.3, 1.0, prob.n_elem))
    K = fem.assemble(nx, ny, nz, Ee, fem.hex8_ke())
    fixed = fem.fixed_dofs_aos(prob)
    f = fem.dof_vector_aos(prob)
    u = solve.solve_direct(K, f, fixed, dims)
    free = fem.free_mask(K.shape[0], fixed)
    Kd = K.toarray()[np.ix_(free, free)]
    want = np.zeros_like(u)
    want[free] = np.linalg.solve(Kd, f[free])  # LU, a different routine
    assert np.linalg.norm(u - want) <= 1e-12 * np.linalg.norm(want)
    assert np.all(u[~free] == 0.0)


def test_banded_path_matches_dense_path():
    prob = synth.cantilever(16, 8, 8)  # > DENSE_LIMIT free DOFs -> banded
    rng = np.random.default_rng(2)
    Ee = fem.simp(rng.uniform(0.3, 1.0, prob.n_elem))
    K = fem.assemble(prob.nx, prob.ny, prob.nz, Ee, fem.hex8_ke())
    fixed = fem.fixed_dofs_aos(prob)
    f = fem.dof_vector_aos(prob)
    ds = solve.DirectSolver(K, fixed, (prob.nx, prob.ny, prob.nz))
    assert ds.mode == "banded"
    u = ds.solve(f)
    assert solve.residual_norm(K, u, f, fixed) < 1e-12
    free = fem.free_mask(K.shape[0], fixed)
    want = np.zeros_like(u)
    want[free] = np.linalg.solve(K.toarray()[np.ix_(free, free)], f[free])
    assert np.linalg.norm(u - want) <= 1e-11 * np.linalg.norm(want)


def test_energy_identity_and_uniform_scaling():
    prob = synth.cantilever(4, 2, 2)
    KE = fem.hex8_ke()
    for rho0 in (1.0, 0.5):
        rho = np.full(prob.n_elem, rho0)
        us, Cs, _ = sens.analyse(prob, rho, KE)
        K = fem.assemble(4, 2, 2, fem.simp(rho), KE)
        assert abs(us[0] @ (K @ us[0]) - Cs[0]) < 1e-12 * abs(Cs[0])
        if rho0 == 1.0:
            u1 = us[0]
        else:
            Eh = fem.simp(np.array([0.5]))[0]
            assert np.linalg.norm(us[0] - u1 / Eh) <= 1e-12 * np.linalg.norm(u1 / Eh)


def _complex_compliance(prob, rho_c, KE):
    Ee = fem.simp(rho_c)
    K = fem.assemble(prob.nx, prob.ny, prob.nz, Ee, KE).toarray()
    fixed = fem.fixed_dofs_aos(prob)
    free = fem.free_mask(K.shape[0], fixed)
    f = fem.dof_vector_aos(prob)[free]
    u = np.linalg.solve(K[np.ix_(free, free)], f.astype(complex))
    return f @ u


def test_sensitivity_complex_step():
    """eq. (6) against the complex-step derivative of C(rho~), exact to
    machine precision (no subtractive cancellation)."""
    prob = synth.cantilever(3, 2, 2)
    KE = fem.hex8_ke()
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.3, 1.0, prob.n_elem)
    _, _, dc = sens.analyse(prob, rho, KE)
    h = 1e-30
    for e in range(prob.n_elem):
        rc = rho.astype(complex)
        rc[e] += 1j * h
        d = _complex_compliance(prob, rc, KE).imag / h
        assert abs(d - dc[e]) <= 1e-12 * np.abs(dc).max()


def test_sensitivity_central_difference_two_cases():
    prob = synth.point_loads_on_face(3, 2, 2, n_case=2, seed=5)
    KE = fem.hex8_ke()
    rho = np.random.default_rng(4).uniform(0.3, 1.0, prob.n_elem)
    _, Cs, dc = sens.analyse(prob, rho, KE)
    e = 5
    h = 1e-6
    rp, rm = rho.copy(), rho.copy()
    rp[e] += h
    rm[e] -= h
    Cp = sum(sens.analyse(prob, rp, KE)[1])
    Cm = sum(sens.analyse(prob, rm, KE)[1])
    assert abs((Cp - Cm) / (2 * h) - dc[e]) < 1e-6 * abs(dc[e])


def test_vectorised_element_dofs_and_product_match_assembly():
    """The array-built element DOF table equals the loop-built one, and the
    element-by-element product equals the assembled K times v."""
    nx, ny, nz = 5, 3, 2
    assert np.array_equal(fem.element_dofs_grid(nx, ny, nz), fem.element_dofs(nx, ny, nz))
    rng = np.random.default_rng(19)
    Ee = rng.uniform(0.1, 1.0, nx * ny * nz)
    KE = fem.hex8_ke()
    v = rng.standard_normal(3 * (nx + 1) * (ny + 1) * (nz + 1))
    K = fem.assemble(nx, ny, nz, Ee, KE)
    y = fem.apply_ebe(nx, ny, nz, Ee, KE, v)
    assert np.abs(y - K @ v).max() <= 1e-14 * np.abs(K @ v).max()


def test_product_at_sampled_nodes_matches_assembly():
    """The row-by-row product at selected nodes (for sampled checks on large
    grids) equals the assembled K v at those nodes: every node of a small
    grid, so corners, edges, faces and interior nodes are all covered, with v
    given through an SoA lookup as the large-grid checks do."""
    nx, ny, nz = 4, 3, 5
    nn = (nx + 1) * (ny + 1) * (nz + 1)
    rng = np.random.default_rng(23)
    Ee = rng.uniform(0.1, 1.0, nx * ny * nz)
    KE = fem.hex8_ke()
    v = rng.standard_normal(3 * nn)
    want = (fem.assemble(nx, ny, nz, Ee, KE) @ v).reshape(-1, 3)
    v_soa = fem.aos_to_soa(v)
    got = fem.apply_ebe_at_nodes(nx, ny, nz, Ee, KE, lambda ids: v_soa[ids % 3, ids // 3],
                                 np.arange(nn))
    assert np.abs(got - want).max() <= 1e-14 * np.abs(want).max()


def test_point_loads_on_one_dof_add_up():
    """Two point loads listed on the same DOF act as one with the summed force."""
    import dataclasses

    prob = synth.cantilever(4, 2, 2)
    (i, j, k, c, v) = prob.loads[0][0]
    split = dataclasses.replace(prob, loads=[[(i, j, k, c, 0.3 * v), (i, j, k, c, 0.7 * v)]
                                             + list(prob.loads[0][1:])])
    assert np.allclose(fem.dof_vector_aos(split), fem.dof_vector_aos(prob), rtol=1e-15, atol=0)
