"""Pins of the oracle's density filter (eqs. 31-33) and of its multigrid
pieces (Algorithm 2) against counts, brute force and invariants."""

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import fem, filt, mg, solve


@pytest.mark.parametrize("r,key", [(1.5, "r1p5"), (2.0, "r2"), (2.5, "r2p5")])
def test_filter_interior_taps(gold, r, key):
    g = gold("filter_taps.txt")
    n = 7
    H, Hs = filt.filter_matrix(n, n, n, r)
    c = 3 + n * (3 + n * 3)  # centre element
    assert H[c].nnz == int(g["taps_" + key])
    if "wsum_" + key in g:
        assert abs(Hs[c] - g["wsum_" + key]) < 1e-13


@pytest.mark.parametrize("r", [1.5, 2.0, 2.5])
def test_filter_vs_brute_force(r):
    nx, ny, nz = 5, 4, 3
    rho = np.random.default_rng(0).uniform(0, 1, nx * ny * nz)
    H, Hs = filt.filter_matrix(nx, ny, nz, r)
    assert np.allclose(filt.forward(H, Hs, rho), filt.brute_force_forward(nx, ny, nz, r, rho),
                       rtol=1e-14, atol=1e-15)


def test_filter_uniform_and_adjoint():
    nx, ny, nz = 6, 5, 4
    H, Hs = filt.filter_matrix(nx, ny, nz, 2.5)
    n = nx * ny * nz
    assert np.allclose(filt.forward(H, Hs, np.full(n, 0.37)), 0.37, rtol=1e-15)
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    lhs = filt.forward(H, Hs, x) @ y
    rhs = x @ filt.adjoint(H, Hs, y)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def test_filter_symmetric_weights():
    H, _ = filt.filter_matrix(4, 3, 3, 2.0)
    assert abs(H - H.T).max() == 0.0


def test_prolongation_reproduces_linear_fields():
    """Trilinear interpolation is exact for (tri)linear fields."""
    ncx, ncy, ncz = 3, 2, 2
    P = mg.prolongation(ncx, ncy, ncz)

    def field(nx, ny, nz, h):
        v = np.zeros((nx + 1) * (ny + 1) * (nz + 1) * 3)
        for k in range(nz + 1):
            for j in range(ny + 1):
                for i in range(nx + 1):
                    x, y, z = i * h, j * h, k * h
                    n = fem.node_id(nx, ny, i, j, k)
                    v[3 * n:3 * n + 3] = (1 + 2 * x - y, 3 * z + x * y, x * y * z - z)
        return v

    assert np.allclose(P @ field(ncx, ncy, ncz, 2.0), field(2 * ncx, 2 * ncy, 2 * ncz, 1.0),
                       atol=1e-13)
    # columns sum to the number of fine nodes a coarse node reaches, weighted
    assert np.allclose(P.sum(axis=0).A.ravel().max(), 8.0)


def test_prolongation_kron_equals_node_loop():
    """The Kronecker-built interpolation is the node-loop one, entry for
    entry, on grids with unequal and odd/even extents."""
    for dims in ((1, 1, 1), (3, 2, 2), (2, 5, 3), (4, 1, 6)):
        A = mg.prolongation(*dims)
        B = mg.prolongation_kron(*dims)
        assert A.shape == B.shape
        assert abs(A - B).max() == 0.0
        assert A.nnz == B.nnz


def _setup(dims, levels, seed=0):
    prob = synth.cantilever(*dims)
    rho = np.random.default_rng(seed).uniform(0.3, 1.0, prob.n_elem)
    K = fem.assemble(*dims, fem.simp(rho), fem.hex8_ke())
    fixed = fem.fixed_dofs_aos(prob)
    return prob, K, fixed


def test_galerkin_operators_spd():
    prob, K, fixed = _setup((8, 4, 4), 3)
    H = mg.Hierarchy(K, fixed, (8, 4, 4), 3)
    for A in H.A:
        assert abs(A - A.T).max() < 1e-13
        assert np.linalg.eigvalsh(A.toarray()).min() > 0


def test_vcycle_symmetric():
    prob, K, fixed = _setup((8, 4, 4), 3)
    H = mg.Hierarchy(K, fixed, (8, 4, 4), 3)
    free = fem.free_mask(K.shape[0], fixed)
    rng = np.random.default_rng(2)
    x = rng.standard_normal(K.shape[0]) * free
    y = rng.standard_normal(K.shape[0]) * free
    a = H.vcycle(x) @ y
    b = x @ H.vcycle(y)
    assert abs(a - b) < 1e-12 * abs(a)


def test_two_level_exact_coarse_reduces_error():
    """Two levels, exact coarse solve: the V-cycle is a contraction on the
    error (spectral radius of I - M^-1 A below 1)."""
    prob, K, fixed = _setup((4, 2, 2), 2)
    H = mg.Hierarchy(K, fixed, (4, 2, 2), 2)
    A = H.A[0].toarray()
    n = A.shape[0]
    M = np.stack([H.vcycle(e) for e in np.eye(n)], axis=1)
    rho = np.abs(np.linalg.eigvals(np.eye(n) - M @ A)).max()
    assert rho < 1.0


def test_mgcg_matches_direct():
    dims = (8, 4, 4)
    prob, K, fixed = _setup(dims, 3, seed=4)
    f = fem.dof_vector_aos(prob)
    u_d = solve.solve_direct(K, f, fixed, dims)
    u, it, rel = mg.mgcg(K, f, fixed, dims, 3, rtol=1e-10)
    assert rel <= 1e-10
    assert np.linalg.norm(u - u_d) <= 1e-8 * np.linalg.norm(u_d)
    assert it < 100


def test_coarse_operators_are_the_energy_of_the_interpolated_field():
    """Algorithm 2's coarse operators, read physically: for a coarse vector v
    on level l, v^T A_l v is the strain energy sum_e E_e u_e^T KE u_e of the
    fine displacement u interpolated from v through every level and held at
    zero on the supports.  Checked on levels 1 and 2 of a 3-level hierarchy
    with element-by-element energies, not the matrix chain, so a coarse
    operator formed from the wrong level or an interpolation that ignores
    the supports fails it."""
    dims = (8, 4, 4)
    prob, K, fixed = _setup(dims, 3, seed=6)
    H = mg.Hierarchy(K, fixed, dims, 3)
    rng = np.random.default_rng(6)
    rho = np.random.default_rng(6).uniform(0.3, 1.0, prob.n_elem)
    Ee = fem.simp(rho)
    edof = fem.element_dofs(*dims)
    KE = fem.hex8_ke()
    free = fem.free_mask(K.shape[0], fixed)
    for level in (1, 2):
        Ps = [mg.prolongation(dims[0] >> k, dims[1] >> k, dims[2] >> k) for k in range(1, level + 1)]
        v = rng.standard_normal(Ps[-1].shape[1])
        u = v
        for P in reversed(Ps):
            u = P @ u
        u = np.where(free, u, 0.0)
        energy = float((Ee * np.einsum("ei,ij,ej->e", u[edof], KE, u[edof])).sum())
        assert abs(v @ (H.A[level] @ v) - energy) <= 1e-12 * energy, f"level {level}"
