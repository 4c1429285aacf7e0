"""GPU parity of every kernel family and of the full analysis step against
the CPU FP64 oracle, through the C ABI.  Tolerances: building blocks to
1e-12 relative (FP64, different summation order); converged solves to the
1e-6 compliance / displacement / sensitivity bar."""

import numpy as np
import pytest
import torch

import synth
from oracle import ca as oca
from oracle import fem, filt, mg, oc, sens, solve

from gpu_util import aos, fixed_tensor, loads_tensor, log, mesh_for, rel, soa, t64

pytestmark = pytest.mark.gpu

SIZES = [(2, 2, 2, 2), (8, 4, 4, 3), (18, 10, 6, 2), (24, 12, 12, 3), (36, 20, 12, 3)]


def _density(prob, seed, lo=0.3, hi=1.0):
    return synth.uniform_iid(prob.nx, prob.ny, prob.nz, lo, hi, seed).ravel()


@pytest.mark.parametrize("nx,ny,nz,lev", SIZES)
def test_operator_apply_matches_assembled(nx, ny, nz, lev):
    log(f"operator apply {nx}x{ny}x{nz}")
    prob = synth.cantilever(nx, ny, nz)
    rho = _density(prob, 11)
    m = mesh_for(prob, mg_levels=lev)
    fixed = fixed_tensor(prob, m)
    m.setup(t64(rho), fixed)
    v = np.random.default_rng(12).standard_normal(3 * m.n_node)
    y = torch.zeros(3 * m.n_node, dtype=torch.float64, device="cuda")
    m.apply(t64(v), y)
    K = fem.assemble(nx, ny, nz, fem.simp(rho), fem.hex8_ke())
    A = fem.operator_with_bc(K, fem.fixed_dofs_aos(prob))
    want = soa(A @ aos(v))
    assert rel(y.cpu().numpy(), want) < 1e-13
    # the solver-internal form: input zero on fixed DOFs, no masking on load
    from paper_2205_00385_amd import aarmr

    vm = aos(v)
    vm[fem.fixed_dofs_aos(prob)] = 0.0
    m.apply(t64(soa(vm)), y, flags=aarmr.INPUT_MASKED)
    assert rel(y.cpu().numpy(), soa(A @ vm)) < 1e-13


def test_operator_apply_is_deterministic():
    prob = synth.cantilever(24, 12, 12)
    m = mesh_for(prob)
    m.setup(t64(_density(prob, 1)), fixed_tensor(prob, m))
    v = t64(np.random.default_rng(0).standard_normal(3 * m.n_node))
    y1 = torch.empty_like(v)
    y2 = torch.empty_like(v)
    m.apply(v, y1)
    m.apply(v, y2)
    assert torch.equal(y1, y2)


# (32, 16, 16, 2): a 4131-DOF coarsest level, 65 Gauss-Jordan block rows,
# which the inverse runs as separate cross and tile launches; (40, 20, 20, 2):
# 7623 DOFs, near the 8192-DOF limit of the dense coarsest inverse
@pytest.mark.parametrize("nx,ny,nz,lev", [(8, 4, 4, 3), (24, 12, 12, 3), (16, 8, 8, 4), (48, 24, 24, 3),
                                          (32, 16, 16, 2), (40, 20, 20, 2)])
def test_coarse_operators_and_vcycle(nx, ny, nz, lev):
    log(f"coarse ops / vcycle {nx}x{ny}x{nz} levels={lev}")
    prob = synth.cantilever(nx, ny, nz)
    rho = _density(prob, 21)
    m = mesh_for(prob, mg_levels=lev)
    m.setup(t64(rho), fixed_tensor(prob, m))
    K = fem.assemble(nx, ny, nz, fem.simp(rho), fem.hex8_ke())
    H = mg.Hierarchy(K, fem.fixed_dofs_aos(prob), (nx, ny, nz), lev)
    rng = np.random.default_rng(22)
    for l in range(1, lev):
        nn = (nx // 2 ** l + 1) * (ny // 2 ** l + 1) * (nz // 2 ** l + 1)
        v = rng.standard_normal(3 * nn)
        y = torch.zeros(3 * nn, dtype=torch.float64, device="cuda")
        m.apply(t64(v), y, level=l)
        want = soa(H.A[l] @ aos(v))
        assert rel(y.cpu().numpy(), want) < 1e-12, f"level {l}"
    free = fem.free_mask(K.shape[0], fem.fixed_dofs_aos(prob))
    r = rng.standard_normal(K.shape[0]) * free
    z = torch.zeros(K.shape[0], dtype=torch.float64, device="cuda")
    m.vcycle(t64(soa(r)), z)
    want = soa(H.vcycle(r, omega=0.6, nu1=1, nu2=1))
    assert rel(z.cpu().numpy(), want) < 1e-9


def test_coarse_galerkin_eight_parent_groups():
    """Levels >= 2 with at least 256 groups of 8 parents along x are built 8
    parents per workgroup.  At 48x64x64 with 4 levels, level 2 (12x16x16) has
    512 such groups, half of them partial (12 = 8 + 4 parents per row), while
    level 3 (6x8x8) is built one parent per workgroup.  Each is checked against
    Algorithm 2's coarse operators composed on the oracle's side alone:
    A_l = Q^T Df K Df Q with Q = P_1 ... P_l the oracle's trilinear
    interpolations and K the oracle's element-by-element product."""
    nx, ny, nz = 48, 64, 64
    log(f"coarse galerkin groups {nx}x{ny}x{nz} levels=4")
    prob = synth.cantilever(nx, ny, nz)
    m = mesh_for(prob, mg_levels=4)
    rho = _density(prob, 23)
    m.setup(t64(rho), fixed_tensor(prob, m))
    free = fem.free_mask(3 * m.n_node, fem.fixed_dofs_aos(prob)).astype(np.float64)
    Ee, KE = fem.simp(rho), fem.hex8_ke()
    edof = fem.element_dofs_grid(nx, ny, nz)
    rng = np.random.default_rng(24)
    for l in (2, 3):
        Ps = [mg.prolongation_kron(nx >> k, ny >> k, nz >> k) for k in range(1, l + 1)]
        v = rng.standard_normal(Ps[-1].shape[1])
        x = v
        for P in reversed(Ps):  # Q v = P_1 (P_2 ( ... P_l v))
            x = P @ x
        y = free * fem.apply_ebe(nx, ny, nz, Ee, KE, free * x, edof)
        for P in Ps:  # Q^T y
            y = P.T @ y
        got = torch.zeros(Ps[-1].shape[1], dtype=torch.float64, device="cuda")
        m.apply(t64(soa(v)), got, level=l)
        err = rel(aos(got.cpu().numpy()), y)
        log(f"  level {l}: rel {err:.2e}")
        assert err < 1e-12, f"level {l}"


def test_energy_matches_oracle():
    prob = synth.cantilever(18, 10, 6)
    m = mesh_for(prob, mg_levels=2)
    m.setup(t64(_density(prob, 3)), fixed_tensor(prob, m))
    u = np.random.default_rng(4).standard_normal(3 * m.n_node)
    e = torch.zeros(m.n_elem, dtype=torch.float64, device="cuda")
    m.element_energy(t64(u), e)
    ua = aos(u)
    ua[fem.fixed_dofs_aos(prob)] = 0.0
    want = sens.element_energy(ua, fem.element_dofs(18, 10, 6), fem.hex8_ke())
    assert rel(e.cpu().numpy(), want) < 1e-13


@pytest.mark.parametrize("r", [1.5, 2.0, 2.5])
@pytest.mark.parametrize("dims", [(6, 4, 2), (18, 10, 6)])
def test_filter_matches_oracle(r, dims):
    nx, ny, nz = dims
    prob = synth.cantilever(nx, ny, nz)
    m = mesh_for(prob, mg_levels=2, rmin=r)
    x = np.random.default_rng(5).uniform(0, 1, m.n_elem)
    H, Hs = filt.filter_matrix(nx, ny, nz, r)
    out = torch.zeros(m.n_elem, dtype=torch.float64, device="cuda")
    m.filter(t64(x), out, mode=0)
    assert rel(out.cpu().numpy(), filt.forward(H, Hs, x)) < 1e-14
    m.filter(t64(x), out, mode=1)
    assert rel(out.cpu().numpy(), filt.adjoint(H, Hs, x)) < 1e-14


def test_solve_cantilever24_matches_direct():
    """The 24x12x12 cantilever: design density U[0.3,1] (seed 1), filter
    r=1.5, 3 levels; u, C and dC/drho against the direct solve."""
    nx, ny, nz = 24, 12, 12
    log("solve cantilever24")
    prob = synth.cantilever(nx, ny, nz)
    x = synth.uniform_iid(nx, ny, nz, 0.3, 1.0, seed=1).ravel()
    from paper_2205_00385_amd import aarmr

    m = mesh_for(prob, mg_levels=3, rmin=1.5, cg_rtol=1e-10)
    fixed = fixed_tensor(prob, m)
    f = loads_tensor(prob, m)
    u = torch.zeros_like(f)
    dc = torch.zeros(m.n_elem, dtype=torch.float64, device="cuda")
    C, st, code = m.solve(t64(x), f, fixed, u, dc=dc, flags=aarmr.FILTER_INPUT)
    H, Hs = filt.filter_matrix(nx, ny, nz, 1.5)
    xphys = filt.forward(H, Hs, x)
    us, Cs, dcp = sens.analyse(prob, xphys)
    log(f"  its={st.iterations[0]} rel={st.rel_residual[0]:.2e} C={C[0]:.12g} ref={Cs[0]:.12g}")
    assert code == aarmr.OK and st.rel_residual[0] <= 1e-10
    assert abs(C[0] - Cs[0]) <= 1e-6 * abs(Cs[0])
    assert rel(u.cpu().numpy(), soa(us[0])) <= 1e-6
    assert rel(dc.cpu().numpy(), filt.adjoint(H, Hs, dcp)) <= 1e-6


def test_solve_multi_case_and_warm_start():
    prob = synth.point_loads_on_face(16, 8, 8, n_case=3, seed=7)
    from paper_2205_00385_amd import aarmr

    m = mesh_for(prob, mg_levels=3, cg_rtol=1e-10, n_rhs_max=4)
    rho = synth.smoothed_field(16, 8, 8, 2.0, 1e-3, 1.0, seed=8).ravel()
    fixed = fixed_tensor(prob, m)
    f = loads_tensor(prob, m)
    u = torch.zeros_like(f)
    dc = torch.zeros(m.n_elem, dtype=torch.float64, device="cuda")
    C, st, code = m.solve(t64(rho), f, fixed, u, dc=dc)
    us, Cs, dcs = sens.analyse(prob, rho)
    n3 = 3 * m.n_node
    for l in range(3):
        assert abs(C[l] - Cs[l]) <= 1e-6 * abs(Cs[l])
        assert rel(u[l * n3:(l + 1) * n3].cpu().numpy(), soa(us[l])) <= 1e-6
    assert rel(dc.cpu().numpy(), dcs) <= 1e-6
    # warm start from the converged solution: no iteration needed
    C2, st2, _ = m.solve(t64(rho), f, fixed, u, flags=aarmr.WARM_START)
    assert all(st2.iterations[l] <= 1 for l in range(3))


def test_solve_bridge_high_contrast():
    """Simply supported beam (four bottom corners fixed, centre load) on a
    thresholded field {1e-3, 1}: MGCG must still reach the oracle."""
    prob = synth.bridge(16, 8, 8)
    m = mesh_for(prob, mg_levels=3, cg_rtol=1e-10)
    rho = synth.thresholded_field(16, 8, 8, 2.0, 1e-3, 1.0, seed=9).ravel()
    f = loads_tensor(prob, m)
    u = torch.zeros_like(f)
    C, st, code = m.solve(t64(rho), f, fixed_tensor(prob, m), u)
    us, Cs, _ = sens.analyse(prob, rho)
    log(f"  bridge its={st.iterations[0]} C={C[0]:.10g} ref={Cs[0]:.10g}")
    assert abs(C[0] - Cs[0]) <= 1e-6 * abs(Cs[0])
    assert rel(u.cpu().numpy(), soa(us[0])) <= 1e-6


def test_invalid_inputs_rejected():
    from paper_2205_00385_amd import aarmr

    prob = synth.cantilever(8, 4, 4)
    m = mesh_for(prob, mg_levels=2)
    fixed = fixed_tensor(prob, m)
    f = loads_tensor(prob, m)
    u = torch.zeros_like(f)
    bad = t64(np.full(m.n_elem, 1.5))
    with pytest.raises(aarmr.AarmrError) as ei:
        m.solve(bad, f, fixed, u)
    assert ei.value.code == aarmr.E_INVALID
    badfix = torch.tensor([3 * m.n_node + 5], dtype=torch.int64, device="cuda")
    with pytest.raises(aarmr.AarmrError) as ei:
        m.solve(t64(np.full(m.n_elem, 0.5)), f, badfix, u)
    assert ei.value.code == aarmr.E_INVALID
    with pytest.raises(aarmr.AarmrError) as ei:
        m.ca_update(t64(np.full(m.n_elem, 0.5)), f, fixed, u)
    assert ei.value.code == aarmr.E_STATE


def test_not_converged_reports_and_writes():
    from paper_2205_00385_amd import aarmr

    prob = synth.cantilever(16, 8, 8)
    m = mesh_for(prob, mg_levels=3, cg_maxit=2)
    f = loads_tensor(prob, m)
    u = torch.zeros_like(f)
    C, st, code = m.solve(t64(np.full(m.n_elem, 0.7)), f, fixed_tensor(prob, m), u)
    assert code == aarmr.E_NOT_CONVERGED
    assert st.iterations[0] == 2 and st.rel_residual[0] > 1e-8
    assert torch.isfinite(u).all() and float(u.abs().max()) > 0
    # the message names the smoother condition a stalled solve may be breaking
    assert "omega" in aarmr.lib().aarmr_last_error().decode()


@pytest.mark.parametrize("orth,form", [("gs", "fp64"), ("svd", "fp64"), ("gs", "refine")])
def test_ca_sequence_matches_oracle_algorithm1(orth, form):
    """Algorithm 1 on both sides over the same density sequence: N_on exact
    (oracle) / converged MGCG (GPU) cycles build the PARM, then CA cycles.
    The accept/reject path, u, C and dc must agree.  The oracle
    orthogonalises by eq. 21's SVD; the GPU by Gram-Schmidt or by the same
    SVD (rank of the kept basis compared too).  In the refinement form the
    MGCG solves that fill the PARM and the fallbacks run in FP32 inside FP64
    refinement, while the reduced model itself stays FP64."""
    from paper_2205_00385_amd import aarmr

    prob = synth.cantilever(16, 8, 8)
    Ns, Nm, N_on, tol = 2, 3, 3, 0.05
    alg = oca.AARMR(prob, Ns=Ns, Nm=Nm, N_on=N_on, eps_tol=tol)
    m = mesh_for(prob, mg_levels=3, cg_rtol=1e-11, Ns=Ns, Nm=Nm, ca_tol=tol,
                 orth=aarmr.ORTH_SVD if orth == "svd" else aarmr.ORTH_GS,
                 precision=aarmr.FP32_REFINE if form == "refine" else aarmr.FP64)
    fixed = fixed_tensor(prob, m)
    f = loads_tensor(prob, m)
    u = torch.zeros_like(f)
    dc = torch.zeros(m.n_elem, dtype=torch.float64, device="cuda")
    base = synth.smoothed_field(16, 8, 8, 2.0, 0.2, 1.0, seed=30).ravel()
    d = synth.smoothed_field(16, 8, 8, 3.0, -1.0, 1.0, seed=32).ravel()
    edof = fem.element_dofs(16, 8, 8)
    KE = fem.hex8_ke()
    paths = []
    for loop in range(1, 10):
        # a smooth drift whose step grows: both CA acceptance and fallback occur
        rho = np.clip(base + 0.02 * loop * d + 4e-4 * loop ** 2 * np.roll(d, 7), 0.05, 1.0)
        (u_ref, path, eps_ref, rank_ref), = alg.cycle(loop, rho)
        if loop <= N_on:
            flags = aarmr.WARM_START | (aarmr.RECORD_PARM if loop > N_on - Ns else 0)
            C, st, _ = m.solve(t64(rho), f, fixed, u, dc=dc, flags=flags)
            gpath = "mgcg"
        else:
            C, st, _ = m.ca_update(t64(rho), f, fixed, u, dc=dc)
            gpath = "ca" if st.accepted[0] else "fallback"
            log(f"  loop {loop}: eps gpu={st.eps[0]:.6e} oracle={eps_ref:.6e} rank {st.rank[0]}/{rank_ref}")
            if abs(st.eps[0] - tol) > 1e-6 * tol:
                assert gpath == path
            assert abs(st.eps[0] - eps_ref) <= 1e-6 * max(eps_ref, 1e-12) + 1e-9
            if orth == "svd":
                assert st.rank[0] == rank_ref
        paths.append(gpath)
        assert rel(u.cpu().numpy(), soa(u_ref)) <= 1e-6
        Cref = float(alg.f[0] @ u_ref)
        assert abs(C[0] - Cref) <= 1e-6 * abs(Cref)
        dref = sens.dc_drho_phys(rho, sens.element_energy(u_ref, edof, KE))
        assert rel(dc.cpu().numpy(), dref) <= 1e-6
    log(f"  paths {paths}")
    assert "ca" in paths and "fallback" in paths


def test_oc_update_matches_oracle():
    nx, ny, nz = 12, 8, 6
    prob = synth.cantilever(nx, ny, nz)
    m = mesh_for(prob, mg_levels=2, rmin=2.0)
    H, Hs = filt.filter_matrix(nx, ny, nz, 2.0)
    rng = np.random.default_rng(41)
    x = rng.uniform(0.1, 0.9, m.n_elem)
    dc = -rng.uniform(0.01, 3.0, m.n_elem)
    dv = filt.adjoint(H, Hs, np.ones(m.n_elem))
    xn, xp, lam = oc.oc_update(x, dc, dv, H, Hs, 0.3)
    gx = torch.zeros(m.n_elem, dtype=torch.float64, device="cuda")
    gp = torch.zeros_like(gx)
    m.oc_update(t64(x), t64(dc), t64(dv), 0.3, 0.2, gx, gp)
    assert rel(gx.cpu().numpy(), xn) < 1e-9
    assert rel(gp.cpu().numpy(), xp) < 1e-9


def test_level1_many_fixed_parents_strided_path():
    """Three fully fixed faces on a 64x32x32 grid flag more level-1 parents
    than the compact copy holds (1024), so the level-1 product reads the
    flagged parents' matrices in place; level 1 and the V-cycle against the
    oracle's sparse Galerkin hierarchy."""
    nx, ny, nz, lev = 64, 32, 32, 3
    base = synth.cantilever(nx, ny, nz)
    fixed = set()
    for i in range(nx + 1):
        for j in range(ny + 1):
            for c in range(3):
                fixed.add((i, j, 0, c))
    for j in range(ny + 1):
        for k in range(nz + 1):
            for c in range(3):
                fixed.add((0, j, k, c))
    for i in range(nx + 1):
        for k in range(nz + 1):
            fixed.add((i, 0, k, 1))
    prob = synth.problems.Problem(nx, ny, nz, sorted(fixed), base.loads, "three faces")
    rho = _density(prob, 31)
    m = mesh_for(prob, mg_levels=lev)
    m.setup(t64(rho), fixed_tensor(prob, m))
    K = fem.assemble(nx, ny, nz, fem.simp(rho), fem.hex8_ke())
    H = mg.Hierarchy(K, fem.fixed_dofs_aos(prob), (nx, ny, nz), lev)
    rng = np.random.default_rng(32)
    nn1 = (nx // 2 + 1) * (ny // 2 + 1) * (nz // 2 + 1)
    v = rng.standard_normal(3 * nn1)
    y = torch.zeros(3 * nn1, dtype=torch.float64, device="cuda")
    m.apply(t64(v), y, level=1)
    assert rel(y.cpu().numpy(), soa(H.A[1] @ aos(v))) < 1e-12
    free = fem.free_mask(K.shape[0], fem.fixed_dofs_aos(prob))
    r = rng.standard_normal(K.shape[0]) * free
    z = torch.zeros(K.shape[0], dtype=torch.float64, device="cuda")
    m.vcycle(t64(soa(r)), z)
    assert rel(z.cpu().numpy(), soa(H.vcycle(r, omega=0.6, nu1=1, nu2=1))) < 1e-9


@pytest.mark.parametrize("dims", [(24, 12, 12), (36, 20, 40)])
def test_autotune_keeps_products_bitwise(dims):
    """The autotuner only changes the z-chunk length of the fine-grid
    operator.  Every chunk length (the tuned one and 2, 3, 5, 7 and all
    planes set explicitly) gives the same bits for the product and for a
    V-cycle; a solve, whose CG dot products are summed per workgroup of the
    product, agrees to rounding (1e-10)."""
    from paper_2205_00385_amd import aarmr

    prob = synth.cantilever(*dims)
    for prec in (aarmr.FP64, aarmr.FP32_REFINE):
        m = mesh_for(prob, mg_levels=3, precision=prec)
        fixed = fixed_tensor(prob, m)
        rho = t64(_density(prob, 41))
        m.setup(rho, fixed)
        v = np.random.default_rng(42).standard_normal(3 * m.n_node)
        y0 = torch.empty(3 * m.n_node, dtype=torch.float64, device="cuda")
        m.apply(t64(v), y0)
        z0 = torch.empty_like(y0)
        r = t64(v * fem.aos_to_soa(fem.free_mask(3 * m.n_node, fem.fixed_dofs_aos(prob))
                                   .astype(np.float64)).ravel())
        m.vcycle(r, z0)
        f = loads_tensor(prob, m)
        u0 = torch.zeros_like(f)
        C0, st0, _ = m.solve(rho, f, fixed, u0)
        tuned = m.autotune()
        log(f"  {dims} precision {prec}: tuned chunk lengths {tuned}")
        # chunk lengths, then tile heights (shape word: rows << 16 | chunk)
        for tz in (None, 2, 3, 5, 7, prob.nz + 1, 8 << 16, 12 << 16, (16 << 16) | 3,
                   (12 << 16) | 2):
            if tz is not None:
                m.set_chunk(tz, tz)
            y1 = torch.empty_like(y0)
            m.apply(t64(v), y1)
            assert torch.equal(y0, y1), f"product, chunk {tz}"
            z1 = torch.empty_like(z0)
            m.vcycle(r, z1)
            assert torch.equal(z0, z1), f"V-cycle, chunk {tz}"
            u1 = torch.zeros_like(f)
            C1, st1, _ = m.solve(rho, f, fixed, u1)
            assert rel(u1.cpu().numpy(), u0.cpu().numpy()) < 1e-10, f"solve, chunk {tz}"
            assert abs(C1[0] - C0[0]) <= 1e-10 * abs(C0[0])
            # the iteration count is not compared: on this slowly converging
            # case (hundreds of iterations) rounding alone moves it
            log(f"    chunk {tz}: {st1.iterations[0]} iterations (default {st0.iterations[0]})")
        with pytest.raises(aarmr.AarmrError):
            m.set_chunk(1, 0)
        with pytest.raises(aarmr.AarmrError):
            m.set_chunk(10 << 16, 0)
        m.close()


def test_rejected_reduced_model_runs_beside_speculative_hierarchy():
    """Three reduced-model steps in a row that are all rejected (ca_tol
    1e-12): from the second on, the MG hierarchy of the new design is built on
    a second stream while the reduced model runs.  Every fallback solution,
    compliance and sensitivity must still be the direct solve's, and the
    reported rank and eps must agree (1e-6) with a fresh mesh taken through
    the same history, whose reduced-model step is its first and so builds
    the hierarchy only after the rejection."""
    from paper_2205_00385_amd import aarmr

    prob = synth.cantilever(16, 8, 8)
    Ns, Nm = 2, 3
    kw = dict(mg_levels=3, cg_rtol=1e-11, Ns=Ns, Nm=Nm, ca_tol=1e-12)
    m = mesh_for(prob, **kw)
    fixed = fixed_tensor(prob, m)
    f = loads_tensor(prob, m)
    base = synth.smoothed_field(16, 8, 8, 2.0, 0.2, 1.0, seed=60).ravel()
    d = synth.smoothed_field(16, 8, 8, 3.0, -1.0, 1.0, seed=61).ravel()
    designs = [np.clip(base + 0.03 * k * d, 0.05, 1.0) for k in range(6)]
    edof = fem.element_dofs(16, 8, 8)
    u = torch.zeros_like(f)
    dc = torch.zeros(m.n_elem, dtype=torch.float64, device="cuda")
    for k in range(Ns):
        m.solve(t64(designs[k]), f, fixed, u, flags=aarmr.RECORD_PARM | (aarmr.WARM_START if k else 0))
    for k in range(Ns, 6):
        rho = designs[k]
        # reference: a fresh mesh taken through the same history, its step not speculative
        # (PARM = the last Ns solutions, reference design k - 1, u_last = m's u)
        m2 = mesh_for(prob, **kw)
        u2 = torch.zeros_like(f)
        for j in range(k):
            m2.solve(t64(designs[j]), f, fixed, u2,
                     flags=aarmr.WARM_START | (aarmr.RECORD_PARM if j >= k - Ns else 0))
        u2.copy_(u)
        C2, st2, _ = m2.ca_update(t64(rho), f, fixed, u2)
        m2.close()
        C, st, code = m.ca_update(t64(rho), f, fixed, u, dc=dc)
        assert code == aarmr.OK and st.accepted[0] == 0
        log(f"  step {k}: eps {st.eps[0]:.3e} rank {st.rank[0]}, fallback {st.mgcg_iterations[0]} it")
        (u_ref,), (C_ref,), dc_ref = sens.analyse(prob, rho)
        assert rel(u.cpu().numpy(), soa(u_ref)) < 1e-8
        assert abs(C[0] - C_ref) <= 1e-8 * abs(C_ref)
        assert rel(dc.cpu().numpy(), dc_ref) < 1e-7
        assert st.rank[0] == st2.rank[0]
        assert abs(st.eps[0] - st2.eps[0]) <= 1e-6 * st2.eps[0]
    m.close()


def test_ca_svd_and_gs_bases_give_same_reduced_solution():
    """Nm > Ns + 1 (dependent CARM columns): the SVD and the Gram-Schmidt
    bases span the same space, so the reduced solution and eps agree."""
    from paper_2205_00385_amd import aarmr

    prob = synth.cantilever(16, 8, 8)
    out = {}
    for orth in (aarmr.ORTH_GS, aarmr.ORTH_SVD):
        m = mesh_for(prob, mg_levels=3, cg_rtol=1e-11, Ns=2, Nm=6, ca_tol=1.0, orth=orth)
        fixed = fixed_tensor(prob, m)
        f = loads_tensor(prob, m)
        u = torch.zeros_like(f)
        base = synth.smoothed_field(16, 8, 8, 2.0, 0.2, 1.0, seed=50).ravel()
        for k in range(2):
            m.solve(t64(np.clip(base + 0.01 * k, 0, 1)), f, fixed, u,
                    flags=aarmr.RECORD_PARM | aarmr.WARM_START)
        C, st, _ = m.ca_update(t64(np.clip(base + 0.03, 0, 1)), f, fixed, u)
        assert st.accepted[0] == 1
        out[orth] = (u.cpu().numpy(), st.eps[0], st.rank[0])
        log(f"  orth {orth}: eps {st.eps[0]:.6e} rank {st.rank[0]}")
    (ug, eg, rg), (us, es, rs) = out[aarmr.ORTH_GS], out[aarmr.ORTH_SVD]
    assert rg == rs
    assert rel(us, ug) <= 1e-9
    assert abs(es - eg) <= 1e-9 * max(eg, 1e-12) + 1e-12


@pytest.mark.parametrize("form", ["fp64", "refine"])
def test_ca_nm6_accepted_branch_48x24x24(form):
    """Algorithm 1 with the benchmark loop's basis size (Nm = 6, Ns = 2) on a
    48x24x24 cantilever: the GPU's reduced-model steps against the oracle's
    (eq. 21's SVD basis, exact solves for the PARM and the fallback).  Small
    smooth design steps first, so the accepted branch (eps < 1%, the paper's
    3D range) is taken, then larger ones until a fallback occurs.  Also in the
    refinement form (the PARM's and the fallback's solves in FP32 inside FP64
    refinement)."""
    from paper_2205_00385_amd import aarmr

    dims = (48, 24, 24)
    prob = synth.cantilever(*dims)
    Ns, Nm, N_on, tol = 2, 6, 2, 1e-2
    alg = oca.AARMR(prob, Ns=Ns, Nm=Nm, N_on=N_on, eps_tol=tol)
    m = mesh_for(prob, mg_levels=4, cg_rtol=1e-11, Ns=Ns, Nm=Nm, ca_tol=tol,
                 precision=aarmr.FP32_REFINE if form == "refine" else aarmr.FP64)
    fixed = fixed_tensor(prob, m)
    f = loads_tensor(prob, m)
    u = torch.zeros_like(f)
    dc = torch.zeros(m.n_elem, dtype=torch.float64, device="cuda")
    base = synth.smoothed_field(*dims, 3.0, 0.2, 1.0, seed=70).ravel()
    d = synth.smoothed_field(*dims, 4.0, -1.0, 1.0, seed=71).ravel()
    edof = fem.element_dofs(*dims)
    KE = fem.hex8_ke()
    steps = [0.0, 0.002, 0.004, 0.006, 0.008, 0.03, 0.15]
    paths = []
    for loop, amp in enumerate(steps, start=1):
        rho = np.clip(base + amp * d, 0.05, 1.0)
        log(f"  Nm=6 loop {loop} ({dims}, step {amp})")
        (u_ref, path, eps_ref, rank_ref), = alg.cycle(loop, rho)
        if loop <= N_on:
            flags = aarmr.WARM_START | (aarmr.RECORD_PARM if loop > N_on - Ns else 0)
            C, st, _ = m.solve(t64(rho), f, fixed, u, dc=dc, flags=flags)
            gpath = "mgcg"
        else:
            C, st, _ = m.ca_update(t64(rho), f, fixed, u, dc=dc)
            gpath = "ca" if st.accepted[0] else "fallback"
            log(f"    eps gpu={st.eps[0]:.6e} oracle={eps_ref:.6e} rank {st.rank[0]}/{rank_ref}")
            if abs(st.eps[0] - tol) > 1e-6 * tol:
                assert gpath == path
            assert abs(st.eps[0] - eps_ref) <= 1e-6 * max(eps_ref, 1e-12) + 1e-9
        paths.append(gpath)
        assert rel(u.cpu().numpy(), soa(u_ref)) <= 1e-6
        Cref = float(alg.f[0] @ u_ref)
        assert abs(C[0] - Cref) <= 1e-6 * abs(Cref)
        dref = sens.dc_drho_phys(rho, sens.element_energy(u_ref, edof, KE))
        assert rel(dc.cpu().numpy(), dref) <= 1e-6
    log(f"  paths {paths}")
    assert paths.count("ca") >= 2 and "fallback" in paths
    m.close()
