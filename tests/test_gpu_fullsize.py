"""Checks at the full sizes of the benchmark, in the launch configuration
bench.py times: the 96x48x48 loop mesh (4 levels, autotuned fine-grid
operator) and the 256x128x128 precision-form mesh.  The oracle cannot
factor these, so the checks are the product itself against the oracle's
element-by-element definition (every output), and for solves the residual
certificate ||f - A u|| / ||f|| computed by the oracle, the energy identity
f^T u = u^T A u and the sensitivity from the oracle's element energies."""

import numpy as np
import pytest
import torch

import synth
from oracle import fem, sens

from gpu_util import log, t64

pytestmark = pytest.mark.gpu


def _aarmr():
    from paper_2205_00385_amd import aarmr

    return aarmr


def _mesh(prob, autotune=True, **kw):
    aarmr = _aarmr()
    m = aarmr.Mesh(aarmr.default_params(nx=prob.nx, ny=prob.ny, nz=prob.nz, **kw))
    if autotune:
        m.autotune()
    return m


def _fixed(prob, m):
    aarmr = _aarmr()
    return torch.tensor(aarmr.fixed_dofs_soa(prob, m.n_node), dtype=torch.int64, device="cuda")


def _op_oracle(prob, Ee, v_aos, fixed_aos, edof):
    """A v = Df K Df v + (I - Df) v by the element-by-element definition."""
    vm = v_aos.copy()
    vm[fixed_aos] = 0.0
    y = fem.apply_ebe(prob.nx, prob.ny, prob.nz, Ee, fem.hex8_ke(), vm, edof)
    y[fixed_aos] = v_aos[fixed_aos]
    return y


def _soa(v):
    return fem.aos_to_soa(v).ravel()


def _aos(v):
    return fem.soa_to_aos(np.asarray(v))


# the loop mesh as timed: rmin 2, Ns 2, Nm 6, CA tolerance 1e-3, autotuned
LOOP = dict(mg_levels=4, cg_rtol=1e-8, cg_maxit=2000, rmin=2.0, Ns=2, Nm=6, ca_tol=1e-3)


@pytest.mark.parametrize("dims,kw,tune,seed", [((96, 48, 48), LOOP, True, 3),
                                              ((256, 128, 128), dict(mg_levels=6), False, 3)])
def test_fine_operator_full_size_every_output(dims, kw, tune, seed):
    """Every output of the fine-grid product on the loop mesh (autotuned
    chunk, as timed) and on the 256x128x128 roofline mesh, smoothed random
    moduli in [1e-3, 1], both the solver form (input zero on fixed DOFs) and
    the general form."""
    aarmr = _aarmr()
    log(f"full-size K.v {dims}")
    prob = synth.cantilever(*dims)
    m = _mesh(prob, autotune=tune, **kw)
    rho = synth.smoothed_field(*dims, 8.0, 1e-3, 1.0, seed=seed).ravel()
    fx = _fixed(prob, m)
    m.setup(t64(rho), fx)
    fixed_aos = fem.fixed_dofs_aos(prob)
    rng = np.random.default_rng(seed + 100)
    v = rng.standard_normal(3 * m.n_node)
    edof = fem.element_dofs_grid(*dims)
    want = _op_oracle(prob, fem.simp(rho), v, fixed_aos, edof)
    y = torch.empty(3 * m.n_node, dtype=torch.float64, device="cuda")
    m.apply(t64(_soa(v)), y)
    err = np.abs(_aos(y.cpu().numpy()) - want).max() / np.abs(want).max()
    log(f"  general form max rel err {err:.2e}")
    assert err < 1e-13
    vm = v.copy()
    vm[fixed_aos] = 0.0
    m.apply(t64(_soa(vm)), y, flags=aarmr.INPUT_MASKED)
    want_m = _op_oracle(prob, fem.simp(rho), vm, fixed_aos, edof)
    err = np.abs(_aos(y.cpu().numpy()) - want_m).max() / np.abs(want_m).max()
    log(f"  solver form max rel err {err:.2e}")
    assert err < 1e-13
    m.close()


def test_loop_mesh_solve_certificate_energy_and_sensitivity():
    """One analysis on the 96x48x48 loop mesh (4 levels, rel. residual 1e-8,
    smoothed random design): the oracle's residual meets the tolerance,
    f^T u = u^T A u, and dc equals the oracle's eq. 6 from the same u."""
    aarmr = _aarmr()
    dims = (96, 48, 48)
    prob = synth.cantilever(*dims)
    m = _mesh(prob, **LOOP)
    rho = synth.smoothed_field(*dims, 4.0, 0.05, 1.0, seed=7).ravel()
    fx = _fixed(prob, m)
    f = t64(np.asarray(aarmr.loads_soa(prob, m.n_node)[0]))
    u = torch.zeros_like(f)
    dc = torch.zeros(m.n_elem, dtype=torch.float64, device="cuda")
    C, st, code = m.solve(t64(rho), f, fx, u, dc=dc)
    assert code == aarmr.OK
    fixed_aos = fem.fixed_dofs_aos(prob)
    ua = _aos(u.cpu().numpy())
    fa = fem.dof_vector_aos(prob)
    fa[fixed_aos] = 0.0
    edof = fem.element_dofs_grid(*dims)
    Ee = fem.simp(rho)
    Au = _op_oracle(prob, Ee, ua, fixed_aos, edof)
    rel = np.linalg.norm(fa - Au) / np.linalg.norm(fa)
    log(f"  iterations {st.iterations[0]}, oracle residual {rel:.3e}, gpu {st.rel_residual[0]:.3e}")
    assert rel <= 1.05e-8
    assert abs(C[0] - fa @ ua) <= 1e-12 * abs(C[0])
    assert abs(ua @ Au - C[0]) <= 1e-8 * abs(C[0])
    want = sens.dc_drho_phys(rho, sens.element_energy(ua, edof, fem.hex8_ke()))
    assert np.abs(dc.cpu().numpy() - want).max() <= 1e-12 * np.abs(want).max()
    m.close()


def test_precision_form_full_size_certificate():
    """The refinement form on the 256x128x128 precision-form mesh (5 levels,
    rel. residual 1e-8): the oracle's FP64 residual meets the tolerance, the
    compliance is within 1e-6 of the FP64 GPU path, and in both forms every
    element's sensitivity equals the oracle's eq. 6 from that form's u."""
    aarmr = _aarmr()
    dims = (256, 128, 128)
    prob = synth.cantilever(*dims)
    rho = synth.smoothed_field(*dims, 8.0, 1e-3, 1.0, seed=3).ravel()
    out = {}
    for prec in (aarmr.FP64, aarmr.FP32_REFINE):
        m = _mesh(prob, autotune=False, mg_levels=5, cg_rtol=1e-8, cg_maxit=2000,
                  precision=prec)
        fx = _fixed(prob, m)
        f = t64(np.asarray(aarmr.loads_soa(prob, m.n_node)[0]))
        u = torch.zeros_like(f)
        dc = torch.zeros(m.n_elem, dtype=torch.float64, device="cuda")
        C, st, code = m.solve(t64(rho), f, fx, u, dc=dc)
        assert code == aarmr.OK
        out[prec] = (C[0], u.cpu().numpy(), st.iterations[0], dc.cpu().numpy())
        m.close()
        del u, f, dc
        torch.cuda.empty_cache()
    fixed_aos = fem.fixed_dofs_aos(prob)
    ua = _aos(out[aarmr.FP32_REFINE][1])
    fa = fem.dof_vector_aos(prob)
    fa[fixed_aos] = 0.0
    Au = _op_oracle(prob, fem.simp(rho), ua, fixed_aos, fem.element_dofs_grid(*dims))
    rel = np.linalg.norm(fa - Au) / np.linalg.norm(fa)
    c64, c32 = out[aarmr.FP64][0], out[aarmr.FP32_REFINE][0]
    log(f"  refinement: {out[aarmr.FP32_REFINE][2]} iterations, oracle residual {rel:.3e}, "
        f"C diff vs FP64 {abs(c32 - c64) / c64:.2e}")
    assert rel <= 1.05e-8
    assert abs(c32 - c64) <= 1e-6 * c64
    # eq. 6 on every element from each form's own displacement (the sensitivity
    # kernel at full size against the oracle's element energies)
    edof = fem.element_dofs_grid(*dims)
    for prec in (aarmr.FP64, aarmr.FP32_REFINE):
        want = sens.dc_drho_phys(rho, sens.element_energy(_aos(out[prec][1]), edof, fem.hex8_ke()))
        err = np.abs(out[prec][3] - want).max() / np.abs(want).max()
        log(f"  dc precision {prec}: max rel err {err:.2e}")
        # an element's energy is formed from nodal displacements dominated by
        # the element's rigid motion (the cantilever's tip rotates), so both
        # sides lose digits to that cancellation: measured 6e-13 here
        assert err < 4e-12


@pytest.mark.parametrize("levels", [5, 6])
def test_full_size_level1_operator_and_vcycle_symmetric(levels):
    """The kernels that take over on large grids only (the separable
    restriction and the LDS-staged interpolation, from 1e5 coarse / 1e6 fine
    nodes; the per-element level-1 product, from 2e5 level-1 elements; the
    level-2 matrices from the fine moduli) at 256x128x128: the level-1
    Galerkin operator and the V-cycle are symmetric, <A x, y> = <x, A y>
    and <M x, y> = <x, M y>, which fails if a restriction weight or index
    differs from the interpolation's or if an element's output entries are
    misplaced; A_1 is positive definite on random vectors."""
    aarmr = _aarmr()
    dims = (256, 128, 128)
    log(f"full-size symmetry, {levels} levels")
    prob = synth.cantilever(*dims)
    rho = synth.smoothed_field(*dims, 8.0, 1e-3, 1.0, seed=3).ravel()
    m = _mesh(prob, autotune=False, mg_levels=levels)
    fx = _fixed(prob, m)
    m.setup(t64(rho), fx)
    g = torch.Generator(device="cuda")
    g.manual_seed(31)
    n1 = 3 * (dims[0] // 2 + 1) * (dims[1] // 2 + 1) * (dims[2] // 2 + 1)
    x1 = torch.randn(n1, dtype=torch.float64, device="cuda", generator=g)
    y1 = torch.randn(n1, dtype=torch.float64, device="cuda", generator=g)
    ax = torch.empty_like(x1)
    ay = torch.empty_like(y1)
    m.apply(x1, ax, level=1)
    m.apply(y1, ay, level=1)
    lhs, rhs = float(ax @ y1), float(x1 @ ay)
    assert abs(lhs - rhs) <= 1e-12 * (float(ax.norm()) * float(y1.norm()))
    assert float(ax @ x1) > 0.0
    n0 = 3 * m.n_node
    x = torch.randn(n0, dtype=torch.float64, device="cuda", generator=g)
    y = torch.randn(n0, dtype=torch.float64, device="cuda", generator=g)
    x[fx] = 0.0
    y[fx] = 0.0
    zx = torch.empty_like(x)
    zy = torch.empty_like(y)
    m.vcycle(x, zx)
    m.vcycle(y, zy)
    lhs, rhs = float(zx @ y), float(x @ zy)
    log(f"  <Mx,y> {lhs:.12e}  <x,My> {rhs:.12e}")
    assert abs(lhs - rhs) <= 1e-11 * (float(zx.norm()) * float(y.norm()))
    assert float(zx @ x) > 0.0
    m.close()


def test_level1_galerkin_identity_per_element_path():
    """The per-element level-1 product (one thread per parent for all 24
    outputs, used from 2e5 level-1 elements) against Algorithm 2's first
    coarse operator composed on the oracle's side, A_1 v = (Df P)^T K (Df P) v,
    with P the oracle's trilinear interpolation and K its element-by-element
    product.  At 160x112x112 level 1 has 80x56x56 = 250880 parents, and the
    clamped face's flagged parents take the stored-matrix rows of the same
    launch."""
    from oracle import mg

    dims = (160, 112, 112)
    log("level-1 galerkin identity 160x112x112, 5 levels")
    prob = synth.cantilever(*dims)
    rho = synth.smoothed_field(*dims, 8.0, 1e-3, 1.0, seed=5).ravel()
    m = _mesh(prob, autotune=False, mg_levels=5)
    fx = _fixed(prob, m)
    m.setup(t64(rho), fx)
    P = mg.prolongation_kron(dims[0] // 2, dims[1] // 2, dims[2] // 2)
    v = np.random.default_rng(41).standard_normal(P.shape[1])
    y1 = torch.zeros(P.shape[1], dtype=torch.float64, device="cuda")
    m.apply(t64(fem.aos_to_soa(v).ravel()), y1, level=1)
    free = fem.free_mask(3 * m.n_node, fem.fixed_dofs_aos(prob)).astype(np.float64)
    y0 = free * fem.apply_ebe(*dims, fem.simp(rho), fem.hex8_ke(), free * (P @ v))
    want = P.T @ y0
    got = fem.soa_to_aos(y1.cpu().numpy())
    err = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    log(f"  rel {err:.3e}")
    assert err < 1e-12
    m.close()


def test_filter_and_oc_on_the_loop_mesh():
    """The optimisation loop's support steps at its own size (96x48x48, filter
    radius 2): every output of the density filter and its adjoint (eqs. 31-33)
    against the oracle's explicit filter matrix, and one OC update from a
    loop-like state (smoothed design, sensitivities of a smoothed field)
    against the oracle's bisection."""
    from oracle import filt, oc

    aarmr = _aarmr()
    dims = (96, 48, 48)
    log("filter and OC on the loop mesh 96x48x48, r = 2")
    prob = synth.cantilever(*dims)
    m = _mesh(prob, autotune=False, **LOOP)
    H, Hs = filt.filter_matrix(*dims, 2.0)
    x = synth.smoothed_field(*dims, 3.0, 0.05, 1.0, seed=21).ravel()
    out = torch.zeros(m.n_elem, dtype=torch.float64, device="cuda")
    m.filter(t64(x), out, mode=0)
    want = filt.forward(H, Hs, x)
    err = np.abs(out.cpu().numpy() - want).max() / np.abs(want).max()
    log(f"  forward max rel err {err:.2e}")
    assert err < 1e-14
    g = -synth.smoothed_field(*dims, 2.0, 0.01, 3.0, seed=22).ravel()
    m.filter(t64(g), out, mode=1)
    want = filt.adjoint(H, Hs, g)
    err = np.abs(out.cpu().numpy() - want).max() / np.abs(want).max()
    log(f"  adjoint max rel err {err:.2e}")
    assert err < 1e-14
    dv = filt.adjoint(H, Hs, np.ones(m.n_elem))
    dc = filt.adjoint(H, Hs, g)
    xn, xp, lam = oc.oc_update(x, dc, dv, H, Hs, 0.3)
    gx = torch.zeros(m.n_elem, dtype=torch.float64, device="cuda")
    gp = torch.zeros_like(gx)
    m.oc_update(t64(x), t64(dc), t64(dv), 0.3, 0.2, gx, gp)
    ex = float(np.linalg.norm(gx.cpu().numpy() - xn) / np.linalg.norm(xn))
    ep = float(np.linalg.norm(gp.cpu().numpy() - xp) / np.linalg.norm(xp))
    log(f"  OC: x rel {ex:.2e}, filtered rel {ep:.2e}, volume {gp.sum().item() / m.n_elem:.6f}")
    assert ex < 1e-9 and ep < 1e-9
    m.close()


def test_zero_load_gives_zero_solution():
    """Degenerate case: no load, u = 0, C = 0 and dc = 0 without iterating."""
    aarmr = _aarmr()
    prob = synth.cantilever(16, 8, 8)
    m = _mesh(prob, autotune=False, mg_levels=3)
    f = torch.zeros(3 * m.n_node, dtype=torch.float64, device="cuda")
    u = torch.ones_like(f)
    dc = torch.ones(m.n_elem, dtype=torch.float64, device="cuda")
    C, st, code = m.solve(t64(np.full(m.n_elem, 0.5)), f, _fixed(prob, m), u, dc=dc,
                          flags=aarmr.WARM_START)
    assert code == aarmr.OK and C[0] == 0.0 and st.iterations[0] == 0
    assert float(u.abs().max()) == 0.0 and float(dc.abs().max()) == 0.0


def test_fine_operator_at_largest_accepted_mesh():
    """The largest grid the mesh check accepts for this shape: 704x384x320
    (86.5 M elements, 261 M DOFs, 7 levels), where the fine product's FP64
    vectors take 0.974 of its 2^31-byte offset range.  The oracle's row-by-row
    product checks sampled outputs: the grid's corners, nodes on both sides of
    the 30-node x and 15-row y tile seams, the last nodes of the grid (the
    largest offsets) and 3000 random nodes, in the general form and in the
    solver form (input zero on fixed DOFs)."""
    aarmr = _aarmr()
    dims = (704, 384, 320)
    nx, ny, nz = dims
    nxp, nyp = nx + 1, ny + 1
    log(f"largest mesh K.v {dims}")
    prob = synth.cantilever(*dims)
    m = _mesh(prob, autotune=False, mg_levels=7)
    nn = m.n_node
    assert 3 * nn * 8 < 2 ** 31 and 3 * nn * 8 > 0.97 * 2 ** 31
    rho = synth.uniform_iid(nx, ny, nz, 1e-3, 1.0, seed=11).ravel()
    fx = _fixed(prob, m)
    m.setup(t64(rho), fx)
    rng = np.random.default_rng(111)
    v = rng.standard_normal((3, nn))
    fixed = np.zeros((3, nn), dtype=bool)
    fixed.ravel()[fx.cpu().numpy()] = True

    def nid(i, j, k):
        return i + nxp * (j + nyp * k)

    sample = [nid(i, j, k) for i in (0, nx) for j in (0, ny) for k in (0, nz)]
    sample += [nid(i, j, k) for i in (0, 1, 29, 30, 31, 59, 60, 61, nx - 1)
               for j in (14, 15, 16, 29, 30, ny - 1) for k in (1, nz // 2, nz - 1)]
    sample += [nn - 1, nn - 2, nn - nxp, nn - nxp * nyp]
    sample = np.unique(np.concatenate([np.array(sample), rng.integers(0, nn, 3000)]))
    vm = np.where(fixed, 0.0, v)
    rows = fem.apply_ebe_at_nodes(nx, ny, nz, fem.simp(rho), fem.hex8_ke(),
                                  lambda ids: vm[ids % 3, ids // 3], sample)
    want = np.where(fixed[:, sample].T, v[:, sample].T, rows)  # identity rows on fixed DOFs
    scale = np.abs(want).max()
    idx = torch.tensor(sample, dtype=torch.int64, device="cuda")
    vt = t64(v.ravel())
    y = torch.empty(3 * nn, dtype=torch.float64, device="cuda")
    m.apply(vt, y)
    got = y.view(3, nn)[:, idx].T.cpu().numpy()
    err = np.abs(got - want).max() / scale
    log(f"  general form, {len(sample)} nodes: max rel err {err:.2e}")
    assert err < 1e-13
    del vt
    vmt = t64(vm.ravel())
    m.apply(vmt, y, flags=aarmr.INPUT_MASKED)
    got = y.view(3, nn)[:, idx].T.cpu().numpy()
    want_m = np.where(fixed[:, sample].T, 0.0, rows)  # the masked input's identity rows
    err = np.abs(got - want_m).max() / scale
    log(f"  solver form: max rel err {err:.2e}")
    assert err < 1e-13
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(5):
        m.apply(vmt, y, flags=aarmr.INPUT_MASKED)
    t1.record()
    t1.synchronize()
    ms = t0.elapsed_time(t1) / 5
    log(f"  solver-form product {ms:.3f} ms, {3 * nn / ms / 1e6:.1f} GDOF/s")
    m.close()


def test_analysis_at_largest_accepted_mesh():
    """One analysis on the largest accepted grid (704x384x320, 261 M DOFs, 7
    levels, rel. residual 1e-8, iid density in [0.3, 1]) in FP64 and in the
    refinement form: the residual ||f - A u|| / ||f|| from the library's FP64
    product (itself checked against the oracle at sampled nodes on this grid)
    meets the tolerance, the compliance equals f^T u and the energy u^T A u,
    and the two forms' compliances agree to 1e-6.  Element-wise iid moduli
    raise lambda_max(D^-1 A) to about 3.9 (3.09 for a uniform design), so the
    damped-Jacobi weight is 0.5: the sweep must keep omega lambda_max < 2 for
    the V-cycle to stay positive definite."""
    aarmr = _aarmr()
    dims = (704, 384, 320)
    prob = synth.cantilever(*dims)
    rho = t64(synth.uniform_iid(*dims, 0.3, 1.0, seed=12).ravel())
    comp = {}
    for prec in (aarmr.FP64, aarmr.FP32_REFINE):
        log(f"largest mesh analysis {dims} precision {prec}")
        m = _mesh(prob, autotune=False, mg_levels=7, cg_rtol=1e-8, cg_maxit=500, omega=0.5,
                  precision=prec)
        fx = _fixed(prob, m)
        f = t64(np.asarray(aarmr.loads_soa(prob, m.n_node)[0]))
        u = torch.zeros_like(f)
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        C, st, code = m.solve(rho, f, fx, u)
        t1.record()
        t1.synchronize()
        assert code == aarmr.OK
        fm = f.clone()
        fm[fx] = 0.0
        Au = torch.empty_like(u)
        m.apply(u, Au)
        Au[fx] = 0.0
        res = float(torch.linalg.vector_norm(fm - Au) / torch.linalg.vector_norm(fm))
        ftu, uau = float(fm @ u), float(u @ Au)
        log(f"  {st.iterations[0]} iterations, {t0.elapsed_time(t1):.0f} ms, residual {res:.3e}, "
            f"C {C[0]:.10g}")
        assert res <= 1.05e-8
        assert abs(C[0] - ftu) <= 1e-12 * abs(C[0])
        assert abs(uau - C[0]) <= 1e-8 * abs(C[0])
        comp[prec] = C[0]
        m.close()
        del m, f, u, fm, Au
        torch.cuda.empty_cache()
    assert abs(comp[aarmr.FP32_REFINE] - comp[aarmr.FP64]) <= 1e-6 * comp[aarmr.FP64]
