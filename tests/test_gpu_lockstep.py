"""Load cases of the refinement form solved in lock step (one set of
launches per iteration for all cases of a mesh): every case must get the
bits of its own single-case solve, and the oracle's solution to the 1e-6
bar.  Covers a zero load case, warm starts and a case count below the
mesh's maximum."""

import numpy as np
import pytest
import torch

import synth
from oracle import fem, sens, solve

from gpu_util import fixed_tensor, log, mesh_for, rel, soa, t64

pytestmark = pytest.mark.gpu


def _aarmr():
    from paper_2205_00385_amd import aarmr

    return aarmr


def _loads(prob, m, cases):
    aarmr = _aarmr()
    return [np.asarray(v) for v in aarmr.loads_soa(prob, m.n_node, cases)]


@pytest.mark.parametrize("dims,n_case,levels", [((24, 16, 16), 4, 3), ((32, 16, 24), 3, 4)])
def test_lockstep_cases_equal_single_case_solves(dims, n_case, levels):
    aarmr = _aarmr()
    prob = synth.point_loads_on_face(*dims, n_case=n_case, seed=81)
    rho = synth.smoothed_field(*dims, 3.0, 1e-3, 1.0, seed=82).ravel()
    multi = mesh_for(prob, mg_levels=levels, n_rhs_max=4, precision=aarmr.FP32_REFINE)
    single = mesh_for(prob, mg_levels=levels, n_rhs_max=1, precision=aarmr.FP32_REFINE)
    fixed = fixed_tensor(prob, multi)
    fl = _loads(prob, multi, None)
    f = t64(np.concatenate(fl))
    u = torch.zeros_like(f)
    dc = torch.zeros(multi.n_elem, dtype=torch.float64, device="cuda")
    C, st, code = multi.solve(t64(rho), f, fixed, u, dc=dc)
    assert code == 0
    n3 = 3 * multi.n_node
    KE = fem.hex8_ke()
    K = fem.assemble(*dims, fem.simp(rho), KE)
    fx = fem.fixed_dofs_aos(prob)
    free = fem.free_mask(K.shape[0], fx)
    edof = fem.element_dofs(*dims)
    dc_ref = np.zeros(multi.n_elem)
    for l in range(n_case):
        u1 = torch.zeros(n3, dtype=torch.float64, device="cuda")
        C1, st1, code1 = single.solve(t64(rho), t64(fl[l]), fixed, u1)
        assert code1 == 0
        log(f"  {dims} case {l}: lock-step {st.iterations[l]} its, alone {st1.iterations[0]} its")
        assert torch.equal(u[l * n3:(l + 1) * n3], u1), f"case {l} differs from its own solve"
        assert C[l] == C1[0]
        fa = fem.dof_vector_aos(prob, l) * free
        ua = solve.solve_direct(K, fa, fx, dims)
        Cr = float(fa @ ua)
        assert abs(C[l] - Cr) <= 1e-6 * abs(Cr)
        assert rel(u1.cpu().numpy(), soa(ua)) <= 1e-6
        dc_ref += sens.dc_drho_phys(rho, sens.element_energy(ua, edof, KE))
    assert rel(dc.cpu().numpy(), dc_ref) <= 1e-6
    # warm start from the converged solutions: nothing left to do
    C2, st2, code2 = multi.solve(t64(rho), f, fixed, u, flags=aarmr.WARM_START)
    assert code2 == 0 and all(st2.iterations[l] == 0 for l in range(n_case))
    multi.close()
    single.close()


def test_lockstep_large_grid_kernels():
    """Lock step on a grid where the large-grid kernels take over (the
    separable restriction from 1e5 coarse nodes, the LDS-staged interpolation
    from 1e6 fine nodes, the per-element level-1 product from 2e5 level-1
    elements), whose load-case strides only the lock-step solve exercises:
    160x112x112, 3 cases, 5 levels.  Every case gets the bits of its own
    single-case solve, and the oracle's FP64 residual of each meets 1e-8."""
    aarmr = _aarmr()
    dims = (160, 112, 112)
    log(f"lock-step large grid {dims}")
    prob = synth.point_loads_on_face(*dims, n_case=3, seed=85)
    rho = synth.smoothed_field(*dims, 6.0, 1e-3, 1.0, seed=86).ravel()
    multi = mesh_for(prob, mg_levels=5, n_rhs_max=3, precision=aarmr.FP32_REFINE)
    single = mesh_for(prob, mg_levels=5, n_rhs_max=1, precision=aarmr.FP32_REFINE)
    fixed = fixed_tensor(prob, multi)
    fl = _loads(prob, multi, None)
    f = t64(np.concatenate(fl))
    u = torch.zeros_like(f)
    C, st, code = multi.solve(t64(rho), f, fixed, u)
    assert code == 0
    n3 = 3 * multi.n_node
    fx = fem.fixed_dofs_aos(prob)
    edof = fem.element_dofs_grid(*dims)
    Ee = fem.simp(rho)
    for l in range(3):
        u1 = torch.zeros(n3, dtype=torch.float64, device="cuda")
        C1, st1, code1 = single.solve(t64(rho), t64(fl[l]), fixed, u1)
        assert code1 == 0
        log(f"  case {l}: lock-step {st.iterations[l]} its, alone {st1.iterations[0]} its")
        assert torch.equal(u[l * n3:(l + 1) * n3], u1), f"case {l} differs from its own solve"
        assert C[l] == C1[0]
        ua = fem.soa_to_aos(u1.cpu().numpy())
        fa = fem.dof_vector_aos(prob, l)
        fa[fx] = 0.0
        um = ua.copy()
        um[fx] = 0.0
        Au = fem.apply_ebe(*dims, Ee, fem.hex8_ke(), um, edof)
        Au[fx] = ua[fx]
        res = np.linalg.norm(fa - Au) / np.linalg.norm(fa)
        assert res <= 1.05e-8, f"case {l}: oracle residual {res:.3e}"
    multi.close()
    single.close()


def test_lockstep_with_a_zero_load_case():
    aarmr = _aarmr()
    dims = (16, 8, 8)
    prob = synth.point_loads_on_face(*dims, n_case=2, seed=83)
    rho = synth.smoothed_field(*dims, 2.0, 1e-2, 1.0, seed=84).ravel()
    m = mesh_for(prob, mg_levels=3, n_rhs_max=3, precision=aarmr.FP32_REFINE)
    fl = _loads(prob, m, None)
    f = t64(np.concatenate([fl[0], np.zeros_like(fl[0]), fl[1]]))
    u = torch.full_like(f, 1.0)
    C, st, code = m.solve(t64(rho), f, fixed_tensor(prob, m), u)
    assert code == 0
    n3 = 3 * m.n_node
    assert C[1] == 0.0 and float(u[n3:2 * n3].abs().max()) == 0.0
    assert st.iterations[1] == 0
    assert st.rel_residual[0] <= 1e-8 and st.rel_residual[2] <= 1e-8
    m.close()


def test_loads_built_on_the_device_equal_host_loads():
    aarmr = _aarmr()
    for prob, nn in ((synth.point_loads_on_face(12, 8, 8, n_case=5, seed=85), 13 * 9 * 9),
                     (synth.inverter2d(16, 8), 17 * 9)):
        host = np.concatenate(aarmr.loads_soa(prob, nn))
        dev = aarmr.loads_device(prob, nn, "cuda")
        assert torch.equal(dev.cpu(), torch.tensor(host))
        sub = aarmr.loads_device(prob, nn, "cuda", cases=[1, 0])
        assert torch.equal(sub.cpu(), torch.tensor(np.concatenate(aarmr.loads_soa(prob, nn, [1, 0]))))
