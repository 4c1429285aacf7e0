"""Parity of the refinement form (precision AARMR_FP32_REFINE: FP32
operator sweeps, V-cycle and inner CG vectors; FP64 residuals, dot-product
accumulation, updates of u and the coarsest inverse) against the CPU FP64
oracle and against the FP64 GPU path.  The bar is the same as for the FP64
path: compliance and displacement within 1e-6 relative at an FP64 relative
residual of cg_rtol."""

import numpy as np
import pytest
import torch

import synth
from oracle import filt, sens

from gpu_util import fixed_tensor, loads_tensor, log, mesh_for, rel, soa, t64

pytestmark = pytest.mark.gpu


def _aarmr():
    from paper_2205_00385_amd import aarmr

    return aarmr


@pytest.mark.parametrize("rtol", [1e-8, 1e-11])
def test_refine_cantilever24_matches_direct(rtol):
    """The 24x12x12 cantilever of the FP64 test (design density U[0.3, 1],
    seed 1, filter r=1.5, 3 levels).  rtol 1e-11 lies below FP32 precision,
    so only the FP64 refinement can reach it."""
    aarmr = _aarmr()
    nx, ny, nz = 24, 12, 12
    log(f"refine cantilever24 rtol={rtol}")
    prob = synth.cantilever(nx, ny, nz)
    x = synth.uniform_iid(nx, ny, nz, 0.3, 1.0, seed=1).ravel()
    m = mesh_for(prob, mg_levels=3, rmin=1.5, cg_rtol=rtol, precision=aarmr.FP32_REFINE)
    fixed = fixed_tensor(prob, m)
    f = loads_tensor(prob, m)
    u = torch.zeros_like(f)
    dc = torch.zeros(m.n_elem, dtype=torch.float64, device="cuda")
    C, st, code = m.solve(t64(x), f, fixed, u, dc=dc, flags=aarmr.FILTER_INPUT)
    H, Hs = filt.filter_matrix(nx, ny, nz, 1.5)
    us, Cs, dcp = sens.analyse(prob, filt.forward(H, Hs, x))
    log(f"  its={st.iterations[0]} rel={st.rel_residual[0]:.2e} C={C[0]:.12g} ref={Cs[0]:.12g}")
    assert code == aarmr.OK and st.rel_residual[0] <= rtol
    assert abs(C[0] - Cs[0]) <= 1e-6 * abs(Cs[0])
    assert rel(u.cpu().numpy(), soa(us[0])) <= 1e-6
    assert rel(dc.cpu().numpy(), filt.adjoint(H, Hs, dcp)) <= 1e-6


def test_refine_bridge_void_contrast():
    """Simply supported beam on a thresholded field whose void is at the
    SIMP floor (rho = 1e-3, E ~ 1e-9): contrast ~1e9 in an FP32 inner solve."""
    aarmr = _aarmr()
    prob = synth.bridge(16, 8, 8)
    m = mesh_for(prob, mg_levels=3, cg_rtol=1e-9, precision=aarmr.FP32_REFINE)
    rho = synth.thresholded_field(16, 8, 8, 2.0, 1e-3, 1.0, seed=9).ravel()
    f = loads_tensor(prob, m)
    u = torch.zeros_like(f)
    C, st, code = m.solve(t64(rho), f, fixed_tensor(prob, m), u)
    us, Cs, _ = sens.analyse(prob, rho)
    log(f"  refine bridge its={st.iterations[0]} rel={st.rel_residual[0]:.2e} C={C[0]:.10g}")
    assert code == aarmr.OK and st.rel_residual[0] <= 1e-9
    assert abs(C[0] - Cs[0]) <= 1e-6 * abs(Cs[0])
    assert rel(u.cpu().numpy(), soa(us[0])) <= 1e-6


def test_refine_multi_case_and_warm_start():
    aarmr = _aarmr()
    prob = synth.point_loads_on_face(16, 8, 8, n_case=3, seed=7)
    m = mesh_for(prob, mg_levels=3, cg_rtol=1e-9, n_rhs_max=4, precision=aarmr.FP32_REFINE)
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
    C2, st2, _ = m.solve(t64(rho), f, fixed, u, flags=aarmr.WARM_START)
    assert all(st2.iterations[l] == 0 for l in range(3))


def test_refine_matches_fp64_gpu_random_field():
    """64x32x32 cantilever on the smoothed random field of the large
    mixed-precision workload (correlation 8 voxels, [1e-3, 1]): the
    refinement form against the FP64 path, both at rtol 1e-8."""
    aarmr = _aarmr()
    nx, ny, nz = 64, 32, 32
    prob = synth.cantilever(nx, ny, nz)
    rho = t64(synth.smoothed_field(nx, ny, nz, 8.0, 1e-3, 1.0, seed=3).ravel())
    out = {}
    for prec in (aarmr.FP64, aarmr.FP32_REFINE):
        m = mesh_for(prob, mg_levels=4, cg_rtol=1e-8, precision=prec)
        f = loads_tensor(prob, m)
        u = torch.zeros_like(f)
        C, st, code = m.solve(rho, f, fixed_tensor(prob, m), u)
        assert code == aarmr.OK and st.rel_residual[0] <= 1e-8
        out[prec] = (C[0], u.cpu().numpy(), st.iterations[0])
        log(f"  prec={prec} its={st.iterations[0]} rel={st.rel_residual[0]:.2e} C={C[0]:.12g}")
        m.close()
    C64, u64, _ = out[aarmr.FP64]
    C32, u32, _ = out[aarmr.FP32_REFINE]
    assert abs(C32 - C64) <= 1e-6 * abs(C64)
    assert rel(u32, u64) <= 1e-6
