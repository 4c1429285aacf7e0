"""The allocation-free OC update (static device scratch, no read-back)
against the regular OC update through the C ABI: bitwise equal outputs on
two calls in a row on one GPU, the second on a smaller mesh, so that the
scratch array's contents from the first call must not leak into the
second."""

import numpy as np
import pytest
import torch

import synth
from oracle import filt
from gpu_util import mesh_for, t64

pytestmark = pytest.mark.gpu


def _case(dims, seed, volfrac):
    prob = synth.cantilever(*dims)
    m = mesh_for(prob, mg_levels=2, rmin=2.0)
    H, Hs = filt.filter_matrix(*dims, 2.0)
    rng = np.random.default_rng(seed)
    x = t64(rng.uniform(0.1, 0.9, m.n_elem))
    dc = t64(-rng.uniform(0.01, 3.0, m.n_elem))
    dv = t64(filt.adjoint(H, Hs, np.ones(m.n_elem)))
    return m, x, dc, dv, volfrac


def test_oc_noalloc_matches_oc_update_twice():
    for dims, seed, vf in (((24, 16, 12), 51, 0.3), ((12, 8, 6), 52, 0.45)):
        print(f"[no-alloc] OC {dims} seed {seed}", flush=True)
        m, x, dc, dv, vf = _case(dims, seed, vf)
        ref_x = torch.zeros_like(x)
        ref_p = torch.zeros_like(x)
        m.oc_update(x, dc, dv, vf, 0.2, ref_x, ref_p)
        got_x = torch.full_like(x, -1.0)
        got_p = torch.full_like(x, -1.0)
        m.oc_update_noalloc(x, dc, dv, vf, 0.2, got_x, got_p)
        torch.cuda.synchronize()
        assert torch.equal(got_x, ref_x)
        assert torch.equal(got_p, ref_p)
        # the volume constraint the bisection targets holds on the output
        assert abs(float(got_p.sum()) / m.n_elem - vf) < 1e-2
