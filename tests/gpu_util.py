"""Helpers of the GPU tests: build meshes and device tensors from the seeded
problem descriptions, and convert between the oracle's AoS vectors and the
library's SoA vectors."""

import numpy as np
import torch

from oracle import fem


def dev():
    return torch.device("cuda:0")


def t64(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), dtype=torch.float64, device=dev())


def mesh_for(prob, **kw):
    from paper_2205_00385_amd import aarmr

    p = aarmr.default_params(nx=prob.nx, ny=prob.ny, nz=prob.nz, **kw)
    return aarmr.Mesh(p)


def fixed_tensor(prob, mesh):
    from paper_2205_00385_amd import aarmr

    return torch.tensor(aarmr.fixed_dofs_soa(prob, mesh.n_node), dtype=torch.int64, device=dev())


def loads_tensor(prob, mesh, cases=None):
    from paper_2205_00385_amd import aarmr

    return t64(np.concatenate([np.asarray(v) for v in aarmr.loads_soa(prob, mesh.n_node, cases)]))


def soa(v_aos):
    return fem.aos_to_soa(v_aos).ravel()


def aos(v_soa):
    return fem.soa_to_aos(np.asarray(v_soa))


def rel(a, b):
    a, b = np.asarray(a).ravel(), np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def log(msg):
    print(msg, flush=True)
