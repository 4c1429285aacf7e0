"""Thin ctypes binding of the AARMR HIP library (``libaarmr.so``).

Argument marshalling only: every call forwards device pointers of torch
tensors and the current HIP stream to the C ABI declared in
``include/aarmr.h``.  There is no CPU fallback: importing this module without
the built library raises, and every call that fails raises
:class:`AarmrError` with the library's message.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libaarmr.so")

OK, E_INVALID, E_HIP, E_NOT_CONVERGED, E_SINGULAR, E_NO_WORKSPACE, E_STATE = range(7)
MAX_RHS, MAX_LEVELS, MAX_BASIS, MAX_SPRINGS = 8, 8, 10, 8
FP64, FP32_REFINE = 0, 1
FILTER_INPUT, RECORD_PARM, WARM_START, INPUT_MASKED, MUTUAL_SENS, REUSE_COARSEST = 1, 2, 4, 8, 16, 32
ORTH_GS, ORTH_SVD = 0, 1


class AarmrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"aarmr error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("E0", ctypes.c_double), ("Emin", ctypes.c_double), ("nu", ctypes.c_double),
        ("penal", ctypes.c_double), ("rmin", ctypes.c_double),
        ("mg_levels", ctypes.c_int32), ("nu_pre", ctypes.c_int32), ("nu_post", ctypes.c_int32),
        ("omega", ctypes.c_double), ("cg_rtol", ctypes.c_double), ("cg_maxit", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("Ns", ctypes.c_int32), ("Nm", ctypes.c_int32),
        ("ca_tol", ctypes.c_double), ("gs_tau", ctypes.c_double), ("n_rhs_max", ctypes.c_int32),
        ("orth", ctypes.c_int32), ("oc_eta", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32 * MAX_RHS),
        ("rel_residual", ctypes.c_double * MAX_RHS),
        ("fine_sweeps", ctypes.c_int64),
        ("setup_ms", ctypes.c_double), ("solve_ms", ctypes.c_double),
        ("coarsest_inversions", ctypes.c_int32),
    ]


class CAStats(ctypes.Structure):
    _fields_ = [
        ("eps", ctypes.c_double * MAX_RHS),
        ("accepted", ctypes.c_int32 * MAX_RHS),
        ("rank", ctypes.c_int32 * MAX_RHS),
        ("mgcg_iterations", ctypes.c_int32 * MAX_RHS),
        ("rel_residual", ctypes.c_double * MAX_RHS),
        ("fine_sweeps", ctypes.c_int64),
        ("coarsest_inversions", ctypes.c_int32),
    ]


class BatchItem(ctypes.Structure):
    _fields_ = [
        ("mesh", ctypes.c_void_p), ("rho", ctypes.c_void_p), ("f", ctypes.c_void_p),
        ("n_rhs", ctypes.c_int32), ("fixed_dofs", ctypes.c_void_p), ("n_fixed", ctypes.c_int64),
        ("u", ctypes.c_void_p), ("compliance", ctypes.c_void_p), ("dc", ctypes.c_void_p),
        ("flags", ctypes.c_int32), ("status", ctypes.c_int32), ("stats", Stats),
        ("done", ctypes.c_int32),
    ]


EXPORTS = [
    "aarmr_default_params", "aarmr_mesh_create", "aarmr_mesh_destroy", "aarmr_workspace_bytes",
    "aarmr_bind_workspace", "aarmr_solve", "aarmr_ca_update", "aarmr_filter", "aarmr_setup",
    "aarmr_apply_operator", "aarmr_vcycle", "aarmr_element_energy", "aarmr_oc_update",
    "aarmr_oc_update_noalloc",
    "aarmr_autotune", "aarmr_set_chunk", "aarmr_batch_solve", "aarmr_batch_submit", "aarmr_batch_poll",
    "aarmr_batch_wait", "aarmr_set_springs", "aarmr_last_error",
]


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python -m paper_2205_00385_amd.build` "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    P, vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.aarmr_default_params.argtypes = [ctypes.POINTER(Params)]
    lib.aarmr_default_params.restype = None
    lib.aarmr_mesh_create.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(P)]
    lib.aarmr_mesh_destroy.argtypes = [P]
    lib.aarmr_mesh_destroy.restype = None
    lib.aarmr_workspace_bytes.argtypes = [P]
    lib.aarmr_workspace_bytes.restype = i64
    lib.aarmr_bind_workspace.argtypes = [P, vp, i64, vp]
    lib.aarmr_solve.argtypes = [P, vp, vp, i32, vp, i64, vp, vp, vp, i32, ctypes.POINTER(Stats), vp]
    lib.aarmr_ca_update.argtypes = [P, vp, vp, i32, vp, i64, vp, vp, vp, i32,
                                    ctypes.POINTER(CAStats), vp]
    lib.aarmr_filter.argtypes = [P, i32, vp, vp, vp]
    lib.aarmr_setup.argtypes = [P, vp, vp, i64, vp]
    lib.aarmr_apply_operator.argtypes = [P, i32, vp, vp, i32, vp]
    lib.aarmr_vcycle.argtypes = [P, vp, vp, vp]
    lib.aarmr_element_energy.argtypes = [P, vp, vp, vp]
    lib.aarmr_oc_update.argtypes = [P, vp, vp, vp, dbl, dbl, vp, vp, vp]
    lib.aarmr_oc_update_noalloc.argtypes = [P, vp, vp, vp, dbl, dbl, vp, vp, vp]
    lib.aarmr_batch_solve.argtypes = [ctypes.POINTER(BatchItem), i32, ctypes.POINTER(P), i32]
    lib.aarmr_batch_submit.argtypes = [ctypes.POINTER(BatchItem), i32, ctypes.POINTER(P), i32,
                                       ctypes.POINTER(P)]
    lib.aarmr_batch_poll.argtypes = [P, ctypes.POINTER(i32)]
    lib.aarmr_batch_wait.argtypes = [P]
    lib.aarmr_autotune.argtypes = [P, ctypes.POINTER(i32), vp]
    lib.aarmr_set_chunk.argtypes = [P, i32, i32]
    lib.aarmr_set_springs.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(dbl), i32]
    lib.aarmr_last_error.argtypes = []
    lib.aarmr_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("aarmr_default_params", "aarmr_mesh_destroy", "aarmr_workspace_bytes",
                        "aarmr_last_error"):
            getattr(lib, name).restype = i32
    return lib


_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


def _check(code: int, allow=()) -> int:
    if code != OK and code not in allow:
        raise AarmrError(code, lib().aarmr_last_error().decode())
    return code


def default_params(**kw) -> Params:
    p = Params()
    lib().aarmr_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _f64(t: torch.Tensor, n: int, name: str) -> torch.Tensor:
    if t.dtype != torch.float64 or t.numel() != n:
        raise ValueError(f"{name}: expected float64 with {n} entries, got {t.dtype} {t.numel()}")
    return t


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Mesh:
    """A grid with its device workspace (allocated through torch)."""

    def __init__(self, params: Params, device: str = "cuda"):
        self.params = params
        h = ctypes.c_void_p()
        _check(lib().aarmr_mesh_create(ctypes.byref(params), ctypes.byref(h)))
        self._h = h
        self.nx, self.ny, self.nz = params.nx, params.ny, params.nz
        # nz == 0: the plane-stress grid of unit squares, 2 DOFs per node
        self.dim = 2 if params.nz == 0 else 3
        self.n_elem = params.nx * params.ny * max(params.nz, 1)
        self.n_node = (params.nx + 1) * (params.ny + 1) * (params.nz + 1)
        self.n_dof = self.dim * self.n_node
        nbytes = lib().aarmr_workspace_bytes(h)
        if nbytes < 0:
            raise AarmrError(E_INVALID, "workspace size query failed")
        self.workspace = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws_ptr = self.workspace.data_ptr() + off
        self.workspace_bytes = int(nbytes)
        _check(lib().aarmr_bind_workspace(h, ctypes.c_void_p(self._ws_ptr), nbytes, _stream()))

    def close(self):
        if getattr(self, "_h", None):
            lib().aarmr_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- main entry points ---------------------------------------------------
    def solve(self, rho, f, fixed, u, compliance=True, dc=None, flags=0):
        n3 = self.n_dof
        n_rhs = f.numel() // n3
        _f64(rho, self.n_elem, "rho")
        _f64(f, n_rhs * n3, "f")
        _f64(u, n_rhs * n3, "u")
        if dc is not None:
            _f64(dc, self.n_elem, "dc")
        C = (ctypes.c_double * MAX_RHS)()
        st = Stats()
        code = lib().aarmr_solve(self._h, _ptr(rho), _ptr(f), n_rhs, _ptr(fixed), fixed.numel(),
                                 _ptr(u), C if compliance else None, _ptr(dc), flags,
                                 ctypes.byref(st), _stream())
        _check(code, allow=(E_NOT_CONVERGED,))
        return [C[i] for i in range(n_rhs)], st, code

    def ca_update(self, rho, f, fixed, u, dc=None, flags=0):
        n3 = self.n_dof
        n_rhs = f.numel() // n3
        _f64(rho, self.n_elem, "rho")
        _f64(f, n_rhs * n3, "f")
        _f64(u, n_rhs * n3, "u")
        C = (ctypes.c_double * MAX_RHS)()
        st = CAStats()
        code = lib().aarmr_ca_update(self._h, _ptr(rho), _ptr(f), n_rhs, _ptr(fixed),
                                     fixed.numel(), _ptr(u), C, _ptr(dc), flags,
                                     ctypes.byref(st), _stream())
        _check(code, allow=(E_NOT_CONVERGED,))
        return [C[i] for i in range(n_rhs)], st, code

    def filter(self, x, out, mode=0):
        _check(lib().aarmr_filter(self._h, mode, _ptr(x), _ptr(out), _stream()))
        return out

    # -- building blocks -----------------------------------------------------
    def setup(self, rho_phys, fixed):
        _check(lib().aarmr_setup(self._h, _ptr(rho_phys), _ptr(fixed), fixed.numel(), _stream()))

    def apply(self, v, y, level=0, flags=0):
        _check(lib().aarmr_apply_operator(self._h, level, _ptr(v), _ptr(y), flags, _stream()))
        return y

    def vcycle(self, r, z):
        _check(lib().aarmr_vcycle(self._h, _ptr(r), _ptr(z), _stream()))
        return z

    def element_energy(self, u, out):
        _check(lib().aarmr_element_energy(self._h, _ptr(u), _ptr(out), _stream()))
        return out

    def autotune(self):
        """Pick the fine-grid operator's z-chunk length by timing; returns the
        chosen (FP64, FP32) lengths (0 = the default)."""
        out = (ctypes.c_int32 * 2)()
        _check(lib().aarmr_autotune(self._h, out, _stream()))
        return out[0], out[1]

    def set_chunk(self, tz64, tz32=0):
        """Set the fine-grid operator's z-chunk lengths (0: the default)."""
        _check(lib().aarmr_set_chunk(self._h, int(tz64), int(tz32)))

    def set_springs(self, dofs, k):
        """Grounded springs (host sequences of SoA DOF ids and stiffnesses)."""
        n = len(dofs)
        d = (ctypes.c_int64 * max(n, 1))(*[int(x) for x in dofs])
        kk = (ctypes.c_double * max(n, 1))(*[float(x) for x in k])
        _check(lib().aarmr_set_springs(self._h, d, kk, n))

    def oc_update(self, x, dc, dv, volfrac, move, x_new, rho_new):
        _check(lib().aarmr_oc_update(self._h, _ptr(x), _ptr(dc), _ptr(dv), float(volfrac),
                                     float(move), _ptr(x_new), _ptr(rho_new), _stream()))

    def oc_update_noalloc(self, x, dc, dv, volfrac, move, x_new, rho_new):
        _check(lib().aarmr_oc_update_noalloc(self._h, _ptr(x), _ptr(dc), _ptr(dv),
                                             float(volfrac), float(move), _ptr(x_new),
                                             _ptr(rho_new), _stream()))


def _batch_items(jobs):
    n = len(jobs)
    items = (BatchItem * n)()
    comp = []
    for i, jb in enumerate(jobs):
        m = jb["mesh"]
        n3 = m.n_dof
        n_rhs = jb["f"].numel() // n3
        _f64(jb["rho"], m.n_elem, "rho")
        _f64(jb["f"], n_rhs * n3, "f")
        _f64(jb["u"], n_rhs * n3, "u")
        C = (ctypes.c_double * MAX_RHS)()
        comp.append(C)
        it = items[i]
        it.mesh = m._h.value
        it.rho = jb["rho"].data_ptr()
        it.f = jb["f"].data_ptr()
        it.n_rhs = n_rhs
        it.fixed_dofs = jb["fixed"].data_ptr() if jb["fixed"].numel() else None
        it.n_fixed = jb["fixed"].numel()
        it.u = jb["u"].data_ptr()
        it.compliance = ctypes.cast(C, ctypes.c_void_p).value
        dc = jb.get("dc")
        it.dc = dc.data_ptr() if dc is not None else None
        it.flags = jb.get("flags", 0)
    return items, comp


def batch_solve(jobs, streams, check=True):
    """Solve independent analyses concurrently (aarmr_batch_solve).

    jobs: list of dicts with keys mesh, rho, f, fixed, u and optionally dc,
    flags; tensors as for Mesh.solve.  streams: torch.cuda.Stream objects.
    Returns (compliances per job, the BatchItem array, return code)."""
    n = len(jobs)
    items, comp = _batch_items(jobs)
    hs = (ctypes.c_void_p * len(streams))(*[s.cuda_stream for s in streams])
    code = lib().aarmr_batch_solve(items, n, hs, len(streams))
    if check:
        _check(code, allow=(E_NOT_CONVERGED,))
    out = [[comp[i][l] for l in range(items[i].n_rhs)] for i in range(n)]
    return out, items, code


class BatchRun:
    """A batch started with aarmr_batch_submit: poll() reports progress
    without blocking, wait() finishes it (returns compliances per job and
    the return code).  The job tensors must stay alive until wait()."""

    def __init__(self, jobs, streams):
        self._jobs = jobs
        self._items, self._comp = _batch_items(jobs)
        self._hs = (ctypes.c_void_p * len(streams))(*[s.cuda_stream for s in streams])
        self._h = ctypes.c_void_p()
        _check(lib().aarmr_batch_submit(self._items, len(jobs), self._hs, len(streams),
                                        ctypes.byref(self._h)))

    @property
    def items(self):
        return self._items

    def poll(self) -> int:
        n = ctypes.c_int32()
        _check(lib().aarmr_batch_poll(self._h, ctypes.byref(n)))
        return n.value

    def wait(self, check=True):
        code = lib().aarmr_batch_wait(self._h)
        self._h = None
        if check:
            _check(code, allow=(E_NOT_CONVERGED,))
        n = len(self._jobs)
        return [[self._comp[i][l] for l in range(self._items[i].n_rhs)] for i in range(n)], code


def fixed_dofs_soa(prob, n_node: int):
    """Flatten a problem's fixed (i, j, k, c) list, or (i, j, c) for a
    plane-stress problem, into sorted unique SoA DOF ids c*n_node + n
    (numpy int64)."""
    import numpy as np

    nx, ny = prob.nx, prob.ny
    if not prob.fixed:
        return np.zeros(0, dtype=np.int64)
    f = np.asarray(prob.fixed, dtype=np.int64)
    if not hasattr(prob, "nz"):
        ids = f[:, 2] * n_node + f[:, 0] + (nx + 1) * f[:, 1]
    else:
        ids = f[:, 3] * n_node + f[:, 0] + (nx + 1) * (f[:, 1] + (ny + 1) * f[:, 2])
    return np.unique(ids)


def springs_soa(prob, n_node: int):
    """A plane-stress problem's springs (i, j, c, k) as (SoA DOF ids, k)."""
    nx = prob.nx
    sp = getattr(prob, "springs", [])
    return [c * n_node + i + (nx + 1) * j for (i, j, c, _) in sp], [k for (*_, k) in sp]


def loads_device(prob, n_node: int, device, cases: Optional[Sequence[int]] = None):
    """The SoA load vectors of loads_soa, concatenated over the cases, built
    directly in device memory (zeros plus the few point loads), for grids
    whose host vectors would cost more to build and copy than the solve."""
    import numpy as np

    nx, ny = prob.nx, prob.ny
    plane = not hasattr(prob, "nz")
    n = (2 if plane else 3) * n_node
    cases = list(range(prob.n_case) if cases is None else cases)
    f = torch.zeros(len(cases) * n, dtype=torch.float64, device=device)
    idx, val = [], []
    for slot, l in enumerate(cases):
        for ld in prob.loads[l]:
            if plane:
                i, j, c, w = ld
                idx.append(slot * n + c * n_node + i + (nx + 1) * j)
            else:
                i, j, k, c, w = ld
                idx.append(slot * n + c * n_node + i + (nx + 1) * (j + (ny + 1) * k))
            val.append(float(w))
    if idx:
        f.index_put_((torch.tensor(idx, dtype=torch.int64, device=device),),
                     torch.tensor(val, dtype=torch.float64, device=device), accumulate=True)
    return f


def loads_soa(prob, n_node: int, cases: Optional[Sequence[int]] = None) -> list:
    """Flatten a problem's point loads into SoA vectors [case][dim * n_node]
    (dim = 2 for a plane-stress problem, whose loads are (i, j, c, value));
    numpy float64 arrays, repeated points summed."""
    import numpy as np

    nx, ny = prob.nx, prob.ny
    plane = not hasattr(prob, "nz")
    cases = range(prob.n_case) if cases is None else cases
    out = []
    for l in cases:
        v = np.zeros((2 if plane else 3) * n_node)
        lds = prob.loads[l]
        if lds:
            a = np.asarray(lds, dtype=np.float64)
            ii = a[:, :-1].astype(np.int64)
            if plane:
                idx = ii[:, 2] * n_node + ii[:, 0] + (nx + 1) * ii[:, 1]
            else:
                idx = ii[:, 3] * n_node + ii[:, 0] + (nx + 1) * (ii[:, 1] + (ny + 1) * ii[:, 2])
            np.add.at(v, idx, a[:, -1])
        out.append(v)
    return out
