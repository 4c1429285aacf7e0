"""The C ABI library loads, exports every symbol include/aarmr.h declares and
validates parameters on the host (no GPU needed, no compute calls)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "aarmr.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(aarmr_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2205_00385_amd import aarmr

    return aarmr.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header():
    from paper_2205_00385_amd import aarmr

    assert set(aarmr.EXPORTS) == set(declared_functions())


def test_struct_sizes_match_header_layout(lib):
    from paper_2205_00385_amd import aarmr

    p = aarmr.default_params()
    assert p.E0 == 1.0 and p.Emin == 1e-9 and p.nu == 0.3 and p.penal == 3.0
    assert p.mg_levels == 3 and p.Ns == 2 and p.Nm == 2 and p.rmin == 2.5
    assert p.cg_rtol == 1e-8 and p.n_rhs_max == 1


def _create(lib, **kw):
    from paper_2205_00385_amd import aarmr

    p = aarmr.default_params(**kw)
    h = ctypes.c_void_p()
    code = lib.aarmr_mesh_create(ctypes.byref(p), ctypes.byref(h))
    return code, h


@pytest.mark.parametrize("kw", [
    dict(nx=0),
    dict(nx=6, ny=6, nz=6, mg_levels=4),      # not divisible by 8
    dict(mg_levels=1),
    dict(mg_levels=9),
    dict(Ns=0), dict(Nm=11), dict(n_rhs_max=9), dict(nu=0.5), dict(Emin=0.0),
    dict(cg_maxit=0), dict(precision=7), dict(omega=0.0),
    dict(nx=256, ny=256, nz=256, mg_levels=2),  # coarsest dense too large
    # 449^3 nodes: 3 * n_node * 8 bytes exceed the fine product's 2^31 offsets
    dict(nx=448, ny=448, nz=448, mg_levels=7),
])
def test_mesh_create_rejects(lib, kw):
    from paper_2205_00385_amd import aarmr

    code, h = _create(lib, **kw)
    assert code == aarmr.E_INVALID
    assert lib.aarmr_last_error().decode() != ""


def test_workspace_bytes_and_unbound_calls(lib):
    from paper_2205_00385_amd import aarmr

    code, h = _create(lib, nx=24, ny=12, nz=12, mg_levels=3)
    assert code == aarmr.OK
    try:
        nb = lib.aarmr_workspace_bytes(h)
        nn = 25 * 13 * 13
        assert nb > 8 * 3 * nn * 10  # at least the CG and V-cycle vectors
        assert nb % 256 == 0
        # compute entry points refuse to run before a workspace is bound
        assert lib.aarmr_vcycle(h, None, None, None) == aarmr.E_NO_WORKSPACE
        assert lib.aarmr_filter(h, 0, None, None, None) == aarmr.E_NO_WORKSPACE
    finally:
        lib.aarmr_mesh_destroy(h)


def test_workspace_grows_with_parm_and_cases(lib):
    from paper_2205_00385_amd import aarmr

    sizes = []
    for kw in (dict(Ns=2, n_rhs_max=1), dict(Ns=4, n_rhs_max=1), dict(Ns=4, n_rhs_max=3)):
        code, h = _create(lib, nx=16, ny=8, nz=8, mg_levels=3, **kw)
        assert code == aarmr.OK
        sizes.append(lib.aarmr_workspace_bytes(h))
        lib.aarmr_mesh_destroy(h)
    assert sizes[0] < sizes[1] < sizes[2]


def test_missing_library_fails_loudly(tmp_path):
    """Without the built HIP library the binding raises at load time: there is
    no CPU fallback for any entry point."""
    from paper_2205_00385_amd import aarmr

    with pytest.raises(ImportError, match="no CPU fallback"):
        aarmr.load_library(str(tmp_path / "libaarmr.so"))
