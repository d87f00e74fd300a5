"""The C ABI library loads and exports every entry point include/wigner.h declares
(no compute call: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wigner.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b((?:wk|sp)_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for need in ("wk_kernel_eval", "wk_kernel_bwd", "wk_gamma_tables", "sp_init", "sp_step",
                 "sp_annihilate", "sp_density", "wk_surrogate_fwd", "wk_surrogate_bwd",
                 "wk_mse_grad", "wk_sgd_update", "wk_last_error", "wk_version"):
        assert need in names


def test_library_exports_every_declared_symbol():
    from paper_1806_00082_amd import _lib
    lib = _lib.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert lib.wk_version() == 1


def test_python_binding_names_match_header():
    from paper_1806_00082_amd import _lib
    assert set(_lib.SIGNATURES) <= set(declared_functions())


def test_host_validation_without_gpu():
    """Argument checks run on the host before anything is enqueued."""
    from paper_1806_00082_amd import _lib
    lib = _lib.lib()
    m = _lib.WkMesh(1, 10, 1, 7, 0.65)           # odd n_m is rejected
    rc = lib.wk_kernel_eval(ctypes.byref(m), None, 1, None, 10, 0, 0, None, None)
    assert rc == _lib.WK_EINVAL
    assert b"n_m" in lib.wk_last_error()
    m = _lib.WkMesh(1, 10, 1, 8, 0.65)
    assert lib.wk_kernel_eval(ctypes.byref(m), None, 0, None, 10, 0, 0, None, None) == 0  # empty
    g = _lib.SpGeom(1, 10, 1, 8, 16, -8, 0, 0, 0.1, 0)
    assert lib.sp_workspace_size(ctypes.byref(g)) > 0


def test_particle_calls_reject_aliased_buffers_without_gpu():
    """sp_step and sp_annihilate write `out` while reading `in`: the same buffers twice are
    refused on the host (the pointers are never dereferenced)."""
    from paper_1806_00082_amd import _lib
    lib = _lib.lib()
    g = _lib.SpGeom(1, 10, 1, 8, 16, -8, 0, 0, 0.1, 0)
    p = _lib.SpParticles(0x1000, None, 0x2000, None, 0x3000, 100, 0x4000)
    q = _lib.SpParticles(0x5000, None, 0x6000, None, 0x7000, 100, 0x8000)
    ws = int(lib.sp_workspace_size(ctypes.byref(g)))
    f = 0x9000
    rc = lib.sp_step(ctypes.byref(g), f, f, f, f, None, 0, ctypes.byref(p), ctypes.byref(p), None,
                     0, f, f, ws, None)
    assert rc == _lib.WK_EINVAL and b"different buffers" in lib.wk_last_error()
    rc = lib.sp_annihilate(ctypes.byref(g), ctypes.byref(q), ctypes.byref(q), f, 0, 0, f, f, ws, None)
    assert rc == _lib.WK_EINVAL and b"different buffers" in lib.wk_last_error()
    rc = lib.sp_step(ctypes.byref(g), f, f, f, f, f, 0, ctypes.byref(p), ctypes.byref(q), None,
                     0, f, f, ws, None)
    assert rc == _lib.WK_EINVAL and b"guide_len" in lib.wk_last_error()
    rc = lib.sp_step(ctypes.byref(g), f, f, f, f, None, 0, ctypes.byref(p), ctypes.byref(q), None,
                     0, f, f, ws - 1, None)
    assert rc == _lib.WK_EINVAL and b"workspace" in lib.wk_last_error()
