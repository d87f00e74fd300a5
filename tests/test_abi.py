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
    assert lib.wk_version() == 4


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
    # wk_kernel_tables checks its precision on the host (the pointers are never touched)
    fake = ctypes.c_void_p(4096)
    for dim, ny in ((1, 1), (2, 6)):
        m = _lib.WkMesh(dim, 10, ny, 8, 0.65)
        rc = lib.wk_kernel_tables(ctypes.byref(m), fake, 1, None, 10 * ny, 42, 0.5, fake, fake, fake, fake,
                                  None, 0, None)
        assert rc == _lib.WK_EINVAL
        assert b"precision" in lib.wk_last_error()


def test_workspace_contracts_without_gpu():
    """Workspace queries and checks of the calls whose scratch is the caller's (host only)."""
    from paper_1806_00082_amd import _lib
    lib = _lib.lib()
    m = _lib.WkMesh(1, 64, 1, 32, 0.65)
    n = lib.wk_surrogate_fwd_workspace(ctypes.byref(m), 4)
    assert n > 0
    assert lib.wk_surrogate_fwd_workspace(ctypes.byref(m), 3) == 0      # N must be a power of two
    fake = ctypes.c_void_p(16)                                           # never dereferenced
    rc = lib.wk_surrogate_fwd(ctypes.byref(m), 4, fake, fake, fake, fake, 1, None, 64, _lib.WK_FP32,
                              fake, fake, n - 1, None)
    assert rc == _lib.WK_EINVAL and b"workspace" in lib.wk_last_error()
    rc = lib.wk_surrogate_fwd(ctypes.byref(m), 4, fake, fake, fake, fake, 1, None, 64, _lib.WK_FP16,
                              fake, fake, n, None)
    assert rc == _lib.WK_EINVAL and b"prec" in lib.wk_last_error()
    # the adjoint: FP64 and FP32 workspaces, cell lists, bad precision
    w64 = lib.wk_kernel_bwd_workspace(ctypes.byref(m), 2, 10, _lib.WK_FP64)
    w32 = lib.wk_kernel_bwd_workspace(ctypes.byref(m), 2, 10, _lib.WK_FP32)
    assert w64 > w32 > 0 and lib.wk_kernel_bwd_workspace(ctypes.byref(m), 2, 10, _lib.WK_BF16) == 0
    rc = lib.wk_kernel_bwd(ctypes.byref(m), fake, 2, None, 10, _lib.WK_FP64, _lib.WK_HALF, fake, fake,
                           w64, None)
    assert rc == _lib.WK_EINVAL and b"n_cells must be nx" in lib.wk_last_error()
    rc = lib.wk_kernel_bwd(ctypes.byref(m), fake, 2, fake, 10, _lib.WK_FP64, _lib.WK_HALF, fake, fake,
                           w64 - 1, None)
    assert rc == _lib.WK_EINVAL and b"workspace" in lib.wk_last_error()
    # pair removal: scratch sized by the input capacity
    g = _lib.SpGeom(1, 10, 1, 8, 16, -8, 0, 0, 0.1, 0)
    assert lib.sp_pairs_scratch_size(ctypes.byref(g), 1000) > lib.sp_pairs_scratch_size(ctypes.byref(g), 10) > 0
    assert lib.sp_pairs_scratch_size(ctypes.byref(g), -1) == 0
    # set-up validates before touching a device
    bad = _lib.WkMesh(1, 64, 1, 31, 0.65)
    assert lib.wk_prepare(ctypes.byref(bad), None) == _lib.WK_EINVAL


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
                     0, None, 0, f, f, ws, None)
    assert rc == _lib.WK_EINVAL and b"different buffers" in lib.wk_last_error()
    rc = lib.sp_annihilate(ctypes.byref(g), ctypes.byref(q), ctypes.byref(q), f, 0, None, 0, f, f, ws, None)
    assert rc == _lib.WK_EINVAL and b"different buffers" in lib.wk_last_error()
    for bad in (-1, 3):
        rc = lib.sp_annihilate(ctypes.byref(g), ctypes.byref(p), ctypes.byref(q), f, bad, None, 0, f, f, ws,
                               None)
        assert rc == _lib.WK_EINVAL and b"hist_ready" in lib.wk_last_error()
        rc = lib.sp_annihilate_pairs(ctypes.byref(g), ctypes.byref(p), ctypes.byref(q), f, bad, f, f, ws,
                                     f, 1 << 40, None)
        assert rc == _lib.WK_EINVAL and b"hist_ready" in lib.wk_last_error()
    rc = lib.sp_step(ctypes.byref(g), f, f, f, f, f, 0, ctypes.byref(p), ctypes.byref(q), None,
                     0, None, 0, f, f, ws, None)
    assert rc == _lib.WK_EINVAL and b"guide_len" in lib.wk_last_error()
    rc = lib.sp_step(ctypes.byref(g), f, f, f, f, None, 0, ctypes.byref(p), ctypes.byref(q), None,
                     0, None, 0, f, f, ws - 1, None)
    assert rc == _lib.WK_EINVAL and b"workspace" in lib.wk_last_error()
    for bad in (-1, 2):
        rc = lib.sp_step(ctypes.byref(g), f, f, f, f, None, 0, ctypes.byref(p), ctypes.byref(q), f,
                         bad, None, 0, f, f, ws, None)
        assert rc == _lib.WK_EINVAL and b"hist_mode" in lib.wk_last_error()
    # keys come with a histogram and are 16-byte aligned
    rc = lib.sp_step(ctypes.byref(g), f, f, f, f, None, 0, ctypes.byref(p), ctypes.byref(q), None,
                     0, f, 0, f, f, ws, None)
    assert rc == _lib.WK_EINVAL and b"keys" in lib.wk_last_error()
    rc = lib.sp_step(ctypes.byref(g), f, f, f, f, None, 0, ctypes.byref(p), ctypes.byref(q), f,
                     0, f + 4, 0, f, f, ws, None)
    assert rc == _lib.WK_EINVAL and b"aligned" in lib.wk_last_error()
    rc = lib.sp_annihilate(ctypes.byref(g), ctypes.byref(p), ctypes.byref(q), f, 0, f + 4, 0, f, f, ws, None)
    assert rc == _lib.WK_EINVAL and b"aligned" in lib.wk_last_error()


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of the parameter structs have the sizes and field offsets the C
    compiler gives the header's structs."""
    import shutil
    import subprocess
    from paper_1806_00082_amd import _lib
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    mirrors = {"wk_mesh": _lib.WkMesh, "sp_geom": _lib.SpGeom, "sp_particles": _lib.SpParticles}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "wigner.h"', "int main(void) {"]
    for cname, cls in mirrors.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


def test_momentum_width_rules():
    """Momentum storage width: chosen per buffer (int32, int16 or int8), the narrowest that
    holds the window widened by the largest pair offset; refused when the buffers of a call
    disagree (checked on the host before any library call)."""
    import torch
    from paper_1806_00082_amd import inputs, ops
    md = inputs.config_c1().mesh.as_dict(1.0)          # M in [-30, 30), n_m = 30
    assert ops.fits_m16(md) and ops.fits_m_bytes(md, 1) and ops.narrowest_m_bytes(md) == 1
    assert not ops.fits_m16(dict(md, M_min=-40000))
    assert ops.narrowest_m_bytes(dict(md, M_min=-113)) == 1    # -113 - 15 = -128
    assert ops.narrowest_m_bytes(dict(md, M_min=-114)) == 2
    assert ops.narrowest_m_bytes(dict(md, M_min=-32768 + 15)) == 2
    assert ops.narrowest_m_bytes(dict(md, M_min=-32768 + 14)) == 4
    md2 = inputs.config_c5().mesh.as_dict(0.5)        # 2-D: M in [-32, 32), n_m = 32
    assert ops.narrowest_m_bytes(md2) == 1
    assert not ops.fits_m_bytes(md2, 4)                # 2-D momenta are at most 16 bits
    a = ops.DeviceParticles(1, 8, True, device="cpu")
    b = ops.DeviceParticles(1, 8, True, device="cpu", m16=True)
    c = ops.DeviceParticles(2, 8, False, device="cpu")
    d = ops.DeviceParticles(2, 8, False, device="cpu", m_bytes=1)
    e = ops.DeviceParticles(1, 8, False, device="cpu", m_bytes=1)
    assert a.M.dtype == torch.int32 and b.M.dtype == torch.int16
    assert c.M.dtype == torch.int16 and c.My.dtype == torch.int16 and c.m_bytes == 2
    assert d.M.dtype == torch.int8 and d.My.dtype == torch.int8 and e.M.dtype == torch.int8
    with pytest.raises(ValueError):
        ops.DeviceParticles(2, 8, False, device="cpu", m_bytes=4)
    with pytest.raises(ValueError):
        ops.DeviceParticles(1, 8, False, device="cpu", m_bytes=3)
    with pytest.raises(ValueError):
        ops.sp_annihilate(md, 0, a, b, None, 0, None, None)
    with pytest.raises(ValueError):
        ops.sp_annihilate(md, 0, b, e, None, 0, None, None)
    assert ops.geom_struct(md, 0, 2).m_bytes == 2


def test_momentum_width_checked_by_the_library():
    """sp_workspace_size validates the geometry (0 = refused) without touching a device: the
    momentum type must hold the window widened by n_m / 2, and 2-D momenta are not int32."""
    from paper_1806_00082_amd import _lib
    lib = _lib.lib()

    def ok(dim, n_m, n_k, M_min, mb):
        g = _lib.SpGeom(dim, 10, 1 if dim == 1 else 10, n_m, n_k, M_min, 0, mb, 0.1, 0)
        return lib.sp_workspace_size(ctypes.byref(g)) > 0

    assert ok(1, 30, 60, -30, 1) and ok(1, 30, 60, -30, 2) and ok(1, 30, 60, -30, 4) and ok(1, 30, 60, -30, 0)
    assert ok(1, 30, 60, -113, 1) and not ok(1, 30, 60, -114, 1)        # low end: -113 - 15 = -128
    assert ok(1, 30, 226, -113, 1) and not ok(1, 30, 227, -113, 1)      # high end: -113 + 225 + 15 = 127
    assert ok(2, 32, 64, -32, 1) and ok(2, 32, 64, -32, 2) and ok(2, 32, 64, -32, 0)
    assert not ok(2, 32, 64, -32, 4) and not ok(1, 30, 60, -30, 3) and not ok(2, 32, 64, -32, -1)
    assert not ok(2, 32, 64, -32768, 2) and ok(2, 32, 64, -32768 + 16, 2)
