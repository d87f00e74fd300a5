"""GPU tests of the C-ABI contract: explicit set-up (wk_prepare), caller-owned workspaces
(two streams evaluating eq.(5) with different weights at once), and the adjoint of eq.(4)
on cell lists in FP64 and FP32 against the oracle's adjoint."""
import ctypes

import numpy as np
import pytest
import torch

from gpu_helpers import HB, dev, to_np
from paper_1806_00082_amd import _lib as L
from paper_1806_00082_amd import inputs, learn, ops

pytestmark = pytest.mark.gpu


def _fold_full(Gf):
    """dL/dK on the unique momenta m = 1..P from a full-table gradient (m = -P..P-1):
    G(m) - G(-m) for m < P and -G(-P) for m = P (layout conversion of the test inputs)."""
    n_m = Gf.shape[-1]
    P = n_m // 2
    G1 = np.empty(Gf.shape[:-1] + (P,))
    G1[..., : P - 1] = Gf[..., P + 1:] - Gf[..., 1:P][..., ::-1]
    G1[..., P - 1] = -Gf[..., 0]
    return G1


@pytest.mark.parametrize("nx,n_m,layout", [(37, 20, "half"), (300, 256, "half"), (150, 64, "full"),
                                          (90, 30, "full"), (64, 2, "half"), (1024, 256, "full")])
def test_kernel_adjoint_cells_fp64(orc, nx, n_m, layout):
    """Cell lists with repeats, both edges, any order; one and several column blocks."""
    B, P = 2, n_m // 2
    rng = np.random.default_rng(nx + n_m)
    cells = np.concatenate([[0, nx - 1, nx // 2, nx // 2, 1, nx - 2], rng.integers(0, nx, 37)]).astype(np.int32)
    width = P if layout == "half" else n_m
    G = rng.normal(size=(B, len(cells), width))
    G1 = G if layout == "half" else _fold_full(G)
    ref = orc.kernel_bwd_1d(G1, n_m, HB, nx=nx, cells=cells)
    got = to_np(ops.kernel_bwd(torch.from_numpy(G.reshape(B * len(cells), width)).to(dev()), nx, n_m, B,
                               layout=layout, cells=torch.from_numpy(cells).to(dev())))
    scale = max(np.abs(ref).max(), 1e-300)
    assert np.abs(got - ref).max() <= 1e-12 * scale


@pytest.mark.parametrize("nx,n_m,cells", [(300, 256, False), (257, 64, True), (90, 30, True),
                                          (1024, 256, True), (40, 80, False)])
def test_kernel_adjoint_fp32(orc, nx, n_m, cells):
    """FP32 operands and sums: within the rounding of P-term FP32 products and 2P-term FP32
    gathers, u32 (3P) sum |terms|, against the FP64 oracle on the same (float) gradient."""
    B, P = 2, n_m // 2
    rng = np.random.default_rng(7 * nx + n_m)
    cl = (np.concatenate([[0, nx - 1, 5, 5], rng.integers(0, nx, 60)]).astype(np.int32) if cells else None)
    nc = nx if cl is None else len(cl)
    G = rng.normal(size=(B, nc, P)).astype(np.float32)
    ref = orc.kernel_bwd_1d(G.astype(np.float64), n_m, HB, nx=nx, cells=cl)
    refabs = orc.kernel_bwd_1d(np.abs(G).astype(np.float64), n_m, HB, nx=nx, cells=cl)  # sign-free scale
    got = to_np(ops.kernel_bwd(torch.from_numpy(G.reshape(B * nc, P)).to(dev()), nx, n_m, B, layout="half",
                               cells=None if cl is None else torch.from_numpy(cl).to(dev())))
    err = np.abs(got - ref).max()
    # bound: each of the ~3P FP32 roundings on a path is relative to a partial sum no larger
    # than sum |c| |G| over the row, ~P |c| max|G| per GD entry, and a dV sums 2P entries
    bound = 3 * P * 2.0 ** -24 * (2 * P) * P * (2.0 / (HB * n_m)) * np.abs(G).max()
    print(f"fp32 adjoint nx={nx} n_m={n_m}: err {err:.3e}, bound {bound:.3e}, scale {np.abs(ref).max():.3e}")
    assert err <= bound
    assert err <= 1e-4 * np.abs(refabs).max()


def test_unprepared_n_m_is_rejected():
    """Without wk_prepare for an n_m the contraction refuses (nothing allocated in the call)."""
    lib = L.lib()
    n_m, nx = 94, 50                       # an n_m no other test uses
    m = ops.mesh_struct(1, nx, 1, n_m)
    V = torch.zeros((1, nx), dtype=torch.float64, device=dev())
    K = torch.empty((nx, n_m), dtype=torch.float64, device=dev())
    rc = lib.wk_kernel_eval(ctypes.byref(m), ctypes.c_void_p(V.data_ptr()), 1, None, nx, L.WK_FP64,
                            L.WK_FULL, ctypes.c_void_p(K.data_ptr()), ops._stream())
    assert rc == L.WK_EINVAL and b"wk_prepare" in lib.wk_last_error()
    ops.prepare(n_m)
    ops.kernel_eval(V, n_m, out=K)
    torch.cuda.synchronize()
    assert float(K.abs().max()) == 0.0     # constant potential: K = 0 exactly


def test_surrogate_fwd_two_streams():
    """Two streams run eq.(5) at once with different weights, each on its own workspace: both
    equal their single-stream results bit for bit (no hidden shared scratch)."""
    nx, n_m, N, B = 1024, 256, 4, 32
    V = torch.from_numpy(inputs.random_potentials(B, nx, 0.5, seed=3)).to(dev())
    g = torch.Generator().manual_seed(0)
    w1 = [t.to(dev()) for t in (1 + 0.1 * torch.randn(N, generator=g), 0.25 + 0.01 * torch.randn(N, generator=g),
                                -0.01 * (1 + 0.1 * torch.randn(n_m // N, generator=g)))]
    w2 = [t.to(dev()) for t in (1 + 0.1 * torch.randn(N, generator=g), 0.25 + 0.01 * torch.randn(N, generator=g),
                                -0.01 * (1 + 0.1 * torch.randn(n_m // N, generator=g)))]
    for prec in ("fp32", "bf16"):
        ref1 = learn.surrogate_fwd(V, n_m, N, *w1, prec=prec)
        ref2 = learn.surrogate_fwd(V, n_m, N, *w2, prec=prec)
        torch.cuda.synchronize()
        assert not torch.equal(ref1, ref2)
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        ws1 = learn.surrogate_fwd_workspace(n_m, N, dev())
        ws2 = learn.surrogate_fwd_workspace(n_m, N, dev())
        o1, o2 = torch.empty_like(ref1), torch.empty_like(ref2)
        torch.cuda.synchronize()
        for _ in range(3):
            with torch.cuda.stream(s1):
                learn.surrogate_fwd(V, n_m, N, *w1, prec=prec, out=o1, ws=ws1)
            with torch.cuda.stream(s2):
                learn.surrogate_fwd(V, n_m, N, *w2, prec=prec, out=o2, ws=ws2)
            torch.cuda.synchronize()
            assert torch.equal(o1, ref1) and torch.equal(o2, ref2), prec
