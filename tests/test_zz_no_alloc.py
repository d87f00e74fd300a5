"""wk_surrogate_fwd_static (the forward of eq.(5) that allocates nothing, its scratch a
library-owned device array) against wk_surrogate_fwd with a caller workspace, through the C
ABI: two calls in a row, the second smaller, each bit-identical to the workspace form."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1806_00082_amd import _lib as L
from paper_1806_00082_amd import inputs, ops

pytestmark = pytest.mark.gpu


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _weights(n_m, N, seed, dev):
    g = torch.Generator().manual_seed(seed)
    c = -2.0 / (inputs.HBAR_EVFS * n_m)
    return [t.to(torch.float32).to(dev) for t in (1 + 0.1 * torch.randn(N, generator=g),
                                                  1.0 / N + 0.01 * torch.randn(N, generator=g),
                                                  c * (1 + 0.1 * torch.randn(n_m // N, generator=g)))]


def _both(lib, nx, n_m, N, B, prec, cells, seed):
    dev = torch.device("cuda:0")
    V = torch.from_numpy(inputs.random_potentials(B, nx, 0.5, seed=seed)).to(dev)
    wV, wT, W = _weights(n_m, N, seed, dev)
    nc = nx if cells is None else len(cells)
    cl = None if cells is None else torch.as_tensor(cells, dtype=torch.int32, device=dev)
    P = n_m // 2
    dt = torch.float64 if prec == L.WK_FP64 else torch.float32
    ref = torch.full((B * nc, P), float("nan"), dtype=dt, device=dev)
    got = torch.full((B * nc, P), float("nan"), dtype=dt, device=dev)
    m = ops.mesh_struct(1, nx, 1, n_m)
    wsz = lib.wk_surrogate_fwd_workspace(ctypes.byref(m), N)
    ws = torch.empty(wsz, dtype=torch.uint8, device=dev)
    s = ops._stream()
    print(f"no-alloc forward nx={nx} n_m={n_m} N={N} B={B} prec={prec} cells={cells is not None}", flush=True)
    L.check(lib.wk_surrogate_fwd(ctypes.byref(m), N, _p(wV), _p(wT), _p(W), _p(V), B, _p(cl), nc, prec,
                                 _p(ref), _p(ws), wsz, s), "wk_surrogate_fwd")
    L.check(lib.wk_surrogate_fwd_static(ctypes.byref(m), N, _p(wV), _p(wT), _p(W), _p(V), B, _p(cl), nc,
                                        prec, _p(got), s), "wk_surrogate_fwd_static")
    torch.cuda.synchronize()
    assert not torch.isnan(ref).any()
    assert torch.equal(got, ref)


def test_static_forward_matches_workspace_forward_twice():
    lib = L.lib()
    # the larger call first, then a smaller one (fewer rows, narrower tables, a cell list)
    _both(lib, 1024, 256, 2, 8, L.WK_FP32, None, 1)
    _both(lib, 300, 64, 4, 2, L.WK_BF16, [0, 299, 5, 5, 150, 1], 2)


def test_static_forward_fp64_and_limit():
    lib = L.lib()
    _both(lib, 90, 32, 2, 3, L.WK_FP64, None, 3)
    assert lib.wk_surrogate_fwd_static_max() == 4 << 20
    # n_m = 2048 with N = 8 (H = 256) needs more scratch than the static array holds: refused
    # on the host before anything is enqueued
    m = ops.mesh_struct(1, 4096, 1, 2048)
    assert lib.wk_surrogate_fwd_workspace(ctypes.byref(m), 8) > lib.wk_surrogate_fwd_static_max()
    fake = ctypes.c_void_p(16)
    rc = lib.wk_surrogate_fwd_static(ctypes.byref(m), 8, fake, fake, fake, fake, 1, None, 4096, L.WK_FP32,
                                     fake, None)
    assert rc == L.WK_EINVAL and b"static" in lib.wk_last_error()
