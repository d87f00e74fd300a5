"""GPU parity of the three added forms against the FP64 oracle:
(1) precision: BF16/FP16 MFMA contraction with FP32 accumulation and hi/lo split correction;
(3) differentiation: the hand-written adjoint of eq.(4) and of eq.(5);
(4) learned: the eq.(5) network forward, backward, loss, update and training."""
import math

import numpy as np
import pytest
import torch

from gpu_helpers import HB, dev, normwise, to_np
from paper_1806_00082_amd import inputs, learn, ops

pytestmark = pytest.mark.gpu

# Normwise bounds (max |err| / max |K| per potential).  Single-pass forms: one rounding of
# each operand (u_bf16 = 2^-8, u_fp16 = 2^-11) plus FP32 sums; split forms: the operands
# carry 16 (bf16) or 22 (fp16) bits and the dropped lo*lo term is ~u^2.
LOWP_TOL = {"bf16": 1e-2, "fp16": 2e-3, "bf16x3": 5e-5, "fp16x3": 1e-5}
U_IN = {"bf16": 2.0 ** -8, "fp16": 2.0 ** -11}
# Underflow: a rounded operand is d (1 + delta) + eta with |eta| below the smallest normal
# of the format (the matrix cores may flush subnormals): 2^-126 for bf16, 2^-14 for fp16.
ETA_IN = {"bf16": 2.0 ** -126, "fp16": 2.0 ** -14}


@pytest.mark.parametrize("prec", ["bf16", "fp16", "bf16x3", "fp16x3"])
@pytest.mark.parametrize("nx,n_m,B", [(300, 64, 3), (2048, 512, 2), (100, 30, 2), (1024, 256, 2),
                                      (300, 134, 2), (90, 1024, 1), (70, 1100, 1), (41, 6, 2)])
def test_lowp_kernel_error_bounds(orc, prec, nx, n_m, B):
    """Both layouts; every fold tile shape (H = n_m / 4 below 32, in (32, 64], above 64), odd
    P, whole-row staging (one column block, P % 4 == 0) and per-entry stores (several column
    blocks, odd P, the full layout), rows built from the LDS window and from L2 (n_m = 1100)."""
    print(f"lowp {prec} nx={nx} n_m={n_m}", flush=True)
    V = inputs.random_potentials(B, nx, 0.5, seed=nx + 7)
    ref = orc.kernel_1d(V, n_m, HB)
    Vd = torch.from_numpy(V).to(dev())
    full = to_np(ops.kernel_eval(Vd, n_m, prec=prec, layout="full")).astype(np.float64)
    half = to_np(ops.kernel_eval(Vd, n_m, prec=prec, layout="half")).astype(np.float64)
    assert normwise(full.reshape(B, -1), ref.reshape(B, -1)) <= LOWP_TOL[prec]
    assert normwise(half.reshape(B, -1), orc.full_to_half(ref).reshape(B, -1)) <= LOWP_TOL[prec]
    if prec in U_IN:
        # per-entry bound: |dK| <= (2u + u^2 + (P-1) u32) |c| sum_j |S D| (+ output rounding)
        P = n_m // 2
        u, u32 = U_IN[prec], 2.0 ** -24
        c = 2.0 / (HB * n_m)
        j = np.arange(1, P + 1)
        m = np.arange(1, P + 1)
        S = np.abs(np.sin(2 * np.pi * np.outer(j, m) / n_m))
        for b in range(B):
            Vb = V[b]
            idx = np.arange(nx)
            D = np.abs(Vb[np.clip(idx[:, None] + j[None, :], 0, nx - 1)] -
                       Vb[np.clip(idx[:, None] - j[None, :], 0, nx - 1)])
            eta = ETA_IN[prec]
            bound = (2 * u + u * u + (P - 1) * u32) * c * (D @ S) + u32 * np.abs(orc.full_to_half(ref[b])) \
                + 2 * c * eta * S.sum(axis=0)[None, :]
            err = np.abs(half.reshape(B, nx, P)[b] - orc.full_to_half(ref[b]))
            assert np.all(err <= bound * 1.0001 + 1e-300)


def test_lowp_cell_list_and_constant(orc):
    nx, n_m = 200, 64
    V = inputs.random_potentials(2, nx, 0.5, seed=3)
    cells = np.array([0, 199, 50, 50, 7], np.int32)
    ref = orc.kernel_1d(V, n_m, HB, cells=cells)
    got = to_np(ops.kernel_eval(torch.from_numpy(V).to(dev()), n_m, cells=torch.from_numpy(cells).to(dev()),
                                prec="bf16x3")).astype(np.float64)
    assert normwise(got.reshape(2, -1), ref.reshape(2, -1)) <= LOWP_TOL["bf16x3"]
    Z = torch.full((1, 100), 0.2, dtype=torch.float64, device=dev())
    for prec in LOWP_TOL:
        assert torch.count_nonzero(ops.kernel_eval(Z, 32, prec=prec)).item() == 0


def test_lowp_full_size_sampled(orc):
    """Precision batch at full size (4096 x 2048 x 512), BF16 and BF16x3, sampled rows."""
    c3 = inputs.C3
    B, nx, n_m = c3["B"], c3["nx"], c3["n_m"]
    V = inputs.random_potentials(B, nx, c3["dx"], seed=c3["seed"])
    Vd = torch.from_numpy(V).to(dev())
    rows = np.array([0, 1, nx - 1, 5 * nx + 17, B * nx - 1, 1234567, 7654321])
    for prec in ("bf16", "bf16x3"):
        K = ops.kernel_eval(Vd, n_m, prec=prec, layout="half")
        got = to_np(K[torch.from_numpy(rows).to(dev())]).astype(np.float64)
        del K
        for k, r in enumerate(rows):
            b, i = divmod(int(r), nx)
            ref = orc.full_to_half(orc.kernel_1d(V[b], n_m, HB))[0]
            scale = np.abs(ref).max()
            assert np.abs(got[k] - ref[i]).max() <= LOWP_TOL[prec] * scale, (prec, b, i)


# ----------------------------------------------------------------------------- adjoint
@pytest.mark.parametrize("nx,n_m,B", [(90, 30, 2), (257, 64, 3), (40, 80, 1), (300, 256, 2), (40, 2, 1), (70, 6, 2)])
def test_kernel_adjoint_matches_oracle(orc, nx, n_m, B):
    P = n_m // 2
    rng = np.random.default_rng(nx)
    G = rng.normal(size=(B, nx, P))
    ref = orc.kernel_bwd_1d(G, n_m, HB)
    got = to_np(ops.kernel_bwd(torch.from_numpy(G).to(dev()), nx, n_m, B, layout="half"))
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_kernel_adjoint_full_layout_dot_product():
    """<G, K(dV)> = <K^T G, dV> with the GPU forward and backward, full table layout."""
    nx, n_m, B = 150, 40, 2
    g = torch.Generator(device="cpu").manual_seed(0)
    G = torch.randn((B * nx, n_m), generator=g, dtype=torch.float64).to(dev())
    dV = torch.randn((B, nx), generator=g, dtype=torch.float64).to(dev())
    K = ops.kernel_eval(dV, n_m, layout="full")
    lhs = float((G * K).sum())
    rhs = float((ops.kernel_bwd(G, nx, n_m, B, layout="full") * dV).sum())
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_wigner_kernel_gradcheck():
    V = torch.randn((2, 24), dtype=torch.float64, device=dev(), requires_grad=True)
    fn = lambda v: learn.WignerKernelFn.apply(v, 8, "full")
    assert torch.autograd.gradcheck(fn, (V,), eps=1e-6, atol=1e-8, rtol=1e-6)
    fn = lambda v: learn.WignerKernelFn.apply(v, 12, "half")
    assert torch.autograd.gradcheck(fn, (V,), eps=1e-6, atol=1e-8, rtol=1e-6)


# ----------------------------------------------------------------------------- surrogate
def _weights(n_m, N, seed, analytic=False):
    if analytic:
        return [np.asarray(w) for w in ( np.ones(N), np.full(N, 1.0 / N), np.full(n_m // N, -2.0 / (HB * n_m)))]
    rng = np.random.default_rng(seed)
    return [rng.normal(1.0, 0.1, N), rng.normal(1.0 / N, 0.05, N), rng.normal(-2.0 / (HB * n_m), 0.01, n_m // N)]


def _f32(ws):
    return [torch.from_numpy(np.asarray(w, np.float32)).to(dev()) for w in ws]


@pytest.mark.parametrize("N", [1, 2, 4, 8])
@pytest.mark.parametrize("analytic", [True, False])
def test_surrogate_fwd(orc, N, analytic):
    nx, n_m, B = 150, 64, 2
    V = inputs.random_potentials(B, nx, 0.5, seed=N)
    w = _weights(n_m, N, N, analytic)
    w32 = [np.asarray(x, np.float32).astype(np.float64) for x in w]   # the device holds floats
    ref = orc.surrogate_fwd(V, n_m, N, *w32)
    Vd = torch.from_numpy(V).to(dev())
    wd = _f32(w)
    got64 = to_np(learn.surrogate_fwd(Vd, n_m, N, *wd, prec="fp64"))
    assert normwise(got64.reshape(B, -1), ref.reshape(B, -1)) <= 1e-12
    got32 = to_np(learn.surrogate_fwd(Vd, n_m, N, *wd, prec="fp32")).astype(np.float64)
    assert normwise(got32.reshape(B, -1), ref.reshape(B, -1)) <= 2e-5
    gotbf = to_np(learn.surrogate_fwd(Vd, n_m, N, *wd, prec="bf16")).astype(np.float64)
    assert normwise(gotbf.reshape(B, -1), ref.reshape(B, -1)) <= 3e-2
    if analytic and N == 1:
        exact = orc.full_to_half(orc.kernel_1d(V, n_m, HB))
        assert normwise(got64.reshape(B, -1), exact.reshape(B, -1)) <= 1e-6   # float weights


@pytest.mark.parametrize("N", [1, 2, 4, 8])
def test_surrogate_fwd_wide(orc, N):
    """The learned-kernel shape (256 momenta): hidden width 256 / 128 / 64 / 32; tiles inside
    one potential (window) and across two (gathered rows), a ragged last tile.  FP32 with
    H = 256 takes the path without the LDS-resident table."""
    nx, n_m, B = 300, 256, 2
    print(f"surrogate fwd n_m={n_m} N={N}", flush=True)
    V = inputs.random_potentials(B, nx, 0.5, seed=40 + N)
    w = _weights(n_m, N, 40 + N, False)
    w32 = [np.asarray(x, np.float32).astype(np.float64) for x in w]
    ref = orc.surrogate_fwd(V, n_m, N, *w32)
    Vd = torch.from_numpy(V).to(dev())
    wd = _f32(w)
    got32 = to_np(learn.surrogate_fwd(Vd, n_m, N, *wd, prec="fp32")).astype(np.float64)
    assert normwise(got32.reshape(B, -1), ref.reshape(B, -1)) <= 2e-5
    gotbf = to_np(learn.surrogate_fwd(Vd, n_m, N, *wd, prec="bf16")).astype(np.float64)
    assert normwise(gotbf.reshape(B, -1), ref.reshape(B, -1)) <= 3e-2


def test_surrogate_fwd_cells(orc):
    nx, n_m, N = 120, 32, 2
    V = inputs.random_potentials(3, nx, 0.5, seed=5)
    w = _weights(n_m, N, 1)
    w32 = [np.asarray(x, np.float32).astype(np.float64) for x in w]
    cells = np.array([0, 119, 60, 3, 3], np.int32)
    ref = orc.surrogate_fwd(V, n_m, N, *w32, cells=cells)
    got = to_np(learn.surrogate_fwd(torch.from_numpy(V).to(dev()), n_m, N, *_f32(w),
                                    cells=torch.from_numpy(cells).to(dev()), prec="fp64"))
    assert normwise(got.reshape(3, -1), ref.reshape(3, -1)) <= 1e-12


@pytest.mark.parametrize("N", [1, 2, 4])
def test_surrogate_bwd_vs_oracle(orc, N):
    """FP32 hand-written gradients against the FP64 oracle gradients."""
    _bwd_case(orc, N, 130, 32, 3)


@pytest.mark.parametrize("N", [1, 2, 4, 8])
def test_surrogate_bwd_wide(orc, N):
    """The learned-kernel shape (256 momenta, H = 256 / 128 / 64 / 32): tiles inside one
    potential and across two, a ragged last tile; H = 256 takes the path without LDS tables."""
    print(f"surrogate bwd n_m=256 N={N}", flush=True)
    _bwd_case(orc, N, 300, 256, 2)


def test_surrogate_bwd_cells(orc):
    """Gradients over a cell list (arbitrary order, duplicates, both mesh edges)."""
    nx, n_m, N, B = 90, 64, 2, 2
    rng = np.random.default_rng(5)
    V = inputs.random_potentials(B, nx, 0.5, seed=6)
    w = _weights(n_m, N, 7)
    w32 = [np.asarray(x, np.float32).astype(np.float64) for x in w]
    cells = np.array([0, 89, 45, 45, 3, 88] * 7 + [17], np.int32)
    E = rng.normal(size=(B, len(cells), n_m // 2)).astype(np.float32)
    dwV, dwT, dW, _ = orc.surrogate_bwd(V, n_m, N, *w32, E.astype(np.float64), cells=cells, want_dV=False)
    g = learn.surrogate_bwd(torch.from_numpy(V).to(dev()), n_m, N, *_f32(w),
                            torch.from_numpy(E.reshape(B * len(cells), -1)).to(dev()),
                            cells=torch.from_numpy(cells).to(dev()))
    for got, ref in zip(g[:3], (dwV, dwT, dW)):
        got = to_np(got).astype(np.float64).reshape(ref.shape)
        assert np.abs(got - ref).max() <= 1e-4 * np.abs(ref).max(), (got, ref)


def _bwd_case(orc, N, nx, n_m, B):
    rng = np.random.default_rng(40 + N)
    V = inputs.random_potentials(B, nx, 0.5, seed=N + 30)
    w = _weights(n_m, N, N)
    w32 = [np.asarray(x, np.float32).astype(np.float64) for x in w]
    E = rng.normal(size=(B, nx, n_m // 2)).astype(np.float32)
    dwV, dwT, dW, dV = orc.surrogate_bwd(V, n_m, N, *w32, E.astype(np.float64))
    g = learn.surrogate_bwd(torch.from_numpy(V).to(dev()), n_m, N, *_f32(w),
                            torch.from_numpy(E.reshape(B * nx, -1)).to(dev()), want_dV=True)
    for got, ref in zip(g, (dwV, dwT, dW, dV)):
        got = to_np(got).astype(np.float64).reshape(ref.shape)
        assert np.abs(got - ref).max() <= 1e-4 * np.abs(ref).max(), (got, ref)


def test_surrogate_autograd_matches_bwd(orc):
    nx, n_m, N = 64, 16, 2
    V = torch.from_numpy(inputs.random_potentials(2, nx, 0.5, seed=2)).to(dev()).requires_grad_(True)
    wV, wT, W = [t.requires_grad_(True) for t in _f32(_weights(n_m, N, 3))]
    Kh = learn.SurrogateFn.apply(V, wV, wT, W, n_m, N)
    En = np.random.default_rng(5).normal(size=tuple(Kh.shape)).astype(np.float32)
    (Kh * torch.from_numpy(En).to(dev())).sum().backward()
    ref = orc.surrogate_bwd(inputs.random_potentials(2, nx, 0.5, seed=2), n_m, N,
                            *[w.astype(np.float32).astype(np.float64) for w in _weights(n_m, N, 3)],
                            En.astype(np.float64).reshape(2, nx, -1))
    for got, r in zip((wV.grad, wT.grad, W.grad, V.grad), ref):
        got = to_np(got).astype(np.float64).reshape(r.shape)
        assert np.abs(got - r).max() <= 1e-4 * np.abs(r).max()


def test_mse_grad_and_sgd(orc):
    """Loss and dloss/dKh against the oracle's MSE of Sec. 3 (FP32 network outputs, FP64
    labels); the update is w - lr g elementwise."""
    g = torch.Generator(device="cpu").manual_seed(1)
    Kh = torch.randn(1000, generator=g).to(torch.float32).to(dev())
    K = torch.randn(1000, generator=g, dtype=torch.float64).to(dev())
    E, loss = learn.mse_grad(Kh, K, 3.0)
    ref_loss, ref_E = orc.mse_grad(to_np(Kh).astype(np.float64), to_np(K), 3.0)
    assert abs(float(loss) - ref_loss) <= 1e-12 * ref_loss
    assert np.allclose(to_np(E).astype(np.float64), ref_E, rtol=1e-6, atol=0)
    w = torch.ones(10, device=dev())
    learn.sgd_update(w, torch.arange(10, dtype=torch.float32, device=dev()), 0.5)
    assert torch.equal(w.cpu(), 1 - 0.5 * torch.arange(10, dtype=torch.float32))


def test_training_recovers_from_perturbed_weights():
    """Learned form, trained on the GPU by the library's own kernels: SGD from weights 20-30%
    off the barycentric ones reaches the accuracy of the barycentric network, which is the
    optimum of eq.(5) on this data (see the least-squares test on the oracle)."""
    nx, n_m, N = 256, 64, 4
    Vtr = torch.from_numpy(inputs.random_potentials(512, nx, 0.5, seed=0)).to(dev())
    Vte = torch.from_numpy(inputs.random_potentials(64, nx, 0.5, seed=1)).to(dev())
    wV, wT, W = learn.analytic_weights(n_m, N)
    r_bary = learn.surrogate_rms_error(Vte, n_m, N, wV, wT, W)
    g = torch.Generator().manual_seed(N)
    pert = (wV * (1 + 0.3 * torch.randn(N, generator=g)).to(dev()),
            wT * (1 + 0.01 * torch.randn(N, generator=g)).to(dev()),
            W * (0.8 + 0.2 * torch.rand(n_m // N, generator=g)).to(dev()))
    r0 = learn.surrogate_rms_error(Vte, n_m, N, *pert)
    res = learn.train_surrogate(Vtr, n_m, N, epochs=8, batch=32, lr=(10.0, 1e-5, 10.0), init=pert)
    r1 = learn.surrogate_rms_error(Vte, n_m, N, res.wV, res.wT, res.W)
    print(f"held-out rms: perturbed {r0:.4f} -> trained {r1:.4f} (barycentric {r_bary:.4f})")
    assert res.losses[-1] < res.losses[0]
    assert r1 < 0.9 * r0 and r1 <= 1.02 * r_bary


def test_surrogate_driven_run_vs_exact():
    """The trained-form kernel (N = 2, barycentric weights) drives the barrier run on the
    1024-cell, 256-m mesh next to the exact kernel: creation rates agree within 15% and the
    densities stay close (physics tolerances; the paper reports only visual agreement)."""
    from paper_1806_00082_amd.sim import Simulator
    cfg = inputs.config_c4_run(N0=1e6, steps=240)
    n_m = cfg.mesh.n_m
    out = {}
    for kind, N in (("exact", 1), ("surrogate", 2)):
        sim = Simulator(cfg, kernel=kind, N=N, weights=learn.analytic_weights(n_m, N),
                        prec="fp32" if kind == "surrogate" else "fp64", cap_factor=4.0)
        sim.run(240)
        assert not sim.overflowed()
        g = to_np(sim.gamma[:sim.n_rows])
        slot = to_np(sim.cell_slot)
        out[kind] = (to_np(sim.density()), np.where(slot >= 0, g[np.maximum(slot, 0)], 0.0))
    (rx, gx), (rs, gs) = out["exact"], out["surrogate"]
    both = (gx > 0) & (gs > 0)
    assert np.abs(gs[both] - gx[both]).max() <= 0.15 * gx.max()
    xc = (np.arange(cfg.mesh.nx) + 0.5) * cfg.mesh.dx
    assert abs((rs * xc).sum() / rs.sum() - (rx * xc).sum() / rx.sum()) < 8.0
    assert np.abs(rs - rx).sum() < 0.35


# ----------------------------------------------------------------------------- 2-D, 16-bit
# Rounding units of the two 16-bit formats; a split (hi, lo) operand carries the value to
# within about u^2.
U16 = {"bf16": 2.0 ** -8, "fp16": 2.0 ** -11, "bf16x3": 2.0 ** -8, "fp16x3": 2.0 ** -11}
LOWP2D_TOL = {"bf16": 2e-2, "fp16": 3e-3, "bf16x3": 1e-4, "fp16x3": 2e-5}


@pytest.mark.parametrize("prec", ["bf16", "fp16", "bf16x3", "fp16x3"])
@pytest.mark.parametrize("nx,ny,n_m", [(20, 18, 8), (24, 21, 16), (256, 256, 32)])
def test_2d_lowp_kernel_error_bounds(orc, prec, nx, ny, n_m):
    """The d = 2 kernel with 16-bit operands against the oracle's direct FP64 sum.  Per entry:
    each product of the two stages has |trig| <= 1 and weights <= 1, so every partial sum is
    at most sum_j |D_j| over the window (twice, sine and cosine parts), and the error is at most
    2 |c2| sum_j |D_j| (e + (K1 + K2) u32) with e = 6u for one pass (D, trig and the stage-1
    result rounded, two products) and 6u^2 + 2 u32 for the split forms, plus the underflow of
    the rounded operands below the format's smallest normal.  Normwise: the stated
    tolerances.  Sampled cells on the 2-D workload's mesh (with the dot), all cells on the small
    meshes, both mesh edges included."""
    mesh = inputs.Mesh2D(nx=nx, ny=ny, dx=0.5, n_m=n_m, pos_f64=False)
    if nx == 256:
        V = inputs.gaussian_dot_2d(mesh, 0.2, 4.0, 64.0, 64.0)[None]
        rng = np.random.default_rng(3)
        cy, cx = rng.integers(100, 156, 40), rng.integers(100, 156, 40)   # near the dot
        cells = np.concatenate([cy * nx + cx, [0, nx - 1, nx * ny - 1, (ny // 2) * nx + nx // 2 - 9],
                                rng.integers(0, nx * ny, 20)]).astype(np.int32)
    else:
        V = np.stack([inputs.gaussian_dot_2d(mesh, 0.3, 1.5, 4.0 + 2 * b, 5.0) for b in range(2)])
        cells = None
    ref = orc.kernel_2d(V, n_m, HB, cells=cells)
    got = to_np(ops.kernel_eval(torch.from_numpy(V).to(dev()), n_m, cells=None if cells is None else
                                torch.from_numpy(cells).to(dev()), prec=prec)).astype(np.float64)
    B = V.shape[0]
    ref = ref.reshape(B, -1, n_m, n_m)
    got = got.reshape(ref.shape)
    err = normwise(got, ref)
    # per-entry bound from the window's absolute differences
    P = n_m // 2
    u, u32 = U16[prec], 2.0 ** -24
    e = (6 * u * u + 2 * u32) if prec.endswith("x3") else 6 * u
    J = 2 * P + 1
    K1, K2 = -(-J // 32) * 32, 2 * (-(-J // 16) * 16)
    c2 = 1.0 / (HB * n_m * n_m)
    # underflow: a rounded operand is v (1 + delta) + eta, |eta| below the format's smallest
    # normal; D is rounded (hi and lo) in J^2 entries used by both trig parts, the stage-1
    # result (hi and lo) in K2 entries
    eta = ETA_IN["bf16" if prec.startswith("bf16") else "fp16"]
    under = c2 * eta * (4 * J * J + 2 * K2)
    worst = 0.0
    ids = np.arange(nx * ny) if cells is None else cells
    for b in range(B):
        for r, cid in enumerate(ids):
            iy, ix = divmod(int(cid), nx)
            yy = np.clip(iy + np.arange(-P, P + 1), 0, ny - 1)
            xx = np.clip(ix + np.arange(-P, P + 1), 0, nx - 1)
            yym = np.clip(iy - np.arange(-P, P + 1), 0, ny - 1)
            xxm = np.clip(ix - np.arange(-P, P + 1), 0, nx - 1)
            D = V[b][np.ix_(yy, xx)] - V[b][np.ix_(yym, xxm)]
            bound = 2 * c2 * np.abs(D).sum() * (e + (K1 + K2) * u32) + under + 1e-300
            worst = max(worst, np.abs(got[b, r] - ref[b, r]).max() / bound)
    print(f"2-D {prec} n_m={n_m}: normwise {err:.3e}, worst error / per-entry bound {worst:.3f}")
    assert worst <= 1.0
    assert err <= LOWP2D_TOL[prec]


# ----------------------------------------------------------------------------- 2-D eq.(5)
@pytest.mark.parametrize("N", [1, 2, 4, 8])
@pytest.mark.parametrize("nx,ny,n_m", [(13, 9, 8), (20, 17, 16), (256, 256, 32)])
def test_surrogate_2d_vs_oracle(orc, N, nx, ny, n_m):
    """eq.(5) in d = 2 (FP64) against the oracle: analytic weights and perturbed ones, every cell
    of the small meshes (windows clamped at both edges) and sampled cells of the 2-D workload's
    mesh; N = 1 with analytic weights is also the d = 2 kernel of the GPU."""
    if N >= n_m:
        pytest.skip("N must be below n_m")
    mesh = inputs.Mesh2D(nx=nx, ny=ny, dx=0.5, n_m=n_m, pos_f64=False)
    V = inputs.gaussian_dot_2d(mesh, 0.2, 2.0 if nx < 100 else 4.0, nx * 0.2, ny * 0.3)[None]
    if nx == 256:
        rng = np.random.default_rng(N)
        cells = np.concatenate([[0, nx - 1, nx * ny - 1], rng.integers(0, nx * ny, 40),
                                (rng.integers(90, 110, 20) * nx + rng.integers(40, 60, 20))]).astype(np.int32)
    else:
        cells = None
    H = n_m // N
    rng = np.random.default_rng(7 + N)
    for analytic in (True, False):
        w = orc.analytic_weights_2d(n_m, N, HB)
        if not analytic:
            w = (w[0] * rng.normal(1, 0.1, N * N), w[1] + rng.normal(0, 0.01, N), w[2] + rng.normal(0, 0.01, N),
                 w[3] * rng.normal(1, 0.1, H * H))
        w32 = [np.asarray(x, np.float32) for x in w]
        ref = orc.surrogate_fwd_2d(V, n_m, N, *[x.astype(np.float64) for x in w32], cells=cells)
        got = to_np(learn.surrogate_fwd_2d(torch.from_numpy(V).to(dev()), n_m, N,
                                           *[torch.from_numpy(x).to(dev()) for x in w32],
                                           cells=None if cells is None else torch.from_numpy(cells).to(dev())))
        err = normwise(got.reshape(1, -1), ref.reshape(1, -1))
        assert err <= 1e-12, (N, analytic, err)
        if N == 1 and analytic:
            kk = to_np(ops.kernel_eval(torch.from_numpy(V).to(dev()), n_m,
                                       cells=None if cells is None else torch.from_numpy(cells).to(dev())))
            # W = c2 held in FP32: relative rounding at most 2^-24
            assert normwise(got.reshape(1, -1), kk.reshape(1, -1)) <= 2.0 ** -23


@pytest.mark.parametrize("N", [1, 2, 4])
@pytest.mark.parametrize("nx,ny,n_m,use_cells,glen", [(13, 9, 8, False, 0), (20, 17, 16, True, 64),
                                                      (40, 33, 32, True, 256), (37, 30, 32, False, 7)])
def test_surrogate_tables_2d_equals_two_step(N, nx, ny, n_m, use_cells, glen):
    """eq.(5) in d = 2 straight into the creation tables equals surrogate_fwd_2d followed by
    gamma_tables and sampling_guide on the GPU, bit for bit (out-of-mesh ids included), with
    perturbed weights."""
    mesh = inputs.Mesh2D(nx=nx, ny=ny, dx=0.5, n_m=n_m, pos_f64=False)
    V = torch.from_numpy(inputs.gaussian_dot_2d(mesh, 0.25, 1.5, nx * 0.3, ny * 0.4)[None]).to(dev())
    rng = np.random.default_rng(N + nx)
    H = n_m // N
    wV, wTx, wTy, W = learn.analytic_weights_2d(n_m, N)
    w = [wV * torch.from_numpy(rng.normal(1, 0.1, N * N).astype(np.float32)).to(dev()),
         wTx + torch.from_numpy(rng.normal(0, 0.01, N).astype(np.float32)).to(dev()),
         wTy + torch.from_numpy(rng.normal(0, 0.01, N).astype(np.float32)).to(dev()),
         W * torch.from_numpy(rng.normal(1, 0.1, H * H).astype(np.float32)).to(dev())]
    cells = None
    if use_cells:
        ids = np.concatenate([rng.permutation(nx * ny)[: nx * ny // 2], [-1, nx * ny]]).astype(np.int32)
        cells = torch.from_numpy(ids).to(dev())
    dt = 0.5
    g, n0, thr, cdf, guide = learn.surrogate_tables_2d(V, n_m, N, *w, dt, cells=cells, guide_len=glen)
    K = learn.surrogate_fwd_2d(V, n_m, N, *w, cells=cells)
    g2, n02, thr2, cdf2 = ops.gamma_tables(K.reshape(K.shape[0], -1), n_m, dt, dim=2)
    assert torch.equal(g, g2) and torch.equal(n0, n02) and torch.equal(thr, thr2)
    assert torch.equal(cdf, cdf2)
    if glen:
        assert torch.equal(guide, ops.sampling_guide(cdf2, glen))
    else:
        assert guide is None
    assert float(g.max()) > 0


def test_surrogate_2d_simulator_fused_equals_two_step():
    """The 2-D time loop driven by eq.(5) (N = 2, barycentric weights): creation tables straight
    from the network's rows give the same tables and trajectory as rows -> tables."""
    from paper_1806_00082_amd.sim import Simulator
    mesh = inputs.Mesh2D(nx=40, ny=36, dx=0.5, n_m=16, pos_f64=False)
    V = inputs.gaussian_dot_2d(mesh, 0.2, 1.5, 10.0, 9.0)
    bc = inputs.packet_bin_counts_2d(mesh, 5e4, 6.0, 9.0, 1.2, inputs.k_for_energy(0.1), 0.0)
    cfg = inputs.RunConfig("small2d", mesh, V, bc, int(bc.sum()), 0.5, 10, seed=5)
    w = learn.analytic_weights_2d(16, 2)
    fused = Simulator(cfg, kernel="surrogate", N=2, weights=w)
    two = Simulator(cfg, kernel="surrogate", N=2, weights=w, fused_tables=False)
    assert fused.fused and not two.fused and fused.Kbuf is None
    for k in range(10):
        fused.step()
        two.step()
        n = fused.count()
        assert n == two.count(), k
        for f in ("x", "y", "M", "My", "s"):
            assert torch.equal(getattr(fused.a, f)[:n], getattr(two.a, f)[:n]), (k, f)
    r = fused.n_rows
    assert r == two.n_rows and r > 0
    for f in ("gamma", "n0", "thr", "cdf", "guide"):
        assert torch.equal(getattr(fused, f)[:r], getattr(two, f)[:r]), f
