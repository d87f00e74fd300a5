"""Differentiation and learned-kernel forms.

* ``WignerKernelFn``: eq.(4) as a torch.autograd.Function whose backward is the hand-written
  adjoint kernel (wk_kernel_bwd) with respect to the potential samples.
* ``SurrogateFn``: the trainable network of eq.(5) (Sec. 2.3) with the hand-written
  backward (wk_surrogate_bwd) with respect to (V, wV, wT, W).
* ``train_surrogate``: the supervised training of Sec. 3 -- random Gaussian-bell potentials,
  exact kernels from the quadrature as labels, MSE, stochastic gradient descent -- with
  every step (labels, forward, loss, backward, update) in the library's kernels.

Weights are FP32 device tensors: wV, wT of length N and W of length n_m / N.  W is trained
in units of the analytic weight c = -2/(hbar n_m) (the update is scaled by c^2), so all
three groups are O(1) and one learning rate serves them.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass, field

import torch

from . import _lib as L
from . import ops
from .inputs import HBAR_EVFS


def analytic_weights(n_m: int, N: int, hbar: float = HBAR_EVFS, device="cuda"):
    """wV = 1, wT = 1/N, W = -2/(hbar n_m): eq.(4) for N = 1, the barycentric form for N = 2."""
    H = n_m // N
    return (torch.ones(N, dtype=torch.float32, device=device),
            torch.full((N,), 1.0 / N, dtype=torch.float32, device=device),
            torch.full((H,), -2.0 / (hbar * n_m), dtype=torch.float32, device=device))


# ----------------------------------------------------------------------------- raw calls
def surrogate_fwd_workspace(n_m: int, N: int, device, hbar: float = HBAR_EVFS) -> torch.Tensor:
    """Scratch buffer for surrogate_fwd (the per-call W sin(u m) and prefactor tables)."""
    m = ops.mesh_struct(1, 1, 1, n_m, hbar)
    n = int(L.lib().wk_surrogate_fwd_workspace(ctypes.byref(m), N))
    if n == 0:
        L.check(L.WK_EINVAL, "wk_surrogate_fwd_workspace")
    return torch.empty(n, dtype=torch.uint8, device=device)


def surrogate_fwd(V, n_m: int, N: int, wV, wT, W, cells=None, prec: str = "fp32",
                  hbar: float = HBAR_EVFS, out=None, ws=None):
    """Half table [B * n_cells][P] of eq.(5); float32 (fp32, bf16) or float64 (fp64).
    ws: surrogate_fwd_workspace() buffer (allocated here when None); calls sharing one must
    not overlap."""
    if V.dim() == 1:
        V = V[None]
    B, nx = V.shape
    n_cells = nx if cells is None else int(cells.numel())
    P = n_m // 2
    p = {"fp64": L.WK_FP64, "bf16": L.WK_BF16, "fp32": L.WK_FP32}[prec]
    dt = torch.float64 if prec == "fp64" else torch.float32
    if out is None:
        out = torch.empty((B * n_cells, P), dtype=dt, device=V.device)
    if ws is None:
        ws = surrogate_fwd_workspace(n_m, N, V.device, hbar)
    m = ops.mesh_struct(1, nx, 1, n_m, hbar)
    c = None if cells is None else cells.to(torch.int32).contiguous()
    L.check(L.lib().wk_surrogate_fwd(ctypes.byref(m), N, ops._ptr(wV), ops._ptr(wT), ops._ptr(W),
                                     ops._ptr(V.contiguous()), B, ops._ptr(c), n_cells, p,
                                     ops._ptr(out), ops._ptr(ws), ws.numel(), ops._stream()),
            "wk_surrogate_fwd")
    return out


def analytic_weights_2d(n_m: int, N: int, hbar: float = HBAR_EVFS, device="cuda"):
    """wV = 1 (N x N), wTx = wTy = 1/N, W = -2/(hbar n_m^2): the d = 2 kernel for N = 1."""
    H = n_m // N
    return (torch.ones(N * N, dtype=torch.float32, device=device),
            torch.full((N,), 1.0 / N, dtype=torch.float32, device=device),
            torch.full((N,), 1.0 / N, dtype=torch.float32, device=device),
            torch.full((H * H,), -2.0 / (hbar * n_m * n_m), dtype=torch.float32, device=device))


def surrogate_fwd_2d(V, n_m: int, N: int, wV, wTx, wTy, W, cells=None, hbar: float = HBAR_EVFS, out=None):
    """eq.(5) in d = 2 (FP64): full tables [B * n_cells][n_m][n_m] of V [B][ny][nx]."""
    if V.dim() == 2:
        V = V[None]
    B, ny, nx = V.shape
    n_cells = nx * ny if cells is None else int(cells.numel())
    if out is None:
        out = torch.empty((B * n_cells, n_m, n_m), dtype=torch.float64, device=V.device)
    m = ops.mesh_struct(2, nx, ny, n_m, hbar)
    c = None if cells is None else cells.to(torch.int32).contiguous()
    L.check(L.lib().wk_surrogate_fwd_2d(ctypes.byref(m), N, ops._ptr(wV), ops._ptr(wTx), ops._ptr(wTy),
                                        ops._ptr(W), ops._ptr(V.contiguous()), B, ops._ptr(c), n_cells,
                                        ops._ptr(out), ops._stream()), "wk_surrogate_fwd_2d")
    return out


def surrogate_tables_2d(V, n_m: int, N: int, wV, wTx, wTy, W, dt: float, cells=None, guide_len: int = 0,
                        hbar: float = HBAR_EVFS, out=None):
    """eq.(5) in d = 2 turned straight into the creation tables (the rows stay on chip).
    Returns (gamma, n0, thr, cdf, guide or None) as ops.kernel_tables; `out` may supply them."""
    if V.dim() == 2:
        V = V[None]
    B, ny, nx = V.shape
    n_cells = nx * ny if cells is None else int(cells.numel())
    R, width = B * n_cells, n_m * n_m
    dev = V.device
    if out is None:
        out = (torch.empty(R, dtype=torch.float64, device=dev), torch.empty(R, dtype=torch.int32, device=dev),
               torch.empty(R, dtype=torch.int32, device=dev), torch.empty((R, width), dtype=torch.int64, device=dev),
               torch.empty((R, guide_len + 1), dtype=torch.int32, device=dev) if guide_len else None)
    g, n0, thr, cdf, guide = out
    for t, shape in ((g, (R,)), (n0, (R,)), (thr, (R,)), (cdf, (R, width))):
        if tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError(f"surrogate_tables_2d: output of shape {tuple(t.shape)}, expected {shape}")
    if guide is not None and (tuple(guide.shape) != (R, guide_len + 1) or not guide.is_contiguous()):
        raise ValueError("surrogate_tables_2d: guide must be a contiguous [rows][guide_len + 1] tensor")
    m = ops.mesh_struct(2, nx, ny, n_m, hbar)
    c = None if cells is None else cells.to(torch.int32).contiguous()
    L.check(L.lib().wk_surrogate_tables_2d(ctypes.byref(m), N, ops._ptr(wV), ops._ptr(wTx), ops._ptr(wTy),
                                           ops._ptr(W), ops._ptr(V.contiguous()), B, ops._ptr(c), n_cells,
                                           float(dt), ops._ptr(g), ops._ptr(n0), ops._ptr(thr), ops._ptr(cdf),
                                           ops._ptr(guide), guide_len if guide is not None else 0,
                                           ops._stream()), "wk_surrogate_tables_2d")
    return g, n0, thr, cdf, guide


def surrogate_bwd(V, n_m: int, N: int, wV, wT, W, E, cells=None, want_dV: bool = False,
                  hbar: float = HBAR_EVFS, ws=None):
    if V.dim() == 1:
        V = V[None]
    B, nx = V.shape
    n_cells = nx if cells is None else int(cells.numel())
    m = ops.mesh_struct(1, nx, 1, n_m, hbar)
    need = int(L.lib().wk_surrogate_workspace(ctypes.byref(m), N, B, n_cells))
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=V.device)
    dwV = torch.empty(N, dtype=torch.float32, device=V.device)
    dwT = torch.empty(N, dtype=torch.float32, device=V.device)
    dW = torch.empty(n_m // N, dtype=torch.float32, device=V.device)
    dV = torch.zeros((B, nx), dtype=torch.float64, device=V.device) if want_dV else None
    c = None if cells is None else cells.to(torch.int32).contiguous()
    L.check(L.lib().wk_surrogate_bwd(ctypes.byref(m), N, ops._ptr(wV), ops._ptr(wT), ops._ptr(W),
                                     ops._ptr(V.contiguous()), B, ops._ptr(c), n_cells,
                                     ops._ptr(E.contiguous()), ops._ptr(dwV), ops._ptr(dwT),
                                     ops._ptr(dW), ops._ptr(dV), ops._ptr(ws), ws.numel(),
                                     ops._stream()), "wk_surrogate_bwd")
    return dwV, dwT, dW, dV


def mse_grad(Kh, K, inv_scale: float, E=None, loss=None, ws=None):
    n = Kh.numel()
    dev = Kh.device
    if E is None:
        E = torch.empty_like(Kh, dtype=torch.float32)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float64, device=dev)
    if ws is None:
        ws = torch.empty(8 * 1024, dtype=torch.uint8, device=dev)
    L.check(L.lib().wk_mse_grad(ops._ptr(Kh), ops._ptr(K), n, float(inv_scale), ops._ptr(E),
                                ops._ptr(loss), ops._ptr(ws), ws.numel(), ops._stream()),
            "wk_mse_grad")
    return E, loss


def sgd_update(w, g, lr: float):
    L.check(L.lib().wk_sgd_update(ops._ptr(w), ops._ptr(g), w.numel(), float(lr), ops._stream()),
            "wk_sgd_update")


# ----------------------------------------------------------------------------- autograd
class WignerKernelFn(torch.autograd.Function):
    """K = eq.(4)(V) on all cells (FP64), with the adjoint kernel as backward."""

    @staticmethod
    def forward(ctx, V, n_m: int, layout: str = "full", hbar: float = HBAR_EVFS):
        ctx.shape = tuple(V.shape)
        ctx.n_m, ctx.layout, ctx.hbar = n_m, layout, hbar
        return ops.kernel_eval(V.detach(), n_m, layout=layout, hbar=hbar)

    @staticmethod
    def backward(ctx, G):
        B, nx = ctx.shape if len(ctx.shape) == 2 else (1, ctx.shape[0])
        dV = ops.kernel_bwd(G.contiguous().to(torch.float64), nx, ctx.n_m, B, layout=ctx.layout,
                            hbar=ctx.hbar)
        return dV.reshape(ctx.shape), None, None, None


class SurrogateFn(torch.autograd.Function):
    """Kh = eq.(5)(V; wV, wT, W) on all cells (FP32), with the hand-written backward."""

    @staticmethod
    def forward(ctx, V, wV, wT, W, n_m: int, N: int, hbar: float = HBAR_EVFS):
        ctx.save_for_backward(V, wV, wT, W)
        ctx.n_m, ctx.N, ctx.hbar = n_m, N, hbar
        return surrogate_fwd(V.detach(), n_m, N, wV.detach(), wT.detach(), W.detach(),
                             prec="fp32", hbar=hbar)

    @staticmethod
    def backward(ctx, E):
        V, wV, wT, W = ctx.saved_tensors
        dwV, dwT, dW, dV = surrogate_bwd(V, ctx.n_m, ctx.N, wV, wT, W,
                                         E.contiguous().to(torch.float32),
                                         want_dV=ctx.needs_input_grad[0], hbar=ctx.hbar)
        if dV is not None:
            dV = dV.reshape(V.shape).to(V.dtype)
        return dV, dwV, dwT, dW, None, None, None


# ----------------------------------------------------------------------------- training
@dataclass
class TrainResult:
    wV: torch.Tensor
    wT: torch.Tensor
    W: torch.Tensor
    losses: list = field(default_factory=list)     # mean batch loss per epoch
    steps: int = 0
    seconds: float = 0.0


class SGDState:
    """Device buffers of one training step (Sec. 3) for batches of `batch` potentials of nx
    cells: label, forward and gradient tables, the loss, and the three calls' workspaces."""

    def __init__(self, n_m: int, N: int, batch: int, nx: int, device, hbar: float = HBAR_EVFS):
        P = n_m // 2
        self.n_m, self.N, self.batch, self.nx, self.hbar = n_m, N, batch, nx, hbar
        self.c = -2.0 / (hbar * n_m)
        self.inv_scale = 1.0 / abs(self.c)
        self.Kh = torch.empty((batch * nx, P), dtype=torch.float32, device=device)
        self.Klab = torch.empty((batch * nx, P), dtype=torch.float64, device=device)
        self.E = torch.empty_like(self.Kh)
        self.loss = torch.empty(1, dtype=torch.float64, device=device)
        self.mse_ws = torch.empty(8 * 1024, dtype=torch.uint8, device=device)
        self.fwd_ws = surrogate_fwd_workspace(n_m, N, device, hbar)
        m = ops.mesh_struct(1, nx, 1, n_m, hbar)
        self.bwd_ws = torch.empty(int(L.lib().wk_surrogate_workspace(ctypes.byref(m), N, batch, nx)),
                                  dtype=torch.uint8, device=device)

    def step(self, Vb, weights, lr, labels=None):
        """One SGD step on the batch Vb [batch][nx] (all cells), in place on `weights`:
        exact eq.(4) half tables as labels (FP64, unless `labels` [batch * nx][P] is given),
        eq.(5) forward in FP32, MSE on targets scaled by 1 / |c|, backward, then
        w -= lr * g per group with W stepped in units of c (lr_W c^2).  The loss before the
        step is left in self.loss (device)."""
        lr_V, lr_T, lr_W = (lr, lr, lr) if isinstance(lr, (int, float)) else lr
        wV, wT, W = weights
        if labels is None:
            ops.kernel_eval(Vb, self.n_m, layout="half", hbar=self.hbar, out=self.Klab)
            labels = self.Klab
        surrogate_fwd(Vb, self.n_m, self.N, wV, wT, W, prec="fp32", hbar=self.hbar, out=self.Kh,
                      ws=self.fwd_ws)
        mse_grad(self.Kh, labels, self.inv_scale, E=self.E, loss=self.loss, ws=self.mse_ws)
        dwV, dwT, dW, _ = surrogate_bwd(Vb, self.n_m, self.N, wV, wT, W, self.E, hbar=self.hbar,
                                        ws=self.bwd_ws)
        sgd_update(wV, dwV, lr_V)
        sgd_update(wT, dwT, lr_T)
        sgd_update(W, dW, lr_W * self.c * self.c)
        return self.loss


def sgd_steps(V: torch.Tensor, batches, n_m: int, N: int, lr, init, hbar: float = HBAR_EVFS):
    """SGD steps on the given batches (lists of potential indices into V [n_pot][nx]) from
    the weights `init`; returns (wV, wT, W) and the loss before each step (host floats)."""
    w = [t.clone() for t in init]
    nx = V.shape[1]
    st = SGDState(n_m, N, len(batches[0]), nx, V.device, hbar)
    losses = []
    for idx in batches:
        Vb = V.index_select(0, torch.as_tensor(idx, dtype=torch.long, device=V.device)).contiguous()
        losses.append(float(st.step(Vb, w, lr).item()))
    return w, losses


def train_surrogate(V_train: torch.Tensor, n_m: int, N: int, epochs: int, batch: int,
                    lr, hbar: float = HBAR_EVFS, init=None, labels=None,
                    seed: int = 0, log=None, epoch_end=None) -> TrainResult:
    """SGD on the MSE between eq.(5) and the exact eq.(4) half tables (Sec. 3).

    V_train: [n_pot][nx] float64 device tensor.  labels: optional precomputed exact half
    tables [n_pot][nx][P] (float64); otherwise each batch's labels are computed on the fly
    with the FP64 kernel contraction.  Batches are drawn by a seeded permutation per epoch.
    lr: one step size, or (lr_wV, lr_wT, lr_W) per parameter group -- the angle weights wT
    multiply offsets up to n_m/2 and momenta up to n_m/2 inside the sine, so their gradient
    is orders of magnitude larger than the others' and they need a much smaller step.
    epoch_end(ep, weights): optional callback after each epoch (e.g. held-out error).
    """
    dev = V_train.device
    n_pot, nx = V_train.shape
    w = [t.clone() for t in (init or analytic_weights(n_m, N, hbar, dev))]
    st = SGDState(n_m, N, batch, nx, dev, hbar)
    P = n_m // 2
    gen = torch.Generator(device="cpu")
    gen.manual_seed(seed)
    res = TrainResult(*w)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for ep in range(epochs):
        perm = torch.randperm(n_pot, generator=gen)
        ep_loss = torch.zeros(1, dtype=torch.float64, device=dev)
        nb = 0
        for k in range(0, n_pot - batch + 1, batch):
            idx = perm[k:k + batch].to(dev)
            Vb = V_train.index_select(0, idx)
            lab = None if labels is None else labels.index_select(0, idx).reshape(batch * nx, P)
            ep_loss += st.step(Vb, w, lr, labels=lab)
            nb += 1
            res.steps += 1
        res.losses.append(float((ep_loss / max(nb, 1)).item()))
        if log:
            log(f"epoch {ep}: loss {res.losses[-1]:.6e}")
        if epoch_end:
            epoch_end(ep, w)
    ev1.record()
    torch.cuda.synchronize()
    res.seconds = ev0.elapsed_time(ev1) / 1e3
    return res


def surrogate_error(V: torch.Tensor, n_m: int, N: int, wV, wT, W, hbar: float = HBAR_EVFS,
                    prec: str = "fp32") -> float:
    """Normwise error max|Kh - K| / max|K| per potential (max over the batch), exact K in FP64."""
    B, nx = V.shape
    K = ops.kernel_eval(V, n_m, layout="half", hbar=hbar).reshape(B, -1)
    Kh = surrogate_fwd(V, n_m, N, wV, wT, W, prec=prec, hbar=hbar).reshape(B, -1).to(torch.float64)
    err = (Kh - K).abs().amax(dim=1) / K.abs().amax(dim=1).clamp_min(1e-300)
    return float(err.max().item())


def surrogate_rms_error(V: torch.Tensor, n_m: int, N: int, wV, wT, W, hbar: float = HBAR_EVFS,
                        prec: str = "fp32") -> float:
    """sqrt(mean (Kh - K)^2) / sqrt(mean K^2) over the batch: the quantity SGD minimises."""
    K = ops.kernel_eval(V, n_m, layout="half", hbar=hbar)
    Kh = surrogate_fwd(V, n_m, N, wV, wT, W, prec=prec, hbar=hbar).to(torch.float64)
    return float(((Kh - K) ** 2).mean().sqrt() / (K ** 2).mean().sqrt())
