"""CPU oracle for the signed-particle Wigner Monte Carlo hot path (arXiv:1806.00082).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product library
(``paper_1806_00082_amd``) never imports it and shares no code with it.

The arithmetic lives in ``wk_oracle.c`` (plain C, FP64, single thread, built with
``-O2 -ffp-contract=off``).  This module only marshals numpy arrays into it and adds
small numpy helpers for the read-out (rule 1 of Sec. 2.1).  Every function names the
passage of the paper it follows.

Parity status (see the tests for each pin):
  kernel_1d, kernel_1d_literal ... pinned (DST-I, Parseval, closed forms, brute force)
  kernel_2d ...................... pinned (reduction to 1-D, oddness, brute force)
  kernel_bwd_1d .................. pinned (adjoint dot-product identity)
  gamma_tables ................... pinned (positive-part sum, sampling law)
  philox4x32_10 .................. pinned (published known-answer vectors)
  sp_init / sp_step / sp_annihilate pinned (hand-traced cases, invariants, free drift)
  sp_annihilate_pairs ............ pinned (explicit pair matching by brute force,
                                   net sign per bin, survivors an exact subsequence)
  surrogate_fwd .................. pinned (N=1 equals eq.(4); N=2 equals the
                                   barycentric form of Sec. 2.3)
  surrogate_bwd .................. pinned (finite differences in high precision)
  surrogate_fwd_2d ............... pinned (N = 1 equals the d = 2 kernel; a potential of x
                                   alone gives the 1-D network on the my = 0 row, 0 elsewhere)
  mse_grad, sgd_step ............. pinned (finite differences of the loss, first-order
                                   descent prediction, fixed point at zero residual)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wk_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ST_N, ST_PAIRS, ST_ABS_X, ST_ABS_M, ST_NEEDED, ST_KEPT, ST_REGEN, ST_MIXED = range(8)


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC",
             "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, u64, f64 = ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        L.oracle_philox4x32_10.argtypes = [P, P, P]
        L.oracle_philox4x32_10.restype = None
        for name in ("oracle_kernel_1d", "oracle_kernel_1d_literal"):
            getattr(L, name).argtypes = [i32, i32, f64, P, i32, P, i32, P]
            getattr(L, name).restype = i32
        L.oracle_kernel_2d.argtypes = [i32, i32, i32, f64, P, i32, P, i32, P]
        L.oracle_kernel_2d.restype = i32
        L.oracle_kernel_bwd_1d.argtypes = [i32, i32, f64, P, i32, P, i32, P]
        L.oracle_kernel_bwd_1d.restype = i32
        L.oracle_gamma_tables.argtypes = [i32, P, i32, f64, P, P, P, P]
        L.oracle_gamma_tables.restype = i32
        L.oracle_sp_init.argtypes = [i32, i32, i32, i32, i32, i32, u64, P, P, P, P, P, P, i64]
        L.oracle_sp_init.restype = i64
        L.oracle_sp_step.argtypes = [i32, i32, i32, i32, i32, i32, i32, f64, u64, i64,
                                     P, P, P, P, i64, P, P, P, P, P, i64, P]
        L.oracle_sp_step.restype = i64
        L.oracle_sp_annihilate.argtypes = [i32, i32, i32, i32, i32, i32, u64, i64, i64,
                                           P, P, P, P, P, P, P, P, P, P, i64, P, P, P]
        L.oracle_sp_annihilate.restype = i64
        L.oracle_sp_annihilate_pairs.argtypes = [i32, i32, i32, i32, i32, i32, i64,
                                                 P, P, P, P, P, P, P, P, P, P, i64, P, P, P]
        L.oracle_sp_annihilate_pairs.restype = i64
        L.oracle_surrogate_fwd.argtypes = [i32, i32, i32, P, P, P, P, i32, P, i32, P]
        L.oracle_surrogate_fwd.restype = i32
        L.oracle_surrogate_bwd.argtypes = [i32, i32, i32, P, P, P, P, i32, P, i32, P, P, P, P, P]
        L.oracle_surrogate_bwd.restype = i32
        L.oracle_surrogate_fwd_2d.argtypes = [i32, i32, i32, i32, P, P, P, P, P, i32, P, i32, P]
        L.oracle_surrogate_fwd_2d.restype = i32
        L.oracle_mse_grad.argtypes = [P, P, i64, f64, P]
        L.oracle_mse_grad.restype = f64
        L.oracle_sgd_step.argtypes = [i32, i32, i32, f64, P, i32, P, f64, f64, f64, f64, P, P, P]
        L.oracle_sgd_step.restype = f64
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _cells(cells):
    return None if cells is None else np.ascontiguousarray(cells, dtype=np.int32)


def _check(rc, what):
    if rc < 0:
        raise ValueError(f"oracle {what} failed with code {rc}")
    return rc


# ----------------------------------------------------------------------------- RNG
def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 block (Salmon et al., SC'11) -> 4 uint32 words."""
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_p(c), _p(k), _p(out))
    return out


# ----------------------------------------------------------------------------- kernel
def kernel_1d(V, n_m: int, hbar: float, cells=None, literal: bool = False) -> np.ndarray:
    """Full table [B][n_cells][n_m] of eq.(4) (Sec. 2.2), m = t - n_m/2."""
    V = _f64(np.atleast_2d(V))
    B, nx = V.shape
    c = _cells(cells)
    nc = nx if c is None else len(c)
    K = np.empty((B, nc, n_m))
    fn = lib().oracle_kernel_1d_literal if literal else lib().oracle_kernel_1d
    _check(fn(nx, n_m, hbar, _p(V), B, _p(c), nc, _p(K)), "kernel_1d")
    return K


def kernel_2d(V, n_m: int, hbar: float, cells=None) -> np.ndarray:
    """Full table [B][n_cells][n_m(y)][n_m(x)] of the d = 2 form of eq.(4)."""
    V = _f64(V)
    if V.ndim == 2:
        V = V[None]
    B, ny, nx = V.shape
    c = _cells(cells)
    nc = nx * ny if c is None else len(c)
    K = np.empty((B, nc, n_m, n_m))
    _check(lib().oracle_kernel_2d(nx, ny, n_m, hbar, _p(V), B, _p(c), nc, _p(K)), "kernel_2d")
    return K


def kernel_bwd_1d(G, n_m: int, hbar: float, nx: int | None = None, cells=None) -> np.ndarray:
    """dV of <G, K_half(V)> for the half table of eq.(4) on the requested cells (all cells
    when `cells` is None): the adjoint of eq.(4) in V, which is linear in V."""
    G = _f64(G)
    B, nc, P = G.shape
    assert P == n_m // 2
    c = _cells(cells)
    if c is None:
        nx = nc if nx is None else nx
        assert nx == nc
    else:
        assert nx is not None and len(c) == nc
    dV = np.zeros((B, nx))
    _check(lib().oracle_kernel_bwd_1d(nx, n_m, hbar, _p(G), B, _p(c), nc, _p(dV)), "kernel_bwd_1d")
    return dV


def full_to_half(K: np.ndarray) -> np.ndarray:
    """Half table (m = 1..P) from a full 1-D table (m = -P..P-1); K(P) = -K(-P)."""
    n_m = K.shape[-1]
    P = n_m // 2
    H = np.empty(K.shape[:-1] + (P,))
    H[..., : P - 1] = K[..., P + 1:]
    H[..., P - 1] = -K[..., 0]
    return H


def half_to_full(H: np.ndarray) -> np.ndarray:
    """Full 1-D table from a half table by oddness K(-m) = -K(m), K(0) = 0."""
    P = H.shape[-1]
    K = np.zeros(H.shape[:-1] + (2 * P,), dtype=H.dtype)
    K[..., P + 1:] = H[..., : P - 1]
    K[..., 1:P] = -H[..., : P - 1][..., ::-1]
    K[..., 0] = -H[..., P - 1]
    return K


# ----------------------------------------------------------------------------- tables
def gamma_tables(K, dt: float):
    """eq.(1) per row and the integer sampling tables (gamma, n0, thr, cdf)."""
    K = _f64(K)
    width = K.shape[-1]
    Kr = K.reshape(-1, width)
    n = Kr.shape[0]
    g = np.empty(n)
    n0 = np.empty(n, np.uint32)
    thr = np.empty(n, np.uint32)
    cdf = np.empty((n, width), np.uint64)
    _check(lib().oracle_gamma_tables(width, _p(Kr), n, dt, _p(g), _p(n0), _p(thr), _p(cdf)),
           "gamma_tables")
    return g, n0, thr, cdf


# ----------------------------------------------------------------------------- particles
class Particles:
    """Struct-of-arrays particle store on the host (positions in cell units)."""

    def __init__(self, dim: int, capacity: int, pos_f64: bool):
        ft = np.float64 if pos_f64 else np.float32
        mt = np.int32 if dim == 1 else np.int16
        self.dim, self.pos_f64, self.capacity = dim, pos_f64, capacity
        self.x = np.zeros(capacity, ft)
        self.y = np.zeros(capacity if dim == 2 else 0, ft)
        self.M = np.zeros(capacity, mt)
        self.My = np.zeros(capacity if dim == 2 else 0, mt)
        self.s = np.zeros(capacity, np.int8)
        self.n = 0

    def ptrs(self):
        y = _p(self.y) if self.dim == 2 else None
        My = _p(self.My) if self.dim == 2 else None
        return _p(self.x), y, _p(self.M), My, _p(self.s)

    def view(self):
        n = self.n
        d = {"x": self.x[:n].copy(), "M": self.M[:n].copy(), "s": self.s[:n].copy()}
        if self.dim == 2:
            d["y"] = self.y[:n].copy()
            d["My"] = self.My[:n].copy()
        return d


def sp_init(mesh: dict, bin_counts, capacity: int, seed: int) -> Particles:
    """Particles of the initial Wigner function, bin by bin (eq.(6) counts given)."""
    dim = mesh["dim"]
    p = Particles(dim, capacity, mesh["pos_f64"])
    bc = np.ascontiguousarray(bin_counts, dtype=np.int32)
    x, y, M, My, s = p.ptrs()
    n = lib().oracle_sp_init(dim, mesh["nx"], mesh.get("ny", 1), mesh["n_k"], mesh["M_min"],
                             int(mesh["pos_f64"]), seed, _p(bc), x, y, M, My, s, capacity)
    p.n = _check(n, "sp_init")
    return p


def sp_step(mesh: dict, p: Particles, tables, cell_slot, step: int, seed: int):
    """Postulate II + free drift + absorbing boundaries for one time step (Sec. 2.1)."""
    n0, thr, cdf = tables
    cs = np.ascontiguousarray(cell_slot, dtype=np.int32)
    n0 = np.ascontiguousarray(n0, dtype=np.uint32)
    thr = np.ascontiguousarray(thr, dtype=np.uint32)
    cdf = np.ascontiguousarray(cdf, dtype=np.uint64)
    stats = np.zeros(8, np.int64)
    x, y, M, My, s = p.ptrs()
    n = lib().oracle_sp_step(p.dim, mesh["nx"], mesh.get("ny", 1), mesh["n_m"], mesh["n_k"],
                             mesh["M_min"], int(p.pos_f64), mesh["vdt"], seed, step,
                             _p(cs), _p(n0), _p(thr), _p(cdf), p.n, x, y, M, My, s,
                             p.capacity, _p(stats))
    if n == -2:
        return None, stats
    p.n = _check(n, "sp_step")
    return p, stats


def sp_annihilate(mesh: dict, p: Particles, step: int, seed: int, capacity=None):
    """Rule 2 on the (cell, momentum) grid; returns (new particles, H+, H-, stats)."""
    dim = p.dim
    q = Particles(dim, capacity or max(p.capacity, 1), p.pos_f64)
    n_bins = mesh["nx"] * mesh.get("ny", 1) * mesh["n_k"] ** dim
    hp = np.zeros(n_bins, np.int32)
    hm = np.zeros(n_bins, np.int32)
    stats = np.zeros(8, np.int64)
    x, y, M, My, s = p.ptrs()
    xo, yo, Mo, Myo, so = q.ptrs()
    n = lib().oracle_sp_annihilate(dim, mesh["nx"], mesh.get("ny", 1), mesh["n_k"], mesh["M_min"],
                                   int(p.pos_f64), seed, step, p.n, x, y, M, My, s,
                                   xo, yo, Mo, Myo, so, q.capacity, _p(hp), _p(hm), _p(stats))
    q.n = _check(n, "sp_annihilate")
    return q, hp, hm, stats


def sp_annihilate_pairs(mesh: dict, p: Particles, capacity=None):
    """Rule 2 as literal pair removal (k-th positive meets k-th negative of a bin, input
    order); returns (kept particles, H+, H-, stats)."""
    dim = p.dim
    q = Particles(dim, capacity or max(p.capacity, 1), p.pos_f64)
    n_bins = mesh["nx"] * mesh.get("ny", 1) * mesh["n_k"] ** dim
    hp = np.zeros(n_bins, np.int32)
    hm = np.zeros(n_bins, np.int32)
    stats = np.zeros(8, np.int64)
    x, y, M, My, s = p.ptrs()
    xo, yo, Mo, Myo, so = q.ptrs()
    n = lib().oracle_sp_annihilate_pairs(dim, mesh["nx"], mesh.get("ny", 1), mesh["n_k"], mesh["M_min"],
                                         int(p.pos_f64), p.n, x, y, M, My, s, xo, yo, Mo, Myo, so,
                                         q.capacity, _p(hp), _p(hm), _p(stats))
    q.n = _check(n, "sp_annihilate_pairs")
    return q, hp, hm, stats


def density(hp, hm, mesh: dict, N0: float):
    """Rule 1: signed histogram / N0 -> Wigner function f(c, M) and density rho(c)."""
    f = (hp.astype(np.int64) - hm.astype(np.int64)).astype(np.float64) / N0
    if mesh["dim"] == 1:
        f = f.reshape(mesh["nx"], mesh["n_k"])
        return f, f.sum(axis=1)
    f = f.reshape(mesh["ny"], mesh["nx"], mesh["n_k"], mesh["n_k"])
    return f, f.sum(axis=(2, 3))


# ----------------------------------------------------------------------------- surrogate
def surrogate_fwd(V, n_m: int, N: int, wV, wT, W, cells=None) -> np.ndarray:
    """eq.(5): half table [B][n_cells][P] (m = 1..P) of the grouped network."""
    V = _f64(np.atleast_2d(V))
    B, nx = V.shape
    c = _cells(cells)
    nc = nx if c is None else len(c)
    wV, wT, W = _f64(wV), _f64(wT), _f64(W)
    Kh = np.empty((B, nc, n_m // 2))
    _check(lib().oracle_surrogate_fwd(nx, n_m, N, _p(wV), _p(wT), _p(W), _p(V), B, _p(c), nc,
                                      _p(Kh)), "surrogate_fwd")
    return Kh


def surrogate_bwd(V, n_m: int, N: int, wV, wT, W, E, cells=None, want_dV: bool = True):
    """Gradients of sum(E * Kh) w.r.t. (wV, wT, W, V) for eq.(5)."""
    V = _f64(np.atleast_2d(V))
    B, nx = V.shape
    c = _cells(cells)
    nc = nx if c is None else len(c)
    wV, wT, W, E = _f64(wV), _f64(wT), _f64(W), _f64(E)
    dwV = np.zeros(N)
    dwT = np.zeros(N)
    dW = np.zeros(n_m // N)
    dV = np.zeros((B, nx)) if want_dV else None
    _check(lib().oracle_surrogate_bwd(nx, n_m, N, _p(wV), _p(wT), _p(W), _p(V), B, _p(c), nc,
                                      _p(E), _p(dwV), _p(dwT), _p(dW), _p(dV)), "surrogate_bwd")
    return dwV, dwT, dW, dV


def surrogate_fwd_2d(V, n_m: int, N: int, wV, wTx, wTy, W, cells=None) -> np.ndarray:
    """eq.(5) in d = 2: full table [B][n_cells][n_m(y)][n_m(x)]."""
    V = _f64(V)
    if V.ndim == 2:
        V = V[None]
    B, ny, nx = V.shape
    c = _cells(cells)
    nc = nx * ny if c is None else len(c)
    wV, wTx, wTy, W = _f64(wV), _f64(wTx), _f64(wTy), _f64(W)
    Kh = np.empty((B, nc, n_m, n_m))
    _check(lib().oracle_surrogate_fwd_2d(nx, ny, n_m, N, _p(wV), _p(wTx), _p(wTy), _p(W), _p(V), B, _p(c), nc,
                                         _p(Kh)), "surrogate_fwd_2d")
    return Kh


def analytic_weights_2d(n_m: int, N: int, hbar: float):
    """wV = 1 (N x N), wTx = wTy = 1/N, W = -2/(hbar n_m^2) ((n_m/N)^2 groups)."""
    H = n_m // N
    return (np.ones(N * N), np.full(N, 1.0 / N), np.full(N, 1.0 / N), np.full(H * H, -2.0 / (hbar * n_m * n_m)))


def analytic_weights(n_m: int, N: int, hbar: float):
    """Barycentric weights of Sec. 2.3: wV = 1, wT = 1/N, W = -2/(hbar n_m)."""
    return (np.ones(N), np.full(N, 1.0 / N), np.full(n_m // N, -2.0 / (hbar * n_m)))


# ----------------------------------------------------------------------------- training
def mse_grad(Kh, K, inv_scale: float):
    """MSE of Sec. 3 on targets scaled by inv_scale: (loss, dloss/dKh)."""
    Kh, K = _f64(Kh), _f64(K)
    E = np.empty_like(Kh)
    loss = lib().oracle_mse_grad(_p(Kh), _p(K), Kh.size, float(inv_scale), _p(E))
    return loss, E


def sgd_step(V, K, n_m: int, N: int, hbar: float, weights, lr, inv_scale: float | None = None):
    """One SGD step of Sec. 3 on a batch (all cells) with labels K [B][nx][P]; returns
    (loss before the step, (wV, wT, W) after it).  lr: one value or (lr_V, lr_T, lr_W), W
    stepped in units of c = -2/(hbar n_m)."""
    V = _f64(np.atleast_2d(V))
    B, nx = V.shape
    K = _f64(K)
    assert K.shape == (B, nx, n_m // 2)
    lr_V, lr_T, lr_W = (lr, lr, lr) if np.isscalar(lr) else lr
    if inv_scale is None:
        inv_scale = hbar * n_m / 2.0
    wV, wT, W = (_f64(w).copy() for w in weights)
    loss = lib().oracle_sgd_step(nx, n_m, N, hbar, _p(V), B, _p(K), float(inv_scale), float(lr_V),
                                 float(lr_T), float(lr_W), _p(wV), _p(wT), _p(W))
    if loss < 0:
        raise ValueError("oracle sgd_step failed")
    return loss, (wV, wT, W)
