"""Torch-facing wrappers of the C ABI: argument marshalling only.

Torch provides device memory and the current stream; every computation happens in the
HIP kernels of libwigner.so.  Tensors must already live on the HIP device.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L
from .inputs import HBAR_EVFS


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need_cuda(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise L.WignerError("libwigner works on device tensors only")


def mesh_struct(dim: int, nx: int, ny: int, n_m: int, hbar: float = HBAR_EVFS) -> L.WkMesh:
    return L.WkMesh(dim, nx, ny, n_m, hbar)


# ----------------------------------------------------------------------------- set-up
_prepared = set()


def prepare(n_m: int, device=None, hbar: float = HBAR_EVFS):
    """wk_prepare for n_m on `device` (default: the current one), once per process: builds the
    library's sine tables for the 1-D contractions (allocates and synchronises)."""
    dev = torch.cuda.current_device() if device is None else torch.device(device).index
    dev = torch.cuda.current_device() if dev is None else dev
    key = (dev, int(n_m))
    if key in _prepared:
        return
    m = mesh_struct(1, 1, 1, n_m, hbar)
    with torch.cuda.device(dev):
        L.check(L.lib().wk_prepare(ctypes.byref(m), _stream()), "wk_prepare")
    _prepared.add(key)


# ----------------------------------------------------------------------------- kernel
def kernel_eval(V: torch.Tensor, n_m: int, cells: torch.Tensor | None = None, prec: str = "fp64",
                layout: str = "full", hbar: float = HBAR_EVFS, out: torch.Tensor | None = None):
    """eq.(4) on the requested cells.  V: [B][nx] (1-D) or [B][ny][nx] (2-D) float64."""
    _need_cuda(V, cells)
    if V.dim() == 1:
        V = V[None]
    dim = 1 if V.dim() == 2 else 2
    B = V.shape[0]
    nx = V.shape[-1]
    ny = 1 if dim == 1 else V.shape[-2]
    V = V.contiguous()
    assert V.dtype == torch.float64
    n_cells = nx * ny if cells is None else int(cells.numel())
    if cells is not None:
        cells = cells.to(torch.int32).contiguous()
    P = n_m // 2
    lay = L.WK_HALF if layout == "half" else L.WK_FULL
    p = L.PREC[prec]
    dt = torch.float64 if p == L.WK_FP64 else torch.float32
    if dim == 1:
        shape = (B * n_cells, P if lay == L.WK_HALF else n_m)
    else:
        shape = (B * n_cells, n_m, n_m)
    if out is None:
        out = torch.empty(shape, dtype=dt, device=V.device)
    if dim == 1:
        prepare(n_m, V.device)
    m = mesh_struct(dim, nx, ny, n_m, hbar)
    L.check(L.lib().wk_kernel_eval(ctypes.byref(m), _ptr(V), B, _ptr(cells), n_cells, p, lay,
                                   _ptr(out), _stream()), "wk_kernel_eval")
    return out


def kernel_bwd(G: torch.Tensor, nx: int, n_m: int, B: int, layout: str = "full",
               hbar: float = HBAR_EVFS, dV: torch.Tensor | None = None,
               cells: torch.Tensor | None = None):
    """Adjoint of eq.(4) in V on the rows of kernel_eval (all cells, or `cells`): G is float64
    (FP64 product) or float32 (FP32 product); dV [B][nx] float64 is accumulated into."""
    _need_cuda(G, cells)
    prec = {torch.float64: L.WK_FP64, torch.float32: L.WK_FP32}[G.dtype]
    n_cells = nx if cells is None else int(cells.numel())
    if cells is not None:
        cells = cells.to(torch.int32).contiguous()
    m = mesh_struct(1, nx, 1, n_m, hbar)
    prepare(n_m, G.device)
    if dV is None:
        dV = torch.zeros((B, nx), dtype=torch.float64, device=G.device)
    wsz = L.lib().wk_kernel_bwd_workspace(ctypes.byref(m), B, n_cells, prec)
    ws = torch.empty(max(int(wsz), 8), dtype=torch.uint8, device=G.device)
    lay = L.WK_HALF if layout == "half" else L.WK_FULL
    L.check(L.lib().wk_kernel_bwd(ctypes.byref(m), _ptr(G.contiguous()), B, _ptr(cells), n_cells, prec,
                                  lay, _ptr(dV), _ptr(ws), int(wsz), _stream()), "wk_kernel_bwd")
    return dV


def gamma_tables(K: torch.Tensor, n_m: int, dt: float, dim: int = 1, layout: str = "full",
                 hbar: float = HBAR_EVFS):
    """Returns (gamma f64, n0 u32-as-int32, thr u32-as-int32, cdf u64-as-int64)."""
    _need_cuda(K)
    K = K.contiguous()
    width = n_m if dim == 1 else n_m * n_m
    lay = L.WK_HALF if layout == "half" else L.WK_FULL
    row_len = n_m // 2 if lay == L.WK_HALF else width
    n_rows = K.numel() // row_len
    dev = K.device
    g = torch.empty(n_rows, dtype=torch.float64, device=dev)
    n0 = torch.empty(n_rows, dtype=torch.int32, device=dev)
    thr = torch.empty(n_rows, dtype=torch.int32, device=dev)
    cdf = torch.empty((n_rows, width), dtype=torch.int64, device=dev)
    m = mesh_struct(dim, 1, 1, n_m, hbar)
    L.check(L.lib().wk_gamma_tables(ctypes.byref(m), _ptr(K), int(K.dtype == torch.float64), lay,
                                    n_rows, dt, _ptr(g), _ptr(n0), _ptr(thr), _ptr(cdf), _stream()),
            "wk_gamma_tables")
    return g, n0, thr, cdf


def kernel_tables(V: torch.Tensor, n_m: int, dt: float, cells: torch.Tensor | None = None,
                  guide_len: int = 0, hbar: float = HBAR_EVFS, out=None, prec: str = "fp64"):
    """eq.(4) rows of the requested cells turned straight into the creation tables (the rows
    stay on chip).  V [B][nx] (1-D) or [B][ny][nx] (2-D); prec "fp64" or a 16-bit form
    ("bf16", "fp16", "bf16x3", "fp16x3": the tables of its FP32 rows).
    Returns (gamma, n0, thr, cdf, guide or None) as gamma_tables and sampling_guide would;
    `out` may supply those five tensors (row slices are fine)."""
    _need_cuda(V, cells)
    if V.dim() == 1:
        V = V[None]
    assert V.dim() in (2, 3) and V.dtype == torch.float64, "FP64 potentials [B][nx] or [B][ny][nx]"
    V = V.contiguous()
    dim = V.dim() - 1
    B, nx = V.shape[0], V.shape[-1]
    ny = 1 if dim == 1 else V.shape[1]
    width = n_m if dim == 1 else n_m * n_m
    n_cells = nx * ny if cells is None else int(cells.numel())
    if cells is not None:
        cells = cells.to(torch.int32).contiguous()
    R = B * n_cells
    dev = V.device
    if out is None:
        out = (torch.empty(R, dtype=torch.float64, device=dev), torch.empty(R, dtype=torch.int32, device=dev),
               torch.empty(R, dtype=torch.int32, device=dev), torch.empty((R, width), dtype=torch.int64, device=dev),
               torch.empty((R, guide_len + 1), dtype=torch.int32, device=dev) if guide_len else None)
    g, n0, thr, cdf, guide = out
    for t, shape in ((g, (R,)), (n0, (R,)), (thr, (R,)), (cdf, (R, width))):
        if tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError(f"kernel_tables: output of shape {tuple(t.shape)}, expected {shape}")
    if guide is not None and (tuple(guide.shape) != (R, guide_len + 1) or not guide.is_contiguous()):
        raise ValueError("kernel_tables: guide must be a contiguous [rows][guide_len + 1] tensor")
    if dim == 1:
        prepare(n_m, V.device)
    m = mesh_struct(dim, nx, ny, n_m, hbar)
    L.check(L.lib().wk_kernel_tables(ctypes.byref(m), _ptr(V), B, _ptr(cells), n_cells, L.PREC[prec], float(dt),
                                     _ptr(g), _ptr(n0), _ptr(thr), _ptr(cdf), _ptr(guide),
                                     guide_len if guide is not None else 0, _stream()), "wk_kernel_tables")
    return g, n0, thr, cdf, guide


# ----------------------------------------------------------------------------- particles
def geom_struct(mesh: dict, seed: int, m_bytes: int = 0) -> L.SpGeom:
    """m_bytes: bytes per stored momentum index (0 = the library default: 4 in 1-D, 2 in 2-D)."""
    return L.SpGeom(mesh["dim"], mesh["nx"], mesh.get("ny", 1), mesh["n_m"], mesh["n_k"],
                    mesh["M_min"], int(mesh["pos_f64"]), int(m_bytes), float(mesh["vdt"]), seed)


_M_RANGE = {1: (-128, 127), 2: (-32768, 32767), 4: (-2 ** 31, 2 ** 31 - 1)}


def fits_m_bytes(mesh: dict, m_bytes: int) -> bool:
    """Whether momenta of m_bytes bytes hold the window widened by the largest pair offset
    (children outside the window are stored, dead, with their momenta)."""
    lo = mesh["M_min"] - mesh["n_m"] // 2
    hi = mesh["M_min"] + mesh["n_k"] - 1 + mesh["n_m"] // 2
    tmin, tmax = _M_RANGE[m_bytes]
    return tmin <= lo and hi <= tmax and (m_bytes != 4 or mesh["dim"] == 1)


def fits_m16(mesh: dict) -> bool:
    return fits_m_bytes(mesh, 2)


def narrowest_m_bytes(mesh: dict) -> int:
    """The narrowest momentum storage the mesh's window fits (fewer bytes streamed per pass)."""
    for mb in (1, 2, 4):
        if fits_m_bytes(mesh, mb):
            return mb
    raise ValueError("momentum window does not fit int32")


def _m_bytes(*parts) -> int:
    widths = {p.m_bytes for p in parts}
    if len(widths) != 1:
        raise ValueError("the particle buffers of one call must use the same momentum width")
    return widths.pop()


class DeviceParticles:
    """Struct-of-arrays particle buffer in HBM (positions in cell units)."""

    def __init__(self, dim: int, capacity: int, pos_f64: bool, device="cuda", m16: bool = False,
                 m_bytes: int | None = None):
        """m_bytes: bytes per momentum index, 4 (1-D only), 2 or 1 (default: 4 in 1-D, 2 in
        2-D; m16 = True selects 2); the library refuses a width the mesh's window does not
        fit.  With FP32 positions a 1-D particle takes 9, 7 or 6 bytes, a 2-D one 13 or 11."""
        ft = torch.float64 if pos_f64 else torch.float32
        if m_bytes is None:
            m_bytes = 2 if (m16 or dim == 2) else 4
        if m_bytes not in (1, 2, 4) or (m_bytes == 4 and dim != 1):
            raise ValueError("m_bytes must be 1, 2 or (1-D) 4")
        self.m_bytes = int(m_bytes)
        mt = {1: torch.int8, 2: torch.int16, 4: torch.int32}[self.m_bytes]
        self.dim, self.pos_f64, self.capacity = dim, pos_f64, int(capacity)
        self.x = torch.zeros(capacity, dtype=ft, device=device)
        self.y = torch.zeros(capacity, dtype=ft, device=device) if dim == 2 else None
        self.M = torch.zeros(capacity, dtype=mt, device=device)
        self.My = torch.zeros(capacity, dtype=mt, device=device) if dim == 2 else None
        self.s = torch.zeros(capacity, dtype=torch.int8, device=device)
        self.d_n = torch.zeros(1, dtype=torch.int64, device=device)

    def struct(self) -> L.SpParticles:
        return L.SpParticles(self.x.data_ptr(), self.y.data_ptr() if self.y is not None else None,
                             self.M.data_ptr(), self.My.data_ptr() if self.My is not None else None,
                             self.s.data_ptr(), self.capacity, self.d_n.data_ptr())

    def count(self) -> int:
        return int(self.d_n.item())

    def load(self, n: int, x, M, s, y=None, My=None):
        """Copy host arrays in (test helper for given particle states)."""
        dev = self.x.device
        self.x[:n] = torch.as_tensor(x, device=dev).to(self.x.dtype)
        self.M[:n] = torch.as_tensor(M, device=dev).to(self.M.dtype)
        self.s[:n] = torch.as_tensor(s, device=dev).to(torch.int8)
        if self.dim == 2:
            self.y[:n] = torch.as_tensor(y, device=dev).to(self.y.dtype)
            self.My[:n] = torch.as_tensor(My, device=dev).to(self.My.dtype)
        self.d_n.fill_(n)

    def view(self) -> dict:
        n = self.count()
        d = {"x": self.x[:n].cpu().numpy(), "M": self.M[:n].cpu().numpy(), "s": self.s[:n].cpu().numpy()}
        if self.dim == 2:
            d["y"] = self.y[:n].cpu().numpy()
            d["My"] = self.My[:n].cpu().numpy()
        return d


def sp_workspace(mesh: dict, seed: int = 0, device="cuda") -> torch.Tensor:
    g = geom_struct(mesh, seed)
    n = int(L.lib().sp_workspace_size(ctypes.byref(g)))
    if n == 0:
        L.check(L.WK_EINVAL, "sp_workspace_size")
    return torch.empty(n, dtype=torch.uint8, device=device)


def new_stats(device="cuda") -> torch.Tensor:
    return torch.zeros(L.ST_COUNT, dtype=torch.int64, device=device)


def sp_init(mesh: dict, seed: int, bin_counts: torch.Tensor, out: DeviceParticles,
            stats: torch.Tensor, ws: torch.Tensor):
    g = geom_struct(mesh, seed, _m_bytes(out))
    ps = out.struct()
    L.check(L.lib().sp_init(ctypes.byref(g), _ptr(bin_counts.to(torch.int32).contiguous()),
                            ctypes.byref(ps), _ptr(stats), _ptr(ws), ws.numel(), _stream()),
            "sp_init")


def sampling_guide(cdf: torch.Tensor, guide_len: int, out: torch.Tensor | None = None):
    """Guide table [rows][guide_len + 1] (int32 holding uint32) of CDF rows [rows][width]."""
    _need_cuda(cdf)
    rows, width = cdf.shape
    if out is None:
        out = torch.empty((rows, guide_len + 1), dtype=torch.int32, device=cdf.device)
    L.check(L.lib().wk_sampling_guide(_ptr(cdf), rows, width, guide_len, _ptr(out), _stream()),
            "wk_sampling_guide")
    return out


def sp_step(mesh: dict, seed: int, cell_slot, n0, thr, cdf, pin: DeviceParticles,
            pout: DeviceParticles, step: int, stats: torch.Tensor, ws: torch.Tensor,
            hist: torch.Tensor | None = None, guide: torch.Tensor | None = None, hist_mode: int = 0,
            keys: torch.Tensor | None = None):
    """One step from pin to pout.  hist (optional): receives the signed histogram of the
    ensemble after the step; hist_mode 1: `hist` is unchanged since the last histogram
    build on this workspace, so only its marked blocks need clearing.  guide (optional):
    sampling_guide() of the cdf rows.  keys (optional, with hist): 32-bit [pout.capacity]
    receiving every output particle's histogram key."""
    g = geom_struct(mesh, seed, _m_bytes(pin, pout))
    a, b = pin.struct(), pout.struct()
    glen = 0 if guide is None else guide.shape[1] - 1
    L.check(L.lib().sp_step(ctypes.byref(g), _ptr(cell_slot), _ptr(n0), _ptr(thr), _ptr(cdf),
                            _ptr(guide), glen, ctypes.byref(a), ctypes.byref(b), _ptr(hist),
                            int(hist_mode), _ptr(keys), step,
                            _ptr(stats), _ptr(ws), ws.numel(), _stream()), "sp_step")


def sp_annihilate(mesh: dict, seed: int, pin: DeviceParticles, pout: DeviceParticles,
                  hist: torch.Tensor, step: int, stats: torch.Tensor, ws: torch.Tensor,
                  hist_ready: int = 0, keys: torch.Tensor | None = None):
    """hist_ready: 0 = build the histogram here; 1 (or True) = `hist` already holds the
    histogram of `pin`; 2 = it is what the last sp_step on this workspace built, unchanged
    (the annihilation then reads only the blocks that step marked).  keys: the keys sp_step
    wrote for `pin` (optional)."""
    g = geom_struct(mesh, seed, _m_bytes(pin, pout))
    a, b = pin.struct(), pout.struct()
    L.check(L.lib().sp_annihilate(ctypes.byref(g), ctypes.byref(a), ctypes.byref(b), _ptr(hist),
                                  int(hist_ready), _ptr(keys), step, _ptr(stats), _ptr(ws), ws.numel(),
                                  _stream()), "sp_annihilate")


def sp_pairs_scratch(mesh: dict, capacity: int, device="cuda") -> torch.Tensor:
    """Scratch buffer of sp_annihilate_pairs for input buffers of `capacity` particles."""
    g = geom_struct(mesh, 0)
    n = int(L.lib().sp_pairs_scratch_size(ctypes.byref(g), int(capacity)))
    if n == 0:
        L.check(L.WK_EINVAL, "sp_pairs_scratch_size")
    return torch.empty(n, dtype=torch.uint8, device=device)


def sp_annihilate_pairs(mesh: dict, pin: DeviceParticles, pout: DeviceParticles, hist: torch.Tensor,
                        stats: torch.Tensor, ws: torch.Tensor, scratch: torch.Tensor,
                        hist_ready: int = 0):
    """Rule 2 as literal pair removal (survivors keep their exact positions); hist_ready as
    for sp_annihilate."""
    g = geom_struct(mesh, 0, _m_bytes(pin, pout))
    a, b = pin.struct(), pout.struct()
    L.check(L.lib().sp_annihilate_pairs(ctypes.byref(g), ctypes.byref(a), ctypes.byref(b), _ptr(hist),
                                        int(hist_ready), _ptr(stats), _ptr(ws), ws.numel(),
                                        _ptr(scratch), scratch.numel(), _stream()), "sp_annihilate_pairs")


def sp_density(mesh: dict, hist: torch.Tensor, N0: float, rho: torch.Tensor | None = None):
    g = geom_struct(mesh, 0)
    if rho is None:
        rho = torch.empty(mesh["nx"] * mesh.get("ny", 1), dtype=torch.float64, device=hist.device)
    L.check(L.lib().sp_density(ctypes.byref(g), _ptr(hist), float(N0), _ptr(rho), _stream()),
            "sp_density")
    return rho


def n_bins(mesh: dict) -> int:
    return mesh["nx"] * mesh.get("ny", 1) * mesh["n_k"] ** mesh["dim"]
