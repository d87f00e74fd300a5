"""Time loop of the signed-particle method (Sec. 2.1, Sec. 3): host-side orchestration of the
library's kernels, no computation in Python.

Per step: (every `refresh_every` steps) kernel rows for newly occupied cells -> creation
tables (one fused pass for exact FP64 rows, the rows staying on chip); sp_step
(creation at rate gamma, drift, absorbing boundaries, and the signed histogram of rule 1 of
the result); sp_annihilate (rule 2 on that histogram).  The particle
count stays in device memory; the host synchronises only to size the occasional kernel-row
refresh and to read statistics.

Annihilation (rule 2): "regenerate" replaces the particles of each bin holding both signs by
|H+ - H-| fresh particles of the net sign; "pairs" removes opposite-sign pairs and keeps the
other particles exactly where they are.

Kernel sources (the paper's two steps, Sec. 4): "exact" = eq.(4) on MFMA in FP64 or a reduced
precision; "surrogate" = the trained network of eq.(5) (in 2-D its d = 2 form, FP64, weights
(wV, wTx, wTy, W)); "given" = rows the caller computed
(`rows`, one per cell, every cell evaluated at start).  Rows are evaluated only for cells
within a margin of the occupied ones ("occupied", the paper's memory/speed point) or for
every cell at start ("all"); both give the same trajectory bit for bit when the margin
covers the drift between refreshes.

`run(steps, log=f)` writes one JSON line of statistics per step; `save` / `restore` write and
read the state carried between steps, and a restored run continues bit for bit.
"""
from __future__ import annotations

import ctypes
import json
import math
import time

import torch

from . import _lib as L
from . import learn, ops


class Simulator:
    def __init__(self, cfg, kernel: str = "exact", prec: str = "fp64", mode: str = "occupied",
                 refresh_every: int = 8, cap_factor: float = 3.0, weights=None, N: int = 2,
                 device="cuda", hist_in_step: bool = True, rows=None, m_bytes=None,
                 fused_tables: bool = True, annihilation: str = "regenerate", keys: bool = True):
        self.cfg = cfg
        self.md = cfg.mesh.as_dict(cfg.dt)
        md = self.md
        self.dim = md["dim"]
        self.kernel, self.prec, self.mode = kernel, prec, mode
        if annihilation not in ("regenerate", "pairs"):
            raise ValueError("annihilation must be 'regenerate' or 'pairs'")
        self.annihilation = annihilation
        self.hist_in_step = hist_in_step   # sp_step builds the histogram sp_annihilate uses
        self.refresh_every = max(1, int(refresh_every))
        self.N, self.weights = N, weights
        self.seed = cfg.seed
        self.dev = torch.device(device)
        self.n_m = md["n_m"]
        self.n_cells = md["nx"] * md.get("ny", 1)
        self.width = self.n_m if self.dim == 1 else self.n_m * self.n_m
        self.half = self.dim == 1                       # 1-D rows are kept as half tables
        self.row_len = self.n_m // 2 if self.half else self.width
        V = torch.as_tensor(cfg.V, dtype=torch.float64)
        self.V = (V[None] if V.dim() == self.dim else V).contiguous().to(self.dev)
        # per-cell creation tables (rows handed out as cells become occupied)
        self.cell_slot = torch.full((self.n_cells,), -1, dtype=torch.int32, device=self.dev)
        self.gamma = torch.zeros(self.n_cells, dtype=torch.float64, device=self.dev)
        self.n0 = torch.zeros(self.n_cells, dtype=torch.int32, device=self.dev)
        self.thr = torch.zeros(self.n_cells, dtype=torch.int32, device=self.dev)
        self.cdf = torch.zeros((self.n_cells, self.width), dtype=torch.int64, device=self.dev)
        self.glen = min(self.width, 256)                # guide buckets for the CDF search
        self.guide = torch.zeros((self.n_cells, self.glen + 1), dtype=torch.int32, device=self.dev)
        # exact rows go straight into the creation tables (wk_kernel_tables): the kernel rows
        # then never exist in device memory
        self.fused = fused_tables and (
            (kernel == "exact" and ((self.dim == 1 and 4 <= self.n_m <= 514) or (self.dim == 2 and self.n_m in (8, 16, 32))))
            or (kernel == "surrogate" and self.dim == 2))
        if self.fused:
            self.Kbuf = None
        elif kernel == "given":
            if mode != "all":
                raise ValueError("given kernel rows need mode='all'")
            if (rows is None or rows.device.type != self.dev.type or rows.dtype not in (torch.float64, torch.float32)
                    or tuple(rows.shape) != (self.n_cells, self.row_len) or not rows.is_contiguous()):
                raise ValueError(f"rows must be a contiguous [{self.n_cells}][{self.row_len}] float "
                                 f"tensor on {self.dev}")
            self.Kbuf = rows
        else:
            kdt = (torch.float64 if ((kernel == "exact" and prec == "fp64") or (kernel == "surrogate" and self.dim == 2))
                   else torch.float32)
            self.Kbuf = torch.empty((self.n_cells, self.row_len), dtype=kdt, device=self.dev)
        self.surr_ws = (learn.surrogate_fwd_workspace(self.n_m, N, self.dev)
                        if kernel == "surrogate" and self.dim == 1 else None)
        self.new_cells = torch.empty(self.n_cells, dtype=torch.int32, device=self.dev)
        self.d_count = torch.zeros(1, dtype=torch.int64, device=self.dev)
        self.n_rows = 0
        # particles
        bc = torch.as_tensor(cfg.bin_counts, dtype=torch.int32)
        n0 = int(bc.sum())
        self.capacity = int(cap_factor * n0) + 1024
        # momenta in the narrowest integer type the window allows (int8 for the workloads here:
        # 6-byte 1-D and 11-byte 2-D particles with FP32 positions)
        m_bytes = m_bytes if m_bytes is not None else ops.narrowest_m_bytes(md)
        self.a = ops.DeviceParticles(self.dim, self.capacity, md["pos_f64"], self.dev, m_bytes=m_bytes)
        self.b = ops.DeviceParticles(self.dim, self.capacity, md["pos_f64"], self.dev, m_bytes=m_bytes)
        self.stats = ops.new_stats(self.dev)
        self.ws = ops.sp_workspace(md, self.seed, self.dev)
        self.hist = torch.zeros(2 * ops.n_bins(md), dtype=torch.int32, device=self.dev)
        # every particle's histogram key from sp_step, read back by the annihilation's counting
        # pass in place of the particles (the rule-2 regeneration path, 2-D: an 11-byte particle
        # against a 4-byte key; a 1-D particle of 6 bytes gains nothing from it)
        self.keys = (torch.empty(self.capacity, dtype=torch.int32, device=self.dev)
                     if keys and self.dim == 2 and hist_in_step and annihilation == "regenerate" else None)
        self.pair_scratch = (ops.sp_pairs_scratch(md, self.capacity, self.dev)
                             if annihilation == "pairs" else None)
        ops.sp_init(md, self.seed, bc.to(self.dev), self.a, self.stats, self.ws)
        self.step_index = 0
        # the initial ensemble is single-signed: this pass only builds the histogram
        ops.sp_annihilate(md, self.seed, self.a, self.b, self.hist, 0xFFFFFFFF, self.stats, self.ws)
        self.a, self.b = self.b, self.a
        # `hist` is what the last histogram build on `ws` left (its block map is valid), so the
        # next step need clear only the marked blocks; false after a restore
        self.hist_marked = True
        vmax = max(abs(md["M_min"]), abs(md["M_min"] + md["n_k"] - 1)) * abs(md["vdt"])
        self.margin = int(math.ceil(self.refresh_every * vmax)) + 1
        if mode == "all":
            self._rows_for(torch.arange(self.n_cells, dtype=torch.int32, device=self.dev), self.n_cells)
            self.cell_slot.copy_(torch.arange(self.n_cells, dtype=torch.int32, device=self.dev))
        else:
            self.refresh()

    # ------------------------------------------------------------------ kernel rows
    def _rows_for(self, cells: torch.Tensor, count: int):
        """Kernel rows + creation tables for `count` cells, appended at row self.n_rows."""
        if count == 0:
            return
        r0 = self.n_rows
        if self.fused:
            tabs = (self.gamma[r0:r0 + count], self.n0[r0:r0 + count], self.thr[r0:r0 + count],
                    self.cdf[r0:r0 + count], self.guide[r0:r0 + count])
            if self.kernel == "surrogate":
                learn.surrogate_tables_2d(self.V, self.n_m, self.N, *self.weights, float(self.cfg.dt),
                                          cells=cells[:count], guide_len=self.glen, out=tabs)
            else:
                ops.kernel_tables(self.V, self.n_m, float(self.cfg.dt), cells=cells[:count], guide_len=self.glen,
                                  prec=self.prec, out=tabs)
            self.n_rows += count
            return
        K = self.Kbuf[:count]
        if self.kernel == "given":
            pass                                        # rows already in place (all cells)
        elif self.kernel == "exact":
            ops.kernel_eval(self.V, self.n_m, cells=cells[:count], prec=self.prec,
                            layout="half" if self.half else "full", out=K)
        elif self.dim == 2:
            learn.surrogate_fwd_2d(self.V, self.n_m, self.N, *self.weights, cells=cells[:count],
                                   out=K.view(count, self.n_m, self.n_m))
        else:
            wV, wT, W = self.weights
            learn.surrogate_fwd(self.V, self.n_m, self.N, wV, wT, W, cells=cells[:count],
                                prec=self.prec if self.prec in ("fp64", "bf16") else "fp32", out=K,
                                ws=self.surr_ws)
        m = ops.mesh_struct(self.dim, 1, 1, self.n_m)
        L.check(L.lib().wk_gamma_tables(
            ctypes.byref(m), ops._ptr(K), int(K.dtype == torch.float64),
            L.WK_HALF if self.half else L.WK_FULL, count, float(self.cfg.dt),
            ctypes.c_void_p(self.gamma.data_ptr() + 8 * r0), ctypes.c_void_p(self.n0.data_ptr() + 4 * r0),
            ctypes.c_void_p(self.thr.data_ptr() + 4 * r0),
            ctypes.c_void_p(self.cdf.data_ptr() + 8 * self.width * r0), ops._stream()), "wk_gamma_tables")
        ops.sampling_guide(self.cdf[r0:r0 + count], self.glen, out=self.guide[r0:r0 + count])
        self.n_rows += count

    def refresh(self) -> int:
        """Rows for the cells near occupied ones that have none yet (one host sync)."""
        g = ops.geom_struct(self.md, self.seed)
        L.check(L.lib().sp_cells_to_evaluate(ctypes.byref(g), ops._ptr(self.hist),
                                             1 if self.hist_marked else 0, self.margin,
                                             ops._ptr(self.cell_slot), ops._ptr(self.new_cells),
                                             ops._ptr(self.d_count), ops._ptr(self.ws),
                                             self.ws.numel(), ops._stream()), "sp_cells_to_evaluate")
        count = int(self.d_count.item())
        if count:
            self._rows_for(self.new_cells, count)
            L.check(L.lib().sp_assign_slots(ops._ptr(self.new_cells), ops._ptr(self.d_count), count,
                                            self.n_rows - count, ops._ptr(self.cell_slot),
                                            ops._stream()), "sp_assign_slots")
        return count

    # ------------------------------------------------------------------ time loop
    def step(self):
        s = self.step_index
        if self.mode == "occupied" and s > 0 and s % self.refresh_every == 0:
            self.refresh()
        ops.sp_step(self.md, self.seed, self.cell_slot, self.n0, self.thr, self.cdf, self.a,
                    self.b, s, self.stats, self.ws, hist=self.hist if self.hist_in_step else None,
                    guide=self.guide, hist_mode=1 if self.hist_marked else 0, keys=self.keys)
        if self.annihilation == "pairs":
            ops.sp_annihilate_pairs(self.md, self.b, self.a, self.hist, self.stats, self.ws,
                                    self.pair_scratch, hist_ready=2 if self.hist_in_step else 0)
        else:
            ops.sp_annihilate(self.md, self.seed, self.b, self.a, self.hist, s, self.stats, self.ws,
                              hist_ready=2 if self.hist_in_step else 0, keys=self.keys)
        self.step_index += 1
        self.hist_marked = True   # built by sp_step, or by the annihilation itself

    def run(self, steps: int, log=None):
        """`steps` time steps; with `log` (a writable text file) one JSON line of
        `metrics()` per step, at one host synchronisation per step."""
        t0 = time.perf_counter()
        for _ in range(steps):
            self.step()
            if log is not None:
                rec = self.metrics()
                rec["wall_s"] = round(time.perf_counter() - t0, 6)
                log.write(json.dumps(rec) + "\n")

    def count(self) -> int:
        return self.a.count()

    def overflowed(self) -> bool:
        return bool(self.stats[L.ST_OVERFLOW].item())

    def density(self):
        return ops.sp_density(self.md, self.hist, float(self.cfg.N0))

    # ------------------------------------------------------------------ metrics, checkpoints
    def metrics(self) -> dict:
        """The statistics of the step just taken (one host synchronisation)."""
        S = self.stats.cpu().tolist()
        return {"step": self.step_index - 1, "particles": S[L.ST_N], "pairs": S[L.ST_PAIRS],
                "absorbed_x": S[L.ST_ABS_X], "absorbed_m": S[L.ST_ABS_M], "kept": S[L.ST_KEPT],
                "regenerated": S[L.ST_REGEN], "mixed_bins": S[L.ST_MIXED], "rows": self.n_rows,
                "overflow": bool(S[L.ST_OVERFLOW])}

    def _identity(self) -> dict:
        """What a checkpoint must agree on with the simulator it is restored into."""
        return {"mesh": self.md, "seed": int(self.seed), "kernel": self.kernel, "prec": self.prec,
                "mode": self.mode, "refresh_every": self.refresh_every, "N": int(self.N),
                "annihilation": self.annihilation, "hist_in_step": bool(self.hist_in_step),
                "fused": bool(self.fused), "glen": self.glen, "m_bytes": self.a.m_bytes}

    def checkpoint(self) -> dict:
        """The state the time loop carries from one step to the next, copied to host memory:
        the ensemble, the signed histogram, the running statistics, the step index and the
        creation tables of the cells evaluated so far.  Pair creation draws from a
        counter-based generator keyed by (seed, step, particle index) and every pass is
        order-defined, so a simulator restored from this state continues bit for bit as the
        uninterrupted run does."""
        n, r = self.count(), self.n_rows
        host = lambda t: t.detach().to("cpu").clone()
        st = {"identity": json.dumps(self._identity(), sort_keys=True),
              "step_index": torch.tensor(self.step_index, dtype=torch.int64),
              "n_rows": torch.tensor(r, dtype=torch.int64), "V": host(self.V),
              "hist": host(self.hist), "stats": host(self.stats), "cell_slot": host(self.cell_slot),
              "gamma": host(self.gamma[:r]), "n0": host(self.n0[:r]), "thr": host(self.thr[:r]),
              "cdf": host(self.cdf[:r]), "guide": host(self.guide[:r])}
        for f in ("x", "y", "M", "My", "s"):
            t = getattr(self.a, f)
            if t is not None:
                st["p_" + f] = host(t[:n])
        for i, w in enumerate(self.weights or ()):
            st[f"w{i}"] = host(torch.as_tensor(w))
        return st

    def save(self, path):
        torch.save(self.checkpoint(), path)

    def restore(self, state):
        """Loads a checkpoint (a dict from `checkpoint()` or a file from `save()`) into this
        simulator, which must have been built with the same configuration, potential and
        weights (refused otherwise).  Files are read without unpickling code."""
        if not isinstance(state, dict):
            state = torch.load(state, map_location="cpu", weights_only=True)
        if state["identity"] != json.dumps(self._identity(), sort_keys=True):
            raise ValueError("checkpoint was written by a simulator of another configuration")
        if not torch.equal(state["V"], self.V.cpu()):
            raise ValueError("checkpoint was written for another potential")
        for i, w in enumerate(self.weights or ()):
            if not torch.equal(state[f"w{i}"], torch.as_tensor(w).cpu()):
                raise ValueError("checkpoint was written with other kernel weights")
        n, r = state["p_x"].numel(), int(state["n_rows"])
        if n > self.a.capacity:
            raise ValueError(f"checkpoint holds {n} particles, the buffers {self.a.capacity}")
        for f in ("x", "y", "M", "My", "s"):
            t = getattr(self.a, f)
            if t is not None:
                t[:n].copy_(state["p_" + f])
        self.a.d_n.fill_(n)
        for name in ("hist", "stats", "cell_slot"):
            getattr(self, name).copy_(state[name])
        for name in ("gamma", "n0", "thr", "cdf", "guide"):
            getattr(self, name)[:r].copy_(state[name])
        self.n_rows = r
        self.step_index = int(state["step_index"])
        self.hist_marked = False  # the workspace's block map does not describe the restored histogram
