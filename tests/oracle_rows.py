"""Oracle eq.(4) rows of the d = 2 form for many cells, computed by a pool of processes
(test infrastructure: only the oracle and numpy are imported here, so spawned workers start
without touching any device)."""
import multiprocessing as mp
import os

import numpy as np


def _rows(args):
    import oracle as orc
    V, n_m, hbar, cells = args
    return orc.kernel_2d(V, n_m, hbar, cells=cells)[0]


def kernel_2d_rows(V, n_m, hbar, cells, workers=None):
    """[len(cells)][n_m * n_m] rows of the oracle's direct d = 2 sum."""
    workers = workers or max(1, min(16, os.cpu_count() or 1))
    chunks = [c for c in np.array_split(np.asarray(cells, np.int32), workers * 4) if len(c)]
    with mp.get_context("spawn").Pool(workers) as pool:
        rows = pool.map(_rows, [(V, n_m, hbar, c) for c in chunks])
    return np.concatenate(rows).reshape(len(cells), n_m * n_m)


def reachable_cells(occupied, pad):
    """Cells within `pad` cells (per axis) of an occupied one, flat ids in ascending order."""
    occ = np.asarray(occupied, bool)
    reach = np.zeros_like(occ)
    ny, nx = occ.shape
    for dy in range(-pad, pad + 1):
        for dx in range(-pad, pad + 1):
            sh = np.zeros_like(occ)
            ys = slice(max(dy, 0), ny + min(dy, 0))
            yd = slice(max(-dy, 0), ny + min(-dy, 0))
            xs = slice(max(dx, 0), nx + min(dx, 0))
            xd = slice(max(-dx, 0), nx + min(-dx, 0))
            sh[ys, xs] = occ[yd, xd]
            reach |= sh
    return np.flatnonzero(reach).astype(np.int32)
