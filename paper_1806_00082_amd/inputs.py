"""Seeded synthetic inputs and workload definitions.

This module holds the inputs both the HIP path and the CPU oracle consume, and none of
the method's arithmetic (no Wigner kernel, no creation rate, no particle rules).  It
defines the meshes, the potentials (Gaussian barriers and random Gaussian-bell
potentials, Sec. 3), the initial Wigner function of eq.(6) turned into per-bin particle
counts, and the physical constants (CODATA 2018).

Units: nm, fs, eV.  Positions handed to the particle passes are in units of the cell
width.  Momentum indices count Delta k = pi / L_C (the momentum grid of eq.(3), read as
Delta p = pi hbar / L_C).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# CODATA 2018: hbar = 1.054571817e-34 J s, e = 1.602176634e-19 C, m_e = 9.1093837015e-31 kg.
HBAR_EVFS = 0.6582119569          # hbar in eV fs
HBAR_OVER_ME = 0.115767636        # hbar / m_e in nm^2 / fs


def k_for_energy(E_eV: float) -> float:
    """Wave number (1/nm) of a free electron of kinetic energy E: E = hbar^2 k^2 / (2 m)."""
    return math.sqrt(2.0 * E_eV / (HBAR_EVFS * HBAR_OVER_ME))


@dataclass
class Mesh1D:
    nx: int
    dx: float
    n_m: int
    pos_f64: bool = True

    @property
    def dim(self):
        return 1

    @property
    def L_C(self):
        return self.n_m * self.dx

    @property
    def dk(self):
        return math.pi / self.L_C

    @property
    def n_k(self):            # particle momentum window [M_min, M_min + n_k)
        return 2 * self.n_m

    @property
    def M_min(self):
        return -self.n_m

    def centres(self):
        return (np.arange(self.nx) + 0.5) * self.dx

    def vdt(self, dt: float) -> float:
        """Drift per step and per unit of momentum index, in cells: (hbar/m) dk dt / dx."""
        return HBAR_OVER_ME * self.dk * dt / self.dx

    def as_dict(self, dt: float):
        return {"dim": 1, "nx": self.nx, "ny": 1, "n_m": self.n_m, "n_k": self.n_k,
                "M_min": self.M_min, "pos_f64": self.pos_f64, "vdt": self.vdt(dt)}


@dataclass
class Mesh2D:
    nx: int
    ny: int
    dx: float
    n_m: int
    pos_f64: bool = False

    @property
    def dim(self):
        return 2

    @property
    def L_C(self):
        return self.n_m * self.dx

    @property
    def dk(self):
        return math.pi / self.L_C

    @property
    def n_k(self):
        return self.n_m

    @property
    def M_min(self):
        return -(self.n_m // 2)

    def vdt(self, dt: float) -> float:
        return HBAR_OVER_ME * self.dk * dt / self.dx

    def as_dict(self, dt: float):
        return {"dim": 2, "nx": self.nx, "ny": self.ny, "n_m": self.n_m, "n_k": self.n_k,
                "M_min": self.M_min, "pos_f64": self.pos_f64, "vdt": self.vdt(dt)}


# ----------------------------------------------------------------------------- potentials
def gaussian_barrier_1d(mesh: Mesh1D, height: float, sigma: float, centre: float) -> np.ndarray:
    x = mesh.centres()
    return height * np.exp(-((x - centre) ** 2) / (2.0 * sigma * sigma))


def gaussian_dot_2d(mesh: Mesh2D, height: float, sigma: float, cx: float, cy: float) -> np.ndarray:
    x = (np.arange(mesh.nx) + 0.5) * mesh.dx
    y = (np.arange(mesh.ny) + 0.5) * mesh.dx
    r2 = (x[None, :] - cx) ** 2 + (y[:, None] - cy) ** 2
    return height * np.exp(-r2 / (2.0 * sigma * sigma))


def random_potentials(B: int, nx: int, dx: float, seed: int, hmax: float = 0.5,
                      smin: float = 1.0, smax: float = 5.0, qmax: int = 4) -> np.ndarray:
    """B potentials, each a sum of Q ~ U{1..qmax} Gaussian bells with heights U(0, hmax) eV,
    widths U(smin, smax) nm and centres U(0, nx dx) (the data set of Sec. 3)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = (np.arange(nx) + 0.5) * dx
    V = np.zeros((B, nx))
    for b in range(B):
        q = int(rng.integers(1, qmax + 1))
        h = rng.uniform(0.0, hmax, q)
        s = rng.uniform(smin, smax, q)
        c = rng.uniform(0.0, nx * dx, q)
        V[b] = (h[:, None] * np.exp(-((x[None, :] - c[:, None]) ** 2) / (2.0 * s[:, None] ** 2))).sum(0)
    return V


# ----------------------------------------------------------------------------- initial state
def _cell_weights(n: int, dx: float, x0: float, sigma: float) -> np.ndarray:
    """Integral of exp(-(x-x0)^2/sigma^2) over each cell (erf closed form)."""
    from scipy.special import erf
    edges = np.arange(n + 1) * dx
    e = erf((edges - x0) / sigma)
    return 0.5 * math.sqrt(math.pi) * sigma * (e[1:] - e[:-1])


def _mom_weights(n_k: int, M_min: int, dk: float, k0: float, sigma: float) -> np.ndarray:
    M = np.arange(M_min, M_min + n_k)
    return np.exp(-((M * dk - k0) ** 2) * sigma * sigma)


def _round_counts(F: np.ndarray, N0: float) -> np.ndarray:
    c = np.floor(F / F.sum() * N0 + 0.5)
    return c.astype(np.int32)


def packet_bin_counts_1d(mesh: Mesh1D, N0: float, x0: float, sigma: float, k0: float) -> np.ndarray:
    """Per-bin counts of eq.(6) on the (cell, M) grid, bin = cell * n_k + (M - M_min)."""
    fx = _cell_weights(mesh.nx, mesh.dx, x0, sigma)
    fk = _mom_weights(mesh.n_k, mesh.M_min, mesh.dk, k0, sigma)
    return _round_counts(np.outer(fx, fk).ravel(), N0)


def packet_bin_counts_2d(mesh: Mesh2D, N0: float, x0: float, y0: float, sigma: float,
                         kx0: float, ky0: float) -> np.ndarray:
    """Bins ((cy * nx + cx) * n_k + (My - M_min)) * n_k + (Mx - M_min)."""
    fx = _cell_weights(mesh.nx, mesh.dx, x0, sigma)
    fy = _cell_weights(mesh.ny, mesh.dx, y0, sigma)
    gx = _mom_weights(mesh.n_k, mesh.M_min, mesh.dk, kx0, sigma)
    gy = _mom_weights(mesh.n_k, mesh.M_min, mesh.dk, ky0, sigma)
    F = fy[:, None, None, None] * fx[None, :, None, None] * gy[None, None, :, None] * gx[None, None, None, :]
    return _round_counts(F.ravel(), N0)


# ----------------------------------------------------------------------------- workloads
@dataclass
class RunConfig:
    """A barrier/packet time-loop workload."""
    name: str
    mesh: object
    V: np.ndarray
    bin_counts: np.ndarray
    N0: int
    dt: float
    steps: int
    seed: int = 0
    meta: dict = field(default_factory=dict)


def config_c1() -> RunConfig:
    """1-D plain FP64: 100 cells of 1 nm, L_C = 30 nm, barrier 0.3 eV sigma 3 nm at 50 nm,
    packet at 25 nm sigma 5 nm with 0.1 eV, 1e5 particles, dt 1 fs, 100 steps."""
    mesh = Mesh1D(nx=100, dx=1.0, n_m=30, pos_f64=True)
    V = gaussian_barrier_1d(mesh, 0.3, 3.0, 50.0)
    k0 = k_for_energy(0.1)
    bc = packet_bin_counts_1d(mesh, 1e5, 25.0, 5.0, k0)
    return RunConfig("c1_1d_fp64_100cells_30m_1e5p", mesh, V, bc, int(1e5), 1.0, 100,
                     meta={"k0": k0})


def config_c2(N0: float = 1e7, steps: int = 400) -> RunConfig:
    """1-D paper-shaped run: 400 cells of 0.5 nm, L_C = 40 nm, barrier 0.3 eV sigma 2 nm at
    100 nm, packet at 50 nm sigma 10 nm with 0.1 eV, 1e7 particles (FP32), 400 x 0.5 fs."""
    mesh = Mesh1D(nx=400, dx=0.5, n_m=80, pos_f64=False)
    V = gaussian_barrier_1d(mesh, 0.3, 2.0, 100.0)
    k0 = k_for_energy(0.1)
    bc = packet_bin_counts_1d(mesh, N0, 50.0, 10.0, k0)
    return RunConfig("c2_1d_400cells_80m_1e7p_fp32", mesh, V, bc, int(N0), 0.5, steps,
                     meta={"k0": k0})


def config_c4_run(N0: float = 1e7, steps: int = 400) -> RunConfig:
    """C2 physics on the 1024-cell, 256-m mesh of the learned-kernel workload."""
    mesh = Mesh1D(nx=1024, dx=0.5, n_m=256, pos_f64=False)
    V = gaussian_barrier_1d(mesh, 0.3, 2.0, 256.0)
    k0 = k_for_energy(0.1)
    bc = packet_bin_counts_1d(mesh, N0, 206.0, 10.0, k0)
    return RunConfig("c4_1d_1024cells_256m_1e7p_fp32", mesh, V, bc, int(N0), 0.5, steps,
                     meta={"k0": k0})


def config_c5(N0: float = 5e7, steps: int = 200) -> RunConfig:
    """2-D: 256 x 256 cells of 0.5 nm, L_C = 16 nm (32 x 32 m), dot 0.2 eV sigma 4 nm at
    (64, 64) nm, packet sigma 8 nm at (32, 64) nm with 0.1 eV along +x, 5e7 particles."""
    mesh = Mesh2D(nx=256, ny=256, dx=0.5, n_m=32, pos_f64=False)
    V = gaussian_dot_2d(mesh, 0.2, 4.0, 64.0, 64.0)
    k0 = k_for_energy(0.1)
    bc = packet_bin_counts_2d(mesh, N0, 32.0, 64.0, 8.0, k0, 0.0)
    return RunConfig("c5_2d_256x256_32x32m_5e7p_fp32", mesh, V, bc, int(N0), 0.5, steps,
                     meta={"k0": k0})


# Kernel-batch workloads (precision and learned forms).
C3 = {"B": 4096, "nx": 2048, "n_m": 512, "dx": 0.5, "seed": 0}
C4 = {"B": 100000, "nx": 1024, "n_m": 256, "dx": 0.5, "seed": 0, "test_seed": 1, "test_B": 1000}
