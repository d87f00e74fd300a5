"""Split-step Fourier solution of the 1-D Schrodinger equation, the physics reference for the
barrier and free-packet checks (test infrastructure; not part of either implementation).

A Gaussian state psi ~ exp(-(x-x0)^2/(2 sigma^2) + i k0 x) has exactly the Wigner function of
eq.(6) read with the printed sigma; it is propagated with Strang splitting on a fine periodic
grid much larger than the simulation domain."""
import numpy as np

from paper_1806_00082_amd.inputs import HBAR_EVFS, HBAR_OVER_ME


def densities(x0, sigma, k0, barrier, times, nx, dx, dxs=0.05, dts=0.025, pad=200.0):
    """Cell-integrated |psi|^2 on [0, nx dx) at each time (fs); barrier = (U, s, b) or None."""
    L = nx * dx
    xs = np.arange(-pad, L + pad, dxs)
    ks = 2 * np.pi * np.fft.fftfreq(len(xs), d=dxs)
    psi = np.exp(-(xs - x0) ** 2 / (2 * sigma ** 2) + 1j * k0 * xs)
    psi /= np.sqrt((np.abs(psi) ** 2).sum() * dxs)
    Vs = np.zeros_like(xs) if barrier is None else barrier[0] * np.exp(-(xs - barrier[2]) ** 2 / (2 * barrier[1] ** 2))
    kin = np.exp(-1j * HBAR_OVER_ME * ks ** 2 * dts / 2)
    half = np.exp(-1j * Vs * dts / (2 * HBAR_EVFS))
    inside = (xs >= 0) & (xs < L)
    cell = np.floor(xs[inside] / dx).astype(np.int64)
    out, t = [], 0.0
    for T in times:
        for _ in range(int(round((T - t) / dts))):
            psi = half * np.fft.ifft(kin * np.fft.fft(half * psi))
        t = T
        out.append(np.bincount(cell, weights=(np.abs(psi) ** 2)[inside] * dxs, minlength=nx))
    return out
