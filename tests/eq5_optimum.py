"""Least-squares optimum of the trainable network of eq.(5) (Sec. 2.3) over a data set,
in closed form (test-side analysis; numpy only).

The network's angle weights wT enter only through u_g = (2 pi / n_m)((N g - P) S + T) with
S = sum_p wT_p and T = sum_p p wT_p, and for fixed (S, T) the network is linear in the
products C[g, p] = W_g wV_p.  Its mean squared error against the exact kernel of eq.(4),
K(i, m) = c sum_{o = -P}^{P-1} sin(2 pi o m / n_m) V(i + o) (clamped indices, the j-sum of
eq.(4) unfolded onto one side), over all cells i, momenta m = 1..P and potentials, is then
the quadratic form  C^T G C - 2 C^T r + y^T y  whose coefficients need only the lagged
correlation R[o, o'] = sum_{b,i} V_b(i + o) V_b(i + o') of the data and sums over m of sines.
Minimising over an unconstrained C (a relaxation of the product W_g wV_p) and scanning
(S, T) bounds from below every MSE the network can reach, jointly over (wV, wT, W).
"""
import numpy as np


def lagged_correlation(V, P):
    """R[a, b] = sum over potentials and cells of V(clamp(i + o_a)) V(clamp(i + o_b)),
    o = -P..P-1 (index a = o + P)."""
    V = np.atleast_2d(V)
    nx = V.shape[1]
    idx = np.clip(np.arange(nx)[:, None] + np.arange(-P, P)[None, :], 0, nx - 1)
    R = np.zeros((2 * P, 2 * P))
    for v in V:
        X = v[idx]
        R += X.T @ X
    return R


def quadratic_form(R, n_m, N, S, T, hbar):
    """(G, r, yy, count_per_row) of the MSE sum over all (potential, cell, m) as a function
    of C [H * N] (index g * N + p)."""
    P, H = n_m // 2, n_m // N
    c = -2.0 / (hbar * n_m)
    m = np.arange(1, P + 1)
    Pi = np.ones(P)
    for s in range(int(round(np.log2(N)))):
        Pi *= np.cos(np.pi * 2 ** s * m / n_m)
    u = (2 * np.pi / n_m) * ((N * np.arange(H) - P) * S + T)
    sg = np.sin(np.outer(u, m))                                        # [H][P]
    so = np.sin(np.outer(np.arange(-P, P), m) * 2 * np.pi / n_m)       # [2P][P]
    off = (N * np.arange(H)[:, None] + np.arange(N)[None, :]).ravel()   # o + P of (g, p)
    gi = np.repeat(np.arange(H), N)
    Tt = (sg * Pi ** 2) @ sg.T
    G = Tt[np.ix_(gi, gi)] * R[np.ix_(off, off)]
    M = (sg * Pi) @ so.T                                               # [H][2P]
    r = c * np.einsum("kn,kn->k", M[gi], R[off])
    yy = c * c * np.einsum("am,bm,ab->", so, so, R)
    return G, r, yy


def mse(G, r, yy, C):
    return float(C @ G @ C - 2.0 * C @ r + yy)


def barycentric_C(n_m, N, hbar):
    return np.full((n_m // N) * N, -2.0 / (hbar * n_m))


def best_C(G, r):
    return np.linalg.lstsq(G, r, rcond=None)[0]
