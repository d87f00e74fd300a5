"""Pins of the oracle's Wigner kernel (eq.(4), Sec. 2.2) against mathematics it must obey.

None of these re-types the oracle's sum: each checks it against a library transform, a
closed form, a high-precision brute force, or an invariant of the kernel.
"""
import math

import mpmath
import numpy as np
import pytest
import scipy.fft

from paper_1806_00082_amd import inputs

HB = inputs.HBAR_EVFS


def _diffs(V, i, P):
    """D_i(j) = V(i+j) - V(i-j), j = 1..P, nearest-edge value outside the mesh."""
    nx = len(V)
    j = np.arange(1, P + 1)
    return V[np.clip(i + j, 0, nx - 1)] - V[np.clip(i - j, 0, nx - 1)]


@pytest.mark.parametrize("nx,n_m", [(64, 16), (100, 30), (200, 80), (96, 64)])
def test_dst1_identity(orc, nx, n_m):
    """For m = 1..P-1 the folded eq.(4) is a type-I discrete sine transform of the
    potential differences: K(i, .) = (c/2) DST-I(D_i(1..P-1)) with c = -2/(hbar n_m)."""
    rng = np.random.default_rng(1)
    V = rng.normal(size=nx)
    P = n_m // 2
    K = orc.kernel_1d(V, n_m, HB)[0]
    c = -2.0 / (HB * n_m)
    kmax = np.abs(K).max()
    for i in range(nx):
        D = _diffs(V, i, P)
        ref = 0.5 * c * scipy.fft.dst(D[: P - 1], type=1)
        got = K[i, P + 1:]
        assert np.max(np.abs(got - ref)) <= 1e-13 * kmax


def test_parseval_and_inversion(orc):
    """Orthogonality of the DST-I basis: sum_m K^2 = c^2 (P/2) sum_{j<P} D^2, and D is
    recovered from K by the inverse transform."""
    n_m, nx = 40, 120
    P = n_m // 2
    V = np.random.default_rng(2).uniform(0, 0.5, nx)
    K = orc.kernel_1d(V, n_m, HB)[0]
    c = -2.0 / (HB * n_m)
    for i in (0, 7, 60, 119):
        D = _diffs(V, i, P)[: P - 1]
        k = K[i, P + 1:]
        lhs = np.sum(k * k)
        rhs = c * c * (P / 2.0) * np.sum(D * D)
        assert abs(lhs - rhs) <= 1e-13 * rhs
        Drec = (2.0 / (P * c)) * scipy.fft.dst(k, type=1) / 2.0
        assert np.max(np.abs(Drec - D)) <= 1e-12 * np.abs(D).max()


def test_real_odd_periodic(orc):
    """V_W is real and odd in m; K(i,0) = K(i,-P) = 0 exactly (sin 0, sin(pi m))."""
    n_m, nx = 30, 50
    P = n_m // 2
    V = np.random.default_rng(3).normal(size=nx)
    K = orc.kernel_1d(V, n_m, HB)[0]
    assert np.all(K[:, P] == 0.0)
    assert np.all(K[:, 0] == 0.0)
    for m in range(1, P):
        assert np.max(np.abs(K[:, P + m] + K[:, P - m])) <= 1e-15 * np.abs(K).max()


def test_constant_potential_vanishes(orc):
    """A constant potential has no Wigner kernel, on every cell (edges included)."""
    V = np.full(37, 0.731)
    K = orc.kernel_1d(V, 24, HB)
    assert np.all(K == 0.0)


@pytest.mark.parametrize("n_m", [16, 30, 80])
def test_linear_potential_closed_form(orc, n_m):
    """V = F x: D_i(j) = 2 F j dx on interior cells and the sum sum_j j sin(j a) has a closed
    form, giving K(i,m) = (F dx / hbar) (-1)^m cot(pi m / n_m), independent of i."""
    P = n_m // 2
    dx, F = 0.5, 0.013
    nx = 3 * n_m
    x = (np.arange(nx) + 0.5) * dx
    K = orc.kernel_1d(F * x, n_m, HB)[0]
    m = np.arange(-P + 1, P)
    m = m[m != 0]
    ref = (F * dx / HB) * (-1.0) ** m * (1.0 / np.tan(np.pi * m / n_m))
    for i in range(P, nx - P):
        got = K[i, m + P]
        assert np.max(np.abs(got - ref)) <= 1e-13 * np.abs(ref).max()


def test_gaussian_continuum_limit(orc):
    """Gaussian barrier U exp(-(x-b)^2/(2 s^2)) well inside the coherence window: the finite
    sum equals the continuous transform -(2 U s sqrt(2 pi)/(hbar L_C)) exp(-2 k^2 s^2)
    sin(2 k (b - x)), up to the Gaussian tail beyond the window (exp(-18) relative)."""
    mesh = inputs.Mesh1D(nx=400, dx=0.5, n_m=80)
    U, s, b = 0.3, 2.0, 100.0
    V = inputs.gaussian_barrier_1d(mesh, U, s, b)
    K = orc.kernel_1d(V, mesh.n_m, HB)[0]
    P = mesh.n_m // 2
    x = mesh.centres()
    k = (np.arange(mesh.n_m) - P) * mesh.dk
    ok = np.abs(x - b) <= mesh.L_C / 2 - 6 * s
    assert ok.sum() > 10
    ref = -(2 * U * s * math.sqrt(2 * math.pi) / (HB * mesh.L_C)) * np.exp(-2 * (k * s) ** 2)[None, :] \
        * np.sin(2 * k[None, :] * (b - x[ok, None]))
    # tail bound: |c| * 2 * sum of the neglected samples <= |c| * 2 * U * exp(-18) * (L_C/dx)
    bound = (2.0 / (HB * mesh.n_m)) * 2 * U * math.exp(-18.0) * mesh.n_m
    assert np.max(np.abs(K[ok] - ref)) <= bound + 1e-12


def test_literal_and_folded_agree(orc):
    """The printed form (offsets -P..P, both terms) and the folded form agree to rounding."""
    rng = np.random.default_rng(4)
    V = rng.normal(size=(3, 45))
    cells = np.array([0, 1, 5, 22, 44, 44, 3], dtype=np.int32)
    Kf = orc.kernel_1d(V, 20, HB, cells=cells)
    Kl = orc.kernel_1d(V, 20, HB, cells=cells, literal=True)
    assert np.max(np.abs(Kf - Kl)) <= 1e-14 * np.abs(Kf).max()


def _mp_kernel(V, i, m, n_m):
    """eq.(4) term by term in 50-digit arithmetic."""
    mpmath.mp.dps = 50
    P = n_m // 2
    nx = len(V)
    acc = mpmath.mpf(0)
    for j in range(-P, P + 1):
        vp = mpmath.mpf(float(V[min(max(i + j, 0), nx - 1)]))
        vm = mpmath.mpf(float(V[min(max(i - j, 0), nx - 1)]))
        acc += mpmath.sin(2 * mpmath.pi * j * m / n_m) * (vp - vm)
    return -acc / (mpmath.mpf(HB) * n_m)


@pytest.mark.parametrize("nx,n_m", [(8, 4), (20, 16), (32, 12)])
def test_brute_force_high_precision(orc, nx, n_m):
    """Tiny meshes: both oracle forms equal eq.(4) evaluated in 50 digits."""
    V = np.random.default_rng(5 + nx).uniform(-1, 1, nx)
    P = n_m // 2
    Kf = orc.kernel_1d(V, n_m, HB)[0]
    Kl = orc.kernel_1d(V, n_m, HB, literal=True)[0]
    ref = np.array([[float(_mp_kernel(V, i, t - P, n_m)) for t in range(n_m)] for i in range(nx)])
    scale = np.abs(ref).max()
    assert np.max(np.abs(Kf - ref)) <= 1e-15 * scale * P
    assert np.max(np.abs(Kl - ref)) <= 1e-15 * scale * P


def test_linearity_and_shift(orc):
    rng = np.random.default_rng(6)
    V1, V2 = rng.normal(size=60), rng.normal(size=60)
    a = 0.37
    K1, K2 = orc.kernel_1d(V1, 16, HB)[0], orc.kernel_1d(V2, 16, HB)[0]
    K12 = orc.kernel_1d(V1 + a * V2, 16, HB)[0]
    assert np.max(np.abs(K12 - (K1 + a * K2))) <= 1e-14 * np.abs(K12).max()
    # shift-equivariance on cells whose window stays inside the mesh
    Vs = np.roll(V1, 3)
    Ks = orc.kernel_1d(Vs, 16, HB)[0]
    for i in range(8 + 3, 60 - 8):
        assert np.max(np.abs(Ks[i] - K1[i - 3])) <= 1e-14 * np.abs(K1).max()


def test_classical_limit_sign(orc):
    """Sign convention of eq.(4) with the creation rule (+s at M+m'): for V = F x the
    creation term sum_m' K(m') f(M - m') is the classical force term (F/(hbar dk)) df/dM
    on a smooth momentum distribution (Newton: dk/dt = -F/hbar moves f towards -M)."""
    n_m, dx = 80, 0.5
    F = 0.01
    mesh = inputs.Mesh1D(nx=3 * n_m, dx=dx, n_m=n_m)
    K = orc.kernel_1d(F * mesh.centres(), n_m, HB)[0][n_m + 3]
    P = n_m // 2
    Ms = np.arange(-400, 401)
    f = np.exp(-((Ms * mesh.dk - 0.5) ** 2) / (2 * 0.4 ** 2))
    fd = -f * (Ms * mesh.dk - 0.5) * mesh.dk / 0.4 ** 2      # df/dM
    for M in (-10, 0, 5, 12):
        lhs = sum(K[t] * f[M - (t - P) + 400] for t in range(n_m))
        rhs = F / (HB * mesh.dk) * fd[M + 400]
        assert abs(lhs / rhs - 1.0) < 0.01


# ----------------------------------------------------------------------------- 2-D
def test_2d_reduces_to_1d(orc):
    """V(x, y) = V1(x): the y sum of the half-weighted sines is n_m delta(m_y), so
    K2(i; m_x, m_y) = delta(m_y, 0) K1(i_x; m_x)."""
    n_m, nx, ny = 8, 12, 7
    P = n_m // 2
    V1 = np.random.default_rng(7).normal(size=nx)
    V2 = np.tile(V1, (ny, 1))
    K2 = orc.kernel_2d(V2, n_m, HB)[0].reshape(ny, nx, n_m, n_m)
    K1 = orc.kernel_1d(V1, n_m, HB)[0]
    scale = np.abs(K1).max()
    for iy in range(ny):
        assert np.max(np.abs(K2[iy, :, P, :] - K1)) <= 1e-13 * scale
        others = np.delete(K2[iy], P, axis=1)
        assert np.max(np.abs(others)) <= 1e-13 * scale


def test_2d_odd_and_constant(orc):
    n_m = 8
    P = n_m // 2
    V = np.random.default_rng(8).normal(size=(6, 9))
    K = orc.kernel_2d(V, n_m, HB)[0]
    for tx in range(1, n_m):
        for ty in range(1, n_m):
            assert np.max(np.abs(K[:, ty, tx] + K[:, 2 * P - ty, 2 * P - tx])) <= 1e-14 * np.abs(K).max()
    assert np.all(K[:, P, P] == 0.0)
    assert np.all(orc.kernel_2d(np.full((5, 5), 2.0), n_m, HB) == 0.0)


def test_2d_separable_equals_direct(orc):
    """sin(a + b) = sin a cos b + cos a sin b splits the d = 2 sum into two products of
    per-axis matrices: K = c2 (S_y D C_x^T + C_y D S_x^T) with D_j = V(i+j) - V(i-j)."""
    n_m, nx, ny = 8, 10, 9
    P = n_m // 2
    V = np.random.default_rng(9).normal(size=(ny, nx))
    K = orc.kernel_2d(V, n_m, HB)[0]
    j = np.arange(-P, P + 1)
    w = np.where(np.abs(j) == P, 0.5, 1.0)
    m = np.arange(-P, P)
    S = np.sin(2 * np.pi * np.outer(m, j) / n_m) * w[None, :]
    C = np.cos(2 * np.pi * np.outer(m, j) / n_m) * w[None, :]
    c2 = -1.0 / (HB * n_m * n_m)
    for iy in range(ny):
        for ix in range(nx):
            yy_p = np.clip(iy + j, 0, ny - 1)
            yy_m = np.clip(iy - j, 0, ny - 1)
            xx_p = np.clip(ix + j, 0, nx - 1)
            xx_m = np.clip(ix - j, 0, nx - 1)
            D = V[np.ix_(yy_p, xx_p)] - V[np.ix_(yy_m, xx_m)]
            ref = c2 * (S @ D @ C.T + C @ D @ S.T)
            assert np.max(np.abs(K[iy * nx + ix] - ref)) <= 1e-13 * np.abs(ref).max() + 1e-300


def test_2d_brute_force_high_precision(orc):
    mpmath.mp.dps = 40
    n_m, nx, ny = 4, 3, 3
    P = n_m // 2
    V = np.random.default_rng(10).uniform(-1, 1, (ny, nx))
    K = orc.kernel_2d(V, n_m, HB)[0]
    for cid in range(nx * ny):
        ix, iy = cid % nx, cid // nx
        for ty in range(n_m):
            for tx in range(n_m):
                mx, my = tx - P, ty - P
                acc = mpmath.mpf(0)
                for jy in range(-P, P + 1):
                    for jx in range(-P, P + 1):
                        w = mpmath.mpf(0.5 if abs(jx) == P else 1) * mpmath.mpf(0.5 if abs(jy) == P else 1)
                        vp = V[min(max(iy + jy, 0), ny - 1), min(max(ix + jx, 0), nx - 1)]
                        vm = V[min(max(iy - jy, 0), ny - 1), min(max(ix - jx, 0), nx - 1)]
                        acc += w * mpmath.sin(2 * mpmath.pi * (mx * jx + my * jy) / n_m) * (mpmath.mpf(vp) - mpmath.mpf(vm))
                ref = float(-acc / (mpmath.mpf(HB) * n_m * n_m))
                assert abs(K[cid, ty, tx] - ref) <= 1e-14


# ----------------------------------------------------------------------------- adjoint
def test_kernel_adjoint_dot_product(orc):
    """V -> K_half is linear, so <G, K(dV)> = <K^T G, dV> for any G, dV."""
    rng = np.random.default_rng(11)
    n_m, nx, B = 24, 50, 2
    P = n_m // 2
    G = rng.normal(size=(B, nx, P))
    dV = rng.normal(size=(B, nx))
    Kh = orc.full_to_half(orc.kernel_1d(dV, n_m, HB))
    lhs = np.sum(G * Kh)
    rhs = np.sum(orc.kernel_bwd_1d(G, n_m, HB) * dV)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_kernel_adjoint_cells_dot_product(orc):
    """The same identity on a cell list with repeats and both edges: rows of the forward on
    `cells` against the adjoint on `cells` (the forward is pinned independently above)."""
    rng = np.random.default_rng(12)
    n_m, nx, B = 20, 37, 3
    P = n_m // 2
    cells = np.array([0, 5, 5, 36, 18, 1, 35, 20, 9], dtype=np.int32)
    G = rng.normal(size=(B, len(cells), P))
    dV = rng.normal(size=(B, nx))
    Kh = orc.full_to_half(orc.kernel_1d(dV, n_m, HB, cells=cells))
    lhs = np.sum(G * Kh)
    rhs = np.sum(orc.kernel_bwd_1d(G, n_m, HB, nx=nx, cells=cells) * dV)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # the all-cells list in order is the all-cells adjoint
    Ga = rng.normal(size=(B, nx, P))
    a = orc.kernel_bwd_1d(Ga, n_m, HB)
    b = orc.kernel_bwd_1d(Ga, n_m, HB, nx=nx, cells=np.arange(nx, dtype=np.int32))
    assert np.array_equal(a, b)


def test_kernel_adjoint_cells_finite_difference(orc):
    """K is linear in V, so one finite difference per coordinate is exact up to rounding:
    dL/dV[l] = L(e_l) for L(V) = <G, K(V)> on the cell list."""
    rng = np.random.default_rng(13)
    n_m, nx = 12, 15
    P = n_m // 2
    cells = np.array([2, 14, 7, 0, 7], dtype=np.int32)
    G = rng.normal(size=(1, len(cells), P))
    grad = orc.kernel_bwd_1d(G, n_m, HB, nx=nx, cells=cells)[0]
    for l in range(nx):
        e = np.zeros(nx)
        e[l] = 1.0
        fd = np.sum(G * orc.full_to_half(orc.kernel_1d(e, n_m, HB, cells=cells)))
        assert abs(fd - grad[l]) <= 1e-13 * max(1.0, abs(fd)) / HB
