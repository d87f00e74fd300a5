"""Pins of the oracle's trainable kernel network, eq.(5) of Sec. 2.3, and its gradients."""
import numpy as np
import pytest

from paper_1806_00082_amd import inputs

HB = inputs.HBAR_EVFS


def test_n1_analytic_is_exact(orc):
    """N = 1 with the analytic weights (w_l = -2 dx/(hbar L_C)) is eq.(4) itself."""
    V = inputs.random_potentials(2, 200, 0.5, seed=4)
    n_m = 64
    wV, wT, W = orc.analytic_weights(n_m, 1, HB)
    Kh = orc.surrogate_fwd(V, n_m, 1, wV, wT, W)
    Kx = orc.full_to_half(orc.kernel_1d(V, n_m, HB))
    assert np.max(np.abs(Kh - Kx)) <= 1e-12 * np.abs(Kx).max()


@pytest.mark.parametrize("N", [2, 4, 8])
def test_barycentric_exact_on_blockwise_constant(orc, N):
    """sum_{p<N} sin(a + p d) = sin(a + (N-1)d/2) sin(N d/2)/sin(d/2), and for N = 2^L
    sin(N d/2)/sin(d/2) = N prod_{s<L} cos(2^s d/2).  So when V is constant on every group
    of N window cells, eq.(5) with wV = 1, wT = 1/N, W = c equals eq.(4) exactly."""
    n_m, nx = 32, 160
    P = n_m // 2
    rng = np.random.default_rng(N)
    blocks = rng.normal(size=nx // N)
    V = np.repeat(blocks, N)                        # constant on [kN, kN+N)
    wV, wT, W = orc.analytic_weights(n_m, N, HB)
    Kh = orc.surrogate_fwd(V, n_m, N, wV, wT, W)[0]
    Kx = orc.full_to_half(orc.kernel_1d(V, n_m, HB))[0]
    aligned = [i for i in range(P, nx - P) if (i - P) % N == 0]
    assert len(aligned) > 5
    scale = np.abs(Kx[aligned]).max()
    assert np.max(np.abs(Kh[aligned] - Kx[aligned])) <= 1e-12 * scale
    # and it is only an approximation for a generic potential
    V2 = rng.normal(size=nx)
    Kh2 = orc.surrogate_fwd(V2, n_m, N, wV, wT, W)[0]
    Kx2 = orc.full_to_half(orc.kernel_1d(V2, n_m, HB))[0]
    assert np.max(np.abs(Kh2 - Kx2)) > 1e-3 * np.abs(Kx2).max()


def test_n2_matches_printed_two_term_form(orc):
    """N = 2 analytic weights give the two-term form derived in Sec. 2.3:
    c cos(pi m / n_m) sum_g [V(2g) + V(2g+1)] sin((theta_2g + theta_2g+1)/2)."""
    n_m, nx = 20, 50
    P = n_m // 2
    V = np.random.default_rng(12).normal(size=nx)
    wV, wT, W = orc.analytic_weights(n_m, 2, HB)
    Kh = orc.surrogate_fwd(V, n_m, 2, wV, wT, W)[0]
    c = -2.0 / (HB * n_m)
    i = 25
    for m in range(1, P + 1):
        acc = 0.0
        for g in range(P):
            o0, o1 = -P + 2 * g, -P + 2 * g + 1
            th0, th1 = 2 * np.pi * o0 * m / n_m, 2 * np.pi * o1 * m / n_m
            acc += (V[i + o0] + V[i + o1]) * np.sin(0.5 * (th0 + th1))
        ref = c * np.cos(np.pi * m / n_m) * acc
        assert abs(Kh[i, m - 1] - ref) <= 1e-12 * max(1.0, abs(ref))


@pytest.mark.parametrize("N", [1, 2, 4])
def test_surrogate_gradients_finite_differences(orc, N):
    """Analytic gradients of <E, Kh> against central differences of the forward."""
    n_m, nx, B = 16, 40, 2
    rng = np.random.default_rng(20 + N)
    V = rng.normal(size=(B, nx))
    wV = rng.normal(size=N)
    wT = rng.normal(size=N) / N
    W = rng.normal(size=n_m // N)
    cells = np.array([0, 3, 17, 39, 20], np.int32)
    E = rng.normal(size=(B, len(cells), n_m // 2))
    dwV, dwT, dW, dV = orc.surrogate_bwd(V, n_m, N, wV, wT, W, E, cells=cells)

    def f(wV_, wT_, W_, V_):
        return np.sum(E * orc.surrogate_fwd(V_, n_m, N, wV_, wT_, W_, cells=cells))

    h = 1e-6
    for arr, grad, idx in ((wV, dwV, range(N)), (wT, dwT, range(N)), (W, dW, range(0, n_m // N, 3))):
        for k in idx:
            a = arr.copy()
            a[k] += h
            args_p = [wV, wT, W, V]
            args_p[[id(wV), id(wT), id(W)].index(id(arr))] = a
            fp = f(*args_p)
            a[k] -= 2 * h
            fm = f(*args_p)
            fd = (fp - fm) / (2 * h)
            assert abs(grad[k] - fd) <= 1e-6 * max(1.0, abs(fd))
    for (b, l) in ((0, 0), (1, 5), (0, 20), (1, 39)):
        Vp = V.copy()
        Vp[b, l] += h
        fp = f(wV, wT, W, Vp)
        Vp[b, l] -= 2 * h
        fm = f(wV, wT, W, Vp)
        fd = (fp - fm) / (2 * h)
        assert abs(dV[b, l] - fd) <= 1e-6 * max(1.0, abs(fd))


def test_barycentric_weights_near_least_squares_optimum(orc):
    """With wV, wT at the barycentric values eq.(5) is linear in W, so the best W is a
    least-squares problem: on random Gaussian-bell potentials it improves the held-out RMS
    error by under 1% -- the trainable form has little room beyond the barycentric network."""
    nx, n_m, N = 128, 32, 2
    H = n_m // N
    wV, wT, W = orc.analytic_weights(n_m, N, HB)
    Vtr = inputs.random_potentials(24, nx, 0.5, seed=0)
    Vte = inputs.random_potentials(24, nx, 0.5, seed=1)

    def feats(V):
        return np.stack([orc.surrogate_fwd(V, n_m, N, wV, wT, np.eye(H)[g]).ravel() for g in range(H)], 1)

    Ftr, Fte = feats(Vtr), feats(Vte)
    Ktr = orc.full_to_half(orc.kernel_1d(Vtr, n_m, HB)).ravel()
    Kte = orc.full_to_half(orc.kernel_1d(Vte, n_m, HB)).ravel()
    Wopt = np.linalg.lstsq(Ftr, Ktr, rcond=None)[0]
    rms = lambda w: np.sqrt(np.mean((Fte @ w - Kte) ** 2) / np.mean(Kte ** 2))
    assert rms(Wopt) > 0.99 * rms(W)
    assert rms(W) < 0.15


# ----------------------------------------------------------------------------- d = 2
def _v2(seed, nx, ny):
    rng = np.random.default_rng(seed)
    x = (np.arange(nx) + 0.5) * 0.5
    y = (np.arange(ny) + 0.5) * 0.5
    V = np.zeros((ny, nx))
    for _ in range(3):
        cx, cy, h, s = rng.uniform(0, nx * 0.5), rng.uniform(0, ny * 0.5), rng.uniform(0, 0.4), rng.uniform(1, 3)
        V += h * np.exp(-((x[None] - cx) ** 2 + (y[:, None] - cy) ** 2) / (2 * s * s))
    return V


@pytest.mark.parametrize("n_m", [4, 8, 16])
def test_surrogate_2d_n1_is_the_2d_kernel(orc, n_m):
    """With N = 1 and the analytic weights the d = 2 network is the d = 2 kernel of eq.(4)
    (pinned independently by brute force and by its reduction to 1-D), on every cell of a mesh
    smaller than the window (both edge clampings and the end-point means in play)."""
    nx, ny = 13, 9
    V = _v2(1, nx, ny)
    ref = orc.kernel_2d(V, n_m, HB)
    got = orc.surrogate_fwd_2d(V, n_m, 1, *orc.analytic_weights_2d(n_m, 1, HB))
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("N", [2, 4])
def test_surrogate_2d_reduces_to_1d_for_a_potential_of_x(orc, N):
    """V(x, y) = V1(x): the my = 0 row is the 1-D network of eq.(5) (pinned against eq.(4) and
    the barycentric form) evaluated with the end-point mean in the window, and every other row
    vanishes (the sum over gy of the phases cancels or the cos prefactor is 0)."""
    n_m, nx, ny = 16, 30, 7
    P = n_m // 2
    rng = np.random.default_rng(N)
    V1 = rng.uniform(0, 0.3, nx)
    V = np.tile(V1, (ny, 1))
    wV1, wT1, W1 = rng.normal(1, 0.1, N), rng.normal(1.0 / N, 0.02, N), rng.normal(-2 / (HB * n_m), 1e-3, n_m // N)
    H = n_m // N
    # 2-D weights that reduce to the 1-D ones: wV(px, py) = wV1(px) / N, W(gx, gy) = W1(gx) / H
    wV2 = np.tile(wV1 / N, N)
    W2 = np.tile(W1 / H, H)
    cells = np.array([P, 15, nx - 1 - P, 2 * nx + 11, 5 * nx + 19], dtype=np.int32)  # interior in x
    got = orc.surrogate_fwd_2d(V, n_m, N, wV2, wT1, np.full(N, 1.0 / N), W2, cells=cells)[0]
    for r, cid in enumerate(cells):
        ix = int(cid) % nx
        # the 1-D window of this cell with the end point -P holding the mean of both ends
        Vc = V1.copy()
        Vc[ix - P] = 0.5 * (V1[ix - P] + V1[ix + P])
        full1 = orc.half_to_full(orc.surrogate_fwd(Vc[None], n_m, N, wV1, wT1, W1,
                                                   cells=np.array([ix], np.int32))[0])[0]
        row0 = got[r, P]          # my = 0
        assert np.abs(row0 - full1).max() <= 1e-12 * np.abs(full1).max()
        others = np.delete(got[r], P, axis=0)
        assert np.abs(others).max() <= 1e-12 * np.abs(full1).max()
