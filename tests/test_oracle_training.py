"""Pins of the oracle's training step (Sec. 3: supervised SGD on the MSE between the network
of eq.(5) and the exact kernel of eq.(4)).  Everything here runs on the CPU.

The step is pinned against the loss it descends, computed from the independently pinned
forward of eq.(5): the gradient the step applies must equal finite differences of that loss,
per parameter group and with W stepped in units of c; a zero residual must be a fixed point.
"""
import numpy as np
import pytest

from paper_1806_00082_amd import inputs

HB = inputs.HBAR_EVFS


def _case(seed, nx=24, n_m=16, N=2, B=2):
    rng = np.random.default_rng(seed)
    V = inputs.random_potentials(B, nx, 0.5, seed)
    c = -2.0 / (HB * n_m)
    w = (rng.normal(1.0, 0.05, N), rng.normal(1.0 / N, 0.02, N), c * rng.normal(1.0, 0.05, n_m // N))
    return V, w, c


def _loss(orc, V, K, n_m, N, w, inv_scale):
    Kh = orc.surrogate_fwd(V, n_m, N, *w)
    return float(np.mean(((Kh - K) * inv_scale) ** 2))


def test_mse_grad_is_the_derivative_of_the_loss(orc):
    rng = np.random.default_rng(0)
    Kh, K = rng.normal(size=50), rng.normal(size=50)
    s = 3.0
    loss, E = orc.mse_grad(Kh, K, s)
    assert loss == pytest.approx(np.mean(((Kh - K) * s) ** 2), rel=1e-14)
    h = 1e-4
    for k in (0, 17, 49):
        up, dn = Kh.copy(), Kh.copy()
        up[k] += h
        dn[k] -= h
        fd = (orc.mse_grad(up, K, s)[0] - orc.mse_grad(dn, K, s)[0]) / (2 * h)
        assert abs(fd - E[k]) <= 1e-9 * max(1.0, abs(E[k]))


@pytest.mark.parametrize("N", [1, 2, 4])
def test_sgd_step_applies_the_loss_gradient(orc, N):
    """(w0 - w1) / lr is the finite-difference gradient of the loss, per group; for W the
    step is lr c^2 dL/dW (W in units of c)."""
    n_m = 16
    V, w0, c = _case(1, n_m=n_m, N=N)
    K = orc.full_to_half(orc.kernel_1d(V, n_m, HB))
    inv = 1.0 / abs(c)
    lr = (0.3, 0.002, 0.5)
    loss0, w1 = orc.sgd_step(V, K, n_m, N, HB, w0, lr, inv_scale=inv)
    assert loss0 == pytest.approx(_loss(orc, V, K, n_m, N, w0, inv), rel=1e-12)
    scale = (lr[0], lr[1], lr[2] * c * c)
    for gi in range(3):
        g_step = (w0[gi] - w1[gi]) / scale[gi]
        for k in range(len(w0[gi])):
            h = 1e-6 * max(1.0, abs(w0[gi][k]))
            wp = [a.copy() for a in w0]
            wm = [a.copy() for a in w0]
            wp[gi][k] += h
            wm[gi][k] -= h
            fd = (_loss(orc, V, K, n_m, N, wp, inv) - _loss(orc, V, K, n_m, N, wm, inv)) / (2 * h)
            tol = 1e-6 * max(np.abs(g_step).max(), 1e-3 / abs(c) if gi == 2 else 1e-3)
            assert abs(g_step[k] - fd) <= tol, (N, gi, k, g_step[k], fd)


def test_sgd_step_descends(orc):
    """A small step lowers the loss by lr |g|^2 to first order (one group at a time)."""
    n_m, N = 16, 2
    V, w0, c = _case(2, n_m=n_m, N=N)
    K = orc.full_to_half(orc.kernel_1d(V, n_m, HB))
    inv = 1.0 / abs(c)
    for gi, lr in ((0, 1e-3), (1, 1e-6), (2, 1e-3)):
        lrs = [0.0, 0.0, 0.0]
        lrs[gi] = lr
        loss0, w1 = orc.sgd_step(V, K, n_m, N, HB, w0, tuple(lrs), inv_scale=inv)
        step = w0[gi] - w1[gi]
        scale = lr * (c * c if gi == 2 else 1.0)
        g = step / scale
        pred = loss0 - scale * float(np.sum(g * g))
        got = _loss(orc, V, K, n_m, N, w1, inv)
        assert got < loss0
        assert abs(got - pred) <= 0.05 * (loss0 - pred), (gi, loss0, pred, got)


def test_sgd_fixed_point_at_zero_residual(orc):
    n_m, N = 16, 4
    V, w0, c = _case(3, n_m=n_m, N=N)
    K = orc.surrogate_fwd(V, n_m, N, *w0)
    loss0, w1 = orc.sgd_step(V, K, n_m, N, HB, w0, (1.0, 1.0, 1.0))
    assert loss0 == 0.0
    for a, b in zip(w0, w1):
        assert np.array_equal(a, b)
