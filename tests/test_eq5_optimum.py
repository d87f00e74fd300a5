"""What training can gain for the network of eq.(5) (Sec. 2.3, trained as in Sec. 3): the
least-squares optimum of the form, jointly over (wV, wT, W), against the barycentric
(untrained, analytic) weights, on random Gaussian-bell potentials (the data law of Sec. 3).
CPU only: the closed-form MSE (tests/eq5_optimum.py) is first pinned against the oracle's
eq.(5) forward and eq.(4) kernel, then used at the learned-kernel shape."""
import numpy as np
import pytest

import eq5_optimum as opt
from paper_1806_00082_amd import inputs

HB = inputs.HBAR_EVFS


@pytest.mark.parametrize("N", [1, 2, 4])
def test_closed_form_mse_matches_the_oracle(orc, N):
    """The quadratic form reproduces sum (Kh - K)^2 computed by the oracle for the barycentric
    weights, and for random weights given as C = W wV with their (S, T)."""
    n_m, nx = 16, 40
    V = inputs.random_potentials(3, nx, 0.5, seed=5)
    K = orc.full_to_half(orc.kernel_1d(V, n_m, HB))
    R = opt.lagged_correlation(V, n_m // 2)
    rng = np.random.default_rng(N)
    c = -2.0 / (HB * n_m)
    for wV, wT, W in (orc.analytic_weights(n_m, N, HB),
                      (rng.normal(1, 0.2, N), rng.normal(1.0 / N, 0.05, N), c * rng.normal(1, 0.2, n_m // N))):
        Kh = orc.surrogate_fwd(V, n_m, N, wV, wT, W)
        ref = float(np.sum((Kh - K) ** 2))
        S, T = float(np.sum(wT)), float(np.sum(np.arange(N) * wT))
        G, r, yy = opt.quadratic_form(R, n_m, N, S, T, HB)
        C = np.outer(W, wV).ravel()
        assert opt.mse(G, r, yy, C) == pytest.approx(ref, rel=1e-9)
        assert yy == pytest.approx(float(np.sum(K ** 2)), rel=1e-12)


@pytest.mark.parametrize("N", [2, 4, 8])
def test_joint_optimum_gains_little_over_barycentric(N):
    """At the learned-kernel shape (1024 cells, 256 momenta, H = 128 / 64 / 32), fitted on 300
    potentials and scored on 200 held-out ones: the best network of the form is within a few
    per cent (relative MSE) of the barycentric one, so training can gain at most that much."""
    n_m, nx = 256, 1024
    Vtr = inputs.random_potentials(300, nx, 0.5, seed=0)
    Vte = inputs.random_potentials(200, nx, 0.5, seed=1)
    P = n_m // 2
    Rtr, Rte = opt.lagged_correlation(Vtr, P), opt.lagged_correlation(Vte, P)
    S0, T0 = 1.0, (N - 1) / 2.0
    Gt, rt, yt = opt.quadratic_form(Rte, n_m, N, S0, T0, HB)
    bary = opt.mse(Gt, rt, yt, opt.barycentric_C(n_m, N, HB)) / yt
    best = bary
    for S in (0.98, 1.0, 1.02):
        for T in (T0 - 0.25, T0, T0 + 0.25):
            G, r, _ = opt.quadratic_form(Rtr, n_m, N, S, T, HB)
            C = opt.best_C(G, r)
            Gt, rt, yt = opt.quadratic_form(Rte, n_m, N, S, T, HB)
            best = min(best, opt.mse(Gt, rt, yt, C) / yt)
    gain = 1.0 - best / bary
    print(f"N={N} (H={n_m // N}): held-out relative MSE barycentric {bary:.5f}, best of the form "
          f"{best:.5f}, gain {100 * gain:.2f} % (rms {np.sqrt(bary):.4f} -> {np.sqrt(best):.4f})")
    assert 0.0 <= gain < 0.05
