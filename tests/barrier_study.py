"""Oracle-only physics study of the 0.1 eV packet on the 0.3 eV barrier (CPU; test
infrastructure): the signed-particle density of the oracle's time loop against the
split-step Schrodinger density of the same Gaussian state.

    python tests/barrier_study.py seeds   # offsets of the mean position over six seeds
    python tests/barrier_study.py seeds pairs   # the same with rule 2 as literal pair removal
    python tests/barrier_study.py lc      # L1 distance vs coherence length and cell width

The first gives the statistics behind the bounds of test_barrier_reflection_tracks_schrodinger;
the second asks whether the gap between the two densities shrinks with the coherence length
L_C or the cell width, whether it survives averaging over seeds (a bias) or not (sampling
noise), and whether it depends on the reading of rule 2 (regeneration of mixed bins, or
literal pair removal)."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

import oracle as orc  # noqa: E402
import schrodinger  # noqa: E402
from paper_1806_00082_amd import inputs  # noqa: E402

HB = inputs.HBAR_EVFS


def run(seed, N0=1e5, times=(100.0, 150.0, 200.0), dx=0.5, L_C=40.0, U=0.3, x0=80.0, sigma=5.0, dt=0.5,
        pairs=False):
    """Oracle time loop on a 200 nm domain; returns the particle densities at `times`, the
    Schrodinger densities and the cell centres.  pairs: rule 2 as literal pair removal
    (survivors keep their exact positions) instead of the regeneration of mixed bins."""
    nx = int(round(200.0 / dx))
    n_m = int(round(L_C / dx))
    mesh = inputs.Mesh1D(nx=nx, dx=dx, n_m=n_m, pos_f64=False)
    V = inputs.gaussian_barrier_1d(mesh, U, 2.0, 100.0)
    k0 = inputs.k_for_energy(0.1)
    bc = inputs.packet_bin_counts_1d(mesh, N0, x0, sigma, k0)
    md = mesh.as_dict(dt)
    K = orc.kernel_1d(V, n_m, HB)[0]
    _, n0, thr, cdf = orc.gamma_tables(K, dt)
    p = orc.sp_init(md, bc, 40 * int(bc.sum()), seed=seed)
    slot = np.arange(nx, dtype=np.int32)
    out, t, st = [], 0.0, 0
    for T in times:
        while t < T - 1e-9:
            p, _ = orc.sp_step(md, p, (n0, thr, cdf), slot, step=st, seed=seed)
            if pairs:
                p, hp, hm, _ = orc.sp_annihilate_pairs(md, p)
            else:
                p, hp, hm, _ = orc.sp_annihilate(md, p, step=st, seed=seed)
            t += dt
            st += 1
        rho = (hp.astype(np.float64) - hm.astype(np.float64)).reshape(nx, -1).sum(1) / bc.sum()
        out.append(rho)
    ref = schrodinger.densities(x0, sigma, k0, (U, 2.0, 100.0), times, nx, dx)
    return out, ref, (np.arange(nx) + 0.5) * dx


def _seed_offsets(args):
    seed, pairs = args
    out, ref, xc = run(seed, pairs=pairs)
    return [(r * xc).sum() / r.sum() - (s * xc).sum() / s.sum() for r, s in zip(out, ref)]


def seeds_study(n_seeds=6, pairs=False):
    """Offset of the mean position from the Schrodinger one at 100, 150 and 200 fs, per seed."""
    from multiprocessing import get_context
    with get_context("spawn").Pool(min(n_seeds, 6)) as pool:
        offs = np.array(pool.map(_seed_offsets, [(seed, pairs) for seed in range(n_seeds)]))
    return offs.mean(0), offs.std(0, ddof=1), offs


def _lc_case(args):
    L_C, dx, pairs, seed, T = args
    out, ref, xc = run(seed, times=(T,), dx=dx, L_C=L_C, pairs=pairs)
    return out[0], ref[0], xc


def lc_study(T=200.0, n_seeds=4):
    """L1 between the particle and Schrodinger densities at T for L_C = 40, 80 nm at
    dx = 0.5 nm, L_C = 40 nm at dx = 0.25 nm, and L_C = 40 nm at dx = 0.5 nm with rule 2 as
    literal pair removal, over `n_seeds` seeds each, on the whole domain,
    in front of the barrier (x < 96 nm, the reflected packet) and past it (x > 104 nm).

    A gap that is the method's discretisation error would shrink as L_C or the cell width
    improves and survive averaging over seeds; sampling noise is measured by the L1 between two
    seeds' densities divided by sqrt(2), and averaging n seeds divides it by sqrt(n)."""
    from multiprocessing import get_context
    cases = [(40.0, 0.5, False), (80.0, 0.5, False), (40.0, 0.25, False), (40.0, 0.5, True)]
    jobs = [(L_C, dx, pairs, s, T) for L_C, dx, pairs in cases for s in range(n_seeds)]
    with get_context("spawn").Pool(min(len(jobs), 6)) as pool:
        res = pool.map(_lc_case, jobs)
    rows = []
    for i, (L_C, dx, pairs) in enumerate(cases):
        runs = res[i * n_seeds:(i + 1) * n_seeds]
        s_ref, xc = runs[0][1], runs[0][2]
        regions = {"all": np.ones_like(xc, bool), "front": xc < 96.0, "past": xc > 104.0}
        row = {"L_C": L_C, "dx": dx, "rule2": "pairs" if pairs else "regenerate"}
        mean = np.mean([r for r, _, _ in runs], axis=0)
        for name, m in regions.items():
            single = np.mean([np.abs(r[m] - s_ref[m]).sum() for r, _, _ in runs])
            noise = np.mean([np.abs(runs[a][0][m] - runs[a + 1][0][m]).sum() / np.sqrt(2)
                             for a in range(0, n_seeds - 1, 2)])
            row[name] = {"L1_one_seed": round(float(single), 4), "noise_one_seed": round(float(noise), 4),
                         f"L1_mean_of_{n_seeds}": round(float(np.abs(mean[m] - s_ref[m]).sum()), 4)}
        row["transmitted"] = {"particles": round(float(mean[regions["past"]].sum()), 5),
                              "schrodinger": float(s_ref[regions["past"]].sum())}
        rows.append(row)
    return rows


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "seeds"
    if what == "seeds":
        mean, std, offs = seeds_study(pairs="pairs" in sys.argv[2:])
        print("offset of the mean position (particles - Schrodinger), nm, at 100 / 150 / 200 fs")
        print("per seed:\n", np.round(offs, 3))
        print("mean", np.round(mean, 3), "std", np.round(std, 3))
    else:
        for r in lc_study():
            print(r)
