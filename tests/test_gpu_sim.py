"""Time-loop level checks on the GPU: the occupied-cell kernel refresh gives the same
trajectory as evaluating every cell; the simulator equals the oracle loop; physics sanity."""
import ctypes
import math

import numpy as np
import pytest
import torch

from gpu_helpers import HB, assert_particles_equal, dev, host_tables_to_device, to_np
from paper_1806_00082_amd import _lib as L
from paper_1806_00082_amd import inputs, ops
from paper_1806_00082_amd.sim import Simulator

pytestmark = pytest.mark.gpu


def test_occupied_mode_equals_all_cells():
    """Kernel rows only near occupied cells (refreshed every 8 steps) reproduce, bit for bit,
    the run with rows for every cell: the paper's 'only where needed' costs nothing in results."""
    cfg = inputs.config_c2(N0=3e5)
    a = Simulator(cfg, mode="occupied", refresh_every=8)
    b = Simulator(cfg, mode="all")
    for _ in range(60):
        a.step()
        b.step()
    assert a.n_rows < b.n_rows
    assert_particles_equal(a.a.view(), b.a.view(), "occupied vs all")


def test_full_size_run_repeatable_both_histogram_paths():
    """The 1e7-particle run, 40 steps, three times: twice with the histogram built inside
    sp_step and once with sp_annihilate building it.  Every run must give the same ensemble
    bit for bit (output order is defined by the data alone, not by scheduling)."""
    cfg = inputs.config_c2()
    print("full-size repeatability: 3 x 40 steps of 1e7 particles", flush=True)
    runs = [Simulator(cfg, hist_in_step=True), Simulator(cfg, hist_in_step=True),
            Simulator(cfg, hist_in_step=False)]
    for sim in runs:
        sim.run(40)
    torch.cuda.synchronize()
    ref = runs[0]
    S0 = to_np(ref.stats)
    assert S0[L.ST_OVERFLOW] == 0 and S0[L.ST_CUM_PAIRS] > 0 and S0[L.ST_CUM_REGEN] > 0
    n = ref.count()
    for k, sim in enumerate(runs[1:], 1):
        S = to_np(sim.stats)
        assert np.array_equal(S[L.ST_CUM_STEPS:L.ST_COUNT], S0[L.ST_CUM_STEPS:L.ST_COUNT]), k
        assert sim.count() == n, k
        for f in ("x", "M", "s"):
            assert torch.equal(getattr(sim.a, f)[:n], getattr(ref.a, f)[:n]), (k, f)
        assert torch.equal(sim.hist, ref.hist), k


@pytest.mark.parametrize("f64", [True, False])
def test_simulator_equals_oracle_loop(orc, f64):
    """Rows -> tables -> steps: the simulator given the oracle's kernel rows (FP64, or rounded to
    FP32 as the reduced-precision forms store them) equals the oracle loop on the same rows."""
    cfg = inputs.config_c1()
    md = cfg.mesh.as_dict(cfg.dt)
    Kf = orc.kernel_1d(cfg.V, cfg.mesh.n_m, HB)[0]
    if not f64:
        Kf = Kf.astype(np.float32).astype(np.float64)
    rows = torch.from_numpy(np.ascontiguousarray(orc.full_to_half(Kf)).astype(
        np.float64 if f64 else np.float32)).to(dev())
    sim = Simulator(cfg, kernel="given", mode="all", rows=rows)
    g, n0, thr, cdf = orc.gamma_tables(Kf, cfg.dt)
    assert np.array_equal(to_np(sim.gamma), g)
    assert np.array_equal(to_np(sim.cdf).view(np.uint64), cdf)
    cap = sim.capacity
    hp = orc.sp_init(md, cfg.bin_counts, cap, seed=cfg.seed)
    slot = np.arange(md["nx"], dtype=np.int32)
    for s in range(8):
        hp, _ = orc.sp_step(md, hp, (n0, thr, cdf), slot, step=s, seed=cfg.seed)
        hp, _, _, _ = orc.sp_annihilate(md, hp, step=s, seed=cfg.seed, capacity=cap)
        sim.step()
    assert_particles_equal(sim.a.view(), hp.view(), f"simulator vs oracle ({'fp64' if f64 else 'fp32'} rows)")


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("bf16x3", 5e-5)])
def test_simulator_rows_and_rates_match_oracle(orc, prec, tol):
    """The simulator's own kernel rows (eq.(4) on the GPU) against the oracle's, normwise, and
    the creation rates built from them against the oracle's rates from its own rows."""
    cfg = inputs.config_c1()
    sim = Simulator(cfg, mode="all", prec=prec, fused_tables=False)
    Kf = orc.kernel_1d(cfg.V, cfg.mesh.n_m, HB)[0]
    got = to_np(sim.Kbuf).astype(np.float64)
    ref = orc.full_to_half(Kf)
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()
    g = orc.gamma_tables(Kf, cfg.dt)[0]
    # gamma sums n_m rows entries of size <= max|K|: the row error bound carries over
    assert np.abs(to_np(sim.gamma) - g).max() <= cfg.mesh.n_m * tol * np.abs(ref).max()


@pytest.mark.parametrize("mode,prec", [("all", "fp64"), ("occupied", "fp64"), ("occupied", "bf16"),
                                       ("all", "bf16x3"), ("occupied", "fp16x3")])
def test_fused_tables_simulator_equals_two_step(mode, prec):
    """Rows straight into the creation tables (kernel rows never in device memory) give the
    same tables and, step for step, the same particles as rows -> tables in two passes, for
    the FP64 kernel and the 16-bit forms."""
    cfg = inputs.config_c2(N0=2e5)
    fused = Simulator(cfg, mode=mode, prec=prec)
    two = Simulator(cfg, mode=mode, prec=prec, fused_tables=False)
    assert fused.fused and not two.fused
    for k in range(12):
        fused.step()
        two.step()
        n = fused.count()
        assert n == two.count(), k
        for f in ("x", "M", "s"):
            assert torch.equal(getattr(fused.a, f)[:n], getattr(two.a, f)[:n]), (k, f)
    r = fused.n_rows
    assert r == two.n_rows
    for f in ("gamma", "n0", "thr", "cdf", "guide"):
        assert torch.equal(getattr(fused, f)[:r], getattr(two, f)[:r]), f


@pytest.mark.parametrize("prec", ["fp64", "bf16", "fp16x3"])
def test_fused_tables_2d_simulator_equals_two_step(prec):
    """d = 2, rows near occupied cells: the fused rows -> tables pass gives the same tables and
    trajectory as the two-step form (FP64 and 16-bit kernels)."""
    mesh = inputs.Mesh2D(nx=40, ny=36, dx=0.5, n_m=16, pos_f64=False)
    V = inputs.gaussian_dot_2d(mesh, 0.2, 1.5, 10.0, 9.0)
    bc = inputs.packet_bin_counts_2d(mesh, 5e4, 6.0, 9.0, 1.2, inputs.k_for_energy(0.1), 0.0)
    cfg = inputs.RunConfig("small2d", mesh, V, bc, int(bc.sum()), 0.5, 10, seed=5)
    fused = Simulator(cfg, prec=prec)
    two = Simulator(cfg, prec=prec, fused_tables=False)
    assert fused.fused and not two.fused
    for k in range(10):
        fused.step()
        two.step()
        n = fused.count()
        assert n == two.count(), k
        for f in ("x", "y", "M", "My", "s"):
            assert torch.equal(getattr(fused.a, f)[:n], getattr(two.a, f)[:n]), (k, f)
    r = fused.n_rows
    assert r == two.n_rows and r > 0
    for f in ("gamma", "n0", "thr", "cdf", "guide"):
        assert torch.equal(getattr(fused, f)[:r], getattr(two, f)[:r]), f


def test_2d_full_size_histogram_recount():
    """The 2-D workload at full size (5e7 particles): the signed histogram a step builds (LDS
    hash aggregation, with global atomics for the keys that overflow it) equals a host recount
    of the particles the step wrote."""
    cfg = inputs.config_c5()
    sim = Simulator(cfg)
    for _ in range(3):
        sim.step()
    md = sim.md
    out = ops.DeviceParticles(2, sim.capacity, md["pos_f64"], m_bytes=sim.a.m_bytes)
    hist = torch.zeros_like(sim.hist)
    ops.sp_step(md, sim.seed, sim.cell_slot, sim.n0, sim.thr, sim.cdf, sim.a, out, sim.step_index,
                sim.stats, sim.ws, hist=hist, guide=sim.guide)
    assert not sim.overflowed()
    v = out.view()
    live = v["s"] != 0
    cx = np.floor(v["x"][live]).astype(np.int64)
    cy = np.floor(v["y"][live]).astype(np.int64)
    kx = v["M"][live].astype(np.int64) - md["M_min"]
    ky = v["My"][live].astype(np.int64) - md["M_min"]
    b = ((cy * md["nx"] + cx) * md["n_k"] + ky) * md["n_k"] + kx
    nb = ops.n_bins(md)
    pos = v["s"][live] > 0
    h = to_np(hist)
    assert np.array_equal(h[:nb], np.bincount(b[pos], minlength=nb))
    assert np.array_equal(h[nb:], np.bincount(b[~pos], minlength=nb))
    assert live.sum() > 4e7


def test_2d_simulator_equals_oracle_loop(orc):
    mesh = inputs.Mesh2D(nx=20, ny=18, dx=0.5, n_m=16, pos_f64=False)
    V = inputs.gaussian_dot_2d(mesh, 0.2, 1.5, 5.0, 4.5)
    bc = inputs.packet_bin_counts_2d(mesh, 2e4, 3.0, 4.5, 1.2, inputs.k_for_energy(0.1), 0.0)
    cfg = inputs.RunConfig("tiny2d", mesh, V, bc, int(bc.sum()), 0.5, 5, seed=4)
    md = mesh.as_dict(cfg.dt)
    K = orc.kernel_2d(V, 16, HB).reshape(-1, 256)
    sim = Simulator(cfg, kernel="given", mode="all", rows=torch.from_numpy(np.ascontiguousarray(K)).to(dev()))
    got = to_np(ops.kernel_eval(torch.from_numpy(V[None]).to(dev()), 16,
                                cells=torch.arange(20 * 18, dtype=torch.int32, device=dev())))
    assert np.abs(got.reshape(-1, 256) - K).max() <= 1e-10 * np.abs(K).max()
    g, n0, thr, cdf = orc.gamma_tables(K, cfg.dt)
    hp = orc.sp_init(md, bc, sim.capacity, seed=cfg.seed)
    slot = np.arange(20 * 18, dtype=np.int32)
    for s in range(5):
        hp, _ = orc.sp_step(md, hp, (n0, thr, cdf), slot, step=s, seed=cfg.seed)
        hp, _, _, st = orc.sp_annihilate(md, hp, step=s, seed=cfg.seed, capacity=sim.capacity)
        sim.step()
    assert_particles_equal(sim.a.view(), hp.view(), "2-D simulator vs oracle")


def test_free_packet_moments_gpu():
    """V = 0 on the GPU at 1e6 particles: no creation, no annihilation; the mean position moves
    by t <v> and the variance grows as Var x0 + t^2 Var v (x0 and v independent in eq.(6))."""
    mesh = inputs.Mesh1D(nx=400, dx=0.5, n_m=80, pos_f64=True)
    k0 = inputs.k_for_energy(0.1)
    bc = inputs.packet_bin_counts_1d(mesh, 1e6, 50.0, 10.0, k0)
    cfg = inputs.RunConfig("free", mesh, np.zeros(mesh.nx), bc, int(bc.sum()), 0.5, 50)
    sim = Simulator(cfg, mode="all")
    v0 = sim.a.view()
    x0, M0 = v0["x"].astype(np.float64), v0["M"].astype(np.float64)
    steps = 50
    sim.run(steps)
    assert int(sim.stats[L.ST_CUM_PAIRS]) == 0
    v = sim.a.view()
    assert len(v["x"]) == len(x0)
    vdt = mesh.vdt(cfg.dt)
    assert np.array_equal(v["M"], v0["M"])
    assert abs(v["x"].mean() - (x0.mean() + steps * vdt * M0.mean())) < 1e-9
    var_ref = x0.var() + (steps * vdt) ** 2 * M0.var() + 2 * steps * vdt * np.cov(x0, M0, bias=True)[0, 1]
    assert abs(v["x"].var() - var_ref) < 1e-8 * var_ref


def test_barrier_reflection_gpu():
    """1e6-particle packet reflected by the 0.3 eV barrier on the GPU: no bin holds both signs
    after annihilation, the sign-weighted momentum reverses and the mean position follows the
    Schrodinger solution (the oracle's physics check, at 10x the particles)."""
    import schrodinger
    mesh = inputs.Mesh1D(nx=400, dx=0.5, n_m=80, pos_f64=False)
    V = inputs.gaussian_barrier_1d(mesh, 0.3, 2.0, 100.0)
    k0 = inputs.k_for_energy(0.1)
    bc = inputs.packet_bin_counts_1d(mesh, 1e6, 80.0, 5.0, k0)
    cfg = inputs.RunConfig("reflect", mesh, V, bc, int(bc.sum()), 0.5, 400)
    sim = Simulator(cfg, cap_factor=4.0)
    ref = schrodinger.densities(80.0, 5.0, k0, (0.3, 2.0, 100.0), (100.0, 200.0), 400, 0.5)
    xc = (np.arange(400) + 0.5) * 0.5
    nb = ops.n_bins(sim.md)
    for T, rs in zip((100.0, 200.0), ref):
        while sim.step_index < int(T / 0.5):
            sim.step()
        rho = to_np(sim.density())
        assert abs((rho * xc).sum() / rho.sum() - (rs * xc).sum() / rs.sum()) < 1.5
    assert not sim.overflowed()
    v = sim.a.view()
    assert np.all(v["s"] != 0)
    M = v["M"].astype(np.int64)                  # stored in the narrowest type (int8 here)
    b = (np.floor(v["x"]).astype(np.int64) * sim.md["n_k"] + (M - sim.md["M_min"]))
    pos = np.bincount(b[v["s"] > 0], minlength=nb)
    neg = np.bincount(b[v["s"] < 0], minlength=nb)
    assert not np.any((pos > 0) & (neg > 0))
    s = v["s"].astype(np.float64)
    assert (s * M).sum() / s.sum() < -0.8 * k0 / mesh.dk


@pytest.mark.parametrize("dim,nx,ny,margin", [(1, 300, 1, 3), (2, 37, 23, 2), (2, 64, 50, 0), (2, 20, 70, 25)])
def test_cells_to_evaluate_box(dim, nx, ny, margin):
    """sp_cells_to_evaluate against the box test written out: every cell without a table row
    that has an occupied cell within `margin` cells along each axis, in ascending order."""
    print(f"cells to evaluate dim={dim} {nx}x{ny} margin={margin}", flush=True)
    n_m = 8
    mesh = inputs.Mesh1D(nx, 1.0, n_m) if dim == 1 else inputs.Mesh2D(nx, ny, 0.5, n_m)
    md = mesh.as_dict(0.5)
    rng = np.random.default_rng(nx * 7 + margin)
    n_cells = nx * ny
    per_cell = ops.n_bins(md) // n_cells
    hist = np.zeros((2, n_cells, per_cell), np.int32)
    occ = rng.random(n_cells) < 0.03
    for c in np.flatnonzero(occ):                        # an occupied cell holds a particle
        hist[rng.integers(2), c, rng.integers(per_cell)] = 1 + rng.integers(3)
    slot = np.where(rng.random(n_cells) < 0.2, rng.integers(0, 1000, n_cells), -1).astype(np.int32)
    grid = occ.reshape(ny, nx)
    want = []
    for c in range(n_cells):
        cy, cx = divmod(c, nx)
        box = grid[max(cy - margin, 0):cy + margin + 1, max(cx - margin, 0):cx + margin + 1]
        if slot[c] < 0 and box.any():
            want.append(c)
    d_hist = torch.from_numpy(hist.reshape(-1)).to(dev())
    d_slot = torch.from_numpy(slot).to(dev())
    new_cells = torch.full((n_cells,), -7, dtype=torch.int32, device=dev())
    d_count = torch.zeros(1, dtype=torch.int64, device=dev())
    ws = ops.sp_workspace(md, 0, dev())
    g = ops.geom_struct(md, 0)
    L.check(L.lib().sp_cells_to_evaluate(ctypes.byref(g), ops._ptr(d_hist), 0, margin, ops._ptr(d_slot),
                                         ops._ptr(new_cells), ops._ptr(d_count), ops._ptr(ws), ws.numel(),
                                         ops._stream()), "sp_cells_to_evaluate")
    count = int(d_count.item())
    assert count == len(want)
    assert to_np(new_cells[:count]).tolist() == want


@pytest.mark.parametrize("nx,ny,n_m", [(256, 256, 32), (40, 36, 16)])
def test_cells_to_evaluate_from_block_map(nx, ny, n_m):
    """2-D, after simulator steps: the occupancy scan that skips the cells under unmarked blocks
    of the workspace's block map (hist_mode 1) finds the same cells as the scan of the whole
    histogram (hist_mode 0), with every cell's table row withdrawn so that all occupied
    neighbourhoods count."""
    if nx == 256:
        cfg = inputs.config_c5(N0=5e6)
    else:
        mesh = inputs.Mesh2D(nx=nx, ny=ny, dx=0.5, n_m=n_m, pos_f64=False)
        V = inputs.gaussian_dot_2d(mesh, 0.2, 1.5, 10.0, 9.0)
        bc = inputs.packet_bin_counts_2d(mesh, 5e4, 6.0, 9.0, 1.2, inputs.k_for_energy(0.1), 0.0)
        cfg = inputs.RunConfig("small2d", mesh, V, bc, int(bc.sum()), 0.5, 10, seed=5)
    sim = Simulator(cfg)
    sim.run(9)
    assert sim.hist_marked
    none = torch.full_like(sim.cell_slot, -1)
    got = []
    for mode in (0, 1, 0):
        d_count = torch.zeros(1, dtype=torch.int64, device=dev())
        new_cells = torch.full_like(sim.new_cells, -7)
        g = ops.geom_struct(sim.md, sim.seed)
        L.check(L.lib().sp_cells_to_evaluate(ctypes.byref(g), ops._ptr(sim.hist), mode, 2, ops._ptr(none),
                                             ops._ptr(new_cells), ops._ptr(d_count), ops._ptr(sim.ws),
                                             sim.ws.numel(), ops._stream()), "sp_cells_to_evaluate")
        n = int(d_count.item())
        got.append(to_np(new_cells[:n]).tolist())
    assert got[0] == got[1] == got[2] and len(got[0]) > 0
    # the cells found hold particles or neighbour one: every occupied cell is among them
    per_cell = ops.n_bins(sim.md) // (nx * ny)
    h = to_np(sim.hist).reshape(2, nx * ny, per_cell)
    occupied = np.flatnonzero((h != 0).any(axis=(0, 2)))
    assert set(occupied.tolist()) <= set(got[0])
