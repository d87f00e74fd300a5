"""Benchmark of the signed-particle Wigner Monte Carlo hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-forms] [--no-cpu]

Headline workload: the 2-D run (256 x 256 cells of 0.5 nm, L_C = 16 nm -> 32 x 32
pseudo-momenta, Gaussian dot 0.2 eV sigma 4 nm at (64, 64) nm, Gaussian packet sigma 8 nm at
(32, 64) nm with 0.1 eV along +x, 5e7 signed particles in FP32, dt = 0.5 fs, annihilation
every step), the largest workload that fits one GPU.  One step = kernel rows for newly
occupied cells (every 8 steps, straight into the creation tables) + sp_step (creation at
rate gamma, drift, absorbing boundaries, signed histogram) + sp_annihilate.  W warm-up
steps, then exactly K timed steps (default W + K = the run's 200 steps).

value = particle-steps/s = sum over timed steps of the particle count at the start of the
step, divided by the time between the events bracketing the K steps (inputs resident in HBM).

Also reported (same JSON line): the 1-D paper-shaped run (400 cells, 1e7 particles) as a
secondary line; kernel entries/s of eq.(4) on the precision batch (4096 potentials x 2048
cells x 512 m) in FP64 and the BF16/FP16 (+split) forms with their normwise error against
the FP64 path; the learned eq.(5) forward, its training on 1e5 random potentials
(1024 cells x 256 m) and the run it drives; the CPU oracle timed on bounded samples.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Wigner kernel entries/s + particle-steps/s; BF16/surrogate vs FP64 at stated err"
HBM_PEAK_GBS = 8000.0
MTYPE = {1: "int8", 2: "int16", 4: "int32"}   # momentum storage by bytes per index
PEAK_TFLOPS = {"fp64": 78.6, "bf16": 2500.0, "fp16": 2500.0, "bf16x3": 2500.0, "fp16x3": 2500.0,
               "fp32": 157.3}


# HBM traffic per launch (GB) of the particle kernels of each workload over its timed steps,
# from two rocprofv3 counter runs (FETCH_SIZE, then WRITE_SIZE) of `bench.py --no-forms
# --no-cpu --no-trace --copy-calibration` (2-D: the headline; 1-D: with --headline-1d), scaled
# by what the counters read for a 1 GiB device copy (fetch x2.0, write x1.0).  Taken for the
# kernels as they are now; an entry is dropped when its kernel changes until the counters are
# taken again.
TRAFFIC = {"1d": {"step_count": 0.0611, "step_apply": 0.1353, "annih_bins": 0.0008,
                  "annih_count": 0.0626, "annih_write": 0.1224},
           "2d": {"step_count": 0.7616, "step_apply": 2.4723, "annih_bins": 0.1212,
                  "annih_count": 0.3085, "annih_write": 1.2755}}


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


# Algorithmic HBM bytes per launch of each particle kernel, from the running sums the
# library keeps (S = stats): what the pass must move at minimum with PB-byte particles
# (FP32 positions, 8-bit momenta: 1-D x 4 + M 1 + s 1 = 6; 2-D x 4 + y 4 + M 1 + My 1 + s 1
# = 11), the step's 4-byte histogram key of every output particle (read by the annihilation's
# counting pass instead of the particle), the annihilation's keep bits (one per input
# particle, written by the counting pass and read by the writing pass, which then reads the
# kept particles only) and, where a pass
# clears or walks the 2-D signed histogram (2 x 4 B x 67M bins, beyond every cache), the part
# of it that pass touches.  Not counted: the 1-D histogram and all tables (L2-resident), the
# 1-bit mixed-bin map (1/64 of the histogram) and the pair counts the two sp_step passes hand
# over (an implementation choice).
def kernel_bytes(PB: int, dim: int, hist_bytes: int, walked_bytes=None, cleared_bytes=None,
                 keys: bool = False):
    """walked_bytes: histogram bytes the bin pass had to read over the run (2-D: the blocks
    of bins that held counts, which the step marks); cleared_bytes: those the counting pass
    had to clear (the blocks the previous step marked).  None = the whole histogram each
    step.  keys: the step writes every output particle's 4-byte histogram key and the
    annihilation's counting pass reads those instead of the particles."""
    KY = 4 if keys else 0
    pos = 4 * dim + 1            # what the counting pass reads: positions and sign
    H = hist_bytes if dim == 2 else 0
    walk = (lambda S, L: H * S[L.ST_CUM_STEPS]) if walked_bytes is None else (lambda S, L: walked_bytes)
    clear = (lambda S, L: H * S[L.ST_CUM_STEPS]) if cleared_bytes is None else (lambda S, L: cleared_bytes)
    return {
        "step_count": lambda S, L: pos * S[L.ST_CUM_N] + clear(S, L),                # + histogram clear
        # read, write (2 children per pair), and the keys of the output
        "step_apply": lambda S, L: (2 * PB * (S[L.ST_CUM_N] + S[L.ST_CUM_PAIRS])
                                    + KY * (S[L.ST_CUM_N] + 2 * S[L.ST_CUM_PAIRS])),
        "annih_bins": walk,                                                           # histogram walk
        # read, and one keep bit per particle written
        "annih_count": lambda S, L: (KY or PB) * S[L.ST_CUM_ANNIH_IN] + S[L.ST_CUM_ANNIH_IN] / 8,
        # the keep bits and the kept particles read, kept + placed written
        "annih_write": lambda S, L: (S[L.ST_CUM_ANNIH_IN] / 8 + PB * (2 * S[L.ST_CUM_KEPT]
                                                                   + S[L.ST_CUM_REGEN])),
    }


def run_particles(cfg, steps: int, warmup: int, traced: bool, annihilation: str = "regenerate",
                  m_bytes=None, ms_ref=None, keys: bool = True):
    """A time-loop workload.  traced=True replays the identical (bit-exact, same seed) run with
    per-kernel events, used only for the per-kernel roofline; the reported value comes from
    the untraced run, whose time (ms_ref) the whole-step roofline uses.  m_bytes: momentum
    storage (default: the narrowest that fits)."""
    import torch
    from paper_1806_00082_amd import _lib as L
    from paper_1806_00082_amd import ops
    from paper_1806_00082_amd.sim import Simulator

    sim = Simulator(cfg, kernel="exact", prec="fp64", mode="occupied", refresh_every=8,
                    annihilation=annihilation, m_bytes=m_bytes, keys=keys)
    for _ in range(warmup):
        sim.step()
    sim.stats[L.ST_CUM_STEPS:L.ST_COUNT].zero_()
    if traced:
        L.check(L.lib().wk_trace_enable(steps * 24 + 64), "wk_trace_enable")
    torch.cuda.synchronize()
    # traced replica, 2-D: the blocks of bins each step's histogram holds counts in, which the
    # bin pass of the annihilation reads (measured between the steps, on the GPU, outside the
    # traced kernels)
    walked = torch.zeros((), dtype=torch.int64, device=sim.dev) if traced and sim.dim == 2 else None
    blk = 256
    while -(-ops.n_bins(sim.md) // blk) > 65536:
        blk *= 2

    def marked_blocks():
        h = sim.hist.view(2, -1)
        pad = (-h.shape[1]) % blk
        if pad:
            h = torch.nn.functional.pad(h, (0, pad))
        return (h.view(2, -1, blk) != 0).any(dim=2).any(dim=0).sum()

    # the first timed step clears what the last warm-up step built
    first = marked_blocks() if walked is not None else None
    last = None
    t0, t1 = _events()
    wall0 = time.perf_counter()
    t0.record()
    for _ in range(steps):
        sim.step()
        if walked is not None:
            last = marked_blocks()
            walked += last
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t0.elapsed_time(t1)
    S = [int(v) for v in sim.stats.cpu().tolist()]
    assert S[L.ST_OVERFLOW] == 0, "particle buffer overflowed during the timed run"
    assert S[L.ST_CUM_STEPS] == steps
    dim = sim.dim
    out = {"cfg": cfg, "ms": ms, "wall_s": wall, "particle_steps": float(S[L.ST_CUM_N]),
           "pairs": S[L.ST_CUM_PAIRS], "regen": S[L.ST_CUM_REGEN], "n_last": int(sim.count()),
           "rows": sim.n_rows, "stats": S}
    pbytes = (8 if sim.md["pos_f64"] else 4) * dim + sim.a.m_bytes * dim + 1
    out["particle_bytes"] = pbytes
    out["m_bytes"] = sim.a.m_bytes
    use_keys = sim.keys is not None
    hist_bytes = 2 * 4 * ops.n_bins(sim.md)
    del sim
    torch.cuda.empty_cache()
    if not traced:
        return out
    L.check(L.lib().wk_trace_disable(), "wk_trace_disable")
    walked_bytes = None if walked is None else int(walked.item()) * blk * 2 * 4
    cleared_bytes = (None if walked is None
                     else int((walked + first - last).item()) * blk * 2 * 4)
    out["walked_hist_fraction"] = (None if walked_bytes is None
                                   else round(walked_bytes / (hist_bytes * steps), 4))
    KB = kernel_bytes(pbytes, dim, hist_bytes, walked_bytes, cleared_bytes, keys=use_keys)
    kernels = {}
    for name in L.trace_names():
        tot, cnt = L.trace_read(name)
        kernels[name] = {"ms_total": round(tot, 3), "launches": cnt, "us_avg": round(1e3 * tot / max(cnt, 1), 2)}
        if name in KB:
            b = KB[name](S, L)
            kernels[name]["alg_GB_per_launch"] = round(b / max(cnt, 1) / 1e9, 4)
            kernels[name]["alg_GBps"] = round(b / (tot * 1e-3) / 1e9, 1)
            t = TRAFFIC["2d" if dim == 2 else "1d"].get(name)
            if t is not None:
                kernels[name]["traffic_GB_per_launch"] = t
    dom = max((k for k in kernels if k in KB), key=lambda k: kernels[k]["ms_total"])
    ach = kernels[dom]["alg_GBps"]
    traffic = TRAFFIC["2d" if dim == 2 else "1d"].get(dom)
    out["kernels"] = kernels
    out["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                       "traffic": traffic,
                       "alg_GB_per_launch": kernels[dom]["alg_GB_per_launch"],
                       "us_per_launch": kernels[dom]["us_avg"]}
    # the whole step against the sum of its kernels' algorithmic bytes
    tot_b = sum(KB[k](S, L) for k in KB)
    ms_step = ms if ms_ref is None else ms_ref
    out["step_roofline"] = {"alg_GB_per_step": round(tot_b / steps / 1e9, 4),
                            "achieved_GBps": round(tot_b / (ms_step * 1e-3) / 1e9, 1),
                            "frac": round(tot_b / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    return out


def run_kernel_forms():
    """eq.(4) on the precision batch in every form, error vs the FP64 path."""
    import numpy as np
    import torch
    from paper_1806_00082_amd import inputs, ops

    c3 = inputs.C3
    B, nx, n_m = c3["B"], c3["nx"], c3["n_m"]
    P = n_m // 2
    V = torch.from_numpy(inputs.random_potentials(B, nx, c3["dx"], seed=c3["seed"])).cuda()
    entries = B * nx * n_m
    # FLOP of the direct sum of eq.(4) (the unit of "alg_TFLOPs"), and the MFMA FLOP each form
    # issues: every form runs the odd/even fold (two H x H products per row, H = P / 2), three
    # times for the split forms.
    flops = 2.0 * (P - 1) ** 2 * B * nx
    H = P // 2
    issued = {"fp64": 4.0 * H * H, "bf16": 4.0 * H * H, "fp16": 4.0 * H * H,
              "bf16x3": 12.0 * H * H, "fp16x3": 12.0 * H * H}
    out = {"workload": "precision batch: 4096 potentials x 2048 cells x 512 m, half table"}
    ref = ops.kernel_eval(V, n_m, layout="half")
    refmax = ref.reshape(B, -1).abs().amax(dim=1)
    for prec in ("fp64", "bf16", "fp16", "bf16x3", "fp16x3"):
        buf = ref if prec == "fp64" else torch.empty((B * nx, P), dtype=torch.float32, device="cuda")
        ops.kernel_eval(V, n_m, prec=prec, layout="half", out=buf)
        torch.cuda.synchronize()
        e0, e1 = _events()
        reps = 3
        e0.record()
        for _ in range(reps):
            ops.kernel_eval(V, n_m, prec=prec, layout="half", out=buf)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        tf = flops / (ms * 1e-3) / 1e12
        mtf = issued[prec] * B * nx / (ms * 1e-3) / 1e12
        wbytes = B * nx * P * (8 if prec == "fp64" else 4)
        rec = {"ms": round(ms, 3), "entries_per_s": entries / (ms * 1e-3),
               "alg_TFLOPs": round(tf, 2), "mfma_TFLOPs": round(mtf, 2),
               "mfma_frac": round(mtf / PEAK_TFLOPS[prec], 4),
               "write_GBps": round(wbytes / (ms * 1e-3) / 1e9, 1)}
        if prec != "fp64":
            err = 0.0
            for b0 in range(0, B, 256):
                d = (buf[b0 * nx:(b0 + 256) * nx].double() - ref[b0 * nx:(b0 + 256) * nx]).reshape(-1, nx * P)
                err = max(err, float((d.abs().amax(dim=1) / refmax[b0:b0 + 256]).max()))
            rec["normwise_err_vs_fp64"] = err
            del buf
        out[prec] = rec
    del ref
    torch.cuda.empty_cache()
    return out


def run_learning(B=64, N=4, reps=5):
    """One SGD step of the eq.(5) training loop on 64 potentials x 1024 cells x 256 m (exact
    FP64 labels, FP32 forward, MSE gradient, backward, update), its parts, and the eq.(4)
    adjoint on the same batch."""
    import torch
    from paper_1806_00082_amd import inputs, learn, ops

    c4 = inputs.C4
    nx, n_m = c4["nx"], c4["n_m"]
    P = n_m // 2
    dev = torch.device("cuda")
    V = torch.from_numpy(inputs.random_potentials(B, nx, c4["dx"], seed=c4["test_seed"])).to(dev)
    wV, wT, W = learn.analytic_weights(n_m, N, device=dev)
    inv_scale = 1.0 / abs(-2.0 / (inputs.HBAR_EVFS * n_m))
    Klab = torch.empty((B * nx, P), dtype=torch.float64, device=dev)
    Kh = torch.empty((B * nx, P), dtype=torch.float32, device=dev)
    E = torch.empty_like(Kh)
    loss = torch.empty(1, dtype=torch.float64, device=dev)
    mws = torch.empty(8 * 1024, dtype=torch.uint8, device=dev)
    fws = learn.surrogate_fwd_workspace(n_m, N, dev)
    G = torch.randn((B * nx, P), dtype=torch.float64, device=dev, generator=torch.Generator(device=dev).manual_seed(1))
    dV = torch.zeros((B, nx), dtype=torch.float64, device=dev)

    def labels():
        ops.kernel_eval(V, n_m, layout="half", out=Klab)

    def fwd():
        learn.surrogate_fwd(V, n_m, N, wV, wT, W, prec="fp32", out=Kh, ws=fws)

    def mse():
        learn.mse_grad(Kh, Klab, inv_scale, E=E, loss=loss, ws=mws)

    grads = {}

    def bwd():
        grads["g"] = learn.surrogate_bwd(V, n_m, N, wV, wT, W, E)

    def sgd():
        dwV, dwT, dW, _ = grads["g"]
        learn.sgd_update(wV, dwV, 0.0)
        learn.sgd_update(wT, dwT, 0.0)
        learn.sgd_update(W, dW, 0.0)

    def adjoint():
        ops.kernel_bwd(G, nx, n_m, B, layout="half", dV=dV)

    def step():
        labels(), fwd(), mse(), bwd(), sgd()

    def timeit(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = _events()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return round(e0.elapsed_time(e1) / reps, 4)

    out = {"workload": f"{B} potentials x {nx} cells x {n_m} m, N={N} (H={n_m // N}), lr 0 (timing)"}
    for name, fn in (("labels_fp64", labels), ("surrogate_fwd_fp32", fwd), ("mse_grad", mse),
                     ("surrogate_bwd", bwd), ("sgd_update_x3", sgd), ("train_step", step),
                     ("kernel_adjoint_fp64", adjoint)):
        out[name + "_ms"] = timeit(fn)
    del Klab, Kh, E, G
    torch.cuda.empty_cache()
    return out


def run_learning_c4(n_train=100000, n_test=1000, sweep_epochs=3, train_epochs=6, batch=64,
                    driven_particles=1e7, driven_steps=400):
    """The learned form at its workload (Sec. 3): eq.(5) trained by SGD on the MSE against
    exact eq.(4) labels (computed per batch in FP64) for n_train random Gaussian-bell
    potentials of 1024 cells x 256 m, scored on n_test held-out ones, for H = 128, 64, 32
    (N = 2, 4, 8).  (a) One learning rate for every weight group, the paper's three values,
    from weights perturbed off the barycentric ones (the Fig. 3 analogue: mean batch loss per
    epoch).  (b) Per-group steps below each group's stability limit, from the barycentric
    weights: what training gains on held-out data.  (c) The trained N = 2 network drives the
    1e7-particle barrier run on the same mesh next to the exact kernel and the untrained one."""
    import numpy as np
    import torch
    from paper_1806_00082_amd import inputs, learn
    from paper_1806_00082_amd.sim import Simulator

    c4 = inputs.C4
    nx, n_m, dx = c4["nx"], c4["n_m"], c4["dx"]
    dev = torch.device("cuda")
    t0 = time.perf_counter()
    Vtr = torch.from_numpy(inputs.random_potentials(n_train, nx, dx, seed=c4["seed"])).to(dev)
    Vte = torch.from_numpy(inputs.random_potentials(n_test, nx, dx, seed=c4["test_seed"])).to(dev)
    out = {"workload": f"{n_train} training / {n_test} held-out potentials x {nx} cells x {n_m} m, "
                       f"batch {batch}, labels eq.(4) FP64 per batch, forward/backward FP32",
           "data_gen_s": round(time.perf_counter() - t0, 1)}
    g = torch.Generator().manual_seed(0)
    per_group_lr = (2.0, 5e-4, 30.0)
    trained = {}
    for N in (2, 4, 8):
        H = n_m // N
        wb = learn.analytic_weights(n_m, N, device=dev)
        rec = {"barycentric": {"held_out_rel_rms": learn.surrogate_rms_error(Vte, n_m, N, *wb),
                               "held_out_normwise": learn.surrogate_error(Vte, n_m, N, *wb)}}
        pert = (wb[0] * (1 + 0.3 * torch.randn(N, generator=g)).to(dev),
                wb[1] * (1 + 0.01 * torch.randn(N, generator=g)).to(dev),
                wb[2] * (0.8 + 0.2 * torch.rand(H, generator=g)).to(dev))
        rec["perturbed_start_rel_rms"] = learn.surrogate_rms_error(Vte, n_m, N, *pert)
        sweep = {}
        for lr in (1e-3, 1e-4, 1e-5):
            r = learn.train_surrogate(Vtr, n_m, N, epochs=sweep_epochs, batch=batch, lr=lr, init=pert, seed=1)
            fin = [float(w.abs().max()) for w in (r.wV, r.wT, r.W)]
            sweep[f"{lr:g}"] = {"epoch_loss": [round(x, 6) for x in r.losses],
                                "held_out_rel_rms": (learn.surrogate_rms_error(Vte, n_m, N, r.wV, r.wT, r.W)
                                                     if all(np.isfinite(fin)) else float("nan")),
                                "steps_per_s": round(r.steps / r.seconds, 1)}
        rec["lr_sweep_single_lr"] = sweep
        r = learn.train_surrogate(Vtr, n_m, N, epochs=train_epochs, batch=batch, lr=per_group_lr, init=wb, seed=2)
        rms = learn.surrogate_rms_error(Vte, n_m, N, r.wV, r.wT, r.W)
        rec["trained"] = {"lr_per_group": per_group_lr, "epochs": train_epochs,
                          "epoch_loss": [round(x, 6) for x in r.losses],
                          "held_out_rel_rms": rms,
                          "held_out_normwise": learn.surrogate_error(Vte, n_m, N, r.wV, r.wT, r.W),
                          "mse_gain_vs_barycentric": 1.0 - (rms / rec["barycentric"]["held_out_rel_rms"]) ** 2,
                          "seconds": round(r.seconds, 2), "steps": r.steps,
                          "weights": {"wV": r.wV.tolist(), "wT": r.wT.tolist(),
                                      "W_over_c_mean": float((r.W / wb[2]).mean()),
                                      "W_over_c_min": float((r.W / wb[2]).min()),
                                      "W_over_c_max": float((r.W / wb[2]).max())}}
        trained[N] = (r.wV, r.wT, r.W)
        out[f"N{N}_H{H}"] = rec
    del Vtr, Vte
    torch.cuda.empty_cache()
    if driven_steps:
        cfg = inputs.config_c4_run(N0=driven_particles, steps=driven_steps)
        runs = {}
        for tag, kind, N, w in (("exact_fp64", "exact", 1, None),
                                ("surrogate_N2_trained", "surrogate", 2, trained[2]),
                                ("surrogate_N2_barycentric", "surrogate", 2, learn.analytic_weights(n_m, 2))):
            sim = Simulator(cfg, kernel=kind, N=N, weights=w, prec="fp64" if kind == "exact" else "fp32",
                            cap_factor=3.0)
            torch.cuda.synchronize()
            e0, e1 = _events()
            e0.record()
            sim.run(driven_steps)
            e1.record()
            torch.cuda.synchronize()
            assert not sim.overflowed()
            gam = sim.gamma[:sim.n_rows].cpu().numpy()
            slot = sim.cell_slot.cpu().numpy()
            runs[tag] = {"ms_per_step": round(e0.elapsed_time(e1) / driven_steps, 4), "n_last": sim.count(),
                         "rho": sim.density().cpu().numpy(),
                         "gamma": np.where(slot >= 0, gam[np.maximum(slot, 0)], 0.0)}
            del sim
            torch.cuda.empty_cache()
        xc = (np.arange(cfg.mesh.nx) + 0.5) * cfg.mesh.dx
        ref = runs["exact_fp64"]
        drv = {"workload": f"1-D barrier run on {cfg.mesh.nx} cells x {n_m} m, {driven_particles:.0e} particles, "
                           f"{driven_steps} x {cfg.dt} fs"}
        for tag, r in runs.items():
            both = (ref["gamma"] > 0) & (r["gamma"] > 0)
            drv[tag] = {"ms_per_step": r["ms_per_step"], "n_last": r["n_last"],
                        "mean_x_nm": float((r["rho"] * xc).sum() / r["rho"].sum()),
                        "rho_L1_vs_exact": float(np.abs(r["rho"] - ref["rho"]).sum()),
                        "gamma_max_rel_diff_vs_exact": float(np.abs(r["gamma"][both] - ref["gamma"][both]).max()
                                                             / ref["gamma"].max())}
        out["driven_run"] = drv
    return out


def run_annihilation_modes():
    """Rule 2 read two ways on both time-loop workloads: regeneration of mixed bins (the
    headline) and literal pair removal (survivors keep their positions; a stable radix sort
    of the mixed bins' particles).  The trajectories differ (different readings), so each
    mode is timed on its own run: ms per step and particle-steps/s untraced, and its
    annihilation kernels from a traced replica."""
    from paper_1806_00082_amd import inputs

    out = {}
    for tag, cfg, steps, warm in (("workload_2d", inputs.config_c5(), 190, 10),
                                  ("workload_1d", inputs.config_c2(), 390, 10)):
        rec = {}
        for mode in ("regenerate", "pairs"):
            u = run_particles(cfg, steps, warm, traced=False, annihilation=mode)
            r = run_particles(cfg, steps, warm, traced=True, annihilation=mode, ms_ref=u["ms"])
            k = r["kernels"]
            annih = {n: v["us_avg"] for n, v in k.items()
                     if n.startswith(("annih", "pair", "radix", "hist_"))}
            rec[mode] = {"ms_per_step": round(u["ms"] / steps, 4),
                         "particle_steps_per_s": u["particle_steps"] / (u["ms"] * 1e-3),
                         "n_last": u["n_last"], "annihilation_kernels_us": annih,
                         "annihilation_us_per_step": round(sum(v["ms_total"] for n, v in k.items()
                                                               if n in annih) * 1e3 / steps, 1)}
        out[tag] = rec
    return out


def run_forms_2d(steps=60, warmup=10):
    """The 2-D workload's kernel in every form, side by side: eq.(4) in FP64, BF16, FP16 and
    the split forms, and eq.(5) in d = 2 (FP64, barycentric weights, N = 2 and 4), on every cell
    of its 256 x 256 mesh (kernel entries/s, normwise error against FP64); then the time loop
    driven by the exact FP64 rows (fused tables), the BF16 x3 and BF16 rows and the N = 2
    network: ms per step and the density's L1 distance from the FP64-driven run."""
    import numpy as np
    import torch
    from paper_1806_00082_amd import inputs, learn, ops
    from paper_1806_00082_amd.sim import Simulator

    cfg = inputs.config_c5()
    n_m = cfg.mesh.n_m
    V = torch.from_numpy(cfg.V[None]).cuda()
    R = cfg.mesh.nx * cfg.mesh.ny
    entries = R * n_m * n_m

    def timeit(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        e0, e1 = _events()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {"kernel": {"workload": f"2-D kernel on all {R} cells of the 256 x 256 mesh, {n_m} x {n_m} m"}}
    ref = ops.kernel_eval(V, n_m)
    kmax = float(ref.abs().max())
    for prec in ("fp64", "bf16", "fp16", "bf16x3", "fp16x3"):
        buf = ref if prec == "fp64" else torch.empty(ref.shape, dtype=torch.float32, device="cuda")
        ms = timeit(lambda: ops.kernel_eval(V, n_m, prec=prec, out=buf))
        rec = {"ms": round(ms, 4), "entries_per_s": entries / (ms * 1e-3)}
        if prec != "fp64":
            rec["normwise_err_vs_fp64"] = float((buf.double() - ref).abs().max()) / kmax
        out["kernel"][prec] = rec
        del buf
    for N in (2, 4):
        w = learn.analytic_weights_2d(n_m, N)
        buf = torch.empty(ref.shape, dtype=torch.float64, device="cuda")
        ms = timeit(lambda: learn.surrogate_fwd_2d(V, n_m, N, *w, out=buf))
        out["kernel"][f"surrogate_N{N}_fp64"] = {"ms": round(ms, 4), "entries_per_s": entries / (ms * 1e-3),
                                                 "normwise_err_vs_exact": float((buf - ref).abs().max()) / kmax}
        del buf
    del ref
    torch.cuda.empty_cache()
    # creation tables of every cell: rows straight into the tables against rows -> tables
    W = n_m * n_m
    tabs = (torch.empty(R, dtype=torch.float64, device="cuda"), torch.empty(R, dtype=torch.int32, device="cuda"),
            torch.empty(R, dtype=torch.int32, device="cuda"), torch.empty((R, W), dtype=torch.int64, device="cuda"),
            torch.empty((R, 257), dtype=torch.int32, device="cuda"))
    out["tables"] = {"workload": f"creation tables (eq.(1)) of all {R} cells, guide of 256 buckets"}
    for prec in ("fp64", "bf16", "bf16x3"):
        K = torch.empty((R, W), dtype=torch.float64 if prec == "fp64" else torch.float32, device="cuda")

        def two_step():
            ops.kernel_eval(V, n_m, prec=prec, out=K)
            g, n0, thr, cdf = ops.gamma_tables(K, n_m, cfg.dt, dim=2)
            ops.sampling_guide(cdf, 256, out=tabs[4])

        out["tables"][prec] = {
            "fused_ms": round(timeit(lambda: ops.kernel_tables(V, n_m, cfg.dt, guide_len=256, out=tabs, prec=prec)), 4),
            "two_step_ms": round(timeit(two_step), 4),
            "kernel_rows_MB_two_step": round(K.numel() * K.element_size() / 1e6, 1)}
        del K
        torch.cuda.empty_cache()
    w2 = learn.analytic_weights_2d(n_m, 2)
    K = torch.empty((R, W), dtype=torch.float64, device="cuda")

    def two_step_surr():
        learn.surrogate_fwd_2d(V, n_m, 2, *w2, out=K.view(R, n_m, n_m))
        g, n0, thr, cdf = ops.gamma_tables(K, n_m, cfg.dt, dim=2)
        ops.sampling_guide(cdf, 256, out=tabs[4])

    out["tables"]["surrogate_N2_fp64"] = {
        "fused_ms": round(timeit(lambda: learn.surrogate_tables_2d(V, n_m, 2, *w2, cfg.dt, guide_len=256,
                                                                   out=tabs)), 4),
        "two_step_ms": round(timeit(two_step_surr), 4),
        "kernel_rows_MB_two_step": round(K.numel() * 8 / 1e6, 1)}
    del tabs, K
    torch.cuda.empty_cache()
    runs = {}
    for tag, kw in (("exact_fp64", dict(kernel="exact", prec="fp64")),
                    ("exact_bf16x3", dict(kernel="exact", prec="bf16x3")),
                    ("exact_bf16", dict(kernel="exact", prec="bf16")),
                    ("surrogate_N2_fp64", dict(kernel="surrogate", N=2, weights=learn.analytic_weights_2d(n_m, 2)))):
        sim = Simulator(cfg, **kw)
        sim.run(warmup)
        torch.cuda.synchronize()
        e0, e1 = _events()
        e0.record()
        sim.run(steps)
        e1.record()
        torch.cuda.synchronize()
        assert not sim.overflowed()
        runs[tag] = {"ms_per_step": round(e0.elapsed_time(e1) / steps, 4), "n_last": sim.count(),
                     "rho": sim.density().cpu().numpy()}
        del sim
        torch.cuda.empty_cache()
    out["time_loop"] = {"workload": f"2-D run, {warmup} + {steps} steps, 5e7 particles at start"}
    for tag, r in runs.items():
        out["time_loop"][tag] = {"ms_per_step": r["ms_per_step"], "n_last": r["n_last"],
                                 "rho_L1_vs_fp64": float(np.abs(r["rho"] - runs["exact_fp64"]["rho"]).sum())}
    return out


def run_surrogate_forms():
    """eq.(5) forward (analytic barycentric weights) vs the exact kernel, 1024 cells x 256 m."""
    import torch
    from paper_1806_00082_amd import inputs, learn, ops

    c4 = inputs.C4
    nx, n_m, B = c4["nx"], c4["n_m"], 512
    P = n_m // 2
    V = torch.from_numpy(inputs.random_potentials(B, nx, c4["dx"], seed=c4["test_seed"])).cuda()
    entries = B * nx * n_m
    res = {"workload": f"{B} potentials x {nx} cells x {n_m} m, half table"}

    def timeit(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        e0, e1 = _events()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    K = torch.empty((B * nx, P), dtype=torch.float64, device="cuda")
    ms = timeit(lambda: ops.kernel_eval(V, n_m, layout="half", out=K))
    res["exact_fp64"] = {"ms": round(ms, 3), "entries_per_s": entries / (ms * 1e-3)}
    Kb = torch.empty((B * nx, P), dtype=torch.float32, device="cuda")
    ms = timeit(lambda: ops.kernel_eval(V, n_m, prec="bf16", layout="half", out=Kb))
    res["exact_bf16"] = {"ms": round(ms, 3), "entries_per_s": entries / (ms * 1e-3)}
    kmax = K.reshape(B, -1).abs().amax(dim=1)
    # N sweep of eq.(5): N cos factors, H = n_m / N sinusoid groups (N = 1 is eq.(4) itself)
    for N in (1, 2, 4, 8, 16):
        w = learn.analytic_weights(n_m, N)
        fws = learn.surrogate_fwd_workspace(n_m, N, "cuda")
        for prec in ("fp32", "bf16"):
            ms = timeit(lambda: learn.surrogate_fwd(V, n_m, N, *w, prec=prec, out=Kb, ws=fws))
            err = float(((Kb.double() - K).reshape(B, -1).abs().amax(dim=1) / kmax).max())
            res[f"N{N}_H{n_m // N}_{prec}"] = {"ms": round(ms, 3), "entries_per_s": entries / (ms * 1e-3),
                                              "normwise_err_vs_exact": err}
    return res


def run_tables_forms(reps=5):
    """Creation tables (eq.(1), postulate II) from eq.(4) rows: the fused pass whose kernel rows
    stay on chip against kernel_eval + gamma_tables + sampling_guide, and the device memory the
    two-step form needs for the rows."""
    import torch
    from paper_1806_00082_amd import inputs, ops

    out = {}
    cases = (("1e7-particle run, every cell: 1 x 400 cells x 80 m", 1, 400, 80, 80),
             ("learned-kernel shape: 64 potentials x 1024 cells x 256 m", 64, 1024, 256, 256),
             ("64 potentials x 2048 cells x 512 m", 64, 2048, 512, 256))
    for name, B, nx, n_m, glen in cases:
        V = torch.from_numpy(inputs.random_potentials(B, nx, 0.5, seed=5)).cuda()
        R = B * nx
        bufs = (torch.empty(R, dtype=torch.float64, device="cuda"), torch.empty(R, dtype=torch.int32, device="cuda"),
                torch.empty(R, dtype=torch.int32, device="cuda"),
                torch.empty((R, n_m), dtype=torch.int64, device="cuda"),
                torch.empty((R, glen + 1), dtype=torch.int32, device="cuda"))
        rec = {"rows": R, "kernel_rows_MB_two_step": round(R * (n_m // 2) * 8 / 1e6, 1)}
        for prec in ("fp64", "bf16", "bf16x3"):
            K = torch.empty((R, n_m // 2), dtype=torch.float64 if prec == "fp64" else torch.float32,
                            device="cuda")

            def fused():
                ops.kernel_tables(V, n_m, 0.5, guide_len=glen, out=bufs, prec=prec)

            def two_step():
                ops.kernel_eval(V, n_m, layout="half", out=K, prec=prec)
                g, n0, thr, cdf = ops.gamma_tables(K, n_m, 0.5, layout="half")
                ops.sampling_guide(cdf, glen, out=bufs[4])

            r = rec if prec == "fp64" else rec.setdefault(prec, {})
            for tag, fn in (("fused_ms", fused), ("two_step_ms", two_step)):
                fn()
                torch.cuda.synchronize()
                e0, e1 = _events()
                e0.record()
                for _ in range(reps):
                    fn()
                e1.record()
                torch.cuda.synchronize()
                r[tag] = round(e0.elapsed_time(e1) / reps, 4)
        out[name] = rec
        del V, bufs, K
        torch.cuda.empty_cache()
    return out


def _oracle_rows_2d(args):
    """Worker: oracle eq.(4) rows (direct d = 2 sum) for a chunk of cells."""
    import oracle as orc
    V, n_m, hbar, cells = args
    return orc.kernel_2d(V, n_m, hbar, cells=cells)[0]


def run_cpu_particles(sample_steps: int):
    """The oracle (single-threaded C, one core) on the first steps of the headline run: its
    sp_step and sp_annihilate over all 5e7 particles.  The oracle's kernel rows and creation
    tables for the cells the particles can reach in those steps are built first, untimed, by
    a pool of oracle processes."""
    import multiprocessing as mp

    import numpy as np
    import oracle as orc
    from paper_1806_00082_amd import inputs

    cfg = inputs.config_c5()
    md = cfg.mesh.as_dict(cfg.dt)
    nx, ny, n_m = md["nx"], md["ny"], md["n_m"]
    occ = cfg.bin_counts.reshape(ny, nx, -1).sum(-1) > 0
    pad = int(np.ceil(sample_steps * abs(md["vdt"]) * max(abs(md["M_min"]), md["M_min"] + md["n_k"]))) + 1
    reach = np.zeros_like(occ)
    for dy in range(-pad, pad + 1):
        for dx in range(-pad, pad + 1):
            reach |= np.roll(np.roll(occ, dy, 0), dx, 1)
    cells = np.flatnonzero(reach).astype(np.int32)
    workers = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    chunks = np.array_split(cells, workers * 4)
    with mp.get_context("spawn").Pool(workers) as pool:
        rows = pool.map(_oracle_rows_2d, [(cfg.V, n_m, inputs.HBAR_EVFS, c) for c in chunks])
    K = np.concatenate(rows).reshape(len(cells), n_m * n_m)
    _, n0, thr, cdf = orc.gamma_tables(K, cfg.dt)
    slot = np.full(nx * ny, -1, np.int32)
    slot[cells] = np.arange(len(cells), dtype=np.int32)
    t_tables = time.perf_counter() - t0
    n_init = int(cfg.bin_counts.sum())
    p = orc.sp_init(md, cfg.bin_counts, int(1.3 * n_init), seed=cfg.seed)
    ps = 0
    t0 = time.perf_counter()
    for s in range(sample_steps):
        ps += p.n
        p, _ = orc.sp_step(md, p, (n0, thr, cdf), slot, step=s, seed=cfg.seed)
        p, _, _, _ = orc.sp_annihilate(md, p, step=s, seed=cfg.seed, capacity=p.capacity)
    dt = time.perf_counter() - t0
    return {"value": ps / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"first {sample_steps} steps of the 2-D 5e7-particle run (sp_step + sp_annihilate, "
                      f"{ps:.3g} particle-steps in {dt:.1f} s on one host core; the oracle's kernel rows and "
                      f"creation tables for the {len(cells)} reachable cells built beforehand, untimed, in "
                      f"{t_tables:.1f} s by {workers} oracle processes)"}


def run_cpu_kernel(n_pot: int):
    """The oracle's eq.(4) (single-threaded C, one core) on the first potentials of the
    precision batch (2048 cells x 512 m each)."""
    import oracle as orc
    from paper_1806_00082_amd import inputs

    c3 = inputs.C3
    V = inputs.random_potentials(n_pot, c3["nx"], c3["dx"], seed=c3["seed"])
    t0 = time.perf_counter()
    orc.kernel_1d(V, c3["n_m"], inputs.HBAR_EVFS)
    dt = time.perf_counter() - t0
    entries = n_pot * c3["nx"] * c3["n_m"]
    return {"value": entries / dt, "unit": "kernel entries/s", "cores": 1, "kind": "oracle",
            "sample": f"eq.(4) full tables of the first {n_pot} potentials of the precision batch "
                      f"({entries} entries in {dt:.1f} s on one host core)"}


def host_info():
    info = {"cpu_count": os.cpu_count()}
    try:
        info["affinity_cores"] = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["model"] = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return info


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=190)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--no-keys", action="store_true",
                    help="headline run without the step's histogram keys (the annihilation rereads the particles)")
    ap.add_argument("--m-bytes", type=int, default=None, choices=(1, 2, 4),
                    help="momentum storage of the headline run (default: the narrowest that fits)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--cpu-potentials", type=int, default=2)
    ap.add_argument("--headline-1d", action="store_true",
                    help="time the 1-D 1e7-particle run as the headline (for its counter runs)")
    ap.add_argument("--no-trace", action="store_true",
                    help="skip the traced replica (for counter runs under rocprofv3 --pmc)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with three plain 1 GiB device copies (counter calibration)")
    ap.add_argument("--forms-only", action="store_true",
                    help="only the eq.(4) precision batch (for counter runs on the contraction)")
    ap.add_argument("--learning-only", action="store_true",
                    help="only the training study of eq.(5) (with --train-epochs, --sweep-epochs)")
    ap.add_argument("--forms-2d-only", action="store_true",
                    help="only the 2-D kernel forms and the runs they drive")
    ap.add_argument("--annihilation-only", action="store_true",
                    help="only the comparison of the two readings of rule 2")
    ap.add_argument("--train-epochs", type=int, default=6)
    ap.add_argument("--sweep-epochs", type=int, default=3)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(particles, cells and kernel rows are not sharded across devices).", file=sys.stderr)
        sys.exit(2)
    import torch
    if torch.cuda.device_count() < 1:          # counts devices without initialising HIP
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    # the CPU oracle legs run first, before anything touches the GPU
    cpu = cpu_kernel = None
    if not (args.no_cpu or args.forms_only or args.learning_only or args.headline_1d
            or args.annihilation_only or args.forms_2d_only):
        print("cpu baseline: oracle particle passes", file=sys.stderr, flush=True)
        cpu = run_cpu_particles(args.cpu_steps)
        print("cpu baseline: oracle eq.(4)", file=sys.stderr, flush=True)
        cpu_kernel = run_cpu_kernel(args.cpu_potentials)
        cpu["host"] = cpu_kernel["host"] = host_info()
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    from paper_1806_00082_amd import inputs
    if args.forms_only:
        print(json.dumps({"forms": {"kernel_eq4": run_kernel_forms()}}))
        return
    if args.forms_2d_only:
        print(json.dumps({"forms": {"forms_2d": run_forms_2d()}}))
        return
    if args.annihilation_only:
        print(json.dumps({"forms": {"annihilation_modes": run_annihilation_modes()}}))
        return
    if args.learning_only:
        print(json.dumps({"forms": {"learning_c4": run_learning_c4(sweep_epochs=args.sweep_epochs,
                                                                   train_epochs=args.train_epochs)}}))
        return
    cfg = inputs.config_c2() if args.headline_1d else inputs.config_c5()
    print(f"headline: {cfg.name}, {args.warmup} + {args.steps} steps", file=sys.stderr, flush=True)
    h = run_particles(cfg, args.steps, args.warmup, traced=False, m_bytes=args.m_bytes, keys=not args.no_keys)
    tr = h
    if not args.no_trace:
        tr = run_particles(cfg, args.steps, args.warmup, traced=True, m_bytes=args.m_bytes, ms_ref=h["ms"],
                           keys=not args.no_keys)
        assert tr["stats"][11:16] == h["stats"][11:16], "traced replica diverged from the timed run"
    forms = {}
    if not args.no_forms and not args.headline_1d:
        print("secondary: 1-D 1e7-particle run", file=sys.stderr, flush=True)
        c2 = inputs.config_c2()
        s1 = run_particles(c2, 390, 10, traced=False)
        s1t = run_particles(c2, 390, 10, traced=True, ms_ref=s1["ms"])
        assert s1t["stats"][11:16] == s1["stats"][11:16], "traced replica diverged from the timed run"
        forms["workload_1d"] = {
            "workload": f"{c2.name}: 1-D, 400 cells x 80 m, 1e7 particles, 390 timed steps",
            "ms_per_step": round(s1["ms"] / 390, 4),
            "particle_steps_per_s": s1["particle_steps"] / (s1["ms"] * 1e-3),
            "note": f"double-buffered {s1['particle_bytes']}-byte particles (2 x "
                    f"{round(s1['particle_bytes'] * 1e7 / 1e6)} MB) fit the 256 MB MALL: its HBM fraction "
                    "is a cache-assisted figure, the headline's 2-D run is not",
            "roofline": s1t["roofline"], "step_roofline": s1t["step_roofline"], "kernels": s1t["kernels"]}
        for name, fn in (("forms_2d", run_forms_2d), ("annihilation_modes", run_annihilation_modes),
                         ("kernel_eq4", run_kernel_forms), ("surrogate_eq5", run_surrogate_forms),
                         ("learning", run_learning), ("tables", run_tables_forms),
                         ("learning_c4", lambda: run_learning_c4(sweep_epochs=args.sweep_epochs,
                                                                 train_epochs=args.train_epochs))):
            print(f"forms: {name}", file=sys.stderr, flush=True)
            forms[name] = fn()
        if cpu_kernel is not None:
            k = forms["kernel_eq4"]["fp64"]
            forms["kernel_eq4"]["cpu_baseline"] = cpu_kernel
            forms["kernel_eq4"]["fp64"]["vs_cpu_oracle"] = round(k["entries_per_s"] / cpu_kernel["value"], 1)
    value = h["particle_steps"] / (h["ms"] * 1e-3)
    dim = cfg.mesh.dim
    config = {"workload": cfg.name, "dim": dim, "dx_nm": cfg.mesh.dx, "n_m": cfg.mesh.n_m,
              "particles_initial": int(cfg.bin_counts.sum()), "dt_fs": cfg.dt,
              "annihilation": "every step", "kernel": "exact fp64 rows near occupied cells, fused into the "
                                                     "creation tables",
              "particle_layout": (f"x, y fp32, Mx, My {MTYPE[h['m_bytes']]}, s int8 ({h['particle_bytes']} B)"
                                  if dim == 2 else
                                  f"x fp32, M {MTYPE[h['m_bytes']]}, s int8 ({h['particle_bytes']} B)")}
    config["cells"] = (f"{cfg.mesh.nx}x{cfg.mesh.ny}" if dim == 2 else cfg.mesh.nx)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"{MTYPE[h['m_bytes']]}+fp32 (fp64 kernel and tables)",
        "data": "synthetic",
        "config": config,
        "run": {"n_last": h["n_last"], "pairs_created": h["pairs"], "regenerated": h["regen"],
                "kernel_rows_evaluated": h["rows"], "wall_s": round(h["wall_s"], 3),
                "traced_replica_ms_per_step": round(tr["ms"] / args.steps, 4),
                "histogram_fraction_walked": tr.get("walked_hist_fraction"),
                "kernels": tr.get("kernels"), "step_roofline": tr.get("step_roofline")},
        "roofline": tr.get("roofline"),
        "cpu_baseline": cpu,
        "forms": forms,
    }
    print(json.dumps(line))
    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
