"""Benchmark of the signed-particle Wigner Monte Carlo hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-forms] [--no-cpu]

Headline workload: the 1-D paper-shaped run (400 cells of 0.5 nm, L_C = 40 nm -> 80
pseudo-momenta, Gaussian barrier 0.3 eV sigma 2 nm at 100 nm, Gaussian packet at 50 nm
sigma 10 nm with 0.1 eV, 1e7 signed particles in FP32, dt = 0.5 fs, annihilation every
step).  One step = kernel rows for newly occupied cells (every 8 steps) + creation tables +
sp_step (creation at rate gamma, drift, absorbing boundaries) + sp_annihilate.  W warm-up
steps, then exactly K timed steps (default W + K = the run's 400 steps).

value = particle-steps/s = sum over timed steps of the particle count at the start of the
step, divided by the time between the events bracketing the K steps (inputs resident in HBM).

Also reported (same JSON line): kernel entries/s of eq.(4) on the precision batch (4096
potentials x 2048 cells x 512 m) in FP64 and the BF16/FP16 (+split) forms with their
normwise error against the FP64 path, and the learned eq.(5) forward on 1024-cell, 256-m
potentials; the CPU oracle timed on a bounded sample of the headline run.
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
PEAK_TFLOPS = {"fp64": 78.6, "bf16": 2500.0, "fp16": 2500.0, "bf16x3": 2500.0, "fp16x3": 2500.0,
               "fp32": 157.3}


# HBM traffic per launch (GB) over the timed steps of this benchmark, from two rocprofv3
# counter runs (FETCH_SIZE, then WRITE_SIZE) of `bench.py --no-forms --no-cpu --no-trace
# --copy-calibration`, scaled by what the counters read for a 1 GiB device copy (fetch x2.0,
# write x1.0).  Taken for the kernels as they are now; an entry is dropped when its kernel
# changes until the counters are taken again.
TRAFFIC = {"step_count": 0.0671, "step_apply": 0.2082, "annih_count": 0.0920,
           "annih_scan": 0.0001, "annih_write": 0.1693}


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


# Algorithmic HBM bytes per launch of each particle kernel, from the running sums the
# library keeps (S = stats): what the pass must move at minimum with PB-byte particles (the
# headline's: x 4 + M 2 + s 1 = 7, FP32 positions and 16-bit momenta).  The histogram and
# the tables are L2-resident; the pair counts the two sp_step passes hand over are not
# counted (an implementation choice).
def kernel_bytes(PB: int):
    return {
        "step_count": lambda S, L: 5 * S[L.ST_CUM_N],                                # read x 4 + s 1
        "step_apply": lambda S, L: 2 * PB * (S[L.ST_CUM_N] + S[L.ST_CUM_PAIRS]),    # read, write; 2 children
        "annih_count": lambda S, L: PB * S[L.ST_CUM_ANNIH_IN],                       # read
        "annih_write": lambda S, L: PB * (S[L.ST_CUM_ANNIH_IN] + S[L.ST_CUM_KEPT]
                                          + S[L.ST_CUM_REGEN]),                      # read, write kept + placed
    }


def run_headline(steps: int, warmup: int, traced: bool):
    """The headline run.  traced=True replays the identical (bit-exact, same seed) run with
    per-kernel events, used only for the per-kernel roofline; the headline value comes from
    the untraced run."""
    import torch
    from paper_1806_00082_amd import _lib as L
    from paper_1806_00082_amd import inputs
    from paper_1806_00082_amd.sim import Simulator

    cfg = inputs.config_c2()
    sim = Simulator(cfg, kernel="exact", prec="fp64", mode="occupied", refresh_every=8)
    for _ in range(warmup):
        sim.step()
    sim.stats[L.ST_CUM_STEPS:L.ST_COUNT].zero_()
    if traced:
        L.check(L.lib().wk_trace_enable(steps * 24 + 64), "wk_trace_enable")
    torch.cuda.synchronize()
    t0, t1 = _events()
    wall0 = time.perf_counter()
    t0.record()
    for _ in range(steps):
        sim.step()
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t0.elapsed_time(t1)
    S = [int(v) for v in sim.stats.cpu().tolist()]
    assert S[L.ST_OVERFLOW] == 0, "particle buffer overflowed during the timed run"
    assert S[L.ST_CUM_STEPS] == steps
    out = {"cfg": cfg, "ms": ms, "wall_s": wall, "particle_steps": float(S[L.ST_CUM_N]),
           "pairs": S[L.ST_CUM_PAIRS], "regen": S[L.ST_CUM_REGEN], "n_last": int(sim.count()),
           "rows": sim.n_rows, "stats": S}
    if not traced:
        return out
    L.check(L.lib().wk_trace_disable(), "wk_trace_disable")
    pbytes = (8 if sim.md["pos_f64"] else 4) + (2 if sim.a.m16 else 4) + 1
    out["particle_bytes"] = pbytes
    KB = kernel_bytes(pbytes)
    kernels = {}
    for name in L.trace_names():
        tot, cnt = L.trace_read(name)
        kernels[name] = {"ms_total": round(tot, 3), "launches": cnt, "us_avg": round(1e3 * tot / max(cnt, 1), 2)}
        if name in KB:
            b = KB[name](S, L)
            kernels[name]["alg_GB"] = round(b / 1e9, 3)
            kernels[name]["alg_GBps"] = round(b / (tot * 1e-3) / 1e9, 1)
    dom = max((k for k in kernels if k in KB), key=lambda k: kernels[k]["ms_total"])
    ach = kernels[dom]["alg_GBps"]
    out["kernels"] = kernels
    out["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                       "traffic": TRAFFIC.get(dom)}
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


def run_2d(steps=40, warmup=8, fused_tables=True):
    """The 2-D workload: 256 x 256 cells of 0.5 nm, 32 x 32 momenta, 5e7 particles, exact FP64
    kernel rows formed near occupied cells (refreshed every 8 steps) straight into the creation
    tables, annihilation every step."""
    import torch
    from paper_1806_00082_amd import _lib as L
    from paper_1806_00082_amd import inputs
    from paper_1806_00082_amd.sim import Simulator

    cfg = inputs.config_c5()
    sim = Simulator(cfg, fused_tables=fused_tables)
    sim.run(warmup)
    torch.cuda.synchronize()
    sim.stats[L.ST_CUM_STEPS:L.ST_COUNT].zero_()
    e0, e1 = _events()
    e0.record()
    sim.run(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    S = sim.stats.cpu().tolist()
    out = {"workload": "2-D: 256x256 cells, 32x32 m, 5e7 particles, exact fp64 rows near occupied cells",
           "steps": steps, "ms_per_step": round(ms / steps, 4),
           "particle_steps_per_s": S[L.ST_CUM_N] / (ms * 1e-3), "n_last": sim.count(),
           "kernel_rows": sim.n_rows,
           "kernel_row_table_MB": 0.0 if sim.fused else round(sim.Kbuf.numel() * sim.Kbuf.element_size() / 1e6, 1)}
    del sim
    torch.cuda.empty_cache()
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
        K = torch.empty((R, n_m // 2), dtype=torch.float64, device="cuda")

        def fused():
            ops.kernel_tables(V, n_m, 0.5, guide_len=glen, out=bufs)

        def two_step():
            ops.kernel_eval(V, n_m, layout="half", out=K)
            g, n0, thr, cdf = ops.gamma_tables(K, n_m, 0.5, layout="half")
            ops.sampling_guide(cdf, glen, out=bufs[4])

        rec = {"rows": R, "kernel_rows_MB_two_step": round(K.numel() * 8 / 1e6, 1)}
        for tag, fn in (("fused_ms", fused), ("two_step_ms", two_step)):
            fn()
            torch.cuda.synchronize()
            e0, e1 = _events()
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            rec[tag] = round(e0.elapsed_time(e1) / reps, 4)
        out[name] = rec
        del V, bufs, K
        torch.cuda.empty_cache()
    return out


def run_cpu_baseline(sample_steps: int):
    """The oracle (single-threaded C, one core) on the first steps of the headline run."""
    import numpy as np
    import oracle as orc
    from paper_1806_00082_amd import inputs

    cfg = inputs.config_c2()
    md = cfg.mesh.as_dict(cfg.dt)
    K = orc.kernel_1d(cfg.V, cfg.mesh.n_m, inputs.HBAR_EVFS)[0]
    _, n0, thr, cdf = orc.gamma_tables(K, cfg.dt)
    p = orc.sp_init(md, cfg.bin_counts, 3 * int(cfg.bin_counts.sum()), seed=cfg.seed)
    slot = np.arange(md["nx"], dtype=np.int32)
    ps = 0
    t0 = time.perf_counter()
    for s in range(sample_steps):
        ps += p.n
        p, _ = orc.sp_step(md, p, (n0, thr, cdf), slot, step=s, seed=cfg.seed)
        p, _, _, _ = orc.sp_annihilate(md, p, step=s, seed=cfg.seed)
    dt = time.perf_counter() - t0
    return {"value": ps / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"first {sample_steps} steps of the 1e7-particle run (sp_step + sp_annihilate), "
                      f"{dt:.1f} s on one host core"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=390)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--no-trace", action="store_true",
                    help="skip the traced replica (for counter runs under rocprofv3 --pmc)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with three plain 1 GiB device copies (counter calibration)")
    ap.add_argument("--forms-only", action="store_true",
                    help="only the eq.(4) precision batch (for counter runs on the contraction)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(particles, cells and kernel rows are not sharded across devices).", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.forms_only:
        print(json.dumps({"forms": {"kernel_eq4": run_kernel_forms()}}))
        return
    h = run_headline(args.steps, args.warmup, traced=False)
    tr = h
    if not args.no_trace:
        tr = run_headline(args.steps, args.warmup, traced=True)
        assert tr["stats"][11:16] == h["stats"][11:16], "traced replica diverged from the timed run"
    forms = {} if args.no_forms else {"kernel_eq4": run_kernel_forms(), "surrogate_eq5": run_surrogate_forms(),
                                      "learning": run_learning(), "tables": run_tables_forms(),
                                      "workload_2d": run_2d()}
    cpu = None if args.no_cpu else run_cpu_baseline(args.cpu_steps)
    value = h["particle_steps"] / (h["ms"] * 1e-3)
    cfg = h["cfg"]
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
        "dtype": "int16+fp32 (fp64 kernel and tables)",
        "data": "synthetic",
        "config": {"workload": cfg.name, "cells": cfg.mesh.nx, "dx_nm": cfg.mesh.dx,
                   "n_m": cfg.mesh.n_m, "particles_initial": int(cfg.bin_counts.sum()),
                   "dt_fs": cfg.dt, "annihilation": "every step", "kernel": "exact fp64, occupied cells",
                   "particle_layout": "x fp32, M int16, s int8 (7 B)"},
        "run": {"n_last": h["n_last"], "pairs_created": h["pairs"], "regenerated": h["regen"],
                "kernel_rows_evaluated": h["rows"], "wall_s": round(h["wall_s"], 3),
                "traced_replica_ms_per_step": round(tr["ms"] / args.steps, 4),
                "kernels": tr.get("kernels")},
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
