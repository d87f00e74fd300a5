"""Checkpoint / resume and per-step metrics of the time loop, on the GPU: a run stopped,
written to disk and restored into a fresh simulator continues bit for bit as the
uninterrupted run (counter-based draws keyed by step and particle index, order-defined
passes); the JSONL metrics agree with the running statistics."""
import io
import json

import numpy as np
import pytest
import torch

from gpu_helpers import to_np
from paper_1806_00082_amd import _lib as L
from paper_1806_00082_amd import inputs
from paper_1806_00082_amd.sim import Simulator

pytestmark = pytest.mark.gpu


def _small_2d(seed=5):
    mesh = inputs.Mesh2D(nx=40, ny=36, dx=0.5, n_m=16, pos_f64=False)
    V = inputs.gaussian_dot_2d(mesh, 0.2, 1.5, 10.0, 9.0)
    bc = inputs.packet_bin_counts_2d(mesh, 5e4, 6.0, 9.0, 1.2, inputs.k_for_energy(0.1), 0.0)
    return inputs.RunConfig("small2d", mesh, V, bc, int(bc.sum()), 0.5, 10, seed=seed)


CASES = [
    ("1d-regenerate", lambda: inputs.config_c2(N0=3e5), {}, 9),
    ("1d-regenerate-at-refresh", lambda: inputs.config_c2(N0=3e5), {}, 8),
    ("1d-pairs", lambda: inputs.config_c2(N0=3e5), {"annihilation": "pairs"}, 9),
    ("1d-two-step-bf16", lambda: inputs.config_c2(N0=3e5), {"prec": "bf16", "fused_tables": False}, 9),
    ("2d-regenerate", _small_2d, {}, 9),
    ("2d-pairs", _small_2d, {"annihilation": "pairs"}, 9),
]


def _assert_same_state(a: Simulator, b: Simulator, tag):
    n = a.count()
    assert n == b.count(), tag
    for f in ("x", "y", "M", "My", "s"):
        t = getattr(a.a, f)
        if t is not None:
            assert torch.equal(t[:n], getattr(b.a, f)[:n]), (tag, f)
    assert torch.equal(a.hist, b.hist), tag
    assert torch.equal(a.stats, b.stats), tag
    assert a.n_rows == b.n_rows and a.step_index == b.step_index, tag
    assert torch.equal(a.cell_slot, b.cell_slot), tag
    r = a.n_rows
    for f in ("gamma", "n0", "thr", "cdf", "guide"):
        assert torch.equal(getattr(a, f)[:r], getattr(b, f)[:r]), (tag, f)


@pytest.mark.parametrize("name,make,kw,stop", CASES, ids=[c[0] for c in CASES])
def test_resume_from_file_is_bit_exact(tmp_path, name, make, kw, stop):
    total = 23
    print(f"checkpoint resume {name}: stop at {stop} of {total} steps", flush=True)
    cfg = make()
    whole = Simulator(cfg, **kw)
    whole.run(total)
    first = Simulator(cfg, **kw)
    first.run(stop)
    path = tmp_path / "state.pt"
    first.save(path)
    del first
    resumed = Simulator(cfg, **kw)
    resumed.restore(path)
    resumed.run(total - stop)
    torch.cuda.synchronize()
    assert not whole.overflowed()
    assert int(to_np(whole.stats)[L.ST_CUM_PAIRS]) > 0
    _assert_same_state(whole, resumed, name)


def test_restore_refuses_another_run(tmp_path):
    cfg = inputs.config_c2(N0=1e5)
    sim = Simulator(cfg)
    sim.run(3)
    path = tmp_path / "state.pt"
    sim.save(path)
    other_seed = inputs.config_c2(N0=1e5)
    other_seed.seed = cfg.seed + 1
    with pytest.raises(ValueError, match="configuration"):
        Simulator(other_seed).restore(path)
    with pytest.raises(ValueError, match="configuration"):
        Simulator(cfg, annihilation="pairs").restore(path)
    other_V = inputs.config_c2(N0=1e5)
    other_V.V = np.asarray(other_V.V) * 1.5
    with pytest.raises(ValueError, match="potential"):
        Simulator(other_V).restore(path)
    small = Simulator(inputs.config_c2(N0=1e3))      # same run, buffers for 4e3 particles
    with pytest.raises(ValueError, match="particles"):
        small.restore(path)


def test_metrics_jsonl_agree_with_running_statistics():
    cfg = _small_2d()
    sim = Simulator(cfg)
    S0 = to_np(sim.stats)          # the set-up's histogram pass counts as one annihilation
    log = io.StringIO()
    sim.run(7, log=log)
    recs = [json.loads(l) for l in log.getvalue().splitlines()]
    assert [r["step"] for r in recs] == list(range(7))
    S = to_np(sim.stats) - S0
    assert recs[-1]["particles"] == sim.count() == S[L.ST_N] + S0[L.ST_N]
    assert sum(r["pairs"] for r in recs) == S[L.ST_CUM_PAIRS] > 0
    assert sum(r["kept"] for r in recs) == S[L.ST_CUM_KEPT]
    assert sum(r["regenerated"] for r in recs) == S[L.ST_CUM_REGEN] > 0
    assert S[L.ST_CUM_STEPS] == 7
    assert all(not r["overflow"] and r["rows"] > 0 for r in recs)
    assert all(b["wall_s"] >= a["wall_s"] for a, b in zip(recs, recs[1:]))
