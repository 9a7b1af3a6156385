"""Batches (rf_batch_*: several segments bound once and run by one call),
schedule tuning (rf_plan_set_tuning) and the autotuner.  Results must equal
the per-segment search bit for bit, on every run and under every schedule.

Graph capture of a batch is switched off in the library: its one run ended
the host process with a segmentation fault inside rf_batch_create's stream
capture, and no cause was found in the capture sequence by reading it, so
the captured form is not run here."""
import sys

import numpy as np
import pytest

import rfgen
from helpers import gpu_plan, upload

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _seg(nant, nint, npix, seed, k):
    c = npix // 2
    return rfgen.Preset(name=f"batch-{k}", nant=nant, nint=nint, tint_s=0.005, f_lo_ghz=1.0,
                        f_hi_ghz=2.0, nchan=48 + 16 * k, npol=2, dms=np.linspace(0, 200, 5 + k),
                        widths=[1, 2, 4], npix=npix, seed=seed,
                        pulses=[rfgen.Pulse(dm_idx=2, width_idx=k % 3, t0=8, x=c + 6, y=c - 4,
                                            snr=30.0)])


@pytest.fixture(scope="module")
def segs(torch):
    out = []
    for k, (nant, nint, npix, dt) in enumerate([(27, 48, 256, 0), (19, 64, 128, 0),
                                                (27, 40, 512, 0), (10, 56, 256, 1)]):
        p = _seg(nant, nint, npix, 60 + k, k)
        g = gpu_plan(p, vis_dtype=dt)
        dv = upload(p.make_vis(), dt)
        rows, n, st = g.search_segment(dv, cap=4096, with_stats=True)
        torch.cuda.synchronize()
        out.append((p, g, dv, rows, n, st))
        say("eager", p.name, "candidates", n)
    return out


def test_batch_runs_equal_eager(torch, segs):
    import paper_1802_03084_amd as rf
    b = rf.Batch([g for _, g, _, _, _, _ in segs], [dv for _, _, dv, _, _, _ in segs], cap=4096,
                 with_stats=True)
    say("batch of", len(segs))
    for rep in range(3):  # every run, including the first, equals the per-segment search
        res = b.run()
        for (p, g, dv, rows0, n0, st0), (rows, n, st) in zip(segs, res):
            assert n == n0, (rep, p.name)
            assert np.array_equal(rows, rows0), (rep, p.name)
            assert np.array_equal(st.view(np.int32), st0.view(np.int32)), (rep, p.name)
        # other work of the program between runs
        p, g, dv, rows0, n0, _ = segs[rep % len(segs)]
        rows, n, _ = g.search_segment(dv, cap=4096)
        torch.cuda.synchronize()
        assert n == n0 and np.array_equal(rows, rows0)
    b.close()


def test_schedule_does_not_change_results(torch, segs):
    p, g, dv, rows0, n0, st0 = segs[0]
    for lanes, budget in [(1, 16), (3, 64), (4, 4096), (2, 240)]:
        g.set_tuning(lanes, budget)
        assert g.tuning == (lanes, budget)
        rows, n, st = g.search_segment(dv, cap=4096, with_stats=True)
        say("schedule", lanes, budget, n)
        assert n == n0 and np.array_equal(rows, rows0)
        assert np.array_equal(st.view(np.int32), st0.view(np.int32))


def test_autotune_picks_caches_and_keeps_results(torch, segs, tmp_path):
    from paper_1802_03084_amd import autotune
    p, g, dv, rows0, n0, st0 = segs[2]
    cache = str(tmp_path / "tuning.json")
    lanes, budget, info = autotune.tune(g, dv, ndm=2, cache_path=cache, reps=1)
    say("autotune", lanes, budget, info)
    assert (lanes, budget) in autotune.CANDIDATES and not info["cached"]
    assert g.tuning == (lanes, budget)
    g.set_tuning(2, 240)
    lanes2, budget2, info2 = autotune.tune(g, dv, cache_path=cache)
    assert info2["cached"] and (lanes2, budget2) == (lanes, budget) and g.tuning == (lanes, budget)
    rows, n, st = g.search_segment(dv, cap=4096, with_stats=True)
    assert n == n0 and np.array_equal(rows, rows0)
