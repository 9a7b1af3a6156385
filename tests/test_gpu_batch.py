"""Batches (rf_batch_*: several segments bound once and run by one call),
schedule tuning (rf_plan_set_tuning) and the autotuner.  Results must equal
the per-segment search bit for bit, on every run and under every schedule,
eager or captured into HIP graphs (replayed several times with other work of
the program and synchronisations between the replays; capture is switched
off in the library for now).  The batching workload (segments of uneven
shape, FP16 storage, 512^2 to 2048^2) runs as one batch and is checked
against the oracle on sampled images."""
import sys

import numpy as np
import pytest

import oracle
import rfgen
from helpers import cand_keys, gpu_plan, oracle_plan, upload

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


@pytest.mark.parametrize("graph", [
    False,
    pytest.param(True, marks=pytest.mark.skip(
        reason="graph capture of a batch is switched off in the library (RF_EUNSUPPORTED): both "
               "captured runs ended the process with a host segmentation fault inside "
               "rf_batch_create, and no cause has been shown")),
])
def test_batch_runs_equal_eager(torch, segs, graph):
    import paper_1802_03084_amd as rf
    b = rf.Batch([g for _, g, _, _, _, _ in segs], [dv for _, _, dv, _, _, _ in segs], cap=4096,
                 with_stats=True, graph=graph)
    say("batch of", len(segs), "graph" if graph else "eager", "nodes", b.graph_nodes)
    assert (b.graph_nodes > 0) == graph
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


def test_batch_of_plans_with_different_lane_counts(torch, segs):
    """A batch whose segments' plans run 1, 2, 3 and 4 lane streams (the
    batch creates the largest number) equals the per-segment searches."""
    import paper_1802_03084_amd as rf
    tunings = [(1, 64), (2, 240), (3, 96), (4, 4096)]
    try:
        for (p, g, dv, rows0, n0, st0), t in zip(segs, tunings):
            g.set_tuning(*t)
        b = rf.Batch([x[1] for x in segs], [x[2] for x in segs], cap=4096, with_stats=True)
        for rep in range(2):
            res = b.run()
            for (p, g, dv, rows0, n0, st0), (rows, n, st) in zip(segs, res):
                say("lanes", g.tuning, p.name, n)
                assert n == n0 and np.array_equal(rows, rows0), (rep, p.name)
                assert np.array_equal(st.view(np.int32), st0.view(np.int32)), (rep, p.name)
        b.close()
    finally:
        for _, g, _, _, _, _ in segs:
            g.set_tuning(2, 240)


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


@pytest.fixture(scope="module")
def batching_segs(torch):
    """Eight segments of the batching workload (every nint from 256 to 4096,
    128 and 256 channels, every image size 512^2 to 2048^2), FP16 storage
    generated on the device, three of their DM trials each (the first, the
    pulse's, the last)."""
    from paper_1802_03084_amd import mock
    out = []
    for s in range(8):
        ndm = rfgen.batching_dm_count(s)
        p = rfgen.batching(s, keep_dms=[0, ndm // 3, ndm - 1])
        g = gpu_plan(p, vis_dtype=1)
        dv = mock.synthesize(g, p.seed, p.mocks())
        rows, n, st = g.search_segment(dv, cap=65536, with_stats=True)
        torch.cuda.synchronize()
        say("batching segment", s, p.nint, "x", p.nchan, f"{p.npix}^2", "candidates", n)
        out.append((p, g, dv, rows, n, st))
    return out


def test_batching_workload_batch_equals_per_segment(torch, batching_segs):
    import paper_1802_03084_amd as rf
    b = rf.Batch([x[1] for x in batching_segs], [x[2] for x in batching_segs], cap=65536,
                 with_stats=True)
    say("batching workload as one batch")
    for rep in range(2):
        res = b.run()
        for (p, g, dv, rows0, n0, st0), (rows, n, st) in zip(batching_segs, res):
            assert n == n0, (rep, p.name)
            assert np.array_equal(rows, rows0), (rep, p.name)
            assert np.array_equal(st.view(np.int32), st0.view(np.int32)), (rep, p.name)
            for q in p.pulses:
                assert (q.dm_idx, q.width_idx, q.t0, q.x, q.y) in cand_keys(rows), (p.name, q)
        p, g, dv, rows0, n0, _ = batching_segs[rep]
        rows, n, _ = g.search_segment(dv, cap=65536)
        torch.cuda.synchronize()
        assert n == n0 and np.array_equal(rows, rows0)
    b.close()


def test_batching_workload_sampled_oracle(torch, batching_segs):
    """Two DM trials per segment (the first and the pulse's), the pulse image
    and images spread over every width, against the oracle on the stored
    FP16 values: statistics within the float32 image bar, position exact
    outside the margin guard."""
    tol = 1e-5
    rng = np.random.default_rng(5)
    for p, g, dv, rows, n, st in batching_segs:
        host = dv.cpu().numpy()
        o = oracle_plan(p)
        keys = set()
        for q in p.pulses:
            keys.add((q.dm_idx, q.width_idx, q.t0 // p.widths[q.width_idx]))
        for i in (0, p.pulses[0].dm_idx if p.pulses else 1):
            for j in range(len(p.widths)):
                keys.add((i, j, int(rng.integers(0, p.nint // p.widths[j]))))
        say("batching oracle", p.name, len(keys), "images")
        for (i, j, k) in sorted(keys):
            img = oracle.image_at(host, o, i, j, k)
            peak, x, y, sigma, snr = oracle.image_stats(img)
            s = st[g.image_base(i, j) + k]
            amax = float(np.max(np.abs(img)))
            assert abs(float(s["peak"]) - peak) <= tol * amax, (p.name, i, j, k)
            assert abs(float(s["sigma"]) - sigma) <= 1.4826 * tol * amax, (p.name, i, j, k)
            if not oracle.is_marginal(img, snr, o.threshold, tol):
                assert (int(s["x"]), int(s["y"])) == (x, y), (p.name, i, j, k)
                assert (snr > o.threshold) == (float(s["snr"]) > o.threshold), (p.name, i, j, k)


def test_graph_batches_are_refused(torch, segs):
    """RF_BATCH_GRAPH is refused (RF_EUNSUPPORTED) and leaves nothing behind."""
    import paper_1802_03084_amd as rf
    with pytest.raises(rf.RFError) as e:
        rf.Batch([segs[0][1]], [segs[0][2]], cap=16, graph=True)
    assert e.value.status == -6
