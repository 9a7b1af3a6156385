"""Serving through the C ABI (rf_server_*): segments of different shapes
admitted by an HBM budget and searched concurrently on slot streams.  Each
segment's result must be the same alone and in the mix; a budget that holds
one request at a time must serialise admission without changing results."""
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


def _sub(nant, tint, nint, seed, k):
    c = 128
    return rfgen.Preset(name=f"serve-{nant}", nant=nant, nint=nint, tint_s=tint, f_lo_ghz=1.272,
                        f_hi_ghz=1.528, nchan=64, npol=2, dms=np.linspace(0, 300, 6),
                        widths=[1, 2, 4], npix=256, seed=seed,
                        pulses=[rfgen.Pulse(dm_idx=2 + k, width_idx=k, t0=8 + 4 * k,
                                            x=c + 7 - 3 * k, y=c - 5 + 2 * k, snr=30.0)])


def _host(torch, vis, dtype):
    arr = np.ascontiguousarray(vis.astype(np.complex64)) if dtype == 0 else np.ascontiguousarray(rfgen.to_cf16(vis))
    return torch.from_numpy(arr).pin_memory()


@pytest.fixture(scope="module")
def segments(torch):
    """(plan, pinned host segment, rows alone, count alone) for three subarray
    shapes and one FP16-storage plan."""
    out = []
    cases = [(_sub(10, 0.005, 64, 41, 0), 0), (_sub(19, 0.010, 32, 42, 1), 0),
             (_sub(27, 0.005, 64, 43, 2), 0), (_sub(27, 0.005, 64, 44, 1), 1)]
    for p, dt in cases:
        g = gpu_plan(p, vis_dtype=dt)
        vis = p.make_vis()
        rows, n, _ = g.search_segment(upload(vis, dt), cap=4096)
        torch.cuda.synchronize()
        out.append((p, g, _host(torch, vis, dt), rows, n))
        say("alone", p.name, "dtype", dt, "candidates", n)
    return out


def test_served_in_mix_equals_alone(torch, segments):
    import paper_1802_03084_amd as rf
    need = sum(rf.Server.request_bytes(g, 4096) for _, g, _, _, _ in segments)
    arena = torch.empty(2 * need + (1 << 20), dtype=torch.uint8, device="cuda")
    srv = rf.Server(arena, nslots=3)
    say("serving mix, arena", arena.numel())
    tickets = []
    for rep in range(2):
        for i, (p, g, h, _, _) in enumerate(segments):
            tickets.append((i, srv.submit(g, h, cap=4096)))
    spans = []
    for i, t in tickets:
        rows, n, tm = srv.wait(t)
        _, _, _, rows0, n0 = segments[i]
        assert n == n0, i
        assert np.array_equal(rows, rows0), i
        assert tm["latency_s"] >= 0 and tm["done_s"] >= tm["started_s"] >= tm["released_s"]
        spans.append((tm["started_s"], tm["done_s"]))
    srv.close()
    # continuous batching: requests were on the device together (one was
    # admitted before another had finished)
    spans.sort()
    assert any(s2 < d1 for (s1, d1), (s2, d2) in zip(spans, spans[1:])), spans
    p0 = segments[0][0]
    q = p0.pulses[0]
    assert (q.dm_idx, q.width_idx, q.t0, q.x, q.y) in cand_keys(segments[0][3])


def test_budget_serialises_admission(torch, segments):
    """An arena that holds one request: requests run one after another, each
    admitted only after the previous one freed its block, with results as
    alone."""
    import paper_1802_03084_amd as rf
    p, g, h, rows0, n0 = segments[2]
    need = rf.Server.request_bytes(g, 4096)
    arena = torch.empty(need + need // 2, dtype=torch.uint8, device="cuda")
    srv = rf.Server(arena, nslots=3)
    say("serving under a one-request budget")
    ts = [srv.submit(g, h, cap=4096) for _ in range(3)]
    res = [srv.wait(t) for t in ts]
    srv.close()
    for rows, n, _ in res:
        assert n == n0 and np.array_equal(rows, rows0)
    spans = sorted((tm["started_s"], tm["done_s"]) for _, _, tm in res)
    for (s1, d1), (s2, d2) in zip(spans, spans[1:]):
        assert s2 >= d1  # the next admission waited for the block


def test_request_larger_than_arena_rejected(torch, segments):
    import paper_1802_03084_amd as rf
    p, g, h, _, _ = segments[0]
    arena = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    srv = rf.Server(arena, nslots=1)
    with pytest.raises(rf.RFError) as e:
        srv.submit(g, h, cap=4096)
    assert e.value.status == -4
    srv.close()


def test_failed_request_is_drained_before_its_memory_is_reused(torch, segments):
    """A request that fails after its copy was enqueued (fault injection) must
    not leave work in flight in its arena block: with an arena that holds one
    request and two slots, the next request is admitted into the same block
    on the other slot, and its results must equal the alone run."""
    import paper_1802_03084_amd as rf
    p, g, h, rows0, n0 = segments[2]
    need = rf.Server.request_bytes(g, 4096)
    arena = torch.empty(need + need // 2, dtype=torch.uint8, device="cuda")
    srv = rf.Server(arena, nslots=2)
    say("serving: failed request, then reuse of its block")
    for rep in range(3):
        bad = srv.submit(g, h, cap=4096, flags=rf.Server.FAIL_AFTER_COPY)
        good = srv.submit(g, h, cap=4096)
        with pytest.raises(rf.RFError) as e:
            srv.wait(bad)
        assert e.value.status == -5
        rows, n, _ = srv.wait(good)
        assert n == n0 and np.array_equal(rows, rows0), rep
    srv.close()


def test_served_results_match_the_oracle(torch, segments):
    """The served segments' candidate keys against the CPU oracle (float32
    storage: 1e-5 bar; FP16 storage: 3e-3 against the oracle on the unrounded
    input), images inside the margin guard excluded and counted."""
    import paper_1802_03084_amd as rf
    need = sum(rf.Server.request_bytes(g, 4096) for _, g, _, _, _ in segments)
    arena = torch.empty(need + (1 << 20), dtype=torch.uint8, device="cuda")
    srv = rf.Server(arena, nslots=3)
    tickets = [srv.submit(g, h, cap=4096) for _, g, h, _, _ in segments]
    served = [srv.wait(t) for t in tickets]
    srv.close()
    for (p, g, h, _, _), (rows, n, _) in zip(segments, served):
        tol = 1e-5 if g.vis_dtype == 0 else 3e-3
        vis = p.make_vis()
        o = oracle_plan(p)
        ostats, ocands, oimgs = oracle.search(vis, o, keep_images=True)
        marginal = {key for key, st in ostats.items()
                    if oracle.is_marginal(oimgs[key], st[4], o.threshold, tol)}
        want = [c[:5] for c in ocands if (c[0], c[1], c[2] // p.widths[c[1]]) not in marginal]
        got = [k for k in cand_keys(rows) if (k[0], k[1], k[2] // p.widths[k[1]]) not in marginal]
        say("served vs oracle", p.name, "storage", g.vis_dtype, "candidates", n, "marginal", len(marginal))
        assert got == want
        q = p.pulses[0]
        assert (q.dm_idx, q.width_idx, q.t0, q.x, q.y) in cand_keys(rows)
