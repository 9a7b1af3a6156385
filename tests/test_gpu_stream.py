"""The streaming front end: mean-visibility subtraction (rf_subtract_mean)
against the oracle, and overlapping segments with candidate windows over a
long stream: a steady source is removed, every pulse is found exactly once at
its time in the stream, also next to segment boundaries; the served form with
mean subtraction equals the same steps run alone."""
import sys

import numpy as np
import pytest

import oracle
import rfgen
from helpers import cand_keys, gpu_plan, upload

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("dtype", [0, 1])
def test_subtract_mean_matches_oracle(torch, dtype):
    p = rfgen.smallcase(nint=37, nchan=48, seed=71)
    say("subtract mean, storage", dtype)
    g = gpu_plan(p, vis_dtype=dtype)
    vis = p.make_vis()
    vis = vis + (0.7 - 0.3j)  # a common offset the subtraction must remove
    dv = upload(vis, dtype)
    g.subtract_mean(dv)
    got = dv.cpu().numpy()
    if dtype == 1:
        got = rfgen.from_cf16(got)
    ref = oracle.subtract_mean(vis)
    amax = np.max(np.abs(ref))
    err = np.max(np.abs(got - ref)) / amax
    say("max rel error", err)
    assert err <= (1e-6 if dtype == 0 else 3e-3)
    if dtype == 1:  # against the oracle on the rounded input: the output rounding only
        ref16 = oracle.subtract_mean(rfgen.from_cf16(rfgen.to_cf16(vis)))
        assert np.max(np.abs(got - ref16)) / amax <= 1e-3


def _stream():
    """184 integrations (4 segments of 64 overlapping by 24), a steady source
    and four pulses, two at segment-window boundaries."""
    n = 256
    c = n // 2
    pulses = [rfgen.Pulse(dm_idx=4, width_idx=0, t0=8, x=c + 9, y=c - 6, snr=25.0),
              rfgen.Pulse(dm_idx=3, width_idx=1, t0=38, x=c - 12, y=c + 7, snr=25.0),
              rfgen.Pulse(dm_idx=2, width_idx=2, t0=40, x=c + 5, y=c + 11, snr=25.0),
              rfgen.Pulse(dm_idx=1, width_idx=0, t0=124, x=c - 8, y=c - 13, snr=25.0)]
    p = rfgen.Preset(name="stream", nant=19, nint=184, tint_s=0.005, f_lo_ghz=1.272,
                     f_hi_ghz=1.528, nchan=64, npol=2, dms=np.linspace(0, 100, 5),
                     widths=[1, 2, 4], npix=n, seed=81, pulses=pulses)
    vis = p.make_vis()
    du, dv = p.cell()
    l, m = rfgen.pixel_to_lm(c + 20, c - 15, n, du, dv)
    amp = 15.0 / np.sqrt(2.0 * p.nbl * p.nchan)  # S/N 15 in every width-1 image
    rfgen.add_pulse(vis, p.uvw(), p.freq(), p.tint_s, p.kdm, 0.0, 0, p.nint, l, m, amp)
    return p, vis, (c + 20, c - 15)


def test_stream_segments_find_each_pulse_once(torch):
    from paper_1802_03084_amd import stream
    p, vis, steady = _stream()
    seg_nint, overlap = 64, 24
    segs = stream.segments(p.nint, seg_nint, overlap)
    say("stream segments", segs)
    found, found_raw = [], []
    plans = {}
    for start, tb, te in segs:
        q = rfgen.Preset(name="seg", nant=19, nint=seg_nint, tint_s=p.tint_s, f_lo_ghz=p.f_lo_ghz,
                         f_hi_ghz=p.f_hi_ghz, nchan=p.nchan, npol=2, dms=p.dms, widths=p.widths,
                         npix=p.npix, seed=0, pulses=[])
        if te not in plans:
            plans[te] = gpu_plan(q, t_begin=tb, t_end=te)
        g = plans[te]
        assert overlap >= stream.min_overlap(g)
        seg = np.ascontiguousarray(vis[start:start + seg_nint])
        rows_raw, _, _ = g.search_segment(upload(seg), cap=4096)
        dvs = upload(seg)
        g.subtract_mean(dvs)
        rows, _, _ = g.search_segment(dvs, cap=4096)
        for (i, j, t, x, y) in cand_keys(rows):
            found.append((i, j, start + t, x, y))
        for (i, j, t, x, y) in cand_keys(rows_raw):
            found_raw.append((i, j, start + t, x, y))
    for q in p.pulses:
        key = (q.dm_idx, q.width_idx, q.t0, q.x, q.y)
        assert found.count(key) == 1, (key, found.count(key))
    assert not any((x, y) == steady for (_, _, _, x, y) in found), "steady source not removed"
    assert sum((x, y) == steady for (_, _, _, x, y) in found_raw) > 0, "steady source too faint"


def test_served_with_mean_subtraction_equals_alone(torch):
    import paper_1802_03084_amd as rf
    p, vis, _ = _stream()
    q = rfgen.Preset(name="seg", nant=19, nint=64, tint_s=p.tint_s, f_lo_ghz=p.f_lo_ghz,
                     f_hi_ghz=p.f_hi_ghz, nchan=p.nchan, npol=2, dms=p.dms, widths=p.widths,
                     npix=p.npix, seed=0, pulses=[])
    g = gpu_plan(q)
    seg = np.ascontiguousarray(vis[40:104])
    dvs = upload(seg)
    g.subtract_mean(dvs)
    rows0, n0, _ = g.search_segment(dvs, cap=4096)
    host = torch.from_numpy(seg.astype(np.complex64)).pin_memory()
    arena = torch.empty(2 * rf.Server.request_bytes(g, 4096), dtype=torch.uint8, device="cuda")
    srv = rf.Server(arena, nslots=2)
    ts = [srv.submit(g, host, cap=4096, subtract_mean=True) for _ in range(2)]
    for t in ts:
        rows, n, _ = srv.wait(t)
        assert n == n0 and np.array_equal(rows, rows0)
    srv.close()
