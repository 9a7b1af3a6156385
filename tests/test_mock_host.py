"""Host logic of the mock-transient tools (paper_1802_03084_amd.mock):
drawing, matching and binning, on synthetic geometry and candidate lists."""
import math

import numpy as np
import pytest

import rfgen
from paper_1802_03084_amd import mock

CAND = np.dtype([("dm_idx", "<i4"), ("width_idx", "<i4"), ("t_int", "<i4"), ("x", "<i4"),
                 ("y", "<i4"), ("snr", "<f4"), ("peak", "<f4"), ("sigma", "<f4")])


def geom(nint=2048):
    p = rfgen.survey()
    du, dv = p.cell()
    return mock.Geometry(nint=nint, tint_s=p.tint_s, freq_ghz=p.freq(), dms=p.dms, widths=p.widths,
                         npix=p.npix, du=du, dv=dv, W=p.nbl * p.nchan)


def test_amplitude_gives_the_ideal_snr():
    """amp (2 w W)^1/2 = snr: the matched-filter S/N of a box of w unit-noise
    integrations averaged over two polarisations and W samples."""
    g = geom()
    for snr, w in [(6.0, 1), (20.0, 8), (7.5, 3.3)]:
        assert math.isclose(g.amplitude(snr, w) * math.sqrt(2 * w * g.W), snr, rel_tol=1e-12)


def test_on_grid_draws():
    g = geom()
    rng = np.random.default_rng(3)
    recs = mock.draw(g, 5, rng, snr=(5, 30))
    sweep_max = g.sweep(float(g.dms.max()))
    ends = []
    for r in recs:
        assert r.dm in set(g.dms.tolist()) and int(r.width) in g.widths
        assert r.t0 == int(r.t0) and int(r.t0) % int(r.width) == 0
        assert r.x == int(r.x) and r.y == int(r.y)
        assert abs(r.x - g.npix / 2) <= g.npix / 16 and abs(r.y - g.npix / 2) <= g.npix / 16
        assert 5 <= r.snr <= 30
        assert r.t0 + g.sweep(r.dm) + r.width <= g.nint
        l, m = g.lm(r.x, r.y)
        assert (r.l, r.m) == (l, m)
        ends.append((r.t0, r.t0 + g.sweep(r.dm) + r.width))
    for (a0, a1), (b0, b1) in zip(ends, ends[1:]):
        assert a1 <= b0, "sweeps of different mocks must not overlap in time"
    assert sweep_max > 300


def test_off_grid_draws_and_too_many():
    g = geom()
    rng = np.random.default_rng(4)
    recs = mock.draw(g, 4, rng, on_grid=False)
    assert any(r.dm not in set(g.dms.tolist()) for r in recs)
    assert all(1 <= r.width <= 8 for r in recs)
    with pytest.raises(ValueError):
        mock.draw(g, 20, rng)


def test_match_keeps_the_brightest_nearby_candidate():
    g = geom()
    r = mock.MockRecord(seg=0, dm=100.0, t0=400.0, width=2.0, x=520.0, y=500.0, snr=20.0, amp=1.0)
    far = mock.MockRecord(seg=0, dm=100.0, t0=1200.0, width=1.0, x=400.0, y=400.0, snr=20.0, amp=1.0)
    rows = np.zeros(4, CAND)
    rows[0] = (12, 1, 400, 520, 500, 15.0, 0, 0)
    rows[1] = (13, 1, 400, 521, 499, 18.0, 0, 0)    # brighter, within 2 pixels
    rows[2] = (13, 1, 400, 530, 500, 40.0, 0, 0)    # too far in x
    rows[3] = (13, 1, 900, 520, 500, 50.0, 0, 0)    # wrong time
    mock.match([r, far], rows, g)
    assert r.found and r.found_key == [13, 1, 400, 521, 499] and r.found_snr == 18.0
    assert not far.found
    mock.match([far], np.zeros(0, CAND), g)
    assert not far.found


def test_efficiency_bins():
    recs = []
    for k in range(10):
        r = mock.MockRecord(seg=0, dm=0.0, t0=0.0, width=1.0, x=0, y=0, snr=float(k + 1), amp=1.0)
        r.found = k >= 5
        r.found_snr = r.snr * 0.9 if r.found else 0.0
        recs.append(r)
    tab = mock.efficiency(recs, "snr", bins=[1, 5.5, 10])
    assert [t["n"] for t in tab] == [5, 5]
    assert [t["found"] for t in tab] == [0, 5]
    assert tab[1]["fraction"] == 1.0 and math.isclose(tab[1]["snr_ratio"], 0.9)
    assert math.isnan(tab[0]["snr_ratio"])
