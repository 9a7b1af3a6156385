"""Periodicity search through the C ABI (rf_search_periodic) against the
oracle's: every (DM, frequency) amplitude image's statistics and the
candidate list, on a small case (CF32 and CF16) and at the survey's transform
length and image size (2048 integrations, 1024^2), with a dispersed pulse
train injected."""
import sys

import numpy as np
import pytest

import oracle
import rfgen
from helpers import gpu_plan, oracle_plan, upload

pytestmark = pytest.mark.gpu

TOL = 1e-5


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _train(p, dm, period, phase, x, y, snr):
    """Noise plus a train of width-1 pulses every `period` integrations from
    pixel (x, y); snr is the fluctuation S/N of the fundamental (amplitude
    A / period against (2 T nbl nchan)^-1/2)."""
    vis = p.make_vis(with_pulses=False)
    du, dv = p.cell()
    l, m = rfgen.pixel_to_lm(x, y, p.npix, du, dv)
    amp = snr * period / np.sqrt(2.0 * p.nint * p.nbl * p.nchan)
    for t0 in range(phase, p.nint, period):
        rfgen.add_pulse(vis, p.uvw(), p.freq(), p.tint_s, p.kdm, dm, t0, 1, l, m, amp)
    return vis


def _compare(g, p, vis_host, dvis, select=None):
    o = oracle_plan(p)
    rows, n, st = g.search_periodic(dvis, cap=4096, with_stats=True)
    assert n == len(rows)
    ostats, ocands, oimgs = oracle.periodic_search(vis_host, o, select=select, keep_images=True)
    nf = p.nint // 2
    marginal = set()
    for key, ref in ostats.items():
        i, f = key
        s = st[i * nf + f - 1]
        peak, x, y, sigma, snr = ref
        amax = float(np.max(oimgs[key]))
        if oracle.is_marginal(oimgs[key], snr, o.threshold, TOL):
            marginal.add(key)
        else:
            assert (int(s["x"]), int(s["y"])) == (x, y), key
        assert abs(float(s["peak"]) - peak) <= TOL * amax, (key, float(s["peak"]), peak)
        assert abs(float(s["sigma"]) - sigma) <= TOL * amax, (key, float(s["sigma"]), sigma)
    got = [(int(r["dm_idx"]), int(r["t_int"]), int(r["x"]), int(r["y"])) for r in rows
           if (int(r["dm_idx"]), int(r["t_int"])) not in marginal
           and (select is None or (int(r["dm_idx"]), int(r["t_int"])) in select)]
    want = [c[:4] for c in ocands if (c[0], c[1]) not in marginal]
    assert sorted(got) == sorted(want)
    assert all(int(r["width_idx"]) == -1 for r in rows)
    say("periodic: images", len(ostats), "candidates", len(want), "marginal", len(marginal))
    return rows


@pytest.mark.parametrize("dtype,nint", [(0, 32), (1, 32), (0, 64), (1, 256)])
def test_periodic_small_matches_oracle(torch, dtype, nint):
    """Every (DM, frequency) image: the radix-2 time transform (32) and the
    register/LDS one (64, 256)."""
    p = rfgen.smallcase(nant=10, nint=nint, nchan=48, npix=128, seed=17)
    p.dms = np.array([0.0, 40.0])
    p.widths = [1]
    p.pulses = []
    c = p.npix // 2
    vis = _train(p, 40.0, 8, 3, c + 5, c - 4, snr=25.0)
    host = vis if dtype == 0 else rfgen.to_cf16(vis)
    g = gpu_plan(p, vis_dtype=dtype)
    say("periodic small, dtype", dtype, "nint", nint)
    rows = _compare(g, p, host, upload(vis, dtype))
    assert (1, nint // 8, c + 5, c - 4) in [(int(r["dm_idx"]), int(r["t_int"]), int(r["x"]),
                                             int(r["y"])) for r in rows]


def test_periodic_survey_transform(torch):
    """2048-integration transform and 1024^2 images: the pulse train's DM
    trial at its first harmonics, the band edges and a spread of other
    frequencies against the oracle."""
    p = rfgen.Preset(name="psr", nant=10, nint=2048, tint_s=0.010, f_lo_ghz=1.0, f_hi_ghz=2.0,
                     nchan=64, npol=2, dms=np.array([0.0, 150.0, 300.0]), widths=[1], npix=1024,
                     seed=23)
    c = p.npix // 2
    vis = _train(p, 150.0, 64, 17, c - 20, c + 11, snr=30.0)
    g = gpu_plan(p)
    say("periodic survey transform")
    freqs = {1, 2, 31, 32, 33, 64, 96, 128, 257, 500, 777, 1023, 1024}
    rows = _compare(g, p, vis, upload(vis), select={(1, f) for f in freqs})
    keys = [(int(r["dm_idx"]), int(r["t_int"]), int(r["x"]), int(r["y"])) for r in rows]
    assert (1, 32, c - 20, c + 11) in keys      # fundamental: 2048 / 64


def test_periodic_rejects_bad_shapes(torch):
    import paper_1802_03084_amd as rf
    p = rfgen.smallcase(nant=10, nint=37, nchan=48, npix=128)
    g = gpu_plan(p)
    with pytest.raises(rf.RFError) as e:
        g.search_periodic(g.empty_vis())
    assert e.value.status == -3
