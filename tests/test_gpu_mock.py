"""Mock transients and counter-based noise on the device, through the C ABI
(rf_inject, rf_noise), against the oracle's injection and the host-side
definition of the noise stream; then the search over injected mocks against
the oracle's search, and the efficiency curve's shape."""
import sys

import numpy as np
import pytest

import oracle
import rfgen
from helpers import cand_keys, gpu_plan, oracle_plan, upload
from rfgen import philox

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _ulps(a, b, dtype):
    """|a - b| in units of the storage format's spacing at b."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    sp = np.spacing(np.abs(b).astype(dtype)).astype(np.float64)
    return np.abs(a - b) / sp


def _host(t, dtype):
    x = t.cpu().numpy()
    return x if dtype == 0 else x.view(np.float16)


def _compare_storage(got, want, dtype, what):
    if dtype == 0:
        g = np.stack([got.real, got.imag], -1)
        w = np.stack([want.real, want.imag], -1)
        fdt = np.float32
    else:
        g, w, fdt = got, want, np.float16
    exact = float(np.mean(g == w))
    worst = float(np.max(_ulps(g, w, fdt))) if g.size else 0.0
    say(what, "exact fraction", exact, "worst ulps", worst)
    assert worst <= 1.0, what
    assert exact >= 0.9999, what


def _small(npol=2, nchan=47, nant=10, nint=37):
    p = rfgen.smallcase(nant=nant, nint=nint, nchan=nchan, npix=128, npol=npol)
    p.pulses = []
    return p


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("npol", [2, 1])
def test_noise_matches_generator(torch, dtype, npol):
    """rf_noise equals the host definition of the stream (Philox4x32-10 +
    Box-Muller): a window that starts mid-stream, with an odd number of
    complex values per integration when npol == 1."""
    p = _small(npol=npol)
    g = gpu_plan(p, vis_dtype=dtype)
    seed, sid, t_first = 12345678901, 3, 5
    say("noise", "dtype", dtype, "npol", npol)
    v = g.noise(seed=seed, stream_id=sid, t_first=t_first)
    torch.cuda.synchronize()
    ref = philox.segment(seed, p.nint, p.nbl, p.nchan, p.npol, t_first=t_first, stream=sid)
    want = ref if dtype == 0 else rfgen.to_cf16(ref)
    _compare_storage(_host(v, dtype), want, dtype, f"noise dtype {dtype} npol {npol}")


def _mocks(p):
    du, dv = p.cell()
    n = p.npix
    l0, m0 = rfgen.pixel_to_lm(n // 2 + 5, n // 2 - 3, n, du, dv)
    return [
        dict(dm=float(p.dms[1]), t0=4.0, width=2.0, l=l0, m=m0, amp=0.3),        # on a trial
        dict(dm=37.7, t0=10.3, width=3.6, l=-0.004, m=0.006, amp=0.11),         # fractional
        dict(dm=60.0, t0=4.5, width=1.0, l=0.001, m=0.0, amp=0.5),              # overlaps the first
        dict(dm=120.0, t0=-3.2, width=5.0, l=0.0, m=-0.002, amp=0.2),           # starts before 0
        dict(dm=0.0, t0=35.5, width=4.0, l=0.02, m=0.013, amp=0.7),             # runs past the end
    ]


@pytest.mark.parametrize("dtype", [0, 1])
def test_inject_matches_oracle(torch, dtype):
    p = _small()
    vis = p.make_vis(with_pulses=False)
    stored = vis.astype(np.complex64) if dtype == 0 else rfgen.to_cf16(vis)
    g = gpu_plan(p, vis_dtype=dtype)
    mocks = _mocks(p)
    say("inject", "dtype", dtype, "mocks", len(mocks))
    dv = upload(vis, dtype)
    g.inject(dv, mocks)
    got = _host(dv, dtype)
    want = oracle.inject(stored, mocks, p.freq(), p.uvw(), p.tint_s, p.kdm)
    _compare_storage(got, want, dtype, f"inject dtype {dtype}")
    assert np.any(got != stored), "nothing was injected"


def test_inject_many_mocks_in_order(torch):
    """More mocks than one launch carries, overlapping each other: added in
    array order across launches."""
    p = _small()
    vis = p.make_vis(with_pulses=False)
    rng = np.random.default_rng(9)
    mocks = [dict(dm=float(rng.uniform(0, 120)), t0=float(rng.uniform(-5, 35)),
                  width=float(rng.uniform(0.3, 6)), l=float(rng.uniform(-0.01, 0.01)),
                  m=float(rng.uniform(-0.01, 0.01)), amp=float(rng.uniform(0.01, 0.5)))
             for _ in range(150)]
    g = gpu_plan(p, vis_dtype=1)
    dv = upload(vis, 1)
    say("inject 150 mocks")
    g.inject(dv, mocks)
    want = oracle.inject(rfgen.to_cf16(vis), mocks, p.freq(), p.uvw(), p.tint_s, p.kdm)
    _compare_storage(_host(dv, 1), want, 1, "inject 150 mocks")


def test_windowed_injection_equals_whole(torch):
    """Noise and mocks written window by window (t_first) give the values of
    the whole segment written at once, bit for bit."""
    from paper_1802_03084_amd import mock
    p = _small()
    g = gpu_plan(p)
    mocks = _mocks(p)
    whole = g.noise(seed=8, stream_id=1)
    g.inject(whole, mocks)
    say("windowed injection")
    for t0, n in [(0, 16), (16, 21), (9, 5)]:
        sp = mock._staging_plan(g, n)
        part = sp.noise(seed=8, stream_id=1, t_first=t0)
        sp.inject(part, mocks, t_first=t0)
        assert torch.equal(part, whole[t0:t0 + n]), (t0, n)


def test_synthesize_fp16_rounds_once(torch):
    """mock.synthesize on float16 storage: RNE16 of the complex64 segment
    with the mocks, through CF32 windows of a few integrations."""
    from paper_1802_03084_amd import mock
    p = _small()
    g = gpu_plan(p, vis_dtype=1)
    mocks = _mocks(p)
    say("synthesize fp16")
    v = mock.synthesize(g, 99, mocks, stream_id=2, chunk_ints=10)
    noise = philox.segment(99, p.nint, p.nbl, p.nchan, p.npol, stream=2)
    want = rfgen.to_cf16(oracle.inject(noise, mocks, p.freq(), p.uvw(), p.tint_s, p.kdm))
    _compare_storage(_host(v, 1), want, 1, "synthesize fp16")


def test_inject_rejects_bad_mocks(torch):
    import paper_1802_03084_amd as rf
    p = _small()
    g = gpu_plan(p)
    dv = g.empty_vis()
    for bad in [dict(width=0.0), dict(width=-1.0), dict(t0=float("nan")), dict(amp=float("inf"))]:
        mk = dict(dm=10.0, t0=1.0, width=1.0, l=0.0, m=0.0, amp=1.0)
        mk.update(bad)
        with pytest.raises(rf.RFError) as e:
            g.inject(dv, [mk])
        assert e.value.status == -3
    g.inject(dv, [])   # nothing to add is fine


@pytest.mark.parametrize("dtype", [0, 1])
def test_injected_search_matches_oracle(torch, dtype):
    """Mocks injected on the device and searched by the fused path give the
    oracle's candidates (oracle: the same injection on the host, then its
    search), and the on-trial mocks are found at their exact keys."""
    p = rfgen.smallcase(nant=19, nint=48, nchan=64, npix=128, seed=21)
    p.pulses = []
    du, dv_ = p.cell()
    n = p.npix
    pix = [(n // 2 + 6, n // 2 - 4), (n // 2 - 9, n // 2 + 2)]
    mocks = []
    for (x, y), (i, j, t0) in zip(pix, [(1, 1, 8), (0, 0, 30)]):
        l, m = rfgen.pixel_to_lm(x, y, n, du, dv_)
        w = p.widths[j]
        mocks.append(dict(dm=float(p.dms[i]), t0=float(t0), width=float(w), l=l, m=m,
                          amp=20.0 / np.sqrt(2.0 * w * p.nbl * p.nchan)))
    mocks.append(dict(dm=90.0, t0=20.4, width=2.7, l=0.003, m=-0.002,
                      amp=14.0 / np.sqrt(2.0 * 2.7 * p.nbl * p.nchan)))
    vis = p.make_vis(with_pulses=False)
    stored = vis.astype(np.complex64) if dtype == 0 else rfgen.to_cf16(vis)
    g = gpu_plan(p, vis_dtype=dtype)
    dvis = upload(vis, dtype)
    say("injected search", "dtype", dtype)
    g.inject(dvis, mocks)
    rows, _, st = g.search_segment(dvis, cap=4096, with_stats=True)
    o = oracle_plan(p)
    host = oracle.inject(stored, mocks, p.freq(), p.uvw(), p.tint_s, p.kdm)
    ostats, ocands, oimgs = oracle.search(host, o, keep_images=True)
    tol = 1e-5
    marginal = set()
    for key, ref in ostats.items():
        i, j, k = key
        s = st[g.image_base(i, j) + k]
        peak, x, y, sigma, snr = ref
        amax = float(np.max(np.abs(oimgs[key])))
        if oracle.is_marginal(oimgs[key], snr, o.threshold, tol):
            marginal.add(key)
        else:
            assert (int(s["x"]), int(s["y"])) == (x, y), key
        assert abs(float(s["peak"]) - peak) <= tol * amax, key
    want = [c[:5] for c in ocands if (c[0], c[1], c[2] // p.widths[c[1]]) not in marginal]
    got = [kk for kk in cand_keys(rows) if (kk[0], kk[1], kk[2] // p.widths[kk[1]]) not in marginal]
    assert got == want
    keys = cand_keys(rows)
    assert (1, 1, 8) + pix[0] in keys and (0, 0, 30) + pix[1] in keys


def test_efficiency_curve(torch):
    """Bright on-trial mocks are all recovered, at their exact keys when
    bright enough; faint ones almost never pass the 6 sigma threshold."""
    from paper_1802_03084_amd import mock
    p = rfgen.Preset(name="eff", nant=19, nint=512, tint_s=0.005, f_lo_ghz=1.0, f_hi_ghz=2.0,
                     nchan=64, npol=2, dms=np.linspace(0, 200, 8), widths=[1, 2, 4], npix=256,
                     seed=31)
    g = gpu_plan(p, vis_dtype=1)
    say("efficiency curve")
    hi = mock.run(g, nseg=4, per_seg=3, seed=5, snr=(15.0, 40.0))
    lo = mock.run(g, nseg=4, per_seg=3, seed=6, snr=(2.5, 3.5), noise_seed=77)
    for r in hi:
        assert r.found, r
        dm_idx = int(np.argmin(np.abs(p.dms - r.dm)))
        w_idx = p.widths.index(int(r.width))
        assert r.found_key == [dm_idx, w_idx, int(r.t0), int(r.x), int(r.y)], r
        assert 0.7 < r.found_snr / r.snr < 1.3, r
    assert sum(r.found for r in lo) <= 3
    tab = mock.efficiency(hi + lo, "snr", bins=[2.5, 3.5, 40.0])
    assert tab[1]["fraction"] == 1.0 and tab[0]["fraction"] <= 0.25
