"""HIP path against the CPU oracle, step by step and end to end.

Bars: integer tables, dedispersed visibilities and candidate keys are
bit-exact; float results agree to 1e-5 of the reference maximum (float32
storage) or 3e-3 (float16 storage against the float64 oracle on the
unrounded input).  Every call goes through librf's C ABI.
"""
import sys

import numpy as np
import pytest

import oracle
import rfgen
from helpers import cand_keys, gpu_plan, oracle_plan, rel_err, upload

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL16 = 3e-3


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


PRESETS = {
    "tiny": rfgen.tiny,
    "small": rfgen.smallcase,
    "small_n64_p1": lambda: rfgen.smallcase(nant=6, nint=9, nchan=20, npix=64, npol=1, seed=9),
    "small_n512": lambda: rfgen.smallcase(nant=12, nint=7, nchan=33, npix=512, seed=8),
}


@pytest.mark.parametrize("name", ["tiny", "small", "small_n64_p1", "small_n512", "survey"])
def test_plan_tables_bit_exact(torch, name):
    p = rfgen.survey() if name == "survey" else PRESETS[name]()
    say("tables", name)
    g = gpu_plan(p)
    o = oracle_plan(p)
    assert np.array_equal(g.delays(), o.delays)
    cells = g.cells()
    assert np.array_equal(cells[..., 0], o.iu)
    assert np.array_equal(cells[..., 1], o.iv)
    assert g.W == o.W
    assert g.info["max_delay"] == int(o.delays.max())


@pytest.mark.parametrize("name", ["tiny", "small", "small_n64_p1"])
@pytest.mark.parametrize("dtype", [0, 1])
def test_dedisperse_bit_exact(torch, name, dtype):
    p = PRESETS[name]()
    say("dedisperse", name, dtype)
    vis = p.make_vis()
    g = gpu_plan(p, vis_dtype=dtype)
    o = oracle_plan(p)
    dv = upload(vis, dtype)
    host = dv.cpu().numpy()
    for i in range(len(p.dms)):
        out = g.dedisperse(dv, i).cpu().numpy()
        ref = oracle.dedisperse(oracle.as_complex(host), o.delays[i])
        if dtype == 0:
            assert np.array_equal(out.astype(np.complex128), ref), i
        else:
            assert np.array_equal(oracle.as_complex(out), ref), i


@pytest.mark.parametrize("name", ["tiny", "small", "small_n64_p1"])
@pytest.mark.parametrize("dtype", [0, 1])
def test_resample(torch, name, dtype):
    p = PRESETS[name]()
    say("resample", name, dtype)
    vis = p.make_vis()
    g = gpu_plan(p, vis_dtype=dtype)
    dv = upload(vis, dtype)
    ref_in = oracle.as_complex(dv.cpu().numpy())
    for w in (1, 2, 3, 4, 8, p.nint):
        out = g.resample(dv, w).cpu().numpy()
        ref = oracle.resample(ref_in, w)
        assert out.shape == ref.shape
        assert rel_err(out.real, ref.real) < 1e-6 and rel_err(out.imag, ref.imag) < 1e-6, w


@pytest.mark.parametrize("name", ["tiny", "small", "small_n64_p1", "small_n512"])
def test_grid_and_image(torch, name):
    p = PRESETS[name]()
    say("grid+image", name)
    vis = p.make_vis()
    g = gpu_plan(p)
    o = oracle_plan(p)
    nimg = min(p.nint, 5)   # odd count: the last image has no partner
    dv = upload(vis[:nimg])
    grid = g.grid(dv)
    gh = grid.cpu().numpy()
    img = g.image(grid).cpu().numpy()
    for k in range(nimg):
        G = oracle.grid(oracle.stokes_i(vis[k].astype(np.complex128)), o.iu, o.iv, o.valid, p.npix)
        assert rel_err(gh[k].real, G.real) < TOL32 and rel_err(gh[k].imag, G.imag) < TOL32
        ref = oracle.image(G, o.W)
        e = rel_err(img[k], ref)
        assert e < TOL32, (k, e)


@pytest.mark.parametrize("name", ["tiny", "small"])
def test_search_stats_exact_on_same_image(torch, name):
    """Given the same float32 image, peak, argmax and the lower median are
    exact order statistics and must match bit for bit."""
    p = PRESETS[name]()
    say("search stats", name)
    g = gpu_plan(p)
    vis = p.make_vis()
    nimg = min(p.nint, 6)
    img_t = g.image(g.grid(upload(vis[:nimg])))
    # plant ties and a flat image
    img_t[1].fill_(0.25)
    img_t[2, 3, 5] = float(img_t[2].max()) + 1.0
    img_t[2, 7, 1] = float(img_t[2, 3, 5])
    img = img_t.cpu().numpy()
    tags = np.array([[0, 0, k] for k in range(nimg)], np.int32)
    rows, n, st = g.search(img_t, tags, cap=64)
    for k in range(nimg):
        flat = img[k].ravel()
        idx = int(np.argmax(flat))
        a = np.sort(np.abs(flat))
        med = a[(a.size - 1) // 2]
        assert st[k]["peak"] == flat[idx]
        assert (st[k]["x"], st[k]["y"]) == (idx % p.npix, idx // p.npix)
        assert st[k]["sigma"] == np.float32(1.4826) * med
    assert (st[2]["x"], st[2]["y"]) == (5, 3), "ties go to the lowest flat index"


def _segment_parity(p, dtype, tol):
    o = oracle_plan(p)
    g = gpu_plan(p, vis_dtype=dtype)
    vis = p.make_vis()
    dv = upload(vis, dtype)
    rows, n, st = g.search_segment(dv, cap=4096, with_stats=True)
    ostats, ocands, oimgs = oracle.search(vis, o, keep_images=True)
    assert n == len(rows)
    marginal = set()
    for key, ref in ostats.items():
        i, j, k = key
        s = st[g.image_base(i, j) + k]
        peak, x, y, sigma, snr = ref
        if oracle.is_marginal(oimgs[key], snr, o.threshold, tol):
            marginal.add(key)
        else:
            assert (int(s["x"]), int(s["y"])) == (x, y), key
        # an order statistic moves by at most the largest pixel error, which
        # the image bar bounds by tol * max|ref|
        amax = float(np.max(np.abs(oimgs[key])))
        assert abs(s["peak"] - peak) <= tol * amax, key
        assert abs(s["sigma"] - sigma) <= 1.4826 * tol * amax, key
    want = [c[:5] for c in ocands if (c[0], c[1], c[2] // p.widths[c[1]]) not in marginal]
    got = [k for k in cand_keys(rows)
           if (k[0], k[1], k[2] // p.widths[k[1]]) not in marginal]
    assert got == want
    return rows, marginal


@pytest.mark.parametrize("dtype,tol", [(0, TOL32), (1, TOL16)])
def test_segment_tiny(torch, dtype, tol):
    p = rfgen.tiny()
    say("segment tiny", dtype)
    rows, marginal = _segment_parity(p, dtype, tol)
    pulse = p.pulses[0]
    assert cand_keys(rows) == [(pulse.dm_idx, pulse.width_idx, pulse.t0, pulse.x, pulse.y)]
    say("marginal images excluded from the exact comparison:", len(marginal))
    assert (pulse.dm_idx, pulse.width_idx, pulse.t0) not in marginal


@pytest.mark.parametrize("dtype,tol", [(0, TOL32), (1, TOL16)])
def test_segment_small(torch, dtype, tol):
    p = rfgen.smallcase()
    say("segment small", dtype)
    rows, _ = _segment_parity(p, dtype, tol)
    pulse = p.pulses[0]
    assert (pulse.dm_idx, pulse.width_idx, pulse.t0, pulse.x, pulse.y) in cand_keys(rows)


def test_segment_window_and_capacity(torch):
    p = rfgen.tiny()
    say("segment window/cap")
    vis = upload(p.make_vis())
    g = gpu_plan(p, t_begin=1)
    rows, n, _ = g.search_segment(vis, cap=16)
    assert n == 0
    p2 = rfgen.tiny()
    p2.threshold = 0.5   # every image is a candidate
    g2 = gpu_plan(p2)
    rows, n, _ = g2.search_segment(vis, cap=7)
    assert n == p2.n_images() and len(rows) == 7


@pytest.mark.parametrize("name", ["tiny", "small", "small_n64_p1", "small_n512"])
@pytest.mark.parametrize("dtype", [0, 1])
def test_fused_equals_steps(torch, name, dtype):
    """rf_search_segment (fused) and rf_search_segment_steps (plain chain)
    give bit-identical statistics and candidates."""
    p = PRESETS[name]()
    say("fused vs steps", name, dtype)
    g = gpu_plan(p, vis_dtype=dtype)
    dv = upload(p.make_vis(), dtype)
    r1, n1, s1 = g.search_segment(dv, cap=4096, with_stats=True)
    r2, n2, s2 = g.search_segment(dv, cap=4096, with_stats=True, steps=True)
    assert n1 == n2
    assert np.array_equal(r1, r2)
    assert np.array_equal(s1.view(np.int32), s2.view(np.int32))


def test_fused_bright_source_exact_fallback(torch):
    """A very bright pulse moves the image rms far from the noise median, so
    the median bracket misses and the exact recomputation must take over."""
    p = rfgen.tiny()
    p.pulses = [rfgen.Pulse(dm_idx=1, width_idx=0, t0=3, x=140, y=120, snr=400.0)]
    say("bright source fallback")
    g = gpu_plan(p)
    o = oracle_plan(p)
    vis = p.make_vis()
    dv = upload(vis)
    r1, n1, s1 = g.search_segment(dv, cap=4096, with_stats=True)
    r2, n2, s2 = g.search_segment(dv, cap=4096, with_stats=True, steps=True)
    assert np.array_equal(s1.view(np.int32), s2.view(np.int32))
    assert np.array_equal(r1, r2)
    key = (1, 0, 3)
    st, _, im = oracle.search(vis, o, select={key}, keep_images=True)
    ref = st[key]
    s = s1[g.image_base(1, 0) + 3]
    assert (int(s["x"]), int(s["y"])) == (140, 120)
    amax = float(np.max(np.abs(im[key])))
    assert abs(s["sigma"] - ref[3]) <= 1.4826 * TOL32 * amax
    assert s["snr"] > 50


def test_profile_modes_match_search(torch):
    """rf_search_segment_profile, serial and concurrent, returns the same
    candidates as rf_search_segment and times the same launches; a mode other
    than 0 or 1 is rejected."""
    import ctypes
    from paper_1802_03084_amd import _lib
    p = rfgen.smallcase(nint=24, npix=256, seed=31)
    say("profile modes")
    g = gpu_plan(p)
    dv = upload(p.make_vis())
    r0, n0, _ = g.search_segment(dv, cap=4096)
    t1, r1, n1 = g.profile_segment(dv, cap=4096, concurrent=False)
    t2, r2, n2 = g.profile_segment(dv, cap=4096, concurrent=True)
    assert n0 == n1 == n2
    assert np.array_equal(r0, r1) and np.array_equal(r0, r2)
    for k in ("drs", "grid", "rows", "cols", "select"):
        assert t1[k][1] == t2[k][1] > 0, k
        assert t1[k][0] > 0 and t2[k][0] > 0, k
    kt = _lib.KernelTimes()
    kt.concurrent = 2
    ws = g.workspace(_lib.RF_OP_SEGMENT)
    cand = torch.empty((16, 8), dtype=torch.int32, device=dv.device)
    ncand = torch.zeros(1, dtype=torch.int32, device=dv.device)
    st = _lib.load().rf_search_segment_profile(g._h, ctypes.c_void_p(dv.data_ptr()),
                                               ctypes.c_void_p(cand.data_ptr()), 16,
                                               ctypes.c_void_p(ncand.data_ptr()), None,
                                               ctypes.c_void_p(ws.data_ptr()), ws.numel(), None,
                                               ctypes.byref(kt))
    assert st == _lib.RF_EINVAL


def _band_preset(n, nint, pulses=(), seed=13):
    """Few integrations of the survey band (1024^2: 256 channels over 1-2 GHz,
    10 ms) or of the large band (2048^2: 1024 channels over 2-4 GHz, 1 ms)."""
    if n == 1024:
        return rfgen.Preset(name="survey-band", nant=27, nint=nint, tint_s=0.010, f_lo_ghz=1.0,
                            f_hi_ghz=2.0, nchan=256, npol=2, dms=np.array([0.0, 40.0]),
                            widths=[1, 2], npix=n, seed=seed, pulses=list(pulses))
    return rfgen.Preset(name="large-band", nant=27, nint=nint, tint_s=0.001, f_lo_ghz=2.0,
                        f_hi_ghz=4.0, nchan=1024, npol=2, dms=np.array([0.0, 30.0]),
                        widths=[1, 2], npix=n, seed=seed, pulses=list(pulses))


@pytest.mark.parametrize("n", [1024, 2048])
def test_image_full_size_elementwise(torch, n):
    """rf_image, the dense transform of the exact fallback, the second-tier
    products and the periodicity search, element by element against the
    oracle's image at the survey (1024^2) and large (2048^2) sizes: three
    images, the last without a partner in its transform pair."""
    p = _band_preset(n, 3)
    say("rf_image element-wise", n)
    vis = p.make_vis()
    g = gpu_plan(p)
    o = oracle_plan(p)
    img = g.image(g.grid(upload(vis))).cpu().numpy()
    for k in range(p.nint):
        G = oracle.grid(oracle.stokes_i(vis[k].astype(np.complex128)), o.iu, o.iv, o.valid, n)
        ref = oracle.image(G, o.W)
        e = rel_err(img[k], ref)
        say(f"  image {k}: max |diff| / max |ref| = {e:.2e}")
        assert e < TOL32, (k, e)


def test_fused_bright_source_exact_fallback_2048(torch):
    """The exact fallback at 2048^2: a very bright pulse moves the rms far
    from the noise median, the bracket misses, the image is recomputed by the
    dense step chain; fused and step results are identical and sigma matches
    the oracle's exact lower median."""
    n = 2048
    p = _band_preset(n, 6, [rfgen.Pulse(dm_idx=1, width_idx=0, t0=2, x=n // 2 + 70, y=n // 2 - 41,
                                        snr=600.0)])
    say("bright source fallback 2048")
    g = gpu_plan(p)
    o = oracle_plan(p)
    vis = p.make_vis()
    dv = upload(vis)
    times, _, _ = g.profile_segment(dv, cap=4096)
    assert times["fallback"][1] >= 1, times
    r1, n1, s1 = g.search_segment(dv, cap=4096, with_stats=True)
    r2, n2, s2 = g.search_segment(dv, cap=4096, with_stats=True, steps=True)
    assert np.array_equal(s1.view(np.int32), s2.view(np.int32))
    assert np.array_equal(r1, r2)
    key = (1, 0, 2)
    st, _, im = oracle.search(vis, o, select={key}, keep_images=True)
    peak, x, y, sigma, snr = st[key]
    s = s1[g.image_base(1, 0) + 2]
    assert (int(s["x"]), int(s["y"])) == (x, y) == (n // 2 + 70, n // 2 - 41)
    amax = float(np.max(np.abs(im[key])))
    assert abs(s["peak"] - peak) <= TOL32 * amax
    assert abs(s["sigma"] - sigma) <= 1.4826 * TOL32 * amax
    assert s["snr"] > 50


def test_segment_begin_end_equals_search(torch):
    """rf_search_segment_begin / _end: two searches in flight at once on two
    streams (a bright-source segment whose image takes the exact fallback,
    and a plain one), each equal to rf_search_segment bit for bit."""
    pa = rfgen.tiny()
    pa.pulses = [rfgen.Pulse(dm_idx=1, width_idx=0, t0=3, x=140, y=120, snr=400.0)]
    pb = rfgen.smallcase(seed=23)
    say("segment begin/end")
    out = []
    for p in (pa, pb):
        g = gpu_plan(p)
        dv = upload(p.make_vis())
        out.append((g, dv, g.search_segment(dv, cap=4096, with_stats=True)))
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    jobs = [g.search_segment_begin(dv, cap=4096, with_stats=True, stream=st)
            for (g, dv, _), st in zip(out, (s1, s2))]
    for (g, dv, (rows0, n0, st0)), job in zip(out, jobs):
        rows, n, st = g.search_segment_end(job)
        assert n == n0 and np.array_equal(rows, rows0)
        assert np.array_equal(st.view(np.int32), st0.view(np.int32))
