"""Pins for the CPU oracle: checks against values fixed by the paper or by
mathematics, never against the oracle's own formula.

Each check takes an implementation namespace `o` (the oracle module, or a copy
with a planted mistake) and raises AssertionError when the implementation is
wrong.  test_oracle_pins.py runs them on the oracle; test_oracle_mutants.py
runs them on oracles with planted mistakes and requires that they fail.
"""
import json
import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def paper_values():
    with open(os.path.join(GOLDEN, "paper_values.json")) as f:
        return json.load(f)


def centres(lo, hi, n):
    return lo + (np.arange(n) + 0.5) * (hi - lo) / n


# ---------------------------------------------------------------- delay table

def check_delay_law(o):
    """The printed law: tau = 4.15 ms DM / nu^2 (section 2.1 footnote).
    Against an effectively infinite reference frequency, with 1 us
    integrations, DM 1 at 1 GHz is 4150 us, DM 100 at 2 GHz is 103750 us and
    DM 7 at 0.5 GHz is 4 * 7 * 4150 us."""
    pv = paper_values()["dispersion_law"]
    k = pv["delay_ms_per_dm_at_1ghz"] * 1e-3
    f = np.array([1.0, 2.0, 0.5, 1e9])
    d = o.delay_table(f, np.array([1.0, 100.0, 7.0]), 1e-6, k)
    assert d.shape == (3, 4)
    assert int(d[0, 0]) == 4150, d
    assert int(d[1, 1]) == 103750, d
    assert int(d[2, 2]) == 4 * 7 * 4150, d
    assert (d[:, 3] == 0).all()


def check_delay_properties(o):
    f = centres(1.0, 2.0, 64)
    dms = np.linspace(0, 500, 11)
    d = o.delay_table(f, dms, 0.005, 4.15e-3)
    assert d.dtype == np.int32
    assert (d[0] == 0).all(), "DM = 0 must not shift anything"
    assert (d[:, -1] == 0).all(), "the top channel is the reference"
    assert (d >= 0).all()
    assert (np.diff(d, axis=1) <= 0).all(), "delay must not grow with frequency"
    assert (np.diff(d, axis=0) >= 0).all(), "delay must not shrink with DM"


def check_delay_hand_values(o):
    hv = paper_values()["hand_values"]
    t = hv["tiny_dm100_chan0"]
    d = o.delay_table(centres(t["f_lo_ghz"], t["f_hi_ghz"], t["nchan"]),
                      np.array([t["dm"]]), t["tint_s"], 4.15e-3)
    assert int(d[0, t["chan"]]) == t["delay"], d[0, :4]
    for key in ("survey_dm1000_max", "large_dm3000_max"):
        s = hv[key]
        d = o.delay_table(centres(s["f_lo_ghz"], s["f_hi_ghz"], s["nchan"]),
                          np.array([s["dm"]]), s["tint_s"], 4.15e-3)
        assert int(d.max()) == s["delay_max"], (key, int(d.max()))


def check_delay_rounding(o):
    """Whole-integration rounding is round-half-even: with K DM = 1.25 s GHz^2,
    nu = 2 GHz against an infinite reference and t_int = 0.125 s the exact
    delay is 2.5 integrations -> 2; with K DM = 1.75 it is 3.5 -> 4."""
    f = np.array([2.0, 1e150])
    d = o.delay_table(f, np.array([1.25, 1.75]), 0.125, 1.0)
    assert int(d[0, 0]) == 2 and int(d[1, 0]) == 4, d


def check_sweep_example(o):
    """Section 3.2: DM 2000 over 256 MHz at 1.4 GHz sweeps 'roughly 2 s'."""
    s = paper_values()["sweep_example"]
    lo = s["centre_ghz"] - s["bandwidth_mhz"] / 2000.0
    hi = s["centre_ghz"] + s["bandwidth_mhz"] / 2000.0
    d = o.delay_table(np.array([lo, hi]), np.array([s["dm"]]), 1e-3, 4.15e-3)
    sweep = d[0, 0] * 1e-3
    assert 0.7 * s["approx_sweep_s"] < sweep < 1.05 * s["approx_sweep_s"], sweep


# ---------------------------------------------------------------- cell table

def check_cells(o):
    """Hand values: a 1000 m east baseline at 1.5 GHz spans
    1000 * 1.5e9 / 299792458 = 5003.46 wavelengths -> cell 50 at du = 100;
    a 250 m north baseline at the same frequency is 1250.87 wavelengths ->
    cell 13 at dv = 100 (while u is 0)."""
    uvw = np.array([[1000.0, 0.0, 0.0], [0.0, 250.0, 0.0], [-1000.0, -250.0, 0.0]])
    iu, iv = o.cell_table(uvw, np.array([1.5, 3.0]), 100.0, 100.0)
    assert iu.shape == (3, 2)
    assert int(iu[0, 0]) == 50 and int(iv[0, 0]) == 0
    assert int(iu[1, 0]) == 0 and int(iv[1, 0]) == 13
    assert int(iu[2, 0]) == -50 and int(iv[2, 0]) == -13
    assert int(iu[0, 1]) == 100 and int(iv[1, 1]) == 25  # 10006.9 -> 100; 2501.7 -> 25
    assert o.valid_cells(np.array([63, 64, -63, -64]), np.array([0, 0, 0, 0]), 128).tolist() == [True, False, True, False]


# ---------------------------------------------------------------- dedispersion

def check_dedisperse(o):
    rng = np.random.default_rng(11)
    T, B, C, P = 12, 3, 5, 2
    vis = rng.standard_normal((T, B, C, P)) + 1j * rng.standard_normal((T, B, C, P))
    assert np.array_equal(o.dedisperse(vis, np.zeros(C, np.int32)), vis), "DM = 0 is the identity"
    d = np.array([4, 3, 2, 0, 13], np.int32)
    # an impulse arriving at t0 + d[c] in every channel lands at t0
    imp = np.zeros((T, B, C, P), complex)
    t0 = 5
    for c in range(C):
        if t0 + d[c] < T:
            imp[t0 + d[c], :, c, :] = 1.0
    out = o.dedisperse(imp, d)
    for c in range(C):
        col = out[:, 0, c, 0]
        if t0 + d[c] < T:
            assert col[t0] == 1.0 and np.count_nonzero(col) == 1, (c, col)
        else:
            assert np.count_nonzero(col) == 0
    # what moves in from past the end is zero; nothing else is touched
    out = o.dedisperse(vis, d)
    assert (out[T - 4:, :, 0, :] == 0).all()
    assert np.array_equal(out[: T - 4, :, 0, :], vis[4:, :, 0, :])
    assert (out[:, :, 4, :] == 0).all()
    assert np.array_equal(out[:, :, 3, :], vis[:, :, 3, :])


# ---------------------------------------------------------------- resampling

def check_resample(o):
    rng = np.random.default_rng(12)
    x = rng.standard_normal((13, 2, 3, 2)) + 1j * rng.standard_normal((13, 2, 3, 2))
    assert np.array_equal(o.resample(x, 1), x)
    r4 = o.resample(x, 4)
    assert r4.shape == (3, 2, 3, 2), "the remainder is dropped"
    # a linear ramp t -> mean over [k w, (k+1) w) is k w + (w - 1)/2
    ramp = np.arange(13, dtype=float)[:, None, None, None] * np.ones((1, 2, 3, 2))
    r = o.resample(ramp.astype(complex), 4)
    assert np.allclose(r[:, 0, 0, 0].real, [1.5, 5.5, 9.5], rtol=0, atol=1e-15)
    assert np.allclose(o.resample(np.full((8, 1, 1, 1), 3.0 + 2j), 8), 3.0 + 2j)
    # resampling twice by 2 equals resampling by 4
    assert np.allclose(o.resample(o.resample(x, 2), 2), r4, rtol=0, atol=1e-14)
    # flux is conserved over the kept samples
    assert np.allclose(r4.sum(axis=0) * 4, x[:12].sum(axis=0), rtol=0, atol=1e-12)


def check_stokes(o):
    v = np.zeros((2, 3, 2), complex)
    v[..., 0] = 1 + 2j
    v[..., 1] = 3 - 4j
    assert np.allclose(o.stokes_i(v), 2 - 1j)
    assert np.allclose(o.stokes_i(v[..., :1]), 1 + 2j)


# ---------------------------------------------------------------- gridding

def check_grid(o):
    N = 16
    iu = np.array([[3, -2], [3, 7]])
    iv = np.array([[-5, 0], [-5, 9]])
    valid = o.valid_cells(iu, iv, N)
    assert valid.tolist() == [[True, True], [True, False]]
    vi = np.array([[1 + 1j, 2.0], [0.5j, 100.0]])
    G = o.grid(vi, iu, iv, valid, N)
    assert G.shape == (N, N)
    assert G[N - 5, 3] == 1 + 1.5j, "two samples in one cell add; negative v wraps"
    assert G[0, N - 2] == 2.0, "negative u wraps to column N - 2"
    assert np.count_nonzero(G) == 2
    assert np.isclose(G.sum(), (1 + 1j) + 2 + 0.5j), "dropped samples do not reach the grid"


# ---------------------------------------------------------------- imaging

def _dft_image(vi, iu, iv, N, W):
    """Brute force: direct sum over samples of the image definition."""
    X = np.arange(N) - N / 2
    img = np.zeros((N, N))
    for a, u, v in zip(vi, iu, iv):
        ph = 2 * np.pi * (u * X[None, :] + v * X[:, None]) / N
        img += (a * np.exp(1j * ph)).real
    return img / W


def check_image_dft(o):
    """FFT imaging equals a brute-force direct DFT of the samples (N <= 64)."""
    rng = np.random.default_rng(13)
    for N in (16, 32, 64):
        n = 40
        iu = rng.integers(-N // 2 + 1, N // 2, n)
        iv = rng.integers(-N // 2 + 1, N // 2, n)
        vi = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        W = n
        G = o.grid(vi, iu, iv, np.ones(n, bool), N)
        img = o.image(G, W)
        ref = _dft_image(vi, iu, iv, N, W)
        assert np.max(np.abs(img - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref))), N


def check_image_single_cell(o):
    """One unit sample at cell (iu, iv) = (3, -5) images to
    cos(2 pi (3 (X - N/2) - 5 (Y - N/2)) / N) / W (orientation and sign)."""
    N = 32
    G = np.zeros((N, N), complex)
    G[(-5) % N, 3] = 1.0
    img = o.image(G, 7)
    X = np.arange(N) - N / 2
    ref = np.cos(2 * np.pi * (3 * X[None, :] - 5 * X[:, None]) / N) / 7
    assert np.allclose(img, ref, rtol=0, atol=1e-13)
    # a quarter-turn phase makes it -sin(...)
    G[(-5) % N, 3] = 1j
    ref = -np.sin(2 * np.pi * (3 * X[None, :] - 5 * X[:, None]) / N) / 7
    assert np.allclose(o.image(G, 7), ref, rtol=0, atol=1e-13)


def check_image_point_source(o):
    """A source at the phase centre (V = A on every sample) images to A at
    pixel (N/2, N/2), which is the global maximum."""
    rng = np.random.default_rng(14)
    N = 64
    n = 300
    iu = rng.integers(-N // 2 + 1, N // 2, n)
    iv = rng.integers(-N // 2 + 1, N // 2, n)
    A = 0.37
    img = o.image(o.grid(np.full(n, A, complex), iu, iv, np.ones(n, bool), N), n)
    assert abs(img[N // 2, N // 2] - A) < 1e-14
    assert np.argmax(img) == (N // 2) * N + N // 2


def check_image_parseval(o):
    """sum img^2 = N^2/(2 W^2) (sum |G|^2 + Re sum G[k] G[-k]); sum img =
    N^2 Re G[0, 0] / W."""
    rng = np.random.default_rng(15)
    N, W = 32, 9
    G = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    img = o.image(G, W)
    Gm = np.roll(np.flip(G, axis=(0, 1)), 1, axis=(0, 1))  # G[-k]
    lhs = float((img ** 2).sum())
    rhs = N * N / (2 * W * W) * (float((np.abs(G) ** 2).sum()) + float((G * Gm).sum().real))
    assert abs(lhs - rhs) < 1e-10 * rhs
    assert abs(img.sum() - N * N * G[0, 0].real / W) < 1e-9


def check_image_offset_source(o):
    """A source at pixel (X0, Y0), simulated with exact phases and gridded to
    the nearest cell, peaks at (X0, Y0) above 0.98 of its flux."""
    import rfgen
    N = 128
    uvw = rfgen.baseline_uvw(rfgen.y_array_positions(27))
    f = centres(1.0, 2.0, 32)
    du = rfgen.default_cell_size(uvw, f, N)
    iu, iv = o.cell_table(uvw, f, du, du)
    valid = o.valid_cells(iu, iv, N)
    for X0, Y0 in ((N // 2 + 5, N // 2 - 3), (N // 2 - 8, N // 2 + 7)):
        l, m = rfgen.pixel_to_lm(X0, Y0, N, du, du)
        ul = uvw[:, 0:1] * f[None, :] * 1e9 / rfgen.C_LIGHT
        vl = uvw[:, 1:2] * f[None, :] * 1e9 / rfgen.C_LIGHT
        vi = 0.5 * np.exp(-2j * np.pi * (ul * l + vl * m))
        img = o.image(o.grid(vi, iu, iv, valid, N), int(valid.sum()))
        y, x = divmod(int(np.argmax(img)), N)
        assert (x, y) == (X0, Y0), (x, y)
        assert img[y, x] > 0.98 * 0.5


def check_image_linear(o):
    rng = np.random.default_rng(16)
    N = 16
    G1 = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    G2 = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    assert np.allclose(o.image(2 * G1 - G2, 5), 2 * o.image(G1, 5) - o.image(G2, 5), atol=1e-12)


# ---------------------------------------------------------------- statistics

def check_stats(o):
    rng = np.random.default_rng(17)
    img = rng.standard_normal((32, 32))
    img[7, 9] = 50.0
    img[20, 3] = 50.0   # tie: the lower flat index (row 7) wins
    peak, x, y, sigma, snr = o.image_stats(img)
    assert (peak, x, y) == (50.0, 9, 7)
    a = np.sort(np.abs(img.ravel()))
    assert sigma == 1.4826 * a[(a.size - 1) // 2], "lower median of |img|"
    assert snr == peak / sigma
    # a negative extreme is not a peak; all-zero images have S/N 0
    img2 = -np.abs(img)
    img2[0, 0] = 1.0
    assert o.image_stats(img2)[:3] == (1.0, 0, 0)
    assert o.image_stats(np.zeros((8, 8)))[4] == 0.0
    # S/N is scale free
    assert abs(o.image_stats(3 * img)[4] - snr) < 1e-12 * snr


def check_noise_sigma(o):
    """Unit complex noise per polarisation, averaged over 2 polarisations and
    w samples, gives image noise (2 w W)^-1/2 (MAD estimate within 5%)."""
    import rfgen
    N, nchan = 128, 32
    uvw = rfgen.baseline_uvw(rfgen.y_array_positions(27))
    f = centres(1.0, 2.0, nchan)
    du = rfgen.default_cell_size(uvw, f, N)
    iu, iv = o.cell_table(uvw, f, du, du)
    valid = o.valid_cells(iu, iv, N)
    W = int(valid.sum())
    vis = rfgen.noise_vis(21, 8, uvw.shape[0], nchan, 2)
    for w in (1, 2):
        rs = o.resample(vis.astype(np.complex128), w)
        sig = [o.image_stats(o.image(o.grid(o.stokes_i(rs[k]), iu, iv, valid, N), W))[3]
               for k in range(rs.shape[0])]
        pred = (2 * w * W) ** -0.5
        assert abs(np.mean(sig) / pred - 1) < 0.05, (w, np.mean(sig), pred)


# ---------------------------------------------------------------- windowed forms

def _window_case(o):
    """A small plan whose largest delays reach and pass the segment length,
    with widths that leave a remainder (T = 13)."""
    from rfgen import synth
    uvw = synth.baseline_uvw(synth.y_array_positions(8))
    f = centres(1.0, 2.0, 10)
    N = 32
    du = synth.default_cell_size(uvw, f, N)
    plan = o.Plan(f, uvw, 0.005, np.array([0.0, 8.0, 30.0]), [1, 2, 4], N, du, du, nint=13)
    return plan, uvw, f


def check_dedisperse_window(o):
    """Rows [t0, t1) of the dedispersed segment, formed without the rest (for
    sampling single images of large segments).  A pulse arriving at t* + d[c]
    in channel c lands at row t* - t0 in every channel whose arrival is inside
    the segment; rows past T - d[c] hold zeros (delays equal to and beyond T
    included); the window equals the same rows of the whole-segment
    dedispersion; float16 storage is widened exactly."""
    T, B, C, P = 11, 2, 6, 2
    d = np.array([14, 11, 10, 5, 1, 0], np.int32)
    ts = 3
    imp = np.zeros((T, B, C, P), np.complex128)
    for c in range(C):
        if ts + d[c] < T:
            imp[ts + d[c], :, c, :] = 1.0 - 0.5j
    ones = np.ones((T, B, C, P), np.complex128)
    rng = np.random.default_rng(33)
    vis = rng.standard_normal((T, B, C, P)) + 1j * rng.standard_normal((T, B, C, P))
    whole = o.dedisperse(vis, d)
    for t0, t1 in [(0, T), (0, 1), (3, 4), (2, 9), (T - 1, T), (4, 7)]:
        win = o.dedisperse_window(imp, d, t0, t1)
        assert win.shape == (t1 - t0, B, C, P), win.shape
        for c in range(C):
            col = win[:, 0, c, 0]
            if t0 <= ts < t1 and ts + d[c] < T:
                assert col[ts - t0] == 1.0 - 0.5j and np.count_nonzero(col) == 1, (t0, t1, c, col)
            else:
                assert np.count_nonzero(col) == 0, (t0, t1, c, col)
        filled = o.dedisperse_window(ones, d, t0, t1)[:, 1, :, 1]
        for c in range(C):
            n_in = max(0, min(t1, T - int(d[c])) - t0)
            assert (filled[:n_in, c] == 1.0).all() and (filled[n_in:, c] == 0.0).all(), (t0, t1, c)
        assert np.array_equal(o.dedisperse_window(vis, d, t0, t1), whole[t0:t1])
    v16 = np.zeros((T, B, C, P, 2), np.float16)
    v16[..., 0] = vis.real.astype(np.float16)
    v16[..., 1] = vis.imag.astype(np.float16)
    want = o.dedisperse(v16[..., 0].astype(np.float64) + 1j * v16[..., 1].astype(np.float64), d)
    assert np.array_equal(o.dedisperse_window(v16, d, 2, 9), want[2:9])


def check_image_at(o):
    """One image of the search, formed from its own window of integrations,
    is bit for bit the image the whole-segment search forms for that (DM
    trial, width, integration): every key, trials whose delays reach past the
    segment and the last box of the widest width included."""
    plan, uvw, f = _window_case(o)
    rng = np.random.default_rng(34)
    vis = rng.standard_normal((13, uvw.shape[0], 10, 2)) + 1j * rng.standard_normal((13, uvw.shape[0], 10, 2))
    d = plan.delays
    assert d[2].max() > 13 and 0 < d[1].max() < 13 and (d[2] == 0).any(), d
    _, _, images = o.search(vis, plan, keep_images=True)
    assert len(images) == 3 * (13 + 6 + 3)
    for (i, j, k), img in images.items():
        got = o.image_at(vis, plan, i, j, k)
        assert np.array_equal(got, img), (i, j, k, float(np.max(np.abs(got - img))))


def check_is_marginal(o):
    """The margin guard on hand-built images: an S/N within 10 tol (relative)
    of the threshold, or top two pixels within 10 tol (relative) of each
    other, is marginal; clear cases are not; an all-zero image is."""
    def img_with(top, second):
        a = np.zeros((8, 8))
        a[:] = np.linspace(-0.5, 0.5, 64).reshape(8, 8)
        a[2, 5] = top
        a[6, 1] = second
        return a
    tol = 1e-5
    assert not o.is_marginal(img_with(1.0, 0.9), 7.0, 6.0, tol)
    # S/N side: |snr - thr| = 3e-4 < 10 tol thr = 6e-4; 9e-4 is not
    assert o.is_marginal(img_with(1.0, 0.9), 6.0003, 6.0, tol)
    assert o.is_marginal(img_with(1.0, 0.9), 5.9997, 6.0, tol)
    assert not o.is_marginal(img_with(1.0, 0.9), 6.0009, 6.0, tol)
    # gap side: a relative gap of 5e-5 is under 10 tol; 2e-4 is not
    assert o.is_marginal(img_with(1.0, 1.0 - 5e-5), 7.0, 6.0, tol)
    assert not o.is_marginal(img_with(1.0, 1.0 - 2e-4), 7.0, 6.0, tol)
    # relative to the top pixel: the same gap at 100x the scale is the same
    assert o.is_marginal(img_with(100.0, 100.0 - 5e-3), 7.0, 6.0, tol)
    assert not o.is_marginal(img_with(100.0, 100.0 - 2e-2), 7.0, 6.0, tol)
    # a tied top pair is marginal; a lone top pixel far above the rest is not
    assert o.is_marginal(img_with(1.0, 1.0), 7.0, 6.0, tol)
    assert o.is_marginal(np.zeros((8, 8)), 0.0, 6.0, tol)
    # the looser tolerance of float16 storage widens both sides
    assert o.is_marginal(img_with(1.0, 1.0 - 2e-2), 7.0, 6.0, 3e-3)
    assert o.is_marginal(img_with(1.0, 0.5), 6.1, 6.0, 3e-3)


# ---------------------------------------------------------------- mean subtraction

def check_subtract_mean(o):
    """Closed forms of subtracting the segment's time mean (section 3.1): a
    constant source vanishes; an impulse A at t0 in an empty segment leaves
    A (1 - 1/T) at t0 and -A/T elsewhere; the output's time mean is zero;
    adding a constant to every integration changes nothing."""
    rng = np.random.default_rng(5)
    T, B, C, P = 12, 3, 5, 2
    const = rng.standard_normal((B, C, P)) + 1j * rng.standard_normal((B, C, P))
    out = o.subtract_mean(np.broadcast_to(const, (T, B, C, P)))
    assert np.max(np.abs(out)) < 1e-12, "a constant source must vanish"
    imp = np.zeros((T, B, C, P), np.complex128)
    imp[4, 1, 2, 0] = 3.0 - 2.0j
    out = o.subtract_mean(imp)
    assert abs(out[4, 1, 2, 0] - (3.0 - 2.0j) * (1 - 1 / T)) < 1e-12
    assert abs(out[7, 1, 2, 0] + (3.0 - 2.0j) / T) < 1e-12
    assert np.max(np.abs(out[:, 0])) < 1e-15, "other baselines untouched"
    x = rng.standard_normal((T, B, C, P)) + 1j * rng.standard_normal((T, B, C, P))
    y = o.subtract_mean(x)
    assert np.max(np.abs(y.sum(axis=0))) < 1e-12
    assert np.max(np.abs(o.subtract_mean(x + const[None]) - y)) < 1e-12

# ---------------------------------------------------------------- mock injection

def _mock(**kw):
    m = dict(dm=0.0, t0=0.0, width=1.0, l=0.0, m=0.0, amp=1.0)
    m.update(kw)
    return m


def _one_baseline(u_m=0.0, v_m=0.0):
    return np.array([[u_m, v_m, 0.0]])


def check_inject_boxcar(o):
    """A DM 0 mock at the phase centre starting on an integration boundary
    adds exactly amp to `width` whole integrations of every baseline,
    channel and polarisation, and nothing elsewhere."""
    T, B, C, P = 10, 3, 4, 2
    uvw = np.array([[10.0, -3.0, 0.0], [0.0, 7.5, 0.0], [-120.0, 44.0, 0.0]])
    f = centres(1.0, 2.0, C)
    vis = np.zeros((T, B, C, P), np.complex64)
    out = o.inject(vis, [_mock(t0=3.0, width=2.0, amp=0.5)], f, uvw, 0.005, 4.15e-3)
    want = np.zeros((T, B, C, P), np.complex64)
    want[3:5] = 0.5
    assert out.dtype == np.complex64 and np.array_equal(out, want)


def check_inject_fractional(o):
    """Fractional start and width split the flux by overlap: [2.25, 3.75)
    puts 3/4 of amp in integrations 2 and 3; [5.5, 8.0) puts 1/2, 1, 1."""
    C = 2
    f = centres(1.0, 2.0, C)
    vis = np.zeros((10, 1, C, 1), np.complex64)
    out = o.inject(vis, [_mock(t0=2.25, width=1.5, amp=2.0)], f, _one_baseline(), 0.01, 4.15e-3)
    got = out[:, 0, 0, 0].real
    want = np.zeros(10)
    want[2] = want[3] = 1.5
    assert np.array_equal(got, want), got
    out = o.inject(vis, [_mock(t0=5.5, width=2.5, amp=1.0)], f, _one_baseline(), 0.01, 4.15e-3)
    got = out[:, 0, 1, 0].real
    want = np.zeros(10)
    want[5], want[6], want[7] = 0.5, 1.0, 1.0
    assert np.array_equal(got, want), got


def check_inject_dispersion(o):
    """The sweep follows the printed law (4.15 ms DM / nu^2, section 2.1
    footnote), relative to the highest channel: channels at 1 GHz and 2 GHz,
    DM 10, 1 ms integrations: the 1 GHz channel arrives 31.125 ms after the
    2 GHz one, so a width-1 pulse at t0 = 4 lands in integrations 35 and 36
    (7/8 and 1/8 of its flux) at 1 GHz and in integration 4 at 2 GHz."""
    k = paper_values()["dispersion_law"]["delay_ms_per_dm_at_1ghz"] * 1e-3
    f = np.array([1.0, 2.0])
    vis = np.zeros((48, 1, 2, 1), np.complex64)
    out = o.inject(vis, [_mock(dm=10.0, t0=4.0, width=1.0, amp=1.0)], f, _one_baseline(), 1e-3, k)
    lo = out[:, 0, 0, 0].real.astype(np.float64)
    hi = out[:, 0, 1, 0].real.astype(np.float64)
    assert np.nonzero(hi)[0].tolist() == [4] and hi[4] == 1.0, hi
    assert np.nonzero(lo)[0].tolist() == [35, 36], np.nonzero(lo)
    assert abs(lo[35] - 0.875) < 1e-6 and abs(lo[36] - 0.125) < 1e-6, lo[35:37]


def check_inject_phase(o):
    """Visibility of a point source: amp exp(-2 pi i (u l + v m)), u and v in
    wavelengths.  A baseline of c / 1 GHz metres east is one wavelength at
    1 GHz: l = 1/4 gives -i amp, l = 1/8 gives amp (1 - i)/sqrt(2); a north
    baseline with m = -1/4 gives +i amp."""
    lam = 299792458.0 / 1e9
    f = np.array([1.0])
    vis = np.zeros((2, 1, 1, 2), np.complex64)
    for uvw, l, m, want in [(_one_baseline(u_m=lam), 0.25, 0.0, -1j),
                            (_one_baseline(u_m=lam), 0.125, 0.0, (1 - 1j) / math.sqrt(2)),
                            (_one_baseline(v_m=lam), 0.0, -0.25, 1j),
                            (_one_baseline(u_m=2 * lam, v_m=lam), 0.125, 0.25, -1.0)]:
        out = o.inject(vis, [_mock(l=l, m=m, amp=3.0)], f, uvw, 0.005, 4.15e-3)
        assert np.max(np.abs(out[0, 0, 0, :] - 3.0 * want)) < 1e-6, (l, m, out[0, 0, 0])
        assert np.max(np.abs(out[1])) == 0.0


def check_inject_flux(o):
    """Flux conservation: a mock wholly inside the segment adds amp * width
    times its phasor, summed over time, in every (baseline, channel); the
    phasor has modulus amp regardless of frequency."""
    rng = np.random.default_rng(11)
    T, C = 64, 16
    uvw = np.column_stack([rng.uniform(-800, 800, 5), rng.uniform(-800, 800, 5), np.zeros(5)])
    f = centres(1.0, 2.0, C)
    mk = _mock(dm=37.3, t0=6.3, width=3.7, l=0.004, m=-0.007, amp=1.0)
    vis = np.zeros((T, 5, C, 1), np.complex128)
    t = np.arange(T)[:, None, None]
    sig = o.mock_signal(mk, t, np.arange(5)[None, :, None], np.arange(C)[None, None, :], f, uvw,
                        0.005, 4.15e-3)
    tot = sig.sum(axis=0)
    assert np.max(np.abs(np.abs(tot) - 3.7)) < 1e-12, np.abs(tot)
    # the sum over time is width times the single-integration phasor
    one = o.mock_signal(dict(mk, dm=0.0, t0=0.0, width=1.0), np.zeros((1, 1, 1), int),
                        np.arange(5)[None, :, None], np.arange(C)[None, None, :], f, uvw, 0.005, 4.15e-3)
    assert np.max(np.abs(tot - 3.7 * one[0])) < 1e-12
    del vis


def check_inject_images_at_pixel(o):
    """A mock placed at pixel (X0, Y0) (l = (X0 - N/2)/(N du), likewise m)
    images at (X0, Y0) with a peak close to its amplitude: injection and
    imaging follow one sign convention."""
    from rfgen import synth
    pos = synth.y_array_positions(27)
    uvw = synth.baseline_uvw(pos)
    f = centres(1.0, 2.0, 32)
    N = 128
    du = synth.default_cell_size(uvw, f, N)
    iu, iv = o.cell_table(uvw, f, du, du)
    valid = o.valid_cells(iu, iv, N)
    W = int(np.count_nonzero(valid))
    for X0, Y0 in [(N // 2 + 5, N // 2 - 3), (N // 2 - 7, N // 2 + 6)]:
        l, m = (X0 - N / 2) / (N * du), (Y0 - N / 2) / (N * du)
        vis = np.zeros((1, uvw.shape[0], 32, 2), np.complex64)
        out = o.inject(vis, [_mock(l=l, m=m, amp=0.8)], f, uvw, 0.005, 4.15e-3)
        img = o.image(o.grid(o.stokes_i(o.as_complex(out[0])), iu, iv, valid, N), W)
        peak, x, y, _, _ = o.image_stats(img)
        assert (x, y) == (X0, Y0), (x, y, X0, Y0)
        assert 0.98 * 0.8 <= peak <= 0.8 * (1 + 1e-6), peak


def _exact_round(x, mant_bits, emin):
    """Round-to-nearest-even of the float x to a binary format with
    mant_bits stored fraction bits and minimum normal exponent emin, by exact
    rational arithmetic (brute force on the rounding definition)."""
    from fractions import Fraction
    if x == 0.0:
        return 0.0
    X = Fraction(abs(x))
    e = 0
    while Fraction(2) ** e > X:
        e -= 1
    while Fraction(2) ** (e + 1) <= X:
        e += 1
    q = Fraction(2) ** (max(e, emin) - mant_bits)
    n = X / q
    fl = n.numerator // n.denominator
    r = n - fl
    if r > Fraction(1, 2) or (r == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return math.copysign(float(fl * q), x)


def check_inject_storage_rounding(o):
    """A mock's float64 sum with the stored value is rounded once, to nearest
    even, to the storage type: exact ties and values a hair off a tie go the
    way the rounding definition says, for float16 and float32 storage."""
    f = np.array([1.0])
    for storage, mant, emin, old in [("cf16", 10, -14, 1.0), ("cf16", 10, -14, -0.3330078125),
                                     ("cf32", 23, -126, 1.0), ("cf32", 23, -126, 0.1)]:
        dt = np.float16 if storage == "cf16" else np.float32
        ulp = float(np.spacing(dt(old)))
        for d in (0.5 * ulp, 1.5 * ulp, 0.5 * ulp * (1 + 2.0 ** -30), 0.5 * ulp * (1 - 2.0 ** -30), 0.25 * ulp):
            if storage == "cf16":
                vis = np.zeros((1, 1, 1, 1, 2), np.float16)
                vis[..., 0] = old
                out = o.inject(vis, [_mock(amp=d)], f, _one_baseline(), 0.005, 4.15e-3)
                got = float(out[0, 0, 0, 0, 0])
                assert out.dtype == np.float16
            else:
                vis = np.full((1, 1, 1, 1), old, np.complex64)
                out = o.inject(vis, [_mock(amp=d)], f, _one_baseline(), 0.005, 4.15e-3)
                got = float(out[0, 0, 0, 0].real)
            want = _exact_round(float(dt(old)) + d, mant, emin)
            assert got == want, (storage, old, d, got, want)


def check_inject_order(o):
    """Two mocks are added one after the other, each rounded to the storage:
    in float16, 1 + 2^-11 + 2^-11 is 1 (each addition is a tie to even),
    not 1 + 2^-10."""
    f = np.array([1.0])
    vis = np.zeros((1, 1, 1, 1, 2), np.float16)
    vis[..., 0] = 1.0
    out = o.inject(vis, [_mock(amp=2.0 ** -11), _mock(amp=2.0 ** -11)], f, _one_baseline(), 0.005, 4.15e-3)
    assert float(out[0, 0, 0, 0, 0]) == 1.0


# ---------------------------------------------------------------- second-tier products

def check_cutout(o):
    """The cutout is the image rolled so the candidate pixel sits at (half,
    half) (numpy.roll as the library special case), wrapping at every edge."""
    rng = np.random.default_rng(2)
    img = rng.standard_normal((32, 32))
    for x, y, h in [(10, 20, 4), (0, 31, 5), (31, 0, 16), (16, 16, 1)]:
        cut = o.candidate_cutout(img, x, y, h)
        want = np.roll(img, (h - y, h - x), axis=(0, 1))[:2 * h, :2 * h]
        assert cut.shape == (2 * h, 2 * h) and np.array_equal(cut, want), (x, y, h)
        assert cut[h, h] == img[y, x]


def _spectrum_case(o):
    from rfgen import synth
    uvw = synth.baseline_uvw(synth.y_array_positions(10))
    f = centres(1.0, 2.0, 12)
    N = 64
    du = 0.6 * synth.default_cell_size(uvw, f, N)   # some pairs fall off the grid
    plan = o.Plan(f, uvw, 0.005, np.array([0.0, 40.0]), [1, 2], N, du, du, nint=20)
    return plan, uvw, f, N, du


def check_spectrum_splits_pixel(o):
    """Weighted by the channel's gridded baselines and divided by W, a
    spectrum row adds up to the candidate pixel of that row's image: the
    spectrum splits the image pixel by channel."""
    plan, uvw, f, N, du = _spectrum_case(o)
    n_c = plan.valid.sum(axis=0)
    assert n_c.min() < n_c.max() and n_c.min() < uvw.shape[0], "the case must drop some pairs"
    rng = np.random.default_rng(8)
    vis = rng.standard_normal((20, uvw.shape[0], 12, 2)) + 1j * rng.standard_normal((20, uvw.shape[0], 12, 2))
    for i, j, k, x, y in [(1, 1, 4, 37, 25), (0, 0, 19, 3, 60), (1, 0, 0, 32, 32)]:
        spec = o.candidate_spectrum(vis, plan, i, j, k, x, y, 5)
        K = 20 // plan.widths[j]
        for s in range(5):
            kk = k - 2 + s
            got = float((spec[s] * n_c).sum() / plan.W)
            if 0 <= kk < K:
                want = o.image_at(vis, plan, i, j, kk)[y, x]
                assert abs(got - want) < 1e-12, (i, j, k, s, got, want)
            else:
                assert np.all(spec[s] == 0.0)


def check_spectrum_point_source(o):
    """A steady source at the phase centre (V = A everywhere) has the
    spectrum A in every channel with a gridded baseline, in every row inside
    the segment, toward pixel (N/2, N/2)."""
    plan, uvw, f, N, du = _spectrum_case(o)
    vis = np.full((20, uvw.shape[0], 12, 2), 0.7 - 0.2j)
    spec = o.candidate_spectrum(vis, plan, 0, 1, 9, N // 2, N // 2, 4)
    n_c = plan.valid.sum(axis=0)
    assert np.max(np.abs(spec[:3][:, n_c > 0] - 0.7)) < 1e-12
    assert np.all(spec[3] == 0.0), "row k + 1 = 10 is past the 10 width-2 integrations"


def check_spectrum_pulse(o):
    """A noise-free pulse from pixel (x0, y0) at DM 0 in integration 6: toward
    that pixel its row holds nearly the full flux in every gridded channel
    (nearest-cell phase error <= pi |dx| / N), every other row is zero; toward
    the mirrored pixel the flux is not there."""
    from rfgen import synth
    plan, uvw, f, N, du = _spectrum_case(o)
    x0, y0 = N // 2 + 3, N // 2 - 2
    l, m = synth.pixel_to_lm(x0, y0, N, du, du)
    vis = np.zeros((20, uvw.shape[0], 12, 2), np.complex128)
    synth.add_pulse(vis, uvw, f, 0.005, 4.15e-3, 0.0, 6, 1, l, m, 0.5)
    spec = o.candidate_spectrum(vis, plan, 0, 0, 6, x0, y0, 3)
    n_c = plan.valid.sum(axis=0)
    assert np.all(spec[0] == 0) and np.all(spec[2] == 0)
    row = spec[1][n_c > 0]
    assert np.all(row > 0.5 * 0.95) and np.all(row <= 0.5 + 1e-12), row
    away = o.candidate_spectrum(vis, plan, 0, 0, 6, N - x0, N - y0, 3)[1][n_c > 0]
    assert np.mean(away) < 0.5 * 0.5, away


# ---------------------------------------------------------------- periodicity search

def check_time_spectrum(o):
    """The fluctuation spectrum is the 1/T-normalised forward DFT along time:
    brute force on a short series; a steady source sits in bin 0; a comb of
    pulses every P integrations has A / P in every multiple of T / P and
    nothing else."""
    rng = np.random.default_rng(4)
    T = 12
    x = rng.standard_normal((T, 3)) + 1j * rng.standard_normal((T, 3))
    F = o.time_spectrum(x)
    for f in range(T):
        want = sum(x[t] * np.exp(-2j * np.pi * f * t / T) for t in range(T)) / T
        assert np.max(np.abs(F[f] - want)) < 1e-12, f
    F = o.time_spectrum(np.full((16, 2), 0.4 - 0.1j))
    assert np.max(np.abs(F[0] - (0.4 - 0.1j))) < 1e-15 and np.max(np.abs(F[1:])) < 1e-15
    comb = np.zeros((24, 1), complex)
    comb[3::6] = 1.5
    F = o.time_spectrum(comb)
    for f in range(24):
        want = 1.5 / 6 if f % 4 == 0 else 0.0
        assert abs(abs(F[f, 0]) - want) < 1e-14, f


def check_complex_image(o):
    """The complex image: brute-force inverse DFT on a small grid, and its
    real and imaginary parts are the real images of G and -iG."""
    rng = np.random.default_rng(6)
    N = 16
    G = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    I = o.complex_image(G, 7)
    ky, kx = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    for Y, X in [(0, 0), (8, 8), (3, 12), (15, 1)]:
        want = np.sum(G * np.exp(2j * np.pi * (kx * (X - N // 2) + ky * (Y - N // 2)) / N)) / 7
        assert abs(I[Y, X] - want) < 1e-12, (X, Y)
    assert np.max(np.abs(I.real - o.image(G, 7))) < 1e-12
    assert np.max(np.abs(I.imag - o.image(-1j * G, 7))) < 1e-12


def check_amplitude_stats(o):
    """sqrt(2 ln 2) is the median of a unit Rayleigh amplitude (scipy as the
    library special case); the estimate recovers the per-quadrature noise of
    a complex Gaussian field; ties go to the lowest index."""
    from scipy import stats as sst
    assert abs(o.RAYLEIGH_MEDIAN - sst.rayleigh.median()) < 1e-12
    rng = np.random.default_rng(12)
    A = np.abs(0.3 * (rng.standard_normal((512, 512)) + 1j * rng.standard_normal((512, 512))))
    peak, x, y, sigma, snr = o.amplitude_stats(A)
    assert abs(sigma / 0.3 - 1) < 0.01, sigma
    assert peak == A.max() and A[y, x] == peak
    B = np.ones((8, 8))
    B[5, 2] = B[2, 6] = 3.0
    assert o.amplitude_stats(B)[1:3] == (6, 2)
    assert o.amplitude_stats(np.zeros((4, 4)))[4] == 0.0


def _periodic_case(o, T=32, dms=(0.0, 40.0)):
    from rfgen import synth
    uvw = synth.baseline_uvw(synth.y_array_positions(10))
    f = centres(1.0, 2.0, 16)
    N = 64
    du = synth.default_cell_size(uvw, f, N)
    plan = o.Plan(f, uvw, 0.005, np.array(dms), [1], N, du, du, nint=T)
    return plan, uvw, f, N, du


def check_periodic_pulse_train(o):
    """A noise-free train of pulses every P = 8 integrations from the phase
    centre, with different flux in the two polarisations, at DM 0: every
    harmonic f = 4, 8, 12, 16 images to the Stokes I amplitude over P at
    pixel (N/2, N/2); the frequencies searched are 1 .. T/2."""
    plan, uvw, f, N, du = _periodic_case(o)
    vis = np.zeros((32, uvw.shape[0], 16, 2), complex)
    vis[2::8, :, :, 0] = 1.2
    vis[2::8, :, :, 1] = 0.4
    stats, cands, _ = o.periodic_search(vis, plan)
    assert sorted({k[1] for k in stats}) == list(range(1, 17))
    for fb in (4, 8, 12, 16):
        peak, x, y, sigma, snr = stats[(0, fb)]
        assert (x, y) == (N // 2, N // 2) and abs(peak - 0.8 / 8) < 1e-12, (fb, peak)
    assert stats[(0, 5)][0] < 1e-12


def check_periodic_dispersed(o):
    """A dispersed pulse train (DM 40, P = 8, from pixel (x0, y0), in
    noise) is found at its DM trial and fundamental frequency, at its pixel,
    and not at DM 0 with the same strength."""
    from rfgen import synth
    plan, uvw, f, N, du = _periodic_case(o)
    rng = np.random.default_rng(3)
    vis = 0.05 * (rng.standard_normal((32, uvw.shape[0], 16, 2)) + 1j * rng.standard_normal((32, uvw.shape[0], 16, 2)))
    x0, y0 = N // 2 + 4, N // 2 - 3
    l, m = synth.pixel_to_lm(x0, y0, N, du, du)
    for t0 in range(1, 32, 8):
        synth.add_pulse(vis, uvw, f, 0.005, 4.15e-3, 40.0, t0, 1, l, m, 1.0)
    stats, cands, _ = o.periodic_search(vis, plan)
    peak, x, y, sigma, snr = stats[(1, 4)]
    assert (x, y) == (x0, y0) and snr > 20, (x, y, snr)
    assert (1, 4, x0, y0) in [c[:4] for c in cands]
    assert stats[(0, 4)][4] < 0.6 * snr


def check_periodic_noise_sigma(o):
    """Noise only: the per-quadrature noise of a frequency's image is
    (2 T W)^-1/2 for unit complex noise per polarisation (the fluctuation
    spectrum divides by T), recovered to 5%."""
    plan, uvw, f, N, du = _periodic_case(o, T=16, dms=(0.0,))
    rng = np.random.default_rng(21)
    vis = rng.standard_normal((16, uvw.shape[0], 16, 2)) + 1j * rng.standard_normal((16, uvw.shape[0], 16, 2))
    stats, _, _ = o.periodic_search(vis, plan, select={(0, 3), (0, 7)})
    want = (2 * 16 * plan.W) ** -0.5
    for key, st in stats.items():
        assert abs(st[3] / want - 1) < 0.05, (key, st[3], want)


# ---------------------------------------------------------------- layout

def check_table1_layout():
    """Table 1 rates follow from 351 baselines x channels x 2 pols x 8-byte
    complex64 per integration: the layout the search consumes."""
    t = paper_values()["table1"]
    for row in t["rows"]:
        rate = t["baselines"] * row["channels"] * t["npol"] * np.dtype(np.complex64).itemsize / (row["tint_ms"] * 1e-3) / 1e6
        assert abs(rate / row["rate_mb_s"] - 1) < 0.05, (row, rate)


ALL_CHECKS = [
    check_delay_law, check_delay_properties, check_delay_hand_values, check_delay_rounding,
    check_sweep_example, check_cells, check_dedisperse, check_resample, check_stokes,
    check_grid, check_image_dft, check_image_single_cell, check_image_point_source,
    check_image_parseval, check_image_offset_source, check_image_linear, check_stats,
    check_noise_sigma, check_subtract_mean, check_inject_boxcar, check_inject_fractional,
    check_inject_dispersion, check_inject_phase, check_inject_flux, check_inject_images_at_pixel,
    check_inject_storage_rounding, check_inject_order, check_cutout, check_spectrum_splits_pixel,
    check_spectrum_point_source, check_spectrum_pulse, check_time_spectrum, check_complex_image,
    check_amplitude_stats, check_periodic_pulse_train, check_periodic_dispersed,
    check_periodic_noise_sigma, check_dedisperse_window, check_image_at, check_is_marginal,
]
