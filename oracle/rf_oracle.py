"""CPU oracle for the realfast search hot path (test infrastructure only).

THIS IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it.  The product path (the HIP library
and its Python binding) never calls it and shares no code with it.

It is a plain, slow, obviously correct numpy implementation in float64 /
complex128 of what the search computes, step by step, in the order of the
search loop of Law et al. 2018 (section 3.1 and the caption of Figure 2:
loops over trial dispersion measures and sampling times; each dedispersed,
time-resampled Stokes I image is thresholded on S/N).  The paper states the
method in words only; where it is silent the readings used are written next
to the function that needs them and listed together in the design notes.

Functions and the passages they follow:
  delay_table   section 2.1 footnote (cold-plasma delay 4.15 ms DM / nu^2)
  cell_table    sections 2.2 and 3.1 (visibility-domain processing, FFT imaging)
  dedisperse    section 2.2 (dedispersion in the visibility domain), 3.1
  resample      section 2.2 (matched filters over pulse widths), Figure 2
                (loop over trial sampling times)
  stokes_i      section 3.1 (a Stokes I image per DM and width)
  grid          section 2.2 item 3 (FFT imaging); gridding itself unstated
  image         section 3.1 / 3.2 (2-D FFT imaging)
  image_stats   section 3.1 (point sources above an S/N threshold, ~6 sigma)
  search        section 3.1 / Figure 2 (the whole loop)
  subtract_mean section 3.1 (mean visibility subtracted on timescales below
                the fringe rate), 3.2 (segments of about that length)
  mock_signal   section 3.3 (mock transients inserted into the data to
                measure the search's efficiency), 2.1 footnote (their sweep)
  inject(_at)   the same, applied to stored visibilities with the storage
                rounding (one rounding per mock, mocks in order)
  time_spectrum, complex_image, amplitude_stats, periodic_search
                section 3.1 footnote (a segment transformed to frequencies
                along time, each frequency imaged), Figure 2 caption (a
                modification of the innermost loop)
  candidate_cutout, candidate_spectrum
                section 3.1 (a second, higher threshold, ~7 sigma, selects
                candidates for visualisation), 3.3 (the candidate's image
                and spectrum)
  dedisperse_window, image_at
                the same dedispersion and imaging restricted to the
                integrations of one image (section 2.2, 3.1), for sampling
                single images of segments too large to search whole
  is_marginal   the parity margin guard (not a step of the method): images
                whose S/N or top-two pixel gap lie within 10 tol of a
                decision may flip between two correct float implementations

Parity pins live in tests/test_oracle_*.py; every function above is pinned
there against closed forms, brute force, library special cases or the values
the paper prints.  Readings that no paper value can pin (edge handling,
resampling kind, gridding kernel, cell size, sigma estimator) are marked
"parity unpinned" below: only their internal consistency is checked.
"""
import math

import numpy as np

C_LIGHT = 299792458.0          # m/s
MAD_TO_SIGMA = 1.4826          # 1 / Phi^-1(3/4): MAD of a Gaussian -> sigma


class Plan:
    """Everything the search needs besides the visibilities (the pipeline
    state of section 3.2: metadata plus preferences define it uniquely)."""

    def __init__(self, freq_ghz, uvw_m, tint_s, dms, widths, npix, du, dv,
                 kdm=4.15e-3, threshold=6.0, t_begin=0, t_end=None, nint=None):
        self.freq = np.asarray(freq_ghz, dtype=np.float64)
        self.uvw = np.asarray(uvw_m, dtype=np.float64)
        self.tint = float(tint_s)
        self.dms = np.asarray(dms, dtype=np.float64)
        self.widths = [int(w) for w in widths]
        self.npix = int(npix)
        self.du = float(du)
        self.dv = float(dv)
        self.kdm = float(kdm)
        self.threshold = float(threshold)
        self.nint = nint
        self.t_begin = int(t_begin)
        self.t_end = int(t_end) if t_end is not None else (nint if nint is not None else 1 << 30)
        self.delays = delay_table(self.freq, self.dms, self.tint, self.kdm)
        self.iu, self.iv = cell_table(self.uvw, self.freq, self.du, self.dv)
        self.valid = valid_cells(self.iu, self.iv, self.npix)
        self.W = int(np.count_nonzero(self.valid))


def delay_table(freq_ghz, dms, tint_s, kdm):
    """Integer dispersion delay, in integrations, of every (DM trial, channel).

    Cold-plasma law (section 2.1 footnote): tau = K DM / nu^2, K = 4.15 ms
    GHz^2 per pc cm^-3.  Readings: delays are relative to the highest channel
    (which never moves, so every delay is >= 0); the delay in seconds is
    rounded to whole integrations with round-half-even.  Each product, sum and
    quotient below is one IEEE float64 operation in exactly this order:
        d = rint(((K * DM) * (1/(nu*nu) - 1/(nu_ref*nu_ref))) / t_int)
    Returns int32 [ndm][nchan].
    """
    f = np.asarray(freq_ghz, dtype=np.float64)
    dm = np.asarray(dms, dtype=np.float64)
    nu_ref = np.max(f)
    inv = 1.0 / (f * f)
    inv_ref = 1.0 / (nu_ref * nu_ref)
    lag = (kdm * dm)[:, None] * (inv - inv_ref)[None, :]
    return np.rint(lag / tint_s).astype(np.int32)


def cell_table(uvw_m, freq_ghz, du, dv):
    """Nearest uv cell of every (baseline, channel): (iu, iv) int32 [nbl][nchan].

    u in wavelengths is u_m * nu / c; the cell is rint(u_lambda / du) (round
    half even), each step one float64 operation in this order:
        iu = rint(((u_m * (nu_ghz * 1e9)) / c) / du)
    and likewise for v.  Reading (gridding is not described in the paper):
    nearest-cell assignment with no convolution kernel, w ignored.
    """
    f_hz = np.asarray(freq_ghz, dtype=np.float64) * 1e9
    u = np.asarray(uvw_m, dtype=np.float64)[:, 0]
    v = np.asarray(uvw_m, dtype=np.float64)[:, 1]
    iu = np.rint(((u[:, None] * f_hz[None, :]) / C_LIGHT) / du).astype(np.int32)
    iv = np.rint(((v[:, None] * f_hz[None, :]) / C_LIGHT) / dv).astype(np.int32)
    return iu, iv


def valid_cells(iu, iv, npix):
    """A (baseline, channel) pair is imaged iff |iu|, |iv| <= N/2 - 1."""
    lim = npix // 2 - 1
    return (np.abs(iu) <= lim) & (np.abs(iv) <= lim)


def subtract_mean(vis):
    """Mean-visibility subtraction over one segment (section 3.1: the mean
    visibility in time is subtracted on timescales shorter than the fringe
    rate, which removes constant sources; section 3.2: segments are about
    that long).

    out[t, b, c, p] = vis[t, b, c, p] - (1/T) sum_t' vis[t', b, c, p].
    Reading: the mean is taken over the whole segment, per baseline, channel
    and polarisation, and subtracted from every integration of it (the paper
    gives the time scale, not the window).  complex128.
    """
    v = np.asarray(vis).astype(np.complex128)
    T = v.shape[0]
    total = np.zeros(v.shape[1:], dtype=np.complex128)
    for t in range(T):
        total += v[t]
    return v - (total / T)[None]


def dedisperse(vis, delay_row):
    """Visibility-domain dedispersion for one DM trial (section 2.2).

    out[t, b, c, p] = vis[t + d[c], b, c, p] if t + d[c] < T, else 0.
    Reading (parity unpinned: the paper handles edges with overlapping
    segments, section 3.2): samples shifted in from past the end of the
    segment are zero.  Pure data movement; returns complex128.
    """
    vis = np.asarray(vis)
    T = vis.shape[0]
    out = np.zeros(vis.shape, dtype=np.complex128)
    for c, d in enumerate(np.asarray(delay_row)):
        d = int(d)
        if d < T:
            out[: T - d, :, c, :] = vis[d:, :, c, :]
    return out


def resample(x, w):
    """Boxcar resampling to sampling time w (Figure 2 loop over sampling time).

    out[k] = (sum_{j<w} x[k w + j]) / w for k < floor(T / w); the remainder is
    dropped.  Reading (parity unpinned): a decimating mean, not a sliding one.
    """
    T = x.shape[0]
    K = T // w
    acc = np.zeros((K,) + x.shape[1:], dtype=np.complex128)
    for j in range(w):
        acc += x[j: K * w: w]
    return acc / w


def stokes_i(v):
    """Stokes I from the polarisation axis (last): mean of the two
    polarisations, or the single one when npol == 1 (section 3.1)."""
    if v.shape[-1] == 1:
        return v[..., 0].astype(np.complex128)
    return (v[..., 0] + v[..., 1]) / 2.0


def grid(vi, iu, iv, valid, npix):
    """Natural-weight nearest-cell gridding of one Stokes I sample set.

    G[iv mod N, iu mod N] += V_I[b, c] over valid pairs; complex128 [N][N].
    """
    G = np.zeros((npix, npix), dtype=np.complex128)
    np.add.at(G, (np.mod(iv[valid], npix), np.mod(iu[valid], npix)), vi[valid])
    return G


def image(G, W):
    """Stokes I image from a grid (2-D FFT imaging, section 3.2).

    img[Y, X] = (1/W) Re sum_{iu,iv} G[iv, iu] exp(+2 pi i (iu (X - N/2) +
    iv (Y - N/2)) / N), i.e. the unnormalised inverse DFT, shifted so the
    phase centre is pixel (N/2, N/2), divided by the number of gridded
    samples W.  numpy's inverse FFT is the library step.
    """
    N = G.shape[0]
    F = np.fft.ifft2(G) * (N * N)
    return np.fft.fftshift(F).real / W


def image_stats(img):
    """(peak, X, Y, sigma, snr) of one image (section 3.1 thresholding).

    peak is the signed maximum; ties go to the lowest Y*N + X.  Reading
    (parity unpinned): sigma = 1.4826 * lower median of |img| (a median
    absolute deviation about zero; the image mean is zero because the
    zero-spacing cell is empty).  snr = peak / sigma, 0 when sigma == 0.
    """
    N = img.shape[1]
    flat = img.ravel()
    idx = int(np.argmax(flat))
    peak = float(flat[idx])
    a = np.abs(flat)
    k = (a.size - 1) // 2
    med = float(np.partition(a, k)[k])
    sigma = MAD_TO_SIGMA * med
    snr = peak / sigma if sigma != 0.0 else 0.0
    return peak, idx % N, idx // N, sigma, snr


def make_image(vis_int, plan):
    """Image of one resampled integration vis_int [nbl][nchan][npol]."""
    vi = stokes_i(vis_int)
    G = grid(vi, plan.iu, plan.iv, plan.valid, plan.npix)
    return image(G, plan.W)


def search(vis, plan, select=None, keep_images=False):
    """The search loop of Figure 2: for each DM trial dedisperse, for each
    sampling time resample, image every integration and threshold it.

    vis: complex [T][nbl][nchan][npol] (or float16 [..., 2] storage).
    select: optional set of (dm_idx, width_idx, k) to image; default all.
    Returns (stats, candidates, images):
      stats: dict (i, j, k) -> (peak, X, Y, sigma, snr)
      candidates: list of (i, j, t_int, X, Y, snr, peak, sigma) for images
        with snr > threshold and t_begin <= k*w < t_end, in (i, j, k) order.
    """
    vis = as_complex(vis)
    T = vis.shape[0]
    stats, cands, images = {}, [], {}
    dm_set = range(len(plan.dms)) if select is None else sorted({s[0] for s in select})
    for i in dm_set:
        dd = dedisperse(vis, plan.delays[i])
        for j, w in enumerate(plan.widths):
            if select is not None and not any(s[0] == i and s[1] == j for s in select):
                continue
            rs = resample(dd, w)
            for k in range(T // w):
                if select is not None and (i, j, k) not in select:
                    continue
                img = make_image(rs[k], plan)
                st = image_stats(img)
                stats[(i, j, k)] = st
                if keep_images:
                    images[(i, j, k)] = img
                peak, x, y, sigma, snr = st
                t_int = k * w
                if snr > plan.threshold and plan.t_begin <= t_int < plan.t_end:
                    cands.append((i, j, t_int, x, y, snr, peak, sigma))
    return stats, cands, images


def as_complex(vis):
    """complex64/complex128 arrays pass through; float16 [..., 2] storage is
    widened exactly to complex128."""
    vis = np.asarray(vis)
    if np.iscomplexobj(vis):
        return vis
    if vis.dtype == np.float16 and vis.shape[-1] == 2:
        return vis[..., 0].astype(np.float64) + 1j * vis[..., 1].astype(np.float64)
    raise TypeError("visibilities must be complex or float16 [..., 2]")


def is_marginal(img, snr, threshold, tol):
    """Margin guard for candidate parity: an image whose S/N is within 10 tol
    (relative) of the threshold, or whose top two pixels are within 10 tol
    (relative) of each other, may legitimately flip between two correct
    float implementations."""
    if abs(snr - threshold) < 10 * tol * threshold:
        return True
    flat = np.sort(img.ravel())
    top, second = flat[-1], flat[-2]
    if top == 0.0:
        return True
    return (top - second) / abs(top) < 10 * tol


def dedisperse_window(vis, delay_row, t0, t1):
    """Rows [t0, t1) of dedisperse(vis, delay_row), without forming the rest
    (for sampling single images of a large segment).  float16 [..., 2]
    storage is widened exactly, slice by slice."""
    T = vis.shape[0]
    shape = (t1 - t0,) + tuple(vis.shape[1:4])
    out = np.zeros(shape, dtype=np.complex128)
    for c, d in enumerate(np.asarray(delay_row)):
        for t in range(t0, t1):
            s = t + int(d)
            if s < T:
                out[t - t0, :, c, :] = as_complex(vis[s, :, c])
    return out


def image_at(vis, plan, i, j, k):
    """The image of DM trial i, width index j, resampled integration k."""
    w = plan.widths[j]
    dd = dedisperse_window(vis, plan.delays[i], k * w, k * w + w)
    return make_image(resample(dd, w)[0], plan)


def mock_signal(mock, t, b, c, freq_ghz, uvw_m, tint_s, kdm):
    """Complex visibility of one mock transient at integration t, baseline b,
    channel c (broadcastable int arrays); complex128.

    A mock (section 3.3: mock sources inserted into calibrated data test the
    search's efficiency) is a dispersed boxcar point source, given as a dict
    with dm (pc cm^-3), t0 (arrival at the highest channel, in integrations
    from the segment start, may be fractional), width (integrations, > 0),
    l, m (direction cosines from the phase centre) and amp (flux in
    visibility units, the same in every polarisation).  In channel c it
    arrives later by the cold-plasma lag K DM (1/nu_c^2 - 1/nu_top^2)
    seconds (section 2.1 footnote); integration t holds the part of
    [start, start + width) that overlaps [t, t + 1), so the flux is
    conserved.  A point source at (l, m) has visibility
    amp exp(-2 pi i (u l + v m)) with u, v in wavelengths (the sign
    convention the imaging inverts).  Every step is one float64 operation in
    the order written:
        lag   = (K * DM) * (1/(nu*nu) - 1/(nu_top*nu_top))
        start = t0 + lag / t_int;  end = start + width
        frac  = min(t + 1, end) - max(t, start), nothing where frac <= 0
        u_l   = (u_m * (nu * 1e9)) / c;  v_l likewise
        phase = -(2 pi * (u_l * l + v_l * m))
        value = (amp * frac) * (cos(phase) + i sin(phase))
    """
    f = np.asarray(freq_ghz, dtype=np.float64)
    uvw = np.asarray(uvw_m, dtype=np.float64)
    t, b, c = np.broadcast_arrays(np.asarray(t), np.asarray(b), np.asarray(c))
    nu = f[c]
    nu_top = np.max(f)
    lag = (kdm * mock["dm"]) * (1.0 / (nu * nu) - 1.0 / (nu_top * nu_top))
    start = mock["t0"] + lag / tint_s
    end = start + mock["width"]
    tt = t.astype(np.float64)
    frac = np.minimum(tt + 1.0, end) - np.maximum(tt, start)
    frac = np.where(frac > 0.0, frac, 0.0)
    f_hz = nu * 1e9
    u_l = (uvw[b, 0] * f_hz) / C_LIGHT
    v_l = (uvw[b, 1] * f_hz) / C_LIGHT
    phase = -(2.0 * math.pi * (u_l * mock["l"] + v_l * mock["m"]))
    s = mock["amp"] * frac
    return s * np.cos(phase) + 1j * (s * np.sin(phase))


def round_storage(z, storage):
    """Round complex128 values to the visibility storage: complex64
    ("cf32"), or float16 [..., 2] ("cf16"), each part rounded to nearest
    even directly from float64."""
    z = np.asarray(z)
    if storage == "cf32":
        return z.astype(np.complex64)
    out = np.empty(z.shape + (2,), dtype=np.float16)
    out[..., 0] = z.real.astype(np.float16)
    out[..., 1] = z.imag.astype(np.float16)
    return out


def inject_at(values, t, b, c, mocks, freq_ghz, uvw_m, tint_s, kdm):
    """Stored values after adding mocks, at any set of positions.

    values: complex64 [..., npol] or float16 [..., npol, 2], the stored
    visibilities at integration t, baseline b, channel c (int arrays
    broadcastable to values' leading shape).  Mocks are added one at a time
    in the given order; after each, every value is the stored value plus the
    mock's signal (mock_signal), formed in float64 and rounded once to the
    storage type.  Returns a new array of the same type.
    """
    storage = "cf32" if np.iscomplexobj(values) else "cf16"
    cur = np.array(values, copy=True)
    for mk in mocks:
        sig = mock_signal(mk, t, b, c, freq_ghz, uvw_m, tint_s, kdm)[..., None]
        cur = round_storage(as_complex(cur).astype(np.complex128) + sig, storage)
    return cur


def inject(vis, mocks, freq_ghz, uvw_m, tint_s, kdm, t_first=0):
    """Add mock transients to a stored segment (section 3.3): vis is complex64
    [T][nbl][nchan][npol] or float16 [T][nbl][nchan][npol][2], integrations
    t_first .. t_first + T - 1; see inject_at."""
    T, B, C = vis.shape[0], vis.shape[1], vis.shape[2]
    t = (np.arange(T) + t_first)[:, None, None]
    b = np.arange(B)[None, :, None]
    c = np.arange(C)[None, None, :]
    return inject_at(vis, t, b, c, mocks, freq_ghz, uvw_m, tint_s, kdm)


def candidate_cutout(img, x, y, half):
    """Second-tier product (section 3.1: candidates above a higher threshold,
    typically 7 sigma, get visualisations; section 3.3: the candidate's image
    and spectrum): the 2 half x 2 half window of the candidate's image whose
    pixel (half, half) is the candidate pixel (x, y); the image is periodic
    (an inverse DFT), so the window wraps at the edges.
        out[r][q] = img[(y - half + r) mod N][(x - half + q) mod N]
    """
    N = img.shape[0]
    rows = np.mod(y - half + np.arange(2 * half), N)
    cols = np.mod(x - half + np.arange(2 * half), N)
    return img[np.ix_(rows, cols)]


def candidate_spectrum(vis, plan, i, j, k, x, y, nspec):
    """Second-tier product: the dedispersed dynamic spectrum toward the
    candidate pixel (x, y), float64 [nspec][nchan].

    Row s is resampled integration kk = k - nspec // 2 + s of DM trial i and
    width index j (zero when kk is outside [0, T // w)); column c is the mean
    over the channel's gridded baselines of the Stokes I sample turned to the
    pixel with the gridding's own cell phases:
        spec[s][c] = (1/n_c) sum_{b: (b,c) gridded}
                     Re( V_I[kk][b][c] exp(+2 pi i (iu (x - N/2) + iv (y - N/2)) / N) )
    (0 for a channel with no gridded baseline).  So sum_c n_c spec[s][c] / W
    is the image of (i, j, kk) at (x, y): the spectrum splits that pixel by
    channel.
    """
    w = plan.widths[j]
    T = vis.shape[0]
    K = T // w
    N = plan.npix
    dX, dY = x - N // 2, y - N // 2
    phase = np.exp(2j * np.pi * ((plan.iu * dX + plan.iv * dY) % N) / N)
    valid = plan.valid
    n_c = valid.sum(axis=0)
    out = np.zeros((nspec, plan.iu.shape[1]), dtype=np.float64)
    for s in range(nspec):
        kk = k - nspec // 2 + s
        if not 0 <= kk < K:
            continue
        dd = dedisperse_window(vis, plan.delays[i], kk * w, kk * w + w)
        vi = stokes_i(resample(dd, w)[0])
        turned = np.where(valid, (vi * phase).real, 0.0)
        tot = turned.sum(axis=0)
        out[s] = np.where(n_c > 0, tot / np.maximum(n_c, 1), 0.0)
    return out


# Median of the amplitude of a complex Gaussian with unit variance per
# quadrature (a Rayleigh variable of scale 1): sqrt(2 ln 2).
RAYLEIGH_MEDIAN = math.sqrt(2.0 * math.log(2.0))


def time_spectrum(vi):
    """Fluctuation spectrum of a segment along time (section 3.1 footnote:
    a time segment is Fourier transformed to frequencies): complex
    [T][...] -> F[f] = (1/T) sum_t vi[t] exp(-2 pi i f t / T).  A steady
    source of flux A gives F[0] = A; numpy's FFT is the library step."""
    T = vi.shape[0]
    return np.fft.fft(np.asarray(vi, dtype=np.complex128), axis=0) / T


def complex_image(G, W):
    """The image of a grid without taking the real part: (1/W) times the
    shifted unnormalised inverse DFT (the same sum as `image`).  A fluctuation
    frequency's grid has no Hermitian symmetry, so its sky is complex."""
    N = G.shape[0]
    return np.fft.fftshift(np.fft.ifft2(G) * (N * N)) / W


def amplitude_stats(A):
    """(peak, X, Y, sigma, snr) of an amplitude image A = |complex image|.

    Readings (parity unpinned: the paper states the periodicity search in one
    sentence): the statistic is the amplitude, whose peak is the fluctuation
    amplitude of a point source; sigma is the noise per quadrature, estimated
    as the lower median of A over sqrt(2 ln 2) (the median of the amplitude
    of a complex Gaussian); snr = peak / sigma (0 when sigma == 0).  Ties go
    to the lowest Y*N + X as in image_stats."""
    N = A.shape[1]
    flat = A.ravel()
    idx = int(np.argmax(flat))
    peak = float(flat[idx])
    k = (flat.size - 1) // 2
    med = float(np.partition(flat, k)[k])
    sigma = med / RAYLEIGH_MEDIAN
    snr = peak / sigma if sigma != 0.0 else 0.0
    return peak, idx % N, idx // N, sigma, snr


def periodic_search(vis, plan, select=None, keep_images=False):
    """Periodicity search (section 3.1 footnote; Figure 2 caption: a
    modification of the innermost loop).  For each DM trial: dedisperse,
    form Stokes I, take the fluctuation spectrum along time, and image and
    threshold every frequency f = 1 .. T // 2 (f = 0 is the steady sky; for
    a real source flux, f and T - f carry the same signal).

    Readings: the DM loop stays outside (a periodic source is dispersed too);
    the segment length T is the transform length (zero-filled tail as in
    dedisperse); widths do not apply.  select: optional set of (dm_idx, f).
    Returns (stats, candidates, images): stats (i, f) -> (peak, X, Y, sigma,
    snr) of the amplitude image; candidates (i, f, X, Y, snr, peak, sigma) in
    (i, f) order for snr > threshold.
    """
    vis = as_complex(vis)
    T = vis.shape[0]
    N = plan.npix
    stats, cands, images = {}, [], {}
    dm_set = range(len(plan.dms)) if select is None else sorted({s[0] for s in select})
    for i in dm_set:
        F = time_spectrum(stokes_i(dedisperse(vis, plan.delays[i])))
        for f in range(1, T // 2 + 1):
            if select is not None and (i, f) not in select:
                continue
            G = grid(F[f], plan.iu, plan.iv, plan.valid, N)
            A = np.abs(complex_image(G, plan.W))
            st = amplitude_stats(A)
            stats[(i, f)] = st
            if keep_images:
                images[(i, f)] = A
            peak, x, y, sigma, snr = st
            if snr > plan.threshold:
                cands.append((i, f, x, y, snr, peak, sigma))
    return stats, cands, images
