"""Forward model: antennas -> baselines -> visibilities with noise and pulses.

Everything here is a simulation of the input data, written from the physics of
an interferometer (Law et al. 2018, section 2.2: visibilities are correlations
between antenna pairs, N_bl = N_ant (N_ant - 1) / 2) and of a dispersed pulse
(section 2.1 footnote: the cold-plasma delay scales as DM / nu^2).  It is not
the search: no integer delay table, no uv cells, no images are computed here.
"""
import math

import numpy as np

C_LIGHT = 299792458.0  # m/s


def y_array_positions(n_ant=27, arm_m=1000.0, power=1.716):
    """Antenna positions of a synthetic three-arm Y array, metres, [n_ant][3].

    Three arms at azimuths 0, 120 and 240 degrees, nine stations per arm at
    r_k = arm_m * (k/9)**power, k = 1..9 (power-law station spacing).  With
    n_ant == 27 the antenna order is arm-major (index = arm*9 + k - 1).  A
    smaller subarray takes the innermost stations round-robin over the arms
    and is then ordered arm-major.  x is east, y north, z = 0.
    """
    if not 2 <= n_ant <= 27:
        raise ValueError("n_ant must be in [2, 27]")
    picks = []
    for k in range(1, 10):
        for arm in range(3):
            picks.append((arm, k))
    picks = sorted(picks[:n_ant])
    pos = np.zeros((n_ant, 3), dtype=np.float64)
    for i, (arm, k) in enumerate(picks):
        az = math.radians(120.0 * arm)
        r = arm_m * (k / 9.0) ** power
        pos[i, 0] = r * math.sin(az)
        pos[i, 1] = r * math.cos(az)
    return pos


def baseline_uvw(pos):
    """Baseline vectors b = pos_j - pos_i for i < j, metres, [nbl][3].

    The phase centre is the zenith, so (u, v, w) = (dx, dy, 0) and w plays no
    part in the imaging.
    """
    n = pos.shape[0]
    rows = []
    for i in range(n):
        for j in range(i + 1, n):
            d = pos[j] - pos[i]
            rows.append((d[0], d[1], 0.0))
    return np.asarray(rows, dtype=np.float64)


def channel_centres(f_lo_ghz, f_hi_ghz, nchan):
    """Channel centre frequencies in GHz: f_lo + (c + 1/2) * (f_hi - f_lo) / nchan."""
    bw = (f_hi_ghz - f_lo_ghz) / nchan
    return f_lo_ghz + (np.arange(nchan, dtype=np.float64) + 0.5) * bw


def default_cell_size(uvw_m, freq_ghz, npix):
    """uv cell (wavelengths) that makes the longest projected spacing land at
    N/2 - 2 cells from the origin, i.e. about two pixels per synthesised beam."""
    fmax = float(np.max(freq_ghz)) * 1e9
    umax = float(np.max(np.abs(uvw_m[:, :2]))) * fmax / C_LIGHT
    return umax / (npix / 2 - 2)


def noise_vis(seed, nint, nbl, nchan, npol):
    """Complex64 visibilities [nint][nbl][nchan][npol]; Re and Im i.i.d. N(0,1).

    Recipe: numpy default_rng(seed).standard_normal in float32, first the whole
    real-part array, then the whole imaginary-part array.
    """
    rng = np.random.default_rng(seed)
    shape = (nint, nbl, nchan, npol)
    vis = np.empty(shape, dtype=np.complex64)
    vis.real = rng.standard_normal(shape, dtype=np.float32)
    vis.imag = rng.standard_normal(shape, dtype=np.float32)
    return vis


def pixel_to_lm(x_pix, y_pix, npix, du, dv):
    """Direction cosines of image pixel (X, Y) for a grid of npix cells of size
    du x dv wavelengths, with the phase centre at pixel (N/2, N/2)."""
    return (x_pix - npix / 2) / (npix * du), (y_pix - npix / 2) / (npix * dv)


def add_pulse(vis, uvw_m, freq_ghz, tint_s, kdm, dm, t_start, width, l, m, amp):
    """Add a dispersed boxcar pulse from direction (l, m) to vis in place.

    Physical model: at the top channel the pulse starts at t_start * tint_s
    seconds and lasts width * tint_s.  In channel c it arrives later by
    kdm * dm * (nu_c**-2 - nu_top**-2) seconds (cold-plasma law, nu in GHz).
    Integration j integrates flux over [j tint, (j+1) tint), so a pulse that
    straddles two integrations splits its flux between them.  Every
    polarisation sees the same flux (an unpolarised source).  The visibility of
    a point source of flux S at (l, m) on baseline (u, v) at frequency nu is
    S * exp(-2 pi i (u l + v m) nu / c).
    """
    nint, nbl, nchan, npol = vis.shape
    nu_top = float(np.max(freq_ghz))
    lag_s = kdm * dm * (1.0 / freq_ghz**2 - 1.0 / nu_top**2)
    start = t_start + lag_s / tint_s  # in integrations, per channel
    u_lam = uvw_m[:, 0:1] * (freq_ghz[None, :] * 1e9) / C_LIGHT
    v_lam = uvw_m[:, 1:2] * (freq_ghz[None, :] * 1e9) / C_LIGHT
    phasor = np.exp(-2j * np.pi * (u_lam * l + v_lam * m))  # [nbl][nchan]
    for c in range(nchan):
        a = start[c]
        b = a + width
        j0 = int(math.floor(a))
        j1 = int(math.ceil(b))
        for j in range(max(j0, 0), min(j1, nint)):
            frac = min(j + 1.0, b) - max(float(j), a)
            if frac <= 0.0:
                continue
            val = (amp * frac) * phasor[:, c]
            for p in range(npol):
                vis[j, :, c, p] += val.astype(vis.dtype)


def to_cf16(vis):
    """Complex64 [...] -> float16 [..., 2] (re, im), round-to-nearest-even."""
    out = np.empty(vis.shape + (2,), dtype=np.float16)
    out[..., 0] = vis.real.astype(np.float16)
    out[..., 1] = vis.imag.astype(np.float16)
    return out


def from_cf16(v16):
    """float16 [..., 2] -> complex128 (exact widening)."""
    return v16[..., 0].astype(np.float64) + 1j * v16[..., 1].astype(np.float64)
