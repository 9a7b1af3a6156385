"""Planted mistakes in the oracle must be caught by its pins.

Each mutant copies the oracle's namespace and replaces one function with a
plausibly wrong version (a dropped term, a wrong sign, a swapped index, a
transposed operand).  At least one pin must reject every mutant; otherwise the
pins would not be evidence that the oracle is right.
"""
import math
import types

import numpy as np
import pytest

import oracle
from oracle import rf_oracle as ro
from oracle.rf_oracle import C_LIGHT
import pins


def mutant(**repl):
    """The oracle's namespace with some functions replaced.  Every oracle
    function is rebound to globals holding the replacements, so a function
    that calls a replaced one (inject -> mock_signal) sees the mistake too."""
    g = dict(ro.__dict__)
    g.update(repl)
    ns = {}
    for k, v in g.items():
        if k.startswith("__"):
            continue
        if isinstance(v, types.FunctionType) and v.__module__ == ro.__name__ and k not in repl:
            v = types.FunctionType(v.__code__, g, v.__name__, v.__defaults__, v.__closure__)
            g[k] = v
        ns[k] = v
    return types.SimpleNamespace(**ns)


def _delay_inv_nu(freq, dms, tint, kdm):             # 1/nu instead of 1/nu^2
    f = np.asarray(freq, float)
    lag = (kdm * np.asarray(dms, float))[:, None] * (1.0 / f - 1.0 / f.max())[None, :]
    return np.rint(lag / tint).astype(np.int32)


def _delay_floor(freq, dms, tint, kdm):              # floor instead of rint
    f = np.asarray(freq, float)
    lag = (kdm * np.asarray(dms, float))[:, None] * (1.0 / (f * f) - 1.0 / (f.max() ** 2))[None, :]
    return np.floor(lag / tint).astype(np.int32)


def _delay_ref_low(freq, dms, tint, kdm):            # reference at the bottom channel
    f = np.asarray(freq, float)
    lag = (kdm * np.asarray(dms, float))[:, None] * (1.0 / (f.min() ** 2) - 1.0 / (f * f))[None, :]
    return np.rint(lag / tint).astype(np.int32)


def _dedisperse_backwards(vis, d):                   # t - d instead of t + d
    T = vis.shape[0]
    out = np.zeros(vis.shape, complex)
    for c, dd in enumerate(d):
        dd = int(dd)
        if dd < T:
            out[dd:, :, c, :] = vis[: T - dd, :, c, :]
    return out


def _resample_sum(x, w):                             # sum instead of mean
    return ro.resample(x, w) * w


def _resample_sliding(x, w):                         # sliding boxcar
    K = x.shape[0] - w + 1
    return np.stack([x[k:k + w].mean(axis=0) for k in range(K)])


def _stokes_sum(v):                                  # dropped 1/2
    return v[..., 0] + v[..., 1] if v.shape[-1] == 2 else v[..., 0]


def _grid_transposed(vi, iu, iv, valid, N):          # u and v swapped
    return ro.grid(vi, iv, iu, valid, N)


def _grid_no_wrap(vi, iu, iv, valid, N):             # negative cells clipped
    G = np.zeros((N, N), complex)
    m = valid & (iu >= 0) & (iv >= 0)
    np.add.at(G, (iv[m], iu[m]), vi[m])
    return G


def _image_forward(G, W):                            # forward instead of inverse DFT
    N = G.shape[0]
    return np.fft.fftshift(np.fft.fft2(G)).real / W


def _image_noshift(G, W):                            # fftshift dropped
    N = G.shape[0]
    return (np.fft.ifft2(G) * N * N).real / W


def _image_no_norm(G, W):                            # 1/W dropped
    N = G.shape[0]
    return np.fft.fftshift(np.fft.ifft2(G) * N * N).real


def _image_transposed(G, W):                         # image transposed
    return ro.image(G, W).T


def _image_abs(G, W):                                # |.| instead of Re
    N = G.shape[0]
    return np.abs(np.fft.fftshift(np.fft.ifft2(G) * N * N)) / W


def _stats_mean(img):                                # sigma from the mean |img|
    p, x, y, _, _ = ro.image_stats(img)
    s = 1.4826 * float(np.mean(np.abs(img)))
    return p, x, y, s, (p / s if s else 0.0)


def _stats_std(img):                                 # sigma = standard deviation
    p, x, y, _, _ = ro.image_stats(img)
    s = float(np.std(img))
    return p, x, y, s, (p / s if s else 0.0)


def _stats_absmax(img):                              # peak of |img|
    N = img.shape[1]
    idx = int(np.argmax(np.abs(img)))
    _, _, _, s, _ = ro.image_stats(img)
    p = float(np.abs(img).ravel()[idx])
    return p, idx % N, idx // N, s, (p / s if s else 0.0)


def _stats_xy_swapped(img):                          # X and Y swapped
    p, x, y, s, snr = ro.image_stats(img)
    return p, y, x, s, snr


def _cells_no_freq(uvw, freq, du, dv):               # frequency dropped from u
    u = np.asarray(uvw)[:, 0:1] * np.ones((1, len(freq)))
    v = np.asarray(uvw)[:, 1:2] * np.ones((1, len(freq)))
    return np.rint(u / du).astype(np.int32), np.rint(v / dv).astype(np.int32)


def _mean_over_baselines(vis):                     # mean over the wrong axis
    v = np.asarray(vis).astype(np.complex128)
    return v - v.mean(axis=1, keepdims=True)


def _mean_unbiased(vis):                           # divides by T - 1
    v = np.asarray(vis).astype(np.complex128)
    return v - v.sum(axis=0, keepdims=True) / (v.shape[0] - 1)


def _mean_of_first(vis):                           # subtracts the first integration
    v = np.asarray(vis).astype(np.complex128)
    return v - v[:1]


def _signal_with(**change):
    """mock_signal with one planted change (keyword switches below)."""
    def sig(mock, t, b, c, freq_ghz, uvw_m, tint_s, kdm):
        f = np.asarray(freq_ghz, float)
        uvw = np.asarray(uvw_m, float)
        t, b, c = np.broadcast_arrays(np.asarray(t), np.asarray(b), np.asarray(c))
        nu = f[c]
        ref = f.min() if change.get("ref_low") else f.max()
        power = 1 if change.get("inv_nu") else 2
        lag = (kdm * mock["dm"]) * (1.0 / nu ** power - 1.0 / ref ** power)
        if change.get("lag_sign"):
            lag = -lag
        start = mock["t0"] + lag / tint_s
        width = 1.0 if change.get("no_width") else mock["width"]
        end = start + width
        tt = t.astype(float)
        if change.get("no_split"):
            frac = np.where(tt == np.floor(start), width, 0.0)
        else:
            frac = np.maximum(np.minimum(tt + 1.0, end) - np.maximum(tt, start), 0.0)
        f_hz = nu * 1e9
        u_l = (uvw[b, 0] * f_hz) / C_LIGHT
        v_l = (uvw[b, 1] * f_hz) / C_LIGHT
        l, m = (mock["m"], mock["l"]) if change.get("lm_swapped") else (mock["l"], mock["m"])
        sign = 1.0 if change.get("phase_sign") else -1.0
        phase = sign * (2.0 * math.pi * (u_l * l + v_l * m))
        s = mock["amp"] * frac
        return s * np.cos(phase) + 1j * (s * np.sin(phase))
    return sig


def _inject_first_pol(vis, mocks, freq, uvw, tint, kdm, t_first=0):  # only polarisation 0
    out = ro.inject(vis, mocks, freq, uvw, tint, kdm, t_first)
    out[:, :, :, 1:] = vis[:, :, :, 1:]
    return out


def _inject_once(values, t, b, c, mocks, freq, uvw, tint, kdm):   # one rounding for all mocks
    storage = "cf32" if np.iscomplexobj(values) else "cf16"
    tot = ro.as_complex(values).astype(complex)
    for mk in mocks:
        tot = tot + ro.mock_signal(mk, t, b, c, freq, uvw, tint, kdm)[..., None]
    return ro.round_storage(tot, storage)


def _round_via_f32(z, storage):                                      # float16 via float32
    z = np.asarray(z)
    if storage == "cf32":
        return z.astype(np.complex64)
    out = np.empty(z.shape + (2,), np.float16)
    out[..., 0] = z.real.astype(np.float32).astype(np.float16)
    out[..., 1] = z.imag.astype(np.float32).astype(np.float16)
    return out


def _spectrum_with(conj=False, no_dd=False, per_nbl=False, shift=0):
    def spec(vis, plan, i, j, k, x, y, nspec):
        w = plan.widths[j]
        T = vis.shape[0]
        N = plan.npix
        sign = -1.0 if conj else 1.0
        phase = np.exp(sign * 2j * np.pi * ((plan.iu * (x - N // 2) + plan.iv * (y - N // 2)) % N) / N)
        n_c = plan.valid.sum(axis=0)
        den = np.full_like(n_c, plan.iu.shape[0]) if per_nbl else np.maximum(n_c, 1)
        out = np.zeros((nspec, plan.iu.shape[1]))
        for s_ in range(nspec):
            kk = k - nspec // 2 + s_ + shift
            if not 0 <= kk < T // w:
                continue
            d = np.zeros_like(plan.delays[i]) if no_dd else plan.delays[i]
            dd = ro.dedisperse_window(vis, d, kk * w, kk * w + w)
            vi = ro.stokes_i(ro.resample(dd, w)[0])
            out[s_] = np.where(n_c > 0, np.where(plan.valid, (vi * phase).real, 0).sum(axis=0) / den, 0)
        return out
    return spec


def _cutout_transposed(img, x, y, half):
    return ro.candidate_cutout(img, x, y, half).T


def _cutout_off_by_one(img, x, y, half):
    return ro.candidate_cutout(img, x, y + 1, half)


def _tspec_unnormalised(vi):                         # 1/T dropped
    return np.fft.fft(np.asarray(vi, complex), axis=0)


def _tspec_inverse(vi):                              # exp(+2 pi i f t / T)
    T = vi.shape[0]
    return np.fft.ifft(np.asarray(vi, complex), axis=0)


def _cimage_real(G, W):                              # real part only
    return ro.image(G, W).astype(complex)


def _astats_gaussian(A):                             # transient sigma estimator
    p, x, y, _, _ = ro.amplitude_stats(A)
    s = 1.4826 * float(np.median(A))
    return p, x, y, s, (p / s if s else 0.0)


def _periodic_with(zero_freq=False, first_pol=False, no_dd=False):
    def search(vis, plan, select=None, keep_images=False):
        vis = ro.as_complex(vis)
        T = vis.shape[0]
        stats, cands = {}, []
        for i in range(len(plan.dms)):
            d = np.zeros_like(plan.delays[i]) if no_dd else plan.delays[i]
            dd = ro.dedisperse(vis, d)
            vi = dd[..., 0] if first_pol else ro.stokes_i(dd)
            F = ro.time_spectrum(vi)
            freqs = range(0, T // 2) if zero_freq else range(1, T // 2 + 1)
            for f in freqs:
                if select is not None and (i, f) not in select:
                    continue
                G = ro.grid(F[f], plan.iu, plan.iv, plan.valid, plan.npix)
                st = ro.amplitude_stats(np.abs(ro.complex_image(G, plan.W)))
                stats[(i, f)] = st
                if st[4] > plan.threshold:
                    cands.append((i, f, st[1], st[2], st[4], st[0], st[3]))
        return stats, cands, {}
    return search


def _window_with(backwards=False, past_end=False, shift=0):
    def win(vis, delay_row, t0, t1):
        T = vis.shape[0]
        out = np.zeros((t1 - t0,) + tuple(vis.shape[1:4]), complex)
        for c, d in enumerate(np.asarray(delay_row)):
            for t in range(t0, t1):
                s = (t - int(d) if backwards else t + int(d)) + shift
                if past_end:
                    ok = s <= T                               # one sample past the end
                else:
                    ok = 0 <= s < T
                if ok:
                    out[t - t0, :, c, :] = ro.as_complex(vis[s, :, c])
        return out
    return win


def _image_at_next(vis, plan, i, j, k):               # box starts at k*w + 1
    w = plan.widths[j]
    dd = ro.dedisperse_window(vis, plan.delays[i], k * w + 1, k * w + w + 1)
    return ro.make_image(ro.resample(dd, w)[0], plan)


def _image_at_first_width(vis, plan, i, j, k):        # window of width 1
    dd = ro.dedisperse_window(vis, plan.delays[i], k, k + 1)
    return ro.make_image(dd[0], plan)


def _marginal_with(abs_snr=False, one_tol=False, abs_gap=False, bottom=False):
    def marg(img, snr, threshold, tol):
        f = 1 if one_tol else 10
        lim = f * tol if abs_snr else f * tol * threshold
        if abs(snr - threshold) < lim:
            return True
        flat = np.sort(img.ravel())
        top, second = (flat[0], flat[1]) if bottom else (flat[-1], flat[-2])
        if top == 0.0:
            return True
        gap = abs(top - second)
        return (gap if abs_gap else gap / abs(top)) < f * tol
    return marg


MUTANTS = {
    "mean over baselines": dict(subtract_mean=_mean_over_baselines),
    "mean unbiased": dict(subtract_mean=_mean_unbiased),
    "mean of first": dict(subtract_mean=_mean_of_first),
    "delay 1/nu": dict(delay_table=_delay_inv_nu),
    "delay floor": dict(delay_table=_delay_floor),
    "delay ref at bottom": dict(delay_table=_delay_ref_low),
    "dedisperse backwards": dict(dedisperse=_dedisperse_backwards),
    "resample sum": dict(resample=_resample_sum),
    "resample sliding": dict(resample=_resample_sliding),
    "stokes sum": dict(stokes_i=_stokes_sum),
    "grid transposed": dict(grid=_grid_transposed),
    "grid no wrap": dict(grid=_grid_no_wrap),
    "image forward": dict(image=_image_forward),
    "image no shift": dict(image=_image_noshift),
    "image no 1/W": dict(image=_image_no_norm),
    "image transposed": dict(image=_image_transposed),
    "image abs": dict(image=_image_abs),
    "sigma mean": dict(image_stats=_stats_mean),
    "sigma std": dict(image_stats=_stats_std),
    "peak abs": dict(image_stats=_stats_absmax),
    "stats xy swapped": dict(image_stats=_stats_xy_swapped),
    "cells no freq": dict(cell_table=_cells_no_freq),
    "mock phase sign": dict(mock_signal=_signal_with(phase_sign=True)),
    "mock lag 1/nu": dict(mock_signal=_signal_with(inv_nu=True)),
    "mock lag ref at bottom": dict(mock_signal=_signal_with(ref_low=True)),
    "mock lag sign": dict(mock_signal=_signal_with(lag_sign=True)),
    "mock width ignored": dict(mock_signal=_signal_with(no_width=True)),
    "mock flux not split": dict(mock_signal=_signal_with(no_split=True)),
    "mock l m swapped": dict(mock_signal=_signal_with(lm_swapped=True)),
    "mock first pol only": dict(inject=_inject_first_pol),
    "mock single rounding": dict(inject_at=_inject_once),
    "mock f16 via f32": dict(round_storage=_round_via_f32),
    "spectrum phase conjugated": dict(candidate_spectrum=_spectrum_with(conj=True)),
    "spectrum not dedispersed": dict(candidate_spectrum=_spectrum_with(no_dd=True)),
    "spectrum over all baselines": dict(candidate_spectrum=_spectrum_with(per_nbl=True)),
    "spectrum rows shifted": dict(candidate_spectrum=_spectrum_with(shift=1)),
    "cutout transposed": dict(candidate_cutout=_cutout_transposed),
    "cutout off by one": dict(candidate_cutout=_cutout_off_by_one),
    "time spectrum unnormalised": dict(time_spectrum=_tspec_unnormalised),
    "time spectrum inverse": dict(time_spectrum=_tspec_inverse),
    "complex image real part": dict(complex_image=_cimage_real),
    "amplitude sigma gaussian": dict(amplitude_stats=_astats_gaussian),
    "periodic includes f=0": dict(periodic_search=_periodic_with(zero_freq=True)),
    "periodic first pol": dict(periodic_search=_periodic_with(first_pol=True)),
    "periodic not dedispersed": dict(periodic_search=_periodic_with(no_dd=True)),
    "window t - d": dict(dedisperse_window=_window_with(backwards=True)),
    "window reads past the end": dict(dedisperse_window=_window_with(past_end=True)),
    "window off by one": dict(dedisperse_window=_window_with(shift=1)),
    "image_at next box": dict(image_at=_image_at_next),
    "image_at width ignored": dict(image_at=_image_at_first_width),
    "marginal absolute snr": dict(is_marginal=_marginal_with(abs_snr=True)),
    "marginal without 10x": dict(is_marginal=_marginal_with(one_tol=True)),
    "marginal absolute gap": dict(is_marginal=_marginal_with(abs_gap=True)),
    "marginal bottom pixels": dict(is_marginal=_marginal_with(bottom=True)),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    o = mutant(**MUTANTS[name])
    failed = []
    for check in pins.ALL_CHECKS:
        try:
            check(o)
        except (AssertionError, ValueError, IndexError):
            failed.append(check.__name__)
    assert failed, f"no pin catches the planted mistake '{name}'"


def test_unmutated_passes_everything():
    o = mutant()
    for check in pins.ALL_CHECKS:
        check(o)
