"""Workload presets: the observing shapes searched by the library.

Each preset fixes the synthetic geometry, band, time sampling, trial grids,
image size, seeds and injected pulses.  Shapes follow the observing
configurations of Law et al. 2018 (Table 1: 351 baselines from 27 antennas,
two polarisations, 256 channels, ms integrations) and the searched trial
grids described in section 3.1 (images per DM and pulse width).
"""
from dataclasses import dataclass, field
from typing import List

import numpy as np

from . import synth


@dataclass(frozen=True)
class Pulse:
    dm_idx: int
    width_idx: int
    t0: int          # start integration at the top of the band (multiple of width)
    x: int           # pixel column of the source
    y: int           # pixel row of the source
    snr: float = 20.0


@dataclass
class Preset:
    name: str
    nant: int
    nint: int
    tint_s: float
    f_lo_ghz: float
    f_hi_ghz: float
    nchan: int
    npol: int
    dms: np.ndarray
    widths: List[int]
    npix: int
    seed: int
    pulses: List[Pulse] = field(default_factory=list)
    kdm: float = 4.15e-3      # s GHz^2 / (pc cm^-3), section 2.1 footnote
    threshold: float = 6.0    # sigma, section 3.1
    t_begin: int = 0
    t_end: int = -1           # -1 means nint

    def __post_init__(self):
        self.dms = np.asarray(self.dms, dtype=np.float64)
        if self.t_end < 0:
            self.t_end = self.nint

    @property
    def nbl(self):
        return self.nant * (self.nant - 1) // 2

    def uvw(self):
        return synth.baseline_uvw(synth.y_array_positions(self.nant))

    def freq(self):
        return synth.channel_centres(self.f_lo_ghz, self.f_hi_ghz, self.nchan)

    def cell(self):
        du = synth.default_cell_size(self.uvw(), self.freq(), self.npix)
        return du, du

    def n_images(self):
        return len(self.dms) * sum(self.nint // w for w in self.widths)

    def pulse_amp(self, p: Pulse):
        """Flux giving matched-filter S/N p.snr when every (baseline, channel)
        pair is imaged: the image noise is (2 w nbl nchan)^-1/2 for unit
        complex Gaussian noise per polarisation averaged over w samples and
        two polarisations."""
        w = self.widths[p.width_idx]
        return p.snr / np.sqrt(2.0 * w * self.nbl * self.nchan)

    def mocks(self):
        """The pulses as mock-transient parameters (dm, t0, width, l, m, amp)
        for device-side injection into device-generated noise."""
        du, dv = self.cell()
        out = []
        for p in self.pulses:
            l, m = synth.pixel_to_lm(p.x, p.y, self.npix, du, dv)
            out.append(dict(dm=float(self.dms[p.dm_idx]), t0=float(p.t0),
                            width=float(self.widths[p.width_idx]), l=l, m=m,
                            amp=float(self.pulse_amp(p))))
        return out

    def make_vis(self, with_pulses=True):
        vis = synth.noise_vis(self.seed, self.nint, self.nbl, self.nchan, self.npol)
        if with_pulses:
            uvw, freq = self.uvw(), self.freq()
            du, dv = self.cell()
            for p in self.pulses:
                l, m = synth.pixel_to_lm(p.x, p.y, self.npix, du, dv)
                synth.add_pulse(vis, uvw, freq, self.tint_s, self.kdm,
                                float(self.dms[p.dm_idx]), p.t0,
                                self.widths[p.width_idx], l, m, self.pulse_amp(p))
        return vis


def tiny():
    """27-antenna Y array, 32 x 5 ms, 64 channels over 1-2 GHz, 2 pols, DM
    {0,50,100,150}, width 1, 256^2 image; one DM=100 pulse at S/N 20."""
    return Preset(name="tiny", nant=27, nint=32, tint_s=0.005, f_lo_ghz=1.0,
                  f_hi_ghz=2.0, nchan=64, npol=2, dms=np.linspace(0, 150, 4),
                  widths=[1], npix=256, seed=0,
                  pulses=[Pulse(dm_idx=2, width_idx=0, t0=0, x=138, y=121)])


def survey():
    """351 baselines, 2048 x 10 ms, 256 channels over 1-2 GHz, 2 pols, DM
    0-1000 in 128 trials, widths {1,2,4,8}, 1024^2 image; five S/N 20 pulses."""
    n = 1024
    c = n // 2
    pulses = [
        Pulse(dm_idx=7, width_idx=0, t0=16, x=c + 10, y=c - 7),
        Pulse(dm_idx=25, width_idx=1, t0=400, x=c - 23, y=c + 15),
        Pulse(dm_idx=51, width_idx=2, t0=800, x=c + 31, y=c + 40),
        Pulse(dm_idx=76, width_idx=3, t0=1200, x=c - 45, y=c - 12),
        Pulse(dm_idx=101, width_idx=1, t0=1600, x=c + 5, y=c + 52),
    ]
    return Preset(name="survey", nant=27, nint=2048, tint_s=0.010, f_lo_ghz=1.0,
                  f_hi_ghz=2.0, nchan=256, npol=2, dms=np.linspace(0, 1000, 128),
                  widths=[1, 2, 4, 8], npix=1024, seed=1, pulses=pulses)


def large():
    """351 baselines, 8192 x 1 ms, 1024 channels over 2-4 GHz, 2 pols, DM
    0-3000 in 400 trials, widths {1,2,4,8,16,32}, 2048^2 images; five S/N 20
    pulses at DM 150-2560.  47 GB as complex64: its noise is generated on the
    device (rfgen.philox defines the same values on the host, seed 4)."""
    n = 2048
    c = n // 2
    pulses = [
        Pulse(dm_idx=20, width_idx=0, t0=100, x=c + 60, y=c - 45),
        Pulse(dm_idx=100, width_idx=2, t0=1200, x=c - 80, y=c + 33),
        Pulse(dm_idx=180, width_idx=5, t0=2400, x=c + 17, y=c + 101),
        Pulse(dm_idx=260, width_idx=3, t0=3800, x=c - 120, y=c - 7),
        Pulse(dm_idx=340, width_idx=1, t0=5400, x=c + 9, y=c + 64),
    ]
    return Preset(name="large", nant=27, nint=8192, tint_s=0.001, f_lo_ghz=2.0,
                  f_hi_ghz=4.0, nchan=1024, npol=2, dms=np.linspace(0, 3000, 400),
                  widths=[1, 2, 4, 8, 16, 32], npix=n, seed=4, pulses=pulses)


def smallcase(nant=10, nint=37, nchan=48, npix=128, seed=5, npol=2):
    """A small ragged shape for parity tests: sizes that are not multiples of
    the kernels' tiles, three DMs, widths {1,2,4}, one pulse."""
    c = npix // 2
    return Preset(name="small", nant=nant, nint=nint, tint_s=0.005, f_lo_ghz=1.0,
                  f_hi_ghz=2.0, nchan=nchan, npol=npol,
                  dms=np.array([0.0, 60.0, 120.0]), widths=[1, 2, 4], npix=npix,
                  seed=seed, pulses=[Pulse(dm_idx=1, width_idx=1, t0=4, x=c + 5, y=c - 3)])


# Serving subarrays: antennas, integration time, integrations per 10.24 s segment
SUBARRAYS = {"A": (10, 0.005, 2048), "B": (19, 0.010, 1024), "C": (27, 0.005, 2048)}


def serving(sub="C", seed=None):
    """One segment of a serving subarray: 10.24 s of data, 256 channels over
    the L band of Table 1 (1.272-1.528 GHz), 2 pols, DM 0-1000 in 64 trials,
    widths {1,2,4,8}, 512^2 images; one S/N 20 pulse.  Subarrays A (10
    antennas, 5 ms), B (19, 10 ms), C (27, 5 ms)."""
    nant, tint, nint = SUBARRAYS[sub]
    n = 512
    c = n // 2
    k = "ABC".index(sub)
    return Preset(name=f"serving-{sub}", nant=nant, nint=nint, tint_s=tint, f_lo_ghz=1.272,
                  f_hi_ghz=1.528, nchan=256, npol=2, dms=np.linspace(0, 1000, 64),
                  widths=[1, 2, 4, 8], npix=n, seed=3 + k if seed is None else seed,
                  pulses=[Pulse(dm_idx=20 + 9 * k, width_idx=k, t0=64 * (k + 1),
                                x=c + 11 - 5 * k, y=c - 9 + 4 * k)])


def batching(s, keep_dms=None):
    """Segment s (0..63) of the batching workload: segments of uneven shape
    searched together (section 3.2: the stream is cut into independent
    segments).  351 baselines, 5 ms integrations over 1-2 GHz, 2 pols;
    nint = 256 * 2^(s mod 5), nchan = 128 * 2^(floor(s/5) mod 3), image side
    512 * 2^(s mod 3), 64 + (37 s mod 193) DM trials over 0-1000, widths
    {1,2,4,8}; one S/N 20 pulse at a third of the DM grid, seed 2 + s.  Meant
    for FP16 storage, generated on the device (rf_noise seed 2 + s plus the
    pulse as a mock).  keep_dms: a subset of the DM indices (the grid is
    unchanged; the pulse's index is remapped, and the pulse dropped if its
    trial is not kept)."""
    nint = 256 * 2 ** (s % 5)
    nchan = 128 * 2 ** ((s // 5) % 3)
    n = 512 * 2 ** (s % 3)
    ndm = 64 + (37 * s) % 193
    dms = np.linspace(0, 1000, ndm)
    j = s % 4
    w = [1, 2, 4, 8][j]
    c = n // 2
    pulse = Pulse(dm_idx=ndm // 3, width_idx=j, t0=w * ((nint // 8) // w),
                  x=c + 17 - 5 * (s % 7), y=c - 11 + 4 * (s % 5))
    pulses = [pulse]
    if keep_dms is not None:
        keep = sorted(set(int(i) for i in keep_dms))
        dms = dms[keep]
        pulses = [Pulse(dm_idx=keep.index(pulse.dm_idx), width_idx=j, t0=pulse.t0, x=pulse.x,
                        y=pulse.y)] if pulse.dm_idx in keep else []
    return Preset(name=f"batching-{s}", nant=27, nint=nint, tint_s=0.005, f_lo_ghz=1.0,
                  f_hi_ghz=2.0, nchan=nchan, npol=2, dms=dms, widths=[1, 2, 4, 8], npix=n,
                  seed=2 + s, pulses=pulses)


BATCHING_SEGMENTS = 64


def batching_dm_count(s):
    return 64 + (37 * s) % 193


def preset_by_name(name):
    if name.startswith("serving-"):
        return serving(name.split("-", 1)[1])
    return {"tiny": tiny, "survey": survey, "small": smallcase, "large": large}[name]()
