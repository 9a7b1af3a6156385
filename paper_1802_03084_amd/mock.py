"""Mock transients and efficiency curves.

The pipeline measures its own efficiency and sensitivity by inserting mock
transients into the data it searches and recording which it recovers (Law et
al. 2018, section 3.3, the mock source database).  This module draws mocks
for a plan, synthesises segments of counter-based noise with the mocks on
the device (rf_noise, rf_inject; each value rounded to the storage once),
runs the fused search and matches candidates to mocks; `efficiency` bins the records into recovered fraction and S/N
ratio against injected S/N, DM and width.

A mock's injected S/N is the matched-filter S/N of an ideal detection: the
full band, every gridded sample, a boxcar exactly `width` integrations long
and aligned with one resampled integration.  With unit complex Gaussian
noise per polarisation, the image noise of a w-integration box averaged over
two polarisations and W gridded samples is (2 w W)^-1/2, so amp = snr (2 w
W)^-1/2.  Off-grid mocks (DM between trials, fractional start, width that is
not a trial width) lose S/N to smearing, which is what the curves measure.

    from paper_1802_03084_amd import mock
    recs = mock.run(plan, nseg=8, per_seg=4, seed=1, snr=(4, 30))
    table = mock.efficiency(recs, "snr", bins=[4, 6, 8, 10, 15, 20, 30])
"""
import json
import math
from dataclasses import asdict, dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class Geometry:
    """What drawing and matching mocks needs to know about a plan."""
    nint: int
    tint_s: float
    freq_ghz: np.ndarray
    dms: np.ndarray
    widths: List[int]
    npix: int
    du: float
    dv: float
    W: int
    kdm: float = 4.15e-3
    threshold: float = 6.0
    npol: int = 2

    @classmethod
    def from_plan(cls, plan):
        return cls(nint=plan.nint, tint_s=plan.tint_s, freq_ghz=np.asarray(plan.freq_ghz),
                   dms=np.asarray(plan.dms), widths=list(plan.widths), npix=plan.npix,
                   du=plan.du, dv=plan.dv, W=plan.W, kdm=plan.kdm,
                   threshold=plan.threshold, npol=plan.npol)

    def sweep(self, dm):
        """Arrival lag of the lowest channel after the highest, integrations."""
        f = np.asarray(self.freq_ghz, dtype=np.float64)
        return self.kdm * dm * (1.0 / f.min() ** 2 - 1.0 / f.max() ** 2) / self.tint_s

    def lm(self, x, y):
        """Direction cosines of pixel (x, y); the phase centre is (N/2, N/2)."""
        n = self.npix
        return (x - n / 2) / (n * self.du), (y - n / 2) / (n * self.dv)

    def amplitude(self, snr, width):
        return snr / math.sqrt(2.0 * width * self.W * (self.npol / 2.0))


@dataclass
class MockRecord:
    """One inserted mock and what the search made of it."""
    seg: int
    dm: float
    t0: float
    width: float
    x: float
    y: float
    snr: float                 # injected (ideal matched-filter) S/N
    amp: float
    l: float = 0.0
    m: float = 0.0
    found: bool = False
    found_snr: float = 0.0
    found_key: Optional[list] = field(default=None)   # [dm_idx, width_idx, t_int, x, y]

    def as_mock(self):
        return dict(dm=self.dm, t0=self.t0, width=self.width, l=self.l, m=self.m, amp=self.amp)


def draw(geom, n, rng, snr=(5.0, 30.0), on_grid=True, box=0.125, seg=0):
    """n mocks in disjoint time slots of one segment.

    on_grid: DM on a trial value, width a trial width, start a multiple of
    the width, integer pixel (an exact detection is possible); otherwise DM
    uniform over the trial range, width log-uniform over the trial range,
    start and position continuous.  S/N log-uniform in [snr[0], snr[1]];
    position uniform in the central `box` fraction of the image.  Raises if
    the segment cannot hold n slots of the largest sweep plus width.
    """
    dms = np.asarray(geom.dms, dtype=np.float64)
    wmax = max(geom.widths)
    slot = int(math.ceil(geom.sweep(float(dms.max())))) + 2 * wmax + 2
    if n * slot > geom.nint:
        raise ValueError(f"{n} mocks need {n * slot} integrations, the segment has {geom.nint}")
    half = max(1, int(geom.npix * box / 2))
    recs = []
    for k in range(n):
        lo = k * slot
        if on_grid:
            i = int(rng.integers(0, len(dms)))
            dm = float(dms[i])
            w = float(geom.widths[int(rng.integers(0, len(geom.widths)))])
            room = slot - int(math.ceil(geom.sweep(dm))) - int(w) - 1
            t0 = float(lo + int(w) * int(rng.integers(0, max(1, room // int(w)))))
            x = float(geom.npix // 2 + int(rng.integers(-half, half + 1)))
            y = float(geom.npix // 2 + int(rng.integers(-half, half + 1)))
        else:
            dm = float(rng.uniform(dms.min(), dms.max()))
            w = float(math.exp(rng.uniform(math.log(min(geom.widths)), math.log(wmax))))
            room = slot - geom.sweep(dm) - w - 1
            t0 = lo + float(rng.uniform(0, max(room, 0.0)))
            x = geom.npix / 2 + float(rng.uniform(-half, half))
            y = geom.npix / 2 + float(rng.uniform(-half, half))
        s = float(math.exp(rng.uniform(math.log(snr[0]), math.log(snr[1]))))
        l, m = geom.lm(x, y)
        recs.append(MockRecord(seg=seg, dm=dm, t0=t0, width=w, x=x, y=y, snr=s,
                               amp=geom.amplitude(s, w), l=l, m=m))
    return recs


def match(recs, rows, geom, pix_tol=2.0):
    """Marks each mock found when a candidate lies within pix_tol pixels of it
    and starts within its time slot: t_int in [t0 - max width, t0 + width].
    The brightest such candidate is kept.  rows: the search's candidate
    array (fields dm_idx, width_idx, t_int, x, y, snr)."""
    wmax = max(geom.widths)
    for r in recs:
        if len(rows) == 0:
            continue
        t = rows["t_int"].astype(np.float64)
        sel = ((t >= r.t0 - wmax) & (t <= r.t0 + r.width)
               & (np.abs(rows["x"] - r.x) <= pix_tol) & (np.abs(rows["y"] - r.y) <= pix_tol))
        if not np.any(sel):
            continue
        best = np.flatnonzero(sel)[int(np.argmax(rows["snr"][sel]))]
        c = rows[best]
        r.found = True
        r.found_snr = float(c["snr"])
        r.found_key = [int(c[f]) for f in ("dm_idx", "width_idx", "t_int", "x", "y")]
    return recs


def efficiency(recs, by="snr", bins=None):
    """Recovered fraction per bin of `by` (snr, dm or width): a list of dicts
    with the bin edges, the number of mocks, the number found, the fraction
    and the mean recovered / injected S/N of the found ones."""
    vals = np.array([getattr(r, by) for r in recs], dtype=np.float64)
    if bins is None:
        bins = np.unique(vals) if by == "width" else np.linspace(vals.min(), vals.max(), 6)
    edges = np.asarray(bins, dtype=np.float64)
    out = []
    for a, b in zip(edges[:-1], edges[1:]):
        last = b == edges[-1]
        sel = [r for r, v in zip(recs, vals) if a <= v < b or (last and v == b)]
        found = [r for r in sel if r.found]
        out.append(dict(lo=float(a), hi=float(b), n=len(sel), found=len(found),
                        fraction=(len(found) / len(sel)) if sel else float("nan"),
                        snr_ratio=(float(np.mean([r.found_snr / r.snr for r in found]))
                                   if found else float("nan"))))
    return out


def save(recs, path):
    """Writes the mock records as JSON (the mock source database)."""
    with open(path, "w") as f:
        json.dump([asdict(r) for r in recs], f, indent=1)


def _staging_plan(plan, nint):
    from . import Plan, RF_CF32
    args = dict(plan._args)
    args.update(nint=int(nint), vis_dtype=RF_CF32, dms=np.zeros(1), widths=np.ones(1, np.int32),
                t_begin=0, t_end=int(nint))
    return Plan(**args)


def synthesize(plan, seed, mocks=(), stream_id=0, vis=None, chunk_ints=None, stream=None):
    """A device segment of `plan`'s shape and storage holding counter-based
    noise (rf_noise, stream `stream_id`) plus `mocks`, each value rounded to
    the storage once, as data whose signal was present before it was stored.

    CF32: noise and injection in place.  CF16: windows of chunk_ints
    integrations (default: at most 2 GiB of complex64) are generated and
    injected in a CF32 staging buffer, then rounded to nearest even into the
    segment, so the stored value is RNE16(RNE32(noise + signal)).
    """
    import torch
    from . import RF_CF32
    if vis is None:
        vis = plan.empty_vis()
    if plan.vis_dtype == RF_CF32:
        plan.noise(vis, seed=seed, stream_id=stream_id, stream=stream)
        plan.inject(vis, list(mocks), stream=stream)
        return vis
    per = plan.nbl * plan.nchan * plan.npol
    chunk = int(chunk_ints) if chunk_ints else max(1, min(plan.nint, (1 << 28) // per))
    stage = {}
    for t0 in range(0, plan.nint, chunk):
        n = min(chunk, plan.nint - t0)
        if n not in stage:
            sp = _staging_plan(plan, n)
            stage[n] = (sp, sp.empty_vis())
        sp, buf = stage[n]
        sp.noise(buf, seed=seed, stream_id=stream_id, t_first=t0, stream=stream)
        sp.inject(buf, list(mocks), t_first=t0, stream=stream)
        vis[t0:t0 + n].copy_(torch.view_as_real(buf).to(torch.float16))
    torch.cuda.synchronize()
    return vis


def run(plan, nseg, per_seg, seed, snr=(5.0, 30.0), on_grid=True, box=0.125, cap=65536,
        noise_seed=None, stream=None):
    """Inserts per_seg mocks into each of nseg noise segments of `plan`'s
    shape (rf_noise, stream id = segment index), searches each on the device
    and matches candidates.  Returns the records of every mock."""
    import torch
    geom = Geometry.from_plan(plan)
    rng = np.random.default_rng(seed)
    nseed = seed if noise_seed is None else noise_seed
    from . import RF_OP_SEGMENT
    vis = plan.empty_vis()
    ws = plan.workspace(RF_OP_SEGMENT)
    recs = []
    for s in range(nseg):
        seg = draw(geom, per_seg, rng, snr=snr, on_grid=on_grid, box=box, seg=s)
        synthesize(plan, nseed, [r.as_mock() for r in seg], stream_id=s, vis=vis, stream=stream)
        rows, _, _ = plan.search_segment(vis, cap=cap, ws=ws, stream=stream)
        recs.extend(match(seg, rows, geom))
    del ws, vis
    torch.cuda.synchronize()
    return recs
