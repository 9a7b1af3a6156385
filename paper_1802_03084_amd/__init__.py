"""realfast search hot path on MI355X: Python binding of librf.

Argument marshalling only: every step runs in librf's HIP kernels.  torch
supplies device memory and the current stream.  The binding's names follow
the C ABI (include/rf.h):

    plan = Plan(freq_ghz, uvw_m, tint_s, dms, widths, npix, du, dv, nint=..., npol=2)
    plan.dedisperse(vis, dm_idx)      # rf_dedisperse
    plan.resample(x, width)           # rf_resample
    plan.grid(vis)                    # rf_grid
    plan.image(grid)                  # rf_image
    plan.search(img, tags)            # rf_search
    plan.search_segment(vis)          # rf_search_segment

Visibilities are torch tensors on the GPU: complex64 [nint, nbl, nchan, npol]
for RF_CF32 storage, or float16 [nint, nbl, nchan, npol, 2] for RF_CF16.
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import (RF_CF16, RF_CF32, RF_OP_IMAGE, RF_OP_SEARCH, RF_OP_SEGMENT,  # noqa: F401
                   RF_OP_SEGMENT_STEPS,
                   Candidate, ImageStats, ImageTag, RFError)

__all__ = ["Plan", "Server", "Batch", "RFError", "RF_CF32", "RF_CF16", "load_library", "CAND_DTYPE", "second_tier",
           "STATS_DTYPE"]

CAND_DTYPE = np.dtype([("dm_idx", "<i4"), ("width_idx", "<i4"), ("t_int", "<i4"), ("x", "<i4"),
                       ("y", "<i4"), ("snr", "<f4"), ("peak", "<f4"), ("sigma", "<f4")])
STATS_DTYPE = np.dtype([("peak", "<f4"), ("sigma", "<f4"), ("snr", "<f4"), ("x", "<i4"),
                        ("y", "<i4")])
TAG_DTYPE = np.dtype([("dm_idx", "<i4"), ("width_idx", "<i4"), ("t_int", "<i4")])


def second_tier(rows, threshold=7.0):
    """Candidates above the second, higher threshold (section 3.1: about 7
    sigma), which get image cutouts and spectra (rf_select_tier)."""
    rows = np.ascontiguousarray(rows, dtype=CAND_DTYPE)
    out = np.empty(len(rows), dtype=CAND_DTYPE)
    k = ctypes.c_int32()
    _lib.check(_lib.load().rf_select_tier(rows.ctypes.data_as(ctypes.c_void_p), len(rows),
                                          float(threshold), out.ctypes.data_as(ctypes.c_void_p),
                                          len(out), ctypes.byref(k)), "rf_select_tier")
    return out[: k.value]


def load_library():
    return _lib.load()


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class Plan:
    """An immutable search plan (rf_plan) with its device tables."""

    def __init__(self, freq_ghz, uvw_m, tint_s, dms, widths, npix, du, dv, nint, npol=2,
                 vis_dtype=RF_CF32, kdm=4.15e-3, threshold=6.0, t_begin=0, t_end=None,
                 device="cuda"):
        torch = _torch()
        lib = _lib.load()
        self._freq = np.ascontiguousarray(freq_ghz, dtype=np.float64)
        self._uvw = np.ascontiguousarray(uvw_m, dtype=np.float64).reshape(-1, 3)
        self._dm = np.ascontiguousarray(dms, dtype=np.float64)
        self._width = np.ascontiguousarray(widths, dtype=np.int32)
        self.nint, self.nbl, self.nchan, self.npol = int(nint), self._uvw.shape[0], self._freq.size, int(npol)
        self.vis_dtype = int(vis_dtype)
        self.npix = int(npix)
        self.widths = [int(w) for w in self._width]
        self.ndm = self._dm.size
        d = _lib.PlanDesc()
        d.nint, d.nbl, d.nchan, d.npol = self.nint, self.nbl, self.nchan, self.npol
        d.vis_dtype = self.vis_dtype
        d.tint_s = float(tint_s)
        d.freq_ghz = self._freq.ctypes.data_as(_lib.c_dp)
        d.uvw_m = self._uvw.ctypes.data_as(_lib.c_dp)
        d.dm = self._dm.ctypes.data_as(_lib.c_dp)
        d.ndm = self._dm.size
        d.width = self._width.ctypes.data_as(_lib.c_ip)
        d.nwidth = self._width.size
        d.npix = self.npix
        d.du, d.dv, d.kdm = float(du), float(dv), float(kdm)
        d.threshold = float(threshold)
        d.t_begin = int(t_begin)
        d.t_end = self.nint if t_end is None else int(t_end)
        self._desc = d
        self._args = dict(freq_ghz=self._freq, uvw_m=self._uvw, tint_s=float(tint_s), dms=self._dm,
                          widths=self._width, npix=self.npix, du=float(du), dv=float(dv),
                          nint=self.nint, npol=self.npol, vis_dtype=self.vis_dtype, kdm=float(kdm),
                          threshold=float(threshold), t_begin=int(t_begin), t_end=d.t_end,
                          device=device)
        nbytes = _lib.c_size(0)
        _lib.check(lib.rf_plan_table_bytes(ctypes.byref(d), ctypes.byref(nbytes)), "rf_plan_table_bytes")
        self.device = torch.device(device)
        self.tables = torch.empty(max(1, nbytes.value), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        _lib.check(lib.rf_plan_create(ctypes.byref(d), _ptr(self.tables), nbytes.value, _stream(),
                                      ctypes.byref(h)), "rf_plan_create")
        self._h = h
        info = _lib.PlanInfo()
        _lib.check(lib.rf_plan_query(h, ctypes.byref(info)), "rf_plan_query")
        self.info = {k: getattr(info, k) for k, _ in _lib.PlanInfo._fields_}
        self.n_images = int(info.n_images)
        self.W = int(info.n_valid)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                _lib.load().rf_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    # ---------------------------------------------------------------- helpers
    @property
    def handle(self):
        return self._h

    freq_ghz = property(lambda self: self._freq)
    uvw_m = property(lambda self: self._uvw)
    dms = property(lambda self: self._dm)
    tint_s = property(lambda self: self._args["tint_s"])
    du = property(lambda self: self._args["du"])
    dv = property(lambda self: self._args["dv"])
    kdm = property(lambda self: self._args["kdm"])
    threshold = property(lambda self: self._args["threshold"])

    def subtract_mean(self, vis, stream=None):
        """rf_subtract_mean: in place, each (baseline, channel, polarisation)
        value loses its mean over the segment."""
        self._check_vis(vis, self.nint)
        _lib.check(_lib.load().rf_subtract_mean(self._h, _ptr(vis), _stream(stream)),
                   "rf_subtract_mean")
        return vis

    def inject(self, vis, mocks, t_first=0, stream=None):
        """rf_inject: adds mock transients to vis in place (mocks: dicts or
        objects with dm, t0, width, l, m, amp; added in order); vis holds
        integrations t_first .. t_first + nint - 1 of the mocks' segment."""
        self._check_vis(vis, self.nint)
        arr = (_lib.Mock * max(1, len(mocks)))()
        for k, mk in enumerate(mocks):
            get = mk.get if isinstance(mk, dict) else (lambda f, _m=mk: getattr(_m, f))
            for f, _ in _lib.Mock._fields_:
                setattr(arr[k], f, float(get(f)))
        _lib.check(_lib.load().rf_inject(self._h, ctypes.cast(arr, ctypes.c_void_p), len(mocks),
                                         int(t_first), _ptr(vis), _stream(stream)), "rf_inject")
        return vis

    def noise(self, vis=None, seed=0, stream_id=0, t_first=0, stream=None):
        """rf_noise: fills vis (allocated if None) with the counter-based
        complex Gaussian noise of integrations t_first .. t_first + nint - 1
        of stream (seed, stream_id)."""
        if vis is None:
            vis = self.empty_vis()
        self._check_vis(vis, self.nint)
        _lib.check(_lib.load().rf_noise(self._h, int(seed) & ((1 << 64) - 1), int(stream_id),
                                        int(t_first), _ptr(vis), _stream(stream)), "rf_noise")
        return vis

    def products_workspace_bytes(self, nspec):
        n = _lib.c_size(0)
        _lib.check(_lib.load().rf_products_workspace_bytes(self._h, int(nspec), ctypes.byref(n)),
                   "rf_products_workspace_bytes")
        return n.value

    def candidate_products(self, vis, rows, half=32, nspec=16, cutouts=True, spectra=True,
                           ws=None, stream=None):
        """rf_candidate_products for candidate rows (CAND_DTYPE, e.g. the
        second tier second_tier(rows)): returns (cutouts [n][2 half][2 half],
        spectra [n][nspec][nchan]) float32 device tensors (None when not
        asked for)."""
        torch = _torch()
        self._check_vis(vis, self.nint)
        rows = np.ascontiguousarray(rows, dtype=CAND_DTYPE)
        n = len(rows)
        cut = torch.empty((n, 2 * half, 2 * half), dtype=torch.float32, device=self.device) if cutouts else None
        spec = torch.empty((n, nspec, self.nchan), dtype=torch.float32, device=self.device) if spectra else None
        if ws is None:
            ws = torch.empty(max(1, self.products_workspace_bytes(nspec)), dtype=torch.uint8,
                             device=self.device)
        _lib.check(_lib.load().rf_candidate_products(
            self._h, _ptr(vis), rows.ctypes.data_as(ctypes.c_void_p), n, int(half), int(nspec),
            _ptr(cut), _ptr(spec), _ptr(ws), ws.numel(), _stream(stream)), "rf_candidate_products")
        return cut, spec

    def set_tuning(self, lanes, m_budget_mb):
        """rf_plan_set_tuning: lane streams and the row-transformed batch
        budget (MB) of the fused search; results do not depend on them."""
        _lib.check(_lib.load().rf_plan_set_tuning(self._h, int(lanes), int(m_budget_mb)),
                   "rf_plan_set_tuning")
        info = _lib.PlanInfo()
        _lib.check(_lib.load().rf_plan_query(self._h, ctypes.byref(info)), "rf_plan_query")
        self.info = {k: getattr(info, k) for k, _ in _lib.PlanInfo._fields_}

    @property
    def tuning(self):
        return int(self.info["lanes"]), int(self.info["m_budget_mb"])

    def subplan(self, ndm):
        """A plan of the same shape over the first ndm DM trials (for tuning)."""
        args = dict(self._args)
        args["dms"] = self._dm[: max(1, int(ndm))]
        return Plan(**args)

    def image_base(self, dm_idx, width_idx):
        per_dm = sum(self.nint // w for w in self.widths)
        return dm_idx * per_dm + sum(self.nint // w for w in self.widths[:width_idx])

    def delays(self):
        out = np.empty((self.ndm, self.nchan), dtype=np.int32)
        _lib.check(_lib.load().rf_get_delays(self._h, out.ctypes.data_as(ctypes.c_void_p)), "rf_get_delays")
        return out

    def cells(self):
        out = np.empty((self.nbl, self.nchan, 2), dtype=np.int32)
        _lib.check(_lib.load().rf_get_cells(self._h, out.ctypes.data_as(ctypes.c_void_p)), "rf_get_cells")
        return out

    def workspace_bytes(self, op, nimg=0):
        n = _lib.c_size(0)
        _lib.check(_lib.load().rf_workspace_bytes(self._h, op, nimg, ctypes.byref(n)), "rf_workspace_bytes")
        return n.value

    def workspace(self, op, nimg=0):
        torch = _torch()
        return torch.empty(max(1, self.workspace_bytes(op, nimg)), dtype=torch.uint8, device=self.device)

    def _vis_shape(self, nint):
        if self.vis_dtype == RF_CF32:
            return (nint, self.nbl, self.nchan, self.npol)
        return (nint, self.nbl, self.nchan, self.npol, 2)

    def empty_vis(self, nint=None):
        torch = _torch()
        nint = self.nint if nint is None else nint
        dt = torch.complex64 if self.vis_dtype == RF_CF32 else torch.float16
        return torch.empty(self._vis_shape(nint), dtype=dt, device=self.device)

    def _check_vis(self, t, nint, cf32_only=False, name="vis"):
        torch = _torch()
        want_dt = torch.complex64 if (cf32_only or self.vis_dtype == RF_CF32) else torch.float16
        want_shape = (nint, self.nbl, self.nchan, self.npol) + (() if want_dt == torch.complex64 else (2,))
        if t.dtype != want_dt or tuple(t.shape) != want_shape or not t.is_contiguous() or t.device.type != "cuda":
            raise ValueError(f"{name}: expected contiguous cuda {want_dt} {want_shape}, got "
                             f"{t.dtype} {tuple(t.shape)} on {t.device}")

    # ---------------------------------------------------------------- steps
    def dedisperse(self, vis, dm_idx, out=None, stream=None):
        self._check_vis(vis, self.nint)
        if out is None:
            out = self.empty_vis()
        self._check_vis(out, self.nint, name="out")
        _lib.check(_lib.load().rf_dedisperse(self._h, int(dm_idx), _ptr(vis), _ptr(out), _stream(stream)),
                   "rf_dedisperse")
        return out

    def resample(self, x, width, out=None, stream=None):
        torch = _torch()
        nin = x.shape[0]
        self._check_vis(x, nin, name="x")
        nout = nin // int(width)
        if out is None:
            out = torch.empty((nout, self.nbl, self.nchan, self.npol), dtype=torch.complex64, device=self.device)
        self._check_vis(out, nout, cf32_only=True, name="out")
        _lib.check(_lib.load().rf_resample(self._h, int(width), _ptr(x), nin, _ptr(out), _stream(stream)),
                   "rf_resample")
        return out

    def grid(self, vis, out=None, stream=None):
        torch = _torch()
        nimg = vis.shape[0]
        self._check_vis(vis, nimg, cf32_only=True)
        if out is None:
            out = torch.empty((nimg, self.npix, self.npix), dtype=torch.complex64, device=self.device)
        if out.dtype != torch.complex64 or tuple(out.shape) != (nimg, self.npix, self.npix) or not out.is_contiguous():
            raise ValueError("grid out: expected complex64 [nimg, N, N]")
        _lib.check(_lib.load().rf_grid(self._h, _ptr(vis), nimg, _ptr(out), _stream(stream)), "rf_grid")
        return out

    def image(self, grid, out=None, ws=None, stream=None):
        torch = _torch()
        nimg = grid.shape[0]
        if grid.dtype != torch.complex64 or tuple(grid.shape) != (nimg, self.npix, self.npix) or not grid.is_contiguous():
            raise ValueError("grid: expected complex64 [nimg, N, N]")
        if out is None:
            out = torch.empty((nimg, self.npix, self.npix), dtype=torch.float32, device=self.device)
        if ws is None:
            ws = self.workspace(RF_OP_IMAGE, nimg)
        _lib.check(_lib.load().rf_image(self._h, _ptr(grid), nimg, _ptr(out), _ptr(ws), ws.numel(),
                                        _stream(stream)), "rf_image")
        return out

    def search(self, img, tags, cap=4096, ncand=None, cand=None, with_stats=True, stream=None):
        """Threshold images; tags: int32 [nimg, 3] (dm_idx, width_idx, t_int).
        Returns (candidates sorted by (dm_idx, width_idx, t_int), true count,
        stats structured array or None).  Synchronises the stream."""
        torch = _torch()
        nimg = img.shape[0]
        tags_t = torch.as_tensor(np.ascontiguousarray(tags, dtype=np.int32).reshape(nimg, 3), device=self.device)
        stats = torch.empty((nimg, 5), dtype=torch.int32, device=self.device) if with_stats else None
        if cand is None:
            cand = torch.empty((max(cap, 1), 8), dtype=torch.int32, device=self.device)
        if ncand is None:
            ncand = torch.zeros(1, dtype=torch.int32, device=self.device)
        _lib.check(_lib.load().rf_search(self._h, _ptr(img), nimg, _ptr(tags_t), _ptr(stats), _ptr(cand),
                                         int(cap), _ptr(ncand), None, 0, _stream(stream)), "rf_search")
        return self._collect(cand, ncand, stats, cap)

    def search_segment(self, vis, cap=65536, with_stats=False, ws=None, stream=None, collect=True,
                       steps=False):
        """rf_search_segment (fused), or rf_search_segment_steps with steps=True."""
        torch = _torch()
        self._check_vis(vis, self.nint)
        op = RF_OP_SEGMENT_STEPS if steps else RF_OP_SEGMENT
        with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream()):
            if ws is None:
                ws = self.workspace(op)
            cand = torch.empty((max(cap, 1), 8), dtype=torch.int32, device=self.device)
            ncand = torch.empty(1, dtype=torch.int32, device=self.device)  # zeroed by the search
            stats = (torch.empty((self.n_images, 5), dtype=torch.int32, device=self.device)
                     if with_stats else None)
        fn = _lib.load().rf_search_segment_steps if steps else _lib.load().rf_search_segment
        _lib.check(fn(self._h, _ptr(vis), _ptr(cand), int(cap), _ptr(ncand), _ptr(stats), _ptr(ws),
                      ws.numel(), _stream(stream)), "rf_search_segment" + ("_steps" if steps else ""))
        if not collect:
            return cand, ncand, stats
        if stream is not None:  # results are complete in that stream's order
            stream.synchronize()
        return self._collect(cand, ncand, stats, cap)

    def search_segment_begin(self, vis, cap=65536, with_stats=False, ws=None, stream=None):
        """rf_search_segment_begin: enqueues the fused search and returns at
        once; pass the result to search_segment_end for the candidates."""
        torch = _torch()
        self._check_vis(vis, self.nint)
        # buffers belong to the search's stream; the search sets the count to
        # zero itself (no fill on another stream that could race with it)
        with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream()):
            if ws is None:
                ws = self.workspace(RF_OP_SEGMENT)
            cand = torch.empty((max(cap, 1), 8), dtype=torch.int32, device=self.device)
            ncand = torch.empty(1, dtype=torch.int32, device=self.device)
            stats = (torch.empty((self.n_images, 5), dtype=torch.int32, device=self.device)
                     if with_stats else None)
        job = ctypes.c_void_p()
        _lib.check(_lib.load().rf_search_segment_begin(self._h, _ptr(vis), _ptr(cand), int(cap), _ptr(ncand),
                                                       _ptr(stats), _ptr(ws), ws.numel(), _stream(stream),
                                                       ctypes.byref(job)), "rf_search_segment_begin")
        return {"job": job, "keep": (vis, ws, cand, ncand, stats), "cap": int(cap),
                "stream": stream if stream is not None else _torch().cuda.current_stream()}

    def search_segment_end(self, pending):
        """rf_search_segment_end: waits, runs the exact fallbacks (enqueued on
        the search's stream); returns as search_segment once that stream is
        done."""
        _lib.check(_lib.load().rf_search_segment_end(pending["job"]), "rf_search_segment_end")
        pending["stream"].synchronize()
        _, _, cand, ncand, stats = pending["keep"]
        return self._collect(cand, ncand, stats, pending["cap"])

    def periodic_workspace_bytes(self):
        n = _lib.c_size(0)
        _lib.check(_lib.load().rf_periodic_workspace_bytes(self._h, ctypes.byref(n)),
                   "rf_periodic_workspace_bytes")
        return n.value

    def search_periodic(self, vis, cap=65536, with_stats=False, ws=None, stream=None):
        """rf_search_periodic: candidate rows (width_idx = -1, t_int = the
        frequency bin f), the true count and, with stats, the per-(DM, f)
        amplitude statistics [ndm * nint/2] (row i * nint/2 + f - 1)."""
        torch = _torch()
        self._check_vis(vis, self.nint)
        if ws is None:
            ws = torch.empty(max(1, self.periodic_workspace_bytes()), dtype=torch.uint8,
                             device=self.device)
        cand = torch.empty((max(cap, 1), 8), dtype=torch.int32, device=self.device)
        ncand = torch.zeros(1, dtype=torch.int32, device=self.device)
        nst = self.ndm * (self.nint // 2)
        stats = torch.empty((max(nst, 1), 5), dtype=torch.int32, device=self.device) if with_stats else None
        _lib.check(_lib.load().rf_search_periodic(self._h, _ptr(vis), _ptr(cand), int(cap), _ptr(ncand),
                                                  _ptr(stats), _ptr(ws), ws.numel(), _stream(stream)),
                   "rf_search_periodic")
        return self._collect(cand, ncand, stats, cap)

    def profile_segment(self, vis, cap=65536, ws=None, stream=None, concurrent=False, sample=1):
        """rf_search_segment_profile: one fused search with kernel launches
        event-timed (every sample-th launch of each kind).  concurrent=False
        runs every launch in order on one stream (durations do not overlap);
        True runs the streams of search_segment.
        Returns ({kind: (ms_total, launches timed)}, candidates, count)."""
        torch = _torch()
        self._check_vis(vis, self.nint)
        if ws is None:
            ws = self.workspace(RF_OP_SEGMENT)
        cand = torch.empty((max(cap, 1), 8), dtype=torch.int32, device=self.device)
        ncand = torch.zeros(1, dtype=torch.int32, device=self.device)
        kt = _lib.KernelTimes()
        kt.concurrent = 1 if concurrent else 0
        kt.sample = int(sample)
        _lib.check(_lib.load().rf_search_segment_profile(self._h, _ptr(vis), _ptr(cand), int(cap), _ptr(ncand),
                                                         None, _ptr(ws), ws.numel(), _stream(stream),
                                                         ctypes.byref(kt)), "rf_search_segment_profile")
        rows, n, _ = self._collect(cand, ncand, None, cap)
        times = {k: (kt.ms[i], int(kt.launches[i])) for i, k in enumerate(_lib.KERNEL_KINDS)}
        return times, rows, n

    @staticmethod
    def _collect(cand, ncand, stats, cap):
        n = int(ncand.item())
        rows = cand[: min(n, cap)].cpu().numpy().view(CAND_DTYPE).reshape(-1)
        rows = np.sort(rows, order=["dm_idx", "width_idx", "t_int"])
        st = stats.cpu().numpy().view(STATS_DTYPE).reshape(-1) if stats is not None else None
        return rows, n, st


class Server:
    """rf_server_*: segments released to a request loop, admitted by the HBM
    budget of one device arena and searched concurrently on `nslots` slot
    streams.  The arena is a caller-owned uint8 device tensor; segments are
    host tensors in the plan's layout (pinned for asynchronous copies) that
    must stay alive until their wait returns."""

    def __init__(self, arena, nslots=2):
        self._arena = arena  # keeps the device memory alive
        h = ctypes.c_void_p()
        _lib.check(_lib.load().rf_server_create(_ptr(arena), arena.numel() * arena.element_size(),
                                                int(nslots), ctypes.byref(h)), "rf_server_create")
        self._h = h
        self._keep = {}

    @staticmethod
    def request_bytes(plan, cap=4096):
        n = ctypes.c_size_t()
        _lib.check(_lib.load().rf_server_request_bytes(plan.handle, int(cap), ctypes.byref(n)),
                   "rf_server_request_bytes")
        return n.value

    SUBTRACT_MEAN = 1
    FAIL_AFTER_COPY = 2  # fault injection: the request fails after its copy is enqueued

    def submit(self, plan, h_vis, cap=4096, subtract_mean=False, flags=0):
        """Releases one segment; returns its ticket at once.  subtract_mean:
        the segment's time mean is subtracted on the device before the search.
        flags: further rf_server_submit flags (FAIL_AFTER_COPY for tests)."""
        torch = _torch()
        want_dt = torch.complex64 if plan.vis_dtype == RF_CF32 else torch.float16
        want = (plan.nint, plan.nbl, plan.nchan, plan.npol) + (() if want_dt == torch.complex64 else (2,))
        if h_vis.dtype != want_dt or tuple(h_vis.shape) != want or not h_vis.is_contiguous() \
                or h_vis.device.type != "cpu":
            raise ValueError(f"h_vis: expected contiguous host {want_dt} {want}, got {h_vis.dtype} "
                             f"{tuple(h_vis.shape)} on {h_vis.device}")
        t = ctypes.c_int64()
        _lib.check(_lib.load().rf_server_submit(self._h, plan.handle, _ptr(h_vis), int(cap),
                                                int(flags) | (self.SUBTRACT_MEAN if subtract_mean else 0),
                                                ctypes.byref(t)),
                   "rf_server_submit")
        self._keep[t.value] = (plan, h_vis, int(cap))
        return t.value

    def wait(self, ticket):
        """Blocks until the ticket's segment is done: (rows sorted by (dm_idx,
        width_idx, t_int), true count, {released_s, started_s, done_s, latency_s})."""
        plan, h_vis, cap = self._keep.pop(ticket)
        buf = (Candidate * max(cap, 1))()
        n = ctypes.c_int32()
        tm = _lib.ServeTimes()
        _lib.check(_lib.load().rf_server_wait(self._h, int(ticket), ctypes.cast(buf, ctypes.c_void_p),
                                              cap, ctypes.byref(n), ctypes.byref(tm)), "rf_server_wait")
        k = min(n.value, cap)
        rows = np.frombuffer(bytes(buf)[: k * ctypes.sizeof(Candidate)], dtype=CAND_DTYPE).copy()
        rows = np.sort(rows, order=["dm_idx", "width_idx", "t_int"])
        times = {f: getattr(tm, f) for f, _ in _lib.ServeTimes._fields_}
        return rows, n.value, times

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.check(_lib.load().rf_server_destroy(self._h), "rf_server_destroy")
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """rf_batch_*: the fused searches of several segments (plans of any shapes)
    bound once and run by one call.  The segment tensors are bound at
    creation: refill them in place between runs.  graph=True captures the
    whole batch into one HIP graph at creation (each run is one launch)."""

    GRAPH = 1

    def __init__(self, plans, vis, cap=4096, with_stats=False, graph=False):
        torch = _torch()
        lib = _lib.load()
        n = len(plans)
        if n < 1 or len(vis) != n:
            raise ValueError("one segment tensor per plan")
        for p, v in zip(plans, vis):
            p._check_vis(v, p.nint)
        self.plans, self.vis, self.cap = list(plans), list(vis), int(cap)
        dev = vis[0].device
        self.cand = [torch.empty((max(self.cap, 1), 8), dtype=torch.int32, device=dev) for _ in plans]
        self.ncand = [torch.zeros(1, dtype=torch.int32, device=dev) for _ in plans]
        self.stats = ([torch.empty((p.n_images, 5), dtype=torch.int32, device=dev) for p in plans]
                      if with_stats else None)
        hs = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
        nb = ctypes.c_size_t()
        _lib.check(lib.rf_batch_workspace_bytes(hs, n, ctypes.byref(nb)), "rf_batch_workspace_bytes")
        self.ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
        arr = lambda ts: (ctypes.c_void_p * n)(*[t.data_ptr() for t in ts])  # noqa: E731
        self._keep = (hs, arr(self.vis), arr(self.cand), (ctypes.c_int32 * n)(*([self.cap] * n)),
                      arr(self.ncand), arr(self.stats) if self.stats else None)
        h = ctypes.c_void_p()
        _lib.check(lib.rf_batch_create(hs, n, self._keep[1], self._keep[2], self._keep[3],
                                       self._keep[4], self._keep[5], _ptr(self.ws), nb.value,
                                       self.GRAPH if graph else 0, ctypes.byref(h)), "rf_batch_create")
        self._h = h
        nodes = ctypes.c_size_t()
        _lib.check(lib.rf_batch_graph_nodes(h, ctypes.byref(nodes)), "rf_batch_graph_nodes")
        self.graph_nodes = nodes.value

    def run(self, stream=None, collect=True):
        """Runs every segment (then the exact fallbacks); returns per segment
        (rows sorted by (dm_idx, width_idx, t_int), true count, stats or None)."""
        _lib.check(_lib.load().rf_batch_run(self._h, _stream(stream)), "rf_batch_run")
        if not collect:
            return None
        out = []
        for i in range(len(self.plans)):
            st = self.stats[i] if self.stats else None
            out.append(Plan._collect(self.cand[i], self.ncand[i], st, self.cap))
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.check(_lib.load().rf_batch_destroy(self._h), "rf_batch_destroy")
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

