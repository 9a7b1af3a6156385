"""Shared test plumbing: build matching oracle / GPU plans from a preset."""
import numpy as np

import oracle
import rfgen


def oracle_plan(p, du=None, dv=None):
    if du is None:
        du, dv = p.cell()
    return oracle.Plan(p.freq(), p.uvw(), p.tint_s, p.dms, p.widths, p.npix, du, dv,
                       kdm=p.kdm, threshold=p.threshold, t_begin=p.t_begin, t_end=p.t_end,
                       nint=p.nint)


def gpu_plan(p, vis_dtype=0, du=None, dv=None, **kw):
    import paper_1802_03084_amd as rf
    if du is None:
        du, dv = p.cell()
    args = dict(kdm=p.kdm, threshold=p.threshold, t_begin=p.t_begin, t_end=p.t_end)
    args.update(kw)
    return rf.Plan(p.freq(), p.uvw(), p.tint_s, p.dms, p.widths, p.npix, du, dv, nint=p.nint,
                   npol=p.npol, vis_dtype=vis_dtype, **args)


def upload(vis, vis_dtype=0):
    import torch
    if vis_dtype == 0:
        return torch.from_numpy(np.ascontiguousarray(vis.astype(np.complex64))).cuda()
    return torch.from_numpy(np.ascontiguousarray(rfgen.to_cf16(vis))).cuda()


def rel_err(a, ref):
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.max(np.abs(ref))
    return float(np.max(np.abs(a - ref)) / den) if den > 0 else float(np.max(np.abs(a)))


def cand_keys(rows):
    return [tuple(int(r[f]) for f in ("dm_idx", "width_idx", "t_int", "x", "y")) for r in rows]
