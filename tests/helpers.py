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


# ---------------------------------------------------------------- oracle pool
# Sampled oracle images of a large segment in worker processes: the segment
# is memory-mapped from an .npy file (spawned interpreters that never touch
# the GPU), each worker rebuilds the oracle plan from its arguments.
_POOL = {}


def _pool_init(vis_path, plan_kwargs):
    _POOL["vis"] = np.load(vis_path, mmap_mode="r")
    _POOL["plan"] = oracle.Plan(**plan_kwargs)


def _pool_one(key):
    vis, plan = _POOL["vis"], _POOL["plan"]
    img = oracle.image_at(vis, plan, *key)
    st = oracle.image_stats(img)
    marg = {tol: bool(oracle.is_marginal(img, st[4], plan.threshold, tol)) for tol in (1e-5, 3e-3)}
    return key, st, marg, float(np.max(np.abs(img)))


def oracle_plan_kwargs(p, du=None, dv=None):
    if du is None:
        du, dv = p.cell()
    return dict(freq_ghz=p.freq(), uvw_m=p.uvw(), tint_s=p.tint_s, dms=np.asarray(p.dms),
                widths=list(p.widths), npix=p.npix, du=du, dv=dv, kdm=p.kdm,
                threshold=p.threshold, t_begin=p.t_begin, t_end=p.t_end, nint=p.nint)


def oracle_images_pool(vis_path, plan_kwargs, keys, procs=16, progress=None):
    """{key: (stats, {tol: marginal}, max|img|)} for (dm_idx, width_idx, k)
    keys, computed by oracle.image_at in `procs` spawned processes."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    out = {}
    with ctx.Pool(procs, initializer=_pool_init, initargs=(vis_path, plan_kwargs)) as pool:
        for n, (key, st, marg, amax) in enumerate(pool.imap_unordered(_pool_one, list(keys), chunksize=4)):
            out[key] = (st, marg, amax)
            if progress and (n + 1) % 200 == 0:
                progress(n + 1, len(keys))
    return out
