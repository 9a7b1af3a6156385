"""Second-tier candidate products through the C ABI (rf_candidate_products):
image cutouts and dedispersed spectra against the oracle's, on a ragged
small case (CF32 and CF16, rows at the segment's ends and pixels at the
image edges) and on the survey segment at full size."""
import sys

import numpy as np
import pytest

import oracle
import rfgen
from helpers import gpu_plan, oracle_plan, upload

pytestmark = pytest.mark.gpu

TOL = 1e-5


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rows(keys):
    import paper_1802_03084_amd as rf
    out = np.zeros(len(keys), rf.CAND_DTYPE)
    for n, (i, j, t, x, y) in enumerate(keys):
        out[n] = (i, j, t, x, y, 0.0, 0.0, 0.0)
    return out


def _compare(g, p, o, vis_host, dvis, rows, half, nspec):
    cut, spec = g.candidate_products(dvis, rows, half=half, nspec=nspec)
    cut = cut.cpu().numpy()
    spec = spec.cpu().numpy()
    for n, r in enumerate(rows):
        i, j, t, x, y = (int(r[f]) for f in ("dm_idx", "width_idx", "t_int", "x", "y"))
        k = t // p.widths[j]
        img = oracle.image_at(vis_host, o, i, j, k)
        want_cut = oracle.candidate_cutout(img, x, y, half)
        amax = float(np.max(np.abs(img)))
        assert np.max(np.abs(cut[n] - want_cut)) <= TOL * amax, (n, i, j, t, x, y)
        want_spec = oracle.candidate_spectrum(vis_host, o, i, j, k, x, y, nspec)
        smax = float(np.max(np.abs(want_spec)))
        err = float(np.max(np.abs(spec[n] - want_spec)))
        say("products", (i, j, t, x, y), "cutout err", float(np.max(np.abs(cut[n] - want_cut))) / amax,
            "spectrum err", err / smax if smax else err)
        assert err <= TOL * smax, (n, i, j, t, x, y)
        zero_rows = [s for s in range(nspec) if not 0 <= k - nspec // 2 + s < p.nint // p.widths[j]]
        assert all(np.all(spec[n][s] == 0) for s in zero_rows)


@pytest.mark.parametrize("dtype", [0, 1])
def test_products_match_oracle(torch, dtype):
    p = rfgen.smallcase(nant=10, nint=37, nchan=48, npix=128, seed=15)
    g = gpu_plan(p, vis_dtype=dtype)
    o = oracle_plan(p)
    vis = p.make_vis()
    host = vis if dtype == 0 else rfgen.to_cf16(vis)
    dvis = upload(vis, dtype)
    rows, n, _ = g.search_segment(dvis, cap=4096)
    q = p.pulses[0]
    keys = [(q.dm_idx, q.width_idx, q.t0, q.x, q.y),
            (0, 0, 0, 0, 127),            # first integration, corner pixel
            (2, 2, 32, 127, 0),            # last width-4 integration, opposite corner
            (1, 0, 36, 64, 64)]            # last integration
    for r in rows[:3]:
        keys.append(tuple(int(r[f]) for f in ("dm_idx", "width_idx", "t_int", "x", "y")))
    say("products small, dtype", dtype, "rows", len(keys))
    _compare(g, p, o, host, dvis, _rows(keys), half=16, nspec=7)


def test_products_survey_full_size(torch):
    """The survey segment at full size: the products of the injected pulses
    (all above 7 sigma) against the oracle."""
    import paper_1802_03084_amd as rf
    p = rfgen.survey()
    say("generating the survey segment")
    vis = p.make_vis()
    g = gpu_plan(p)
    o = oracle_plan(p)
    dvis = upload(vis)
    rows, n, _ = g.search_segment(dvis, cap=65536)
    tier = rf.second_tier(rows, 7.0)
    pulse_keys = {(q.dm_idx, q.width_idx, q.t0, q.x, q.y) for q in p.pulses}
    sel = [r for r in tier if tuple(int(r[f]) for f in ("dm_idx", "width_idx", "t_int", "x", "y")) in pulse_keys]
    assert len(sel) == len(p.pulses)
    say("products survey: second tier", len(tier), "of", len(rows))
    _compare(g, p, o, vis, dvis, np.array(sel, dtype=rf.CAND_DTYPE), half=32, nspec=16)


def test_products_reject_bad_rows(torch):
    import paper_1802_03084_amd as rf
    p = rfgen.smallcase(nant=10, nint=37, nchan=48, npix=128)
    g = gpu_plan(p)
    dvis = g.empty_vis()
    for key, half, nspec in [((0, 1, 3, 5, 5), 8, 4),      # t_int not a multiple of the width
                             ((0, 0, 37, 5, 5), 8, 4),     # past the last integration
                             ((3, 0, 0, 5, 5), 8, 4),      # no such DM trial
                             ((0, 0, 0, 128, 5), 8, 4),    # pixel outside
                             ((0, 0, 0, 5, 5), 65, 4),     # cutout larger than the image
                             ((0, 0, 0, 5, 5), 8, 0)]:     # no spectrum rows
        with pytest.raises(rf.RFError) as e:
            g.candidate_products(dvis, _rows([key]), half=half, nspec=nspec)
        assert e.value.status == -3, key

