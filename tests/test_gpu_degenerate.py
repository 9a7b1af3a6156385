"""Degenerate shapes through the C ABI: a plan that grids nothing (W = 0), a
width as long as the segment (and one longer, rejected), a single image, a
zero capacity, and the periodicity search and second-tier products on such
inputs."""
import sys

import numpy as np
import pytest

import rfgen
from helpers import cand_keys, gpu_plan, upload
from test_gpu_fullsize import _shape_parity

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_nothing_gridded(torch):
    """A cell size so small that every (baseline, channel) pair falls off the
    grid: W = 0, every image is identically zero (sigma 0, S/N 0), and so is
    every periodicity image and product."""
    p = rfgen.smallcase(nint=16)
    du, dv = p.cell()
    g = gpu_plan(p, du=du * 1e-3, dv=dv * 1e-3)
    assert g.W == 0 and g.info["n_dropped"] == p.nbl * p.nchan
    vis = upload(p.make_vis())
    say("nothing gridded")
    rows, n, st = g.search_segment(vis, cap=64, with_stats=True)
    assert n == 0 and (st["peak"] == 0).all() and (st["sigma"] == 0).all() and (st["snr"] == 0).all()
    rows_p, n_p, st_p = g.search_periodic(vis, cap=64, with_stats=True)
    assert n_p == 0 and (st_p["peak"] == 0).all() and (st_p["snr"] == 0).all()
    import paper_1802_03084_amd as rf
    key = np.zeros(1, rf.CAND_DTYPE)
    key[0] = (1, 0, 3, 10, 20, 0, 0, 0)
    cut, spec = g.candidate_products(vis, key, half=8, nspec=4)
    assert float(cut.abs().max()) == 0.0 and float(spec.abs().max()) == 0.0


def test_nothing_gridded_survey_shape(torch):
    """W = 0 at the survey shape (351 baselines x 256 channels, 2048
    integrations, 1024^2) with DM trials over 0-500: the step chain that
    produces the zero statistics fills buffers that cover the fused path's
    fallback list, and with the top DM under the full sweep those buffers hold
    data.  No image may be sent to the exact recomputation, twice in a row."""
    p = rfgen.survey()
    p.dms = np.linspace(0, 500, 8)
    p.pulses = []
    du, dv = p.cell()
    g = gpu_plan(p, du=du * 1e-3, dv=dv * 1e-3)
    assert g.W == 0
    vis = upload(p.make_vis())
    for rep in range(2):
        say("nothing gridded, survey shape, run", rep)
        times, rows, n = g.profile_segment(vis, cap=64)
        assert n == 0 and times["fallback"][1] == 0, times
        rows, n, st = g.search_segment(vis, cap=64, with_stats=True)
        assert n == 0 and (st["peak"] == 0).all() and (st["snr"] == 0).all()


def test_widths_up_to_the_segment(torch):
    """A width equal to the segment length gives one image per DM trial (as
    the oracle's); a width longer than the segment is rejected."""
    import paper_1802_03084_amd as rf
    p = rfgen.smallcase(nint=8, seed=9)
    p.widths = [1, 2, 4, 8]
    p.pulses = [rfgen.Pulse(dm_idx=0, width_idx=0, t0=2, x=70, y=60)]
    say("widths up to the segment")
    g = gpu_plan(p)
    assert g.n_images == len(p.dms) * (8 + 4 + 2 + 1)
    rows = _shape_parity(p)
    assert (0, 0, 2, 70, 60) in cand_keys(rows)
    p.nint, p.t_end = 5, 5
    with pytest.raises(rf.RFError) as e:
        gpu_plan(p)
    assert e.value.status == -3


def test_single_image(torch):
    """One DM trial, one width, one integration."""
    p = rfgen.smallcase(nint=1, seed=10)
    p.dms = np.array([0.0])
    p.widths = [1]
    p.pulses = [rfgen.Pulse(dm_idx=0, width_idx=0, t0=0, x=66, y=61)]
    say("single image")
    g = gpu_plan(p)
    assert g.n_images == 1
    rows = _shape_parity(p)
    assert cand_keys(rows) == [(0, 0, 0, 66, 61)]


def test_zero_capacity_reports_the_count(torch):
    p = rfgen.smallcase(seed=11)
    g = gpu_plan(p)
    vis = upload(p.make_vis())
    rows0, n0, _ = g.search_segment(vis, cap=4096)
    assert n0 > 0
    say("zero capacity")
    rows, n, _ = g.search_segment(vis, cap=0)
    assert n == n0 and len(rows) == 0
    rows, n, _ = g.search_segment(vis, cap=1)
    assert n == n0 and len(rows) == 1


def test_periodic_all_zero(torch):
    p = rfgen.smallcase(nint=32)
    g = gpu_plan(p)
    vis = upload(np.zeros((p.nint, p.nbl, p.nchan, p.npol), np.complex64))
    say("periodic all zero")
    rows, n, st = g.search_periodic(vis, cap=64, with_stats=True)
    assert n == 0 and (st["peak"] == 0).all() and (st["sigma"] == 0).all()
