"""End-to-end oracle search on synthetic workloads: injected dispersed pulses
(the paper's own testing idea, section 3.3 mock sources) are recovered at the
DM trial, width, time and pixel they were injected with."""
import json
import os

import numpy as np
import pytest

import oracle
import rfgen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def plan_of(p):
    du, dv = p.cell()
    return oracle.Plan(p.freq(), p.uvw(), p.tint_s, p.dms, p.widths, p.npix, du, dv,
                       kdm=p.kdm, threshold=p.threshold, t_begin=p.t_begin, t_end=p.t_end,
                       nint=p.nint)


def test_tiny_recovers_injected_pulse():
    p = rfgen.tiny()
    plan = plan_of(p)
    _, cands, _ = oracle.search(p.make_vis(), plan)
    pulse = p.pulses[0]
    assert [c[:5] for c in cands] == [(pulse.dm_idx, pulse.width_idx, pulse.t0, pulse.x, pulse.y)]
    assert cands[0][5] > 10.0


def test_tiny_matches_stored_oracle_values():
    with open(os.path.join(GOLDEN, "tiny_oracle.json")) as f:
        gold = json.load(f)
    p = rfgen.tiny()
    plan = plan_of(p)
    stats, cands, _ = oracle.search(p.make_vis(), plan)
    assert plan.W == gold["W"]
    assert plan.delays.tolist() == gold["delays"]
    assert [list(c[:5]) for c in cands] == [c[:5] for c in gold["candidates"]]
    for key, v in gold["stats"].items():
        i, j, k = map(int, key.split(","))
        got = stats[(i, j, k)]
        assert got[1:3] == tuple(v[1:3])
        assert np.allclose(got[0::3][:1] + got[3:], [v[0]] + v[3:], rtol=1e-12)


def test_tiny_noise_only_has_no_candidates():
    p = rfgen.tiny()
    _, cands, _ = oracle.search(p.make_vis(with_pulses=False), plan_of(p))
    assert cands == []


def test_small_ragged_recovers_pulse():
    p = rfgen.smallcase()
    _, cands, _ = oracle.search(p.make_vis(), plan_of(p))
    pulse = p.pulses[0]
    keys = [c[:5] for c in cands]
    w = p.widths[pulse.width_idx]
    assert (pulse.dm_idx, pulse.width_idx, pulse.t0, pulse.x, pulse.y) in keys, keys
    assert w == 2


def test_search_window_excludes_candidates():
    p = rfgen.tiny()
    plan = plan_of(p)
    plan.t_begin = 1
    _, cands, _ = oracle.search(p.make_vis(), plan)
    assert cands == []


def test_cf16_storage_is_widened_exactly():
    p = rfgen.smallcase()
    v = p.make_vis()
    v16 = rfgen.to_cf16(v)
    z = oracle.as_complex(v16)
    assert z.dtype == np.complex128
    assert np.array_equal(z.real, v16[..., 0].astype(np.float64))


@pytest.mark.parametrize("preset", ["tiny", "small"])
def test_image_at_equals_search_on_every_key(preset):
    """The windowed image (used to sample single images of segments too large
    to search whole on the CPU) equals the whole-segment search's image bit
    for bit on every key of the tiny and small workloads: trials whose delays
    pass the segment end (tiny: up to 91 integrations against 32) and the
    last box of the widest width included."""
    p = rfgen.preset_by_name(preset)
    plan = plan_of(p)
    vis = p.make_vis()
    stats, _, images = oracle.search(vis, plan, keep_images=True)
    if preset == "tiny":
        assert plan.delays.max() > p.nint
    assert len(images) == p.n_images()
    for (i, j, k), img in images.items():
        got = oracle.image_at(vis, plan, i, j, k)
        assert np.array_equal(got, img), (i, j, k)
        assert oracle.image_stats(got) == stats[(i, j, k)]
