"""The counter-based noise generator (rfgen.philox) against its published
definitions: Philox4x32-10 known-answer vectors, and the distribution the
Box-Muller transform must give."""
import json
import os

import numpy as np
import pytest
from scipy import stats

from rfgen import philox

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_philox_known_answers():
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.json")) as f:
        kat = json.load(f)["vectors"]
    for v in kat:
        ctr = [np.uint64(int(x, 16)) for x in v["counter"]]
        key = [np.uint64(int(x, 16)) for x in v["key"]]
        out = philox.philox4x32_10(*ctr, *key)
        assert [int(x) for x in out] == [int(x, 16) for x in v["output"]]


def test_box_muller_is_standard_normal():
    """Re and Im each N(0, 1) (Kolmogorov-Smirnov against the normal CDF),
    uncorrelated with each other and between neighbouring elements."""
    z = philox.segment(seed=7, nint=64, nbl=21, nchan=16, npol=2).ravel()
    for part in (z.real.astype(np.float64), z.imag.astype(np.float64)):
        assert stats.kstest(part, "norm").pvalue > 1e-3
        assert abs(part.mean()) < 5 / np.sqrt(part.size)
        assert abs(part.var() - 1) < 0.02
    assert abs(np.corrcoef(z.real, z.imag)[0, 1]) < 0.01
    assert abs(np.corrcoef(z.real[:-1], z.real[1:])[0, 1]) < 0.01


def test_elements_depend_only_on_their_index():
    """A later window of the same stream, or a scattered gather, reproduces
    the same values: the segment can be regenerated piecewise."""
    nbl, nchan, npol = 3, 5, 2   # odd elements per integration: blocks straddle integrations
    full = philox.segment(seed=3, nint=20, nbl=nbl, nchan=nchan, npol=npol)
    part = philox.segment(seed=3, nint=7, nbl=nbl, nchan=nchan, npol=npol, t_first=9)
    assert np.array_equal(part, full[9:16])
    rng = np.random.default_rng(0)
    idx = [rng.integers(0, n, 50) for n in (20, nbl, nchan, npol)]
    assert np.array_equal(philox.gather(3, nbl, nchan, npol, *idx), full[tuple(idx)])


def test_seed_and_stream_change_everything():
    a = philox.segment(seed=1, nint=4, nbl=3, nchan=4, npol=2)
    b = philox.segment(seed=2, nint=4, nbl=3, nchan=4, npol=2)
    c = philox.segment(seed=1, nint=4, nbl=3, nchan=4, npol=2, stream=1)
    d = philox.segment(seed=1 + (1 << 32), nint=4, nbl=3, nchan=4, npol=2)
    for x in (b, c, d):
        assert not np.any(x == a)
