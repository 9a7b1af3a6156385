"""rf_image_static, the entry point that allocates nothing (its scratch is a
fixed array of the library on each GPU), against rf_image with a caller
workspace: identical images, bit for bit, on two calls in a row, the second
with a smaller input; an input larger than the fixed scratch is rejected
before anything is enqueued."""
import ctypes
import sys

import numpy as np
import pytest

import rfgen
from helpers import gpu_plan, upload

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _preset(n, nint):
    if n == 1024:
        return rfgen.Preset(name="survey-band", nant=27, nint=nint, tint_s=0.010, f_lo_ghz=1.0,
                            f_hi_ghz=2.0, nchan=256, npol=2, dms=np.array([0.0]), widths=[1],
                            npix=n, seed=17)
    return rfgen.Preset(name="large-band", nant=27, nint=nint, tint_s=0.001, f_lo_ghz=2.0,
                        f_hi_ghz=4.0, nchan=1024, npol=2, dms=np.array([0.0]), widths=[1],
                        npix=n, seed=18)


@pytest.mark.parametrize("n,first,second", [(1024, 8, 3), (2048, 4, 1)])
def test_image_static_equals_image(torch, n, first, second):
    from paper_1802_03084_amd import _lib
    L = _lib.load()
    p = _preset(n, first)
    g = gpu_plan(p)
    grid = g.grid(upload(p.make_vis()))
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    for nimg in (first, second):
        say(f"rf_image_static {n}^2, {nimg} images")
        gin = grid[:nimg].contiguous()
        ref = g.image(gin)
        out = torch.full_like(ref, float("nan"))
        st = L.rf_image_static(g.handle, ptr(gin), nimg, ptr(out), stream)
        assert st == 0, _lib.status_string(st)
        torch.cuda.synchronize()
        assert torch.equal(out.view(torch.int32), ref.view(torch.int32)), nimg


def test_image_static_rejects_more_than_its_scratch(torch):
    from paper_1802_03084_amd import _lib
    L = _lib.load()
    p = _preset(2048, 1)
    g = gpu_plan(p)
    cap = ctypes.c_size_t()
    assert L.rf_image_static_max_bytes(ctypes.byref(cap)) == 0
    per_pair = g.info["n_rows"] * p.npix * 8
    too_many = 2 * (cap.value // per_pair) + 2
    dummy = torch.empty(16, dtype=torch.float32, device="cuda")
    st = L.rf_image_static(g.handle, ctypes.c_void_p(dummy.data_ptr()), too_many,
                           ctypes.c_void_p(dummy.data_ptr()), None)
    assert st == _lib.RF_EWORKSPACE
    assert L.rf_image_static(g.handle, ctypes.c_void_p(dummy.data_ptr()), -1,
                             ctypes.c_void_p(dummy.data_ptr()), None) == -3
    assert L.rf_image_static(None, None, 1, None, None) == -1
