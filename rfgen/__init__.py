"""Seeded synthetic inputs for the realfast search hot path.

This package simulates what an interferometer would hand to the search:
array geometry, channel frequencies, thermal noise and dispersed point-source
pulses.  It is a forward model of the sky and the instrument only; it holds
none of the search's own arithmetic (delay tables, cell indices, resampling,
gridding, imaging or statistics).  Both the CPU oracle and the GPU library
consume the bytes it produces.
"""
from .synth import (  # noqa: F401
    C_LIGHT,
    y_array_positions,
    baseline_uvw,
    channel_centres,
    default_cell_size,
    noise_vis,
    add_pulse,
    pixel_to_lm,
    to_cf16,
    from_cf16,
)
from .presets import (Preset, Pulse, tiny, survey, large, smallcase, serving, batching,  # noqa: F401
                      BATCHING_SEGMENTS, batching_dm_count, preset_by_name)
from . import philox  # noqa: F401
