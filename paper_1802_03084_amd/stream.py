"""Overlapping segmentation of a visibility stream (section 3.2).

The correlator output is cut into segments of about the inverse fringe rate
(the largest span over which mean-visibility subtraction is accurate), which
overlap so that a dispersed pulse of any allowed sweep lies wholly inside some
segment.  Segment k covers integrations [k step, k step + seg_nint) with
step = seg_nint - overlap; its candidate window is its first `step`
integrations (the last segment's: all of it), so every start time of the
stream lies in exactly one window, and a pulse whose sweep plus box width
fits in the overlap is searched, whole, in the segment whose window holds its
start: each pulse is reported once.
"""


def min_overlap(plan):
    """Integrations a segment must share with the next: the largest
    dispersive delay of the plan plus its widest box."""
    return int(plan.info["max_delay"]) + max(plan.widths)


def segments(n_total, seg_nint, overlap):
    """[(start, t_begin, t_end)] for a stream of n_total integrations: start
    of each segment in the stream, and its candidate window in the segment's
    own integrations.  The stream must hold whole segments:
    n_total = seg_nint + m (seg_nint - overlap) for some m >= 0."""
    step = seg_nint - overlap
    if not 0 <= overlap < seg_nint:
        raise ValueError("need 0 <= overlap < seg_nint")
    if n_total < seg_nint or (n_total - seg_nint) % step:
        raise ValueError("the stream must hold whole segments")
    n = (n_total - seg_nint) // step + 1
    return [(k * step, 0, step if k < n - 1 else seg_nint) for k in range(n)]
