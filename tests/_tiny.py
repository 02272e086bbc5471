"""Hand-built tiny lines for closed-form checks of the oracle."""
import numpy as np

import oracle


def line(traces, cmp_sizes, offsets, dt=0.004, dx=12.5, window=5, op=1, ap=0):
    traces = np.asarray(traces, dtype=np.float64)
    cmp_ptr = np.concatenate([[0], np.cumsum(cmp_sizes)]).astype(np.int64)
    return oracle.Line(traces, cmp_ptr, np.asarray(offsets, dtype=np.float64), dt, dx, window,
                       op, ap, ap)
