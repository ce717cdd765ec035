"""Host check of an assumption the kernels rely on: the quotient i / d computed as
trunc((float(i) + 0.5f) * (1.0f / d)) in IEEE single precision (round to nearest) is exact
over the ranges the kernels use it on (window cells of the largest windows, thread indices,
footprint widths)."""
import numpy as np


def test_float_reciprocal_quotient_is_exact():
    i = np.arange(1 << 21, dtype=np.int64)
    fi = i.astype(np.float32) + np.float32(0.5)
    for d in range(1, 161):
        inv = np.float32(1.0) / np.float32(d)
        q = (fi * inv).astype(np.int64)
        assert np.array_equal(q, i // d), d
