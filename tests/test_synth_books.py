"""The books generator gives its spine edges exactly the requested number of
triangles (the property the sweep-bin parity cases rely on).  CPU only."""

import numpy as np

import oracle
from synth import books


def test_spines_have_the_requested_triangles():
    pages = (5, 9, 300)
    raw = books(pages=pages, page_degree=4.0, seed=3)
    g = oracle.Graph.from_raw(raw)
    edges = g.rcliques(2)
    ds = g.sdeg(2, 3)
    base = 0
    for p in pages:
        spine = np.nonzero((edges[:, 0] == base) & (edges[:, 1] == base + 1))[0]
        assert spine.size == 1 and ds[spine[0]] == p
        # the spine's endpoints see every page of their book and each other
        row_off, col = g.csr()
        assert row_off[base + 1] - row_off[base] == p + 1
        base += 2 + p
    assert base == raw.n
