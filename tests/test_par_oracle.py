"""The threaded range split of the oracle's sweep (a test helper) gives what
one call over the whole range gives."""
import numpy as np

import oracle as O
import par_oracle as P
from paper_2605_14743_amd import workloads as W


def test_ranges_combine_exactly():
    wl = W.config_er20()
    g = wl.graph
    pool = np.array([1, 4, 9, 15])
    kw = dict(seed=3, R=157, r_begin=40, alpha=wl.alpha, k_min=wl.k_min, want_next=True, pool=pool, topk=3,
              **wl.model())
    one = O.sweep(g.n, g.eu, g.ev, **kw)
    par = P.sweep(g.n, g.eu, g.ev, parts=6, **kw)
    for key in ("counts", "counts_w", "center_global", "next_table", "next_table_w"):
        assert np.array_equal(one[key], par[key]), key
    for key in ("bsum", "psi", "psi_w"):
        assert np.allclose(one[key], par[key], rtol=1e-13, atol=0), key
    assert one["stats"] == par["stats"]
