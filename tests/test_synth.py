"""The seeded input generator: reporting progress leaves the draws alone."""
import dataclasses

import numpy as np

from paper_2111_11682_amd import synth


def test_progress_log_does_not_change_the_draws():
    w = synth.WORKLOADS["nfsmall"]
    w = dataclasses.replace(w, M=40_000, nnz=400_000, n_test=1_000)  # 3 user chunks
    heard = []
    a = synth.generate(w, with_tables=False)
    b = synth.generate(w, with_tables=False, log=heard.append)
    assert a.keys() == b.keys()
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    assert any("split drawn" in m for m in heard) and any("items drawn" in m for m in heard)


def test_large_shape_definition():
    w = synth.WORKLOADS["large1b"]
    assert (w.M, w.N, w.nnz, w.F, w.K, w.G * w.p * w.q, w.p, w.q) == \
        (2_000_000, 500_000, 1_000_000_000, 128, 64, 256, 2, 16)
    assert w.zipf_s == 1.3 and w.rscale == 1
