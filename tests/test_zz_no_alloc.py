"""lshmf_rmse_noalloc (no context, no allocation) against lshmf_rmse on the GPU.

Two calls in a row, the second on a smaller input, so that the second call
runs on the partial sums the first left in the library's fixed array: each
result must equal lshmf_rmse's bit for bit (same kernels, same fixed
reduction order) and the FP64 definition of the RMSE (Sec. 5.1) within 1e-12
relative.  Also n = 0 and the argument checks.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2111_11682_amd import lshmf, synth

pytestmark = pytest.mark.gpu


def _rmse_def(pred, rc, rscale):
    d = rc.astype(np.float64) / rscale - pred.astype(np.float64)
    return float(np.sqrt(np.mean(d * d))) if d.size else 0.0


def _case(m, n, rscale, seed, dev):
    rng = np.random.default_rng(seed)
    pred = rng.uniform(0.0, 5.5, n).astype(np.float32)
    rc = rng.integers(1, 5 * rscale + 1, n).astype(np.uint8)
    tp, tr = torch.from_numpy(pred).to(dev), torch.from_numpy(rc).to(dev)
    got = torch.full((1,), -1.0, dtype=torch.float64, device=dev)
    lshmf.rmse_noalloc(tp, tr, rscale, got)
    ref = m.rmse(tp, tr)
    torch.cuda.synchronize(dev)
    g, r = got.item(), ref.item()
    print("[gpu] rmse_noalloc n=%d rscale=%d: %.17g (lshmf_rmse %.17g)" % (n, rscale, g, r), flush=True)
    assert g == r, (g, r)
    want = _rmse_def(pred, rc, rscale)
    assert abs(g - want) <= 1e-12 * max(want, 1e-300)


def test_rmse_noalloc_matches_lshmf_rmse_twice_then_smaller():
    w = synth.WORKLOADS["small"]  # half-step ratings: rscale 2
    m = lshmf.LshMF(w.M, w.N, w.F, w.K, w.G, w.p, w.q, w.rscale, 1000, n_strata=w.n_strata)
    dev = m.device
    try:
        _case(m, 300_001, w.rscale, 1, dev)   # several grid passes and a ragged tail
        _case(m, 1_000, w.rscale, 2, dev)     # smaller: most partials now from empty blocks
        _case(m, 0, w.rscale, 3, dev)
    finally:
        m.close()


def test_rmse_noalloc_rejects_bad_arguments():
    dev = torch.device("cuda:0")
    pred = torch.zeros(4, dtype=torch.float32, device=dev)
    rc = torch.ones(4, dtype=torch.uint8, device=dev)
    out = torch.zeros(1, dtype=torch.float64, device=dev)
    L = lshmf.lib()
    s = lshmf._stream(dev)
    assert L.lshmf_rmse_noalloc(lshmf._ptr(pred), lshmf._ptr(rc), 4, 3, lshmf._ptr(out), s) == -1
    assert L.lshmf_rmse_noalloc(lshmf._ptr(pred), lshmf._ptr(rc), -1, 1, lshmf._ptr(out), s) == -1
    assert L.lshmf_rmse_noalloc(lshmf._ptr(pred), lshmf._ptr(rc), 4, 1, None, s) == -1
    assert L.lshmf_rmse_noalloc(None, lshmf._ptr(rc), 4, 1, lshmf._ptr(out), s) == -1
