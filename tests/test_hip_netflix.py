"""HIP path vs the FP64 oracle at the full Netflix shape (needs an MI355X).

480,189 users x 17,770 items, 98,591,605 training ratings, F = 128, K = 100,
128 hash bits, in the launch configuration bench.py times (1,536 strata),
storage mode BF16 (FP32 masters, BF16 copies that predict reads), then again
with the user rows stored in BF16 only (storage BF16_U).  Hash sums,
signatures and neighbour lists bit for bit, neighbour codes of sampled
records byte for byte; one SGD epoch over all ratings
within 1e-4 element by element (tablecmp.py); held-out RMSE after that epoch,
predicted from the BF16 copies, within 0.5% of the FP64 oracle's, in both
storage modes.
"""
import sys
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as orc
from paper_2111_11682_amd import synth
from nbrcodes import expected_codes
from tablecmp import compare_tables

pytestmark = pytest.mark.gpu

SEED_FILL = 12345


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_netflix_shape_neighbours_epoch_and_bf16_rmse():
    from paper_2111_11682_amd import lshmf
    w = synth.WORKLOADS["netflix"]
    t0 = time.time()
    d = synth.generate(w)
    _say("[gpu] netflix shape: %d train ratings generated in %.0f s" % (d["train_u"].size, time.time() - t0))
    m = lshmf.LshMF(w.M, w.N, w.F, w.K, w.G, w.p, w.q, w.rscale, d["train_u"].size,
                    n_strata=w.n_strata, storage="bf16")
    dev = m.device
    m.ingest(*[torch.from_numpy(d[k]).to(dev) for k in ("train_u", "train_i", "train_rc")])
    m.set_factors(torch.from_numpy(d["U0"]).to(dev), torch.from_numpy(d["V0"]).to(dev))
    m.build_lsh_neighbours(torch.from_numpy(d["H"].view(np.int32)).to(dev), SEED_FILL)
    m.sgd_epoch(w.alpha, w.lam, w.beta, 0)
    m.check()
    _say("[gpu] netflix GPU epoch done; oracle hashing")
    acc, sig = orc.simlsh(w.M, w.N, w.B, d["train_u"], d["train_i"], d["train_rc"], d["H"])
    assert np.array_equal(m.acc.cpu().numpy().astype(np.int64), acc)
    assert np.array_equal(m.sig.cpu().numpy().view(np.uint32), sig)
    del acc
    JK = orc.topk(sig, w.B, w.G, w.p, w.q, w.K, SEED_FILL)
    assert np.array_equal(m.JK.cpu().numpy(), JK)
    _say("[gpu] netflix neighbours bit-exact; oracle epoch")
    t0 = time.time()
    o = orc.Model(w.M, w.N, w.F, w.K, w.rscale, d["train_u"], d["train_i"], d["train_rc"], JK,
                  d["U0"], d["V0"])
    o.sgd_epoch(w.n_strata, w.alpha, w.lam, w.beta, 0)
    _say("[gpu] netflix oracle epoch in %.0f s" % (time.time() - t0))
    # neighbour codes of 200,000 sampled records, every byte
    n = d["train_u"].size
    lay = m.layout()
    x = np.sort(np.random.default_rng(5).choice(n, 200_000, replace=False))
    nib = m.arena_view(lay.nib, n * lay.nstride, torch.uint8).view(n, lay.nstride)
    nib = nib[torch.from_numpy(x).to(dev)].cpu().numpy()
    order = o._sched[w.n_strata][0]
    assert np.array_equal(nib, expected_codes(w.N, w.K, d["train_u"], d["train_i"], d["train_rc"], order[x],
                                                 JK, lay.nstride))
    compare_tables({k: (getattr(m, k).double().cpu().numpy().reshape(getattr(o, k).shape), getattr(o, k))
                    for k in ("U", "V", "bu", "bv", "W", "C")}, 1e-4, _say, "netflix one epoch")
    tu, ti, trc = (torch.from_numpy(d[k]).to(dev) for k in ("test_u", "test_i", "test_rc"))
    r_gpu = m.rmse(m.predict(tu, ti), trc).item()
    r_orc = o.rmse(d["test_u"], d["test_i"], d["test_rc"])
    _say("[gpu] netflix RMSE after one epoch: gpu (BF16 copies) %.6f oracle (FP64) %.6f" % (r_gpu, r_orc))
    assert abs(r_gpu - r_orc) <= 0.005 * r_orc
    m.close()
    # the same epoch with the user rows stored in BF16 only (storage BF16_U)
    m2 = lshmf.LshMF(w.M, w.N, w.F, w.K, w.G, w.p, w.q, w.rscale, d["train_u"].size,
                     n_strata=w.n_strata, storage="bf16u")
    m2.ingest(*[torch.from_numpy(d[k]).to(dev) for k in ("train_u", "train_i", "train_rc")])
    m2.set_factors(torch.from_numpy(d["U0"]).to(dev), torch.from_numpy(d["V0"]).to(dev))
    m2.build_lsh_neighbours(torch.from_numpy(d["H"].view(np.int32)).to(dev), SEED_FILL)
    m2.sgd_epoch(w.alpha, w.lam, w.beta, 0)
    m2.check()
    r16 = m2.rmse(m2.predict(tu, ti), trc).item()
    _say("[gpu] netflix RMSE after one epoch, user rows in BF16 only: gpu %.6f oracle (FP64) %.6f" % (r16, r_orc))
    assert abs(r16 - r_orc) <= 0.005 * r_orc
