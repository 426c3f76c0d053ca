"""HIP path vs the FP64 oracle at the full MovieLens-10M shaped size, in the
launch configuration bench.py times (P = 256 strata, needs an MI355X).

69,878 users x 10,677 items, 9.9M training ratings, F = 64, K = 50, 128 hash
bits.  Hash sums, signatures, neighbour lists and the whole stratified stream
must match bit for bit, the neighbour codes of sampled records byte for
byte; one SGD epoch over all ratings within 1e-4 element by element
(tablecmp.py); predictions on sampled pairs within 1e-5; the held-out RMSE
after all 20 epochs within 0.5% of the oracle's.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as orc
from paper_2111_11682_amd import synth
from nbrcodes import expected_codes
from tablecmp import compare_tables

pytestmark = pytest.mark.gpu

SEED_FILL = 12345
_c = {}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _setup():
    if "m" in _c:
        return _c["w"], _c["d"], _c["m"]
    from paper_2111_11682_amd import lshmf
    w = synth.WORKLOADS["ml10m"]
    d = synth.generate(w)
    _say("[gpu] ml10m full size: %d ratings, P=%d" % (d["train_u"].size, w.n_strata))
    m = lshmf.LshMF(w.M, w.N, w.F, w.K, w.G, w.p, w.q, w.rscale, d["train_u"].size, n_strata=w.n_strata)
    dev = m.device
    m.ingest(*[torch.from_numpy(d[k]).to(dev) for k in ("train_u", "train_i", "train_rc")])
    m.set_factors(torch.from_numpy(d["U0"]).to(dev), torch.from_numpy(d["V0"]).to(dev))
    m.build_lsh_neighbours(torch.from_numpy(d["H"].view(np.int32)).to(dev), SEED_FILL)
    torch.cuda.synchronize()
    assert m.device_status() == 0
    _c.update(w=w, d=d, m=m)
    return w, d, m


def _oracle_neighbours():
    if "JK" not in _c:
        w, d = _c["w"], _c["d"]
        acc, sig = orc.simlsh(w.M, w.N, w.B, d["train_u"], d["train_i"], d["train_rc"], d["H"])
        _c["acc"], _c["sig"] = acc, sig
        _c["JK"] = orc.topk(sig, w.B, w.G, w.p, w.q, w.K, SEED_FILL)
    return _c["acc"], _c["sig"], _c["JK"]


def test_fullsize_hash_and_neighbours_bit_exact():
    w, d, m = _setup()
    acc, sig, JK = _oracle_neighbours()
    assert np.array_equal(m.acc.cpu().numpy().astype(np.int64), acc)
    assert np.array_equal(m.sig.cpu().numpy().view(np.uint32), sig)
    assert np.array_equal(m.JK.cpu().numpy(), JK)


def test_fullsize_stream_order_bit_exact():
    w, d, m = _setup()
    P, nnz = w.n_strata, d["train_u"].size
    order, blk = orc.schedule(P, d["train_u"], d["train_i"])
    _c["sched"] = (order, blk)
    lay = m.layout()
    assert np.array_equal(m.arena_view(lay.blk_ptr, P * P + 1, torch.int64).cpu().numpy(), blk)
    pk = m.arena_view(lay.pk, nnz, torch.int32).cpu().numpy().view(np.uint32)
    assert np.array_equal(pk >> 4, d["train_u"][order].astype(np.uint32))
    assert np.array_equal(pk & 15, d["train_rc"][order].astype(np.uint32))
    assert np.array_equal(m.arena_view(lay.sj, nnz, torch.int32).cpu().numpy(), d["train_i"][order])
    # neighbour codes of 300,000 sampled records, every byte
    _, _, JK = _oracle_neighbours()
    x = np.sort(np.random.default_rng(5).choice(nnz, 300_000, replace=False))
    nib = m.arena_view(lay.nib, nnz * lay.nstride, torch.uint8).view(nnz, lay.nstride)
    nib = nib[torch.from_numpy(x).to(m.device)].cpu().numpy()
    assert np.array_equal(nib, expected_codes(w.N, w.K, d["train_u"], d["train_i"], d["train_rc"], order[x],
                                                 JK, lay.nstride))


def test_fullsize_one_epoch_and_predictions():
    w, d, m = _setup()
    _, _, JK = _oracle_neighbours()
    o = orc.Model(w.M, w.N, w.F, w.K, w.rscale, d["train_u"], d["train_i"], d["train_rc"], JK,
                  d["U0"], d["V0"])
    if "sched" in _c:
        o._sched[w.n_strata] = _c["sched"]
    m.sgd_epoch(w.alpha, w.lam, w.beta, 0)
    torch.cuda.synchronize()
    assert m.device_status() == 0
    o.sgd_epoch(w.n_strata, w.alpha, w.lam, w.beta, 0)
    compare_tables({k: (getattr(m, k).double().cpu().numpy().reshape(getattr(o, k).shape), getattr(o, k))
                    for k in ("U", "V", "bu", "bv", "W", "C")}, 1e-4, _say, "ml10m one epoch")
    # Eq. (rr) on sampled pairs, both sides holding the same seeded tables
    rng = np.random.default_rng(17)
    tabs = dict(U=rng.normal(0, 0.3, (w.M, w.F)), V=rng.normal(0, 0.3, (w.N, w.F)),
                W=rng.normal(0, 0.2, (w.N, w.K)), C=rng.normal(0, 0.2, (w.N, w.K)),
                bu=rng.normal(0, 0.1, w.M), bv=rng.normal(0, 0.1, w.N))
    for k, v in tabs.items():
        t32 = v.astype(np.float32)
        getattr(m, k).copy_(torch.from_numpy(t32))
        getattr(o, k)[...] = t32.astype(np.float64).reshape(getattr(o, k).shape)
    qu, qi = synth.random_queries(w.M, w.N, 20000, 3)
    qu = np.concatenate([qu, d["test_u"][:5000]]).astype(np.int32)
    qi = np.concatenate([qi, d["test_i"][:5000]]).astype(np.int32)
    got = m.predict(torch.from_numpy(qu).cuda(), torch.from_numpy(qi).cuda()).cpu().numpy()
    ref = o.predict(qu, qi)
    assert np.all(np.abs(got - ref) <= 1e-5 * np.maximum(1.0, np.abs(ref)))


def test_fullsize_rmse_after_all_epochs():
    # the whole 20-epoch job from the initial tables, both sides
    w, d, m = _setup()
    _, _, JK = _oracle_neighbours()
    dev = m.device
    m.set_factors(torch.from_numpy(d["U0"]).to(dev), torch.from_numpy(d["V0"]).to(dev))
    o = orc.Model(w.M, w.N, w.F, w.K, w.rscale, d["train_u"], d["train_i"], d["train_rc"], JK,
                  d["U0"], d["V0"])
    if "sched" in _c:
        o._sched[w.n_strata] = _c["sched"]
    for t in range(w.epochs):
        m.sgd_epoch(w.alpha, w.lam, w.beta, t)
        o.sgd_epoch(w.n_strata, w.alpha, w.lam, w.beta, t)
    m.check()
    tu, ti, trc = (torch.from_numpy(d[k]).to(dev) for k in ("test_u", "test_i", "test_rc"))
    r_gpu = m.rmse(m.predict(tu, ti), trc).item()
    r_orc = o.rmse(d["test_u"], d["test_i"], d["test_rc"])
    _say("[gpu] ml10m RMSE after %d epochs: gpu %.6f oracle %.6f" % (w.epochs, r_gpu, r_orc))
    assert abs(r_gpu - r_orc) <= 0.005 * r_orc
