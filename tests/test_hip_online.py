"""Online learning (Sec. 4.3) on the HIP path vs the FP64 oracle (needs an MI355X).

A model is pre-trained on the ratings of the older users and items, then a
stream of batches arrives: ratings of new users, on new items, and further
ratings between existing ones.  Hash sums, signatures and neighbour lists must
match the oracle bit for bit; the fixed baselines of new ids within FP32
rounding; the learned tables within 1e-4 normwise relative after the online
passes and after a further epoch over the grown training set.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as orc
from paper_2111_11682_amd import synth

pytestmark = pytest.mark.gpu

SEED_FILL = 0x0DDB_A11


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(g, r):
    return float(np.abs(g - r).max() / max(np.abs(r).max(), 1e-3)) if r.size else 0.0


def _split_batches(sp, nb, M, N):
    """Batch k brings the k-th share of the new users and items (by id) and an
    even share of the remaining ratings, in stream order."""
    su, si, src = sp["stream_u"], sp["stream_i"], sp["stream_rc"]
    M0, N0 = int(sp["M_old"]), int(sp["N_old"])
    gu = np.where(su >= M0, (su - M0 + 1) / (M - M0), 0.0)
    gi = np.where(si >= N0, (si - N0 + 1) / (N - N0), 0.0)
    g = np.maximum(gu, gi)
    k = np.where(g > 0, np.ceil(g * nb) - 1, np.arange(su.size) % nb).astype(np.int64)
    return [(su[k == b], si[k == b], src[k == b]) for b in range(nb)]


def _setup(name, frac_new, stream_frac, nb, passes):
    from paper_2111_11682_amd import lshmf
    w = synth.WORKLOADS[name]
    d = synth.generate(w)
    sp = synth.online_split(w, d, frac_new=frac_new, stream_frac=stream_frac)
    M0, N0 = int(sp["M_old"]), int(sp["N_old"])
    pu, pi, prc = sp["pretrain_u"], sp["pretrain_i"], sp["pretrain_rc"]
    batches = _split_batches(sp, nb, w.M, w.N)
    P = w.n_strata
    _say("[gpu] online %s: %d x %d pre-trained on %d ratings, %d batches of ~%d"
         % (name, M0, N0, pu.size, nb, batches[0][0].size))

    # oracle: pre-train one epoch on the old ratings
    acc, sig = orc.simlsh(M0, N0, w.B, pu, pi, prc, d["H"][:M0])
    JK = orc.topk(sig, w.B, w.G, w.p, w.q, w.K, SEED_FILL)
    o = orc.Model(M0, N0, w.F, w.K, w.rscale, pu, pi, prc, JK, d["U0"][:M0], d["V0"][:N0])
    o.sgd_epoch(P, w.alpha, w.lam, w.beta, 0)

    # GPU: the same, with room for the whole stream
    m = lshmf.LshMF(M0, N0, w.F, w.K, w.G, w.p, w.q, w.rscale, pu.size, n_strata=P,
                    M_cap=w.M, N_cap=w.N, nnz_cap=d["train_u"].size + 64,
                    batch_cap=max(b[0].size for b in batches))
    dev = m.device
    m.ingest(*[torch.from_numpy(a).to(dev) for a in (pu, pi, prc)])
    m.set_factors(torch.from_numpy(d["U0"][:M0]).to(dev), torch.from_numpy(d["V0"][:N0]).to(dev))
    H = torch.from_numpy(d["H"].view(np.int32)).to(dev)
    m.build_lsh_neighbours(H, SEED_FILL)
    m.sgd_epoch(w.alpha, w.lam, w.beta, 0)
    torch.cuda.synchronize()
    assert m.device_status() == 0

    Mc, Nc = M0, N0
    for k, (bu_, bi_, brc) in enumerate(batches):
        Mn = max(Mc, int(bu_.max()) + 1)
        Nn = max(Nc, int(bi_.max()) + 1)
        o, acc, sig = orc.online_update(o, acc, sig, w.B, w.G, w.p, w.q, SEED_FILL, bu_, bi_, brc,
                                        d["H"][:Mn], d["U0"][Mc:Mn], d["V0"][Nc:Nn], P, w.alpha,
                                        w.lam, w.beta, 1 + k, passes)
        m.online_update(*[torch.from_numpy(a).to(dev) for a in (bu_, bi_, brc)], Mn, Nn, H,
                        SEED_FILL, w.alpha, w.lam, w.beta, 1 + k, passes,
                        U_new=torch.from_numpy(d["U0"][Mc:Mn]).to(dev),
                        V_new=torch.from_numpy(d["V0"][Nc:Nn]).to(dev))
        torch.cuda.synchronize()
        assert m.device_status() == 0
        Mc, Nc = Mn, Nn
    return w, d, m, o, acc, sig, Mc, Nc


def _check_state(m, o, acc, sig, Mc, Nc, tol):
    lay = m.layout()
    assert (lay.M, lay.N, lay.nnz) == (Mc, Nc, o.u.size)
    assert np.array_equal(m.acc[:Nc].cpu().numpy().astype(np.int64), acc)
    assert np.array_equal(m.sig[:Nc].cpu().numpy().view(np.uint32), sig)
    assert np.array_equal(m.JK[:Nc].cpu().numpy(), o.JK)
    assert m.mu.item() == pytest.approx(o.mu, rel=1e-12)
    for k in ("b0", "bh0"):
        g = getattr(m, k)[: (Mc if k == "b0" else Nc)].double().cpu().numpy()
        assert np.all(np.abs(g - getattr(o, k)) <= 1e-6), k
    worst = {}
    for k in ("U", "V", "bu", "bv", "W", "C"):
        r = getattr(o, k)
        g = getattr(m, k)[: r.shape[0]].double().cpu().numpy().reshape(r.shape)
        worst[k] = _rel(g, r)
    assert all(v <= tol for v in worst.values()), worst
    return worst


@pytest.mark.parametrize("name,nb,passes", [("tiny", 2, 1), ("small", 3, 2), ("ml100k", 2, 1), ("nfsmall", 2, 1), ("wide", 2, 1)])
def test_online_update_parity(name, nb, passes):
    w, d, m, o, acc, sig, Mc, Nc = _setup(name, 0.03, 0.2, nb, passes)
    worst = _check_state(m, o, acc, sig, Mc, Nc, 1e-4)
    _say("[gpu] online %s after batches: worst rel %s" % (name, worst))
    # predictions on the grown model, including new users and items
    qu, qi = synth.random_queries(Mc, Nc, 3000, 5)
    got = m.predict(torch.from_numpy(qu).cuda(), torch.from_numpy(qi).cuda()).cpu().numpy()
    ref = o.predict(qu, qi)
    assert np.all(np.abs(got - ref) <= 1e-4 * np.maximum(1.0, np.abs(ref)))
    # a further epoch over the grown training set (the stream is laid out again)
    m.sgd_epoch(w.alpha, w.lam, w.beta, 1 + nb)
    o.sgd_epoch(w.n_strata, w.alpha, w.lam, w.beta, 1 + nb)
    torch.cuda.synchronize()
    assert m.device_status() == 0
    worst = _check_state(m, o, acc, sig, Mc, Nc, 2e-4)
    _say("[gpu] online %s after a further epoch: worst rel %s" % (name, worst))
    lay = m.layout()
    P = w.n_strata
    order, blk = orc.schedule(P, o.u, o.i)
    sj = m.arena_view(lay.sj, o.u.size, torch.int32).cpu().numpy()
    assert np.array_equal(m.arena_view(lay.blk_ptr, P * P + 1, torch.int64).cpu().numpy(), blk)
    assert np.array_equal(sj, o.i[order])


def test_online_update_rejects_and_leaves_state():
    from paper_2111_11682_amd import lshmf
    w, d, m, o, acc, sig, Mc, Nc = _setup("tiny", 0.03, 0.2, 1, 1)
    before = [getattr(m, k).clone() for k in ("U", "V", "bu", "bv", "W", "C", "JK", "acc")]
    H = torch.from_numpy(d["H"].view(np.int32)).cuda()
    u = torch.tensor([0, Mc], dtype=torch.int32, device="cuda")   # user Mc is beyond M_new = Mc
    i = torch.tensor([0, 1], dtype=torch.int32, device="cuda")
    rc = torch.tensor([3, 4], dtype=torch.uint8, device="cuda")
    with pytest.raises(lshmf.LshmfError) as ei:
        m.online_update(u, i, rc, Mc, Nc, H, SEED_FILL, w.alpha, w.lam, w.beta, 5)
    assert ei.value.status == -1
    big = m.dims.batch_cap + 1
    z = torch.zeros(big, dtype=torch.int32, device="cuda")
    with pytest.raises(lshmf.LshmfError) as ei:
        m.online_update(z, z, torch.ones(big, dtype=torch.uint8, device="cuda"), Mc, Nc, H,
                        SEED_FILL, w.alpha, w.lam, w.beta, 5)
    assert ei.value.status == -3
    with pytest.raises(lshmf.LshmfError) as ei:
        m.online_update(u[:1], i[:1], rc[:1], Mc, w.N + 1, H, SEED_FILL, w.alpha, w.lam, w.beta, 5,
                        V_new=torch.zeros(w.N + 1 - Nc, w.F, device="cuda"))
    assert ei.value.status == -3
    torch.cuda.synchronize()
    for a, k in zip(before, ("U", "V", "bu", "bv", "W", "C", "JK", "acc")):
        assert torch.equal(a, getattr(m, k)), k
    # the model still trains
    m.sgd_epoch(w.alpha, w.lam, w.beta, 6)
    torch.cuda.synchronize()
    assert m.device_status() == 0
