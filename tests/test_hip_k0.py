"""K = 0 on the HIP path vs the FP64 oracle (needs an MI355X).

With K = 0 the model is biased MF without the neighbour term: Eq. (rr) keeps
mu + b_i + bh_j + u_i . v_j and Eq. (sgd_update) moves only b, bh, u, v.  The
same kernels run it; the bars are those of the K > 0 parity tests: hash sums
and signatures bit for bit, predictions within 1e-5 relative, one epoch within
1e-4 element by element (tablecmp.py), held-out RMSE within 0.5%.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as orc
from paper_2111_11682_amd import synth
from tablecmp import compare_tables

pytestmark = pytest.mark.gpu

SEED_FILL = 0x5EED_F111


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _models(name, P=None):
    from paper_2111_11682_amd import lshmf
    w = synth.WORKLOADS[name]
    assert w.K == 0
    d = synth.generate(w)
    P = P or w.n_strata
    _say("[gpu] K=0 model %s P=%d nnz=%d" % (name, P, d["train_u"].size))
    m = lshmf.LshMF(w.M, w.N, w.F, 0, w.G, w.p, w.q, w.rscale, d["train_u"].size, n_strata=P)
    dev = m.device
    m.ingest(*[torch.from_numpy(d[k]).to(dev) for k in ("train_u", "train_i", "train_rc")])
    m.set_factors(torch.from_numpy(d["U0"]).to(dev), torch.from_numpy(d["V0"]).to(dev))
    m.build_lsh_neighbours(torch.from_numpy(d["H"].view(np.int32)).to(dev), SEED_FILL)
    torch.cuda.synchronize()
    assert m.device_status() == 0
    o = orc.Model(w.M, w.N, w.F, 0, w.rscale, d["train_u"], d["train_i"], d["train_rc"],
                  np.zeros((w.N, 0), np.int32), d["U0"], d["V0"])
    return w, d, m, o


def _worst(m, o, label):
    return compare_tables({k: (getattr(m, k).double().cpu().numpy().reshape(getattr(o, k).shape), getattr(o, k))
                           for k in ("U", "V", "bu", "bv")}, 1e-4, _say, label)


@pytest.mark.parametrize("name", ["tiny_k0", "ml100k_k0"])
def test_k0_hash_and_predict(name):
    w, d, m, o = _models(name)
    acc, sig = orc.simlsh(w.M, w.N, w.B, d["train_u"], d["train_i"], d["train_rc"], d["H"])
    assert np.array_equal(m.acc.cpu().numpy().astype(np.int64), acc)
    assert np.array_equal(m.sig.cpu().numpy().view(np.uint32), sig)
    rng = np.random.default_rng(3)
    for k, shape in (("U", (w.M, w.F)), ("V", (w.N, w.F)), ("bu", (w.M,)), ("bv", (w.N,))):
        v = rng.normal(scale=0.3, size=shape).astype(np.float32)
        getattr(m, k).copy_(torch.from_numpy(v))
        getattr(o, k)[...] = v.astype(np.float64)
    qu, qi = synth.random_queries(w.M, w.N, 4000, 7)
    got = m.predict(torch.from_numpy(qu).cuda(), torch.from_numpy(qi).cuda()).cpu().numpy()
    ref = o.predict(qu, qi)
    assert np.all(np.abs(got - ref) <= 1e-5 * np.maximum(1.0, np.abs(ref)))


@pytest.mark.parametrize("name", ["tiny_k0", "ml100k_k0"])
def test_k0_one_epoch_parity(name):
    w, d, m, o = _models(name)
    m.sgd_epoch(w.alpha, w.lam, w.beta, 0)
    torch.cuda.synchronize()
    assert m.device_status() == 0
    o.sgd_epoch(w.n_strata, w.alpha, w.lam, w.beta, 0)
    _worst(m, o, "K=0 one epoch " + name)


def test_k0_full_run_rmse_ml100k():
    w, d, m, o = _models("ml100k_k0")
    for t in range(w.epochs):
        m.sgd_epoch(w.alpha, w.lam, w.beta, t)
        o.sgd_epoch(w.n_strata, w.alpha, w.lam, w.beta, t)
    torch.cuda.synchronize()
    assert m.device_status() == 0
    pred = m.predict(torch.from_numpy(d["test_u"]).cuda(), torch.from_numpy(d["test_i"]).cuda())
    r_gpu = m.rmse(pred, torch.from_numpy(d["test_rc"]).cuda()).item()
    r_orc = o.rmse(d["test_u"], d["test_i"], d["test_rc"])
    _say("[gpu] ml100k K=0 RMSE gpu %.6f oracle %.6f" % (r_gpu, r_orc))
    assert abs(r_gpu - r_orc) <= 0.005 * r_orc


def test_k0_bf16_copies():
    # K = 0 with BF16 storage: no W16 / C16 to keep; U16, V16 are the RNE
    # images of the masters after an epoch, and the masters equal FP32 mode's
    from paper_2111_11682_amd import lshmf
    w = synth.WORKLOADS["ml100k_k0"]
    d = synth.generate(w)
    runs = {}
    for storage in ("fp32", "bf16"):
        m = lshmf.LshMF(w.M, w.N, w.F, 0, w.G, w.p, w.q, w.rscale, d["train_u"].size,
                        n_strata=w.n_strata, storage=storage)
        dev = m.device
        m.ingest(*[torch.from_numpy(d[k]).to(dev) for k in ("train_u", "train_i", "train_rc")])
        m.set_factors(torch.from_numpy(d["U0"]).to(dev), torch.from_numpy(d["V0"]).to(dev))
        m.build_lsh_neighbours(torch.from_numpy(d["H"].view(np.int32)).to(dev), SEED_FILL)
        m.sgd_epoch(w.alpha, w.lam, w.beta, 0)
        torch.cuda.synchronize()
        assert m.device_status() == 0
        runs[storage] = m
    a, b = runs["fp32"], runs["bf16"]
    assert torch.equal(a.U, b.U) and torch.equal(a.V, b.V)
    for master, copy in ((b.U, b.U16), (b.V, b.V16)):
        assert torch.equal(copy.cpu().view(torch.int16), master.cpu().to(torch.bfloat16).view(torch.int16))


def test_k0_online_update():
    from paper_2111_11682_amd import lshmf
    w = synth.WORKLOADS["tiny_k0"]
    d = synth.generate(w)
    sp = synth.online_split(w, d, frac_new=0.03, stream_frac=0.2)
    M0, N0 = int(sp["M_old"]), int(sp["N_old"])
    pu, pi, prc = sp["pretrain_u"], sp["pretrain_i"], sp["pretrain_rc"]
    su, si, src = sp["stream_u"], sp["stream_i"], sp["stream_rc"]
    P = w.n_strata
    acc, sig = orc.simlsh(M0, N0, w.B, pu, pi, prc, d["H"][:M0])
    o = orc.Model(M0, N0, w.F, 0, w.rscale, pu, pi, prc, np.zeros((N0, 0), np.int32),
                  d["U0"][:M0], d["V0"][:N0])
    o.sgd_epoch(P, w.alpha, w.lam, w.beta, 0)
    m = lshmf.LshMF(M0, N0, w.F, 0, w.G, w.p, w.q, w.rscale, pu.size, n_strata=P,
                    M_cap=w.M, N_cap=w.N, nnz_cap=d["train_u"].size + 64, batch_cap=su.size)
    dev = m.device
    m.ingest(*[torch.from_numpy(a).to(dev) for a in (pu, pi, prc)])
    m.set_factors(torch.from_numpy(d["U0"][:M0]).to(dev), torch.from_numpy(d["V0"][:N0]).to(dev))
    H = torch.from_numpy(d["H"].view(np.int32)).to(dev)
    m.build_lsh_neighbours(H, SEED_FILL)
    m.sgd_epoch(w.alpha, w.lam, w.beta, 0)
    Mn, Nn = max(M0, int(su.max()) + 1), max(N0, int(si.max()) + 1)
    _say("[gpu] K=0 online tiny: batch of %d, %d new users, %d new items" % (su.size, Mn - M0, Nn - N0))
    o, acc, sig = orc.online_update(o, acc, sig, w.B, w.G, w.p, w.q, SEED_FILL, su, si, src,
                                    d["H"][:Mn], d["U0"][M0:Mn], d["V0"][N0:Nn], P, w.alpha,
                                    w.lam, w.beta, 1, 1)
    m.online_update(*[torch.from_numpy(a).to(dev) for a in (su, si, src)], Mn, Nn, H, SEED_FILL,
                    w.alpha, w.lam, w.beta, 1, 1, U_new=torch.from_numpy(d["U0"][M0:Mn]).to(dev),
                    V_new=torch.from_numpy(d["V0"][N0:Nn]).to(dev))
    torch.cuda.synchronize()
    assert m.device_status() == 0
    assert np.array_equal(m.acc[:Nn].cpu().numpy().astype(np.int64), acc)
    assert np.array_equal(m.sig[:Nn].cpu().numpy().view(np.uint32), sig)
    compare_tables({k: (getattr(m, k)[: getattr(o, k).shape[0]].double().cpu().numpy().reshape(getattr(o, k).shape),
                        getattr(o, k)) for k in ("U", "V", "bu", "bv")}, 1e-4, _say, "K=0 online")


def test_plain_mf_cusgd_parity():
    # Alg. CUSGD++'s model: rhat = u . v, only U and V learned (LSHMF_PLAIN_MF).
    # The oracle runs the same as K = 0 with mu, b0, bh0 and the bias rates zero.
    from paper_2111_11682_amd import lshmf
    w = synth.WORKLOADS["ml100k_k0"]
    d = synth.generate(w)
    m = lshmf.LshMF(w.M, w.N, w.F, 0, w.G, w.p, w.q, w.rscale, d["train_u"].size, n_strata=w.n_strata,
                    model=lshmf.PLAIN_MF)
    dev = m.device
    m.ingest(*[torch.from_numpy(d[k]).to(dev) for k in ("train_u", "train_i", "train_rc")])
    m.set_factors(torch.from_numpy(d["U0"]).to(dev), torch.from_numpy(d["V0"]).to(dev))
    m.build_lsh_neighbours(torch.from_numpy(d["H"].view(np.int32)).to(dev), SEED_FILL)
    assert m.mu.item() == 0.0
    o = orc.Model(w.M, w.N, w.F, 0, w.rscale, d["train_u"], d["train_i"], d["train_rc"],
                  np.zeros((w.N, 0), np.int32), d["U0"], d["V0"],
                  fixed_baselines=(0.0, np.zeros(w.M), np.zeros(w.N)))
    alpha0 = (0.0, 0.0) + tuple(w.alpha[2:])
    lam0 = (0.0, 0.0) + tuple(w.lam[2:])
    for t in range(2):
        m.sgd_epoch(w.alpha, w.lam, w.beta, t)     # the library ignores the bias rates
        o.sgd_epoch(w.n_strata, alpha0, lam0, w.beta, t)
    m.check()
    assert not m.bu.any().item() and not m.bv.any().item()
    compare_tables({k: (getattr(m, k).double().cpu().numpy().reshape(getattr(o, k).shape), getattr(o, k))
                    for k in ("U", "V")}, 1e-4, _say, "plain MF two epochs")
    qu, qi = synth.random_queries(w.M, w.N, 2000, 7)
    got = m.predict(torch.from_numpy(qu).cuda(), torch.from_numpy(qi).cuda()).cpu().numpy()
    ref = np.einsum("nf,nf->n", o.U[qu], o.V[qi])
    assert np.all(np.abs(got - ref) <= 1e-4 * np.maximum(1.0, np.abs(ref)))
