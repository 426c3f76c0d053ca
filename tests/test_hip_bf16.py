"""Storage mode BF16: BF16 copies of U, V, W, C next to FP32 masters (needs an MI355X).

The masters follow exactly the FP32 arithmetic, so they must equal an FP32
mode run bit for bit; every copy must be the round-to-nearest-even image of
its master (checked against torch's CPU conversion); predictions from the
copies must match the oracle evaluated on the same rounded tables; and the
held-out RMSE of a full run must stay within 0.5% of the FP64 oracle's.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as orc
from paper_2111_11682_amd import synth

pytestmark = pytest.mark.gpu

SEED_FILL = 0x5EED_F111


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _model(name, storage):
    from paper_2111_11682_amd import lshmf
    w = synth.WORKLOADS[name]
    d = synth.generate(w)
    _say("[gpu] %s model %s" % (storage, name))
    m = lshmf.LshMF(w.M, w.N, w.F, w.K, w.G, w.p, w.q, w.rscale, d["train_u"].size,
                    n_strata=w.n_strata, storage=storage)
    dev = m.device
    m.ingest(*[torch.from_numpy(d[k]).to(dev) for k in ("train_u", "train_i", "train_rc")])
    m.set_factors(torch.from_numpy(d["U0"]).to(dev), torch.from_numpy(d["V0"]).to(dev))
    m.build_lsh_neighbours(torch.from_numpy(d["H"].view(np.int32)).to(dev), SEED_FILL)
    return w, d, m


def _copies_are_rne(m, rows_u=None, rows_v=None):
    for master, copy in ((m.U, m.U16), (m.V, m.V16), (m.W, m.W16), (m.C, m.C16)):
        ref = master.cpu().to(torch.bfloat16).view(torch.int16)
        assert torch.equal(copy.cpu().view(torch.int16), ref)


def test_bf16_rounding_of_special_values():
    from paper_2111_11682_amd import lshmf
    m = lshmf.LshMF(4, 3, 64, 1, 8, 1, 1, 1, 2, n_strata=1, storage="bf16")
    dev = m.device
    m.ingest(torch.tensor([0, 1], dtype=torch.int32, device=dev),
             torch.tensor([0, 1], dtype=torch.int32, device=dev),
             torch.tensor([3, 4], dtype=torch.uint8, device=dev))
    bits = np.array([0x3F808000, 0x3F818000, 0x3F80FFFF, 0x3F807FFF, 0xBF808000, 0x7F7FFFFF,
                     0x7F800000, 0xFF800000, 0x00000001, 0x80008000, 0x00018000, 0x7F7F8000,
                     0x00000000, 0x80000000, 0x3EAAAAAB, 0xC2F6E979], np.uint32)
    vals = np.resize(bits, 4 * 64).view(np.float32).reshape(4, 64)
    m.U.copy_(torch.from_numpy(vals))
    m.sync_storage()
    torch.cuda.synchronize()
    ref = torch.from_numpy(vals).to(torch.bfloat16).view(torch.int16)
    assert torch.equal(m.U16.cpu().view(torch.int16), ref)


def test_bf16_masters_equal_fp32_mode_and_copies_are_rne():
    outs = {}
    for storage in ("fp32", "bf16"):
        w, d, m = _model("small", storage)
        for t in range(2):
            m.sgd_epoch(w.alpha, w.lam, w.beta, t)
        torch.cuda.synchronize()
        assert m.device_status() == 0
        outs[storage] = [getattr(m, k).cpu().clone() for k in ("U", "V", "bu", "bv", "W", "C")]
        if storage == "bf16":
            _copies_are_rne(m)
    for a, b in zip(outs["fp32"], outs["bf16"]):
        assert torch.equal(a, b)


def test_bf16_predict_matches_oracle_on_rounded_tables():
    w, d, m = _model("ml100k", "bf16")
    acc, sig = orc.simlsh(w.M, w.N, w.B, d["train_u"], d["train_i"], d["train_rc"], d["H"])
    JK = orc.topk(sig, w.B, w.G, w.p, w.q, w.K, SEED_FILL)
    rng = np.random.default_rng(3)
    tabs = dict(U=rng.normal(0, 0.3, (w.M, w.F)), V=rng.normal(0, 0.3, (w.N, w.F)),
                W=rng.normal(0, 0.2, (w.N, w.K)), C=rng.normal(0, 0.2, (w.N, w.K)),
                bu=rng.normal(0, 0.1, w.M), bv=rng.normal(0, 0.1, w.N))
    o = orc.Model(w.M, w.N, w.F, w.K, w.rscale, d["train_u"], d["train_i"], d["train_rc"], JK,
                  d["U0"], d["V0"])
    for k, v in tabs.items():
        t32 = torch.from_numpy(v.astype(np.float32))
        getattr(m, k).copy_(t32)
        # the oracle sees what the copies hold: masters rounded to BF16 (biases stay FP32)
        ref = t32.to(torch.bfloat16).double() if k in ("U", "V", "W", "C") else t32.double()
        getattr(o, k)[...] = ref.numpy().reshape(getattr(o, k).shape)
    m.sync_storage()
    qu, qi = synth.random_queries(w.M, w.N, 5000, 9)
    got = m.predict(torch.from_numpy(qu).cuda(), torch.from_numpy(qi).cuda()).cpu().numpy()
    ref = o.predict(qu, qi)
    assert np.all(np.abs(got - ref) <= 1e-5 * np.maximum(1.0, np.abs(ref)))


def test_bf16_full_run_rmse_ml100k():
    w, d, m = _model("ml100k", "bf16")
    acc, sig = orc.simlsh(w.M, w.N, w.B, d["train_u"], d["train_i"], d["train_rc"], d["H"])
    JK = orc.topk(sig, w.B, w.G, w.p, w.q, w.K, SEED_FILL)
    o = orc.Model(w.M, w.N, w.F, w.K, w.rscale, d["train_u"], d["train_i"], d["train_rc"], JK,
                  d["U0"], d["V0"])
    for t in range(w.epochs):
        m.sgd_epoch(w.alpha, w.lam, w.beta, t)
        o.sgd_epoch(w.n_strata, w.alpha, w.lam, w.beta, t)
    torch.cuda.synchronize()
    assert m.device_status() == 0
    _copies_are_rne(m)
    tu, ti = torch.from_numpy(d["test_u"]).cuda(), torch.from_numpy(d["test_i"]).cuda()
    r_gpu = m.rmse(m.predict(tu, ti), torch.from_numpy(d["test_rc"]).cuda()).item()
    r_orc = o.rmse(d["test_u"], d["test_i"], d["test_rc"])
    _say("[gpu] ml100k BF16 RMSE gpu %.6f oracle %.6f" % (r_gpu, r_orc))
    assert abs(r_gpu - r_orc) <= 0.005 * r_orc


def test_bf16_online_keeps_copies():
    from paper_2111_11682_amd import lshmf
    w = synth.WORKLOADS["small"]
    d = synth.generate(w)
    sp = synth.online_split(w, d, frac_new=0.03, stream_frac=0.2)
    M0, N0 = int(sp["M_old"]), int(sp["N_old"])
    m = lshmf.LshMF(M0, N0, w.F, w.K, w.G, w.p, w.q, w.rscale, sp["pretrain_u"].size,
                    n_strata=w.n_strata, M_cap=w.M, N_cap=w.N, nnz_cap=d["train_u"].size,
                    batch_cap=sp["stream_u"].size, storage="bf16")
    dev = m.device
    m.ingest(*[torch.from_numpy(sp[k]).to(dev) for k in ("pretrain_u", "pretrain_i", "pretrain_rc")])
    m.set_factors(torch.from_numpy(d["U0"][:M0]).to(dev), torch.from_numpy(d["V0"][:N0]).to(dev))
    H = torch.from_numpy(d["H"].view(np.int32)).to(dev)
    m.build_lsh_neighbours(H, SEED_FILL)
    m.sgd_epoch(w.alpha, w.lam, w.beta, 0)
    su, si, src = (torch.from_numpy(sp[k]).to(dev) for k in ("stream_u", "stream_i", "stream_rc"))
    m.online_update(su, si, src, w.M, w.N, H, SEED_FILL, w.alpha, w.lam, w.beta, 1, 1,
                    U_new=torch.from_numpy(d["U0"][M0:]).to(dev),
                    V_new=torch.from_numpy(d["V0"][N0:]).to(dev))
    torch.cuda.synchronize()
    assert m.device_status() == 0
    _copies_are_rne(m)          # online_update ends with the copies rewritten
    m.sgd_epoch(w.alpha, w.lam, w.beta, 2)
    torch.cuda.synchronize()
    assert m.device_status() == 0
    _copies_are_rne(m)
