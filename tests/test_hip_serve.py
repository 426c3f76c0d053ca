"""The serving loop through the C ABI (needs an MI355X).

A request log of online updates and rating queries is replayed by
lshmf_serve, partly back to back (so queries get merged) and partly at
Poisson arrival times.  The answers and the final model must equal, bit for
bit, what the same updates and queries give when issued one at a time; the
refusals (an update above batch_cap, a query above the batch limit) must
leave the model untouched; times must be ordered.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2111_11682_amd import synth

pytestmark = pytest.mark.gpu

SEED_FILL = 0x5E4E


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _pretrained(w, d, sp, batch_cap, storage):
    from paper_2111_11682_amd import lshmf
    M0, N0 = int(sp["M_old"]), int(sp["N_old"])
    m = lshmf.LshMF(M0, N0, w.F, w.K, w.G, w.p, w.q, w.rscale, sp["pretrain_u"].size,
                    n_strata=w.n_strata, M_cap=w.M, N_cap=w.N, nnz_cap=d["train_u"].size + 64,
                    batch_cap=batch_cap, storage=storage)
    dev = m.device
    m.ingest(*[torch.from_numpy(sp[k]).to(dev) for k in ("pretrain_u", "pretrain_i", "pretrain_rc")])
    m.set_factors(torch.from_numpy(d["U0"][:M0]).to(dev), torch.from_numpy(d["V0"][:N0]).to(dev))
    m.build_lsh_neighbours(torch.from_numpy(d["H"].view(np.int32)).to(dev), SEED_FILL)
    for t in range(2):
        m.sgd_epoch(w.alpha, w.lam, w.beta, t)
    torch.cuda.synchronize()
    return m


@pytest.mark.parametrize("storage", ["fp32", "bf16", "bf16u"])
def test_serve_equals_requests_one_at_a_time(storage):
    # fp32 and bf16u: queries and updates on one stream; bf16: queries on a
    # stream of their own, overlapping the next update up to its last step
    w = synth.WORKLOADS["small"]
    d = synth.generate(w)
    sp = synth.online_split(w, d, frac_new=0.03, stream_frac=0.2)
    L = synth.serve_log(sp, w.M, w.N, 100, 2000, 1, 300)
    batch_cap, mqb = 2000, 512
    req = L["req"]
    extra = np.array([(0, w.M, w.N, 0, 0, batch_cap + 1, 0.0), (1, 0, 0, 0, 0, mqb + 1, 0.0)],
                     dtype=req.dtype)
    req = np.concatenate([req[: req.size // 2], extra, req[req.size // 2:]])
    half = req.size // 2
    req["arrival"][half:] = synth.poisson_arrivals(req.size - half, 2000.0)
    _say("[gpu] serve: %d requests, %d update ratings, %d query pairs" %
         (req.size, L["upd_u"].size, L["q_u"].size))
    dev = torch.device("cuda")
    pin = lambda a: torch.from_numpy(a).pin_memory()
    upd = (pin(L["upd_u"]), pin(L["upd_i"]), pin(L["upd_rc"]))
    qry = (pin(L["q_u"]), pin(L["q_i"]))
    U0 = torch.from_numpy(d["U0"]).to(dev)
    V0 = torch.from_numpy(d["V0"]).to(dev)
    H = torch.from_numpy(d["H"].view(np.int32)).to(dev)

    m1 = _pretrained(w, d, sp, batch_cap, storage)
    pred, start, done, status = m1.serve(req, upd, qry, U0, V0, H, SEED_FILL, w.alpha, w.lam, w.beta,
                                         3, 1, max_query_batch=mqb)
    assert m1.device_status() == 0
    assert np.all(status[[i for i in range(req.size) if req["n"][i] not in (batch_cap + 1, mqb + 1)]] == 0)
    assert set(status[[i for i in range(req.size) if req["n"][i] in (batch_cap + 1, mqb + 1)]]) == {-3}
    assert np.all(done >= start) and np.all(start >= req["arrival"] - 1e-6)
    q = req["kind"] == 1
    starts = start[q]
    assert np.any(starts[1:] == starts[:-1]), "no queries were merged"
    lat = (done - req["arrival"])[q & (status == 0)]
    _say("[gpu] serve (%s) query latency p50 %.3f ms p99 %.3f ms" %
         (storage, 1e3 * np.percentile(lat, 50), 1e3 * np.percentile(lat, 99)))

    # the same requests, one call each
    m2 = _pretrained(w, d, sp, batch_cap, storage)
    ref = torch.full_like(pred, float("nan"))
    Mc, Nc = int(sp["M_old"]), int(sp["N_old"])
    for r in range(req.size):
        if status[r] != 0:
            continue
        o, n = int(req["offset"][r]), int(req["n"][r])
        if req["kind"][r] == 0:
            Mn, Nn = int(req["M_new"][r]), int(req["N_new"][r])
            m2.online_update(*[x[o:o + n].to(dev) for x in upd], Mn, Nn, H, SEED_FILL, w.alpha, w.lam,
                             w.beta, 3, 1, U_new=U0[Mc:Mn], V_new=V0[Nc:Nn])
            Mc, Nc = Mn, Nn
        elif n > 0:
            ref[o:o + n] = m2.predict(qry[0][o:o + n].to(dev), qry[1][o:o + n].to(dev)).cpu()
    torch.cuda.synchronize()
    assert torch.equal(pred, ref)
    tabs = ["U", "V", "bu", "bv", "W", "C", "JK", "acc", "sig", "b0", "bh0"]
    if storage != "fp32":
        tabs += ["U16", "V16", "W16", "C16"]
    if storage == "bf16u":
        tabs.remove("U")  # not used in this mode
    for k in tabs:
        assert torch.equal(getattr(m1, k), getattr(m2, k)), k
    lay1, lay2 = m1.layout(), m2.layout()
    assert (lay1.M, lay1.N, lay1.nnz) == (lay2.M, lay2.N, lay2.nnz)
