"""Quality of the neighbour lists of the three hash families (needs an MI355X).

Sec. 5.3 compares top-K methods by the RMSE they lead to, their time and their
space; Sec. 4.1 motivates simLSH by how well it finds similar items without
the N x N similarity matrix.  Here every family's GPU lists (which other tests
show equal to the oracle's bit for bit) are scored by recall@K against two
brute-force references computed by the oracle: the top-K of the cosine of the
Psi-weighted item columns (what the sign hashes estimate) and the top-K of the
paper's GSM (shrunk Pearson correlation, Sec. 3.1).  Random lists score
K / (N - 1).  Every family must beat random; the recall, build time and
space of each are printed for the record.  The p = 3 rows use the paper's
q = 100 bands (with few bands, 24-bit keys rarely collide and the lists are
mostly the random supplement).
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as orc
from paper_2111_11682_amd import synth

pytestmark = pytest.mark.gpu

SEED_FILL = 0x70B_C0DE


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _recall(JK, ref):
    return float(np.mean([len(set(JK[j]) & set(ref[j])) / JK.shape[1] for j in range(JK.shape[0])]))


@pytest.mark.parametrize("base", ["small", "ml100k"])
def test_family_recall_time_space(base):
    from paper_2111_11682_amd import lshmf
    w0 = synth.WORKLOADS[base]
    d = synth.generate(w0)
    u, it, rc = d["train_u"], d["train_i"], d["train_rc"]
    cos_top = orc.topk_by_score(orc.cosine_psi(w0.M, w0.N, u, it, rc), w0.K)
    gsm_top = orc.topk_by_score(orc.gsm(w0.M, w0.N, u, it, rc, w0.rscale), w0.K) if base == "small" else None
    rand = w0.K / (w0.N - 1)
    rows = []
    shapes = [("simLSH", dict(family=0)), ("RP_cos", dict(family=1)), ("minHash", dict(family=2)),
              ("simLSH p=3", dict(family=0, p=3, q=100)), ("RP_cos p=3", dict(family=1, p=3, q=100)),
              ("minHash p=3", dict(family=2, p=3, q=100))]
    for label, kw in shapes:
        import dataclasses
        w = dataclasses.replace(w0, name=base + "_" + label, **kw)
        R = synth.family_rand(w)
        m = lshmf.LshMF(w.M, w.N, w.F, w.K, w.G, w.p, w.q, w.rscale, u.size, n_strata=w.n_strata,
                        hash_family=w.family)
        dev = m.device
        m.ingest(*[torch.from_numpy(x).to(dev) for x in (u, it, rc)])
        m.set_timing(True)
        Rt = torch.from_numpy(R.view(np.int32) if R.dtype == np.uint32 else R).to(dev)
        m.build_lsh_neighbours(Rt, SEED_FILL)
        m.build_lsh_neighbours(Rt, SEED_FILL)  # the second call is timed warm
        ph = m.lsh_phase_ms()
        m.check()
        JK = m.JK.cpu().numpy()
        m.close()
        rc_cos = _recall(JK, cos_top)
        rc_gsm = _recall(JK, gsm_top) if gsm_top is not None else float("nan")
        ms = ph["hash_state"] + ph["signatures"] + ph["banding"] + ph["topk"]
        space = w.N * w.p * w.q * 4 / 2 ** 20
        rows.append((label, w.G, w.p, w.q, rc_cos, rc_gsm, ms, space))
        assert rc_cos > rand, (label, rc_cos, rand)
    _say("[gpu] top-K quality on the %s shape (N=%d, K=%d; random recall %.4f):" % (base, w0.N, w0.K, rand))
    for r in rows:
        _say("[gpu]   %-12s G=%d p=%d q=%-3d recall@K cosine %.4f GSM %.4f  search %.3f ms  space %.4f MiB" % r)
