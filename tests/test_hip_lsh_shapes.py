"""Neighbour search at other hash shapes and families, HIP path vs the oracle
(needs an MI355X).

Sec. 4.1 coarse-grained hashing ANDs p hashes of G bits into one band key and
fine-grained hashing ORs q bands; Sec. 5.3 runs G = 8, p = 3, q = 100 (B = 2400
bits) and compares simLSH with RP_cos and minHash.  For every shape and family
the per-item hash state (integer sums, FP32 projections in their fixed order,
or minima), the signatures and the neighbour lists must match the oracle bit
for bit.
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


def _rand_tensor(w, R, dev):
    t = torch.from_numpy(R.view(np.int32) if R.dtype == np.uint32 else R)
    return t.to(dev)


def build_gpu(w, d, R):
    from paper_2111_11682_amd import lshmf
    m = lshmf.LshMF(w.M, w.N, w.F, w.K, w.G, w.p, w.q, w.rscale, d["train_u"].size,
                    n_strata=w.n_strata, hash_family=w.family)
    dev = m.device
    m.ingest(*[torch.from_numpy(d[k]).to(dev) for k in ("train_u", "train_i", "train_rc")])
    m.set_factors(torch.from_numpy(d["U0"]).to(dev), torch.from_numpy(d["V0"]).to(dev))
    m.build_lsh_neighbours(_rand_tensor(w, R, dev), SEED_FILL)
    m.check()
    return m


def gpu_state(m, w):
    a = m.acc.cpu().numpy()
    if w.family == 0:
        return a.astype(np.int64)
    if w.family == 1:
        return a.view(np.float32)
    nh = w.B // w.G
    return a.reshape(-1)[: w.N * nh].view(np.uint32).reshape(w.N, nh)


SHAPES = ["small_p2", "small_p7", "small_p3q100", "ml100k_p3q100", "nfsmall_p3q100",
          "small_rpcos", "small_minhash", "ml100k_rpcos_p3", "ml100k_minhash_p3"]


@pytest.mark.parametrize("name", SHAPES)
def test_hash_state_signatures_and_lists_bit_exact(name):
    w = synth.WORKLOADS[name]
    d = synth.generate(w)
    u, it, rc, twins = synth.twin_items(d["train_u"], d["train_i"], d["train_rc"], w.N, max(4, w.N // 40))
    d = dict(d, train_u=u, train_i=it, train_rc=rc)
    R = synth.family_rand(w)
    _say("[gpu] hash shape %s: family %d, G=%d p=%d q=%d (B=%d)" % (name, w.family, w.G, w.p, w.q, w.B))
    m = build_gpu(w, d, R)
    st, sig = orc.lsh_build(w.family, w.M, w.N, w.B, w.G, d["train_u"], d["train_i"], d["train_rc"], R,
                            w.rscale)
    JK = orc.topk(sig, w.B, w.G, w.p, w.q, w.K, SEED_FILL)
    got = gpu_state(m, w)
    if w.family == 1:   # FP32 sums in the same order: the same bits
        assert np.array_equal(got.view(np.uint32), st.view(np.uint32))
    else:
        assert np.array_equal(got, st)
    assert np.array_equal(m.sig.cpu().numpy().view(np.uint32), sig)
    assert np.array_equal(m.JK.cpu().numpy(), JK)
    # the lists are not just the random supplement: most slots come from collisions
    keys = orc.band_keys(sig, w.B, w.G, w.p, w.q)
    hits = sum(int((orc.pair_counts(keys, j)[JK[j]] > 0).sum()) for j in range(0, w.N, max(1, w.N // 50)))
    paired = sum(int(b in JK[a]) + int(a in JK[b]) for a, b in twins)
    _say("[gpu] %s: %d colliding slots in the sampled lists, %d of %d twin slots"
         % (name, hits, paired, 2 * len(twins)))
    assert hits > 0
    assert paired >= len(twins)
