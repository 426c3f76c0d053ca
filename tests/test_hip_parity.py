"""HIP path vs the FP64 oracle, through the C ABI (needs an MI355X).

Integer outputs (layout, hash sums, signatures, neighbour lists, neighbour
codes) must match bit for bit; predictions within 1e-5 relative; one SGD
epoch within 1e-4 element by element (floor 0.1 x the table's RMS, see
tablecmp.py); held-out RMSE within 0.5%.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as orc
from paper_2111_11682_amd import synth
from nbrcodes import expected_codes
from tablecmp import compare_tables

pytestmark = pytest.mark.gpu

SEED_FILL = 0x5EED_F111

_cache = {}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def data(name):
    if name not in _cache:
        _cache[name] = synth.generate(synth.WORKLOADS[name])
    return _cache[name]


def gpu_model(name, P=None, F=None):
    from paper_2111_11682_amd import lshmf
    w = synth.WORKLOADS[name]
    d = data(name)
    P = P or w.n_strata
    _say("[gpu] model %s P=%d nnz=%d" % (name, P, d["train_u"].size))
    m = lshmf.LshMF(w.M, w.N, w.F, w.K, w.G, w.p, w.q, w.rscale, d["train_u"].size, n_strata=P)
    dev = m.device
    m._tu = torch.from_numpy(d["train_u"]).to(dev)
    m._ti = torch.from_numpy(d["train_i"]).to(dev)
    m._trc = torch.from_numpy(d["train_rc"]).to(dev)
    m.ingest(m._tu, m._ti, m._trc)
    m.set_factors(torch.from_numpy(d["U0"]).to(dev), torch.from_numpy(d["V0"]).to(dev))
    H = torch.from_numpy(d["H"].view(np.int32)).to(dev)
    m.build_lsh_neighbours(H, SEED_FILL)
    torch.cuda.synchronize()
    assert m.device_status() == 0
    return w, d, m


def oracle_neighbours(name):
    key = ("orc_jk", name)
    if key not in _cache:
        w = synth.WORKLOADS[name]
        d = data(name)
        acc, sig = orc.simlsh(w.M, w.N, w.B, d["train_u"], d["train_i"], d["train_rc"], d["H"])
        JK = orc.topk(sig, w.B, w.G, w.p, w.q, w.K, SEED_FILL)
        _cache[key] = (acc, sig, JK)
    return _cache[key]


def oracle_model(name, JK):
    w = synth.WORKLOADS[name]
    d = data(name)
    return orc.Model(w.M, w.N, w.F, w.K, w.rscale, d["train_u"], d["train_i"], d["train_rc"],
                     JK, d["U0"], d["V0"])


# ---------------------------------------------------------------- hashing
def test_worked_example_on_gpu():
    from paper_2111_11682_amd import lshmf
    # Sec. 4.1 example: three raters with strings 001, 010, 100 rate 3, 4, 5;
    # Psi(r) = r gives sums (-2, -4, -6) and signature 000.  A second item
    # without ratings has zero sums and signature 111.
    _say("[gpu] worked example")
    m = lshmf.LshMF(3, 2, 4, 1, 3, 1, 1, 1, 3, psi_exp=1, n_strata=1)
    dev = m.device
    u = torch.tensor([0, 1, 2], dtype=torch.int32, device=dev)
    i = torch.tensor([0, 0, 0], dtype=torch.int32, device=dev)
    rc = torch.tensor([3, 4, 5], dtype=torch.uint8, device=dev)
    m.ingest(u, i, rc)
    H = torch.tensor([[0b100], [0b010], [0b001]], dtype=torch.int32, device=dev)
    m.build_lsh_neighbours(H, 1)
    torch.cuda.synchronize()
    assert m.acc.cpu().tolist() == [[-2, -4, -6], [0, 0, 0]]
    assert m.sig.cpu().view(torch.int32).tolist() == [[0], [0b111]]
    assert m.JK.cpu().tolist() == [[1], [0]]


@pytest.mark.parametrize("name", ["tiny", "small", "ml100k", "nfsmall", "wide"])
def test_layout_matches_oracle_order(name):
    from paper_2111_11682_amd import lshmf  # noqa: F401
    w, d, m = gpu_model(name)
    P = w.n_strata
    nnz = d["train_u"].size
    lay = m.layout()
    pk = m.arena_view(lay.pk, nnz, torch.int32).cpu().numpy().view(np.uint32)
    sj = m.arena_view(lay.sj, nnz, torch.int32).cpu().numpy()
    dep = m.arena_view(lay.dep, nnz, torch.int32).cpu().numpy()
    blk = m.arena_view(lay.blk_ptr, P * P + 1, torch.int64).cpu().numpy()
    order, oblk = orc.schedule(P, d["train_u"], d["train_i"])
    assert np.array_equal(blk, oblk)
    assert np.array_equal(pk >> 4, d["train_u"][order].astype(np.uint32))
    assert np.array_equal(pk & 15, d["train_rc"][order].astype(np.uint32))
    assert np.array_equal(sj, d["train_i"][order])
    # dep: previous rating of the same user inside the block, as a local index
    users = (pk >> 4).astype(np.int64)
    ref = np.full(nnz, -1, np.int64)
    for b in range(P * P):
        last = {}
        for x in range(blk[b], blk[b + 1]):
            if users[x] in last:
                ref[x] = last[users[x]] - blk[b]
            last[users[x]] = x
    assert np.array_equal(dep, ref)
    # CSR / CSC and the simple-case baselines
    row_ptr = m.arena_view(lay.row_ptr, w.M + 1, torch.int64).cpu().numpy()
    col = m.arena_view(lay.csr_col, nnz, torch.int32).cpu().numpy()
    R = orc.Csr(w.M, d["train_u"], d["train_i"], d["train_rc"])
    assert np.array_equal(row_ptr, R.row_ptr) and np.array_equal(col, R.col[:nnz])
    mu, b0, bh0 = orc.baselines(w.M, w.N, d["train_u"], d["train_i"], d["train_rc"], w.rscale)
    assert m.mu.item() == pytest.approx(mu, rel=1e-15)
    assert np.allclose(m.b0.cpu().numpy(), b0, rtol=0, atol=1e-6)
    assert np.allclose(m.bh0.cpu().numpy(), bh0, rtol=0, atol=1e-6)


@pytest.mark.parametrize("name", ["tiny", "small", "ml100k", "nfsmall", "wide", "manyitems"])
def test_signatures_and_neighbours_bit_exact(name):
    w, d, m = gpu_model(name)
    acc, sig, JK = oracle_neighbours(name)
    assert np.array_equal(m.acc.cpu().numpy(), acc.astype(np.int32))
    assert np.array_equal(m.sig.cpu().numpy().view(np.uint32), sig)
    assert np.array_equal(m.JK.cpu().numpy(), JK)


@pytest.mark.parametrize("name", ["small", "ml100k", "nfsmall", "wide", "manyitems"])
def test_neighbour_codes_exact(name):
    """Every byte of every record, against codes looked up from the triples.
    manyitems has more items than an LDS byte map holds: its rows go through
    hash tables, and its users past 8192 ratings through binary searches."""
    w, d, m = gpu_model(name)
    nnz = d["train_u"].size
    lay = m.layout()
    nib = m.arena_view(lay.nib, nnz * lay.nstride, torch.uint8).cpu().numpy().reshape(nnz, lay.nstride)
    order, _ = orc.schedule(w.n_strata, d["train_u"], d["train_i"])
    _, _, JK = oracle_neighbours(name)
    assert np.array_equal(nib, expected_codes(w.N, w.K, d["train_u"], d["train_i"], d["train_rc"], order, JK,
                                              lay.nstride))


# ---------------------------------------------------------------- predict
def _random_tables(w, seed):
    rng = np.random.default_rng(seed)
    return dict(bu=rng.normal(0, 0.1, w.M), bv=rng.normal(0, 0.1, w.N),
                W=rng.normal(0, 0.1, (w.N, w.K)), C=rng.normal(0, 0.1, (w.N, w.K)))


@pytest.mark.parametrize("name", ["tiny", "small", "ml100k", "nfsmall", "wide"])
def test_predict_parity(name):
    w, d, m = gpu_model(name)
    _, _, JK = oracle_neighbours(name)
    t = _random_tables(w, 1)
    for k, v in t.items():
        getattr(m, k).copy_(torch.from_numpy(v.astype(np.float32)))
    o = oracle_model(name, JK)
    for k, v in t.items():
        getattr(o, k)[...] = v.astype(np.float32).astype(np.float64)
    qu, qi = synth.random_queries(w.M, w.N, 4000, 7)
    qu = np.concatenate([qu, d["train_u"][:1000], [0, w.M - 1]]).astype(np.int32)
    qi = np.concatenate([qi, d["train_i"][:1000], [w.N - 1, 0]]).astype(np.int32)
    got = m.predict(torch.from_numpy(qu).cuda(), torch.from_numpy(qi).cuda()).cpu().numpy()
    ref = o.predict(qu, qi)
    assert np.all(np.abs(got - ref) <= 1e-5 * np.maximum(1.0, np.abs(ref)))
    # out-of-range ids give NaN, the rest of the batch is unaffected
    bad = m.predict(torch.tensor([0, -1, w.M], dtype=torch.int32, device="cuda"),
                    torch.tensor([0, 0, 0], dtype=torch.int32, device="cuda")).cpu().numpy()
    assert np.isfinite(bad[0]) and np.isnan(bad[1]) and np.isnan(bad[2])


# -------------------------------------------------------------------- SGD
def _compare_tables(m, o, tol, label=""):
    pairs = {}
    for k in ("U", "V", "bu", "bv", "W", "C"):
        r = getattr(o, k)
        pairs[k] = (getattr(m, k).double().cpu().numpy().reshape(r.shape), r)
    return compare_tables(pairs, tol, _say, label)


@pytest.mark.parametrize("name", ["tiny", "small", "ml100k", "nfsmall", "wide", "small_p3q100"])
def test_one_epoch_parity(name):
    w, d, m = gpu_model(name)
    _, _, JK = oracle_neighbours(name)
    o = oracle_model(name, JK)
    m.sgd_epoch(w.alpha, w.lam, w.beta, 0)
    torch.cuda.synchronize()
    assert m.device_status() == 0
    o.sgd_epoch(w.n_strata, w.alpha, w.lam, w.beta, 0)
    _compare_tables(m, o, 1e-4, "one epoch " + name)


def test_full_run_rmse_ml100k():
    name = "ml100k"
    w, d, m = gpu_model(name)
    _, _, JK = oracle_neighbours(name)
    o = oracle_model(name, JK)
    for t in range(w.epochs):
        m.sgd_epoch(w.alpha, w.lam, w.beta, t)
        o.sgd_epoch(w.n_strata, w.alpha, w.lam, w.beta, t)
    tu = torch.from_numpy(d["test_u"]).cuda()
    ti = torch.from_numpy(d["test_i"]).cuda()
    trc = torch.from_numpy(d["test_rc"]).cuda()
    pred = m.predict(tu, ti)
    r_gpu = m.rmse(pred, trc).item()
    r_orc = o.rmse(d["test_u"], d["test_i"], d["test_rc"])
    _say("[gpu] ml100k RMSE gpu %.6f oracle %.6f" % (r_gpu, r_orc))
    assert abs(r_gpu - r_orc) <= 0.005 * r_orc
    # the FP64 RMSE reduction itself against a host FP64 sum of the same predictions
    p = pred.cpu().numpy().astype(np.float64)
    ref = math.sqrt(np.mean((d["test_rc"] / w.rscale - p) ** 2))
    assert r_gpu == pytest.approx(ref, rel=1e-12)


def test_runs_are_bit_identical():
    name = "small"
    outs = []
    for _ in range(2):
        w, d, m = gpu_model(name)
        for t in range(2):
            m.sgd_epoch(w.alpha, w.lam, w.beta, t)
        torch.cuda.synchronize()
        outs.append([getattr(m, k).cpu().clone() for k in ("U", "V", "bu", "bv", "W", "C", "JK")])
    for a, b in zip(*outs):
        assert torch.equal(a, b)


def test_block_schedule_invariance():
    # a different stratum count is a different order; the same count must give
    # the same result whatever the waves' timing (bit-identical reruns above);
    # here: the GPU result with P strata equals the oracle run with blocks reversed.
    name = "tiny"
    w, d, m = gpu_model(name)
    _, _, JK = oracle_neighbours(name)
    o = oracle_model(name, JK)
    m.sgd_epoch(w.alpha, w.lam, w.beta, 0)
    o.sgd_epoch(w.n_strata, w.alpha, w.lam, w.beta, 0, reverse_blocks=True)
    _compare_tables(m, o, 1e-4)


def test_ingest_rejects_bad_ids():
    from paper_2111_11682_amd import lshmf
    m = lshmf.LshMF(10, 5, 8, 2, 8, 1, 2, 1, 3, n_strata=2)
    u = torch.tensor([0, 1, 10], dtype=torch.int32, device="cuda")
    i = torch.tensor([0, 1, 2], dtype=torch.int32, device="cuda")
    rc = torch.tensor([1, 2, 3], dtype=torch.uint8, device="cuda")
    with pytest.raises(lshmf.LshmfError) as ei:
        m.ingest(u, i, rc)
    assert ei.value.status == -1
    with pytest.raises(lshmf.LshmfError) as ei:
        m.sgd_epoch([0.01] * 6, [0.01] * 6, 0.0, 0)
    assert ei.value.status == -2


def test_ingest_rejects_a_pair_given_twice():
    # R holds one value per (user, item) pair: a repeated pair is refused
    # before anything is laid out, and the context stays unbound to data
    from paper_2111_11682_amd import lshmf
    m = lshmf.LshMF(10, 5, 8, 2, 8, 1, 2, 1, 4, n_strata=2)
    u = torch.tensor([0, 1, 3, 1], dtype=torch.int32, device="cuda")
    i = torch.tensor([0, 2, 2, 2], dtype=torch.int32, device="cuda")
    rc = torch.tensor([1, 2, 3, 4], dtype=torch.uint8, device="cuda")
    with pytest.raises(lshmf.LshmfError) as ei:
        m.ingest(u, i, rc)
    assert ei.value.status == -1 and "twice" in str(ei.value)
    H = torch.zeros(10, 1, dtype=torch.int32, device="cuda")
    with pytest.raises(lshmf.LshmfError) as ei:
        m.build_lsh_neighbours(H, 1)
    assert ei.value.status == -2
    # the same pairs without the repeat are accepted; the device status is healthy
    m.ingest(u[:3].contiguous(), i[:3].contiguous(), rc[:3].contiguous())
    m.build_lsh_neighbours(H, 1)
    m.check()
