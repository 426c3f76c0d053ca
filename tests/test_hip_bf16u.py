"""Storage mode BF16_U: user rows stored only in BF16 (needs an MI355X).

The SGD reads each user row from HBM as BF16, computes in FP32 and writes it
back rounded to nearest even (inside a block the row passes between ratings
in FP32); the item side keeps FP32 masters.  The arithmetic is no longer
that of the FP64 oracle up to FP32 rounding: every store of a user row drops
to 8 significant bits.  The bar is the one for BF16 storage: held-out RMSE
within 0.5% of the FP64 oracle's.  The tests also show that the FP32 U
table is not read (NaN there changes nothing), and print the one-epoch
distance of every table from the oracle for the record.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as orc
from paper_2111_11682_amd import synth
from tablecmp import table_errors

pytestmark = pytest.mark.gpu

SEED_FILL = 0x5EED_F111


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _model(name, storage, poison_u=False):
    from paper_2111_11682_amd import lshmf
    w = synth.WORKLOADS[name]
    d = synth.generate(w)
    m = lshmf.LshMF(w.M, w.N, w.F, w.K, w.G, w.p, w.q, w.rscale, d["train_u"].size,
                    n_strata=w.n_strata, storage=storage)
    dev = m.device
    m.ingest(*[torch.from_numpy(d[k]).to(dev) for k in ("train_u", "train_i", "train_rc")])
    m.set_factors(torch.from_numpy(d["U0"]).to(dev), torch.from_numpy(d["V0"]).to(dev))
    if poison_u:
        m.U.fill_(float("nan"))
    m.build_lsh_neighbours(torch.from_numpy(d["H"].view(np.int32)).to(dev), SEED_FILL)
    return w, d, m


def _oracle(w, d, JK, epochs):
    o = orc.Model(w.M, w.N, w.F, w.K, w.rscale, d["train_u"], d["train_i"], d["train_rc"], JK,
                  d["U0"], d["V0"])
    for t in range(epochs):
        o.sgd_epoch(w.n_strata, w.alpha, w.lam, w.beta, t)
    return o


@pytest.mark.parametrize("name", ["ml100k", "nfsmall"])
def test_bf16u_full_run_rmse_and_unused_fp32_u(name):
    w, d, m = _model(name, "bf16u", poison_u=True)
    JK = m.JK.cpu().numpy()
    for t in range(w.epochs):
        m.sgd_epoch(w.alpha, w.lam, w.beta, t)
    m.check()
    dev = m.device
    tu, ti, trc = (torch.from_numpy(d[k]).to(dev) for k in ("test_u", "test_i", "test_rc"))
    pred = m.predict(tu, ti)
    assert torch.isfinite(pred).all()        # the NaN-filled FP32 U was never read
    assert torch.isnan(m.U).all()            # ... nor written
    r_gpu = m.rmse(pred, trc).item()
    o = _oracle(w, d, JK, w.epochs)
    r_orc = o.rmse(d["test_u"], d["test_i"], d["test_rc"])
    u16 = m.U16.float().cpu().numpy().astype(np.float64)
    errs = {k: table_errors(g, getattr(o, k)) for k, g in
            (("U", u16), ("V", m.V.double().cpu().numpy()), ("W", m.W.double().cpu().numpy()),
             ("C", m.C.double().cpu().numpy()))}
    _say("[gpu] %s BF16_U after %d epochs: RMSE gpu %.6f oracle %.6f; tables element-wise (floor RMS) / "
         "normwise %s" % (name, w.epochs, r_gpu, r_orc, {k: "%.2e / %.2e" % v for k, v in errs.items()}))
    assert abs(r_gpu - r_orc) <= 0.005 * r_orc


def test_bf16u_one_epoch_against_fp32_mode():
    # the same epoch in FP32 mode and in BF16_U mode: U differs by the BF16
    # rounding of the rows written back, the rest follows from it
    w, d, m32 = _model("ml100k", "fp32")
    _, _, m16 = _model("ml100k", "bf16u")
    for m in (m32, m16):
        m.sgd_epoch(w.alpha, w.lam, w.beta, 0)
        m.check()
    u32 = m32.U.double().cpu().numpy()
    u16 = m16.U16.float().double().cpu().numpy()
    # A user row goes back to HBM once per stratum in which it has ratings, at
    # most P times an epoch, each time within half a BF16 ulp (2^-9
    # relative); twice that sum allows for the FP32 differences the rounded
    # rows cause in later updates.
    rel = np.abs(u16 - u32) / np.maximum(np.abs(u32), np.sqrt(np.mean(u32 * u32)))
    bound = 2 * w.n_strata * 2.0 ** -9
    _say("[gpu] BF16_U vs FP32 mode after one epoch: U max rel %.3e (bound %.3e), V max rel %.3e" % (
        rel.max(), bound, table_errors(m16.V.double().cpu().numpy(), m32.V.double().cpu().numpy())[0]))
    assert rel.max() <= bound
