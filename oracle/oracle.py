"""ctypes front end of the plain FP64 CPU oracle (``lshmf_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of the benchmark.  The product path never imports it.  It
shares no code with the HIP library.

Besides the C oracle, this module holds the brute-force similarity references
used to judge the neighbour sets on tiny matrices (Sec. 3.1 GSM definition:
S = n/(n + lambda_rho) * rho with Pearson rho over co-raters; and the cosine of
the Psi-weighted columns, the quantity whose angle the sign hash estimates).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lshmf_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liblshmf_oracle.so")
_lock = threading.Lock()
_lib = None

ORC_OK = 0


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C99 + OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-std=c99", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Model(C.Structure):
    _fields_ = [("M", C.c_int), ("N", C.c_int), ("F", C.c_int), ("K", C.c_int),
                ("rscale", C.c_int), ("mu", C.c_double),
                ("U", C.c_void_p), ("V", C.c_void_p), ("bu", C.c_void_p), ("bv", C.c_void_p),
                ("W", C.c_void_p), ("C", C.c_void_p), ("b0", C.c_void_p), ("bh0", C.c_void_p),
                ("JK", C.c_void_p)]


class _Csr(C.Structure):
    _fields_ = [("M", C.c_int), ("row_ptr", C.c_void_p), ("col", C.c_void_p), ("rc", C.c_void_p)]


class _Rates(C.Structure):
    _fields_ = [("g", C.c_double * 6), ("lam", C.c_double * 6)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            L = C.CDLL(build())
            vp, i32, i64, u64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_uint64, C.c_double
            L.orc_splitmix64.restype = u64
            L.orc_splitmix64.argtypes = [u64, u64]
            L.orc_simlsh.argtypes = [i32, i32, i32, i64, vp, vp, vp, vp, i32, vp, vp]
            L.orc_simlsh_add.argtypes = [i32, i32, i32, i64, vp, vp, vp, vp, i32, vp]
            L.orc_signs.argtypes = [i32, i32, vp, vp]
            L.orc_signs.restype = None
            L.orc_band_key.restype = u64
            L.orc_band_key.argtypes = [vp, i32, i32, i32]
            L.orc_band_keys.argtypes = [i32, i32, i32, i32, i32, vp, vp]
            L.orc_pair_counts.argtypes = [i32, i32, vp, i32, vp]
            L.orc_topk.argtypes = [i32, i32, i32, i32, i32, i32, vp, u64, vp, i32, vp]
            L.orc_build_csr.argtypes = [i32, i64, vp, vp, vp, vp, vp, vp]
            L.orc_baselines.argtypes = [i32, i32, i64, vp, vp, vp, i32, C.POINTER(dbl), vp, vp]
            L.orc_predict_one.restype = dbl
            L.orc_predict_one.argtypes = [C.POINTER(_Model), C.POINTER(_Csr), i32, i32]
            L.orc_predict.argtypes = [C.POINTER(_Model), C.POINTER(_Csr), i64, vp, vp, vp]
            L.orc_rmse.restype = dbl
            L.orc_rmse.argtypes = [i64, vp, vp, i32]
            L.orc_rates_for_epoch.argtypes = [vp, vp, dbl, i32, C.POINTER(_Rates)]
            L.orc_schedule.argtypes = [i32, i64, vp, vp, vp, vp]
            L.orc_sgd_epoch.argtypes = [C.POINTER(_Model), C.POINTER(_Csr), i64, vp, vp, vp, vp,
                                        vp, i32, C.POINTER(_Rates), i32, i32]
            L.orc_sgd_one.argtypes = [C.POINTER(_Model), C.POINTER(_Csr), C.POINTER(_Rates), i32,
                                      i32, i32, i32]
            L.orc_loss.restype = dbl
            L.orc_loss.argtypes = [C.POINTER(_Model), C.POINTER(_Csr), vp]
            L.orc_sgd_strata.argtypes = [C.POINTER(_Model), C.POINTER(_Csr), vp, vp, vp, vp, vp,
                                         i32, i32, i32, C.POINTER(_Rates), i32, i32]
            L.orc_set_threads.argtypes = [i32]
            L.orc_set_threads.restype = None
            L.orc_max_threads.argtypes = []
            L.orc_max_threads.restype = i32
            L.orc_remap_slots.argtypes = [i32, i32, i32, vp, vp, vp, vp, vp, vp]
            L.orc_rpcos_add.argtypes = [i32, i32, i32, i64, vp, vp, vp, i32, vp, vp]
            L.orc_rpcos_signs.argtypes = [i32, i32, vp, vp]
            L.orc_rpcos_signs.restype = None
            L.orc_minhash_add.argtypes = [i32, i32, i32, i64, vp, vp, vp, vp]
            L.orc_minhash_sig.argtypes = [i32, i32, i32, vp, vp]
            _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _chk(status: int, what: str):
    if status != ORC_OK:
        raise ValueError("oracle %s failed with status %d" % (what, status))


def set_threads(n: int):
    """OpenMP threads of the oracle's parallel loops."""
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def splitmix64(seed: int, counter: int) -> int:
    return int(lib().orc_splitmix64(seed & (2**64 - 1), counter & (2**64 - 1)))


def simlsh(M: int, N: int, B: int, u, it, rc, H, psi_exp: int = 2):
    """Eq. (item_hash): returns (acc int64 [N, B], sig uint32 [N, ceil(B/32)])."""
    u = np.ascontiguousarray(u, np.int32)
    it = np.ascontiguousarray(it, np.int32)
    rc = np.ascontiguousarray(rc, np.uint8)
    H = np.ascontiguousarray(H, np.uint32)
    words = (B + 31) // 32
    assert H.shape == (M, words)
    acc = np.zeros((N, B), np.int64)
    sig = np.zeros((N, words), np.uint32)
    _chk(lib().orc_simlsh(M, N, B, u.size, _p(u), _p(it), _p(rc), _p(H), psi_exp,
                          _p(acc), _p(sig)), "simlsh")
    return acc, sig


def simlsh_add(acc, B: int, u, it, rc, H, psi_exp: int = 2):
    """acc += Psi(r)(2H - 1) over the given ratings (the online update of the
    saved pre-sign sums, Sec. 4.3)."""
    u = np.ascontiguousarray(u, np.int32)
    it = np.ascontiguousarray(it, np.int32)
    rc = np.ascontiguousarray(rc, np.uint8)
    H = np.ascontiguousarray(H, np.uint32)
    assert acc.dtype == np.int64 and acc.flags.c_contiguous
    N = acc.shape[0]
    _chk(lib().orc_simlsh_add(H.shape[0], N, B, u.size, _p(u), _p(it), _p(rc), _p(H), psi_exp,
                              _p(acc)), "simlsh_add")
    return acc


def signs(acc, B: int) -> np.ndarray:
    acc = np.ascontiguousarray(acc, np.int64)
    N = acc.shape[0]
    sig = np.zeros((N, (B + 31) // 32), np.uint32)
    lib().orc_signs(N, B, _p(acc), _p(sig))
    return sig


def band_keys(sig, B: int, G: int, p: int, q: int) -> np.ndarray:
    sig = np.ascontiguousarray(sig, np.uint32)
    N = sig.shape[0]
    keys = np.zeros((N, q), np.uint64)
    _chk(lib().orc_band_keys(N, B, G, p, q, _p(sig), _p(keys)), "band_keys")
    return keys


def pair_counts(keys: np.ndarray, j: int) -> np.ndarray:
    keys = np.ascontiguousarray(keys, np.uint64)
    N, q = keys.shape
    out = np.zeros(N, np.int32)
    _chk(lib().orc_pair_counts(N, q, _p(keys), j, _p(out)), "pair_counts")
    return out


def topk(sig, B: int, G: int, p: int, q: int, K: int, seed_fill: int,
         items: Optional[Sequence[int]] = None) -> np.ndarray:
    """Top-K by band-collision frequency (Alg. CULSH), rows sorted by id."""
    sig = np.ascontiguousarray(sig, np.uint32)
    N = sig.shape[0]
    items = np.arange(N, dtype=np.int32) if items is None else np.ascontiguousarray(items, np.int32)
    JK = np.zeros((items.size, K), np.int32)
    _chk(lib().orc_topk(N, B, G, p, q, K, _p(sig), seed_fill & (2**64 - 1), _p(items),
                        items.size, _p(JK)), "topk")
    return JK


def remap_slots(JK_old, W_old, C_old, JK_new, n_old: int):
    """w and c values after a rebuild of the neighbour lists: each kept
    neighbour brings its value to its new slot, new slots and new items
    (rows >= n_old) start at 0."""
    JK_new = np.ascontiguousarray(JK_new, np.int32)
    N, K = JK_new.shape
    JK_old = np.ascontiguousarray(JK_old, np.int32)
    W_old = np.ascontiguousarray(W_old, np.float64)
    C_old = np.ascontiguousarray(C_old, np.float64)
    assert JK_old.shape[0] >= n_old and W_old.shape[0] >= n_old and C_old.shape[0] >= n_old
    W = np.zeros((N, K))
    Cn = np.zeros((N, K))
    _chk(lib().orc_remap_slots(N, n_old, K, _p(JK_old), _p(W_old), _p(C_old), _p(JK_new), _p(W),
                               _p(Cn)), "remap_slots")
    return W, Cn


# --------------------------------------------------------------------------
# Hash families of the top-K comparison (Sec. 5.3): simLSH, RP_cos, minHash.
# Each keeps a per-item state that ratings are added to, and a signature of
# B = G*p*q bits in the layout the banding step reads.
# --------------------------------------------------------------------------
SIMLSH, RPCOS, MINHASH = 0, 1, 2


def rpcos_add(acc, B: int, u, it, rc, rscale: int, g):
    """acc (float32 [N, B]) += r_ij g_i in FP32, raters ascending per item."""
    u = np.ascontiguousarray(u, np.int32)
    it = np.ascontiguousarray(it, np.int32)
    rc = np.ascontiguousarray(rc, np.uint8)
    g = np.ascontiguousarray(g, np.float32)
    assert acc.dtype == np.float32 and acc.flags.c_contiguous and g.shape[1] == B
    _chk(lib().orc_rpcos_add(g.shape[0], acc.shape[0], B, u.size, _p(u), _p(it), _p(rc), rscale,
                             _p(g), _p(acc)), "rpcos_add")
    return acc


def rpcos_signs(acc, B: int) -> np.ndarray:
    acc = np.ascontiguousarray(acc, np.float32)
    sig = np.zeros((acc.shape[0], (B + 31) // 32), np.uint32)
    lib().orc_rpcos_signs(acc.shape[0], B, _p(acc), _p(sig))
    return sig


def minhash_add(mins, u, it, v):
    """mins (uint32 [N, nh]) = min(mins, v_i) over the raters of each item."""
    u = np.ascontiguousarray(u, np.int32)
    it = np.ascontiguousarray(it, np.int32)
    v = np.ascontiguousarray(v, np.uint32)
    assert mins.dtype == np.uint32 and mins.flags.c_contiguous and v.shape[1] == mins.shape[1]
    _chk(lib().orc_minhash_add(v.shape[0], mins.shape[0], mins.shape[1], u.size, _p(u), _p(it),
                               _p(v), _p(mins)), "minhash_add")
    return mins


def minhash_sig(mins, G: int) -> np.ndarray:
    mins = np.ascontiguousarray(mins, np.uint32)
    N, nh = mins.shape
    sig = np.zeros((N, (nh * G + 31) // 32), np.uint32)
    _chk(lib().orc_minhash_sig(N, nh, G, _p(mins), _p(sig)), "minhash_sig")
    return sig


def lsh_init(family: int, N: int, B: int, G: int):
    """Empty per-item hash state of a family."""
    if family == SIMLSH:
        return np.zeros((N, B), np.int64)
    if family == RPCOS:
        return np.zeros((N, B), np.float32)
    return np.full((N, B // G), 0xFFFFFFFF, np.uint32)


def lsh_add(family: int, state, B: int, G: int, u, it, rc, R, rscale: int, psi_exp: int = 2):
    """Adds ratings to the state; R is the family's random input per user
    (simLSH: bit strings H, RP_cos: Gaussians, minHash: random values)."""
    if family == SIMLSH:
        return simlsh_add(state, B, u, it, rc, R, psi_exp)
    if family == RPCOS:
        return rpcos_add(state, B, u, it, rc, rscale, R)
    return minhash_add(state, u, it, R)


def lsh_sig(family: int, state, B: int, G: int) -> np.ndarray:
    if family == SIMLSH:
        return signs(state, B)
    if family == RPCOS:
        return rpcos_signs(state, B)
    return minhash_sig(state, G)


def lsh_build(family: int, M: int, N: int, B: int, G: int, u, it, rc, R, rscale: int,
              psi_exp: int = 2):
    """(state, signature) of the ratings under one hash family."""
    st = lsh_init(family, N, B, G)
    lsh_add(family, st, B, G, u, it, rc, R, rscale, psi_exp)
    return st, lsh_sig(family, st, B, G)


class Csr:
    """Training ratings grouped by user, items ascending (R(i) lookups)."""

    def __init__(self, M: int, u, it, rc):
        u = np.ascontiguousarray(u, np.int32)
        it = np.ascontiguousarray(it, np.int32)
        rc = np.ascontiguousarray(rc, np.uint8)
        self.M = M
        self.row_ptr = np.zeros(M + 1, np.int64)
        self.col = np.zeros(max(u.size, 1), np.int32)
        self.rc = np.zeros(max(u.size, 1), np.uint8)
        _chk(lib().orc_build_csr(M, u.size, _p(u), _p(it), _p(rc), _p(self.row_ptr),
                                 _p(self.col), _p(self.rc)), "build_csr")
        self.c = _Csr(M, self.row_ptr.ctypes.data, self.col.ctypes.data, self.rc.ctypes.data)


def baselines(M: int, N: int, u, it, rc, rscale: int):
    """Sec. 3.2 simple case: (mu, b0 [M], bh0 [N]) in FP64."""
    u = np.ascontiguousarray(u, np.int32)
    it = np.ascontiguousarray(it, np.int32)
    rc = np.ascontiguousarray(rc, np.uint8)
    mu = C.c_double(0.0)
    b0 = np.zeros(M, np.float64)
    bh0 = np.zeros(N, np.float64)
    _chk(lib().orc_baselines(M, N, u.size, _p(u), _p(it), _p(rc), rscale, C.byref(mu),
                             _p(b0), _p(bh0)), "baselines")
    return mu.value, b0, bh0


def schedule(P: int, u, it):
    """Stratified epoch order: (order [nnz] int64, blk_ptr [P*P+1] int64)."""
    u = np.ascontiguousarray(u, np.int32)
    it = np.ascontiguousarray(it, np.int32)
    order = np.zeros(max(u.size, 1), np.int64)
    blk = np.zeros(P * P + 1, np.int64)
    _chk(lib().orc_schedule(P, u.size, _p(u), _p(it), _p(order), _p(blk)), "schedule")
    return order[: u.size], blk


def rates_for_epoch(alpha, lam, beta: float, t: int):
    a = np.ascontiguousarray(alpha, np.float64)
    l = np.ascontiguousarray(lam, np.float64)
    r = _Rates()
    lib().orc_rates_for_epoch(_p(a), _p(l), beta, t, C.byref(r))
    return np.array(r.g[:]), np.array(r.lam[:])


def rmse(pred, rc, rscale: int) -> float:
    pred = np.ascontiguousarray(pred, np.float64)
    rc = np.ascontiguousarray(rc, np.uint8)
    return float(lib().orc_rmse(pred.size, _p(pred), _p(rc), rscale))


class Model:
    """FP64 LSH-MF model state driven by the oracle's SGD (Alg. CULSH-MF)."""

    def __init__(self, M: int, N: int, F: int, K: int, rscale: int, train_u, train_i, train_rc,
                 JK, U0, V0, W0=None, C0=None, bu0=None, bv0=None, fixed_baselines=None):
        self.M, self.N, self.F, self.K, self.rscale = M, N, F, K, rscale
        self.u = np.ascontiguousarray(train_u, np.int32)
        self.i = np.ascontiguousarray(train_i, np.int32)
        self.rc = np.ascontiguousarray(train_rc, np.uint8)
        if fixed_baselines is None:
            self.mu, self.b0, self.bh0 = baselines(M, N, self.u, self.i, self.rc, rscale)
        else:
            mu, b0, bh0 = fixed_baselines
            self.mu = float(mu)
            self.b0 = np.ascontiguousarray(b0, np.float64).copy()
            self.bh0 = np.ascontiguousarray(bh0, np.float64).copy()
        self.R = Csr(M, self.u, self.i, self.rc)
        self.JK = np.ascontiguousarray(JK, np.int32).reshape(N, K) if K else np.zeros((N, 1), np.int32)
        self.U = np.array(U0, np.float64).reshape(M, F).copy()
        self.V = np.array(V0, np.float64).reshape(N, F).copy()
        kk = max(K, 1)
        self.W = np.zeros((N, kk)) if W0 is None else np.array(W0, np.float64).reshape(N, kk).copy()
        self.C = np.zeros((N, kk)) if C0 is None else np.array(C0, np.float64).reshape(N, kk).copy()
        self.bu = np.zeros(M) if bu0 is None else np.array(bu0, np.float64).copy()
        self.bv = np.zeros(N) if bv0 is None else np.array(bv0, np.float64).copy()
        self._sched = {}

    def _c(self) -> _Model:
        return _Model(self.M, self.N, self.F, self.K, self.rscale, self.mu,
                      self.U.ctypes.data, self.V.ctypes.data, self.bu.ctypes.data,
                      self.bv.ctypes.data, self.W.ctypes.data, self.C.ctypes.data,
                      self.b0.ctypes.data, self.bh0.ctypes.data, self.JK.ctypes.data)

    def predict(self, qu, qi) -> np.ndarray:
        qu = np.ascontiguousarray(qu, np.int32)
        qi = np.ascontiguousarray(qi, np.int32)
        out = np.zeros(qu.size, np.float64)
        m = self._c()
        _chk(lib().orc_predict(C.byref(m), C.byref(self.R.c), qu.size, _p(qu), _p(qi), _p(out)),
             "predict")
        return out

    def sgd_epoch(self, P: int, alpha, lam, beta: float, t: int, reverse_blocks: bool = False,
                  upd: int = 3):
        """One pass over the model's own ratings in the stratified order."""
        if P not in self._sched:
            self._sched[P] = schedule(P, self.u, self.i)
        self._pass(self.u, self.i, self.rc, self._sched[P], P, alpha, lam, beta, t,
                   reverse_blocks, upd)

    def sgd_pass(self, u, it, rc, P: int, alpha, lam, beta: float, t: int, upd: int = 3):
        """One pass over a given subset of ratings, in the stratified order of
        that subset; R(i) is the model's full rating set."""
        u = np.ascontiguousarray(u, np.int32)
        it = np.ascontiguousarray(it, np.int32)
        rc = np.ascontiguousarray(rc, np.uint8)
        if u.size == 0:
            return
        self._pass(u, it, rc, schedule(P, u, it), P, alpha, lam, beta, t, False, upd)

    def _pass(self, u, it, rc, sched, P, alpha, lam, beta, t, reverse_blocks, upd):
        order, blk = sched
        r = _Rates()
        a = np.ascontiguousarray(alpha, np.float64)
        l = np.ascontiguousarray(lam, np.float64)
        lib().orc_rates_for_epoch(_p(a), _p(l), beta, t, C.byref(r))
        m = self._c()
        _chk(lib().orc_sgd_epoch(C.byref(m), C.byref(self.R.c), u.size, _p(u), _p(it), _p(rc),
                                 _p(order), _p(blk), P, C.byref(r), int(reverse_blocks), upd),
             "sgd_epoch")

    def sgd_strata(self, P: int, s0: int, s1: int, alpha, lam, beta: float, t: int, upd: int = 3):
        """Strata [s0, s1) of one epoch over the model's own ratings (a bounded
        sample of an epoch, for timing)."""
        if P not in self._sched:
            self._sched[P] = schedule(P, self.u, self.i)
        order, blk = self._sched[P]
        r = _Rates()
        a = np.ascontiguousarray(alpha, np.float64)
        l = np.ascontiguousarray(lam, np.float64)
        lib().orc_rates_for_epoch(_p(a), _p(l), beta, t, C.byref(r))
        m = self._c()
        _chk(lib().orc_sgd_strata(C.byref(m), C.byref(self.R.c), _p(self.u), _p(self.i),
                                  _p(self.rc), _p(order), _p(blk), P, s0, s1, C.byref(r), 0, upd),
             "sgd_strata")

    def sgd_one(self, i: int, j: int, code: int, g, lam, upd: int = 3):
        """One update (Eq. sgd_update) with explicit rates g and regularisers lam."""
        r = _Rates()
        for x in range(6):
            r.g[x] = float(g[x])
            r.lam[x] = float(lam[x])
        m = self._c()
        _chk(lib().orc_sgd_one(C.byref(m), C.byref(self.R.c), C.byref(r), i, j, code, upd),
             "sgd_one")

    def loss(self, lam) -> float:
        l = np.ascontiguousarray(lam, np.float64)
        m = self._c()
        return float(lib().orc_loss(C.byref(m), C.byref(self.R.c), _p(l)))

    def rmse(self, qu, qi, rc) -> float:
        return rmse(self.predict(qu, qi), rc, self.rscale)


def online_update(m: "Model", acc, sig, B: int, G: int, p: int, q: int, seed_fill: int,
                  new_u, new_i, new_rc, H, U0_new, V0_new, P: int, alpha, lam, beta: float,
                  t: int, passes: int = 1, psi_exp: int = 2, rebuild: bool = False,
                  family: int = SIMLSH):
    """Online learning, Sec. 4.3 and Alg. "Online Learning".

    The batch may bring new users (ids >= m.M) and new items (ids >= m.N).
      1. the saved pre-sign sums of the items the batch touches are increased
         by the batch's terms (new items start from zero) and signs recomputed
         (RP_cos and minHash: their own per-item state, continued the same way);
      2. existing items keep their neighbour lists; every new item gets its
         top-K over all items from the updated signatures.  With `rebuild`
         every item's list is searched again instead, and the w, c values of
         the old items follow their neighbour ids (remap_slots);
      3. mu stays; a new user's / item's fixed baseline is the mean of its
         batch ratings minus mu; existing baselines stay;
      4. `passes` times: (A) ratings of new users on existing items update only
         b_i, u_i; (B) ratings of new items update only bh_j, v_j, w_j, c_j;
         (C) the remaining ratings update both sides.  Each phase runs in the
         stratified order of its own ratings; R(i) includes the batch.
    Returns (new Model, acc, sig).
    """
    new_u = np.ascontiguousarray(new_u, np.int32)
    new_i = np.ascontiguousarray(new_i, np.int32)
    new_rc = np.ascontiguousarray(new_rc, np.uint8)
    M2 = max(m.M, int(new_u.max()) + 1 if new_u.size else 0)
    N2 = max(m.N, int(new_i.max()) + 1 if new_i.size else 0)
    # 1. sums and signs
    acc2 = lsh_init(family, N2, B, G)
    acc2[: m.N] = acc
    lsh_add(family, acc2, B, G, new_u, new_i, new_rc, H, m.rscale, psi_exp)
    sig2 = lsh_sig(family, acc2, B, G)
    # 2. neighbour lists
    K = m.K
    JK2 = np.zeros((N2, K), np.int32)
    if K > 0 and rebuild:
        JK2[:] = topk(sig2, B, G, p, q, K, seed_fill)
    elif K > 0:   # K = 0: no neighbour lists
        JK2[: m.N] = m.JK
        if N2 > m.N:
            JK2[m.N:] = topk(sig2, B, G, p, q, K, seed_fill, items=np.arange(m.N, N2, dtype=np.int32))
    # 3. baselines
    b02 = np.zeros(M2)
    b02[: m.M] = m.b0
    bh02 = np.zeros(N2)
    bh02[: m.N] = m.bh0
    for ids, vals, out, base in ((new_u, new_rc, b02, m.M), (new_i, new_rc, bh02, m.N)):
        sel = ids >= base
        if sel.any():
            cnt = np.bincount(ids[sel], minlength=out.size)
            tot = np.bincount(ids[sel], weights=vals[sel].astype(np.float64) / m.rscale,
                              minlength=out.size)
            nz = cnt > 0
            out[nz] = tot[nz] / cnt[nz] - m.mu
    # the grown model
    U2 = np.zeros((M2, m.F))
    U2[: m.M] = m.U
    U2[m.M:] = np.asarray(U0_new, np.float64).reshape(M2 - m.M, m.F)
    V2 = np.zeros((N2, m.F))
    V2[: m.N] = m.V
    V2[m.N:] = np.asarray(V0_new, np.float64).reshape(N2 - m.N, m.F)
    W2 = np.zeros((N2, max(K, 1)))
    C2 = np.zeros((N2, max(K, 1)))
    if K > 0 and rebuild:
        W2[:], C2[:] = remap_slots(m.JK, m.W, m.C, JK2, m.N)
    else:
        W2[: m.N] = m.W
        C2[: m.N] = m.C
    bu2 = np.zeros(M2)
    bu2[: m.M] = m.bu
    bv2 = np.zeros(N2)
    bv2[: m.N] = m.bv
    u_all = np.concatenate([m.u, new_u])
    i_all = np.concatenate([m.i, new_i])
    rc_all = np.concatenate([m.rc, new_rc])
    m2 = Model(M2, N2, m.F, K, m.rscale, u_all, i_all, rc_all, JK2, U2, V2, W2, C2, bu2, bv2,
               fixed_baselines=(m.mu, b02, bh02))
    # 4. frozen-side passes over the batch
    phaseA = (new_u >= m.M) & (new_i < m.N)
    phaseB = new_i >= m.N
    phaseC = ~(phaseA | phaseB)
    for _ in range(passes):
        for sel, upd in ((phaseA, 1), (phaseB, 2), (phaseC, 3)):
            m2.sgd_pass(new_u[sel], new_i[sel], new_rc[sel], P, alpha, lam, beta, t, upd)
    return m2, acc2, sig2


# --------------------------------------------------------------------------
# Brute-force similarity references for tiny matrices (tests only).
# --------------------------------------------------------------------------
def dense_ratings(M: int, N: int, u, it, rc, rscale: int) -> np.ndarray:
    R = np.zeros((M, N), np.float64)
    R[np.asarray(u), np.asarray(it)] = np.asarray(rc, np.float64) / rscale
    return R


def gsm(M: int, N: int, u, it, rc, rscale: int, lam_rho: float = 100.0) -> np.ndarray:
    """Sec. 3.1: S = n/(n + lambda_rho) * rho, rho = Pearson over co-raters.

    rho is centred on the co-rater means of each item; rho = 0 when fewer than
    two co-raters or a zero variance.  Diagonal set to -inf (no self pairs).
    """
    R = dense_ratings(M, N, u, it, rc, rscale)
    mask = R != 0
    S = np.zeros((N, N))
    for a in range(N):
        for b in range(a + 1, N):
            co = mask[:, a] & mask[:, b]
            n = int(co.sum())
            rho = 0.0
            if n >= 2:
                x = R[co, a] - R[co, a].mean()
                y = R[co, b] - R[co, b].mean()
                den = np.sqrt((x * x).sum() * (y * y).sum())
                rho = float((x * y).sum() / den) if den > 0 else 0.0
            S[a, b] = S[b, a] = n / (n + lam_rho) * rho
    np.fill_diagonal(S, -np.inf)
    return S


def cosine_psi(M: int, N: int, u, it, rc, psi_exp: int = 2) -> np.ndarray:
    """Cosine of the Psi-weighted item columns (what the sign hash estimates)."""
    X = np.zeros((M, N))
    X[np.asarray(u), np.asarray(it)] = np.asarray(rc, np.float64) ** psi_exp
    nrm = np.linalg.norm(X, axis=0)
    nrm[nrm == 0] = 1.0
    Cm = (X.T @ X) / np.outer(nrm, nrm)
    np.fill_diagonal(Cm, -np.inf)
    return Cm


def topk_by_score(S: np.ndarray, K: int) -> np.ndarray:
    """Top-K per row by (score desc, id asc)."""
    N = S.shape[0]
    out = np.zeros((N, K), np.int64)
    ids = np.arange(N)
    for j in range(N):
        order = np.lexsort((ids, -S[j]))
        out[j] = np.sort(order[:K])
    return out


def space_mib_simlsh(N: int, p: int, q: int) -> float:
    """simLSH table as one int32 per G-bit hash: N * p * q * 4 bytes, in MiB."""
    return N * p * q * 4 / 2**20


def space_mib_gsm(N: int) -> float:
    """Dense N x N similarity matrix of 4-byte entries, in MiB."""
    return N * N * 4 / 2**20
