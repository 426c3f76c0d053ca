"""Seeded synthetic rating matrices with the shapes of the paper's workloads.

This module is the only code shared by the HIP path's tests and the oracle.
It produces inputs only -- COO ratings, a train/held-out split, the random
user hash strings H_i (an input of the CULSH algorithm, Sec. 4.1 Alg. 1) and
initial factor tables (an input of the CULSH-MF algorithm, Sec. 4.2 Alg. 3).
It holds none of the method's arithmetic (no hashing, no baselines, no SGD).

Recipe (stand-in for the Netflix / MovieLens data of Sec. 5.1, Table "Data
sets", which are not available):

* item popularity: Zipf(s) over popularity ranks; rank -> item id through a
  seeded permutation so an id carries no popularity signal;
* user degrees: lognormal, rescaled to the exact rating total, clipped to
  [d_min, N // 2];
* each user draws its items by successive sampling without replacement
  (draw with replacement in Zipf order, keep the first d_u distinct items);
* ratings carry planted structure so that held-out RMSE and neighbours are
  informative: z = sqrt(.5) * standardise(a_u + c_i + x_u . y_i) +
  sqrt(.5) * eps, with x, y in R^8 and y drawn around 64 item clusters, then
  r = clip(round(3.5 + 1.1 z)) on the integer 1..5 scale or the half-step
  0.5..5.0 scale;
* ratings are stored as integer codes rc = rscale * r (rscale 1 for integer
  ratings, 2 for half-steps), so rc is in 1..5 or 1..10;
* H_i: B uniformly random bits per user, packed LSB-first in uint32 words;
* U0, V0: k / 2048 with k uniform in [-128, 128), exact in bf16/fp32/fp64.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Dict, Optional, Tuple

import numpy as np

MASTER_SEED = 2111_11682


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    M: int                   # users (rows)
    N: int                   # items (columns)
    nnz: int                 # total ratings before the split
    rscale: int              # 1: integer ratings 1..5; 2: half-steps 0.5..5
    zipf_s: float            # item popularity exponent
    deg_kind: str            # "c1" (min 20 + lognormal extra) or "lognormal"
    deg_mu: float            # lognormal location (log scale)
    deg_sigma: float
    deg_min: int
    n_test: int              # held-out ratings
    F: int
    K: int
    G: int                   # bits per simLSH hash (a byte in the paper)
    p: int                   # hashes per coarse band
    q: int                   # bands (fine-grained OR)
    epochs: int
    alpha: Tuple[float, ...]   # learning rates  (b, bh, u, v, w, c)
    lam: Tuple[float, ...]     # regularisers    (b, bh, u, v, w, c)
    beta: float                # learning-rate decay, Eq. learn_rate
    n_strata: int = 256
    family: int = 0            # hash family: 0 simLSH, 1 RP_cos, 2 minHash
    model: int = 0             # 0 neighbourhood model (Eq. rr), 1 plain MF (Alg. CUSGD++, K = 0)

    @property
    def B(self) -> int:
        return self.G * self.p * self.q


def _ln_mu_for_mean(mean: float, sigma: float) -> float:
    return math.log(mean) - 0.5 * sigma * sigma


# Hyper-parameters: Table "The initial learning speed and regularization
# parameters of CULSH-MF" (MovieLens and Netflix columns) and beta = 0.3.
_ML_ALPHA = (0.035, 0.035, 0.035, 0.035, 0.002, 0.002)
_ML_LAM = (0.02, 0.02, 0.02, 0.02, 0.002, 0.002)
_NF_ALPHA = (0.02, 0.02, 0.02, 0.02, 0.001, 0.001)
_NF_LAM = (0.01, 0.01, 0.01, 0.01, 0.05, 0.05)

WORKLOADS: Dict[str, Workload] = {
    # MovieLens-100k-shaped plain case
    "ml100k": Workload("ml100k", 943, 1682, 100_000, 1, 1.0, "c1", 0.0, 1.0, 20,
                       10_000, 32, 10, 8, 1, 8, 5,
                       (0.01,) * 6, (0.05,) * 6, 0.0, n_strata=16),
    # MovieLens-10M-shaped (Table "Data sets", MovieLens column)
    "ml10m": Workload("ml10m", 69_878, 10_677, 10_000_000, 2, 1.1, "lognormal",
                      _ln_mu_for_mean(143.0, 1.2), 1.2, 20,
                      100_000, 64, 50, 8, 1, 16, 20, _ML_ALPHA, _ML_LAM, 0.3,
                      n_strata=256),
    # Netflix-shaped (Table "Data sets", Netflix column)
    "netflix": Workload("netflix", 480_189, 17_770, 100_000_000, 1, 1.2, "lognormal",
                        4.5, 1.2, 1, 1_408_395, 128, 100, 8, 1, 16, 20,
                        _NF_ALPHA, _NF_LAM, 0.3, n_strata=1536),
    # the largest single-GPU shape: 2M users x 500k items, 1B integer ratings,
    # Zipf s = 1.3 items, F = 128, K = 64, 256 hash bits as (8, 2, 16)
    "large1b": Workload("large1b", 2_000_000, 500_000, 1_000_000_000, 1, 1.3, "lognormal",
                        _ln_mu_for_mean(500.0, 1.2), 1.2, 1, 1_000_000, 128, 64, 8, 2, 16, 20,
                        _NF_ALPHA, _NF_LAM, 0.3, n_strata=4096),
    # small shapes for CPU tests
    "tiny": Workload("tiny", 120, 90, 2_400, 1, 1.0, "c1", 0.0, 1.0, 5,
                     240, 8, 6, 8, 1, 4, 3, (0.01,) * 6, (0.05,) * 6, 0.0,
                     n_strata=4),
    "small": Workload("small", 700, 500, 30_000, 2, 1.1, "lognormal",
                      _ln_mu_for_mean(43.0, 1.0), 1.0, 5,
                      2_000, 64, 50, 8, 1, 16, 2, _ML_ALPHA, _ML_LAM, 0.3,
                      n_strata=8),
    # Netflix-like at 1/100 of the users: F = 128, K = 100 (two lane passes)
    "nfsmall": Workload("nfsmall", 4_800, 1_777, 600_000, 1, 1.2, "lognormal",
                        _ln_mu_for_mean(125.0, 1.2), 1.2, 1, 10_000, 128, 100, 8, 1, 16, 2,
                        _NF_ALPHA, _NF_LAM, 0.3, n_strata=32),
    # wide factors and an odd neighbour count: F = 200, K = 70
    "wide": Workload("wide", 900, 600, 40_000, 2, 1.1, "lognormal",
                     _ln_mu_for_mean(44.0, 1.0), 1.0, 5, 2_000, 200, 70, 8, 1, 8, 2,
                     _ML_ALPHA, _ML_LAM, 0.3, n_strata=12),
    # more items than an LDS byte map holds, a few users past 8192 ratings:
    # neighbour codes by hashed user rows, the long rows in chunks; K = 20
    # mixes whole and partial 8-slot words
    "manyitems": Workload("manyitems", 1_500, 80_000, 1_200_000, 1, 1.0, "lognormal",
                          _ln_mu_for_mean(800.0, 1.2), 1.2, 1, 2_000, 16, 20, 8, 1, 8, 2,
                          _ML_ALPHA, _ML_LAM, 0.3, n_strata=64),
}

# The same workloads with K = 0: biased MF without the neighbour term, on the
# same data (isolates the cost and the effect of the K-neighbour term).
for _name in ("tiny", "ml100k", "ml10m"):
    WORKLOADS[_name + "_k0"] = dataclasses.replace(WORKLOADS[_name], name=_name + "_k0", K=0)

# Other hash shapes and families on the same data (the data depend only on the
# shape fields, not on G, p, q or the family):
#   p = 2 and p = 3 coarse bands; (8, 3, 100) is the paper's simLSH setting of
#   Sec. 5.3 (B = 2400 bits over two 64-word slices); (8, 7, 4) has 56-bit
#   bands, whose keys straddle three signature words; (8, 2, 16) is B = 256.
_SHAPES = {
    "small_p2": ("small", dict(p=2, q=16)),
    "small_p7": ("small", dict(p=7, q=4)),
    "small_p3q100": ("small", dict(p=3, q=100)),
    "ml100k_p3q100": ("ml100k", dict(p=3, q=100)),
    "nfsmall_p3q100": ("nfsmall", dict(p=3, q=100)),
    "ml10m_p3q100": ("ml10m", dict(p=3, q=100)),
    "ml10m_p3q200": ("ml10m", dict(p=3, q=200)),
    "netflix_p3q100": ("netflix", dict(p=3, q=100)),
    # RP_cos and minHash (Sec. 5.3 top-K comparison)
    "small_rpcos": ("small", dict(family=1)),
    "small_minhash": ("small", dict(family=2)),
    "ml100k_rpcos_p3": ("ml100k", dict(family=1, p=3, q=16)),
    "ml100k_minhash_p3": ("ml100k", dict(family=2, p=3, q=16)),
    "ml10m_rpcos": ("ml10m", dict(family=1)),
    "ml10m_minhash": ("ml10m", dict(family=2)),
    "ml100k_rpcos": ("ml100k", dict(family=1)),
    "ml100k_minhash": ("ml100k", dict(family=2)),
    "netflix_p3q200": ("netflix", dict(p=3, q=200)),
    "netflix_rpcos": ("netflix", dict(family=1)),
    "netflix_minhash": ("netflix", dict(family=2)),
}
for _name, (_base, _kw) in _SHAPES.items():
    WORKLOADS[_name] = dataclasses.replace(WORKLOADS[_base], name=_name, **_kw)


def derive_seed(*parts: int) -> int:
    """Independent sub-stream seeds from the master seed (numpy SeedSequence)."""
    ss = np.random.SeedSequence([MASTER_SEED, *parts])
    return int(ss.generate_state(1, dtype=np.uint64)[0])


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, stream])))


def user_degrees(w: Workload, rng: np.random.Generator, M: Optional[int] = None,
                 total: Optional[int] = None) -> np.ndarray:
    M = w.M if M is None else M
    total = w.nnz if total is None else total
    dmax = max(w.N // 2, 1)
    dmin = min(w.deg_min, dmax)
    if w.deg_kind == "c1":
        extra = rng.lognormal(0.0, w.deg_sigma, M)
        raw = dmin + extra * max(total - dmin * M, 0) / extra.sum()
    else:
        raw = rng.lognormal(w.deg_mu, w.deg_sigma, M)
    if total > dmax * M or total < dmin * M:
        raise ValueError("rating total not reachable with the degree bounds")
    d = raw * (total / raw.sum())
    for _ in range(100):           # rescale the unclipped part until the total fits
        d = np.clip(d, dmin, dmax)
        free = (d > dmin) & (d < dmax)
        gap = total - d.sum()
        if abs(gap) < 0.5 or not free.any():
            break
        d[free] *= 1.0 + gap / d[free].sum()
    base = np.floor(d).astype(np.int64)
    base = np.clip(base, dmin, dmax)
    rem = total - int(base.sum())
    frac = d - np.floor(d)
    order = np.argsort(-frac, kind="stable")
    step = 1 if rem > 0 else -1
    k = 0
    while rem != 0:                # largest-remainder rounding to the exact total
        idx = order[k % M]
        nv = base[idx] + step
        if dmin <= nv <= dmax:
            base[idx] = nv
            rem -= step
        k += 1
    return base


def _sample_chunk(need: np.ndarray, cdf: np.ndarray, N: int, rng: np.random.Generator
                  ) -> Tuple[np.ndarray, np.ndarray]:
    """Successive sampling for one chunk of users (local ids 0..len(need)-1)."""
    need = need.astype(np.int64).copy()
    got_u = []
    got_r = []
    chosen = np.empty(0, dtype=np.int64)          # sorted keys user*N + rank
    factor = 1.6
    while True:
        users = np.nonzero(need > 0)[0]
        if users.size == 0:
            break
        T = np.ceil(need[users] * factor).astype(np.int64) + 16
        du = np.repeat(users.astype(np.int64), T)
        ranks = np.searchsorted(cdf, rng.random(du.size), side="right")
        np.minimum(ranks, N - 1, out=ranks)
        keys = du * N + ranks
        uniq, first = np.unique(keys, return_index=True)
        if chosen.size:
            pos = np.searchsorted(chosen, uniq)
            pos = np.minimum(pos, chosen.size - 1)
            fresh = chosen[pos] != uniq
            uniq, first = uniq[fresh], first[fresh]
        order = np.argsort(first, kind="stable")
        uniq, first = uniq[order], first[order]
        uu = uniq // N
        # rank of each fresh item within its user, in draw order
        starts = np.searchsorted(uu, users)
        within = np.arange(uu.size) - np.repeat(starts, np.diff(np.append(starts, uu.size)))
        take = within < need[uu]
        uniq = uniq[take]
        got_u.append(uniq // N)
        got_r.append(uniq % N)
        np.subtract.at(need, uniq // N, 1)
        chosen = np.sort(np.concatenate([chosen, uniq]))
        factor *= 2.0
    u = np.concatenate(got_u) if got_u else np.empty(0, np.int64)
    r = np.concatenate(got_r) if got_r else np.empty(0, np.int64)
    order = np.argsort(u, kind="stable")
    return u[order], r[order]


CHUNK_USERS = 16384


def sample_items(deg: np.ndarray, N: int, s: float, rng: np.random.Generator,
                 log: Optional[Callable[[str], None]] = None) -> Tuple[np.ndarray, np.ndarray]:
    """Successive sampling without replacement from Zipf(s) popularity ranks.

    Users are drawn in fixed chunks of CHUNK_USERS, each chunk from its own
    generator seeded from `rng`, so the result does not depend on how many
    threads draw the chunks.  Returns (user, rank) pairs, users ascending,
    ranks in draw order per user.  `log`, if given, hears every 16th chunk.
    """
    import concurrent.futures
    import os
    w = np.arange(1, N + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    M = deg.shape[0]
    n_chunks = (M + CHUNK_USERS - 1) // CHUNK_USERS
    root = int(rng.integers(0, 2**63))

    def chunk(k):
        lo = k * CHUNK_USERS
        g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([root, k])))
        u, r = _sample_chunk(deg[lo: lo + CHUNK_USERS], cdf, N, g)
        if log is not None and k % 16 == 15:
            log("  items: chunk %d of %d drawn" % (k + 1, n_chunks))
        return u + lo, r

    workers = max(1, min(16, os.cpu_count() or 1, n_chunks))
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        parts = list(ex.map(chunk, range(n_chunks)))
    u = np.concatenate([p[0] for p in parts]) if parts else np.empty(0, np.int64)
    r = np.concatenate([p[1] for p in parts]) if parts else np.empty(0, np.int64)
    return u, r


def planted_ratings(u: np.ndarray, item: np.ndarray, M: int, N: int, rscale: int,
                    rng: np.random.Generator, chunk: int = 8_000_000) -> np.ndarray:
    """Integer rating codes rc = rscale * r with planted low-rank/cluster structure."""
    a = rng.standard_normal(M).astype(np.float32)
    c = rng.standard_normal(N).astype(np.float32)
    x = (rng.standard_normal((M, 8)) / math.sqrt(8.0)).astype(np.float32)
    cent = rng.standard_normal((64, 8)).astype(np.float32)
    cl = rng.integers(0, 64, N)
    y = (cent[cl] + 0.5 * rng.standard_normal((N, 8))).astype(np.float32)
    n = u.shape[0]
    s = np.empty(n, dtype=np.float32)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        uu, ii = u[lo:hi], item[lo:hi]
        s[lo:hi] = a[uu] + c[ii] + np.einsum("ij,ij->i", x[uu], y[ii])
    mean = float(s.mean(dtype=np.float64))
    std = float(s.std(dtype=np.float64)) or 1.0
    rc = np.empty(n, dtype=np.uint8)
    lo_code, hi_code = (1, 5) if rscale == 1 else (1, 10)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        z = math.sqrt(0.5) * (s[lo:hi] - mean) / std + \
            math.sqrt(0.5) * rng.standard_normal(hi - lo).astype(np.float32)
        code = np.rint(rscale * (3.5 + 1.1 * z))
        rc[lo:hi] = np.clip(code, lo_code, hi_code).astype(np.uint8)
    return rc


def init_table(rows: int, F: int, rng: np.random.Generator) -> np.ndarray:
    """k / 2048, k uniform in [-128, 128): uniform on [-1/16, 1/16), exact in bf16."""
    k = rng.integers(-128, 128, size=(rows, F), dtype=np.int32)
    return (k.astype(np.float32) * np.float32(1.0 / 2048.0))


def hash_strings(M: int, B: int, rng: np.random.Generator) -> np.ndarray:
    """H_i: B random bits per user, bit b in word b // 32 at position b % 32."""
    if B % 32:
        words = (B + 31) // 32
    else:
        words = B // 32
    H = rng.integers(0, 1 << 32, size=(M, words), dtype=np.uint64).astype(np.uint32)
    if B % 32:
        H[:, -1] &= np.uint32((1 << (B % 32)) - 1)
    return H


def generate(w: Workload, seed: int = MASTER_SEED, with_tables: bool = True,
             log: Optional[Callable[[str], None]] = None) -> Dict[str, np.ndarray]:
    """All inputs of one workload, deterministic in (w, seed).

    Keys: train_u, train_i, train_rc, test_u, test_i, test_rc (int32/uint8 COO),
    H (uint32 [M, ceil(B/32)]), U0 (f32 [M, F]), V0 (f32 [N, F]).
    `log`, if given, hears each step (the 1B-rating shape takes minutes).
    """
    say = log if log is not None else (lambda msg: None)
    rng_deg = _rng(seed, 1)
    rng_items = _rng(seed, 2)
    rng_perm = _rng(seed, 3)
    rng_rate = _rng(seed, 4)
    rng_split = _rng(seed, 5)
    rng_hash = _rng(seed, 6)
    rng_init = _rng(seed, 7)

    deg = user_degrees(w, rng_deg)
    say("  %s: user degrees drawn" % w.name)
    u, rank = sample_items(deg, w.N, w.zipf_s, rng_items, log)
    user_perm = rng_perm.permutation(w.M)
    item_perm = rng_perm.permutation(w.N)
    uid = user_perm[u].astype(np.int32)
    del u
    iid = item_perm[rank].astype(np.int32)
    del rank
    say("  %s: %d items drawn" % (w.name, uid.shape[0]))
    rc = planted_ratings(uid, iid, w.M, w.N, w.rscale, rng_rate)
    say("  %s: ratings drawn" % w.name)
    order = rng_split.permutation(uid.shape[0])
    test_idx = np.sort(order[: w.n_test])
    train_idx = np.sort(order[w.n_test:])
    del order
    say("  %s: split drawn" % w.name)
    out = {
        "train_u": np.ascontiguousarray(uid[train_idx]),
        "train_i": np.ascontiguousarray(iid[train_idx]),
        "train_rc": np.ascontiguousarray(rc[train_idx]),
        "test_u": np.ascontiguousarray(uid[test_idx]),
        "test_i": np.ascontiguousarray(iid[test_idx]),
        "test_rc": np.ascontiguousarray(rc[test_idx]),
        "H": hash_strings(w.M, w.B, rng_hash),
    }
    if with_tables:
        out["U0"] = init_table(w.M, w.F, rng_init)
        out["V0"] = init_table(w.N, w.F, rng_init)
    return out


def family_rand(w: Workload, M: Optional[int] = None, seed: int = MASTER_SEED) -> np.ndarray:
    """The random draws per user of the workload's hash family (an input of
    the neighbour search, like the strings H_i of simLSH):
      simLSH   uint32 [M, ceil(B/32)]  the bit strings H_i (as generate's "H")
      RP_cos   float32 [M, B]          standard Gaussian directions
      minHash  uint32 [M, B/G]         uniform 32-bit values (a random order
                                       of the users per hash)"""
    M = w.M if M is None else M
    if w.family == 0:
        return hash_strings(M, w.B, _rng(seed, 6))
    if w.family == 1:
        return _rng(seed, 8).standard_normal((M, w.B), dtype=np.float32)
    return _rng(seed, 9).integers(0, 1 << 32, size=(M, w.B // w.G), dtype=np.uint64).astype(np.uint32)


def online_split(w: Workload, d: Dict[str, np.ndarray], frac_new: float = 0.01,
                 stream_frac: float = 0.2, seed: int = MASTER_SEED) -> Dict[str, np.ndarray]:
    """Pre-train / stream split of the training ratings for online learning.

    The users with the top `frac_new` of ids and the items with the top
    `frac_new` of ids are "new": all their ratings go to the stream.  Random
    existing x existing ratings fill the stream up to `stream_frac` of the
    ratings.  Ids are random permutations of popularity, so the new sets are
    random samples.  Returns pretrain_{u,i,rc}, stream_{u,i,rc} (stream in a
    random order), M_old, N_old.
    """
    rng = _rng(seed, 21)
    M_old = w.M - max(1, int(round(frac_new * w.M)))
    N_old = w.N - max(1, int(round(frac_new * w.N)))
    u, i, rc = d["train_u"], d["train_i"], d["train_rc"]
    new = (u >= M_old) | (i >= N_old)
    old_idx = np.nonzero(~new)[0]
    n_fill = max(0, int(round(stream_frac * u.size)) - int(new.sum()))
    fill = rng.choice(old_idx, size=min(n_fill, old_idx.size), replace=False)
    in_stream = new.copy()
    in_stream[fill] = True
    s_idx = np.nonzero(in_stream)[0]
    s_idx = s_idx[rng.permutation(s_idx.size)]
    p_idx = np.nonzero(~in_stream)[0]
    return {"pretrain_u": u[p_idx], "pretrain_i": i[p_idx], "pretrain_rc": rc[p_idx],
            "stream_u": u[s_idx], "stream_i": i[s_idx], "stream_rc": rc[s_idx],
            "M_old": np.int64(M_old), "N_old": np.int64(N_old)}


def random_queries(M: int, N: int, n: int, seed: int) -> Tuple[np.ndarray, np.ndarray]:
    """Uniform (user, item) query pairs for predict."""
    rng = _rng(seed, 11)
    return (rng.integers(0, M, n).astype(np.int32), rng.integers(0, N, n).astype(np.int32))


REQUEST_FIELDS = [("kind", "<i4"), ("M_new", "<i4"), ("N_new", "<i4"), ("reserved", "<i4"),
                  ("offset", "<i8"), ("n", "<i8"), ("arrival", "<f8")]


def serve_log(sp: Dict[str, np.ndarray], M: int, N: int, upd_lo: int, upd_hi: int,
              q_lo: int, q_hi: int, queries_per_update: int = 4, seed: int = MASTER_SEED
              ) -> Dict[str, np.ndarray]:
    """A request log for the serving loop over the stream part of an online split.

    The stream is reordered so that new users and items arrive progressively
    (a rating of a new id is placed by its id's rank among the new ids,
    existing x existing ratings at random), then cut into update batches of
    log-uniform sizes in [upd_lo, upd_hi].  Each update is followed by
    `queries_per_update` query requests of log-uniform sizes in [q_lo, q_hi],
    uniform over the users and items known at that point.  Arrival times are
    left at zero (set them for an offered load).  Returns req (records with
    REQUEST_FIELDS), upd_u/upd_i/upd_rc and q_u/q_i (payloads in request order).
    """
    rng = _rng(seed, 31)
    su, si, src = sp["stream_u"], sp["stream_i"], sp["stream_rc"]
    M0, N0 = int(sp["M_old"]), int(sp["N_old"])
    gu = np.where(su >= M0, (su - M0 + 1) / max(M - M0, 1), 0.0)
    gi = np.where(si >= N0, (si - N0 + 1) / max(N - N0, 1), 0.0)
    key = np.maximum(gu, gi)
    old = key == 0
    key[old] = rng.random(int(old.sum()))
    order = np.argsort(key, kind="stable")
    su, si, src = su[order], si[order], src[order]
    recs, qus, qis = [], [], []
    at, qat = 0, 0
    Mc, Nc = M0, N0
    lo, hi = np.log(upd_lo), np.log(upd_hi)
    while at < su.size:
        n = int(np.exp(rng.uniform(lo, hi)))
        n = min(max(n, 1), su.size - at)
        Mc = max(Mc, int(su[at:at + n].max()) + 1)
        Nc = max(Nc, int(si[at:at + n].max()) + 1)
        recs.append((0, Mc, Nc, 0, at, n, 0.0))
        at += n
        for _ in range(queries_per_update):
            m = int(np.exp(rng.uniform(np.log(q_lo), np.log(q_hi))))
            qus.append(rng.integers(0, Mc, m).astype(np.int32))
            qis.append(rng.integers(0, Nc, m).astype(np.int32))
            recs.append((1, 0, 0, 0, qat, m, 0.0))
            qat += m
    req = np.array(recs, dtype=np.dtype(REQUEST_FIELDS, align=True))
    return {"req": req, "upd_u": su.astype(np.int32), "upd_i": si.astype(np.int32),
            "upd_rc": src.astype(np.uint8),
            "q_u": np.concatenate(qus) if qus else np.zeros(0, np.int32),
            "q_i": np.concatenate(qis) if qis else np.zeros(0, np.int32)}


def poisson_arrivals(n: int, rate: float, seed: int = MASTER_SEED) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate (requests / s)."""
    rng = _rng(seed, 41)
    return np.cumsum(rng.exponential(1.0 / rate, n))


def twin_items(u: np.ndarray, it: np.ndarray, rc: np.ndarray, N: int, n_pairs: int,
               seed: int = MASTER_SEED) -> Tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
    """Training ratings in which n_pairs items are twins of others: item b's
    ratings are replaced by a copy of item a's (same users, same codes), so
    a and b have equal rating columns.  Returns (u, it, rc, pairs [n, 2]),
    rows of the ratings sorted by (item, user).  An input transform for
    tests that need colliding items at any hash width."""
    rng = _rng(seed, 31)
    ids = rng.permutation(N)[: 2 * n_pairs].reshape(n_pairs, 2).astype(np.int32)
    a, b = ids[:, 0], ids[:, 1]
    keep = ~np.isin(it, b)
    src = np.isin(it, a)
    to = np.zeros(N, np.int32)
    to[a] = b
    u2 = np.concatenate([u[keep], u[src]])
    i2 = np.concatenate([it[keep], to[it[src]]])
    r2 = np.concatenate([rc[keep], rc[src]])
    order = np.lexsort((u2, i2))
    return (u2[order].astype(np.int32), i2[order].astype(np.int32), r2[order].astype(np.uint8), ids)


# CULSH-MF against CUSGD++ (Sec. 5.3 comparison at F = 32, 64, 128): the
# neighbourhood model with K = 32 and plain MF (u . v only, K = 0) on the same
# data and learning rates.
for _base in ("ml10m", "netflix"):
    for _F in (32, 64, 128):
        WORKLOADS["%s_f%d_k32" % (_base, _F)] = dataclasses.replace(WORKLOADS[_base], name="%s_f%d_k32" % (_base, _F),
                                                                    F=_F, K=32)
        WORKLOADS["%s_f%d_cusgd" % (_base, _F)] = dataclasses.replace(WORKLOADS[_base],
                                                                      name="%s_f%d_cusgd" % (_base, _F), F=_F, K=0,
                                                                      model=1)
