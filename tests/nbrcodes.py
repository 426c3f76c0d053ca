"""Expected neighbour codes of stream records, looked up from the training
triples: for record x (rating (i, j) of the stream), nibble k holds the
rating code of user i for item JK[j][k], or 0 if i has not rated it; slot k
sits in byte k // 2, low nibble first; nibbles past K are 0."""
import numpy as np


def expected_codes(N, K, train_u, train_i, train_rc, order, JK, nstride):
    """order: training-triple index of each record to check."""
    key = train_u.astype(np.int64) * N + train_i
    srt = np.argsort(key, kind="stable")
    skey, src = key[srt], train_rc[srt]
    u = train_u[order].astype(np.int64)
    nb = JK[train_i[order]].astype(np.int64)
    q = u[:, None] * N + nb
    at = np.minimum(np.searchsorted(skey, q), skey.size - 1)
    code = np.where(skey[at] == q, src[at], 0).astype(np.uint8)
    full = np.zeros((order.size, 2 * nstride), np.uint8)
    full[:, :K] = code
    return full[:, 0::2] | (full[:, 1::2] << 4)
