"""Element-by-element comparison of a model table with the oracle's.

An element passes when |gpu - oracle| <= tol * max(|oracle|, floor), where the
floor is a fraction of the table's RMS value: relative error for every
element of typical size, and an absolute bound (tol * floor) for elements
that sit near zero -- values that cancel to near zero in FP64 keep an FP32
rounding residue of the size of the terms that cancelled.
"""
import numpy as np

FLOOR_OF_RMS = 0.1   # floor = 0.1 x RMS of the oracle's table


def table_errors(g, r, floor_of_rms=FLOOR_OF_RMS):
    """(worst element-wise ratio |g - r| / max(|r|, floor), normwise ratio)."""
    g = np.asarray(g, np.float64)
    r = np.asarray(r, np.float64)
    if r.size == 0:
        return 0.0, 0.0
    d = np.abs(g - r)
    rms = float(np.sqrt(np.mean(r * r)))
    floor = max(floor_of_rms * rms, 1e-12)
    elem = float(np.max(d / np.maximum(np.abs(r), floor)))
    norm = float(d.max() / max(np.abs(r).max(), 1e-3))
    return elem, norm


def compare_tables(pairs, tol, say=print, label=""):
    """pairs: {name: (gpu array, oracle array)}; asserts the element-wise bar."""
    worst = {}
    for k, (g, r) in pairs.items():
        worst[k] = table_errors(g, r)
    say("[cmp] %s element-wise / normwise: %s" % (label, {k: "%.2e / %.2e" % v for k, v in worst.items()}))
    bad = {k: v for k, v in worst.items() if v[0] > tol}
    assert not bad, bad
    return worst
